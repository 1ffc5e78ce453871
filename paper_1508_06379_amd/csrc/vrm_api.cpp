// C ABI of libvrm: context management, argument checking and the order of
// the kernel launches of each entry point (the entry points are documented
// in include/vrm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "vrm_internal.h"

size_t vrm_sort_tmp_bytes(int32_t cap);

namespace {
thread_local std::string g_err;

vrm::LaunchParams launch_params(const vrm_ctx* c, const vrm_params* p)
{
    vrm::LaunchParams L{};
    L.phase1 = c->lp_objective;
    const double h = p->h;
    L.h = (float)h;
    L.lo2 = (float)(p->r * p->r * h * h * (1.0 - 0x1p-20));
    L.hi2 = (float)(p->R * p->R * h * h * (1.0 + 0x1p-20));
    L.lo2f = L.lo2;
    L.hi2f = (float)(p->R_full * p->R_full * h * h * (1.0 + 0x1p-20));
    L.rad = (float)(1.5 * h);
    L.ex2 = (float)(0.25 * h * h);
    // exact offset scaling by 2^-e with 2^e >= h; the rhs and costs absorb s = 2^e / h
    int e = (int)std::ceil(std::log2(h));
    if (std::ldexp(1.0, e) < h) ++e;
    L.scale2e = (float)std::ldexp(1.0, -e);
    double s = std::ldexp(1.0, e) / h;
    double bt = 2.0 / (s * s);
    L.bt_hi = (float)bt;
    L.bt_lo = (float)(bt - (double)L.bt_hi);
    double cs = std::pow(s, p->q + 1);
    L.cs_hi = (float)cs;
    L.cs_lo = (float)(cs - (double)L.cs_hi);
    L.lam = (float)(p->nu / (h * h));
    L.sc = (float)s;
    L.q = p->q;
    L.m = p->q == 2 ? 5 : 9;
    L.det = p->deterministic;
    L.max_cert = c->tuning.cert_rounds > 0 ? c->tuning.cert_rounds : vrm::kMaxCert;
    return L;
}

int check_params(const vrm_params* p)
{
    if (!p) return vrm_fail(VRM_E_ARG, "params is NULL");
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return vrm_fail(VRM_E_ARG, "h must be positive and finite");
    if (!(p->r > 0.0) || !(p->R > p->r) || !std::isfinite(p->R))
        return vrm_fail(VRM_E_ARG, "need 0 < r < R (got r=%g, R=%g)", p->r, p->R);
    if (!(p->R_full >= p->R) || !std::isfinite(p->R_full))
        return vrm_fail(VRM_E_ARG, "need R_full >= R (got %g)", p->R_full);
    if (p->q != 2 && p->q != 3) return vrm_fail(VRM_E_ARG, "q must be 2 or 3 (got %d)", p->q);
    if (!(p->nu >= 0.0) || !std::isfinite(p->nu)) return vrm_fail(VRM_E_ARG, "nu must be >= 0");
    if (!(p->c_diff >= 0.0) || !std::isfinite(p->c_diff)) return vrm_fail(VRM_E_ARG, "c_diff must be >= 0");
    if (!(p->dt >= 0.0) || !std::isfinite(p->dt)) return vrm_fail(VRM_E_ARG, "dt must be >= 0");
    if (p->deterministic != 0 && p->deterministic != 1)
        return vrm_fail(VRM_E_ARG, "deterministic must be 0 or 1 (got %d)", p->deterministic);
    return VRM_OK;
}

int check_cloud(vrm_ctx* c, const vrm_cloud* cl)
{
    if (!c) return vrm_fail(VRM_E_ARG, "context is NULL");
    if (!cl || !cl->x_dev || !cl->y_dev || !cl->gamma_dev || !cl->id_dev || !cl->n_dev)
        return vrm_fail(VRM_E_ARG, "cloud or one of its arrays is NULL");
    if (cl->capacity <= 0 || cl->capacity > c->capacity)
        return vrm_fail(VRM_E_ARG, "cloud capacity %d outside (0, %d]", cl->capacity, c->capacity);
    return VRM_OK;
}

// Read N from the device (synchronises) and remember it.
int read_n(vrm_ctx* c, const vrm_cloud* cl)
{
    int32_t n = 0;
    VRM_HIP(hipMemcpyAsync(&n, cl->n_dev, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    VRM_HIP(hipStreamSynchronize(c->stream));
    if (n < 0 || n > cl->capacity) return vrm_fail(VRM_E_ARG, "particle count %d outside [0, %d]", n, cl->capacity);
    if (c->n_ptr != cl->n_dev || c->cloud_x != cl->x_dev || c->n != n) {
        // another cloud, or the count changed behind the context: cached cells are stale
        c->cells_valid = 0;
        c->sorted = 0;
    }
    c->n = n;
    c->n_ptr = cl->n_dev;
    c->cloud_x = cl->x_dev;
    return VRM_OK;
}

int cached_n(vrm_ctx* c, const vrm_cloud* cl)
{
    if (c->n_ptr != cl->n_dev || !c->n_diffused_valid)
        return vrm_fail(VRM_E_STATE, "no diffused set for this cloud: call vrm_select_diffused, vrm_set_diffused or "
                                     "vrm_insert_particles first");
    return VRM_OK;
}

template <typename T>
int alloc(T** p, size_t count)
{
    void* q = nullptr;
    VRM_HIP(hipMalloc(&q, count * sizeof(T) + 16));
    *p = static_cast<T*>(q);
    return VRM_OK;
}

__global__ void k_copy_mask(int n, const uint8_t* in, uint8_t* out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] ? 1 : 0;
}

__global__ void k_clear_bad(vrm::GridState* g) { g->bad = 0; }
}  // namespace

int vrm_nonfinite(vrm_ctx* c, int32_t bits)
{
    hipLaunchKernelGGL(k_clear_bad, dim3(1), dim3(1), 0, c->stream, c->grid);
    c->cells_valid = 0;
    c->sorted = 0;
    c->n_diffused_valid = 0;
    c->base_valid = 0;
    (void)hipGetLastError();
    return vrm_fail(VRM_E_NONFINITE, "non-finite %s%s%s in the cloud; it was left unchanged",
                    (bits & vrm::kBadPos) ? "position" : "", (bits & vrm::kBadPos) && (bits & vrm::kBadGamma) ? " and " : "",
                    (bits & vrm::kBadGamma) ? "circulation" : "");
}

int vrm_fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int vrm_hip_check(hipError_t e, const char* what)
{
    return vrm_fail(VRM_E_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

extern "C" {

const char* vrm_last_error(void) { return g_err.c_str(); }

const char* vrm_status_string(int code)
{
    switch (code) {
    case VRM_OK: return "ok";
    case VRM_E_ARG: return "invalid argument";
    case VRM_E_CAPACITY: return "capacity exceeded";
    case VRM_E_HIP: return "HIP runtime error";
    case VRM_E_STATE: return "invalid call order";
    case VRM_E_NONFINITE: return "non-finite position or circulation";
    default: return "unknown";
    }
}

int vrm_create(vrm_ctx** out, int device, void* stream, int32_t capacity)
{
    if (!out) return vrm_fail(VRM_E_ARG, "out is NULL");
    *out = nullptr;
    // complete-neighbourhood LPs pack a particle slot in 26 bits
    if (capacity <= 0 || capacity > (1 << 26)) return vrm_fail(VRM_E_ARG, "capacity %d outside (0, 2^26]", capacity);
    VRM_HIP(hipSetDevice(device));
    vrm_ctx* c = new vrm_ctx();
    std::memset(c, 0, sizeof(*c));
    c->graph_enabled = 1;
    vrm_set_tuning(c, nullptr);
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->capacity = capacity;
    c->ncell_cap = 2 * capacity + 4096;
    size_t cap = (size_t)capacity, cap2 = 2 * cap, nc = (size_t)c->ncell_cap + 1;
    int r = VRM_OK;
#define A(ptr, n)                                \
    if (r == VRM_OK) r = alloc(&c->ptr, (n));
    A(grid, 1);
    A(queues, 1);
    A(sel, 1);
    A(counters, (vrm::kCounterStripes * vrm::kCounterStride + sizeof(vrm_counters) - 1) / sizeof(vrm_counters));
    A(cell_of, cap);
    A(rank, cap);
    A(cell_start, nc);
    A(scan_part, 1024);
    A(perm, cap);
    A(xs, cap);
    A(ys, cap);
    A(ids, cap);
    A(diffused, cap);
    A(acc, 2 * cap);
    A(x0, cap);
    A(y0, cap);
    A(g0, cap);
    A(q_small, cap);
    A(q_full, cap);
    A(q_retry, cap);
    A(srec.i, cap);
    A(srec.rank, cap);
    A(srec.pj, cap * VRM_NSEG);
    A(srec.off, cap * 4 * VRM_NSEG);
    c->srec.cap = capacity;
    A(cx, cap2);
    A(cy, cap2);
    A(ckey, cap2);
    A(cstate, cap2);
    A(ccell, cap2);
    A(crank, cap2);
    A(cstart, nc);
    A(cperm, cap2);
    A(akey, cap2);
    A(aidx, cap2);
    A(tmp_f, 3 * cap);
    A(tmp_i, cap);
    A(tmp_u8, cap);
    A(verify_buf, 8);
    A(full_cols, cap * VRM_KMAX);
    A(full_k, cap);
    A(full_order, cap);
    A(khist, 2 * (VRM_KMAX + 1));
    A(lkey, cap);
    A(pivhist, cap);
    A(q_defer, cap);
    A(pmask, cap);
#undef A
    if (r == VRM_OK) {
        c->sort_tmp_bytes = std::max(vrm_sort_tmp_bytes(capacity), vrm_remove_tmp_bytes(capacity));
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, c->sort_tmp_bytes + 256);
        if (e != hipSuccess) r = vrm_hip_check(e, "hipMalloc(sort)");
        c->sort_tmp = p;
    }
    if (r == VRM_OK) {
        void* p = nullptr;
        hipError_t e = hipHostMalloc(&p, sizeof(vrm::HostQueues), hipHostMallocCoherent);
        if (e != hipSuccess) r = vrm_hip_check(e, "hipHostMalloc(queue record)");
        c->q_host = static_cast<vrm::HostQueues*>(p);
        if (c->q_host) std::memset(c->q_host, 0, sizeof(vrm::HostQueues));
    }
    if (r == VRM_OK) {
        hipError_t e = hipMemsetAsync(c->acc, 0, 2 * cap * sizeof(float), c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->counters, 0, vrm::kCounterStripes * vrm::kCounterStride, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->queues, 0, sizeof(vrm::Queues), c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->sel, 0, sizeof(vrm::SelectState), c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->grid, 0, sizeof(vrm::GridState), c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->khist, 0, 2 * (VRM_KMAX + 1) * sizeof(int32_t), c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->pivhist, 0xff, cap, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) r = vrm_hip_check(e, "initialisation");
    }
    if (r != VRM_OK) {
        std::string keep = g_err;
        vrm_destroy(c);
        g_err = keep;
        return r;
    }
    *out = c;
    return VRM_OK;
}

int vrm_destroy(vrm_ctx* c)
{
    if (!c) return VRM_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    void* ptrs[] = {c->grid, c->queues, c->sel, c->counters, c->cell_of, c->rank, c->cell_start, c->scan_part,
                    c->perm, c->xs, c->ys, c->ids, c->diffused, c->acc, c->x0, c->y0, c->g0, c->q_small, c->q_full, c->q_retry,
                    c->srec.i, c->srec.rank, c->srec.pj, c->srec.off, c->cx, c->cy, c->ckey, c->cstate, c->ccell, c->crank, c->cstart, c->cperm,
                    c->akey, c->aidx, c->tmp_f, c->tmp_i, c->tmp_u8, c->verify_buf, c->sort_tmp, c->full_cols,
                    c->full_k, c->full_order, c->khist, c->lkey, c->pivhist, c->q_defer, c->pmask};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->q_host) (void)hipHostFree(c->q_host);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->t_dev) (void)hipFree(c->t_dev);
    if (c->prev) (void)hipFree(c->prev);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->feat) (void)hipFree(c->feat);
    if (c->u_tmp) (void)hipFree(c->u_tmp);
    if (c->pred) (void)hipFree(c->pred);
    vrm_mlp_free(c);
    if (c->ev_start) {
        for (int k = 0; k < vrm::kMaxTimed; ++k) {
            (void)hipEventDestroy(c->ev_start[k]);
            (void)hipEventDestroy(c->ev_stop[k]);
        }
        delete[] c->ev_start;
        delete[] c->ev_stop;
        delete[] c->ev_group;
    }
    delete c;
    return VRM_OK;
}

int vrm_select_diffused(vrm_ctx* c, const vrm_cloud* cl, const vrm_params* p, uint8_t* mask_dev)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = read_n(c, cl);
    if (r) return r;
    double factor = p->c_diff * std::pow(p->h, p->q + 1);
    {
        vrm::ScopedTimer tm(c, VRM_T_SELECT);
        r = vrm_select_run(c, cl->gamma_dev, cl->id_dev, c->n, factor);
    }
    if (r) return r;
    if (mask_dev && c->n > 0) {
        hipLaunchKernelGGL(k_copy_mask, dim3((c->n + 255) / 256), dim3(256), 0, c->stream, c->n, c->diffused, mask_dev);
        VRM_HIP(hipGetLastError());
    }
    c->n_diffused_valid = 1;
    return VRM_OK;
}

int vrm_set_diffused(vrm_ctx* c, const vrm_cloud* cl, const uint8_t* mask_dev)
{
    int r = check_cloud(c, cl);
    if (!r && !mask_dev) r = vrm_fail(VRM_E_ARG, "mask is NULL");
    if (!r) r = read_n(c, cl);
    if (r) return r;
    if (c->n > 0) {
        hipLaunchKernelGGL(k_copy_mask, dim3((c->n + 255) / 256), dim3(256), 0, c->stream, c->n, mask_dev, c->diffused);
        VRM_HIP(hipGetLastError());
    }
    c->n_diffused_valid = 1;
    return VRM_OK;
}

int vrm_build_neighbourhoods(vrm_ctx* c, const vrm_cloud* cl, const vrm_params* p, int32_t* small_idx_dev,
                             int32_t* kfull_dev)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = cached_n(c, cl);
    if (r) return r;
    vrm::LaunchParams L = launch_params(c, p);
    r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, c->n, L);
    if (r) return r;
    c->cells_valid = 1;
    c->sorted = 0;
    return vrm_small_nbhd_run(c, cl, c->n, L, small_idx_dev, kfull_dev);
}

int vrm_insert_particles(vrm_ctx* c, vrm_cloud* cl, const vrm_params* p)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = read_n(c, cl);
    if (r) return r;
    vrm::LaunchParams L = launch_params(c, p);
    double factor = p->c_diff * std::pow(p->h, p->q + 1);
    {
        vrm::ScopedTimer tm(c, VRM_T_SELECT);
        r = vrm_select_run(c, cl->gamma_dev, cl->id_dev, c->n, factor);
    }
    if (r) return r;
    // the cell list of the last reorder is still valid if nothing moved since
    if (!(c->sorted && c->cells_valid)) {
        r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, c->n, L);
        if (r) return r;
        c->cells_valid = 1;
        c->sorted = 0;
    }
    c->n_diffused_valid = 1;
    int n2;
    {
        vrm::ScopedTimer tm(c, VRM_T_INSERT);
        n2 = vrm_insert_run(c, cl, c->n, L);
    }
    if (n2 < 0) return n2;   // the cloud is unchanged
    c->base_valid = 0;
    if (n2 == c->n && c->sorted) return VRM_OK;   // nothing appended, already in cell order
    if (n2 != c->n) {
        r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, n2, L);
        if (r) return r;
    }
    c->n = n2;
    r = vrm_reorder_cloud(c, cl, n2);
    if (r) return r;
    c->cells_valid = 1;
    c->sorted = 1;
    return VRM_OK;
}

int vrm_remove_particles(vrm_ctx* c, vrm_cloud* cl, const vrm_params* p, int32_t* n_removed, int32_t* n_candidates)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = read_n(c, cl);
    if (r) return r;
    vrm::LaunchParams L = launch_params(c, p);
    if (!(c->sorted && c->cells_valid)) {
        r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, c->n, L);
        if (r) return r;
        c->cells_valid = 1;
        c->sorted = 0;
    }
    // the identity LP: rows 1, x, y; rhs e0 (scale-free); cost |r/h|^2 = |X|^2 (2^e / h)^2
    vrm::LaunchParams R = L;
    R.q = 1;
    R.m = 3;
    R.bt_hi = 1.0f;
    R.bt_lo = 0.0f;
    R.cs_hi = (float)((double)L.sc * (double)L.sc);
    R.cs_lo = (float)((double)L.sc * (double)L.sc - (double)R.cs_hi);
    R.phase1 = 0;
    int32_t nc = 0;
    const int m = vrm_remove_run(c, cl, c->n, R, &nc);
    if (m < 0) return m;
    if (n_candidates) *n_candidates = nc;
    if (n_removed) *n_removed = c->n - m;
    if (m != c->n) {
        c->n = m;
        c->cells_valid = 0;
        c->sorted = 0;
        c->n_diffused_valid = 0;
        c->base_valid = 0;
    }
    return VRM_OK;
}

int vrm_solve_fractions(vrm_ctx* c, const vrm_cloud* cl, const vrm_params* p, vrm_stencils* out)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = cached_n(c, cl);
    if (!r && (!out || !out->small_idx_dev || !out->small_f_dev || !out->fii_dev || !out->status_dev ||
               !out->full_k_dev || (!out->full_idx_dev) != (!out->full_f_dev)))
        r = vrm_fail(VRM_E_ARG, "stencil output arrays missing");
    if (r) return r;
    vrm::LaunchParams L = launch_params(c, p);
    if (!c->cells_valid) {
        r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, c->n, L);
        if (r) return r;
        c->cells_valid = 1;
    }
    return vrm_stencil_run(c, cl, c->n, L, out, 0);
}

}  // extern "C"

namespace {

// One SSP-RK3 stage as launches only (no host synchronisation, so that it can
// be captured): the stage kernels read the particle count on the device and
// size their grids for nb >= N.
int stage_launch(vrm_ctx* c, vrm_cloud* cl, const float* u_dev, const float* v_dev, const vrm_params* p, int stage,
                 int nb)
{
    int r;
    vrm::LaunchParams L = launch_params(c, p);
    if (stage == 0) {
        r = vrm_save_base_run(c, cl, nb, L.det);
        if (r) return r;
        c->base_valid = 1;
    }
    if (!c->cells_valid) {
        r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, nb, L, cl->n_dev);
        if (r) return r;
        c->cells_valid = 1;
    }
    r = vrm_stencil_run(c, cl, nb, L, nullptr, 1);
    if (!r) {
        vrm::ScopedTimer tm(c, VRM_T_COMBINE);
        r = vrm_combine_run(c, cl, nb, u_dev, v_dev, p->dt, L.lam, stage, L.det);
    }
    if (r) return r;
    if (u_dev) {
        c->cells_valid = 0;
        c->sorted = 0;
    }
    if (stage == 2) c->base_valid = 0;
    return VRM_OK;
}

// The three stages of a step after insertion; with vortices, the stage times
// are t + c_s dt, or *t_dev + c_s dt when t_dev is given.
int step_stages(vrm_ctx* c, vrm_cloud* cl, const vrm_params* p, const float* vort_dev, int32_t n_vort, double t,
                const double* t_dev, int nb)
{
    static const double tc[3] = {0.0, 1.0, 0.5};
    for (int s = 0; s < 3; ++s) {
        const float *u = nullptr, *v = nullptr;
        if (n_vort > 0) {
            const double ts = t_dev ? tc[s] * p->dt : t + tc[s] * p->dt;
            int r = vrm_velocity_run(c, cl, nb, vort_dev, n_vort, p->nu, ts, c->u_tmp, c->v_tmp, t_dev);
            if (r) return r;
            u = c->u_tmp;
            v = c->v_tmp;
        }
        int r = stage_launch(c, cl, u, v, p, s, nb);
        if (r) return r;
    }
    return VRM_OK;
}

__global__ void k_set_time(double* t_dev, double t) { *t_dev = t; }

// Timer events of the last graph replay into the accumulated totals.
int collect_graph_timing(vrm_ctx* c)
{
    if (!c->graph_pending) return VRM_OK;
    c->graph_pending = 0;
    const int s0 = vrm::kMaxTimed - vrm::kGraphTimed;
    VRM_HIP(hipEventSynchronize(c->ev_stop[s0 + c->graph_slots - 1]));
    for (int k = s0; k < s0 + c->graph_slots; ++k) {
        float ms = 0.0f;
        VRM_HIP(hipEventElapsedTime(&ms, c->ev_start[k], c->ev_stop[k]));
        c->acc_ms[c->ev_group[k]] += ms;
        c->acc_n[c->ev_group[k]] += 1;
        c->launches[c->ev_group[k]] += 1;
    }
    return VRM_OK;
}

void drop_graph(vrm_ctx* c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// What a captured step depends on besides the device state it reads.
void graph_key(vrm_ctx* c, const vrm_cloud* cl, const vrm_params* p, const float* vort_dev, int32_t n_vort,
               unsigned char (&key)[256])
{
    std::memset(key, 0, sizeof(key));
    size_t o = 0;
    auto put = [&](const void* v, size_t n) {
        std::memcpy(key + o, v, n);
        o += n;
    };
    put(cl, sizeof(vrm_cloud));
    put(p, sizeof(vrm_params));
    put(&vort_dev, sizeof(vort_dev));
    put(&n_vort, sizeof(n_vort));
    int flags[4] = {c->timing, c->warm, c->mlp ? c->mlp->loaded : 0, c->lp_objective};
    put(flags, sizeof(flags));
    const void* mp = c->mlp;
    put(&mp, sizeof(mp));
    put(&c->tuning, sizeof(vrm_tuning));
}
static_assert(sizeof(vrm_cloud) + sizeof(vrm_params) + sizeof(void*) + sizeof(int32_t) + 4 * sizeof(int) +
                      sizeof(void*) + sizeof(vrm_tuning) <=
                  256,
              "graph key buffer too small");

}  // namespace

extern "C" {

int vrm_rk_stage(vrm_ctx* c, vrm_cloud* cl, const float* u_dev, const float* v_dev, const vrm_params* p, int stage)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = cached_n(c, cl);
    if (!r && (stage < 0 || stage > 2)) r = vrm_fail(VRM_E_ARG, "stage must be 0, 1 or 2 (got %d)", stage);
    if (!r && ((u_dev == nullptr) != (v_dev == nullptr))) r = vrm_fail(VRM_E_ARG, "u and v must both be given or both NULL");
    if (!r && stage > 0 && !c->base_valid) r = vrm_fail(VRM_E_STATE, "stage %d before stage 0", stage);
    if (r) return r;
    return stage_launch(c, cl, u_dev, v_dev, p, stage, c->n);
}

int vrm_set_tuning(vrm_ctx* c, const vrm_tuning* t)
{
    if (!c) return vrm_fail(VRM_E_ARG, "context is NULL");
    vrm_tuning d{};
    d.lp_small_blocks = 2048;
    d.lp_full_blocks = 2048;
    d.full_stored_cost_n = 200000;
    d.infer_blocks = 768;   // the persistent inference grid: three resident blocks on each of 256 CUs
    d.lp_small_lanes = 64;
    if (t) {
        const int ln = t->lp_small_lanes;
        if (ln < 0 || ln > 64 || (ln & (ln - 1)) != 0)
            return vrm_fail(VRM_E_ARG, "lp_small_lanes must be 0 or a power of two <= 64 (got %d)", ln);
        if (t->lp_small_blocks < 0 || t->lp_full_blocks < 0 || t->infer_blocks < 0 || t->full_stored_cost_n < -1 ||
            t->lp_small_blocks > (1 << 20) || t->lp_full_blocks > (1 << 22) || t->infer_blocks > (1 << 20))
            return vrm_fail(VRM_E_ARG, "tuning values out of range");
        if (t->lp_small_blocks) d.lp_small_blocks = t->lp_small_blocks;
        if (t->lp_full_blocks) d.lp_full_blocks = t->lp_full_blocks;
        if (t->full_stored_cost_n) d.full_stored_cost_n = t->full_stored_cost_n;
        if (t->infer_blocks) d.infer_blocks = t->infer_blocks;
        if (t->lp_small_lanes) d.lp_small_lanes = t->lp_small_lanes;
        if (t->lp_small_coop != 0 && t->lp_small_coop != 1)
            return vrm_fail(VRM_E_ARG, "lp_small_coop must be 0 or 1 (got %d)", t->lp_small_coop);
        d.lp_small_coop = t->lp_small_coop;
        if (t->cert_rounds < 0 || t->cert_rounds > 64)
            return vrm_fail(VRM_E_ARG, "cert_rounds must be in [0, 64] (got %d)", t->cert_rounds);
        d.cert_rounds = t->cert_rounds;
    }
    c->tuning = d;
    return VRM_OK;
}

int vrm_get_tuning(vrm_ctx* c, vrm_tuning* out)
{
    if (!c || !out) return vrm_fail(VRM_E_ARG, "NULL argument");
    *out = c->tuning;
    return VRM_OK;
}

int vrm_set_graph(vrm_ctx* c, int enable)
{
    if (!c) return vrm_fail(VRM_E_ARG, "context is NULL");
    c->graph_enabled = enable ? 1 : 0;
    if (!enable) {
        VRM_HIP(hipStreamSynchronize(c->stream));
        int r = collect_graph_timing(c);
        drop_graph(c);
        if (r) return r;
    }
    return VRM_OK;
}

int vrm_step(vrm_ctx* c, vrm_cloud* cl, const vrm_params* p, const float* vort_dev, int32_t n_vort, double t)
{
    if (n_vort < 0 || (n_vort > 0 && !vort_dev)) return vrm_fail(VRM_E_ARG, "vortex table");
    int r = vrm_insert_particles(c, cl, p);   // synchronises: the previous replay has finished
    if (r) return r;
    r = collect_graph_timing(c);
    if (r) return r;
    if (n_vort > 0 && !c->u_tmp) {
        void* q = nullptr;
        VRM_HIP(hipMalloc(&q, sizeof(float) * (size_t)c->capacity * 2 + 64));
        c->u_tmp = (float*)q;
        c->v_tmp = c->u_tmp + c->capacity;
    }
    const int n = c->n;
    // timer events recorded by graph nodes cannot be read back (hipEventElapsedTime rejects
    // them), so timed steps launch their stages directly
    if (!c->graph_enabled || c->timing || c->graph_failed[0] || n <= 0)
        return step_stages(c, cl, p, vort_dev, n_vort, t, nullptr, n);

    unsigned char key[256];
    graph_key(c, cl, p, vort_dev, n_vort, key);
    const int f0[3] = {c->cells_valid, c->sorted, c->base_valid};
    if (!c->graph_exec || n > c->graph_nb || std::memcmp(key, c->graph_key, sizeof(key)) != 0 ||
        f0[0] != 1 || f0[2] != 0) {
        drop_graph(c);
        if (!c->t_dev) {
            void* q = nullptr;
            VRM_HIP(hipMalloc(&q, 64));
            c->t_dev = (double*)q;
        }
        if (!c->cap_stream) VRM_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        const int nb = std::min(c->capacity, n + std::max(4096, n / 8));
        // the stages are recorded on the capture stream and replayed on the context's stream
        hipStream_t own = c->stream;
        c->stream = c->cap_stream;
        c->capturing = 1;
        c->graph_slots = 0;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        int rr = VRM_OK;
        if (e == hipSuccess) rr = step_stages(c, cl, p, vort_dev, n_vort, 0.0, c->t_dev, nb);
        hipGraph_t g = nullptr;
        hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(c->stream, &g) : e;
        c->capturing = 0;
        c->stream = own;
        hipGraphExec_t ex = nullptr;
        if (e == hipSuccess && e2 == hipSuccess && rr == VRM_OK && g)
            e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        const int f1[3] = {c->cells_valid, c->sorted, c->base_valid};
        c->cells_valid = f0[0];
        c->sorted = f0[1];
        c->base_valid = f0[2];
        if (e != hipSuccess || e2 != hipSuccess || rr != VRM_OK || !ex) {
            // this runtime cannot capture the stages: launch them directly from now on
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            c->graph_failed[0] = 1;
            c->graph_slots = 0;
            return step_stages(c, cl, p, vort_dev, n_vort, t, nullptr, n);
        }
        c->graph = g;
        c->graph_exec = ex;
        c->graph_nb = nb;
        std::memcpy(c->graph_key, key, sizeof(key));
        std::memcpy(c->graph_flags, f1, sizeof(f1));
    }
    hipLaunchKernelGGL(k_set_time, dim3(1), dim3(1), 0, c->stream, c->t_dev, t);
    VRM_HIP(hipGetLastError());
    VRM_HIP(hipGraphLaunch(c->graph_exec, c->stream));
    c->graph_replays += 1;
    c->graph_pending = c->timing && c->graph_slots > 0;
    c->cells_valid = c->graph_flags[0];
    c->sorted = c->graph_flags[1];
    c->base_valid = c->graph_flags[2];
    return VRM_OK;
}

int vrm_verify(vrm_ctx* c, const vrm_cloud* cl, const vrm_params* p, const vrm_stencils* st, double* report_dev)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r && !report_dev) r = vrm_fail(VRM_E_ARG, "report is NULL");
    if (!r && c->n_ptr != cl->n_dev) r = read_n(c, cl);
    if (r) return r;
    vrm::LaunchParams L = launch_params(c, p);
    return vrm_verify_run(c, cl, c->n, L, p->h, st, report_dev);
}

int vrm_read_counters(vrm_ctx* c, vrm_counters* out)
{
    if (!c || !out) return vrm_fail(VRM_E_ARG, "NULL argument");
    // the copies of the counters: accumulated fields are summed, assigned ones are in copy 0
    static thread_local char buf[vrm::kCounterStripes * vrm::kCounterStride];
    int32_t bad = 0;
    VRM_HIP(hipMemcpyAsync(buf, c->counters, sizeof(buf), hipMemcpyDeviceToHost, c->stream));
    VRM_HIP(hipMemcpyAsync(&bad, &c->grid->bad, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
    VRM_HIP(hipStreamSynchronize(c->stream));
    *out = *reinterpret_cast<const vrm_counters*>(buf);
    for (int k = 1; k < vrm::kCounterStripes; ++k) {
        const vrm_counters& s = *reinterpret_cast<const vrm_counters*>(buf + k * vrm::kCounterStride);
        out->n_diffused += s.n_diffused;
        out->n_small += s.n_small;
        out->n_full += s.n_full;
        out->n_infeasible += s.n_infeasible;
        out->n_uncertified += s.n_uncertified;
        out->n_truncated += s.n_truncated;
        out->n_grid_clamped += s.n_grid_clamped;
        out->pivots += s.pivots;
        out->redistributions += s.redistributions;
        out->full_cols += s.full_cols;
        out->warm_hit += s.warm_hit;
        out->warm_phase2 += s.warm_phase2;
        out->warm_cold += s.warm_cold;
        out->cert_rounds += s.cert_rounds;
        out->cert_exact += s.cert_exact;
    }
    out->n = c->n;
    out->graph_replays = c->graph_replays;
    if (bad) return vrm_nonfinite(c, bad);
    return VRM_OK;
}

int vrm_mlp_load(vrm_ctx* c, const float* w)
{
    if (!c || !w) return vrm_fail(VRM_E_ARG, "NULL argument");
    int r = vrm_mlp_alloc(c, 0);
    if (!r) r = vrm_mlp_set_weights(c, w);
    return r;
}

int vrm_mlp_read(vrm_ctx* c, float* w)
{
    if (!c || !w) return vrm_fail(VRM_E_ARG, "NULL argument");
    if (!c->mlp) return vrm_fail(VRM_E_STATE, "no network parameters");
    return vrm_mlp_read_weights(c, w);
}

int vrm_set_warm_start(vrm_ctx* c, int enable)
{
    if (!c) return vrm_fail(VRM_E_ARG, "context is NULL");
    if (enable < 0 || enable > 2) return vrm_fail(VRM_E_ARG, "warm start mode %d (0, 1 or 2)", enable);
    if (enable && c->lp_objective == 2) return vrm_fail(VRM_E_STATE, "the least-squares objective has no warm start");
    if (enable == 2) {
        if (!c->prev) {
            void* p = nullptr;
            VRM_HIP(hipMalloc(&p, sizeof(int32_t) * (size_t)c->capacity * 9 + 64));
            c->prev = (int32_t*)p;
            VRM_HIP(hipMemsetAsync(c->prev, 0xff, sizeof(int32_t) * (size_t)c->capacity * 9, c->stream));
        }
        c->warm = 2;
        return VRM_OK;
    }
    if (enable) {
        if (!c->mlp || !c->mlp->loaded) return vrm_fail(VRM_E_STATE, "warm start needs network parameters (vrm_mlp_load)");
        if (!c->feat) {
            void* p = nullptr;
            VRM_HIP(hipMalloc(&p, sizeof(uint16_t) * (size_t)c->capacity * vrm::kMlpIn + 64));
            c->feat = (uint16_t*)p;
            VRM_HIP(hipMalloc(&p, sizeof(float) * (size_t)c->capacity * vrm::kMlpOut + 64));
            c->pred = (float*)p;
        }
    }
    c->warm = enable ? 1 : 0;
    return VRM_OK;
}

int vrm_collect_training(vrm_ctx* c, const vrm_cloud* cl, const vrm_params* p, uint16_t* x, float* y, int32_t max_rows,
                         int32_t* rows)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = cached_n(c, cl);
    if (!r && (!x || !y || !rows || max_rows <= 0)) r = vrm_fail(VRM_E_ARG, "training buffers");
    if (r) return r;
    vrm::LaunchParams L = launch_params(c, p);
    if (!c->cells_valid) {
        r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, c->n, L);
        if (r) return r;
        c->cells_valid = 1;
    }
    r = vrm_stencil_run(c, cl, c->n, L, nullptr, 0, x, y, max_rows);
    if (r) return r;
    vrm::Queues q;
    VRM_HIP(hipMemcpyAsync(&q, c->queues, sizeof(q), hipMemcpyDeviceToHost, c->stream));
    VRM_HIP(hipStreamSynchronize(c->stream));
    int got = L.m == 5 ? q.last_small : q.last_full;
    *rows = got < max_rows ? got : max_rows;
    return VRM_OK;
}

int vrm_warm_predictions(vrm_ctx* c, const vrm_cloud* cl, const vrm_params* p, float* out_dev, int32_t* particle_dev,
                         int32_t max_rows, int32_t* rows_host)
{
    int r = check_cloud(c, cl);
    if (!r) r = check_params(p);
    if (!r) r = cached_n(c, cl);
    if (!r && (!out_dev || !particle_dev || !rows_host || max_rows <= 0)) r = vrm_fail(VRM_E_ARG, "prediction buffers");
    if (!r && (c->warm != 1 || !c->feat || !c->mlp || !c->mlp->loaded))
        r = vrm_fail(VRM_E_STATE, "needs the learned warm start (vrm_mlp_load, vrm_set_warm_start(ctx, 1))");
    if (r) return r;
    vrm::LaunchParams L = launch_params(c, p);
    if (!c->cells_valid) {
        r = vrm_build_cells(c, cl->x_dev, cl->y_dev, cl->id_dev, c->n, L);
        if (r) return r;
        c->cells_valid = 1;
    }
    r = vrm_warm_predict_run(c, cl, c->n, L, out_dev, particle_dev, max_rows);
    if (r) return r;
    vrm::Queues q;
    VRM_HIP(hipMemcpyAsync(&q, c->queues, sizeof(q), hipMemcpyDeviceToHost, c->stream));
    VRM_HIP(hipStreamSynchronize(c->stream));
    const int got = L.m == 5 ? q.last_small : q.last_full;
    *rows_host = got < max_rows ? got : max_rows;
    return VRM_OK;
}

int vrm_mlp_train_step(vrm_ctx* c, const uint16_t* x, const float* y, int32_t rows, float lr, float wd, float wf,
                       double* loss, float* grad)
{
    if (!c || !x || !y || rows <= 0) return vrm_fail(VRM_E_ARG, "training arguments");
    if (!c->mlp || !c->mlp->loaded) return vrm_fail(VRM_E_STATE, "no network parameters (vrm_mlp_load)");
    int r = vrm_mlp_alloc(c, rows);
    if (!r) r = vrm_mlp_train(c, x, y, rows, lr, wd, wf, loss, grad);
    return r;
}

int vrm_mlp_infer(vrm_ctx* c, const uint16_t* x, int32_t rows, float* y)
{
    if (!c || !x || !y || rows < 0) return vrm_fail(VRM_E_ARG, "inference arguments");
    if (!c->mlp || !c->mlp->loaded) return vrm_fail(VRM_E_STATE, "no network parameters (vrm_mlp_load)");
    vrm::ScopedTimer tm(c, VRM_T_MLP);
    return vrm_mlp_infer_run(c, x, (int)rows, y, nullptr);
}

int vrm_gemm_bf16(vrm_ctx* c, const uint16_t* a, const uint16_t* b, float* out, int32_t M, int32_t N, int32_t K,
                  int ta, int tb)
{
    if (!c || !a || !b || !out || M <= 0 || N <= 0 || K <= 0) return vrm_fail(VRM_E_ARG, "gemm arguments");
    return vrm_gemm_test(c, a, b, out, M, N, K, ta, tb);
}

int vrm_timing(vrm_ctx* c, int enable) { return vrm_timing_groups(c, enable ? (1u << VRM_NTIMER) - 1u : 0u); }

int vrm_timing_groups(vrm_ctx* c, uint32_t groups)
{
    if (!c) return vrm_fail(VRM_E_ARG, "context is NULL");
    groups &= (1u << VRM_NTIMER) - 1u;
    const int enable = groups != 0u;
    if (enable && !c->ev_start) {
        c->ev_start = new hipEvent_t[vrm::kMaxTimed];
        c->ev_stop = new hipEvent_t[vrm::kMaxTimed];
        c->ev_group = new int[vrm::kMaxTimed];
        // timing-only events: no system-scope fence (vrm_read_timing synchronises
        // the stream before reading them)
        for (int k = 0; k < vrm::kMaxTimed; ++k) {
            VRM_HIP(hipEventCreateWithFlags(&c->ev_start[k], hipEventDisableSystemFence));
            VRM_HIP(hipEventCreateWithFlags(&c->ev_stop[k], hipEventDisableSystemFence));
        }
    }
    if (c->graph_pending) {
        VRM_HIP(hipStreamSynchronize(c->stream));
        int r = collect_graph_timing(c);
        if (r) return r;
    }
    c->timing = enable ? 1 : 0;
    c->timing_groups = groups;
    c->ntimed = 0;
    for (int g = 0; g < VRM_NTIMER; ++g) {
        c->launches[g] = 0;
        c->acc_ms[g] = 0.0;
        c->acc_n[g] = 0;
    }
    return VRM_OK;
}

int vrm_read_timing(vrm_ctx* c, double* ms, int64_t* launches)
{
    if (!c) return vrm_fail(VRM_E_ARG, "context is NULL");
    VRM_HIP(hipStreamSynchronize(c->stream));
    int r = collect_graph_timing(c);
    if (r) return r;
    double acc[VRM_NTIMER] = {0};
    int64_t timed[VRM_NTIMER] = {0};
    for (int k = 0; k < c->ntimed; ++k) {
        float t = 0.0f;
        VRM_HIP(hipEventElapsedTime(&t, c->ev_start[k], c->ev_stop[k]));
        acc[c->ev_group[k]] += t;
        timed[c->ev_group[k]] += 1;
    }
    int over = 0;
    for (int g = 0; g < VRM_NTIMER; ++g) {
        if (ms) ms[g] = acc[g] + c->acc_ms[g];
        if (launches) launches[g] = c->launches[g];
        over |= timed[g] + c->acc_n[g] != c->launches[g];
        c->launches[g] = 0;
        c->acc_ms[g] = 0.0;
        c->acc_n[g] = 0;
    }
    c->ntimed = 0;
    return over ? 1 : VRM_OK;
}

int vrm_vortex_velocity(vrm_ctx* c, const vrm_cloud* cl, const float* vort_dev, int32_t n_vort, double nu, double t,
                        float* u_dev, float* v_dev)
{
    int r = check_cloud(c, cl);
    if (!r && (!u_dev || !v_dev || (n_vort > 0 && !vort_dev) || n_vort < 0))
        r = vrm_fail(VRM_E_ARG, "velocity arguments");
    if (!r && c->n_ptr != cl->n_dev) r = read_n(c, cl);
    if (r) return r;
    return vrm_velocity_run(c, cl, c->n, vort_dev, n_vort, nu, t, u_dev, v_dev);
}

int vrm_biot_savart(vrm_ctx* c, const vrm_cloud* cl, double eps, float* u_dev, float* v_dev)
{
    int r = check_cloud(c, cl);
    if (!r && (!u_dev || !v_dev)) r = vrm_fail(VRM_E_ARG, "u and v are required");
    if (!r && !(eps > 0.0)) r = vrm_fail(VRM_E_ARG, "eps must be positive (got %g)", eps);
    if (!r && c->n_ptr != cl->n_dev) r = read_n(c, cl);
    if (r) return r;
    return vrm_biot_savart_run(c, cl, c->n, eps, u_dev, v_dev);
}

int vrm_set_lp_objective(vrm_ctx* c, int mode)
{
    if (!c) return vrm_fail(VRM_E_ARG, "context is NULL");
    if (mode < 0 || mode > 2) return vrm_fail(VRM_E_ARG, "lp objective must be 0, 1 or 2 (got %d)", mode);
    if (mode == 2 && c->warm) return vrm_fail(VRM_E_STATE, "the least-squares objective has no warm start (warm mode %d)", c->warm);
    c->lp_objective = mode;
    return VRM_OK;
}

}  // extern "C"
