// Neighbourhoods, moment-condition LPs and the operator apply of libvrm.
//
// Kirchhart & Obi, Sec. 2 (eqs. neighbourhood, cond_two, cond_alpha, fii,
// momcondmv), Sec. 4.1 (dense simplex on V f = b, f >= 0), Sec. 4.2
// (segments), Sec. 4.3 (small neighbourhoods first, complete ones as a
// fallback), Sec. 3.4 eq. nsode (dGamma_i/dt = nu sum_j f_ji Gamma_j).
//
// Small-neighbourhood LPs (5 rows, 8 columns) keep their columns in
// registers; complete-neighbourhood LPs (up to 48 columns) keep them in LDS.
// Each LP is solved by one thread (vrm_simplex.h).  The fractions are
// scattered into sum_j fhat_ji Gamma_j with atomics.
#include <hip/hip_runtime.h>

#include "vrm_device.h"
#include "vrm_internal.h"
#include "vrm_simplex.h"

using namespace vrm;

namespace {

__device__ __forceinline__ int cell_of_pos(const GridState& g, float x, float y, int& cx, int& cy)
{
    float fx = (x - g.x0) * g.inv_cs;
    float fy = (y - g.y0) * g.inv_cs;
    fx = fminf(fmaxf(fx, 0.0f), (float)(g.nx - 1));
    fy = fminf(fmaxf(fy, 0.0f), (float)(g.ny - 1));
    cx = (int)fx;
    cy = (int)fy;
    return cy * g.nx + cx;
}

// wave-aggregated append of `want` (0/1) items; returns the slot or -1
__device__ __forceinline__ int wave_append(int* counter, bool want)
{
    uint64_t m = __ballot(want);
    int lane = lane_id();
    int before = __popcll(m & ((1ull << lane) - 1ull));
    int total = __popcll(m);
    int leader = total ? __ffsll((unsigned long long)m) - 1 : 0;
    int base = 0;
    if (total && lane == leader) base = atomicAdd(counter, total);
    base = __shfl(base, leader, VRM_WAVE);
    return want ? base + before : -1;
}

// ------------------------------------------------------------- kernels
// Small neighbourhoods (Sec. 4.3) of the diffused particles, in slot order.
__global__ __launch_bounds__(256) void k_small_nbhd(int n, const int32_t* __restrict__ perm,
                                                    const float* __restrict__ xs, const float* __restrict__ ys,
                                                    const int32_t* __restrict__ ids,
                                                    const int32_t* __restrict__ cell_start,
                                                    const uint8_t* __restrict__ diffused, const GridState* gs,
                                                    LaunchParams P, int32_t* __restrict__ small_slot,
                                                    int32_t* q_small, int32_t* q_full, Queues* qs,
                                                    int32_t* out_small_idx, int32_t* out_kfull, int want_kfull)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    bool active = t < n;
    int i = active ? perm[t] : 0;
    bool dif = active && diffused[i];
    int best[VRM_NSEG];
    float bd[VRM_NSEG];
    int kfull = 0;
    int ksmall = 0;
#pragma unroll
    for (int s = 0; s < VRM_NSEG; ++s) {
        best[s] = -1;
        bd[s] = INFINITY;
    }
    if (dif && (P.m <= VRM_NSEG || want_kfull)) {
        GridState g = *gs;
        float xi = xs[t], yi = ys[t];
        int cx, cy;
        cell_of_pos(g, xi, yi, cx, cy);
        for (int oy = -1; oy <= 1; ++oy) {
            int yy = cy + oy;
            if (yy < 0 || yy >= g.ny) continue;
            for (int ox = -1; ox <= 1; ++ox) {
                int xx = cx + ox;
                if (xx < 0 || xx >= g.nx) continue;
                int c = yy * g.nx + xx;
                int u0 = cell_start[c], u1 = cell_start[c + 1];
                for (int u = u0; u < u1; ++u) {
                    if (u == t) continue;
                    float dx = xs[u] - xi;
                    float dy = ys[u] - yi;
                    float d2 = d2_f32(dx, dy);
                    if (d2 < P.lo2) continue;
                    if (d2 <= P.hi2f) ++kfull;
                    if (d2 > P.hi2) continue;
                    int s = segment_f32(dx, dy);
                    float cur = 0.0f;
                    int cb = -1;
#pragma unroll
                    for (int k = 0; k < VRM_NSEG; ++k)
                        if (k == s) {
                            cur = bd[k];
                            cb = best[k];
                        }
                    bool take = d2 < cur || (d2 == cur && cb >= 0 && ids[u] < ids[cb]);
                    if (take) {
#pragma unroll
                        for (int k = 0; k < VRM_NSEG; ++k)
                            if (k == s) {
                                bd[k] = d2;
                                best[k] = u;
                            }
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < VRM_NSEG; ++s) ksmall += best[s] >= 0 ? 1 : 0;
    }
    if (active) {
        if (small_slot) {
#pragma unroll
            for (int s = 0; s < VRM_NSEG; ++s) small_slot[(size_t)t * VRM_NSEG + s] = best[s];
        }
        if (out_small_idx) {
#pragma unroll
            for (int s = 0; s < VRM_NSEG; ++s)
                out_small_idx[(size_t)i * VRM_NSEG + s] = best[s] >= 0 ? perm[best[s]] : -1;
        }
        if (out_kfull) out_kfull[i] = dif ? kfull : 0;
    }
    if (q_small) {
        bool small_ok = dif && P.m <= VRM_NSEG && ksmall >= P.m;
        int p1 = wave_append(&qs->n_small, small_ok);
        if (small_ok) q_small[p1] = t;
        bool full = dif && !small_ok;
        int p2 = wave_append(&qs->n_full, full);
        if (full) q_full[p2] = t;
    }
}

struct StencilOut {
    int32_t* small_idx;
    float* small_f;
    float* fii;
    uint8_t* status;
    int32_t* full_k;
    int32_t* full_idx;
    float* full_f;
};

__device__ __forceinline__ void count_add(int* p, bool v)
{
    uint64_t m = __ballot(v);
    if (m && lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(p, __popcll(m));
}

// Columns of a small-neighbourhood LP, in registers (column j = segment j).
struct RegCols8 {
    int k;
    uint64_t dead;
    float rx[8], ry[8], c[8], rxl[8], ryl[8], cl[8];
    __device__ __forceinline__ void get(int j, float& x, float& y, float& cc) const
    {
        x = 0.0f;
        y = 0.0f;
        cc = 0.0f;
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s == j) {
                x = rx[s];
                y = ry[s];
                cc = c[s];
            }
    }
    __device__ __forceinline__ void exact(int j, df& X, df& Y, df& C) const
    {
        X = Y = C = {0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s == j) {
                X = {rx[s], rxl[s]};
                Y = {ry[s], ryl[s]};
                C = {c[s], cl[s]};
            }
    }
};

// add 2^-10 rank(id) to a double-float cost (exact at these magnitudes)
__device__ __forceinline__ df add_rank(df C, int rank)
{
    df w = two_sum(C.hi, 0.0009765625f * (float)rank);
    w.lo += C.lo;
    return fast_two_sum(w.hi, w.lo);
}

// Small-neighbourhood LPs (5 rows, up to 8 columns), one thread per particle.
__global__ __launch_bounds__(256) void k_lp_small(const int32_t* __restrict__ perm, const float* __restrict__ xs,
                                                  const float* __restrict__ ys, const int32_t* __restrict__ ids,
                                                  const int32_t* __restrict__ small_slot,
                                                  const int32_t* __restrict__ q_small, Queues* qs,
                                                  int32_t* q_full, const float* __restrict__ gamma,
                                                  float* acc, LaunchParams P, StencilOut out, int apply,
                                                  vrm_counters* cnt)
{
    const int nitems = qs->n_small;
    const int stride = gridDim.x * blockDim.x;
    int loops = (nitems + stride - 1) / stride;
    for (int it = 0; it < loops; ++it) {
        int item = blockIdx.x * blockDim.x + threadIdx.x + it * stride;
        bool live = item < nitems;
        int st = 1, piv = 0, certified = 1;
        int t = 0, i = 0;
        if (live) {
            t = q_small[item];
            i = perm[t];
            const float xi = xs[t], yi = ys[t];
            RegCols8 cs;
            int us[8], idv[8];
            cs.k = 8;
            cs.dead = 0;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                int u = small_slot[(size_t)t * VRM_NSEG + s];
                us[s] = u;
                idv[s] = u >= 0 ? ids[u] : 0x7fffffff;
                if (u < 0) {
                    cs.dead |= 1ull << s;
                    cs.rx[s] = cs.ry[s] = cs.c[s] = cs.rxl[s] = cs.ryl[s] = cs.cl[s] = 0.0f;
                    continue;
                }
                df X, Y;
                exact_offset(xi, yi, xs[u], ys[u], P.scale2e, X, Y);
                cs.rx[s] = X.hi;
                cs.rxl[s] = X.lo;
                cs.ry[s] = Y.hi;
                cs.ryl[s] = Y.lo;
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (us[s] < 0) continue;
                int rank = 0;
#pragma unroll
                for (int o = 0; o < 8; ++o) rank += idv[o] < idv[s] ? 1 : 0;
                df C = add_rank(cost_df({cs.rx[s], cs.rxl[s]}, {cs.ry[s], cs.ryl[s]}, P), rank);
                cs.c[s] = C.hi;
                cs.cl[s] = C.lo;
            }
            float fv[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) fv[s] = 0.0f;
            float fii = 0.0f;
            auto store = [&](int j, float v) {
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    if (s == j) fv[s] = v;
            };
            st = solve_lp<5>(cs, P, store, fii, piv, certified);
            if (st == 0) {
                float g = gamma[i];
                if (apply) {
#pragma unroll
                    for (int s = 0; s < 8; ++s)
                        if (fv[s] != 0.0f) atomicAdd(&acc[perm[us[s]]], fv[s] * g);
                    atomicAdd(&acc[i], fii * g);
                }
                if (out.small_f) {
#pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        out.small_idx[(size_t)i * VRM_NSEG + s] = us[s] >= 0 ? perm[us[s]] : -1;
                        out.small_f[(size_t)i * VRM_NSEG + s] = fv[s];
                    }
                    out.fii[i] = fii;
                    out.status[i] = VRM_ST_SMALL;
                }
            }
        }
        bool ok = live && st == 0;
        if (piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        count_add(&cnt->n_small, ok);
        count_add(&cnt->n_uncertified, ok && !certified);
        if (apply) {
            uint64_t m = __ballot(ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
        bool fail = live && st != 0;
        int p = wave_append(&qs->n_full, fail);
        if (fail) q_full[p] = t;
    }
}

constexpr int kFullBlock = 64;

// Columns of a complete-neighbourhood LP, in LDS (column-major per thread).
struct LdsCols {
    int k;
    uint64_t dead;
    float* srx;       // [VRM_KMAX][kFullBlock]
    float* sry;
    float* sc;
    int* smeta;       // (slot << 6) | rank
    int tid;
    float xi, yi;
    const float* xs;
    const float* ys;
    const LaunchParams* P;
    __device__ __forceinline__ void get(int j, float& x, float& y, float& cc) const
    {
        x = srx[j * kFullBlock + tid];
        y = sry[j * kFullBlock + tid];
        cc = sc[j * kFullBlock + tid];
    }
    __device__ __forceinline__ void exact(int j, df& X, df& Y, df& C) const
    {
        int meta = smeta[j * kFullBlock + tid];
        int u = meta >> 6;
        exact_offset(xi, yi, xs[u], ys[u], P->scale2e, X, Y);
        C = add_rank(cost_df(X, Y, *P), meta & 63);
    }
};

__device__ __forceinline__ uint64_t member_key(float d2, int id)
{
    return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)id;
}

// Complete-neighbourhood LPs (Sec. 4.3 fallback), one thread per particle.
template <int M>
__global__ __launch_bounds__(kFullBlock) void k_lp_full(const int32_t* __restrict__ perm,
                                                        const float* __restrict__ xs, const float* __restrict__ ys,
                                                        const int32_t* __restrict__ ids,
                                                        const int32_t* __restrict__ cell_start, const GridState* gs,
                                                        const int32_t* __restrict__ q_full, const Queues* qs,
                                                        const float* __restrict__ gamma, float* acc, LaunchParams P,
                                                        StencilOut out, int apply, vrm_counters* cnt)
{
    __shared__ float s_rx[VRM_KMAX * kFullBlock];
    __shared__ float s_ry[VRM_KMAX * kFullBlock];
    __shared__ float s_c[VRM_KMAX * kFullBlock];
    __shared__ int s_meta[VRM_KMAX * kFullBlock];
    const int tid = threadIdx.x;
    const int nitems = qs->n_full;
    const int stride = gridDim.x * blockDim.x;
    const GridState g = *gs;
    int loops = (nitems + stride - 1) / stride;
    for (int it = 0; it < loops; ++it) {
        int item = blockIdx.x * blockDim.x + tid + it * stride;
        bool live = item < nitems;
        int st = 1, piv = 0, certified = 1, k = 0;
        bool truncated = false;
        if (live) {
            int t = q_full[item];
            int i = perm[t];
            const float xi = xs[t], yi = ys[t];
            int cx, cy;
            cell_of_pos(g, xi, yi, cx, cy);
            // members within R_full; if there are more than KMAX keep the KMAX nearest by (d2, id)
            int count = 0;
            for (int oy = -1; oy <= 1; ++oy) {
                int yy = cy + oy;
                if (yy < 0 || yy >= g.ny) continue;
                for (int ox = -1; ox <= 1; ++ox) {
                    int xx = cx + ox;
                    if (xx < 0 || xx >= g.nx) continue;
                    int c = yy * g.nx + xx;
                    for (int u = cell_start[c]; u < cell_start[c + 1]; ++u) {
                        if (u == t) continue;
                        float d2 = d2_f32(xs[u] - xi, ys[u] - yi);
                        if (d2 < P.lo2f || d2 > P.hi2f) continue;
                        if (count < VRM_KMAX) s_meta[count * kFullBlock + tid] = u;
                        ++count;
                    }
                }
            }
            uint64_t cut = ~0ull;
            if (count > VRM_KMAX) {
                truncated = true;
                // the VRM_KMAX-th smallest key, by bisection over the 64-bit keys
                uint64_t lo = 0, hi = ~0ull;
                while (lo < hi) {
                    uint64_t mid = lo + ((hi - lo) >> 1);
                    int below = 0;
                    for (int oy = -1; oy <= 1; ++oy) {
                        int yy = cy + oy;
                        if (yy < 0 || yy >= g.ny) continue;
                        for (int ox = -1; ox <= 1; ++ox) {
                            int xx = cx + ox;
                            if (xx < 0 || xx >= g.nx) continue;
                            int c = yy * g.nx + xx;
                            for (int u = cell_start[c]; u < cell_start[c + 1]; ++u) {
                                if (u == t) continue;
                                float d2 = d2_f32(xs[u] - xi, ys[u] - yi);
                                if (d2 < P.lo2f || d2 > P.hi2f) continue;
                                below += member_key(d2, ids[u]) <= mid ? 1 : 0;
                            }
                        }
                    }
                    if (below >= VRM_KMAX)
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                cut = lo;
                int kk = 0;
                for (int oy = -1; oy <= 1; ++oy) {
                    int yy = cy + oy;
                    if (yy < 0 || yy >= g.ny) continue;
                    for (int ox = -1; ox <= 1; ++ox) {
                        int xx = cx + ox;
                        if (xx < 0 || xx >= g.nx) continue;
                        int c = yy * g.nx + xx;
                        for (int u = cell_start[c]; u < cell_start[c + 1]; ++u) {
                            if (u == t) continue;
                            float d2 = d2_f32(xs[u] - xi, ys[u] - yi);
                            if (d2 < P.lo2f || d2 > P.hi2f) continue;
                            if (member_key(d2, ids[u]) <= cut && kk < VRM_KMAX) s_meta[kk++ * kFullBlock + tid] = u;
                        }
                    }
                }
                count = kk;
            }
            k = count;
            // columns: exact offsets, id ranks, costs
            for (int j = 0; j < k; ++j) {
                int u = s_meta[j * kFullBlock + tid];
                s_c[j * kFullBlock + tid] = __int_as_float(ids[u]);
            }
            for (int j = 0; j < k; ++j) {
                int u = s_meta[j * kFullBlock + tid];
                int idj = __float_as_int(s_c[j * kFullBlock + tid]);
                int rank = 0;
                for (int o = 0; o < k; ++o) rank += __float_as_int(s_c[o * kFullBlock + tid]) < idj ? 1 : 0;
                s_meta[j * kFullBlock + tid] = (u << 6) | rank;
            }
            for (int j = 0; j < k; ++j) {
                int meta = s_meta[j * kFullBlock + tid];
                df X, Y;
                exact_offset(xi, yi, xs[meta >> 6], ys[meta >> 6], P.scale2e, X, Y);
                df C = add_rank(cost_df(X, Y, P), meta & 63);
                s_rx[j * kFullBlock + tid] = X.hi;
                s_ry[j * kFullBlock + tid] = Y.hi;
                s_c[j * kFullBlock + tid] = C.hi;
            }
            LdsCols cs{k, 0ull, s_rx, s_ry, s_c, s_meta, tid, xi, yi, xs, ys, &P};
            float fii = 0.0f;
            const float g_i = gamma[i];
            int nz = 0;
            auto store = [&](int j, float v) {
                int u = s_meta[j * kFullBlock + tid] >> 6;
                int pj = perm[u];
                if (apply) atomicAdd(&acc[pj], v * g_i);
                if (out.full_idx) {
                    out.full_idx[(size_t)i * VRM_KMAX + nz] = pj;
                    out.full_f[(size_t)i * VRM_KMAX + nz] = v;
                }
                ++nz;
            };
            st = k > 0 ? solve_lp<M>(cs, P, store, fii, piv, certified) : 1;
            if (st == 0) {
                if (apply) atomicAdd(&acc[i], fii * g_i);
                if (out.full_k) {
                    out.full_k[i] = nz;
                    out.fii[i] = fii;
                    out.status[i] = VRM_ST_FULL;
                }
            } else if (out.status) {
                out.status[i] = VRM_ST_INFEASIBLE;
            }
        }
        bool ok = live && st == 0;
        if (piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        if (ok) atomicAdd((unsigned long long*)&cnt->full_cols, (unsigned long long)k);
        count_add(&cnt->n_full, ok);
        count_add(&cnt->n_infeasible, live && !ok);
        count_add(&cnt->n_uncertified, ok && !certified);
        count_add(&cnt->n_truncated, live && truncated);
        if (apply) {
            uint64_t m = __ballot(ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
    }
}

__global__ void k_status_init(int n, const uint8_t* __restrict__ diffused, StencilOut out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out.status[i] = diffused[i] ? VRM_ST_INFEASIBLE : VRM_ST_SKIPPED;
    out.fii[i] = 0.0f;
    if (out.full_k) out.full_k[i] = 0;
#pragma unroll
    for (int s = 0; s < VRM_NSEG; ++s) {
        out.small_idx[(size_t)i * VRM_NSEG + s] = -1;
        out.small_f[(size_t)i * VRM_NSEG + s] = 0.0f;
    }
    if (out.full_idx) {
        for (int s = 0; s < VRM_KMAX; ++s) {
            out.full_idx[(size_t)i * VRM_KMAX + s] = -1;
            out.full_f[(size_t)i * VRM_KMAX + s] = 0.0f;
        }
    }
}

__global__ void k_reset_queues(Queues* q)
{
    q->n_small = 0;
    q->n_full = 0;
}

// persistent launches: enough threads for every CU, each loops over its items
int lp_grid_small(int n) { return n > 0 ? min((n + 255) / 256, 256 * 8) : 1; }
int lp_grid_full(int n) { return n > 0 ? min((n + kFullBlock - 1) / kFullBlock, 256 * 4) : 1; }

}  // namespace

int vrm_small_nbhd_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const LaunchParams& lp, int32_t* small_idx,
                       int32_t* kfull)
{
    (void)cl;
    if (n <= 0) return VRM_OK;
    int nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_small_nbhd, dim3(nb), dim3(256), 0, c->stream, n, c->perm, c->xs, c->ys, c->ids,
                       c->cell_start, c->diffused, c->grid, lp, (int32_t*)nullptr, (int32_t*)nullptr,
                       (int32_t*)nullptr, c->queues, small_idx, kfull, kfull != nullptr ? 1 : 0);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_stencil_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const LaunchParams& lp, const vrm_stencils* st,
                    int apply)
{
    if (n <= 0) return VRM_OK;
    StencilOut out{};
    if (st) {
        out.small_idx = st->small_idx_dev;
        out.small_f = st->small_f_dev;
        out.fii = st->fii_dev;
        out.status = st->status_dev;
        out.full_k = st->full_k_dev;
        out.full_idx = st->full_idx_dev;
        out.full_f = st->full_f_dev;
        hipLaunchKernelGGL(k_status_init, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, c->diffused, out);
        VRM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(1), 0, c->stream, c->queues);
    int nb = (n + 255) / 256;
    {
        ScopedTimer tm(c, VRM_T_NBHD);
        hipLaunchKernelGGL(k_small_nbhd, dim3(nb), dim3(256), 0, c->stream, n, c->perm, c->xs, c->ys, c->ids,
                           c->cell_start, c->diffused, c->grid, lp, c->small_slot, c->q_small, c->q_full, c->queues,
                           (int32_t*)nullptr, (int32_t*)nullptr, 0);
    }
    VRM_HIP(hipGetLastError());
    if (lp.m == 5) {
        {
            ScopedTimer tm(c, VRM_T_LP_SMALL);
            hipLaunchKernelGGL(k_lp_small, dim3(lp_grid_small(n)), dim3(256), 0, c->stream, c->perm, c->xs, c->ys, c->ids,
                               c->small_slot, c->q_small, c->queues, c->q_full, cl->gamma_dev, c->acc, lp, out, apply,
                               c->counters);
        }
        VRM_HIP(hipGetLastError());
        ScopedTimer tm(c, VRM_T_LP_FULL);
        hipLaunchKernelGGL(k_lp_full<5>, dim3(lp_grid_full(n)), dim3(kFullBlock), 0, c->stream, c->perm, c->xs, c->ys, c->ids,
                           c->cell_start, c->grid, c->q_full, c->queues, cl->gamma_dev, c->acc, lp, out, apply,
                           c->counters);
    } else {
        ScopedTimer tm(c, VRM_T_LP_FULL);
        hipLaunchKernelGGL(k_lp_full<9>, dim3(lp_grid_full(n)), dim3(kFullBlock), 0, c->stream, c->perm, c->xs, c->ys, c->ids,
                           c->cell_start, c->grid, c->q_full, c->queues, cl->gamma_dev, c->acc, lp, out, apply,
                           c->counters);
    }
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}
