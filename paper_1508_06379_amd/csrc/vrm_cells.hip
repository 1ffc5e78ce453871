// Cell lists, reduced-operator selection and particle insertion of libvrm.
//
// Cell list: a counting sort of the particles into square cells of edge
// max(R, R_full) h (so a 3 x 3 block of cells covers every neighbourhood),
// over the bounding box found on the device.  Selection: Sec. 3.5, eq.
// reduced_bound, by a radix select on the bits of |Gamma| with FP64 bucket
// sums.  Insertion: Sec. 4.2, with conflicts between candidates resolved to
// the greedy result in (id, segment) order by rounds of the lexicographically
// first independent set.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstring>
#include <mutex>
#include <rocprim/device/device_radix_sort.hpp>

#include "vrm_device.h"
#include "vrm_internal.h"

using namespace vrm;

namespace {

constexpr int kScanBlocks = 512;

__global__ void k_grid_reset(GridState* g)
{
    g->bad &= ~kBadPos;
    g->bbox[0] = 0xffffffffu;
    g->bbox[1] = 0xffffffffu;
    g->bbox[2] = 0u;
    g->bbox[3] = 0u;
}

__global__ __launch_bounds__(256) void k_bbox(const float* __restrict__ x, const float* __restrict__ y, int n,
                                              const int32_t* __restrict__ n_dev, GridState* g)
{
    if (n_dev) n = *n_dev;
    uint32_t mnx = 0xffffffffu, mny = 0xffffffffu, mxx = 0u, mxy = 0u;
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float xv = x[i], yv = y[i];
        if (!(fabsf(xv) <= 3.4028235e38f) || !(fabsf(yv) <= 3.4028235e38f)) {
            bad = true;   // NaN or infinite: reported, never given a cell
            continue;
        }
        uint32_t kx = ordered_key(xv), ky = ordered_key(yv);
        mnx = min(mnx, kx);
        mny = min(mny, ky);
        mxx = max(mxx, kx);
        mxy = max(mxy, ky);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mnx = min(mnx, (uint32_t)__shfl_xor((int)mnx, o, VRM_WAVE));
        mny = min(mny, (uint32_t)__shfl_xor((int)mny, o, VRM_WAVE));
        mxx = max(mxx, (uint32_t)__shfl_xor((int)mxx, o, VRM_WAVE));
        mxy = max(mxy, (uint32_t)__shfl_xor((int)mxy, o, VRM_WAVE));
    }
    __shared__ uint32_t red[4][8];
    int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        red[0][w] = mnx;
        red[1][w] = mny;
        red[2][w] = mxx;
        red[3][w] = mxy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nw = blockDim.x >> 6;
        for (int k = 1; k < nw; ++k) {
            mnx = min(mnx, red[0][k]);
            mny = min(mny, red[1][k]);
            mxx = max(mxx, red[2][k]);
            mxy = max(mxy, red[3][k]);
        }
        atomicMin(&g->bbox[0], mnx);
        atomicMin(&g->bbox[1], mny);
        atomicMax(&g->bbox[2], mxx);
        atomicMax(&g->bbox[3], mxy);
    }
    if (__any(bad) && lane_id() == 0) atomicOr(&g->bad, kBadPos);
}

__global__ void k_grid_params(GridState* g, float cs, int ncell_cap, vrm_counters* cnt)
{
    float xmin = 0.0f, ymin = 0.0f, xmax = 0.0f, ymax = 0.0f;
    if (g->bbox[0] != 0xffffffffu) {
        xmin = ordered_key_inv(g->bbox[0]);
        ymin = ordered_key_inv(g->bbox[1]);
        xmax = ordered_key_inv(g->bbox[2]);
        ymax = ordered_key_inv(g->bbox[3]);
    }
    g->cs = cs;
    g->inv_cs = 1.0f / cs;
    g->x0 = xmin - cs;
    g->y0 = ymin - cs;
    double fx = ((double)xmax - (double)g->x0) * (double)g->inv_cs;
    double fy = ((double)ymax - (double)g->y0) * (double)g->inv_cs;
    long long nx = (long long)fmin(fx, 1.0e9) + 2;
    long long ny = (long long)fmin(fy, 1.0e9) + 2;
    int clamped = 0;
    if (nx * ny > ncell_cap) {
        // keep the aspect ratio; far particles share the edge cells (still exact, slower)
        double f = sqrt((double)ncell_cap / (double)(nx * ny));
        nx = nx * f > 1 ? (long long)(nx * f) : 1;
        ny = ncell_cap / nx;
        clamped = 1;
    }
    g->nx = (int)nx;
    g->ny = (int)ny;
    g->ncells = (int)(nx * ny);
    g->clamped = clamped;
    if (clamped) atomicAdd(&cnt->n_grid_clamped, 1);
}

__device__ __forceinline__ int cell_index(const GridState& g, float x, float y)
{
    float fx = (x - g.x0) * g.inv_cs;
    float fy = (y - g.y0) * g.inv_cs;
    fx = fminf(fmaxf(fx, 0.0f), (float)(g.nx - 1));
    fy = fminf(fmaxf(fy, 0.0f), (float)(g.ny - 1));
    return (int)fy * g.nx + (int)fx;
}

__global__ __launch_bounds__(256) void k_clear_cells(int32_t* start, const GridState* g)
{
    int nc = g->ncells + 1;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) start[c] = 0;
}

__global__ __launch_bounds__(256) void k_count(const float* __restrict__ x, const float* __restrict__ y, int n,
                                               const int32_t* __restrict__ n_dev, const GridState* gs, int32_t* start,
                                               int32_t* cell_of, int32_t* rank)
{
    if (n_dev) n = *n_dev;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    GridState g = *gs;
    if (g.bad & kBadPos) return;   // a non-finite position: no cell indices (the same for every thread)
    const int c = live ? cell_index(g, x[i], y[i]) : -1;
    if (live) cell_of[i] = c;
    // The rank only has to be unique within the cell.  The cloud is kept in cell
    // order, so the lanes of a wave share few cells: in up to eight rounds, the
    // lanes in the cell of the first lane still waiting take consecutive ranks
    // from one atomic; lanes left after that (an unsorted cloud) add alone.
    const int lane = lane_id();
    bool todo = live;
    int r = 0;
    for (int round = 0; round < 8; ++round) {
        const uint64_t act = __ballot(todo);
        if (!act) break;
        const int leader = __ffsll((unsigned long long)act) - 1;
        const int lc = __shfl(c, leader, 64);
        const bool mine = todo && c == lc;
        const uint64_t same = __ballot(mine);
        int base = 0;
        if (lane == leader) base = atomicAdd(&start[lc], __popcll(same));
        base = __shfl(base, leader, 64);
        if (mine) {
            r = base + __popcll(same & ((1ull << lane) - 1ull));
            todo = false;
        }
    }
    if (todo) r = atomicAdd(&start[c], 1);
    if (live) rank[i] = r;
}

// ----- three-kernel exclusive scan over start[0..ncells), total in start[ncells]
__device__ __forceinline__ int block_exclusive_scan(int v, int& total)
{
    __shared__ int wsum[8];
    int lane = lane_id(), w = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, VRM_WAVE);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int nw = blockDim.x >> 6;
    int off = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        int s = wsum[k];
        if (k < w) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

__global__ __launch_bounds__(256) void k_scan_partial(const int32_t* start, const GridState* g, int32_t* part)
{
    int nc = g->ncells;
    int chunk = (nc + kScanBlocks - 1) / kScanBlocks;
    int lo = blockIdx.x * chunk, hi = min(nc, lo + chunk);
    int s = 0;
    for (int c = lo + threadIdx.x; c < hi; c += blockDim.x) s += start[c];
    int tot;
    block_exclusive_scan(s, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlocks) void k_scan_top(int32_t* part)
{
    int v = part[threadIdx.x];
    int tot;
    int ex = block_exclusive_scan(v, tot);
    part[threadIdx.x] = ex;
    if (threadIdx.x == 0) part[kScanBlocks] = tot;
}

__global__ __launch_bounds__(256) void k_scan_final(int32_t* start, const GridState* g, const int32_t* part)
{
    int nc = g->ncells;
    int chunk = (nc + kScanBlocks - 1) / kScanBlocks;
    int lo = blockIdx.x * chunk, hi = min(nc, lo + chunk);
    int carry = part[blockIdx.x];
    for (int base = lo; base < hi; base += blockDim.x) {
        int c = base + threadIdx.x;
        int v = c < hi ? start[c] : 0;
        int tot;
        int ex = block_exclusive_scan(v, tot);
        if (c < hi) start[c] = carry + ex;
        carry += tot;
    }
    if (blockIdx.x == kScanBlocks - 1 && threadIdx.x == 0) start[nc] = part[kScanBlocks];
}

__global__ __launch_bounds__(256) void k_scatter(const float* __restrict__ x, const float* __restrict__ y,
                                                 const int32_t* __restrict__ id, int n,
                                                 const int32_t* __restrict__ n_dev,
                                                 const int32_t* __restrict__ start, const int32_t* __restrict__ cell_of,
                                                 const int32_t* __restrict__ rank, int32_t* perm, float* xs, float* ys,
                                                 int32_t* ids, const GridState* gs)
{
    if (n_dev) n = *n_dev;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (gs->bad & kBadPos)) return;
    int t = start[cell_of[i]] + rank[i];
    perm[t] = i;
    if (xs) {
        xs[t] = x[i];
        ys[t] = y[i];
        ids[t] = id[i];
    }
}

int scan_cells(vrm_ctx* c, int32_t* start)
{
    hipLaunchKernelGGL(k_scan_partial, dim3(kScanBlocks), dim3(256), 0, c->stream, start, c->grid, c->scan_part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlocks), 0, c->stream, c->scan_part);
    hipLaunchKernelGGL(k_scan_final, dim3(kScanBlocks), dim3(256), 0, c->stream, start, c->grid, c->scan_part);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

// ------------------------------------------------------ reduced operator
// Ranking key (Sec. 3.5): the bits of |Gamma| in FP32, monotone in the value
// for non-negative floats; particles with equal keys form one group, left out
// together.  Four 8-bit radix passes resolve the whole key.
__device__ __forceinline__ uint32_t selection_key(float a) { return __float_as_uint(a); }

// also zeroes the diffused count of every counter copy (k_sel_mask adds to it)
__global__ void k_sel_init(SelectState* s, vrm_counters* cnt, GridState* gs)
{
    int t = threadIdx.x;
    if (cnt && t < kCounterStripes)
        reinterpret_cast<vrm_counters*>(reinterpret_cast<char*>(cnt) + t * kCounterStride)->n_diffused = 0;
    if (t == 0) {
        s->norm1 = 0.0;
        s->bound = 0.0;
        s->prefix = 0.0;
        s->key_prefix = 0u;
        s->done = 0u;
        s->threshold = 0u;
        s->max_id = -1;
        gs->bad &= ~kBadGamma;
    }
    s->bin_sum[t] = 0.0;
    s->bin_cnt[t] = 0u;
}

// One radix pass.  A bin holds FP32 values that share at least the top seven
// bits of their exponent, i.e. values in [2^E, 2^(E+2)) that are multiples of
// 2^(E-23); up to 2^26 of them sum to below 2^(E+28), a multiple of 2^(E-23)
// with at most 51 significant bits, so every FP64 bin sum is exact and does
// not depend on the order of the atomics.  The first pass also finds non-finite
// circulations (kBadGamma) and the largest id.
__global__ __launch_bounds__(256) void k_sel_hist(const float* __restrict__ g, const int32_t* __restrict__ ids, int n,
                                                  SelectState* s, int shift, GridState* gs)
{
    __shared__ double h_sum[256];
    __shared__ uint32_t h_cnt[256];
    h_sum[threadIdx.x] = 0.0;
    h_cnt[threadIdx.x] = 0u;
    __syncthreads();
    bool bad = false;
    int mid = -1;
    if (!s->done) {
        uint32_t pre = s->key_prefix;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            float a = fabsf(g[i]);
            uint32_t key = selection_key(a);
            if (shift == 24) {
                bad = bad || key >= 0x7f800000u;
                if (ids) mid = max(mid, ids[i]);
            }
            if (shift < 24 && (key >> (shift + 8)) != (pre >> (shift + 8))) continue;
            int b = (key >> shift) & 255u;
            atomicAdd(&h_sum[b], (double)a);
            atomicAdd(&h_cnt[b], 1u);
        }
    }
    if (shift == 24) {
        for (int o = 32; o > 0; o >>= 1) mid = max(mid, __shfl_xor(mid, o, VRM_WAVE));
        if (lane_id() == 0 && mid >= 0) atomicMax(&s->max_id, mid);
        if (__any(bad) && lane_id() == 0) atomicOr(&gs->bad, kBadGamma);
    }
    __syncthreads();
    if (h_cnt[threadIdx.x]) {
        atomicAdd(&s->bin_sum[threadIdx.x], h_sum[threadIdx.x]);
        atomicAdd(&s->bin_cnt[threadIdx.x], h_cnt[threadIdx.x]);
    }
}

// Pick the bin where the cumulative sum first exceeds the bound (256 threads,
// one bin each; an FP64 block scan in bin order).
__global__ __launch_bounds__(256) void k_sel_pick(SelectState* s, int shift, double factor)
{
    __shared__ double wtot[4];
    __shared__ int first;
    const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
    double v = s->bin_sum[t];
    // inclusive scan of the bin sums (the same association in every run)
    double incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        double u = __shfl_up(incl, o, VRM_WAVE);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wtot[w] = incl;
    if (t == 0) first = 256;
    __syncthreads();
    double off = 0.0, total = 0.0;
    for (int k = 0; k < 4; ++k) {
        if (k < w) off += wtot[k];
        total += wtot[k];
    }
    incl += off;
    if (shift == 24) {
        if (t == 0) {
            s->norm1 = total;
            s->bound = factor * total;
            s->prefix = 0.0;
        }
    }
    __syncthreads();
    const bool done = s->done != 0u;
    const double bound = s->bound, prefix = s->prefix;
    if (!done && prefix + incl > bound) atomicMin(&first, t);
    __syncthreads();
    if (t == 0 && !done) {
        int b = first;
        if (b == 256) {
            // every particle in the current key range is left out
            uint64_t top = (uint64_t)s->key_prefix + ((uint64_t)256 << shift);
            s->threshold = top > 0xffffffffull ? 0xffffffffu : (uint32_t)top;
            s->done = top > 0xffffffffull ? 2u : 1u;
        } else {
            s->key_prefix |= (uint32_t)b << shift;
            if (shift == 0) {
                s->threshold = s->key_prefix;
                s->done = 1u;
            }
        }
    }
    // cumulative sum below the chosen bin (from its own scan) for the next pass
    if (!done && t == first && first < 256) s->prefix = prefix + incl - v;
    __syncthreads();
    s->bin_sum[t] = 0.0;
    s->bin_cnt[t] = 0u;
}

// Diffused: |Gamma| >= fl32(T (1 - 2^-16)), T the first key that does not fit:
// the particle that reaches the bound and every particle within a relative
// 2^-16 below it are diffused (circulations equal in exact arithmetic differ by
// round-off once computed: 2^-16 covers the stated 1e-5 per-value bound and the
// random-walk round-off of FP32 circulations over 10^2 SSP-RK3 steps).
constexpr float kTieBand = 0.9999847412109375f;   // 1 - 2^-16

__global__ __launch_bounds__(256) void k_sel_mask(const float* __restrict__ g, int n, const SelectState* s,
                                                  uint8_t* diffused, uint8_t* mask_out, vrm_counters* cnt)
{
    if (cnt) cnt = counter_stripe(cnt);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool d = false;
    const float band = __uint_as_float(s->threshold) * kTieBand;
    if (i < n) {
        d = s->done == 2u ? false : fabsf(g[i]) >= band;
        diffused[i] = d ? 1 : 0;
        if (mask_out) mask_out[i] = d ? 1 : 0;
    }
    uint64_t m = __ballot(d);
    if (cnt && lane_id() == 0 && m) atomicAdd(&cnt->n_diffused, __popcll(m));
}

// one thread per counter copy
// ------------------------------------------------------------ insertion
// Candidates: every empty segment of a diffused particle (slot order).
// L lanes per particle (aligned groups; L = 4 for clouds up to kCandCoopMaxN
// particles, where one lane per particle leaves the chip mostly idle and the
// chain of loads of one scan sets the time): the lanes scan interleaved
// candidates and OR their occupied segments; the group's lead lane appends.
constexpr int kCandCoopMaxN = 1 << 18;

template <int L>
__global__ __launch_bounds__(256) void k_candidates(int n, const int32_t* __restrict__ perm,
                                                    const float* __restrict__ xs, const float* __restrict__ ys,
                                                    const int32_t* __restrict__ ids,
                                                    const int32_t* __restrict__ cell_start,
                                                    const uint8_t* __restrict__ diffused, const GridState* gs,
                                                    LaunchParams P, Queues* qs, int cand_cap, float* cx, float* cy,
                                                    uint64_t* ckey, uint8_t* cstate)
{
    const int sub = threadIdx.x & (L - 1);
    const int t = blockIdx.x * (256 / L) + threadIdx.x / L;
    int occupied = 0xff;
    float xi = 0.0f, yi = 0.0f;
    if (t < n && !gs->bad && diffused[perm[t]]) {
        occupied = 0;
        GridState g = *gs;
        xi = xs[t];
        yi = ys[t];
        int c0 = cell_index(g, xi, yi);
        int cxi = c0 % g.nx, cyi = c0 / g.nx;
        for (int oy = -1; oy <= 1; ++oy) {
            int yy = cyi + oy;
            if (yy < 0 || yy >= g.ny) continue;
            {
                // the three cells of this row are contiguous in slot order
                int c0 = yy * g.nx + max(cxi - 1, 0), c1 = yy * g.nx + min(cxi + 1, g.nx - 1);
                int u0 = cell_start[c0], u1 = cell_start[c1 + 1];
                // positions read eight at a time: one memory latency per eight candidates
                for (int ub = u0 + sub; ub < u1; ub += 8 * L) {
                    float bx[8], by[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int v = min(ub + L * e, u1 - 1);   // past the end: a repeat, not visited
                        bx[e] = xs[v];
                        by[e] = ys[v];
                    }
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int u = ub + L * e;
                        if (u >= u1 || u == t) continue;
                        float dx = bx[e] - xi;
                        float dy = by[e] - yi;
                        float d2 = d2_f32(dx, dy);
                        if (d2 < P.lo2 || d2 > P.hi2) continue;
                        occupied |= 1 << segment_f32(dx, dy);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int o = 1; o < L; o <<= 1) occupied |= __shfl_xor(occupied, o, VRM_WAVE);
    __shared__ int s_app[17];
    int empty = (~occupied) & 0xff;
    int want = sub == 0 ? __popc(empty) : 0;
    int base = block_append_n(&qs->n_cand, want, s_app);
    if (want) {
        int id = ids[t];
        int k = 0;
        for (int s = 0; s < VRM_NSEG; ++s) {
            if (!(empty & (1 << s))) continue;
            int p = base + k++;
            if (p >= cand_cap) continue;
            float xc, yc;
            candidate_f32(xi, yi, P.rad, s, xc, yc);
            cx[p] = xc;
            cy[p] = yc;
            ckey[p] = ((uint64_t)(uint32_t)id << 3) | (uint64_t)s;
            cstate[p] = 0;
        }
    }
}

// One round of the lexicographically first independent set: a candidate is
// accepted once every conflicting candidate of smaller key is rejected, and
// rejected as soon as one of them is accepted.
__global__ __launch_bounds__(256) void k_mis_round(int nc, const float* __restrict__ cx, const float* __restrict__ cy,
                                                   const uint64_t* __restrict__ ckey, uint8_t* cstate,
                                                   const int32_t* __restrict__ cstart, const int32_t* __restrict__ cperm,
                                                   const GridState* gs, float ex2, Queues* qs)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    bool undecided = false;
    if (a < nc && cstate[a] == 0) {
        GridState g = *gs;
        float xa = cx[a], ya = cy[a];
        uint64_t ka = ckey[a];
        int c0 = cell_index(g, xa, ya);
        int cxa = c0 % g.nx, cya = c0 / g.nx;
        bool any_in = false, any_open = false;
        for (int oy = -1; oy <= 1 && !any_in; ++oy) {
            int yy = cya + oy;
            if (yy < 0 || yy >= g.ny) continue;
            for (int ox = -1; ox <= 1 && !any_in; ++ox) {
                int xx = cxa + ox;
                if (xx < 0 || xx >= g.nx) continue;
                int c = yy * g.nx + xx;
                for (int u = cstart[c]; u < cstart[c + 1]; ++u) {
                    int b = cperm[u];
                    if (b == a || ckey[b] >= ka) continue;
                    float dx = cx[b] - xa;
                    float dy = cy[b] - ya;
                    if (!(d2_f32(dx, dy) < ex2)) continue;
                    uint8_t sb = ((volatile const uint8_t*)cstate)[b];
                    if (sb == 1) {
                        any_in = true;
                        break;
                    }
                    if (sb == 0) any_open = true;
                }
            }
        }
        if (any_in)
            cstate[a] = 2;
        else if (!any_open)
            cstate[a] = 1;
        else
            undecided = true;
    }
    // a flag (the host only asks whether any candidate is left)
    if (undecided) qs->n_undecided = 1;
}

__global__ __launch_bounds__(256) void k_accepted(int nc, const uint64_t* __restrict__ ckey,
                                                  const uint8_t* __restrict__ cstate, Queues* qs, uint64_t* akey,
                                                  int32_t* aidx)
{
    __shared__ int s_app[17];
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    bool acc = a < nc && cstate[a] == 1;
    int p = block_append_n(&qs->n_accepted, acc ? 1 : 0, s_app);
    if (acc) {
        akey[p] = ckey[a];
        aidx[p] = a;
    }
}

// New particles get ids max_id + 1, max_id + 2, ... in key order (the largest
// id of the cloud is found by the selection's first pass), so ids stay unique
// after particles were removed.
__global__ __launch_bounds__(256) void k_append(int n0, int na, const int32_t* __restrict__ aidx_sorted,
                                                const float* __restrict__ cx, const float* __restrict__ cy, float* x,
                                                float* y, float* gamma, int32_t* id, uint8_t* diffused, int32_t* n_dev,
                                                const SelectState* sel)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *n_dev = n0 + na;
    if (r >= na) return;
    int a = aidx_sorted[r];
    x[n0 + r] = cx[a];
    y[n0 + r] = cy[a];
    gamma[n0 + r] = 0.0f;
    id[n0 + r] = sel->max_id + 1 + r;
    diffused[n0 + r] = 0;
}

// Few candidates: the whole conflict resolution in one workgroup.  The
// candidates are sorted by key (bitonic, in LDS) and decided greedily in that
// order, each against the accepted ones; this is the same set as the rounds of
// k_mis_round (the lexicographically first maximal independent set), and the
// accepted ones are appended in key order as after the radix sort.
constexpr int kInsSmallMax = 1024;

__global__ __launch_bounds__(1024) void k_insert_small(int n0, int capacity, int cand_cap,
                                                       const float* __restrict__ cx, const float* __restrict__ cy,
                                                       const uint64_t* __restrict__ ckey, float ex2, float* x, float* y,
                                                       float* gamma, int32_t* id, uint8_t* diffused, int32_t* n_dev,
                                                       Queues* qs, vrm_counters* cnt, const SelectState* sel)
{
    __shared__ uint64_t key[kInsSmallMax];
    __shared__ int32_t src[kInsSmallMax];
    __shared__ float sx[kInsSmallMax], sy[kInsSmallMax];
    __shared__ float ax[kInsSmallMax], ay[kInsSmallMax];
    __shared__ int32_t asrc[kInsSmallMax];
    __shared__ int32_t na_s;
    const int t = threadIdx.x;
    const int nc = qs->n_cand;
    if (nc > kInsSmallMax || nc > cand_cap) {
        if (t == 0) qs->small_state = 0;
        return;
    }
    int np = 1;
    while (np < nc) np <<= 1;
    if (t < np) {
        key[t] = t < nc ? ckey[t] : ~0ull;   // keys are distinct and below 2^35
        src[t] = t;
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            int p = t ^ j;
            if (t < np && p > t) {
                uint64_t a = key[t], b = key[p];
                bool up = (t & k) == 0;
                if ((a > b) == up) {
                    key[t] = b;
                    key[p] = a;
                    int v = src[t];
                    src[t] = src[p];
                    src[p] = v;
                }
            }
            __syncthreads();
        }
    }
    if (t < nc) {
        sx[t] = cx[src[t]];
        sy[t] = cy[src[t]];
    }
    __syncthreads();
    if (t < 64) {
        int na = 0;
        for (int r = 0; r < nc; ++r) {
            float xa = sx[r], ya = sy[r];
            bool conflict = false;
            for (int b = t; b < na; b += 64) {
                float dx = ax[b] - xa;
                float dy = ay[b] - ya;
                conflict |= d2_f32(dx, dy) < ex2;
            }
            if (!__any(conflict)) {
                if (t == 0) {
                    ax[na] = xa;
                    ay[na] = ya;
                    asrc[na] = src[r];
                }
                ++na;
                // the next candidate's lanes read what lane 0 wrote
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        if (t == 0) na_s = na;
    }
    __syncthreads();
    const int na = na_s;
    if (n0 + na > capacity) {
        if (t == 0) {
            qs->n_accepted = na;
            qs->small_state = 2;
            cnt->capacity_needed = n0 + na;
        }
        return;
    }
    const int id0 = sel->max_id + 1;
    for (int r = t; r < na; r += blockDim.x) {
        int a = asrc[r];
        x[n0 + r] = cx[a];
        y[n0 + r] = cy[a];
        gamma[n0 + r] = 0.0f;
        id[n0 + r] = id0 + r;
        diffused[n0 + r] = 0;
    }
    if (t == 0) {
        *n_dev = n0 + na;
        qs->n_accepted = na;
        qs->small_state = 1;
        cnt->n_candidates = nc;
        cnt->n_inserted = na;
        cnt->mis_rounds = 0;
        cnt->n = n0 + na;
    }
}

// ------------------------------------------------------------- reorder
__global__ __launch_bounds__(256) void k_gather_cloud(int n, const int32_t* __restrict__ perm,
                                                      const float* __restrict__ g, const uint8_t* __restrict__ dif,
                                                      float* tg, uint8_t* tdif)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int i = perm[t];
    tg[t] = g[i];
    tdif[t] = dif[i];
}

// the cloud in slot order; the permutation becomes the identity
__global__ __launch_bounds__(256) void k_copy_back(int n, const float* __restrict__ xs, const float* __restrict__ ys,
                                                   const int32_t* __restrict__ ids, const float* __restrict__ tg,
                                                   const uint8_t* __restrict__ tdif, float* x, float* y, int32_t* id,
                                                   float* g, uint8_t* dif, int32_t* perm)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    x[t] = xs[t];
    y[t] = ys[t];
    id[t] = ids[t];
    g[t] = tg[t];
    dif[t] = tdif[t];
    perm[t] = t;
}

__global__ void k_reset_insert(Queues* q)
{
    q->n_cand = 0;
    q->n_undecided = 0;
    q->n_accepted = 0;
    q->small_state = 0;
}
__global__ void k_reset_undecided(Queues* q) { q->n_undecided = 0; }

__global__ void k_insert_counters(const Queues* q, vrm_counters* cnt, int rounds, int n_after)
{
    cnt->n_candidates = q->n_cand;
    cnt->n_inserted = q->n_accepted;
    cnt->mis_rounds = rounds;
    cnt->n = n_after;
}

int blocks_for(int n) { return n > 0 ? (n + 255) / 256 : 1; }

// One thread copies the queue record to the host copy, then writes the
// sequence number with a system-scope release (after a system fence).
__global__ void k_publish_queues(const Queues* q, const GridState* g, HostQueues* h, int32_t seq)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        h->q = *q;
        h->q.nonfinite = g->bad;
        __threadfence_system();
        __hip_atomic_store(&h->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace

// The host spins on the sequence number; every 256 polls it asks the stream:
// an error ends the wait with that error, and a finished stream without the
// record is a state error (so a wait cannot outlast the stream's work).
int vrm_read_queues(vrm_ctx* c, Queues& q)
{
    const int32_t seq = ++c->q_seq;
    hipLaunchKernelGGL(k_publish_queues, dim3(1), dim3(64), 0, c->stream, c->queues, c->grid, c->q_host, seq);
    VRM_HIP(hipGetLastError());
    for (uint64_t k = 1;; ++k) {
        if (__atomic_load_n(&c->q_host->seq, __ATOMIC_ACQUIRE) == seq) break;
        if ((k & 255) == 0) {
            const hipError_t e = hipStreamQuery(c->stream);
            if (e == hipErrorNotReady) continue;
            VRM_HIP(e);
            if (__atomic_load_n(&c->q_host->seq, __ATOMIC_ACQUIRE) == seq) break;
            return vrm_fail(VRM_E_STATE, "queue record not published");
        }
    }
    std::memcpy(&q, const_cast<const Queues*>(&c->q_host->q), sizeof(Queues));
    return VRM_OK;
}

// Cell list of (x, y) into ctx->cell_start / perm / xs, ys, ids (slot order).
int vrm_build_cells(vrm_ctx* c, const float* x, const float* y, const int32_t* id, int32_t n, const LaunchParams& lp,
                    const int32_t* n_dev)
{
    ScopedTimer tm(c, VRM_T_CELLS);
    hipStream_t s = c->stream;
    hipLaunchKernelGGL(k_grid_reset, dim3(1), dim3(1), 0, s, c->grid);
    int nbb = min(256, blocks_for(n));
    hipLaunchKernelGGL(k_bbox, dim3(nbb), dim3(256), 0, s, x, y, n, n_dev, c->grid);
    float Rmax = (float)fmax((double)lp.hi2, (double)lp.hi2f);
    float cs = sqrtf(Rmax) * (1.0f + 1.0f / 1024.0f);
    hipLaunchKernelGGL(k_grid_params, dim3(1), dim3(1), 0, s, c->grid, cs, c->ncell_cap, c->counters);
    hipLaunchKernelGGL(k_clear_cells, dim3(1024), dim3(256), 0, s, c->cell_start, c->grid);
    if (n > 0) {
        hipLaunchKernelGGL(k_count, dim3(blocks_for(n)), dim3(256), 0, s, x, y, n, n_dev, c->grid, c->cell_start,
                           c->cell_of, c->rank);
    }
    VRM_HIP(hipGetLastError());
    int r = scan_cells(c, c->cell_start);
    if (r) return r;
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n)), dim3(256), 0, s, x, y, id, n, n_dev, c->cell_start,
                           c->cell_of, c->rank, c->perm, c->xs, c->ys, c->ids, c->grid);
    }
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_select_run(vrm_ctx* c, const float* gamma, const int32_t* ids, int32_t n, double factor)
{
    hipStream_t s = c->stream;
    static_assert(kCounterStripes <= 256, "k_sel_init zeroes one counter copy per thread");
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, c->sel, c->counters, c->grid);
    int nb = min(2048, blocks_for(n));
    for (int shift = 24; shift >= 0; shift -= 8) {
        if (n > 0) hipLaunchKernelGGL(k_sel_hist, dim3(nb), dim3(256), 0, s, gamma, ids, n, c->sel, shift, c->grid);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, c->sel, shift, factor);
    }
    if (n > 0)
        hipLaunchKernelGGL(k_sel_mask, dim3(blocks_for(n)), dim3(256), 0, s, gamma, n, c->sel, c->diffused,
                           (uint8_t*)nullptr, c->counters);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

// Insertion; the cell list of the cloud must be current.  Returns once the
// stream has run the work enqueued here (the host reads the queue record).
int vrm_insert_run(vrm_ctx* c, vrm_cloud* cl, int32_t n, const LaunchParams& lp)
{
    hipStream_t s = c->stream;
    const int cand_cap = 2 * c->capacity;
    hipLaunchKernelGGL(k_reset_insert, dim3(1), dim3(1), 0, s, c->queues);
    if (n > 0)
        hipLaunchKernelGGL(n <= kCandCoopMaxN ? k_candidates<4> : k_candidates<1>,
                           dim3(n <= kCandCoopMaxN ? (n + 63) / 64 : blocks_for(n)), dim3(256), 0, s, n, c->perm,
                           c->xs, c->ys, c->ids,
                           c->cell_start, c->diffused, c->grid, lp, c->queues, cand_cap, c->cx, c->cy, c->ckey,
                           c->cstate);
    if (n > 0)
        hipLaunchKernelGGL(k_insert_small, dim3(1), dim3(1024), 0, s, n, cl->capacity, cand_cap, c->cx, c->cy, c->ckey,
                           lp.ex2, cl->x_dev, cl->y_dev, cl->gamma_dev, cl->id_dev, c->diffused, cl->n_dev, c->queues,
                           c->counters, c->sel);
    VRM_HIP(hipGetLastError());
    Queues q;
    if (int r = vrm_read_queues(c, q)) return r;
    if (q.nonfinite) return vrm_nonfinite(c, q.nonfinite);
    if (q.small_state == 2)
        return vrm_fail(VRM_E_CAPACITY, "insertion needs %d particles, capacity is %d", n + q.n_accepted,
                        cl->capacity);
    if (q.small_state == 1) return n + q.n_accepted;
    int nc = q.n_cand;
    if (nc > cand_cap) return vrm_fail(VRM_E_CAPACITY, "insertion: %d candidates exceed the buffer of %d", nc, cand_cap);
    int rounds = 0;
    int na = 0;
    if (nc > 0) {
        // cell list of the candidates on the particles' grid
        hipLaunchKernelGGL(k_clear_cells, dim3(1024), dim3(256), 0, s, c->cstart, c->grid);
        hipLaunchKernelGGL(k_count, dim3(blocks_for(nc)), dim3(256), 0, s, c->cx, c->cy, nc, (const int32_t*)nullptr,
                           c->grid, c->cstart, c->ccell, c->crank);
        VRM_HIP(hipGetLastError());
        int r = scan_cells(c, c->cstart);
        if (r) return r;
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(nc)), dim3(256), 0, s, c->cx, c->cy, (const int32_t*)nullptr,
                           nc, (const int32_t*)nullptr, c->cstart, c->ccell, c->crank, c->cperm, (float*)nullptr,
                           (float*)nullptr, (int32_t*)nullptr, c->grid);
        VRM_HIP(hipGetLastError());
        for (;;) {
            const int batch = 4;
            for (int k = 0; k < batch; ++k) {
                hipLaunchKernelGGL(k_reset_undecided, dim3(1), dim3(1), 0, s, c->queues);
                hipLaunchKernelGGL(k_mis_round, dim3(blocks_for(nc)), dim3(256), 0, s, nc, c->cx, c->cy, c->ckey,
                                   c->cstate, c->cstart, c->cperm, c->grid, lp.ex2, c->queues);
            }
            rounds += batch;
            VRM_HIP(hipGetLastError());
            if (int e = vrm_read_queues(c, q)) return e;
            if (q.n_undecided == 0) break;
            if (rounds > 4 * nc + 64)
                return vrm_fail(VRM_E_STATE, "insertion: conflict resolution did not converge");
        }
        hipLaunchKernelGGL(k_accepted, dim3(blocks_for(nc)), dim3(256), 0, s, nc, c->ckey, c->cstate, c->queues,
                           c->akey, c->aidx);
        VRM_HIP(hipGetLastError());
        if (int e = vrm_read_queues(c, q)) return e;
        na = q.n_accepted;
        if (n + na > cl->capacity) {
            int need = n + na;
            hipMemcpyAsync(&c->counters->capacity_needed, &need, sizeof(int), hipMemcpyHostToDevice, s);
            hipStreamSynchronize(s);
            return vrm_fail(VRM_E_CAPACITY, "insertion needs %d particles, capacity is %d", n + na, cl->capacity);
        }
        if (na > 0) {
            // ids and append order follow the (id, segment) keys; sorted pairs go to the reorder scratch
            size_t bytes = c->sort_tmp_bytes;
            uint64_t* kin = c->akey;
            int32_t* vin = c->aidx;
            uint64_t* ksorted = reinterpret_cast<uint64_t*>(c->tmp_f);
            int32_t* vsorted = c->tmp_i;
            VRM_HIP(rocprim::radix_sort_pairs(c->sort_tmp, bytes, kin, ksorted, vin, vsorted, (size_t)na, 0, 35, s));
            hipLaunchKernelGGL(k_append, dim3(blocks_for(na)), dim3(256), 0, s, n, na, vsorted, c->cx, c->cy, cl->x_dev,
                               cl->y_dev, cl->gamma_dev, cl->id_dev, c->diffused, cl->n_dev, c->sel);
            VRM_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_insert_counters, dim3(1), dim3(1), 0, s, c->queues, c->counters, rounds, n + na);
    VRM_HIP(hipGetLastError());
    return n + na;
}

// Reorder the cloud by the current cell list (perm) and make perm the identity.
int vrm_reorder_cloud(vrm_ctx* c, vrm_cloud* cl, int32_t n)
{
    if (n <= 0) return VRM_OK;
    hipStream_t s = c->stream;
    // xs, ys, ids already hold x, y, id in slot order
    hipLaunchKernelGGL(k_gather_cloud, dim3(blocks_for(n)), dim3(256), 0, s, n, c->perm, cl->gamma_dev, c->diffused,
                       c->tmp_f, c->tmp_u8);
    VRM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_copy_back, dim3(blocks_for(n)), dim3(256), 0, s, n, c->xs, c->ys, c->ids, c->tmp_f, c->tmp_u8,
                       cl->x_dev, cl->y_dev, cl->id_dev, cl->gamma_dev, c->diffused, c->perm);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

size_t vrm_sort_tmp_bytes(int32_t cap)
{
    size_t bytes = 0;
    rocprim::radix_sort_pairs((void*)nullptr, bytes, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                              (int32_t*)nullptr, (size_t)cap, 0, 35, (hipStream_t)0);
    return bytes;
}

// ------------------------------------------------- allocation-free selection
// vrm_select_diffused_static: the selection kernels above with their state
// (histogram bins, threshold, the non-finite flag) in a fixed device array
// instead of a context's memory, for callers that cannot allocate.
namespace {
struct StaticSelect {
    SelectState sel;
    GridState grid;
};
constexpr size_t kStaticScratchBytes = 4096;
static_assert(sizeof(StaticSelect) <= kStaticScratchBytes, "static selection state exceeds its array");
constexpr int32_t kStaticMaxN = 1 << 26;   // exact FP64 bin sums (k_sel_hist)
constexpr int kStaticMaxDevices = 64;

__global__ void k_static_reset(GridState* g) { g->bad = 0; }
__global__ void k_static_report(const GridState* g, int32_t* out) { *out = g->bad; }
}  // namespace

// One copy per GPU, held until the process ends; in host code the name stands
// for the symbol, never for the device address (that is static_scratch_ptr's).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_static_mu;
void* g_static_ptr[kStaticMaxDevices];

// the device address of this GPU's copy of scratch (the current device's), looked
// up once per device
int static_scratch_ptr(int dev, void** out)
{
    if (dev < 0 || dev >= kStaticMaxDevices) return vrm_fail(VRM_E_ARG, "device %d outside [0, %d)", dev, kStaticMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* p = nullptr;
        VRM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return vrm_fail(VRM_E_HIP, "hipGetSymbolAddress(scratch) gave no address");
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return VRM_OK;
}
}  // namespace

extern "C" int vrm_select_diffused_static(const float* gamma_dev, int32_t n, double h, int32_t q, double c_diff,
                                          uint8_t* mask_dev, int32_t* nonfinite_dev, void* stream)
{
    if (!gamma_dev || !mask_dev) return vrm_fail(VRM_E_ARG, "gamma and mask are required");
    if (n < 0 || n > kStaticMaxN) return vrm_fail(VRM_E_ARG, "n = %d outside [0, 2^26] (the largest selection this entry point takes)", n);
    if (!(h > 0.0) || !std::isfinite(h)) return vrm_fail(VRM_E_ARG, "h must be positive and finite");
    if (q != 2 && q != 3) return vrm_fail(VRM_E_ARG, "q must be 2 or 3 (got %d)", q);
    if (!(c_diff >= 0.0) || !std::isfinite(c_diff)) return vrm_fail(VRM_E_ARG, "c_diff must be >= 0");
    int dev = 0;
    VRM_HIP(hipGetDevice(&dev));
    void* ptr = nullptr;
    if (int r = static_scratch_ptr(dev, &ptr)) return r;
    StaticSelect* st = static_cast<StaticSelect*>(ptr);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double factor = c_diff * std::pow(h, q + 1);
    hipLaunchKernelGGL(k_static_reset, dim3(1), dim3(1), 0, s, &st->grid);
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, &st->sel, (vrm_counters*)nullptr, &st->grid);
    const int nb = min(2048, blocks_for(n));
    for (int shift = 24; shift >= 0; shift -= 8) {
        if (n > 0)
            hipLaunchKernelGGL(k_sel_hist, dim3(nb), dim3(256), 0, s, gamma_dev, (const int32_t*)nullptr, n, &st->sel,
                               shift, &st->grid);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, &st->sel, shift, factor);
    }
    if (n > 0)
        hipLaunchKernelGGL(k_sel_mask, dim3(blocks_for(n)), dim3(256), 0, s, gamma_dev, n, &st->sel, mask_dev,
                           (uint8_t*)nullptr, (vrm_counters*)nullptr);
    if (nonfinite_dev) hipLaunchKernelGGL(k_static_report, dim3(1), dim3(1), 0, s, &st->grid, nonfinite_dev);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}
