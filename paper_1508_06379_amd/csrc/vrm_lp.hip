// Neighbourhoods, moment-condition LPs and the operator apply of libvrm.
//
// Kirchhart & Obi, Sec. 2 (eqs. neighbourhood, cond_two, cond_alpha, fii,
// momcondmv), Sec. 4.1 (dense simplex on V f = b, f >= 0), Sec. 4.2
// (segments), Sec. 4.3 (small neighbourhoods first, complete ones as a
// fallback), Sec. 3.4 eq. nsode (dGamma_i/dt = nu sum_j f_ji Gamma_j).
//
// Particle removal (Sec. 6, outlook) solves the identity operator's LP with
// the same machinery.
//
// Small-neighbourhood LPs (5 rows, 8 columns) keep their columns in
// registers; complete-neighbourhood LPs (up to 48 columns) keep them in LDS.
// Each LP is solved by one thread (vrm_simplex.h).  The fractions are
// scattered into sum_j fhat_ji Gamma_j with atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

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
// With queues: the LP queues, and the column record of each queued small LP.
__global__ __launch_bounds__(256) void k_small_nbhd(int n, const int32_t* __restrict__ n_dev,
                                                    const int32_t* __restrict__ perm,
                                                    const float* __restrict__ xs, const float* __restrict__ ys,
                                                    const int32_t* __restrict__ ids,
                                                    const int32_t* __restrict__ cell_start,
                                                    const uint8_t* __restrict__ diffused, const GridState* gs,
                                                    LaunchParams P, SmallRec rec, int32_t* q_small,
                                                    int32_t* q_full, Queues* qs,
                                                    int32_t* out_small_idx, int32_t* out_kfull, int want_kfull)
{
    // each thread's closest candidate per segment lives in LDS (indexed by the
    // segment: no register selects per candidate)
    __shared__ float s_bd[VRM_NSEG * 256];
    __shared__ int s_best[VRM_NSEG * 256];
    if (n_dev) n = *n_dev;
    const int tid = threadIdx.x;
    int t = blockIdx.x * blockDim.x + tid;
    bool active = t < n && !gs->bad;   // no cell list while a value is not finite
    int i = active ? perm[t] : 0;
    bool dif = active && diffused[i];
    int best[VRM_NSEG];
    int kfull = 0;
    int ksmall = 0;
#pragma unroll
    for (int s = 0; s < VRM_NSEG; ++s) {
        best[s] = -1;
        s_bd[s * 256 + tid] = INFINITY;
        s_best[s * 256 + tid] = -1;
    }
    if (dif && (P.m <= VRM_NSEG || want_kfull)) {
        GridState g = *gs;
        float xi = xs[t], yi = ys[t];
        int cx, cy;
        cell_of_pos(g, xi, yi, cx, cy);
        for (int oy = -1; oy <= 1; ++oy) {
            int yy = cy + oy;
            if (yy < 0 || yy >= g.ny) continue;
            {
                // the three cells of this row are contiguous in slot order
                int c0 = yy * g.nx + max(cx - 1, 0), c1 = yy * g.nx + min(cx + 1, g.nx - 1);
                int u0 = cell_start[c0], u1 = cell_start[c1 + 1];
                // positions read eight at a time: one memory latency per eight candidates
                for (int ub = u0; ub < u1; ub += 8) {
                    float bx[8], by[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int v = min(ub + e, u1 - 1);   // past the end: a repeat, not visited
                        bx[e] = xs[v];
                        by[e] = ys[v];
                    }
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int u = ub + e;
                        if (u >= u1 || u == t) continue;
                        float dx = bx[e] - xi;
                        float dy = by[e] - yi;
                        float d2 = d2_f32(dx, dy);
                        if (d2 < P.lo2) continue;
                        if (d2 <= P.hi2f) ++kfull;
                        if (d2 > P.hi2) continue;
                        const int at = segment_f32(dx, dy) * 256 + tid;
                        const float cur = s_bd[at];
                        if (d2 <= cur) {
                            bool take = d2 < cur;
                            if (!take) {
                                // equal distance: the smaller id wins
                                const int cb = s_best[at];
                                take = cb >= 0 && ids[u] < ids[cb];
                            }
                            if (take) {
                                s_bd[at] = d2;
                                s_best[at] = u;
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < VRM_NSEG; ++s) {
            best[s] = s_best[s * 256 + tid];
            ksmall += best[s] >= 0 ? 1 : 0;
        }
    }
    if (active) {
        if (out_small_idx) {
#pragma unroll
            for (int s = 0; s < VRM_NSEG; ++s)
                out_small_idx[(size_t)i * VRM_NSEG + s] = best[s] >= 0 ? perm[best[s]] : -1;
        }
        if (out_kfull) out_kfull[i] = dif ? kfull : 0;
    }
    if (q_small) {
        __shared__ int s_app[17];
        bool small_ok = dif && P.m <= VRM_NSEG && ksmall >= P.m;
        int p1 = block_append_n(&qs->n_small, small_ok ? 1 : 0, s_app);
        if (small_ok) {
            q_small[p1] = t;
            rec.i[p1] = i;
            const size_t cap = (size_t)rec.cap;
            const float xi = xs[t], yi = ys[t];
            int idb[VRM_NSEG];
#pragma unroll
            for (int s = 0; s < VRM_NSEG; ++s) idb[s] = best[s] >= 0 ? ids[best[s]] : 0x7fffffff;
            int packed = 0;
#pragma unroll
            for (int s = 0; s < VRM_NSEG; ++s) {
                int rank = 0;
#pragma unroll
                for (int o = 0; o < VRM_NSEG; ++o) rank += idb[o] < idb[s] ? 1 : 0;
                packed |= rank << (3 * s);
                const int u = best[s];
                df X{0.0f, 0.0f}, Y{0.0f, 0.0f};
                int pj = -1;
                if (u >= 0) {
                    exact_offset(xi, yi, xs[u], ys[u], P.scale2e, X, Y);
                    pj = perm[u];
                }
                rec.pj[s * cap + p1] = pj;
                rec.off[(4 * s + 0) * cap + p1] = X.hi;
                rec.off[(4 * s + 1) * cap + p1] = X.lo;
                rec.off[(4 * s + 2) * cap + p1] = Y.hi;
                rec.off[(4 * s + 3) * cap + p1] = Y.lo;
            }
            rec.rank[p1] = packed;
        }
        bool full = dif && !small_ok;
        int p2 = block_append_n(&qs->n_full, full ? 1 : 0, s_app);
        if (full) q_full[p2] = t;
    }
}

// Small neighbourhoods with kNbL lanes per particle (aligned lane groups), for
// clouds too small to fill the chip with one lane per particle, where the chain
// of loads of one particle's scan sets the time.  The lanes of a group scan
// interleaved candidates of the 3 x 3 cells, each keeps its closest candidate
// per segment (ties to the smaller id), and the group takes the minimum of
// (distance, id) per segment: the candidate the one-lane scan keeps, since that
// scan also keeps the lexicographic minimum.  Same outputs and queue records as
// k_small_nbhd; the lead lane of a group appends, the others write their share
// of the segments.
constexpr int kNbL = 4;
constexpr int kNbhdCoopMaxN = 1 << 16;

__global__ __launch_bounds__(256) void k_small_nbhd_coop(int n, const int32_t* __restrict__ n_dev,
                                                         const int32_t* __restrict__ perm,
                                                         const float* __restrict__ xs, const float* __restrict__ ys,
                                                         const int32_t* __restrict__ ids,
                                                         const int32_t* __restrict__ cell_start,
                                                         const uint8_t* __restrict__ diffused, const GridState* gs,
                                                         LaunchParams P, SmallRec rec, int32_t* q_small,
                                                         int32_t* q_full, Queues* qs,
                                                         int32_t* out_small_idx, int32_t* out_kfull, int want_kfull)
{
    __shared__ float s_bd[VRM_NSEG * 256];
    __shared__ int s_best[VRM_NSEG * 256];
    if (n_dev) n = *n_dev;
    const int tid = threadIdx.x, sub = tid & (kNbL - 1);
    const int t = blockIdx.x * (256 / kNbL) + tid / kNbL;
    const bool active = t < n && !gs->bad;   // no cell list while a value is not finite
    const int i = active ? perm[t] : 0;
    const bool dif = active && diffused[i];
    int kfull = 0;
#pragma unroll
    for (int s = 0; s < VRM_NSEG; ++s) {
        s_bd[s * 256 + tid] = INFINITY;
        s_best[s * 256 + tid] = -1;
    }
    if (dif && (P.m <= VRM_NSEG || want_kfull)) {
        GridState g = *gs;
        const float xi = xs[t], yi = ys[t];
        int cx, cy;
        cell_of_pos(g, xi, yi, cx, cy);
        for (int oy = -1; oy <= 1; ++oy) {
            const int yy = cy + oy;
            if (yy < 0 || yy >= g.ny) continue;
            const int c0 = yy * g.nx + max(cx - 1, 0), c1 = yy * g.nx + min(cx + 1, g.nx - 1);
            const int u0 = cell_start[c0], u1 = cell_start[c1 + 1];
            for (int ub = u0 + sub; ub < u1; ub += 8 * kNbL) {
                float bx[8], by[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int v = min(ub + kNbL * e, u1 - 1);
                    bx[e] = xs[v];
                    by[e] = ys[v];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int u = ub + kNbL * e;
                    if (u >= u1 || u == t) continue;
                    const float dx = bx[e] - xi, dy = by[e] - yi;
                    const float d2 = d2_f32(dx, dy);
                    if (d2 < P.lo2) continue;
                    if (d2 <= P.hi2f) ++kfull;
                    if (d2 > P.hi2) continue;
                    const int at = segment_f32(dx, dy) * 256 + tid;
                    const float cur = s_bd[at];
                    if (d2 <= cur) {
                        bool take = d2 < cur;
                        if (!take) {
                            const int cb = s_best[at];
                            take = cb >= 0 && ids[u] < ids[cb];
                        }
                        if (take) {
                            s_bd[at] = d2;
                            s_best[at] = u;
                        }
                    }
                }
            }
        }
    }
    // group minimum of (distance, id) per segment; empty = (inf, INT_MAX, -1)
    float bd[VRM_NSEG];
    int bu[VRM_NSEG], bid[VRM_NSEG];
#pragma unroll
    for (int s = 0; s < VRM_NSEG; ++s) {
        bd[s] = s_bd[s * 256 + tid];
        bu[s] = s_best[s * 256 + tid];
        bid[s] = bu[s] >= 0 ? ids[bu[s]] : 0x7fffffff;
    }
#pragma unroll
    for (int o = 1; o < kNbL; o <<= 1) {
        kfull += __shfl_xor(kfull, o, VRM_WAVE);
#pragma unroll
        for (int s = 0; s < VRM_NSEG; ++s) {
            const float od = __shfl_xor(bd[s], o, VRM_WAVE);
            const int ou = __shfl_xor(bu[s], o, VRM_WAVE), oid = __shfl_xor(bid[s], o, VRM_WAVE);
            if (od < bd[s] || (od == bd[s] && oid < bid[s])) {
                bd[s] = od;
                bu[s] = ou;
                bid[s] = oid;
            }
        }
    }
    int ksmall = 0;
#pragma unroll
    for (int s = 0; s < VRM_NSEG; ++s) ksmall += bu[s] >= 0 ? 1 : 0;
    const bool lead = sub == 0;
    if (active) {
        if (out_small_idx) {
#pragma unroll
            for (int s = 0; s < VRM_NSEG; ++s)
                if ((s & (kNbL - 1)) == sub) out_small_idx[(size_t)i * VRM_NSEG + s] = bu[s] >= 0 ? perm[bu[s]] : -1;
        }
        if (out_kfull && lead) out_kfull[i] = dif ? kfull : 0;
    }
    if (q_small) {
        __shared__ int s_app[17];
        const bool small_ok = dif && P.m <= VRM_NSEG && ksmall >= P.m;
        int p1 = block_append_n(&qs->n_small, small_ok && lead ? 1 : 0, s_app);
        p1 = __shfl(p1, lane_id() & ~(kNbL - 1), VRM_WAVE);
        if (small_ok) {
            const size_t cap = (size_t)rec.cap;
            const float xi = xs[t], yi = ys[t];
            if (lead) {
                int packed = 0;
#pragma unroll
                for (int s = 0; s < VRM_NSEG; ++s) {
                    int rank = 0;
#pragma unroll
                    for (int o = 0; o < VRM_NSEG; ++o) rank += bid[o] < bid[s] ? 1 : 0;
                    packed |= rank << (3 * s);
                }
                q_small[p1] = t;
                rec.i[p1] = i;
                rec.rank[p1] = packed;
            }
#pragma unroll
            for (int s = 0; s < VRM_NSEG; ++s) {
                if ((s & (kNbL - 1)) != sub) continue;
                const int u = bu[s];
                df X{0.0f, 0.0f}, Y{0.0f, 0.0f};
                int pj = -1;
                if (u >= 0) {
                    exact_offset(xi, yi, xs[u], ys[u], P.scale2e, X, Y);
                    pj = perm[u];
                }
                rec.pj[s * cap + p1] = pj;
                rec.off[(4 * s + 0) * cap + p1] = X.hi;
                rec.off[(4 * s + 1) * cap + p1] = X.lo;
                rec.off[(4 * s + 2) * cap + p1] = Y.hi;
                rec.off[(4 * s + 3) * cap + p1] = Y.lo;
            }
        }
        const bool full = dif && !small_ok;
        const int p2 = block_append_n(&qs->n_full, full && lead ? 1 : 0, s_app);
        if (full && lead) q_full[p2] = t;
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
    uint16_t* feat;      // feature rows of solved LPs (collection), or NULL
    float* lab;          // label rows (basis indicators, fractions) of solved LPs, or NULL
    int max_rows;
    const float* pred;   // warm start: small LPs 8 logits, complete ones kMlpOut outputs per queue item; or NULL
    int32_t* prev;       // basis (column ids) of each particle's last stencil, [id][kPrevIds]: recorded if non-NULL
    int prev_cap;        // rows of prev: particles with larger ids keep no basis (they start cold)
    int use_prev;        // warm start from prev instead of pred
    uint64_t* pmask;         // crash basis as a column mask per complete-neighbourhood queue item (size-binned path)
    uint8_t* pivhist;        // by particle id (< prev_cap): pivots of its last cold complete LP
    const int32_t* cloud_id;   // ids by cloud index
};

constexpr int kPrevIds = 9;

// the previous basis of particle `own` as a mask over columns with ids cid(j), j < k
template <class ColId>
__device__ __forceinline__ uint64_t prev_mask(const int32_t* prev, int own, int k, ColId cid)
{
    int pv[kPrevIds];
#pragma unroll
    for (int r = 0; r < kPrevIds; ++r) pv[r] = prev[(size_t)own * kPrevIds + r];
    uint64_t m = 0;
    for (int j = 0; j < k; ++j) {
        const int id = cid(j);
        if (id < 0) continue;
        bool in = false;
#pragma unroll
        for (int r = 0; r < kPrevIds; ++r) in = in || pv[r] == id;
        if (in) m |= 1ull << j;
    }
    return m;
}

// record the basic columns' ids as the particle's basis
template <class ColId>
__device__ __forceinline__ void record_basis(int32_t* prev, int own, uint64_t basis, ColId cid)
{
    int c = 0;
    while (basis && c < kPrevIds) {
        const int j = __ffsll((unsigned long long)basis) - 1;
        basis &= basis - 1;
        prev[(size_t)own * kPrevIds + c++] = cid(j);
    }
    for (; c < kPrevIds; ++c) prev[(size_t)own * kPrevIds + c] = -1;
}

__device__ __forceinline__ void count_add(int* p, bool v)
{
    uint64_t m = __ballot(v);
    if (m && lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(p, __popcll(m));
}
__device__ __forceinline__ void count_add(int64_t* p, bool v)
{
    uint64_t m = __ballot(v);
    if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
        atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__popcll(m));
}

// Tie-break of the canonical cost: 2^-10 rank(id); for the removal LP (q = 1)
// 2^-16 rank^2, convex in the rank because on a lattice the id ranks of
// opposite neighbours are symmetric and would tie under a linear weight.
// Exact in FP32 for ranks < 64.
__device__ __forceinline__ float tie_weight(unsigned rank, int q)
{
    return q == 1 ? 0x1p-16f * (float)(rank * rank) : 0.0009765625f * (float)rank;
}

// add the tie-break to a double-float cost (exact at these magnitudes)
__device__ __forceinline__ df add_rank(df C, int rank, int q)
{
    df w = two_sum(C.hi, tie_weight((unsigned)rank, q));
    w.lo += C.lo;
    return fast_two_sum(w.hi, w.lo);
}

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// feature row of an LP: slot j < 32 holds column j's offset / h, its mask, and q - 2
__device__ __forceinline__ void feature_zero(uint16_t* row)
{
#pragma unroll 4
    for (int a = 0; a < kMlpIn; ++a) row[a] = 0;
}
__device__ __forceinline__ void feature_slot(uint16_t* row, int j, float dxh, float dyh)
{
    row[2 * j] = f2bf(dxh);
    row[2 * j + 1] = f2bf(dyh);
    row[2 * kMlpSlots + j] = 0x3f80;   // 1.0
}
__device__ __forceinline__ void feature_q(uint16_t* row, int q) { row[3 * kMlpSlots] = q == 3 ? 0x3f80 : 0; }

__device__ __forceinline__ void count_warm(vrm_counters* cnt, bool live, int warm)
{
    uint64_t m1 = __ballot(live && warm == 1), m2 = __ballot(live && warm == 2), m3 = __ballot(live && warm == 3);
    if (lane_id() == 0) {
        if (m1) atomicAdd((unsigned long long*)&cnt->warm_hit, (unsigned long long)__popcll(m1));
        if (m2) atomicAdd((unsigned long long*)&cnt->warm_phase2, (unsigned long long)__popcll(m2));
        if (m3) atomicAdd((unsigned long long*)&cnt->warm_cold, (unsigned long long)__popcll(m3));
    }
}

constexpr int kFullBlock = 64;


// LP kernel passes: plain (cold start), warm (from the predicted basis; what
// it cannot settle cheaply goes to the retry queue), retry (cold start over
// the retry queue).  Splitting the passes keeps the cheap warm-started LPs
// from waiting for expensive cold ones in the same wave.
constexpr int kLpPlain = 0;
constexpr int kLpWarm = 1;
constexpr int kLpRetry = 2;

// Columns of an LP in LDS, column-major per thread (stride = threads per block):
// FP32 scaled offsets and cost, and (slot << 6) | id rank for the exact values.
// STORED: FP32 costs in sc, else computed from the offsets when read.
template <int BLK, bool STORED = true>
struct LdsColsT {
    static constexpr int KC = 0;   // column count known at run time only
    static constexpr bool kCoop = false;
    int k;
    uint64_t dead;
    float* srx;
    float* sry;
    float* sc;     // FP32 costs (STORED)
    int* smeta;
    int tid;
    float xi, yi;
    const float* xs;
    const float* ys;
    const LaunchParams* P;
    float* sxlo;   // low parts of the exact scaled offsets (hi parts are srx, sry), or NULL:
    float* sylo;   // then the exact offsets are recomputed from the positions
    static constexpr int kLds = 64;
    __device__ __forceinline__ int active() const { return k; }
    __device__ __forceinline__ bool widen() const { return false; }
    __device__ __forceinline__ void load_lds(int j, float& x, float& y, uint32_t& aux) const { load(j, x, y, aux); }
    __device__ __forceinline__ void get(int j, float& x, float& y, float& cc) const
    {
        x = srx[j * BLK + tid];
        y = sry[j * BLK + tid];
        if constexpr (STORED) {
            cc = sc[j * BLK + tid];
        } else {
            // FP32 cost from the FP32 offset (the exact cost is recomputed for certification)
            const float d2 = x * x + y * y;
            const float w = P->q == 1 ? d2 : P->q == 2 ? d2 * __builtin_sqrtf(d2) : d2 * d2;
            cc = __builtin_fmaf(w, P->cs_hi, tie_weight((unsigned)smeta[j * BLK + tid] & 63u, P->q));
        }
    }
    // Raw column values, for loops that read column j + 1 while working on
    // column j: the offsets, and the FP32 cost (STORED) or the meta word whose
    // rank bits cost_of needs.
    __device__ __forceinline__ void load(int j, float& x, float& y, uint32_t& aux) const
    {
        x = srx[j * BLK + tid];
        y = sry[j * BLK + tid];
        if constexpr (STORED)
            aux = __float_as_uint(sc[j * BLK + tid]);
        else
            aux = (uint32_t)smeta[j * BLK + tid];
    }
    // FP32 cost of a column from load()'s values, for moment order Q (the
    // value get() gives for P->q == Q)
    template <int Q>
    __device__ __forceinline__ float cost_of(float x, float y, uint32_t aux) const
    {
        if constexpr (STORED) {
            return __uint_as_float(aux);
        } else {
            const float d2 = x * x + y * y;
            const float w = Q == 1 ? d2 : Q == 2 ? d2 * __builtin_sqrtf(d2) : d2 * d2;
            return __builtin_fmaf(w, P->cs_hi, tie_weight(aux & 63u, Q));
        }
    }
    __device__ __forceinline__ void exact_xy(int j, df& X, df& Y) const
    {
        if (sxlo) {
            X = {srx[j * BLK + tid], sxlo[j * BLK + tid]};
            Y = {sry[j * BLK + tid], sylo[j * BLK + tid]};
        } else {
            int u = (int)((unsigned)smeta[j * BLK + tid] >> 6);
            exact_offset(xi, yi, xs[u], ys[u], P->scale2e, X, Y);
        }
    }
    __device__ __forceinline__ void exact(int j, df& X, df& Y, df& C) const
    {
        exact_xy(j, X, Y);
        C = add_rank(cost_df(X, Y, *P), smeta[j * BLK + tid] & 63, P->q);
    }
};

// Small-neighbourhood columns: eight, a compile-time count, plus their
// predicted logits in registers (warm pass).
template <int BLK>
struct SmallColsT : LdsColsT<BLK> {
    static constexpr int KC = VRM_NSEG;
    float lg[VRM_NSEG];
};

// Small-neighbourhood columns spread over an aligned group of eight lanes,
// one column (segment) per lane.  Every lane of the group runs the same
// simplex on replicated state; another lane's column is read with a lane
// permute, and reductions over the group use DPP within the 8 lanes.
struct CoopCols {
    static constexpr int KC = VRM_NSEG;
    static constexpr bool kCoop = true;
    int k;
    uint64_t dead;
    int own, base;                 // this lane's column; the group's first lane
    float x, y, c;                 // this lane's column: FP32 scaled offset, cost
    float xlo, ylo;                // low parts of the exact scaled offset
    int meta;                      // (slot << 6) | id rank
    const LaunchParams* P;
    float lg[VRM_NSEG];            // not used (no warm pass in this layout)
    mutable int cj;                // column whose values the last pick left in cx, cy, cc
    mutable float cx, cy, cc;

    __device__ __forceinline__ int active() const { return k; }
    __device__ __forceinline__ bool widen() const { return false; }
    __device__ __forceinline__ static float lane_f(float v, int src) { return __shfl(v, src, 64); }
    __device__ __forceinline__ static int lane_i(int v, int src) { return __shfl(v, src, 64); }
    __device__ __forceinline__ void get(int j, float& rx, float& ry, float& cost) const
    {
        if (j == cj) {
            rx = cx, ry = cy, cost = cc;
            return;
        }
        rx = lane_f(x, base + j);
        ry = lane_f(y, base + j);
        cost = lane_f(c, base + j);
    }
    __device__ __forceinline__ void exact_xy(int j, df& X, df& Y) const
    {
        X = {lane_f(x, base + j), lane_f(xlo, base + j)};
        Y = {lane_f(y, base + j), lane_f(ylo, base + j)};
    }
    __device__ __forceinline__ void exact(int j, df& X, df& Y, df& C) const
    {
        exact_xy(j, X, Y);
        C = add_rank(cost_df(X, Y, *P), lane_i(meta, base + j) & 63, P->q);
    }
    __device__ __forceinline__ void exact_own(df& X, df& Y, df& C) const
    {
        X = {x, xlo};
        Y = {y, ylo};
        C = add_rank(cost_df(X, Y, *P), meta & 63, P->q);
    }
    // value of the lane whose index differs by the DPP pattern: quad_perm
    // [1,0,3,2] (xor 1), [2,3,0,1] (xor 2), and the mirror within 8 lanes
    template <int CTRL>
    __device__ __forceinline__ static int dpp(int v)
    {
        return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
    }
    template <int CTRL>
    __device__ __forceinline__ static void pick_step(float& key, int& j, float& px, float& py, float& pc)
    {
        const float k2 = __int_as_float(dpp<CTRL>(__float_as_int(key)));
        const int j2 = dpp<CTRL>(j);
        const float x2 = __int_as_float(dpp<CTRL>(__float_as_int(px)));
        const float y2 = __int_as_float(dpp<CTRL>(__float_as_int(py)));
        const float c2 = __int_as_float(dpp<CTRL>(__float_as_int(pc)));
        const bool take = k2 < key || (k2 == key && j2 < j);
        key = take ? k2 : key;
        j = take ? j2 : j;
        px = take ? x2 : px;
        py = take ? y2 : py;
        pc = take ? c2 : pc;
    }
    __device__ __forceinline__ int pick(bool ok, float key) const
    {
        float k = ok ? key : __builtin_huge_valf();
        int j = ok ? own : 64;
        float px = x, py = y, pc = c;
        pick_step<0xB1>(k, j, px, py, pc);
        pick_step<0x4E>(k, j, px, py, pc);
        pick_step<0x141>(k, j, px, py, pc);
        cj = j < 64 ? j : -1;
        cx = px, cy = py, cc = pc;
        return cj;
    }
    __device__ __forceinline__ int first(bool ok) const
    {
        const uint64_t g = (__ballot(ok) >> base) & 0xFFull;
        return g ? __ffsll((unsigned long long)g) - 1 : -1;
    }
    __device__ __forceinline__ bool all(bool ok) const { return ((__ballot(!ok) >> base) & 0xFFull) == 0; }
};

// Small-neighbourhood LPs (5 rows, up to 8 columns), one thread per particle;
// the columns (column j = segment j) live in LDS.
constexpr int kSmallBlock = 256;

template <int OBJ>
__global__ __launch_bounds__(kSmallBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_lp_small(const int32_t* __restrict__ perm,
                                                          const float* __restrict__ xs, const float* __restrict__ ys,
                                                          const int32_t* __restrict__ ids, SmallRec rec,
                                                          const int32_t* __restrict__ q_small, Queues* qs,
                                                          int32_t* q_full, const float* __restrict__ gamma,
                                                          float* acc, LaunchParams P, StencilOut out, int apply,
                                                          vrm_counters* cnt, int mode, int32_t* q_retry, int lanes,
                                                          const GridState* gs)
{
    __shared__ float s_rx[8 * kSmallBlock];
    __shared__ float s_ry[8 * kSmallBlock];
    __shared__ float s_xlo[8 * kSmallBlock];
    __shared__ float s_ylo[8 * kSmallBlock];
    __shared__ float s_c[8 * kSmallBlock];
    __shared__ int s_meta[8 * kSmallBlock];
    cnt = counter_stripe(cnt);
    const int tid = threadIdx.x;
    const int nitems = mode == kLpRetry ? qs->n_retry : qs->n_small;
    const size_t cap = (size_t)rec.cap;
    // `lanes` LPs per wave (a power of two <= 64): fewer per wave shortens a wave,
    // which lasts as long as its slowest LP, where the launch has SIMDs to spare
    const int wave = (blockIdx.x * blockDim.x + tid) >> 6, lane = tid & 63;
    const int stride = ((gridDim.x * blockDim.x) >> 6) * lanes;
    const int loops = (nitems + stride - 1) / stride;
    const double dsc = P.det && apply ? det_scale(gs->gmax_bits) : 0.0;
    for (int it = 0; it < loops; ++it) {
        const int item = wave * lanes + lane + it * stride;
        const bool live = lane < lanes && item < nitems;
        int st = 1, piv = 0, certified = 1, warm = 0;
        int t = 0, i = 0, r = 0;
        if (live) {
            r = mode == kLpRetry ? q_retry[item] : item;   // the LP's column record
            t = q_small[r];
            i = rec.i[r];
            const int packed = rec.rank[r];
            uint64_t dead = 0;
            const bool record = mode == kLpPlain && out.feat && item < out.max_rows;
            uint16_t* frow = record ? out.feat + (size_t)item * kMlpIn : nullptr;
            if (record) feature_zero(frow);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int pj = rec.pj[s * cap + r];
                df X{rec.off[(4 * s + 0) * cap + r], rec.off[(4 * s + 1) * cap + r]};
                df Y{rec.off[(4 * s + 2) * cap + r], rec.off[(4 * s + 3) * cap + r]};
                float c = 0.0f;
                int meta = 0;
                if (pj >= 0) {
                    const int rank = (packed >> (3 * s)) & 7;
                    df C = add_rank(cost_df(X, Y, P), rank, P.q);
                    c = C.hi;
                    meta = (int)(((unsigned)pj << 6) | (unsigned)rank);
                    if (record) feature_slot(frow, s, X.hi * P.sc, Y.hi * P.sc);
                } else {
                    dead |= 1ull << s;
                }
                s_rx[s * kSmallBlock + tid] = X.hi;
                s_ry[s * kSmallBlock + tid] = Y.hi;
                s_xlo[s * kSmallBlock + tid] = X.lo;
                s_ylo[s * kSmallBlock + tid] = Y.lo;
                s_c[s * kSmallBlock + tid] = c;
                s_meta[s * kSmallBlock + tid] = meta;
            }
            if (record) feature_q(frow, P.q);
            SmallColsT<kSmallBlock> cs;
            static_cast<LdsColsT<kSmallBlock>&>(cs) = {8, dead, s_rx, s_ry, s_c, s_meta, tid, 0.0f, 0.0f, xs, ys, &P, s_xlo, s_ylo};
            float fv[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) fv[s] = 0.0f;
            float fii = 0.0f;
            auto store = [&](int j, float v) {
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    if (s == j) fv[s] = v;
            };
            const bool warm_pass = mode == kLpWarm && (out.pred || out.use_prev);
            const int own = ids[t];
            auto col_id = [&](int j) {
                return ((dead >> j) & 1ull) ? -1 : out.cloud_id[(unsigned)s_meta[j * kSmallBlock + tid] >> 6];
            };
            uint64_t pref = 0;
            if (warm_pass && out.use_prev) {
                pref = (unsigned)own < (unsigned)out.prev_cap ? prev_mask(out.prev, own, 8, col_id) : 0ull;
            } else if (warm_pass) {
                const float4* lg4 = reinterpret_cast<const float4*>(out.pred + (size_t)r * VRM_NSEG);
                const float4 a = lg4[0], b = lg4[1];
                cs.lg[0] = a.x, cs.lg[1] = a.y, cs.lg[2] = a.z, cs.lg[3] = a.w;
                cs.lg[4] = b.x, cs.lg[5] = b.y, cs.lg[6] = b.z, cs.lg[7] = b.w;
            }
            uint64_t basis = 0;
            st = solve_lp<5, OBJ>(cs, P, store, fii, piv, certified, warm_pass, nullptr, warm, basis,
                             warm_pass && out.use_prev, pref);
            if (st == 0 && out.prev && (unsigned)own < (unsigned)out.prev_cap) record_basis(out.prev, own, basis, col_id);
            if (record) {
                float* lab = out.lab + (size_t)item * kMlpOut;
#pragma unroll
                for (int s = 0; s < kMlpSlots; ++s) {
                    float v = s < 8 ? fv[s] : 0.0f;
                    lab[s] = (st == 0 && v > 0.0f) ? 1.0f : 0.0f;
                    lab[kMlpSlots + s] = st == 0 ? v : 0.0f;
                }
            }
            if (st == 0) {
                float g = gamma[i];
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    bool alive = !((dead >> s) & 1ull);
                    int pj = alive ? (int)((unsigned)s_meta[s * kSmallBlock + tid] >> 6) : -1;
                    if (apply && fv[s] != 0.0f) acc_add(acc, pj, fv[s], g, dsc);
                    if (out.small_f) {
                        out.small_idx[(size_t)i * VRM_NSEG + s] = pj;
                        out.small_f[(size_t)i * VRM_NSEG + s] = fv[s];
                    }
                }
                if (apply) acc_add(acc, i, fii, g, dsc);
                if (out.small_f) {
                    out.fii[i] = fii;
                    out.status[i] = (warm == 1 || warm == 2) ? VRM_ST_WARM : VRM_ST_SMALL;
                }
            }
        }
        bool ok = live && st == 0;
        if (piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        count_add(&cnt->n_small, ok);
        count_add(&cnt->n_uncertified, ok && !certified);
        count_warm(cnt, live, warm);
        if (apply) {
            uint64_t m = __ballot(ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
        bool fail = live && st == 1;
        int p = wave_append(&qs->n_full, fail);
        if (fail) q_full[p] = t;
        bool retry = live && st == 4;
        int pr = wave_append(&qs->n_retry, retry);
        if (retry) q_retry[pr] = r;
    }
}

// Small-neighbourhood LPs with eight lanes each (CoopCols): the same LPs, the
// same pivots and results as k_lp_small, in one eighth of its dependent chain
// per pivot (one column priced per lane).  Plain and phase-I passes only.
template <int OBJ>
__global__ __launch_bounds__(kSmallBlock) void k_lp_small_coop(const float* __restrict__ gamma,
                                                               SmallRec rec, const int32_t* __restrict__ q_small,
                                                               Queues* qs, int32_t* q_full, float* acc,
                                                               LaunchParams P, StencilOut out, int apply,
                                                               vrm_counters* cnt, const GridState* gs)
{
    cnt = counter_stripe(cnt);
    const double dsc = P.det && apply ? det_scale(gs->gmax_bits) : 0.0;
    const int lane = threadIdx.x & 63;
    const int s = lane & 7, base = lane & ~7;
    const bool lead = s == 0;
    const int nitems = qs->n_small;
    const size_t cap = (size_t)rec.cap;
    const int group = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int ngroups = (gridDim.x * blockDim.x) >> 3;
    const int loops = (nitems + ngroups - 1) / ngroups;
    for (int it = 0; it < loops; ++it) {
        const int item = group + it * ngroups;
        const bool live = item < nitems;   // the same for the eight lanes of a group
        int st = 1, piv = 0, certified = 1, t = 0;
        if (live) {
            t = q_small[item];
            const int i = rec.i[item];
            const int pj = rec.pj[s * cap + item];
            const bool alive = pj >= 0;
            df X{rec.off[(4 * s + 0) * cap + item], rec.off[(4 * s + 1) * cap + item]};
            df Y{rec.off[(4 * s + 2) * cap + item], rec.off[(4 * s + 3) * cap + item]};
            const int rank = (rec.rank[item] >> (3 * s)) & 7;
            CoopCols cs;
            cs.k = VRM_NSEG;
            cs.dead = (__ballot(!alive) >> base) & 0xFFull;
            cs.own = s;
            cs.base = base;
            cs.x = X.hi;
            cs.y = Y.hi;
            cs.xlo = X.lo;
            cs.ylo = Y.lo;
            cs.c = alive ? add_rank(cost_df(X, Y, P), rank, P.q).hi : 0.0f;
            cs.meta = alive ? (int)(((unsigned)pj << 6) | (unsigned)rank) : 0;
            cs.P = &P;
            cs.cj = -1;
            float fv = 0.0f, fii = 0.0f;
            auto store = [&](int j, float v) {
                if (j == s) fv = v;
            };
            int warm = 0;
            uint64_t basis = 0;
            st = solve_lp<5, OBJ>(cs, P, store, fii, piv, certified, false, nullptr, warm, basis, false, 0ull);
            if (st == 0) {
                const float g = gamma[i];
                if (apply && fv != 0.0f) acc_add(acc, pj, fv, g, dsc);
                if (apply && lead) acc_add(acc, i, fii, g, dsc);
                if (out.small_f) {
                    out.small_idx[(size_t)i * VRM_NSEG + s] = alive ? pj : -1;
                    out.small_f[(size_t)i * VRM_NSEG + s] = fv;
                    if (lead) {
                        out.fii[i] = fii;
                        out.status[i] = VRM_ST_SMALL;
                    }
                }
            }
        }
        const bool ok = live && lead && st == 0;
        if (lead && piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        count_add(&cnt->n_small, ok);
        count_add(&cnt->n_uncertified, ok && !certified);
        if (apply) {
            uint64_t m = __ballot(ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
        const bool fail = live && lead && st == 1;
        const int p = wave_append(&qs->n_full, fail);
        if (fail) q_full[p] = t;
    }
}

__device__ __forceinline__ uint64_t member_key(float d2, int id)
{
    return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)id;
}

// Complete neighbourhood of slot t within R_full (its VRM_KMAX nearest by (d2, id)
// if larger), sorted nearest first.  Slots go to su[j * kFullBlock], keys to
// sd2 / sid (same layout).  Returns the count.
// Visit every member of the complete neighbourhood of slot t (within R_full,
// not t itself): f(u, d2, id).  The three cells of a grid row are contiguous
// in slot order; their positions and ids are loaded eight at a time, so one
// memory latency covers eight candidates.
template <class F>
__device__ __forceinline__ void for_each_member(int t, float xi, float yi, int cx, int cy, const GridState& g,
                                                const int32_t* __restrict__ cell_start, const float* __restrict__ xs,
                                                const float* __restrict__ ys, const int32_t* __restrict__ ids,
                                                const LaunchParams& P, F&& f)
{
    for (int oy = -1; oy <= 1; ++oy) {
        const int yy = cy + oy;
        if (yy < 0 || yy >= g.ny) continue;
        const int c0 = yy * g.nx + max(cx - 1, 0), c1 = yy * g.nx + min(cx + 1, g.nx - 1);
        const int u0 = cell_start[c0], u1 = cell_start[c1 + 1];
        for (int u = u0; u < u1; u += 8) {
            float bx[8], by[8];
            int bi[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int v = min(u + e, u1 - 1);   // past the end: a repeat of the last slot, not visited
                bx[e] = xs[v];
                by[e] = ys[v];
                bi[e] = ids[v];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (u + e >= u1 || u + e == t) continue;
                const float d2 = d2_f32(bx[e] - xi, by[e] - yi);
                if (d2 < P.lo2f || d2 > P.hi2f) continue;
                f(u + e, d2, bi[e]);
            }
        }
    }
}

__device__ int collect_full(int t, float xi, float yi, const GridState& g, const int32_t* __restrict__ cell_start,
                            const float* __restrict__ xs, const float* __restrict__ ys,
                            const int32_t* __restrict__ ids, const LaunchParams& P, int* su, float* sd2, int* sid,
                            bool& truncated)
{
    int cx, cy;
    cell_of_pos(g, xi, yi, cx, cy);
    int count = 0;
    for_each_member(t, xi, yi, cx, cy, g, cell_start, xs, ys, ids, P, [&](int u, float d2, int id) {
        if (count < VRM_KMAX) {
            su[count * kFullBlock] = u;
            sd2[count * kFullBlock] = d2;
            sid[count * kFullBlock] = id;
        }
        ++count;
    });
    truncated = count > VRM_KMAX;
    if (truncated) {
        // the VRM_KMAX-th smallest key, by bisection over the 64-bit keys
        uint64_t lo = 0, hi = ~0ull;
        while (lo < hi) {
            const uint64_t mid = lo + ((hi - lo) >> 1);
            int below = 0;
            for_each_member(t, xi, yi, cx, cy, g, cell_start, xs, ys, ids, P,
                            [&](int, float d2, int id) { below += member_key(d2, id) <= mid ? 1 : 0; });
            if (below >= VRM_KMAX)
                hi = mid;
            else
                lo = mid + 1;
        }
        int kk = 0;
        for_each_member(t, xi, yi, cx, cy, g, cell_start, xs, ys, ids, P, [&](int u, float d2, int id) {
            if (member_key(d2, id) <= lo && kk < VRM_KMAX) {
                su[kk * kFullBlock] = u;
                sd2[kk * kFullBlock] = d2;
                sid[kk * kFullBlock] = id;
                ++kk;
            }
        });
        count = kk;
    }
    // insertion sort by (d2, id)
    for (int a = 1; a < count; ++a) {
        int u = su[a * kFullBlock];
        float d = sd2[a * kFullBlock];
        int id = sid[a * kFullBlock];
        int b = a - 1;
        while (b >= 0) {
            float db = sd2[b * kFullBlock];
            int ib = sid[b * kFullBlock];
            if (db < d || (db == d && ib < id)) break;
            su[(b + 1) * kFullBlock] = su[b * kFullBlock];
            sd2[(b + 1) * kFullBlock] = db;
            sid[(b + 1) * kFullBlock] = ib;
            --b;
        }
        su[(b + 1) * kFullBlock] = u;
        sd2[(b + 1) * kFullBlock] = d;
        sid[(b + 1) * kFullBlock] = id;
    }
    return count;
}

// Complete-neighbourhood LPs (Sec. 4.3 fallback), one thread per particle.
// SC: FP32 costs stored in LDS (48 KB per block: fewer instructions per
// pricing, three resident blocks per CU) or computed from the offsets when
// priced (36 KB: four blocks per CU).  Small clouds, whose launches are one
// wave's latency, take the first; large ones, throughput-bound, the second.
template <int M, bool SC, int OBJ, bool WARM>
__global__ __launch_bounds__(kFullBlock) void k_lp_full(const int32_t* __restrict__ perm,
                                                        const float* __restrict__ xs, const float* __restrict__ ys,
                                                        const int32_t* __restrict__ ids,
                                                        const int32_t* __restrict__ cell_start, const GridState* gs,
                                                        const int32_t* __restrict__ q_full, Queues* qs,
                                                        const float* __restrict__ gamma, float* acc, LaunchParams P,
                                                        StencilOut out, int apply, vrm_counters* cnt, int mode,
                                                        int32_t* q_retry, int last_launch)
{
    __shared__ float s_rx[VRM_KMAX * kFullBlock];
    __shared__ float s_ry[VRM_KMAX * kFullBlock];
    __shared__ int s_meta[VRM_KMAX * kFullBlock];
    __shared__ float s_c[SC ? VRM_KMAX * kFullBlock : 1];
    cnt = counter_stripe(cnt);
    const int tid = threadIdx.x;
    const int32_t* queue = mode == kLpRetry ? q_retry : q_full;
    const int nitems = mode == kLpRetry ? qs->n_retry : qs->n_full;
    const GridState g = *gs;
    const int stride = gridDim.x * blockDim.x;
    const int loops = (nitems + stride - 1) / stride;
    const double dsc = P.det && apply ? det_scale(g.gmax_bits) : 0.0;
    for (int it = 0; it < loops; ++it) {
        const int item = blockIdx.x * blockDim.x + tid + it * stride;
        const bool live = item < nitems;
        int st = 1, piv = 0, certified = 1, k = 0, warm = 0, t = 0;
        bool truncated = false;
        if (live) {
            t = queue[item];
            int i = perm[t];
            const float xi = xs[t], yi = ys[t];
            // columns nearest first: slots in s_meta, d2 in s_rx, ids in s_ry (as bits) during collection
            k = collect_full(t, xi, yi, g, cell_start, xs, ys, ids, P, s_meta + tid, s_rx + tid,
                             reinterpret_cast<int*>(s_ry) + tid, truncated);
            for (int j = 0; j < k; ++j) {
                int idj = __float_as_int(s_ry[j * kFullBlock + tid]);
                int rank = 0;
                for (int o = 0; o < k; ++o) rank += __float_as_int(s_ry[o * kFullBlock + tid]) < idj ? 1 : 0;
                s_meta[j * kFullBlock + tid] = (int)(((unsigned)s_meta[j * kFullBlock + tid] << 6) | (unsigned)rank);
            }
            const bool rec = mode == kLpPlain && out.feat && item < out.max_rows;
            uint16_t* frow = rec ? out.feat + (size_t)item * kMlpIn : nullptr;
            if (rec) feature_zero(frow);
            // exact offsets of the members, their positions loaded eight at a time
            for (int j0 = 0; j0 < k; j0 += 8) {
                int bm[8];
                float bx[8], by[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) bm[e] = s_meta[min(j0 + e, k - 1) * kFullBlock + tid];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int um = (int)((unsigned)bm[e] >> 6);
                    bx[e] = xs[um];
                    by[e] = ys[um];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int j = j0 + e;
                    if (j >= k) break;
                    df X, Y;
                    exact_offset(xi, yi, bx[e], by[e], P.scale2e, X, Y);
                    s_rx[j * kFullBlock + tid] = X.hi;
                    s_ry[j * kFullBlock + tid] = Y.hi;
                    if constexpr (SC) s_c[j * kFullBlock + tid] = add_rank(cost_df(X, Y, P), bm[e] & 63, P.q).hi;
                    if (rec && j < kMlpSlots) feature_slot(frow, j, X.hi * P.sc, Y.hi * P.sc);
                }
            }
            if (rec) feature_q(frow, P.q);
            LdsColsT<kFullBlock, SC> cs{k, 0ull, s_rx, s_ry, s_c, s_meta, tid, xi, yi, xs, ys, &P, nullptr, nullptr};
            float fii = 0.0f;
            const float g_i = gamma[i];
            int nz = 0;
            float* lab = rec ? out.lab + (size_t)item * kMlpOut : nullptr;
            if (lab)
                for (int a = 0; a < kMlpOut; ++a) lab[a] = 0.0f;
            auto store = [&](int j, float v) {
                int u = (int)((unsigned)s_meta[j * kFullBlock + tid] >> 6);
                int pj = perm[u];
                if (apply) acc_add(acc, pj, v, g_i, dsc);
                if (out.full_idx) {
                    out.full_idx[(size_t)i * VRM_KMAX + nz] = pj;
                    out.full_f[(size_t)i * VRM_KMAX + nz] = v;
                }
                if (lab && j < kMlpSlots) {
                    lab[j] = 1.0f;
                    lab[kMlpSlots + j] = v;
                }
                ++nz;
            };
            const bool warm_pass = mode == kLpWarm && (out.pred || out.use_prev);
            const float* logit = (warm_pass && !out.use_prev) ? out.pred + (size_t)item * kMlpOut : nullptr;
            const int own = ids[t];
            auto col_id = [&](int j) { return ids[(unsigned)s_meta[j * kFullBlock + tid] >> 6]; };
            const uint64_t pref = (warm_pass && out.use_prev && (unsigned)own < (unsigned)out.prev_cap)
                                      ? prev_mask(out.prev, own, k, col_id)
                                      : 0ull;
            uint64_t basis = 0;
            st = k > 0 ? solve_lp<M, OBJ, WARM>(cs, P, store, fii, piv, certified, warm_pass, logit, warm, basis,
                                     warm_pass && out.use_prev, pref)
                       : 1;
            if (st == 0 && out.prev && (unsigned)own < (unsigned)out.prev_cap) record_basis(out.prev, own, basis, col_id);
            if (st == 0) {
                if (apply) acc_add(acc, i, fii, g_i, dsc);
                if (out.full_k) {
                    out.full_k[i] = nz;
                    out.fii[i] = fii;
                    out.status[i] = (warm == 1 || warm == 2) ? VRM_ST_WARM : VRM_ST_FULL;
                }
            } else if (st == 1) {
                if (out.status) out.status[i] = VRM_ST_INFEASIBLE;
                if (lab)
                    for (int a = 0; a < kMlpOut; ++a) lab[a] = 0.0f;
            }
        }
        bool ok = live && st == 0;
        if (piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        if (ok) atomicAdd((unsigned long long*)&cnt->full_cols, (unsigned long long)k);
        count_add(&cnt->n_full, ok);
        count_add(&cnt->n_infeasible, live && st == 1);
        count_add(&cnt->n_uncertified, ok && !certified);
        count_add(&cnt->n_truncated, live && truncated);
        count_warm(cnt, live, warm);
        if (apply) {
            uint64_t m = __ballot(ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
        bool retry = live && st == 4;
        int pr = wave_append(&qs->n_retry, retry);
        if (retry) q_retry[pr] = t;
    }
    if (last_launch) {
        // the last LP launch of a stencil run: its last block to finish empties the
        // queues for the next run (keeping the counts for the host)
        __shared__ int last;
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) last = atomicAdd(&qs->blocks_done, 1) == (int)gridDim.x - 1;
        __syncthreads();
        if (last && threadIdx.x == 0) {
            __threadfence();
            qs->last_small = qs->n_small;
            qs->last_full = qs->n_full;
            qs->n_small = 0;
            qs->n_full = 0;
            qs->n_retry = 0;
            qs->n_defer = 0;
            qs->blocks_done = 0;
        }
    }
}

// ------------------------------------------------ complete LPs, size-binned
// The complete-neighbourhood LPs of q = 3 (9 rows, k = 9..48 columns) in three
// launches: the column lists (k_full_collect: every member within R_full h,
// the VRM_KMAX nearest by (d2, id), nearest first, with their id ranks) go to
// HBM with a histogram of k; a counting sort orders the LPs by decreasing k
// (k_full_bin_starts, k_full_bin_scatter), so the 64 lanes of a wave solve LPs
// of similar size; k_lp_sift solves them with the nearest kSiftW columns in LDS
// as the working set (Sec. 4.3: the closer particles carry the stencil; the
// canonical cost grows like |r|^4), pricing the others from HBM only once the
// working set is exhausted -- the optimum is certified over all k columns.
constexpr int kSiftW = 24;
constexpr int kDeferMinN = 1 << 20;   // particles from which a cold LP launch defers certifications
constexpr int kKBins = VRM_KMAX + 1;
// a record row: (slot << 6) | id rank per column, nearest first
constexpr int kRecRow = VRM_KMAX;

// Column lists with kCollL lanes per LP (aligned lane groups, four LPs per
// wave): the lanes scan interleaved candidates of the three rows of cells and
// append the members (within R_full h) to the group's list in LDS; then every
// lane places its members at once: position = number of members with a
// smaller (d2, id), id rank = number with a smaller id (among the VRM_KMAX
// nearest if there are more).  No sort, no rescans; a list longer than
// kMemCap (rare: an LP keeps at most VRM_KMAX = 48 columns) goes to the retry queue and
// is solved by the one-thread kernel, which collects on its own.
// The previous-basis warm start (WM 2) takes its input here as well: the
// columns whose ids form the particle's previous basis, as a mask per LP
// (pmask).  The network's inputs are read from the records by its inference.
constexpr int kCollL = 16;
constexpr int kMemCap = 64;
constexpr int kCollBlock = 256;
constexpr int kCollGroups = kCollBlock / kCollL;
constexpr int kMemPerLane = kMemCap / kCollL;
// A member is one 64-bit key, the bits of its d2 (a non-negative float, whose
// bits order as the values do) over its id, so one unsigned comparison orders
// (d2, id).  LDS row stride of a group's keys: a multiple of four (16-byte
// reads of two keys) whose remainder mod 32 banks (as 32-bit words) puts the
// four groups of a wave in different banks when they read the same member.
constexpr int kMemStride = kMemCap + 4;
static_assert(kMemCap % 4 == 0 && kMemStride % 4 == 0, "lists are read four members at a time");

// Eight waves per SIMD (64 VGPRs; the LDS of 17.6 KB per block allows nine):
// the scan waits on its loads, and more resident waves hide that.
template <int WM>
__global__ __launch_bounds__(kCollBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_full_collect(const float* __restrict__ xs,
                                                             const float* __restrict__ ys,
                                                             const int32_t* __restrict__ ids,
                                                             const int32_t* __restrict__ cell_start,
                                                             const GridState* gs, const int32_t* __restrict__ q_full,
                                                             Queues* qs, LaunchParams P, int32_t* rec, int32_t* kcol,
                                                             int32_t* khist, int32_t* q_retry, vrm_counters* cnt,
                                                             const int32_t* __restrict__ prev, int prev_cap,
                                                             uint64_t* pmask, const uint8_t* __restrict__ pivhist,
                                                             int32_t* key)
{
    static_assert(WM == 0 || WM == 2, "cold or previous-basis column lists");
    __shared__ __attribute__((aligned(16))) uint64_t s_key[kCollGroups][kMemStride];
    __shared__ int s_u[kCollGroups][kMemStride];
    __shared__ int s_pos[kCollGroups][kMemStride];
    __shared__ int s_hist[kKBins];
    cnt = counter_stripe(cnt);
    const int tid = threadIdx.x, sub = tid & (kCollL - 1), grp = tid / kCollL;
    const int lane = lane_id(), gbase = lane & ~(kCollL - 1);
    for (int b = tid; b < kKBins; b += blockDim.x) s_hist[b] = 0;
    __syncthreads();
    const int nitems = qs->n_full;
    const GridState g = *gs;
    const int ngroups = gridDim.x * kCollGroups;
    const int loops = (nitems + ngroups - 1) / ngroups;
    for (int it = 0; it < loops; ++it) {
        const int r = blockIdx.x * kCollGroups + grp + it * ngroups;
        const bool live = r < nitems;   // the same for the lanes of a group
        int t = 0, cx = 0, cy = 0;
        float xi = 0.0f, yi = 0.0f;
        if (live) {
            t = q_full[r];
            xi = xs[t];
            yi = ys[t];
            cell_of_pos(g, xi, yi, cx, cy);
        }
        int count = 0;
        for (int oy = -1; oy <= 1; ++oy) {
            const int yy = cy + oy;
            int u0 = 0, u1 = 0;
            if (live && yy >= 0 && yy < g.ny) {
                u0 = cell_start[yy * g.nx + max(cx - 1, 0)];
                u1 = cell_start[yy * g.nx + min(cx + 1, g.nx - 1) + 1];
            }
            for (int ub = u0;; ub += kCollL) {
                const bool act = ub < u1;   // group-uniform
                if (!__any(act)) break;
                const int u = ub + sub;
                bool mem = false;
                float d2 = 0.0f;
                if (act && u < u1 && u != t) {
                    d2 = d2_f32(xs[u] - xi, ys[u] - yi);
                    mem = !(d2 < P.lo2f) && !(d2 > P.hi2f);
                }
                const uint32_t m = (uint32_t)(__ballot(mem) >> gbase) & 0xFFFFu;
                if (mem) {
                    const int at = count + __popc(m & ((1u << sub) - 1u));
                    if (at < kMemCap) {
                        s_key[grp][at] = member_key(d2, ids[u]);
                        s_u[grp][at] = u;
                    }
                }
                count += __popc(m);
            }
        }
        const bool over = live && count > kMemCap;
        const int nm = over ? 0 : count;
        // up to three sentinels after the list (never nearer, never a lower id),
        // so the rank loop reads whole groups of four
        const int nm4 = (nm + 3) & ~3;
        if (nm + sub < nm4) {
            s_key[grp][nm + sub] = member_key(__builtin_inff(), 0x7fffffff);
        }
        // the group's appends are read by its other lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // members per lane that any group of the wave has (wave-uniform, so the
        // unused ones of the kMemPerLane are skipped by a scalar branch)
        int nqw = 0;
#pragma unroll
        for (int q = 0; q < kMemPerLane; ++q) nqw += __ballot(nm > kCollL * q) ? 1 : 0;
        // this lane's members: e = sub + kCollL q
        uint64_t mk[kMemPerLane];
        int mi[kMemPerLane], pos[kMemPerLane], rk[kMemPerLane];
#pragma unroll
        for (int q = 0; q < kMemPerLane; ++q) {
            const int e = sub + kCollL * q;
            mk[q] = q < nqw && e < nm ? s_key[grp][e] : 0ull;
            mi[q] = (int)(uint32_t)mk[q];
            pos[q] = 0;
            rk[q] = 0;
        }
        for (int o = 0; o < nm4; o += 4) {
            const ulonglong2 ka = *reinterpret_cast<const ulonglong2*>(&s_key[grp][o]);
            const ulonglong2 kb = *reinterpret_cast<const ulonglong2*>(&s_key[grp][o + 2]);
            const uint64_t kk[4] = {ka.x, ka.y, kb.x, kb.y};
#pragma unroll
            for (int q = 0; q < kMemPerLane; ++q) {
                if (q < nqw) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        pos[q] += kk[w] < mk[q] ? 1 : 0;
                        rk[q] += (uint32_t)kk[w] < (uint32_t)mi[q] ? 1 : 0;
                    }
                }
            }
        }
        const int k = min(nm, VRM_KMAX);
        if (nm > VRM_KMAX) {
            // ranks among the VRM_KMAX nearest only
#pragma unroll
            for (int q = 0; q < kMemPerLane; ++q)
                if (sub + kCollL * q < nm) s_pos[grp][sub + kCollL * q] = pos[q];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int q = 0; q < kMemPerLane; ++q) rk[q] = 0;
            for (int o = 0; o < nm; ++o) {
                const int id = (int)(uint32_t)s_key[grp][o];
                const bool kept = s_pos[grp][o] < VRM_KMAX;
#pragma unroll
                for (int q = 0; q < kMemPerLane; ++q) rk[q] += (kept && id < mi[q]) ? 1 : 0;
            }
        }
        if constexpr (WM == 2) {
            // the previous basis as a column mask: members whose id is one of its ids
            uint64_t m = 0;
            const int own = live ? ids[t] : -1;
            if (live && !over && (unsigned)own < (unsigned)prev_cap) {
                int pv[kPrevIds];
#pragma unroll
                for (int a = 0; a < kPrevIds; ++a) pv[a] = prev[(size_t)own * kPrevIds + a];
#pragma unroll
                for (int q = 0; q < kMemPerLane; ++q) {
                    bool in = false;
#pragma unroll
                    for (int a = 0; a < kPrevIds; ++a) in = in || pv[a] == mi[q];
                    if (sub + kCollL * q < nm && pos[q] < VRM_KMAX && in) m |= 1ull << pos[q];
                }
            }
            uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
#pragma unroll
            for (int o = 1; o < kCollL; o <<= 1) {
                lo |= __shfl_xor(lo, o, 64);
                hi |= __shfl_xor(hi, o, 64);
            }
            if (live && !over && sub == 0) pmask[r] = ((uint64_t)hi << 32) | lo;
        }
        if (live && !over) {
            int32_t* row = rec + (size_t)r * kRecRow;
#pragma unroll
            for (int q = 0; q < kMemPerLane; ++q) {
                const int e = sub + kCollL * q;
                if (e < nm && pos[q] < VRM_KMAX)
                    row[pos[q]] = (int)(((unsigned)s_u[grp][e] << 6) | (unsigned)rk[q]);
            }
            if (sub == 0) {
                kcol[r] = k;
                // the bin of the counting sort: the particle's pivots in its last
                // complete LP when known (cold or network-started solves), else k
                if constexpr (WM == 0) {
                    const int own = ids[t];
                    const int h = (unsigned)own < (unsigned)prev_cap ? pivhist[own] : 255;
                    const int b = h == 255 ? k : min(h, kKBins - 1);
                    key[r] = b;
                    atomicAdd(&s_hist[b], 1);
                } else {
                    key[r] = k;
                    atomicAdd(&s_hist[k], 1);
                }
            }
        }
        if (over && sub == 0) {
            kcol[r] = -1;
            key[r] = -1;   // not binned: the one-thread kernel solves it
        }
        // lists too long for the group: the one-thread kernel solves them from the retry queue
        const int pr = wave_append(&qs->n_retry, over && sub == 0);
        if (over && sub == 0) q_retry[pr] = t;
        count_add(&cnt->n_truncated, live && sub == 0 && nm > VRM_KMAX);
        // the next item's appends must not overwrite the list before every lane is done with it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    for (int b = tid; b < kKBins; b += blockDim.x)
        if (s_hist[b]) atomicAdd(&khist[b], s_hist[b]);
}

// start of each size bin in decreasing k; khist[kKBins .. 2 kKBins) becomes the fill
// pointers, and the histogram is cleared for the next run
__global__ void k_full_bin_starts(int32_t* khist)
{
    if (threadIdx.x == 0) {
        int at = 0;
        for (int k = kKBins - 1; k >= 0; --k) {
            khist[kKBins + k] = at;
            at += khist[k];
            khist[k] = 0;
        }
    }
}

// order[pos] = queue item, grouped by k (decreasing); one atomic per bin and workgroup
__global__ __launch_bounds__(256) void k_full_bin_scatter(const int32_t* __restrict__ kcol, const Queues* qs,
                                                          int32_t* khist, int32_t* order)
{
    __shared__ int s_cnt[kKBins], s_base[kKBins];
    const int tid = threadIdx.x;
    for (int b = tid; b < kKBins; b += blockDim.x) s_cnt[b] = 0;
    __syncthreads();
    const int nitems = qs->n_full;
    const int r = blockIdx.x * blockDim.x + tid;
    int k = -1, local = 0;
    if (r < nitems) {
        k = kcol[r];   // -1: left for the one-thread kernel
        if (k >= 0) local = atomicAdd(&s_cnt[k], 1);
    }
    __syncthreads();
    for (int b = tid; b < kKBins; b += blockDim.x)
        s_base[b] = s_cnt[b] ? atomicAdd(&khist[kKBins + b], s_cnt[b]) : 0;
    __syncthreads();
    if (k >= 0) order[s_base[k] + local] = r;
}

// Working-set column store: the nearest W columns' FP32 scaled offsets and costs
// in LDS (planes of kFullBlock), the others computed from the record row and the
// positions when priced (only after widen()).  Exact offsets always come from the
// positions.
template <int W>
struct SiftCols {
    static constexpr int KC = 0;
    static constexpr bool kCoop = false;
    int k;
    mutable int kw;                 // columns priced: the working set, then all
    uint64_t dead;
    const float* sx;                // LDS planes, this thread's column 0
    const float* sy;
    const float* sc;
    const int32_t* __restrict__ row;   // record row: (slot << 6) | rank
    float xi, yi;
    const float* __restrict__ xs;
    const float* __restrict__ ys;
    const LaunchParams* P;
    static constexpr int kLds = W;
    __device__ __forceinline__ void load_lds(int j, float& x, float& y, uint32_t& aux) const
    {
        x = sx[j * kFullBlock];
        y = sy[j * kFullBlock];
        aux = __float_as_uint(sc[j * kFullBlock]);
    }
    __device__ __forceinline__ int active() const { return kw; }
    __device__ __forceinline__ bool widen() const
    {
        if (kw >= k) return false;
        kw = k;
        return true;
    }
    __device__ __forceinline__ void restart() const { kw = k < W ? k : W; }
    __device__ __forceinline__ void exact_xy(int j, df& X, df& Y) const
    {
        const int u = (int)((unsigned)row[j] >> 6);
        exact_offset(xi, yi, xs[u], ys[u], P->scale2e, X, Y);
    }
    __device__ __forceinline__ void exact(int j, df& X, df& Y, df& C) const
    {
        const int m = row[j];
        const int u = (int)((unsigned)m >> 6);
        exact_offset(xi, yi, xs[u], ys[u], P->scale2e, X, Y);
        C = add_rank(cost_df(X, Y, *P), m & 63, P->q);
    }
    __device__ __forceinline__ void get(int j, float& x, float& y, float& c) const
    {
        if (j < W) {
            x = sx[j * kFullBlock];
            y = sy[j * kFullBlock];
            c = sc[j * kFullBlock];
        } else {
            // FP32 offset (the high part of the exact one: the scale is a power
            // of two) and FP32 cost; the exact ones are recomputed for certification
            const int m = row[j];
            const int u = (int)((unsigned)m >> 6);
            x = (xs[u] - xi) * P->scale2e;
            y = (ys[u] - yi) * P->scale2e;
            const float d2 = x * x + y * y;
            const float w = P->q == 2 ? d2 * __builtin_sqrtf(d2) : d2 * d2;
            c = __builtin_fmaf(w, P->cs_hi, tie_weight((unsigned)m & 63u, P->q));
        }
    }
    __device__ __forceinline__ void load(int j, float& x, float& y, uint32_t& aux) const
    {
        float c;
        get(j, x, y, c);
        aux = __float_as_uint(c);
    }
    template <int Q>
    __device__ __forceinline__ float cost_of(float, float, uint32_t aux) const
    {
        return __uint_as_float(aux);
    }
};

// The network's predicted basis of each complete LP: the m columns of largest
// logit (L[item][kMlpSlots]) among its first min(k, kMlpSlots) (lowest slot
// among equal logits), as a column mask for the crash.
__global__ __launch_bounds__(256) void k_top_mask(const float* __restrict__ pred, const int32_t* __restrict__ kcol,
                                                  const Queues* qs, int m, uint64_t* pmask)
{
    const int nitems = qs->n_full;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nitems; r += gridDim.x * blockDim.x) {
        const int k = kcol[r];   // -1: a list left for the one-thread kernel
        if (k < 0) continue;
        const int kk = min(k, kMlpSlots);
        float v[kMlpSlots];
        const float4* row = reinterpret_cast<const float4*>(pred + (size_t)r * kMlpSlots);
#pragma unroll
        for (int a = 0; a < kMlpSlots / 4; ++a) {
            const float4 q = row[a];
            v[4 * a] = q.x;
            v[4 * a + 1] = q.y;
            v[4 * a + 2] = q.z;
            v[4 * a + 3] = q.w;
        }
        uint64_t mask = 0;
        for (int t = 0; t < m && t < kk; ++t) {
            int best = -1;
            float bv = 0.0f;
#pragma unroll
            for (int j = 0; j < kMlpSlots; ++j) {
                const bool ok = j < kk && !((mask >> j) & 1ull) && (best < 0 || v[j] > bv);
                best = ok ? j : best;
                bv = ok ? v[j] : bv;
            }
            mask |= 1ull << best;
        }
        pmask[r] = mask;
    }
}

// WM: 0 cold; 1 crash from the network's prediction (out.pmask: its top-m
// columns per queue item), finished whatever it takes; 2 crash from the
// previous basis (out.pmask), at most warm_cap pivots, recording the new one;
// 3 the LPs the launch before deferred (the items in q_defer, queue indices
// below the 2^26 capacity limit with two flag bits): certified from their
// bases in out.pmask, or solved cold where a warm attempt ended infeasible;
// the basis is recorded when out.prev is set.  A
// crash basis that is not feasible is repaired by the composite phase I; a
// warm attempt that fails is solved cold in place.  The canonical launches
// (OBJ 0, WM 0 to 2) defer the LPs whose fast certificate fails to a WM 3
// launch: the double-float dual check of a few per cent of the LPs would
// otherwise hold up most waves (a wave runs it when any of its 64 lanes
// needs it).
template <int M, int W, int OBJ, int WM>
__global__ __launch_bounds__(kFullBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_lp_sift(
    const int32_t* __restrict__ perm, const float* __restrict__ xs, const float* __restrict__ ys,
    const int32_t* __restrict__ ids, const int32_t* __restrict__ order, const int32_t* __restrict__ kcol,
    const int32_t* __restrict__ rec, const int32_t* __restrict__ q_full, Queues* qs, const float* __restrict__ gamma,
    float* acc, LaunchParams P, StencilOut out, int apply, vrm_counters* cnt, int last_launch, const GridState* gs,
    int32_t* q_defer, int defer_cold)
{
    // deferral: always for the warm launches (their cold re-solves run there),
    // for the cold one only when the host asks (large clouds)
    const bool defers = WM != 3 && OBJ == 0 && (WM != 0 || defer_cold);
    __shared__ float s_x[W * kFullBlock];
    __shared__ float s_y[W * kFullBlock];
    __shared__ float s_c[W * kFullBlock];
    cnt = counter_stripe(cnt);
    const int tid = threadIdx.x;
    // the binned items, or the deferred ones
    const int nitems = WM == 3 ? qs->n_defer : qs->n_full - qs->n_retry;
    const int stride = gridDim.x * blockDim.x;
    const int loops = (nitems + stride - 1) / stride;
    const double dsc = P.det && apply ? det_scale(gs->gmax_bits) : 0.0;
    for (int it = 0; it < loops; ++it) {
        const int p = blockIdx.x * blockDim.x + tid + it * stride;
        const bool live = p < nitems;
        int st = 1, piv = 0, certified = 1, k = 0, warm = 0, r = 0, was_warm = 0, cold = 0;
        int cstat[2] = {0, 0};
        if (live) {
            if constexpr (WM == 3) {
                // bit 31: the deferring launch had settled the LP from its warm start;
                // bit 30: its warm attempt ended infeasible, solve it cold
                const int e = q_defer[p];
                r = e & 0x3fffffff;
                was_warm = ((unsigned)e >> 31) & 1;
                cold = ((unsigned)e >> 30) & 1;
            } else {
                r = order[p];
            }
            const int t = q_full[r];
            const int i = perm[t];
            k = kcol[r];
            const int32_t* row = rec + (size_t)r * kRecRow;
            const float xi = xs[t], yi = ys[t];
            const int kw = min(k, W);
            // the working set: offsets and costs of the nearest columns, slots read eight at a time
            for (int j0 = 0; j0 < kw; j0 += 8) {
                int bm[8];
                float bx[8], by[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) bm[e] = row[min(j0 + e, kw - 1)];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int u = (int)((unsigned)bm[e] >> 6);
                    bx[e] = xs[u];
                    by[e] = ys[u];
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int j = j0 + e;
                    if (j >= kw) break;
                    df X, Y;
                    exact_offset(xi, yi, bx[e], by[e], P.scale2e, X, Y);
                    s_x[j * kFullBlock + tid] = X.hi;
                    s_y[j * kFullBlock + tid] = Y.hi;
                    s_c[j * kFullBlock + tid] = add_rank(cost_df(X, Y, P), bm[e] & 63, P.q).hi;
                }
            }
            SiftCols<W> cs{k, kw, 0ull, s_x + tid, s_y + tid, s_c + tid, row, xi, yi, xs, ys, &P};
            float fii = 0.0f;
            const float g_i = gamma[i];
            int nz = 0;
            auto store = [&](int j, float v) {
                const int pj = perm[(unsigned)row[j] >> 6];
                if (apply) acc_add(acc, pj, v, g_i, dsc);
                if (out.full_idx) {
                    out.full_idx[(size_t)i * VRM_KMAX + nz] = pj;
                    out.full_f[(size_t)i * VRM_KMAX + nz] = v;
                }
                ++nz;
            };
            uint64_t basis = 0;
            if constexpr (WM == 0) {
                st = solve_lp<M, OBJ, false>(cs, P, store, fii, piv, certified, false, nullptr, warm, basis, false,
                                             0ull, cstat, true, defers);
            } else {
                const uint64_t pref = cold ? 0ull : out.pmask[r];
                // a prediction that is given up is followed by the cold solve in place
                st = solve_lp<M, OBJ, true, true>(cs, P, store, fii, piv, certified, !cold, nullptr, warm, basis,
                                                  !cold, pref, cstat, WM != 1, defers);
                if (WM == 3) warm = cold ? 0 : was_warm;
                // A warm attempt that ends infeasible is not final: its FP32 phase I may
                // stop on a vertex whose basic artificial is within the FP32 tolerance
                // but not zero in exact arithmetic, which the certification rejects.
                // The deferred launch solves it cold, as the plain solver does.
                if (defers && st == 1 && (warm == 1 || warm == 2)) st = 7;
            }
            if (defers && st == 5) out.pmask[r] = basis;
            if (WM == 2 || (WM == 3 && out.prev)) {
                const int own = ids[t];
                auto col_id = [&](int j) { return ids[(unsigned)row[j] >> 6]; };
                if (st == 0 && (unsigned)own < (unsigned)out.prev_cap) record_basis(out.prev, own, basis, col_id);
            }
            if constexpr (WM < 2) {
                // this LP's pivots, the bin of the particle's next complete LP
                const int own = ids[t];
                if (out.pivhist && (unsigned)own < (unsigned)out.prev_cap) out.pivhist[own] = (uint8_t)min(piv, 254);
            }
            if (st == 0) {
                if (apply) acc_add(acc, i, fii, g_i, dsc);
                if (out.full_k) {
                    out.full_k[i] = nz;
                    out.fii[i] = fii;
                    out.status[i] = (warm == 1 || warm == 2) ? VRM_ST_WARM : VRM_ST_FULL;
                }
            } else if (out.status && st != 5 && st != 7) {
                out.status[i] = VRM_ST_INFEASIBLE;
            }
        }
        if (defers) {
            const bool later = live && (st == 5 || st == 7);
            const int dpos = wave_append(&qs->n_defer, later);
            if (later)
                q_defer[dpos] = r | ((warm == 1 || warm == 2) && st == 5 ? (int)0x80000000u : 0) |
                                (st == 7 ? 0x40000000 : 0);
        }
        if constexpr (WM == 1 || WM == 2) count_warm(cnt, live, warm);
        const bool ok = live && st == 0;
        if (piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        if (ok) atomicAdd((unsigned long long*)&cnt->full_cols, (unsigned long long)k);
        if (cstat[0]) atomicAdd((unsigned long long*)&cnt->cert_rounds, (unsigned long long)cstat[0]);
        count_add(&cnt->n_full, ok);
        count_add(&cnt->n_infeasible, live && st == 1);
        count_add(&cnt->n_uncertified, ok && !certified);
        {
            const uint64_t m = __ballot(live && cstat[1]);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->cert_exact, (unsigned long long)__popcll(m));
        }
        if (apply) {
            uint64_t m = __ballot(ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
    }
    if (last_launch) {
        // the last LP launch of a stencil run: its last block to finish empties the
        // queues for the next run (keeping the counts for the host)
        __shared__ int last;
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) last = atomicAdd(&qs->blocks_done, 1) == (int)gridDim.x - 1;
        __syncthreads();
        if (last && threadIdx.x == 0) {
            __threadfence();
            qs->last_small = qs->n_small;
            qs->last_full = qs->n_full;
            qs->n_small = 0;
            qs->n_full = 0;
            qs->n_retry = 0;
            qs->n_defer = 0;
            qs->blocks_done = 0;
        }
    }
}

// ------------------------------------------------------------ particle removal
// Particle removal (Sec. 6, outlook): a particle closer than r h to another
// gives its circulation to its complete neighbourhood (r h .. R_full h) by
// the first-order identity LP -- sum g = 1, sum g r = 0, g >= 0, minimising
// sum g (|r/h|^2 + 2^-16 rank^2) -- and is dropped.  Candidates are taken
// greedily in id order, skipping one within R_full h of a taken candidate (so
// no removed particle receives circulation); one whose LP is infeasible stays.
constexpr uint8_t kRmNone = 0, kRmUndecided = 1, kRmIn = 2, kRmOut = 3;

// candidates: a particle closer than r h to another (per slot); the
// positions of a row's three cells are read eight at a time
// (a non-finite circulation sets kBadGamma; with a non-finite value no slot is a
// candidate)
__global__ __launch_bounds__(256) void k_rm_candidates(int n, const float* __restrict__ xs,
                                                       const float* __restrict__ ys,
                                                       const int32_t* __restrict__ cell_start, GridState* gs,
                                                       LaunchParams P, uint8_t* state, const int32_t* __restrict__ perm,
                                                       const float* __restrict__ gamma)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    // slots exist only for finite positions
    const bool nf = t < n && !(gs->bad & kBadPos) && !(fabsf(gamma[perm[t]]) <= 3.4028235e38f);
    if (__any(nf) && lane_id() == 0) atomicOr(&gs->bad, kBadGamma);
    if (t >= n) return;
    const GridState g = *gs;
    if (g.bad) {
        state[t] = kRmNone;
        return;
    }
    const float xi = xs[t], yi = ys[t];
    int cx, cy;
    cell_of_pos(g, xi, yi, cx, cy);
    bool close = false;
    for (int oy = -1; oy <= 1 && !close; ++oy) {
        const int yy = cy + oy;
        if (yy < 0 || yy >= g.ny) continue;
        const int u0 = cell_start[yy * g.nx + max(cx - 1, 0)];
        const int u1 = cell_start[yy * g.nx + min(cx + 1, g.nx - 1) + 1];
        for (int u = u0; u < u1 && !close; u += 8) {
            float bx[8], by[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int v = min(u + e, u1 - 1);
                bx[e] = xs[v];
                by[e] = ys[v];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e)
                close = close || (u + e < u1 && u + e != t && d2_f32(bx[e] - xi, by[e] - yi) < P.lo2f);
        }
    }
    state[t] = close ? kRmUndecided : kRmNone;
}

// selection predicate: the slot's state
struct RmStateIs {
    const uint8_t* state;
    uint8_t want;
    __device__ bool operator()(int t) const { return state[t] == want; }
};

// One round of the greedy selection in id order: an undecided candidate with a
// taken candidate within R_full h is out; one with no smaller-id candidate
// still undecided there is taken.  States only go from undecided to taken or
// out, so reading a neighbour's state while it changes is safe: both values
// lead to a decision the sequential greedy pass also makes.
__global__ __launch_bounds__(256) void k_rm_mis_round(int nc, const int32_t* __restrict__ cand,
                                                      const float* __restrict__ xs, const float* __restrict__ ys,
                                                      const int32_t* __restrict__ ids,
                                                      const int32_t* __restrict__ cell_start, const GridState* gs,
                                                      LaunchParams P, uint8_t* state, Queues* qs)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    const int t = cand[k];
    volatile uint8_t* vstate = state;   // other threads change it during the round
    if (vstate[t] != kRmUndecided) return;
    const GridState g = *gs;
    const float xi = xs[t], yi = ys[t];
    const int id = ids[t];
    int cx, cy;
    cell_of_pos(g, xi, yi, cx, cy);
    bool in_near = false, smaller_open = false;
    for (int oy = -1; oy <= 1; ++oy) {
        const int yy = cy + oy;
        if (yy < 0 || yy >= g.ny) continue;
        const int u0 = cell_start[yy * g.nx + max(cx - 1, 0)];
        const int u1 = cell_start[yy * g.nx + min(cx + 1, g.nx - 1) + 1];
        for (int u = u0; u < u1; ++u) {
            if (u == t) continue;
            const uint8_t su = vstate[u];
            if (su != kRmUndecided && su != kRmIn) continue;
            if (d2_f32(xs[u] - xi, ys[u] - yi) > P.hi2f) continue;
            if (su == kRmIn)
                in_near = true;
            else if (ids[u] < id)
                smaller_open = true;
        }
    }
    if (in_near)
        vstate[t] = kRmOut;
    else if (!smaller_open)
        vstate[t] = kRmIn;
    else
        qs->n_undecided = 1;
}

// The identity LP of every taken candidate, one thread each; the columns live
// in LDS as for the complete-neighbourhood Laplacian LPs.
template <bool SC>
__global__ __launch_bounds__(kFullBlock) void k_rm_lp(const int32_t* __restrict__ perm, const float* __restrict__ xs,
                                                      const float* __restrict__ ys, const int32_t* __restrict__ ids,
                                                      const int32_t* __restrict__ cell_start, const GridState* gs,
                                                      const int32_t* __restrict__ queue, Queues* qs,
                                                      const float* __restrict__ gamma, float* acc, uint8_t* removed,
                                                      LaunchParams P)
{
    __shared__ float s_rx[VRM_KMAX * kFullBlock];
    __shared__ float s_ry[VRM_KMAX * kFullBlock];
    __shared__ int s_meta[VRM_KMAX * kFullBlock];
    __shared__ float s_c[SC ? VRM_KMAX * kFullBlock : 1];
    const int tid = threadIdx.x;
    const int nitems = qs->n_accepted;
    const GridState g = *gs;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < nitems; base += stride) {
        const int item = base + tid;
        bool ok = false, unc = false;
        if (item < nitems) {
            const int t = queue[item];
            const int i = perm[t];
            const float xi = xs[t], yi = ys[t];
            bool truncated;
            const int k = collect_full(t, xi, yi, g, cell_start, xs, ys, ids, P, s_meta + tid, s_rx + tid,
                                       reinterpret_cast<int*>(s_ry) + tid, truncated);
            for (int j = 0; j < k; ++j) {
                const int idj = __float_as_int(s_ry[j * kFullBlock + tid]);
                int rank = 0;
                for (int o = 0; o < k; ++o) rank += __float_as_int(s_ry[o * kFullBlock + tid]) < idj ? 1 : 0;
                s_meta[j * kFullBlock + tid] = (int)(((unsigned)s_meta[j * kFullBlock + tid] << 6) | (unsigned)rank);
            }
            for (int j = 0; j < k; ++j) {
                const int meta = s_meta[j * kFullBlock + tid];
                const int um = (int)((unsigned)meta >> 6);
                df X, Y;
                exact_offset(xi, yi, xs[um], ys[um], P.scale2e, X, Y);
                s_rx[j * kFullBlock + tid] = X.hi;
                s_ry[j * kFullBlock + tid] = Y.hi;
                if constexpr (SC) s_c[j * kFullBlock + tid] = add_rank(cost_df(X, Y, P), meta & 63, P.q).hi;
            }
            LdsColsT<kFullBlock, SC> cs{k, 0ull, s_rx, s_ry, s_c, s_meta, tid, xi, yi, xs, ys, &P, nullptr, nullptr};
            const float g_i = gamma[i];
            auto store = [&](int j, float v) {
                const int pj = perm[(unsigned)s_meta[j * kFullBlock + tid] >> 6];
                atomicAdd(&acc[pj], v * g_i);
            };
            float fii = 0.0f;
            int piv = 0, certified = 1, warm = 0;
            uint64_t basis = 0;
            const int st = k > 0 ? solve_lp<3, false>(cs, P, store, fii, piv, certified, false, nullptr, warm, basis)
                                 : 1;
            if (st == 0) {
                removed[i] = 1;
                ok = true;
                unc = !certified;
            }
        }
        count_add(&qs->n_removed, ok);
        count_add(&qs->n_rm_uncertified, unc);
    }
}

// received circulation, and the particles that stay
__global__ __launch_bounds__(256) void k_rm_apply(int n, float* gamma, float* acc, const uint8_t* __restrict__ removed,
                                                  int32_t* keep)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    gamma[i] += acc[i];
    acc[i] = 0.0f;
    keep[i] = removed[i] ? 0 : 1;
}

// the particles that stay, in their order, to the scratch arrays
__global__ __launch_bounds__(256) void k_rm_gather(int n, const int32_t* __restrict__ keep,
                                                   const int32_t* __restrict__ pos, const float* __restrict__ x,
                                                   const float* __restrict__ y, const float* __restrict__ g,
                                                   const int32_t* __restrict__ id, float* tx, float* ty, float* tg,
                                                   int32_t* tid)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !keep[i]) return;
    const int j = pos[i];
    tx[j] = x[i];
    ty[j] = y[i];
    tg[j] = g[i];
    tid[j] = id[i];
}

__global__ __launch_bounds__(256) void k_rm_copy(int m, const float* __restrict__ tx, const float* __restrict__ ty,
                                                 const float* __restrict__ tg, const int32_t* __restrict__ tid, float* x,
                                                 float* y, float* g, int32_t* id, int32_t* n_dev)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) *n_dev = m;
    if (j >= m) return;
    x[j] = tx[j];
    y[j] = ty[j];
    g[j] = tg[j];
    id[j] = tid[j];
}

__global__ void k_rm_reset(Queues* q)
{
    q->n_cand = 0;
    q->n_undecided = 0;
    q->n_accepted = 0;
    q->n_removed = 0;
    q->n_rm_uncertified = 0;
}
__global__ void k_rm_reset_undecided(Queues* q) { q->n_undecided = 0; }

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

// persistent launches: enough threads for every CU (at most the tuned number
// of workgroups), each loops over its items
int lp_grid_small(const vrm_ctx* c, int n)
{
    const int per_block = (kSmallBlock / 64) * c->tuning.lp_small_lanes;
    return n > 0 ? min((n + per_block - 1) / per_block, c->tuning.lp_small_blocks) : 1;
}
int lp_grid_full(const vrm_ctx* c, int n)
{
    return n > 0 ? min((n + kFullBlock - 1) / kFullBlock, c->tuning.lp_full_blocks) : 1;
}
// workgroups of the neighbourhood kernel: 256 particles each, or 256 / kNbL
// with kNbL lanes per particle up to kNbhdCoopMaxN particles
int nbhd_blocks(int n) { return n <= kNbhdCoopMaxN ? (n + 256 / kNbL - 1) / (256 / kNbL) : (n + 255) / 256; }
// clouds up to the tuned size launch the complete-LP kernel with stored costs
bool full_stored_costs(const vrm_ctx* c, int n) { return n <= c->tuning.full_stored_cost_n; }

// the instantiation of an LP kernel for the context's objective (0 canonical,
// 1 phase I only, 2 non-negative least squares)
template <class F>
F by_objective(int obj, F canonical, F phase1, F nnls)
{
    return obj == 2 ? nnls : obj == 1 ? phase1 : canonical;
}
template <int M, bool SC>
auto full_kernel(int obj) -> decltype(&k_lp_full<M, SC, 0, false>)
{
    return by_objective(obj, k_lp_full<M, SC, 0, false>, k_lp_full<M, SC, 1, false>, k_lp_full<M, SC, 2, false>);
}

}  // namespace

int vrm_small_nbhd_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const LaunchParams& lp, int32_t* small_idx,
                       int32_t* kfull)
{
    (void)cl;
    if (n <= 0) return VRM_OK;
    const bool coop = n <= kNbhdCoopMaxN;
    hipLaunchKernelGGL(coop ? k_small_nbhd_coop : k_small_nbhd, dim3(nbhd_blocks(n)), dim3(256), 0, c->stream, n,
                       cl->n_dev, c->perm, c->xs, c->ys, c->ids, c->cell_start, c->diffused, c->grid, lp, SmallRec{},
                       (int32_t*)nullptr, (int32_t*)nullptr, c->queues, small_idx, kfull, kfull != nullptr ? 1 : 0);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_stencil_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const LaunchParams& lp, const vrm_stencils* st,
                    int apply, uint16_t* feat_out, float* label_out, int max_rows)
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
    out.feat = feat_out;
    out.lab = label_out;
    out.max_rows = max_rows;
    // the LP queues are empty here: the last LP launch of every run empties them
    {
        ScopedTimer tm(c, VRM_T_NBHD);
        const bool coop = n <= kNbhdCoopMaxN;
        hipLaunchKernelGGL(coop ? k_small_nbhd_coop : k_small_nbhd, dim3(nbhd_blocks(n)), dim3(256), 0, c->stream, n,
                           cl->n_dev, c->perm, c->xs, c->ys, c->ids, c->cell_start, c->diffused, c->grid, lp, c->srec,
                           c->q_small, c->q_full, c->queues, (int32_t*)nullptr, (int32_t*)nullptr, 0);
    }
    VRM_HIP(hipGetLastError());
    const bool net = c->warm == 1 && c->mlp && c->mlp->loaded && !feat_out;
    const bool warm = net || (c->warm == 2 && !feat_out);
    out.cloud_id = cl->id_dev;
    if (c->warm == 2 && c->prev && !feat_out) {
        out.prev = c->prev;
        out.prev_cap = c->capacity;
        out.use_prev = 1;
    }
    if (net && lp.m == 5) {
        // network inputs of the queued small LPs and the forward pass, fused (row count read on the device)
        ScopedTimer tm(c, VRM_T_MLP);
        int r = vrm_mlp_infer_small_run(c, n, &c->queues->n_small, c->srec, lp.sc, lp.q, c->pred);
        if (r) return r;
        out.pred = c->pred;
    }
    // warm: the pass from the predicted bases, then a cold pass over what it left
    const int first = warm ? kLpWarm : kLpPlain;
    if (lp.m == 5) {
        {
            ScopedTimer tm(c, VRM_T_LP_SMALL);
            if (!warm && c->tuning.lp_small_coop && !feat_out && lp.phase1 != 2) {
                // eight lanes per LP (plain or phase-I pass)
                const int per_block = kSmallBlock / 8;
                const int grid = min((n + per_block - 1) / per_block, c->tuning.lp_small_blocks);
                hipLaunchKernelGGL((lp.phase1 == 1 ? k_lp_small_coop<1> : k_lp_small_coop<0>), dim3(max(grid, 1)),
                                   dim3(kSmallBlock), 0, c->stream, cl->gamma_dev, c->srec, c->q_small, c->queues,
                                   c->q_full, c->acc, lp, out, apply, c->counters, c->grid);
                VRM_HIP(hipGetLastError());
            } else {
                for (int mode = first; mode <= (warm ? kLpRetry : kLpPlain); ++mode) {
                    hipLaunchKernelGGL((by_objective(lp.phase1, k_lp_small<0>, k_lp_small<1>, k_lp_small<2>)), dim3(lp_grid_small(c, n)),
                                       dim3(kSmallBlock), 0, c->stream, c->perm, c->xs, c->ys, c->ids, c->srec,
                                       c->q_small, c->queues, c->q_full, cl->gamma_dev, c->acc, lp, out, apply,
                                       c->counters, mode, c->q_retry, c->tuning.lp_small_lanes, c->grid);
                    VRM_HIP(hipGetLastError());
                }
            }
        }
        // fallbacks of the small LPs: no network input for them
        StencilOut o2 = out;
        o2.pred = nullptr;
        o2.feat = nullptr;
        o2.lab = nullptr;
        ScopedTimer tm(c, VRM_T_LP_FULL);
        const bool stored = full_stored_costs(c, n);
        hipLaunchKernelGGL((stored ? full_kernel<5, true>(lp.phase1) : full_kernel<5, false>(lp.phase1)),
                           dim3(min(lp_grid_full(c, n), 64)), dim3(kFullBlock), 0, c->stream, c->perm,
                           c->xs, c->ys, c->ids, c->cell_start, c->grid, c->q_full, c->queues, cl->gamma_dev, c->acc, lp,
                           o2, apply, c->counters, kLpPlain, c->q_retry, 1);
    } else if (!feat_out) {
        // size-binned working-set path: column lists (with the previous basis),
        // counting sort, the network's inference from the lists if it predicts, LPs
        const int wm = net ? 1 : (warm ? 2 : 0);
        {
            ScopedTimer tm(c, VRM_T_FULL_COLS);
            auto collect = wm == 2 ? k_full_collect<2> : k_full_collect<0>;
            hipLaunchKernelGGL(collect, dim3(min((n + kCollGroups - 1) / kCollGroups, 4096)), dim3(kCollBlock), 0,
                               c->stream, c->xs, c->ys, c->ids, c->cell_start, c->grid, c->q_full, c->queues, lp,
                               c->full_cols, c->full_k, c->khist, c->q_retry, c->counters,
                               wm == 2 ? c->prev : nullptr, c->capacity, wm == 2 ? c->pmask : nullptr, c->pivhist,
                               c->lkey);
            hipLaunchKernelGGL(k_full_bin_starts, dim3(1), dim3(64), 0, c->stream, c->khist);
            hipLaunchKernelGGL(k_full_bin_scatter, dim3((n + 255) / 256), dim3(256), 0, c->stream, c->lkey,
                               c->queues, c->khist, c->full_order);
            VRM_HIP(hipGetLastError());
        }
        if (wm == 1) {
            // the predicted bases, from the column lists (row count read on the device)
            ScopedTimer tm(c, VRM_T_MLP);
            const FullRec fr{c->full_cols, kRecRow, c->full_k, c->q_full, c->xs, c->ys, lp.scale2e, lp.sc, lp.q};
            int r = vrm_mlp_infer_full_run(c, n, &c->queues->n_full, fr, c->pred);
            if (r) return r;
            hipLaunchKernelGGL(k_top_mask, dim3(min((n + 255) / 256, 4096)), dim3(256), 0, c->stream, c->pred,
                               c->full_k, c->queues, lp.m, c->pmask);
            VRM_HIP(hipGetLastError());
        }
        out.pmask = c->pmask;
        out.pivhist = c->pivhist;
        out.prev_cap = c->capacity;
        ScopedTimer tm(c, VRM_T_LP_FULL);
        const int obj = lp.phase1;
        // A cold launch defers its exact certifications to a second launch only on
        // large clouds: there a wave would otherwise wait on the few lanes that
        // need them; on small ones every launch is one latency-bound wave per
        // SIMD, and a second launch adds its whole chain.
        const int defer_cold = n >= kDeferMinN ? 1 : 0;
        auto sift = wm == 0 ? by_objective(obj, k_lp_sift<9, kSiftW, 0, 0>, k_lp_sift<9, kSiftW, 1, 0>,
                                           k_lp_sift<9, kSiftW, 2, 0>)
                  : wm == 1 ? (obj == 1 ? k_lp_sift<9, kSiftW, 1, 1> : k_lp_sift<9, kSiftW, 0, 1>)
                            : (obj == 1 ? k_lp_sift<9, kSiftW, 1, 2> : k_lp_sift<9, kSiftW, 0, 2>);
        hipLaunchKernelGGL(sift, dim3(lp_grid_full(c, n)), dim3(kFullBlock), 0, c->stream, c->perm, c->xs, c->ys,
                           c->ids, c->full_order, c->full_k, c->full_cols, c->q_full, c->queues, cl->gamma_dev, c->acc,
                           lp, out, apply, c->counters, 0, c->grid, c->q_defer, defer_cold);
        if (obj == 0 && (wm != 0 || defer_cold)) {
            // what the launch deferred, from the bases (count read on the device)
            hipLaunchKernelGGL((k_lp_sift<9, kSiftW, 0, 3>), dim3(lp_grid_full(c, n)), dim3(kFullBlock), 0, c->stream,
                               c->perm, c->xs, c->ys, c->ids, c->full_order, c->full_k, c->full_cols, c->q_full,
                               c->queues, cl->gamma_dev, c->acc, lp, out, apply, c->counters, 0, c->grid, c->q_defer,
                               0);
        }
        // lists too long for the collection groups (none in practice): the one-thread
        // kernel from the retry queue, cold; as the run's last LP launch it empties the queues
        hipLaunchKernelGGL((full_kernel<9, false>(lp.phase1)), dim3(1), dim3(kFullBlock), 0, c->stream, c->perm, c->xs,
                           c->ys, c->ids, c->cell_start, c->grid, c->q_full, c->queues, cl->gamma_dev, c->acc, lp, out,
                           apply, c->counters, kLpRetry, c->q_retry, 1);
        VRM_HIP(hipGetLastError());
    } else {
        // training collection: the one-thread kernel records features and labels
        ScopedTimer tm(c, VRM_T_LP_FULL);
        const bool stored = full_stored_costs(c, n);
        hipLaunchKernelGGL((stored ? full_kernel<9, true>(lp.phase1) : full_kernel<9, false>(lp.phase1)),
                           dim3(lp_grid_full(c, n)), dim3(kFullBlock), 0, c->stream, c->perm, c->xs, c->ys, c->ids,
                           c->cell_start, c->grid, c->q_full, c->queues, cl->gamma_dev, c->acc, lp, out, apply,
                           c->counters, kLpPlain, c->q_retry, 1);
        VRM_HIP(hipGetLastError());
    }
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

// Network outputs of the queued LPs as the warm pass sees them (test hook of the
// fused inference): small LPs' 8 logits or complete LPs' 64 outputs, and the
// particle of each row.
namespace {
__global__ void k_pred_out(const Queues* qs, int m, const float* __restrict__ pred, const int32_t* __restrict__ rec_i,
                           const int32_t* __restrict__ perm, const int32_t* __restrict__ q_full, int max_rows,
                           float* out, int32_t* particle)
{
    const int nq = m == 5 ? qs->n_small : qs->n_full;
    const int rows = min(nq, max_rows);
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
        // small LPs: the logits of their 8 columns; complete LPs: the 32 basis logits
        for (int a = 0; a < kMlpOut; ++a)
            out[(size_t)r * kMlpOut + a] = m == 5 ? (a < VRM_NSEG ? pred[(size_t)r * VRM_NSEG + a] : 0.0f)
                                                  : (a < kMlpSlots ? pred[(size_t)r * kMlpSlots + a] : 0.0f);
        particle[r] = m == 5 ? rec_i[r] : perm[q_full[r]];
    }
}
__global__ void k_queues_done(Queues* qs)
{
    qs->last_small = qs->n_small;
    qs->last_full = qs->n_full;
    qs->n_small = 0;
    qs->n_full = 0;
    qs->n_retry = 0;
    qs->n_defer = 0;
    qs->blocks_done = 0;
}
}  // namespace

int vrm_warm_predict_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const LaunchParams& lp, float* out,
                         int32_t* particle, int max_rows)
{
    if (n <= 0) return VRM_OK;
    const bool coop = n <= kNbhdCoopMaxN;
    hipLaunchKernelGGL(coop ? k_small_nbhd_coop : k_small_nbhd, dim3(nbhd_blocks(n)), dim3(256), 0, c->stream, n,
                       cl->n_dev, c->perm, c->xs, c->ys, c->ids, c->cell_start, c->diffused, c->grid, lp, c->srec,
                       c->q_small, c->q_full, c->queues, (int32_t*)nullptr, (int32_t*)nullptr, 0);
    VRM_HIP(hipGetLastError());
    int r;
    if (lp.m == 5) {
        r = vrm_mlp_infer_small_run(c, n, &c->queues->n_small, c->srec, lp.sc, lp.q, c->pred);
    } else {
        // the LP path's own kernels: the column lists (their histogram cleared
        // again by the bin starts), then the inference from the lists
        hipLaunchKernelGGL(k_full_collect<0>, dim3(min((n + kCollGroups - 1) / kCollGroups, 4096)), dim3(kCollBlock),
                           0, c->stream, c->xs, c->ys, c->ids, c->cell_start, c->grid, c->q_full, c->queues, lp,
                           c->full_cols, c->full_k, c->khist, c->q_retry, c->counters, nullptr, c->capacity, nullptr,
                           c->pivhist, c->lkey);
        hipLaunchKernelGGL(k_full_bin_starts, dim3(1), dim3(64), 0, c->stream, c->khist);
        VRM_HIP(hipGetLastError());
        const FullRec fr{c->full_cols, kRecRow, c->full_k, c->q_full, c->xs, c->ys, lp.scale2e, lp.sc, lp.q};
        r = vrm_mlp_infer_full_run(c, n, &c->queues->n_full, fr, c->pred);
    }
    if (r) return r;
    hipLaunchKernelGGL(k_pred_out, dim3(256), dim3(256), 0, c->stream, c->queues, lp.m, c->pred, c->srec.i, c->perm,
                       c->q_full, max_rows, out, particle);
    hipLaunchKernelGGL(k_queues_done, dim3(1), dim3(1), 0, c->stream, c->queues);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

// Scratch bytes of the removal's device-wide selections and scan for up to
// cap particles (the context's sort scratch is sized to hold them too).
size_t vrm_remove_tmp_bytes(int32_t cap)
{
    size_t a = 0, b = 0, d = 0;
    int32_t* p = nullptr;
    (void)rocprim::select(nullptr, a, rocprim::counting_iterator<int32_t>(0), p, p, (size_t)cap,
                          RmStateIs{nullptr, kRmUndecided}, (hipStream_t)0);
    (void)rocprim::select(nullptr, b, p, p, p, (size_t)cap, RmStateIs{nullptr, kRmIn}, (hipStream_t)0);
    (void)rocprim::exclusive_scan(nullptr, d, p, p, 0, (size_t)cap, rocprim::plus<int32_t>(), (hipStream_t)0);
    return std::max(a, std::max(b, d));
}

// Particle removal over the current cell list (slot order); synchronises.
// Returns the new particle count or a negative error; the removed count is in
// the queues (n_removed).
int vrm_remove_run(vrm_ctx* c, vrm_cloud* cl, int32_t n, const LaunchParams& lp, int32_t* n_candidates)
{
    hipStream_t s = c->stream;
    const int nb = n > 0 ? (n + 255) / 256 : 1;
    hipLaunchKernelGGL(k_rm_reset, dim3(1), dim3(1), 0, s, c->queues);
    if (n == 0) {
        if (n_candidates) *n_candidates = 0;
        return n;
    }
    hipLaunchKernelGGL(k_rm_candidates, dim3(nb), dim3(256), 0, s, n, c->xs, c->ys, c->cell_start, c->grid, lp,
                       c->cstate, c->perm, cl->gamma_dev);
    VRM_HIP(hipGetLastError());
    // queue of the candidates (slots), then of the taken ones: device-wide selections
    int32_t* cand = c->cperm;
    {
        size_t bytes = 0;
        VRM_HIP(rocprim::select(nullptr, bytes, rocprim::counting_iterator<int32_t>(0), cand, &c->queues->n_cand,
                                (size_t)n, RmStateIs{c->cstate, kRmUndecided}, s));
        if (bytes > c->sort_tmp_bytes + 256)
            return vrm_fail(VRM_E_STATE, "removal: selection needs %zu bytes of scratch", bytes);
        VRM_HIP(rocprim::select(c->sort_tmp, bytes, rocprim::counting_iterator<int32_t>(0), cand,
                                &c->queues->n_cand, (size_t)n, RmStateIs{c->cstate, kRmUndecided}, s));
    }
    Queues q;
    int32_t bad = 0;
    VRM_HIP(hipMemcpyAsync(&q, c->queues, sizeof(Queues), hipMemcpyDeviceToHost, s));
    VRM_HIP(hipMemcpyAsync(&bad, &c->grid->bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VRM_HIP(hipStreamSynchronize(s));
    if (bad) return vrm_nonfinite(c, bad);   // nothing changed yet
    const int nc = q.n_cand;
    if (n_candidates) *n_candidates = nc;
    if (nc == 0) return n;
    const int nbc = (nc + 255) / 256;
    for (int rounds = 0;;) {
        const int batch = 4;
        for (int k = 0; k < batch; ++k) {
            hipLaunchKernelGGL(k_rm_reset_undecided, dim3(1), dim3(1), 0, s, c->queues);
            hipLaunchKernelGGL(k_rm_mis_round, dim3(nbc), dim3(256), 0, s, nc, cand, c->xs, c->ys, c->ids,
                               c->cell_start, c->grid, lp, c->cstate, c->queues);
        }
        rounds += batch;
        VRM_HIP(hipGetLastError());
        VRM_HIP(hipMemcpyAsync(&q, c->queues, sizeof(Queues), hipMemcpyDeviceToHost, s));
        VRM_HIP(hipStreamSynchronize(s));
        if (q.n_undecided == 0) break;
        if (rounds > 4 * nc + 64) return vrm_fail(VRM_E_STATE, "removal: selection did not converge");
    }
    {
        size_t bytes = 0;
        VRM_HIP(rocprim::select(nullptr, bytes, cand, c->aidx, &c->queues->n_accepted, (size_t)nc,
                                RmStateIs{c->cstate, kRmIn}, s));
        if (bytes > c->sort_tmp_bytes + 256)
            return vrm_fail(VRM_E_STATE, "removal: selection needs %zu bytes of scratch", bytes);
        VRM_HIP(rocprim::select(c->sort_tmp, bytes, cand, c->aidx, &c->queues->n_accepted, (size_t)nc,
                                RmStateIs{c->cstate, kRmIn}, s));
    }
    VRM_HIP(hipMemcpyAsync(&q, c->queues, sizeof(Queues), hipMemcpyDeviceToHost, s));
    VRM_HIP(hipStreamSynchronize(s));
    const int na = q.n_accepted;
    VRM_HIP(hipMemsetAsync(c->tmp_u8, 0, (size_t)n, s));
    {
        const bool stored = full_stored_costs(c, n);
        hipLaunchKernelGGL((stored ? k_rm_lp<true> : k_rm_lp<false>), dim3(lp_grid_full(c, na)), dim3(kFullBlock), 0, s,
                           c->perm, c->xs, c->ys, c->ids, c->cell_start, c->grid, c->aidx, c->queues, cl->gamma_dev,
                           c->acc, c->tmp_u8, lp);
        VRM_HIP(hipGetLastError());
    }
    int32_t* keep = c->ccell;
    int32_t* pos = c->crank;
    hipLaunchKernelGGL(k_rm_apply, dim3(nb), dim3(256), 0, s, n, cl->gamma_dev, c->acc, c->tmp_u8, keep);
    VRM_HIP(hipGetLastError());
    VRM_HIP(hipMemcpyAsync(&q, c->queues, sizeof(Queues), hipMemcpyDeviceToHost, s));
    VRM_HIP(hipStreamSynchronize(s));
    const int m = n - q.n_removed;
    if (q.n_removed == 0) return n;
    size_t bytes = 0;
    VRM_HIP(rocprim::exclusive_scan(nullptr, bytes, keep, pos, 0, (size_t)n, rocprim::plus<int32_t>(), s));
    if (bytes > c->sort_tmp_bytes + 256)
        return vrm_fail(VRM_E_STATE, "removal: scan needs %zu bytes of scratch, %zu held", bytes, c->sort_tmp_bytes);
    VRM_HIP(rocprim::exclusive_scan(c->sort_tmp, bytes, keep, pos, 0, (size_t)n, rocprim::plus<int32_t>(), s));
    const size_t cap = (size_t)c->capacity;
    hipLaunchKernelGGL(k_rm_gather, dim3(nb), dim3(256), 0, s, n, keep, pos, cl->x_dev, cl->y_dev, cl->gamma_dev,
                       cl->id_dev, c->tmp_f, c->tmp_f + cap, c->tmp_f + 2 * cap, c->tmp_i);
    VRM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rm_copy, dim3(m > 0 ? (m + 255) / 256 : 1), dim3(256), 0, s, m, c->tmp_f, c->tmp_f + cap,
                       c->tmp_f + 2 * cap, c->tmp_i, cl->x_dev, cl->y_dev, cl->gamma_dev, cl->id_dev, cl->n_dev);
    VRM_HIP(hipGetLastError());
    return m;
}
