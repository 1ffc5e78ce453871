// One-thread revised simplex for the moment-condition LP of one particle
// (Kirchhart & Obi, Sec. 2 eq. momcondmv and Sec. 4.1), and its certification.
//
//   minimise  sum_j c_j f_j   subject to  V f = b,  f >= 0,
//
// V has M rows (the monomials r^alpha, 1 <= |alpha| <= q, of the scaled
// offsets; or 1, x, y when the identity operator is approximated for
// particle removal, Sec. 6) and k <= 64 columns.  As the paper describes, every iteration works
// with the m x m matrix of the current basic columns; here its inverse B^-1
// is kept explicitly in registers and updated by one elementary row
// operation per pivot.  Phase I starts from the artificial basis with a
// right-hand side perturbed by distinct small amounts (steps over degenerate
// vertices), pricing takes the most negative relative reduced cost, with
// Bland's rule as a fallback.  FP32.
//
// The basis it ends with is then certified against the exact problem: the
// basic solution and the prices are refined with residuals evaluated in
// double-float arithmetic from the exact particle offsets, every reduced cost
// is recomputed the same way, and primal (Bland) or dual repair pivots are
// taken until the basis is optimal to a relative 1e-9.
#pragma once
#include "vrm_device.h"
#include "vrm_internal.h"

namespace vrm {

constexpr float kPerturb = 7.62939453125e-06f;   // 2^-17: relative rhs perturbation
constexpr float kTolD = 1e-6f;                    // FP32 pricing tolerance (relative)
constexpr float kTolPiv = 1e-6f;                  // FP32 pivot tolerance (relative to max |alpha|)
constexpr float kTolFeas = 1e-3f;                 // phase-I infeasibility (relative to the rhs)
constexpr float kCertD = 1e-9f;                   // certified reduced-cost tolerance (relative)
constexpr float kCertX = 1e-9f;                   // certified primal tolerance (absolute, fhat units)
constexpr float kNnlsRes = 1e-5f;                 // NNLS: residual of a found support (relative to b)
constexpr int kMaxRefine = 6;
constexpr float kFastMargin = 64.0f;              // fast certificate: FP32 reduced costs clear zero by this many
                                                  // times their error bound (first correction + 2^-23) x scale

// Rows of a column: the monomials r^alpha, 1 <= |alpha| <= q (M = 5, 9), or
// for the identity operator of particle removal (M = 3) 1, x, y.
template <int M>
__device__ __forceinline__ void mono(float x, float y, float (&v)[M])
{
    if constexpr (M == 3) {
        v[0] = 1.0f;
        v[1] = x;
        v[2] = y;
    } else {
        v[0] = x;
        v[1] = y;
        v[2] = x * x;
        v[3] = x * y;
        v[4] = y * y;
        if constexpr (M == 9) {
            v[5] = v[2] * x;
            v[6] = v[2] * y;
            v[7] = x * v[4];
            v[8] = v[4] * y;
        }
    }
}

template <int M>
__device__ __forceinline__ void mono_df(df X, df Y, df (&v)[M])
{
    if constexpr (M == 3) {
        v[0] = {1.0f, 0.0f};
        v[1] = X;
        v[2] = Y;
    } else {
        df XX = df_mul(X, X), XY = df_mul(X, Y), YY = df_mul(Y, Y);
        v[0] = X;
        v[1] = Y;
        v[2] = XX;
        v[3] = XY;
        v[4] = YY;
        if constexpr (M == 9) {
            v[5] = df_mul(XX, X);
            v[6] = df_mul(XX, Y);
            v[7] = df_mul(X, YY);
            v[8] = df_mul(YY, Y);
        }
    }
}

// |r|^(q+1) of the scaled exact offset, times (2^e/h)^(q+1): the canonical
// cost in units of h, double-float (q = 1: |r|^2, the removal LP's cost)
__device__ __forceinline__ df cost_df(df X, df Y, const LaunchParams& P)
{
    df d2 = df_add(df_mul(X, X), df_mul(Y, Y));
    df w = P.q == 1 ? d2 : (P.q == 2) ? df_mul(d2, df_sqrt(d2)) : df_mul(d2, d2);
    return df_mul(w, df{P.cs_hi, P.cs_lo});
}

// exact offset of particle j from particle i, scaled by 2^-e (exact)
__device__ __forceinline__ void exact_offset(float xi, float yi, float xj, float yj, float s, df& X, df& Y)
{
    df dx = two_sum(xj, -xi);
    df dy = two_sum(yj, -yi);
    X = {dx.hi * s, dx.lo * s};
    Y = {dy.hi * s, dy.lo * s};
}

// Right-hand side: 2 h^2 / 4^e at (2,0) and (0,2) for the Laplacian (eq.
// cond_two); the unit vector e0 for the identity (removal, M = 3)
template <int M>
__device__ __forceinline__ bool rhs_row(int a)
{
    return M == 3 ? a == 0 : (a == 2 || a == 4);
}
template <int M>
__device__ __forceinline__ float rhs_hi(int a, const LaunchParams& P) { return rhs_row<M>(a) ? P.bt_hi : 0.0f; }
template <int M>
__device__ __forceinline__ df rhs_df(int a, const LaunchParams& P)
{
    return rhs_row<M>(a) ? df{P.bt_hi, P.bt_lo} : df{0.0f, 0.0f};
}

// Column store interface (CS):
//   int k; uint64_t dead;                            number of columns, absent ones
//   void get(int j, float& rx, float& ry, float& c)  FP32 scaled offset and cost
//   void exact(int j, df& X, df& Y, df& C)           exact offset and cost
//   void exact_xy(int j, df& X, df& Y)               exact offset
// and, for stores with a run-time column count (KC == 0),
//   void load(int j, float& rx, float& ry, uint32_t& aux)  raw values of column j
//   float cost_of<Q>(float rx, float ry, uint32_t aux)      its FP32 cost (order Q)
//   int active()     columns the simplex prices (a prefix of the k; k by default)
//   kLds, load_lds(j, ...)  columns j < kLds are in LDS: load without the general path
//                  (kLds a multiple of four; load_lds(j) reads inside the store's
//                  LDS for every j below min(k, kLds) rounded up to four)
//   bool widen()     price every column from now on; false if that is already so
// The simplex declares phase II optimal, or phase I infeasible, only after
// widen() returned false (a feasible phase I goes on to phase II on the working
// set), so a store whose working set is the nearest columns (most optimal
// stencils use only those) gives the same certified optimum as pricing all of
// them.
// A store with kCoop spreads the columns over a group of lanes, one each
// (own, x, y, c: this lane's column); every lane of the group runs this
// simplex on the same, replicated state, and the loops over columns become
// one column per lane plus a group reduction:
//   int pick(bool ok, float key)  lowest (key, column) among the lanes with ok, or -1
//   int first(bool ok)            lowest column among the lanes with ok, or -1
//   bool all(bool ok)             every lane of the group has ok
//   void exact_own(df& X, df& Y, df& C)  this lane's exact offset and cost
template <int M, class CS>
struct ThreadSimplex {
    static_assert(M == 3 || M == 5 || M == 9, "3 rows: identity, 5: q = 2, 9: q = 3");
    static constexpr int kQ = M == 3 ? 1 : M == 5 ? 2 : 3;   // order of the cost |r|^(kQ+1)
    float Bi[M][M];   // B^-1
    float xb[M];      // basic values (perturbed rhs)
    float cb[M];      // costs of the basic columns (0 for artificial ones)
    int bs[M];        // basic column of each row; >= 64 means artificial (64 + row)
    uint64_t isb;     // basic structural columns
    uint64_t blk;     // columns blocked until the next pivot (no positive pivot element)
    uint64_t dead;    // columns that do not exist
    int cert_rounds;  // certification rounds taken
    int cert_exact;   // 1 once the double-float dual check ran
    // smallest relative reduced cost d / sc (as d * rcp(sc)) of the last pricing
    // pass that priced every existing non-basic column, none of them blocked,
    // and found none to enter; -inf when the last pass was not such a pass
    mutable float cert_key;

    static constexpr int ART = 64;

    __device__ void init(const LaunchParams& P)
    {
#pragma unroll
        for (int r = 0; r < M; ++r) {
#pragma unroll
            for (int a = 0; a < M; ++a) Bi[r][a] = (r == a) ? 1.0f : 0.0f;
            xb[r] = rhs_hi<M>(r, P) + kPerturb * P.bt_hi * (1.0f + 0.618f * (float)r);
            cb[r] = 0.0f;
            bs[r] = ART + r;
        }
        isb = 0;
        blk = 0;
        cert_key = -__builtin_inff();
    }

    __device__ __forceinline__ void prices(bool phase2, float (&y)[M]) const
    {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            float s = 0.0f;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                float w = phase2 ? cb[r] : (bs[r] >= ART ? 1.0f : 0.0f);
                s = __builtin_fmaf(w, Bi[r][a], s);
            }
            y[a] = s;
        }
    }

    __device__ __forceinline__ void column_alpha(float rx, float ry, float (&alpha)[M]) const
    {
        float v[M];
        mono<M>(rx, ry, v);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            float s = 0.0f;
#pragma unroll
            for (int a = 0; a < M; ++a) s = __builtin_fmaf(Bi[r][a], v[a], s);
            alpha[r] = s;
        }
    }

    // Ratio test (Bland's tie-break: lowest basic index); -1 if no row qualifies.
    __device__ int ratio_test(const float (&alpha)[M], const float (&x)[M], bool phase2) const
    {
        float amax = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) amax = fmaxf(amax, fabsf(alpha[r]));
        float eps = kTolPiv * amax;
        int l = -1, bl = 0;
        float best = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bool art = bs[r] >= ART;
            bool ok;
            float ratio;
            if (phase2 && art && fabsf(alpha[r]) > eps) {
                ok = true;   // a redundant row's artificial must stay at zero: it leaves first
                ratio = 0.0f;
            } else {
                ok = alpha[r] > eps;
                ratio = fmaxf(x[r], 0.0f) * __builtin_amdgcn_rcpf(alpha[r]);
            }
            if (ok && (l < 0 || ratio < best || (ratio == best && bs[r] < bl))) {
                l = r;
                best = ratio;
                bl = bs[r];
            }
        }
        return l;
    }

    __device__ void pivot(int l, int e, const float (&alpha)[M], float ce)
    {
        float al = 1.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) al = (r == l) ? alpha[r] : al;
        float inv = 1.0f / al;
        float row[M];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            float v = 0.0f;
#pragma unroll
            for (int r = 0; r < M; ++r) v = (r == l) ? Bi[r][a] : v;
            row[a] = v * inv;
        }
        float xl = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) xl = (r == l) ? xb[r] : xl;
        xl *= inv;
        int old = 0;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bool me = (r == l);
            old = me ? bs[r] : old;
#pragma unroll
            for (int a = 0; a < M; ++a) Bi[r][a] = me ? row[a] : __builtin_fmaf(-alpha[r], row[a], Bi[r][a]);
            xb[r] = me ? xl : __builtin_fmaf(-alpha[r], xl, xb[r]);
            bs[r] = me ? e : bs[r];
            cb[r] = me ? ce : cb[r];
        }
        if (old < ART) isb &= ~(1ull << old);
        isb |= 1ull << e;
        blk = 0;
    }

    // Crash basis from a prediction: the columns of the M largest logits
    // (slots j < 32 are columns j; a store with KC > 0 columns holds them in
    // cs.lg, otherwise they are read from logit), or the columns of the set
    // pref (use_pref), enter in that order, each replacing the
    // artificial row where its pivot element is largest.  Returns true if the
    // resulting basis is complete and primal feasible (phase II can start).
    __device__ bool crash(const CS& cs, const float* logit, int& piv, bool use_pref = false, uint64_t pref = 0)
    {
        const int kk = cs.k < 32 ? cs.k : 32;
        uint64_t chosen = dead;
        // columns enter by decreasing preference until the basis is complete or
        // the candidates run out (a dependent column is passed over)
        int entered = 0;
        for (int t = 0; t < kk && entered < M; ++t) {
            int best = -1;
            float bl = 0.0f;
            if (use_pref) {
                // a given set of columns (the previous basis), in column order
                const uint64_t left = pref & ~chosen;
                if (left) best = __ffsll((unsigned long long)left) - 1;
            } else if constexpr (CS::KC > 0) {
                // the logits of the columns are in registers
#pragma unroll
                for (int j = 0; j < CS::KC; ++j) {
                    if ((chosen >> j) & 1ull) continue;
                    const float z = cs.lg[j];
                    if (best < 0 || z > bl) {
                        best = j;
                        bl = z;
                    }
                }
            } else {
                for (int j = 0; j < kk; ++j) {
                    if ((chosen >> j) & 1ull) continue;
                    float z = logit[j];
                    if (best < 0 || z > bl) {
                        best = j;
                        bl = z;
                    }
                }
            }
            if (best < 0) break;
            chosen |= 1ull << best;
            float rx, ry, c;
            cs.get(best, rx, ry, c);
            float alpha[M];
            column_alpha(rx, ry, alpha);
            float amax = 0.0f, am = 0.0f;
            int l = -1;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                amax = fmaxf(amax, fabsf(alpha[r]));
                if (bs[r] >= ART && fabsf(alpha[r]) > am) {
                    am = fabsf(alpha[r]);
                    l = r;
                }
            }
            if (l < 0 || am <= 1e-4f * amax) continue;   // dependent on the columns already in
            pivot(l, best, alpha, c);
            ++piv;
            ++entered;
        }
        const float tol = 1e-4f * bt_;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            if (bs[r] >= ART) return false;
            if (xb[r] < -tol) return false;
        }
        return true;
    }

    // Guided phase I from a prediction: from the artificial basis the columns
    // of the M largest logits enter in decreasing order by ordinary phase-I
    // pivots (the ratio test chooses the leaving row), so the basis stays
    // primal feasible whatever the prediction; run(…, 1) then finishes
    // phase I and phase II from it without pricing the entered columns.
    __device__ void guided(const CS& cs, const float* logit, int& piv)
    {
        const int kk = cs.k < 32 ? cs.k : 32;
        uint64_t chosen = dead;
        for (int t = 0; t < M && t < kk; ++t) {
            int best = -1;
            float bl = 0.0f;
            if constexpr (CS::KC > 0) {
#pragma unroll
                for (int j = 0; j < CS::KC; ++j) {
                    if ((chosen >> j) & 1ull) continue;
                    const float z = cs.lg[j];
                    if (best < 0 || z > bl) {
                        best = j;
                        bl = z;
                    }
                }
            } else {
                for (int j = 0; j < kk; ++j) {
                    if ((chosen >> j) & 1ull) continue;
                    const float z = logit[j];
                    if (best < 0 || z > bl) {
                        best = j;
                        bl = z;
                    }
                }
            }
            if (best < 0) break;
            chosen |= 1ull << best;
            float rx, ry, c;
            cs.get(best, rx, ry, c);
            float alpha[M];
            column_alpha(rx, ry, alpha);
            const int l = ratio_test(alpha, xb, false);
            if (l < 0) continue;
            pivot(l, best, alpha, c);
            ++piv;
        }
    }

    // Reduced cost d_j = c_j - y . v_j (phase II; 0 - y . v_j in phase I) and
    // the scale sum |c_j| + sum |y_a v_ja| its tolerance is relative to.
    __device__ __forceinline__ static void reduced(const float (&v)[M], float c, const float (&y)[M], bool p2,
                                                   float& d, float& sc)
    {
        d = p2 ? c : 0.0f;
        sc = fabsf(d);
#pragma unroll
        for (int a = 0; a < M; ++a) {
            d = __builtin_fmaf(-y[a], v[a], d);
            sc = __builtin_fmaf(fabsf(y[a]), fabsf(v[a]), sc);
        }
    }

    // The same for the nine rows of q = 3 by Horner's scheme on the cubic
    // y . v(x, y) = x (y0 + y3 Y + x (y2 + y6 Y + y5 x)) + Y (y1 + Y (y4 + y7 x + y8 Y))
    // (9 operations instead of 7 monomials and 9 products), and its scale from
    // |y| and |x|, |Y| (the |monomials| are the monomials of |x|, |Y|).  p2f is
    // 1 in phase II, 0 in phase I: fma(p2f, c, -p) rounds as (p2 ? c : 0) - p
    // for a finite cost.
    __device__ __forceinline__ static void reduced_horner(float x, float Y, float c, const float (&y)[M],
                                                          const float (&ya)[M], float p2f, float& d, float& sc)
    {
        static_assert(M == 9, "cubic rows");
        const float a = __builtin_fmaf(x, y[5], __builtin_fmaf(Y, y[6], y[2]));
        const float b = __builtin_fmaf(x, a, __builtin_fmaf(Y, y[3], y[0]));
        const float e = __builtin_fmaf(Y, y[8], __builtin_fmaf(x, y[7], y[4]));
        const float g = __builtin_fmaf(Y, e, y[1]);
        const float p = __builtin_fmaf(x, b, Y * g);
        const float ax = fabsf(x), ay = fabsf(Y);
        const float aa = __builtin_fmaf(ax, ya[5], __builtin_fmaf(ay, ya[6], ya[2]));
        const float ab = __builtin_fmaf(ax, aa, __builtin_fmaf(ay, ya[3], ya[0]));
        const float ae = __builtin_fmaf(ay, ya[8], __builtin_fmaf(ax, ya[7], ya[4]));
        const float ag = __builtin_fmaf(ay, ae, ya[1]);
        const float ap = __builtin_fmaf(ax, ab, ay * ag);
        d = __builtin_fmaf(p2f, c, -p);
        sc = __builtin_fmaf(p2f, fabsf(c), ap);
    }

    // Entering column: the columns are taken in groups of four in their order
    // (the complete LPs' lists are nearest first), and the choice is made in
    // the first group that holds an improving column: there, the most
    // negative relative reduced cost d / sc (sc: the magnitude of the terms
    // of d, so the choice does not depend on the rows' or columns' scales).
    // On the 16M-particle q = 3 cloud: 14.2 pivots per LP, against 17.2 for
    // the most negative d / sc over all columns and 26.6 for the most negative
    // d, and most iterations price four columns.  Bland (lowest index) after
    // many iterations.  Every store computes the key d * rcp(sc) the same way,
    // forms the same groups and takes the lowest (key, column) in the group,
    // so all kernels follow the same path.
    __device__ __forceinline__ int price(const CS& cs, const float (&y)[M], bool p2, bool bland) const
    {
        const uint64_t excl = isb | blk | dead;
        int e = -1;
        float best = 0.0f;
        auto consider = [&](int j, float d, float sc) -> bool {
            if (!(d < -kTolD * sc)) return false;
            if (bland) {
                e = j;
                return true;
            }
            const float key = d * __builtin_amdgcn_rcpf(sc);
            if (e < 0 || key < best) {
                e = j;
                best = key;
            }
            return false;
        };
        if constexpr (CS::kCoop) {
            // this lane's column, then the group's choice: Bland's first
            // qualifying column, or the first of the most negative d / sc
            float v[M];
            mono<M>(cs.x, cs.y, v);
            float d, sc;
            reduced(v, cs.c, y, p2, d, sc);
            const bool ok = !((excl >> cs.own) & 1ull) && d < -kTolD * sc;
            // the first group of four columns with an improving one
            const int f = cs.first(ok);
            const bool in_group = ok && (cs.own >> 2) == (f >> 2);
            return cs.pick(in_group, bland ? 0.0f : d * __builtin_amdgcn_rcpf(sc));
        } else if constexpr (CS::KC > 0) {
            // compile-time column count: the loop is unrolled
#pragma unroll
            for (int j = 0; j < CS::KC; ++j) {
                if ((j & 3) == 0 && e >= 0) break;   // a group of four held an improving column
                if ((excl >> j) & 1ull) continue;
                float rx, ry, c;
                cs.get(j, rx, ry, c);
                float v[M];
                mono<M>(rx, ry, v);
                float d, sc;
                reduced(v, c, y, p2, d, sc);
                if (consider(j, d, sc)) break;
            }
        } else {
            // Four columns per iteration (their reads issued together), with
            // selects rather than branches.  A qualifying column has a negative
            // key (d < -kTolD sc), so with best starting at 0 "no column yet"
            // needs no test of its own; Bland's rule (the first qualifying
            // column) gives every column the key -1, which only the first
            // one beats.
            const int k = cs.active();
            float ya[M];
#pragma unroll
            for (int a = 0; a < M; ++a) ya[a] = fabsf(y[a]);
            const float p2f = p2 ? 1.0f : 0.0f;
            // the columns past the k are excluded with the others
            const uint64_t out = k < 64 ? excl | (~0ull << k) : excl;
            float mk = __builtin_inff();   // smallest key of the priced columns
            auto column = [&](int j, bool in, float rx, float ry, uint32_t aux) {
                const float c = cs.template cost_of<kQ>(rx, ry, aux);
                float d, sc;
                if constexpr (M == 9) {
                    reduced_horner(rx, ry, c, y, ya, p2f, d, sc);
                } else {
                    float v[M];
                    mono<M>(rx, ry, v);
                    reduced(v, c, y, p2, d, sc);
                }
                const float kraw = d * __builtin_amdgcn_rcpf(sc);
                const float key = bland ? -1.0f : kraw;
                mk = fminf(mk, in ? kraw : __builtin_inff());
                if (in && d < -kTolD * sc && key < best) {
                    e = j;
                    best = key;
                }
            };
            // the columns a store keeps in LDS (all, or its working set): whole
            // groups of four, read without clamping (the rows past the k
            // columns hold stale values, which `out` excludes); then the rest
            static_assert(CS::kLds % 4 == 0, "a store's LDS rows come in groups of four");
            const int k1 = min(k, CS::kLds);
            for (int j0 = 0; j0 < k1; j0 += 4) {
                float rx[4], ry[4];
                uint32_t aux[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) cs.load_lds(j0 + u, rx[u], ry[u], aux[u]);
                const uint32_t ex4 = (uint32_t)(out >> j0);
#pragma unroll
                for (int u = 0; u < 4; ++u) column(j0 + u, !(ex4 & (1u << u)), rx[u], ry[u], aux[u]);
                if (e >= 0) break;   // this group holds an improving column (Bland: its first)
            }
            for (int j0 = k1; j0 < k; j0 += 4) {
                if (e >= 0) break;
                float rx[4], ry[4];
                uint32_t aux[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) cs.load(min(j0 + u, k - 1), rx[u], ry[u], aux[u]);
                const uint32_t ex4 = (uint32_t)(out >> j0);
#pragma unroll
                for (int u = 0; u < 4; ++u) column(j0 + u, !(ex4 & (1u << u)), rx[u], ry[u], aux[u]);
            }
            // a pass over every column (the whole list, nothing blocked) that found
            // none to enter leaves its smallest key to the fast certificate
            cert_key = (e < 0 && blk == 0 && k == cs.k) ? mk : -__builtin_inff();
        }
        return e;
    }

    // FP32 simplex from phase `first` (1: two phases from the artificial basis,
    // 2: phase II from a feasible basis).  0 optimal, 1 infeasible, 2 iteration
    // limit (cap >= 0: at most cap iterations per phase).  Both phases share one
    // loop, so the lanes of a wave step through their own phases together.
    // With acc (phase I only): at the end of phase I the vertex is offered to
    // accept_phase1 (refined basic values into *x); if taken, *accepted is set
    // and run returns 0, else phase II continues.
    // first = 3: phase I from a crash basis that is not primal feasible, by the
    // sum of infeasibilities (the composite method): the objective is the sum of
    // the negative basic values' magnitudes plus the positive artificial
    // values, priced like phase I; the entering column leaves at the first
    // breakpoint (a feasible row that reaches zero, or an infeasible one that
    // climbs to zero), so the objective never grows, and it carries its cost,
    // so phase II starts on the feasible basis this ends on.  Returns 3 if no
    // column improves the infeasibility (the caller then solves cold).
    __device__ int run(const CS& cs, int& piv, int first, int cap = -1, const LaunchParams* acc = nullptr,
                       df* x = nullptr, bool* accepted = nullptr)
    {
        const int k = cs.k;
        const int bland_after = 3 * (k + M);
        const int limit = cap >= 0 ? cap : 10 * (k + M) + 20;
        bool p2 = first == 2;
        bool comp = first == 3;
        const float ctol = 1e-5f * bt_;
        for (int it = 0;; ++it) {
            if (it >= limit) return 2;
            float y[M];
            if (comp) {
                float w[M];
                bool any = false;
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    w[r] = xb[r] < -ctol ? -1.0f : ((bs[r] >= ART && xb[r] > ctol) ? 1.0f : 0.0f);
                    any = any || w[r] != 0.0f;
                }
                if (!any) {
                    // feasible: phase II from here (or, phase I only, this vertex)
                    comp = false;
                    p2 = true;
                    blk = 0;
                    it = -1;
                    if (acc && accept_phase1(cs, *acc, *reinterpret_cast<df(*)[M]>(x))) {
                        *accepted = true;
                        return 0;
                    }
                    continue;
                }
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    float t = 0.0f;
#pragma unroll
                    for (int r = 0; r < M; ++r) t = __builtin_fmaf(w[r], Bi[r][a], t);
                    y[a] = t;
                }
            } else {
                prices(p2, y);
            }
            const int e = price(cs, y, p2, it >= bland_after);
            if (e < 0) {
                if (comp) {
                    if (cs.widen()) continue;
                    return 3;
                }
                // a working set of columns (sifting) is widened to every column
                // when it is done: at the end of phase II, or at the end of a
                // phase I that found it infeasible; a feasible phase I goes on
                // to phase II on the working set
                if (p2) {
                    if (cs.widen()) continue;
                    return 0;
                }
                // end of phase I: feasible iff the artificial variables vanished
                float art = 0.0f;
#pragma unroll
                for (int r = 0; r < M; ++r) art += bs[r] >= ART ? fabsf(xb[r]) : 0.0f;
                if (art > kTolFeas * P_bt()) {
                    if (cs.widen()) continue;
                    return 1;
                }
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    float c = 0.0f;
                    if (bs[r] < ART) {
                        float rx, ry;
                        cs.get(bs[r], rx, ry, c);
                    }
                    cb[r] = c;
                }
                blk = 0;
                p2 = true;
                it = -1;
                if (acc && accept_phase1(cs, *acc, *reinterpret_cast<df(*)[M]>(x))) {
                    *accepted = true;
                    return 0;
                }
                continue;
            }
            float rx, ry, ce;
            cs.get(e, rx, ry, ce);
            float alpha[M];
            column_alpha(rx, ry, alpha);
            const int l = comp ? ratio_composite(alpha, ctol) : ratio_test(alpha, xb, p2);
            if (l < 0) {
                blk |= 1ull << e;
                continue;
            }
            pivot(l, e, alpha, (p2 || comp) ? ce : 0.0f);
            ++piv;
        }
    }

    // ratio test of the composite phase I: the first breakpoint (lowest basic
    // index among equal ratios); -1 if none
    __device__ int ratio_composite(const float (&alpha)[M], float tol) const
    {
        float amax = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) amax = fmaxf(amax, fabsf(alpha[r]));
        const float eps = kTolPiv * amax;
        int l = -1, bl = 0;
        float best = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const bool neg = xb[r] < -tol;
            const bool ok = neg ? alpha[r] < -eps : alpha[r] > eps;
            const float ratio = (neg ? xb[r] : fmaxf(xb[r], 0.0f)) * __builtin_amdgcn_rcpf(alpha[r]);
            if (ok && (l < 0 || ratio < best || (ratio == best && bs[r] < bl))) {
                l = r;
                best = ratio;
                bl = bs[r];
            }
        }
        return l;
    }

    float bt_;
    __device__ __forceinline__ float P_bt() const { return bt_; }

    // exact B x for the basic solution, residual b - B x
    __device__ void primal_residual(const CS& cs, const df (&x)[M], const LaunchParams& P, float (&res)[M]) const
    {
        df acc[M];
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] = {0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < M; ++r) {
            int b = bs[r];
            if (b < ART) {
                df X, Y;
                cs.exact_xy(b, X, Y);
                df v[M];
                mono_df<M>(X, Y, v);
#pragma unroll
                for (int a = 0; a < M; ++a) acc[a] = df_add(acc[a], df_mul(v[a], x[r]));
            } else {
#pragma unroll
                for (int a = 0; a < M; ++a)
                    if (b - ART == a) acc[a] = df_add(acc[a], x[r]);
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) {
            df rr = df_add(rhs_df<M>(a, P), df_neg(acc[a]));
            res[a] = rr.hi + rr.lo;
        }
    }

    // exact c_B - B^T y, per basis row
    __device__ void dual_residual(const CS& cs, const df (&y)[M], float (&res)[M]) const
    {
#pragma unroll
        for (int r = 0; r < M; ++r) {
            int b = bs[r];
            df s{0.0f, 0.0f};
            if (b < ART) {
                df X, Y, C;
                cs.exact(b, X, Y, C);
                df v[M];
                mono_df<M>(X, Y, v);
                s = C;
#pragma unroll
                for (int a = 0; a < M; ++a) s = df_add(s, df_neg(df_mul(v[a], y[a])));
            } else {
#pragma unroll
                for (int a = 0; a < M; ++a)
                    if (b - ART == a) s = df_neg(y[a]);
            }
            res[r] = s.hi + s.lo;
        }
    }

    // Basic solution of the current basis for the exact right-hand side, refined
    // with double-float residuals; returns |first correction| / |x| (how far
    // B^-1 is from the exact inverse).  One refinement step multiplies the
    // error by about that ratio (the error of x0 = B^-1 b is B^-1's error, and
    // the step leaves (I - B^-1 B) times it), so a first correction below
    // 2^-20 of x leaves x accurate to about 2^-40 of x, far below the 1e-9
    // of the certified decisions: no second residual is formed to confirm it.
    __device__ float refine_primal(const CS& cs, const LaunchParams& P, df (&x)[M]) const
    {
#pragma unroll
        for (int r = 0; r < M; ++r) {
            float v = 0.0f;
#pragma unroll
            for (int a = 0; a < M; ++a) v += rhs_row<M>(a) ? Bi[r][a] : 0.0f;
            x[r] = {v * P.bt_hi, 0.0f};
        }
        float first_corr = 1.0f;
        for (int it = 0; it < kMaxRefine; ++it) {
            float res[M];
            primal_residual(cs, x, P, res);
            float dmax = 0.0f, xmax = 0.0f;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                float d = 0.0f;
#pragma unroll
                for (int a = 0; a < M; ++a) d = __builtin_fmaf(Bi[r][a], res[a], d);
                x[r] = df_add(x[r], df{d, 0.0f});
                dmax = fmaxf(dmax, fabsf(d));
                xmax = fmaxf(xmax, fabsf(x[r].hi));
            }
            if (it == 0) first_corr = dmax / fmaxf(xmax, 1e-30f);
            if (dmax <= 9.313225746154785e-10f * xmax || (it == 0 && first_corr <= 9.5367431640625e-07f)) break;
        }
        return first_corr;
    }

    // Phase I only (Sec. 4.1: the first feasible vertex): the refined basic
    // solution is accepted if every structural basic value is >= -1e-9 and
    // every artificial one has vanished.
    __device__ bool accept_phase1(const CS& cs, const LaunchParams& P, df (&x)[M]) const
    {
        refine_primal(cs, P, x);
        bool ok = true;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float v = x[r].hi + x[r].lo;
            ok = ok && (bs[r] < ART ? !(v < -kCertX) : !(fabsf(v) > kCertX));
        }
        return ok;
    }

    // Certify against the exact problem, repairing the basis if needed.
    // 0 optimal, 1 infeasible, 3 not certified; with `defer`, 5 when the first
    // round's fast certificate does not settle it (the basis is left as it is
    // for a later call without `defer`).  x receives the basic values
    // of the final basis (refined for it, also after a last repair pivot).
    __device__ int certify(const CS& cs, const LaunchParams& P, df (&x)[M], int& piv, bool defer = false)
    {
        const int k = cs.k;
        for (int round = 0; round < P.max_cert; ++round) {
            ++cert_rounds;
            const float first_corr = refine_primal(cs, P, x);
            // An artificial variable still basic must vanish in the exact basic
            // solution; one that does not means phase I ended, within its FP32
            // tolerance, on a vertex that is not feasible: the LP is taken as
            // infeasible (its exact phase-I optimum is positive).
#pragma unroll
            for (int r = 0; r < M; ++r)
                if (bs[r] >= ART && fabsf(x[r].hi + x[r].lo) > kCertX) return 1;
            // Fast certificate: when B^-1 is accurate (the first correction is
            // tiny) and every FP32 reduced cost clears zero by 64 times its error
            // bound, the basis is optimal without the double-float dual check.
            if (first_corr <= 1e-5f) {
                // |d - d_exact| <= (error of B^-1 + FP32 rounding) x sc; the error of
                // B^-1 is about the first correction
                const float margin = kFastMargin * (first_corr + 1.1920929e-07f);
                bool primal_ok = true;
#pragma unroll
                for (int r = 0; r < M; ++r)
                    if (bs[r] < ART && x[r].hi + x[r].lo < -kCertX) primal_ok = false;
                if (primal_ok) {
                    float yf[M];
                    prices(true, yf);
                    bool dual_ok = true;
                    const uint64_t excl = isb | dead;
                    if constexpr (CS::kCoop) {
                        float v[M];
                        mono<M>(cs.x, cs.y, v);
                        float d, sc;
                        reduced(v, cs.c, yf, true, d, sc);
                        dual_ok = cs.all(((excl >> cs.own) & 1ull) || !(d < margin * sc));
                    } else if constexpr (CS::KC > 0) {
#pragma unroll
                        for (int j = 0; j < CS::KC; ++j) {
                            if ((excl >> j) & 1ull) continue;
                            float rx, ry, c;
                            cs.get(j, rx, ry, c);
                            float v[M];
                            mono<M>(rx, ry, v);
                            float d, sc;
                            reduced(v, c, yf, true, d, sc);
                            dual_ok = dual_ok && !(d < margin * sc);
                        }
                    } else if (round == 0 && cert_key >= margin * 1.00000095367431640625f) {
                        // the last pricing pass of the simplex priced every column with
                        // these prices (no pivot since) and its smallest d * rcp(sc)
                        // clears the margin by more than the reciprocal's error
                        dual_ok = true;
                    } else {
                        auto column = [&](int j, bool in, float rx, float ry, uint32_t aux) {
                            const float c = cs.template cost_of<kQ>(rx, ry, aux);
                            float v[M];
                            mono<M>(rx, ry, v);
                            float d, sc;
                            reduced(v, c, yf, true, d, sc);
                            dual_ok = dual_ok && (!in || ((excl >> j) & 1ull) || !(d < margin * sc));
                        };
                        const int k1 = min(k, CS::kLds);
                        for (int j0 = 0; j0 < k1; j0 += 4) {
                            float rx[4], ry[4];
                            uint32_t aux[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) cs.load_lds(min(j0 + u, k1 - 1), rx[u], ry[u], aux[u]);
#pragma unroll
                            for (int u = 0; u < 4; ++u) column(j0 + u, j0 + u < k1, rx[u], ry[u], aux[u]);
                        }
                        for (int j0 = k1; j0 < k; j0 += 4) {
                            float rx[4], ry[4];
                            uint32_t aux[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) cs.load(min(j0 + u, k - 1), rx[u], ry[u], aux[u]);
#pragma unroll
                            for (int u = 0; u < 4; ++u) column(j0 + u, j0 + u < k, rx[u], ry[u], aux[u]);
                        }
                    }
                    if (dual_ok) return 0;
                }
            }
            if (defer && round == 0) return 5;
            cert_exact = 1;
            float yf[M];
            prices(true, yf);
            df y[M];
#pragma unroll
            for (int a = 0; a < M; ++a) y[a] = {yf[a], 0.0f};
            for (int it = 0; it < kMaxRefine; ++it) {
                float res[M];
                dual_residual(cs, y, res);
                float dmax = 0.0f, ymax = 0.0f;
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    float d = 0.0f;
#pragma unroll
                    for (int r = 0; r < M; ++r) d = __builtin_fmaf(Bi[r][a], res[r], d);
                    y[a] = df_add(y[a], df{d, 0.0f});
                    dmax = fmaxf(dmax, fabsf(d));
                    ymax = fmaxf(ymax, fabsf(y[a].hi));
                }
                if (dmax <= 9.313225746154785e-10f * ymax) break;
            }
            // primal feasibility of the exact basic solution
            int lrow = -1;
            float xmin = -kCertX;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                float v = x[r].hi + x[r].lo;
                if (bs[r] < ART && v < xmin) {
                    xmin = v;
                    lrow = r;
                }
            }
            if (lrow >= 0) {
                // dual repair: row lrow leaves, the entering column by the dual ratio test
                float wrow[M];
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    float v = 0.0f;
#pragma unroll
                    for (int r = 0; r < M; ++r) v = (r == lrow) ? Bi[r][a] : v;
                    wrow[a] = v;
                }
                int e = -1;
                float best = 0.0f;
                // the dual ratio of column j (w: its entry in row lrow of B^-1 V)
                auto dual_ratio = [&](const df& X, const df& Y, const df& C, float& ratio) -> bool {
                    df v[M];
                    mono_df<M>(X, Y, v);
                    float w = 0.0f;
                    df s = C;
#pragma unroll
                    for (int a = 0; a < M; ++a) {
                        w = __builtin_fmaf(wrow[a], v[a].hi, w);
                        s = df_add(s, df_neg(df_mul(v[a], y[a])));
                    }
                    ratio = w < -kTolPiv ? fmaxf(s.hi + s.lo, 0.0f) / (-w) : 0.0f;
                    return w < -kTolPiv;
                };
                if constexpr (CS::kCoop) {
                    df X, Y, C;
                    cs.exact_own(X, Y, C);
                    float ratio;
                    const bool ok = dual_ratio(X, Y, C, ratio) && !(((isb | dead) >> cs.own) & 1ull);
                    e = cs.pick(ok, ratio);
                } else {
                    for (int j = 0; j < k; ++j) {
                        if (((isb | dead) >> j) & 1ull) continue;
                        df X, Y, C;
                        cs.exact(j, X, Y, C);
                        float ratio;
                        if (dual_ratio(X, Y, C, ratio) && (e < 0 || ratio < best)) {
                            e = j;
                            best = ratio;
                        }
                    }
                }
                if (e < 0) return 1;
                float rx, ry, ce;
                cs.get(e, rx, ry, ce);
                float alpha[M];
                column_alpha(rx, ry, alpha);
                pivot(lrow, e, alpha, ce);
                ++piv;
                continue;
            }
            // exact reduced costs; Bland's entering column
            int e = -1;
            // exact reduced cost of column j below its tolerance
            auto negative = [&](const df& X, const df& Y, const df& C) -> bool {
                df v[M];
                mono_df<M>(X, Y, v);
                df s = C;
                float sc = fabsf(C.hi);
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    df p = df_mul(v[a], y[a]);
                    s = df_add(s, df_neg(p));
                    sc += fabsf(p.hi);
                }
                return s.hi + s.lo < -kCertD * sc;
            };
            if constexpr (CS::kCoop) {
                df X, Y, C;
                cs.exact_own(X, Y, C);
                e = cs.first(!(((isb | dead) >> cs.own) & 1ull) && negative(X, Y, C));
            } else {
                for (int j = 0; j < k && e < 0; ++j) {
                    if (((isb | dead) >> j) & 1ull) continue;
                    df X, Y, C;
                    cs.exact(j, X, Y, C);
                    if (negative(X, Y, C)) e = j;
                }
            }
            if (e < 0) return 0;
            float rx, ry, ce;
            cs.get(e, rx, ry, ce);
            float alpha[M], xf[M];
            column_alpha(rx, ry, alpha);
#pragma unroll
            for (int r = 0; r < M; ++r) xf[r] = x[r].hi + x[r].lo;
            int l = ratio_test(alpha, xf, true);
            if (l < 0) return 3;
            pivot(l, e, alpha, ce);
            ++piv;
        }
        // out of rounds right after a repair pivot: the values of the basis now held
        refine_primal(cs, P, x);
        return 3;
    }

    // The refined basic solution satisfies the constraints: every structural
    // value >= -kCertX and every artificial one vanished (a basis whose
    // optimality could not be certified is kept only then).
    __device__ bool primal_feasible(const df (&x)[M]) const
    {
        bool ok = true;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            const float v = x[r].hi + x[r].lo;
            ok = ok && (bs[r] < ART ? !(v < -kCertX) : !(fabsf(v) > kCertX));
        }
        return ok;
    }
};

// Solve, certify and extract the fractions: f (k entries, written through
// store(j, value) for the non-zero ones) and fii = -sum f.
// Returns 0 ok, 1 infeasible, 4 left for a cold solve (warm pass), 5 the
// certification deferred (`defer`: the fast certificate did not settle the
// optimum; nothing is stored and `basis` holds the basic columns);
// *certified = 0 if optimality could not be shown.
// Warm pass (warm_pass): the simplex starts from the crash basis of the
// prediction (logits of the first 32 columns, or the column set pref with
// use_pref); a rejected crash basis, or one that needs more than warm_cap<M>()
// phase-II pivots, is given up (status 4) -- except a network's prediction
// for a 9-row LP, which is always finished in the pass (a rejected crash
// basis becomes a guided phase I, no pivot cap).  basis: the final basic
// columns.  warm = 0 cold, 1 the predicted basis was optimal, 2 phase I/II
// from it, 3 given up.
// phase-II pivots allowed from a predicted basis in the warm pass: a few for
// 5-row LPs (a cold solve takes ~8), more for 9-row ones (~30)
template <int M>
constexpr int warm_cap() { return M == 5 ? 3 : 12; }

// Non-negative least squares (Sec. 4.1's alternative: min_{f >= 0} |V f - b|^2,
// Lawson and Hanson's active-set method) in FP32 to find the stencil's support:
// free the column with the largest negative gradient w_j = v_j . (b - V f) (the
// lowest index among equal ones, relative tolerance kTolD), solve the
// unconstrained least squares on the free columns (Householder QR, at most M
// of them), step back towards it and fix again the entries that reach zero while
// it has a non-positive entry.  The support's exact values then come from the
// double-float refinement of the basis it spans (the columns enter the
// artificial basis by their largest pivot element); a support whose exact
// values are not a non-negative solution of the moment conditions counts as
// infeasible.  Returns 0 or 1 as solve_lp.
// Columns of the least-squares problem in the paper's units: monomials of the
// offset over h (the stored offsets are over 2^e = s h), right-hand side 2 at
// the second-order rows.  The simplex may scale rows (it does not change the
// solution set); least squares may not (row weights change the path).
template <int M, class CS>
__device__ __forceinline__ void nnls_column(const CS& cs, const LaunchParams& P, int j, float (&v)[M])
{
    float rx, ry, cc;
    cs.get(j, rx, ry, cc);
    mono<M>(rx * P.sc, ry * P.sc, v);
}
template <int M>
__device__ __forceinline__ float nnls_rhs(int a) { return rhs_row<M>(a) ? 2.0f : 0.0f; }

// Unconstrained least squares on the free columns set[0..p) (Householder QR);
// false if a column is (numerically) dependent on the ones before it.
template <int M, class CS>
__device__ bool nnls_least_squares(const CS& cs, const LaunchParams& P, const int (&set)[M], int p, float (&z)[M])
{
    float Q[M][M], c[M];
#pragma unroll
    for (int a = 0; a < M; ++a) c[a] = nnls_rhs<M>(a);
#pragma unroll
    for (int t = 0; t < M; ++t) {
        float v[M];
        if (t < p) {
            nnls_column<M>(cs, P, set[t], v);
        } else {
#pragma unroll
            for (int a = 0; a < M; ++a) v[a] = 0.0f;
        }
#pragma unroll
        for (int a = 0; a < M; ++a) Q[a][t] = v[a];
    }
    float scale = 0.0f;
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
        for (int t = 0; t < M; ++t) scale = fmaxf(scale, fabsf(Q[a][t]));
    bool ok = true;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        if (t >= p) continue;
        float nrm = 0.0f;
#pragma unroll
        for (int a = 0; a < M; ++a) nrm = a >= t ? __builtin_fmaf(Q[a][t], Q[a][t], nrm) : nrm;
        nrm = __builtin_sqrtf(nrm);
        ok = ok && nrm > 1e-6f * scale;
        const float alpha = Q[t][t] > 0.0f ? -nrm : nrm;
        float v[M];
#pragma unroll
        for (int a = 0; a < M; ++a) v[a] = a < t ? 0.0f : Q[a][t];
        v[t] -= alpha;
        float vv = 0.0f;
#pragma unroll
        for (int a = 0; a < M; ++a) vv = __builtin_fmaf(v[a], v[a], vv);
        const float inv = vv > 0.0f ? 2.0f / vv : 0.0f;
#pragma unroll
        for (int u = 0; u < M; ++u) {
            if (u < t || u >= p) continue;
            float sd = 0.0f;
#pragma unroll
            for (int a = 0; a < M; ++a) sd = __builtin_fmaf(v[a], Q[a][u], sd);
            sd *= inv;
#pragma unroll
            for (int a = 0; a < M; ++a) Q[a][u] = __builtin_fmaf(-sd, v[a], Q[a][u]);
        }
        float sd = 0.0f;
#pragma unroll
        for (int a = 0; a < M; ++a) sd = __builtin_fmaf(v[a], c[a], sd);
        sd *= inv;
#pragma unroll
        for (int a = 0; a < M; ++a) c[a] = __builtin_fmaf(-sd, v[a], c[a]);
    }
#pragma unroll
    for (int t = M - 1; t >= 0; --t) {
        float sd = c[t];
#pragma unroll
        for (int u = t + 1; u < M; ++u) sd = u < p ? __builtin_fmaf(-Q[t][u], z[u], sd) : sd;
        z[t] = t < p ? sd / Q[t][t] : 0.0f;
    }
    return ok;
}

template <int M, class CS, class Store>
__device__ int solve_nnls(const CS& cs, const LaunchParams& P, Store store, float& fii, int& piv, int& certified,
                          uint64_t& basis)
{
    const int k = cs.k;
    int set[M];
    float fz[M];
#pragma unroll
    for (int t = 0; t < M; ++t) {
        set[t] = 0;
        fz[t] = 0.0f;
    }
    int p = 0;
    uint64_t inP = 0;
    uint64_t tabu = 0;   // freed columns whose least-squares value came out <= 0 (FP32 rounding)
    basis = 0;
    certified = 1;
    fii = 0.0f;
    // first pass: stop once the free columns reproduce b to FP32 accuracy; if
    // the exact values on that support are not a solution (a column with a
    // tiny share is still missing), go on until no gradient is positive
    bool res_stop = true;
    ThreadSimplex<M, CS> lp;
    df x[M];
    for (int pass = 0; pass < 2; ++pass) {
        bool stopped_by_residual = false;
        for (int outer = 0; outer < 3 * M + 8; ++outer) {
            // residual of the current point and the column with the largest negative gradient
            float r[M];
#pragma unroll
            for (int a = 0; a < M; ++a) r[a] = nnls_rhs<M>(a);
#pragma unroll
            for (int t = 0; t < M; ++t) {
                if (t >= p) continue;
                float v[M];
                nnls_column<M>(cs, P, set[t], v);
#pragma unroll
                for (int a = 0; a < M; ++a) r[a] = __builtin_fmaf(-fz[t], v[a], r[a]);
            }
            float rmax = 0.0f;
#pragma unroll
            for (int a = 0; a < M; ++a) rmax = fmaxf(rmax, fabsf(r[a]));
            if (res_stop && p > 0 && rmax <= 2.0f * kNnlsRes) {
                stopped_by_residual = true;
                break;
            }
            int best = -1;
            float wbest = 0.0f;
            for (int j = 0; j < k; ++j) {
                if (((inP | cs.dead | tabu) >> j) & 1ull) continue;
                float v[M];
                nnls_column<M>(cs, P, j, v);
                float w = 0.0f, sc = 0.0f;
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    w = __builtin_fmaf(v[a], r[a], w);
                    sc = __builtin_fmaf(fabsf(v[a]), fabsf(r[a]), sc);
                }
                if (w > kTolD * sc && w > wbest) {
                    best = j;
                    wbest = w;
                }
            }
            if (best < 0 || p == M) break;
#pragma unroll
            for (int t = 0; t < M; ++t)
                if (t == p) {
                    set[t] = best;
                    fz[t] = 0.0f;
                }
            ++p;
            ++piv;
            inP |= 1ull << best;
            for (int inner = 0; inner < M + 2 && p > 0; ++inner) {
                float z[M];
                if (!nnls_least_squares<M>(cs, P, set, p, z)) return 1;
                if (inner == 0) {
                    // in exact arithmetic the freed column's value is positive; if
                    // rounding says otherwise it is fixed again and not freed until
                    // another column has been
                    float znew = 0.0f;
#pragma unroll
                    for (int t = 0; t < M; ++t) znew = t == p - 1 ? z[t] : znew;
                    if (!(znew > 0.0f)) {
                        --p;
                        inP &= ~(1ull << best);
                        tabu |= 1ull << best;
                        break;
                    }
                    tabu = 0;
                }
                bool allpos = true;
#pragma unroll
                for (int t = 0; t < M; ++t) allpos = allpos && (t >= p || z[t] > 0.0f);
                if (allpos) {
#pragma unroll
                    for (int t = 0; t < M; ++t) fz[t] = t < p ? z[t] : 0.0f;
                    break;
                }
                // step from the current point towards z until the first entry
                // reaches zero, and fix the entries at zero again (order kept)
                float alpha = 1.0f;
                int tmin = -1;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    if (t < p && z[t] <= 0.0f) {
                        const float a = fz[t] / (fz[t] - z[t]);
                        if (tmin < 0 || a < alpha) {
                            alpha = a;
                            tmin = t;
                        }
                    }
                }
                alpha = fminf(alpha, 1.0f);
                int q = 0;
                int nset[M];
                float nf[M];
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    nset[t] = 0;
                    nf[t] = 0.0f;
                }
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    if (t >= p) continue;
                    const float v = __builtin_fmaf(alpha, z[t] - fz[t], fz[t]);
                    if (t == tmin || v <= 1e-7f * P.bt_hi) {
                        inP &= ~(1ull << set[t]);
                    } else {
#pragma unroll
                        for (int u = 0; u < M; ++u)
                            if (u == q) {
                                nset[u] = set[t];
                                nf[u] = v;
                            }
                        ++q;
                    }
                }
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    set[t] = nset[t];
                    fz[t] = nf[t];
                }
                p = q;
            }
        }
        if (p == 0) return 1;
        // exact values on the support: its columns enter the artificial basis
        // (each where its pivot element is largest), then the double-float
        // refinement of the basic solution
        lp.bt_ = P.bt_hi;
        lp.init(P);
        lp.dead = cs.dead;
        lp.cert_rounds = 0;
        lp.cert_exact = 0;
        int cp = 0;
        lp.crash(cs, nullptr, cp, true, inP);
        if (lp.accept_phase1(cs, P, x)) break;
        if (!stopped_by_residual) return 1;
        res_stop = false;
    }
    float sum = 0.0f, v[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        const float t = x[r].hi + x[r].lo;
        v[r] = (lp.bs[r] < lp.ART && t > 0.0f) ? t : 0.0f;
        sum += v[r];
    }
    const float tiny = 9.313225746154785e-10f * sum;
    sum = 0.0f;
#pragma unroll
    for (int r = 0; r < M; ++r) {
        v[r] = v[r] < tiny ? 0.0f : v[r];
        sum += v[r];
        if (v[r] != 0.0f) store(lp.bs[r], v[r]);
    }
    fii = -sum;
#pragma unroll
    for (int r = 0; r < M; ++r)
        if (lp.bs[r] < lp.ART) basis |= 1ull << lp.bs[r];
    return 0;
}

// OBJ: 0 the canonical stencil; 1 phase I only (the first feasible vertex,
// P.phase1 = 1); 2 non-negative least squares (P.phase1 = 2).  Each
// instantiation carries only its own code.
// WARM: the warm-pass code compiled in (a kernel that never runs a warm pass
// leaves it out, and with it its registers).
// The end of a simplex solve (run's result st): certification against the
// exact problem, the basic values as fractions (stored with store(column,
// value)), fii = -their sum, and the final basis.  Returns solve_lp's result.
template <int M, class CS, class Store>
__device__ int finish_lp(ThreadSimplex<M, CS>& lp, const CS& cs, const LaunchParams& P, Store store, int st,
                         bool accepted, df (&x)[M], float& fii, int& piv, int& certified, uint64_t& basis, int* stats,
                         bool defer = false)
{
    certified = 1;
    if (st == 1) return 1;
    const int c = accepted ? 0 : lp.certify(cs, P, x, piv, defer);
    if (stats) {
        stats[0] = lp.cert_rounds;
        stats[1] = lp.cert_exact;
    }
    if (c == 1) return 1;
    if (c == 5) {
        // deferred: the caller keeps the basis's columns for the later certification
#pragma unroll
        for (int r = 0; r < M; ++r)
            if (lp.bs[r] < lp.ART) basis |= 1ull << lp.bs[r];
        return 5;
    }
    // not certified optimal: kept only if its exact values meet the moment
    // conditions and the sign condition, else treated as infeasible
    if (c == 3 && !lp.primal_feasible(x)) return 1;
    certified = c == 0 ? 1 : 0;
    float sum = 0.0f;
    float v[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        float t = x[r].hi + x[r].lo;
        v[r] = (lp.bs[r] < lp.ART && t > 0.0f) ? t : 0.0f;
        sum += v[r];
    }
    // a basic value below 2^-30 of the stencil's sum is the round-off of a
    // degenerate vertex (zero in exact arithmetic): make it zero
    float tiny = 9.313225746154785e-10f * sum;
    sum = 0.0f;
#pragma unroll
    for (int r = 0; r < M; ++r) {
        v[r] = v[r] < tiny ? 0.0f : v[r];
        sum += v[r];
        if (v[r] != 0.0f) store(lp.bs[r], v[r]);
    }
    fii = -sum;
#pragma unroll
    for (int r = 0; r < M; ++r)
        if (lp.bs[r] < lp.ART) basis |= 1ull << lp.bs[r];
    return 0;
}

// INPLACE (warm passes): a prediction that is given up (warm = 3) is followed by
// the cold solve in the same call instead of returning 4; the store's
// restart() resets what the warm attempt changed in it (a widened working set).
template <int M, int OBJ, bool WARM = true, bool INPLACE = false, class CS, class Store>
__device__ int solve_lp(const CS& cs, const LaunchParams& P, Store store, float& fii, int& piv, int& certified,
                        bool warm_pass_arg, const float* logit, int& warm, uint64_t& basis, bool use_pref = false,
                        uint64_t pref = 0, int* stats = nullptr, bool capped = true, bool defer = false)
{
    if constexpr (OBJ == 2) {
        warm = 0;
        if (stats) stats[0] = stats[1] = 0;
        return solve_nnls<M>(cs, P, store, fii, piv, certified, basis);
    }
    constexpr bool PH1 = OBJ == 1;
    const bool warm_pass = WARM && warm_pass_arg;
    ThreadSimplex<M, CS> lp;
    lp.bt_ = P.bt_hi;
    lp.init(P);
    lp.dead = cs.dead;
    lp.cert_rounds = 0;
    lp.cert_exact = 0;
    if (stats) stats[0] = stats[1] = 0;
    int st;
    warm = 0;
    basis = 0;
    df x[M];
    bool accepted = false;   // phase I only: the first feasible vertex, exact to the refinement
    if constexpr (WARM && INPLACE) {
        // One simplex call site for the whole LP: phase II from the crash basis
        // if it is feasible, else the composite phase I from it (phase-I-only
        // objective: always, it accepts the first feasible vertex); a warm
        // attempt that fails (no improving column, or the pivot cap when
        // `capped`) is followed by the cold solve.
        int first = 1, cap = -1, mode = 0;
        if (warm_pass) {
            const bool feas = lp.crash(cs, logit, piv, use_pref, pref);
            first = (feas && !PH1) ? 2 : 3;
            mode = first;
            cap = use_pref && capped ? warm_cap<M>() : -1;
        }
        const int p1 = piv;
        for (;;) {
            st = lp.run(cs, piv, first, cap, PH1 ? &P : nullptr, x, PH1 ? &accepted : nullptr);
            if (first != 1 && (st == 2 || st == 3)) {
                mode = 0;
                warm = 3;
                lp.init(P);
                cs.restart();
                first = 1;
                cap = -1;
                continue;
            }
            break;
        }
        if (mode) warm = (mode == 2 && piv == p1) ? 1 : 2;
    } else {
        // a network's prediction for a 9-row LP is finished in this pass, whatever
        // it is worth: a rejected crash basis turns into a guided phase I, and no
        // pivot cap applies (a cold retry of these long LPs would redo the work)
        const bool finish = M == 9 && warm_pass && !use_pref;
        bool guided = false;
        if constexpr (WARM) if (warm_pass) {
            if (!lp.crash(cs, logit, piv, use_pref, pref)) {
                if (!finish) {
                    warm = 3;
                    return 4;
                }
                lp.init(P);
                lp.guided(cs, logit, piv);
                guided = true;
            }
            const int p1 = piv;
            st = guided ? lp.run(cs, piv, 1) : lp.run(cs, piv, 2, finish ? -1 : warm_cap<M>());
            if (st == 2 && !finish) {
                warm = 3;
                return 4;
            }
            warm = (!guided && piv == p1) ? 1 : 2;
        }
        if (!warm_pass) {
            if constexpr (PH1)
                st = lp.run(cs, piv, 1, -1, &P, x, &accepted);
            else
                st = lp.run(cs, piv, 1);
        }
    }
    return finish_lp<M>(lp, cs, P, store, st, accepted, x, fii, piv, certified, basis, stats, defer);
}

}  // namespace vrm
