// Neighbourhoods, moment-condition LPs and the operator apply of libvrm.
//
// Kirchhart & Obi, Sec. 2 (eqs. neighbourhood, cond_two, cond_alpha, fii,
// momcondmv), Sec. 4.1 (dense simplex on V f = b, f >= 0), Sec. 4.2
// (segments), Sec. 4.3 (small neighbourhoods first, complete ones as a
// fallback), Sec. 3.4 eq. nsode (dGamma_i/dt = nu sum_j f_ji Gamma_j).
//
// One LP is solved by an octet: 8 lanes of a wave64.  Every lane owns the
// tableau columns whose index is congruent to its lane number mod 8; the
// tableau keeps the artificial columns, so it carries B^-1 alongside B^-1 V.
// The pivoting runs in FP32 on a slightly perturbed right-hand side (to step
// over degenerate vertices); the final basis is then certified against the
// exact problem with compensated (double-float) residuals: iterative
// refinement of the basic solution and of the prices, exact reduced costs,
// and primal or dual repair pivots until it is optimal.  The canonical cost
// c_j = |r_j/h|^(q+1) + 2^-10 rank(id_j) makes the optimum unique.
#include <hip/hip_runtime.h>

#include "vrm_device.h"
#include "vrm_internal.h"

using namespace vrm;

namespace {

constexpr float kPerturb = 7.62939453125e-06f;   // 2^-17: relative rhs perturbation
constexpr float kTolD = 1e-6f;                    // FP32 pricing tolerance (relative)
constexpr float kTolPiv = 1e-6f;                  // FP32 pivot tolerance (relative to max |alpha|)
constexpr float kTolFeas = 1e-3f;                 // phase-I infeasibility (relative to rhs)
constexpr float kCertD = 1e-9f;                   // certified reduced-cost tolerance (relative)
constexpr float kCertX = 1e-9f;                   // certified primal tolerance (absolute, fhat units)
constexpr int kMaxCert = 8;
constexpr int kMaxRefine = 8;

struct Col {
    float rx, ry, rxl, ryl;   // exact offset (x_j - x_i) 2^-e as hi + lo
    float chi, clo;           // canonical cost, double-float
    int id;                   // particle id (rank tie-break)
    int pidx;                 // particle index (output / scatter target)
    bool valid;
};

template <int M>
__device__ __forceinline__ void monomials_f32(float x, float y, float (&v)[M])
{
    v[0] = x;
    v[1] = y;
    v[2] = x * x;
    v[3] = x * y;
    v[4] = y * y;
    if constexpr (M == 9) {
        v[5] = x * x * x;
        v[6] = x * x * y;
        v[7] = x * y * y;
        v[8] = y * y * y;
    }
}

template <int M>
__device__ __forceinline__ void monomials_df(const Col& c, df (&v)[M])
{
    df X{c.rx, c.rxl}, Y{c.ry, c.ryl};
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

// rhs entry of row r in the scaled units (2 at (2,0) and (0,2))
__device__ __forceinline__ df rhs_df(int r, const LaunchParams& P)
{
    return (r == 2 || r == 4) ? df{P.bt_hi, P.bt_lo} : df{0.0f, 0.0f};
}

// The octet LP.  KS structural column slots (multiple of 8), M rows.
template <int M, int KS>
struct OctetLP {
    static constexpr int SS = KS / 8;                 // structural slots per lane
    static constexpr int AS = (M + 7) / 8;            // artificial slots per lane
    static constexpr int CPL = SS + AS;

    float T[CPL][M];
    bool isb[CPL];
    bool blk[CPL];
    float beta[M];
    int basis[M];
    float cB[M];
    int l8;

    __device__ __forceinline__ int col_id(int c) const
    {
        return c < SS ? c * 8 + l8 : KS + (c - SS) * 8 + l8;
    }
    __device__ __forceinline__ bool art_row_owner(int c, int r) const { return c >= SS && col_id(c) == KS + r; }

    // select slot s of an array held per lane
    __device__ __forceinline__ float sel_T(int s, int r) const
    {
        float v = 0.0f;
#pragma unroll
        for (int c = 0; c < CPL; ++c) v = (c == s) ? T[c][r] : v;
        return v;
    }

    __device__ void init(const Col (&col)[SS], const LaunchParams& P)
    {
        l8 = lane_id() & 7;
#pragma unroll
        for (int c = 0; c < SS; ++c) {
            float v[M];
            monomials_f32<M>(col[c].rx, col[c].ry, v);
#pragma unroll
            for (int r = 0; r < M; ++r) T[c][r] = col[c].valid ? v[r] : 0.0f;
            isb[c] = false;
            blk[c] = false;
        }
#pragma unroll
        for (int c = SS; c < CPL; ++c) {
            int id = col_id(c);
#pragma unroll
            for (int r = 0; r < M; ++r) T[c][r] = (id == KS + r) ? 1.0f : 0.0f;
            isb[c] = (id < KS + M);
            blk[c] = false;
        }
#pragma unroll
        for (int r = 0; r < M; ++r) {
            float b = rhs_df(r, P).hi;
            beta[r] = b + kPerturb * P.bt_hi * (1.0f + 0.618f * (float)r);
            basis[r] = KS + r;
            cB[r] = 0.0f;
        }
    }

    // FP32 pivot on row l with entering column e (alpha = its tableau column).
    __device__ void pivot(int l, int e, const float (&alpha)[M], float ce)
    {
        float al = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) al = (r == l) ? alpha[r] : al;
        float inv = 1.0f / al;
        float ap[M];
#pragma unroll
        for (int r = 0; r < M; ++r) ap[r] = alpha[r] - ((r == l) ? 1.0f : 0.0f);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            float t = 0.0f;
#pragma unroll
            for (int r = 0; r < M; ++r) t = (r == l) ? T[c][r] : t;
            float g = t * inv;
#pragma unroll
            for (int r = 0; r < M; ++r) T[c][r] = __builtin_fmaf(-ap[r], g, T[c][r]);
        }
        {
            float t = 0.0f;
#pragma unroll
            for (int r = 0; r < M; ++r) t = (r == l) ? beta[r] : t;
            float g = t * inv;
#pragma unroll
            for (int r = 0; r < M; ++r) beta[r] = __builtin_fmaf(-ap[r], g, beta[r]);
        }
        int old = 0;
#pragma unroll
        for (int r = 0; r < M; ++r) old = (r == l) ? basis[r] : old;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            basis[r] = (r == l) ? e : basis[r];
            cB[r] = (r == l) ? ce : cB[r];
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            int id = col_id(c);
            if (id == e) isb[c] = true;
            if (id == old) isb[c] = false;
            blk[c] = false;
        }
    }

    // entering column's tableau column and cost, broadcast from its owner
    __device__ void fetch_column(int e, const Col (&col)[SS], float (&alpha)[M], float& ce) const
    {
        int owner = e & 7;
        int slot = e < KS ? (e >> 3) : SS + ((e - KS) >> 3);
#pragma unroll
        for (int r = 0; r < M; ++r) alpha[r] = oct_bcast(sel_T(slot, r), owner);
        float c = 0.0f;
#pragma unroll
        for (int s = 0; s < SS; ++s) c = (s == slot) ? col[s].chi : c;
        ce = oct_bcast(c, owner);
    }

    // Bland's rule ratio test; returns the leaving row or -1.
    __device__ int ratio_test(const float (&alpha)[M], const float (&x)[M], bool phase2) const
    {
        float amax = 0.0f;
#pragma unroll
        for (int r = 0; r < M; ++r) amax = fmaxf(amax, fabsf(alpha[r]));
        float eps = kTolPiv * amax;
        int l = -1;
        float best = 0.0f;
        int bb = 0;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            bool art = basis[r] >= KS;
            float ratio;
            bool ok;
            if (phase2 && art && fabsf(alpha[r]) > eps) {
                ratio = 0.0f;
                ok = true;
            } else {
                ok = alpha[r] > eps;
                ratio = fmaxf(x[r], 0.0f) / alpha[r];
            }
            if (ok && (l < 0 || ratio < best || (ratio == best && basis[r] < bb))) {
                l = r;
                best = ratio;
                bb = basis[r];
            }
        }
        return l;
    }

    // Two-phase FP32 simplex.  Returns 0 feasible/optimal, 1 infeasible, 2 iteration limit.
    __device__ int simplex(const Col (&col)[SS], int& piv)
    {
        for (int phase = 1; phase <= 2; ++phase) {
            int it = 0;
            for (; it < 4 * (KS + M) + 32; ++it) {
                // lowest-index column with a negative reduced cost (Bland)
                int mine = 0x7fffffff;
#pragma unroll
                for (int c = SS - 1; c >= 0; --c) {
                    if (!col[c].valid || isb[c] || blk[c]) continue;
                    float d, sc;
                    if (phase == 1) {
                        d = 0.0f;
                        sc = 0.0f;
#pragma unroll
                        for (int r = 0; r < M; ++r) {
                            bool art = basis[r] >= KS;
                            d -= art ? T[c][r] : 0.0f;
                            sc += art ? fabsf(T[c][r]) : 0.0f;
                        }
                    } else {
                        d = col[c].chi;
                        sc = fabsf(col[c].chi);
#pragma unroll
                        for (int r = 0; r < M; ++r) {
                            float t = cB[r] * T[c][r];
                            d -= t;
                            sc += fabsf(t);
                        }
                    }
                    if (d < -kTolD * sc) mine = col_id(c);
                }
                int e = oct_min_i(mine);
                if (e == 0x7fffffff) break;
                float alpha[M], ce;
                fetch_column(e, col, alpha, ce);
                int l = ratio_test(alpha, beta, phase == 2);
                if (l < 0) {
#pragma unroll
                    for (int c = 0; c < SS; ++c)
                        if (col_id(c) == e) blk[c] = true;
                    continue;
                }
                pivot(l, e, alpha, phase == 2 ? ce : 0.0f);
                ++piv;
            }
            if (it >= 4 * (KS + M) + 32) return 2;
            if (phase == 1) {
                float art = 0.0f;
#pragma unroll
                for (int r = 0; r < M; ++r) art += basis[r] >= KS ? fabsf(beta[r]) : 0.0f;
                if (art > kTolFeas * fabsf(beta[2])) return 1;
                // phase-II prices of the basic structural columns
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    int b = basis[r];
                    float c = 0.0f;
                    if (b < KS) {
                        int owner = b & 7, slot = b >> 3;
                        float mine_c = 0.0f;
#pragma unroll
                        for (int s = 0; s < SS; ++s) mine_c = (s == slot) ? col[s].chi : mine_c;
                        c = oct_bcast(mine_c, owner);
                    }
                    cB[r] = c;
                }
#pragma unroll
                for (int c = 0; c < SS; ++c) blk[c] = false;
            }
        }
        return 0;
    }

    // w = B^-1 v  (v uniform in the octet)
    __device__ void binv_apply(const float (&v)[M], float (&w)[M]) const
    {
        float acc[M];
#pragma unroll
        for (int r = 0; r < M; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int c = SS; c < CPL; ++c) {
            int a = col_id(c) - KS;   // this slot holds column a of B^-1
            float va = 0.0f;
#pragma unroll
            for (int r = 0; r < M; ++r) va = (r == a) ? v[r] : va;
            if (a < M) {
#pragma unroll
                for (int r = 0; r < M; ++r) acc[r] = __builtin_fmaf(T[c][r], va, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < M; ++r) w[r] = oct_sum(acc[r]);
    }

    // w = B^-T v: w_a = (column a of B^-1) . v
    __device__ void binvT_apply(const float (&v)[M], float (&w)[M]) const
    {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            int slot = SS + (a >> 3), owner = a & 7;
            float dot = 0.0f;
#pragma unroll
            for (int r = 0; r < M; ++r) dot = __builtin_fmaf(sel_T(slot, r), v[r], dot);
            w[a] = oct_bcast(dot, owner);
        }
    }

    // accurate B x (x in row order of the basis) -> residual b - B x
    __device__ void primal_residual(const Col (&col)[SS], const df (&x)[M], const LaunchParams& P,
                                    float (&res)[M]) const
    {
        df acc[M];
#pragma unroll
        for (int r = 0; r < M; ++r) acc[r] = {0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < SS; ++c) {
            if (!isb[c]) continue;
            int id = col_id(c);
            df xr{0.0f, 0.0f};
#pragma unroll
            for (int r = 0; r < M; ++r)
                if (basis[r] == id) xr = x[r];
            df v[M];
            monomials_df<M>(col[c], v);
#pragma unroll
            for (int a = 0; a < M; ++a) acc[a] = df_add(acc[a], df_mul(v[a], xr));
        }
        // artificial basic columns (redundant rows) contribute x_r e_a on lane 0
        if (l8 == 0) {
#pragma unroll
            for (int r = 0; r < M; ++r) {
                int b = basis[r];
                if (b >= KS) {
#pragma unroll
                    for (int a = 0; a < M; ++a)
                        if (b - KS == a) acc[a] = df_add(acc[a], x[r]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) {
            df s = oct_sum_df(acc[a]);
            df rr = df_add(rhs_df(a, P), df_neg(s));
            res[a] = rr.hi + rr.lo;
        }
    }

    // accurate dual residual c_B - B^T y, per basis row
    __device__ void dual_residual(const Col (&col)[SS], const df (&y)[M], float (&res)[M]) const
    {
        float mine[M];
#pragma unroll
        for (int r = 0; r < M; ++r) mine[r] = 0.0f;
#pragma unroll
        for (int c = 0; c < SS; ++c) {
            if (!isb[c]) continue;
            int id = col_id(c);
            df v[M];
            monomials_df<M>(col[c], v);
            df s{col[c].chi, col[c].clo};
#pragma unroll
            for (int a = 0; a < M; ++a) s = df_add(s, df_neg(df_mul(v[a], y[a])));
#pragma unroll
            for (int r = 0; r < M; ++r)
                if (basis[r] == id) mine[r] = s.hi + s.lo;
        }
#pragma unroll
        for (int r = 0; r < M; ++r) {
            int b = basis[r];
            float v;
            if (b < KS) {
                v = oct_bcast(mine[r], b & 7);
            } else {
                // artificial basic column e_a with cost 0: residual = -y_a
                float ya = 0.0f;
#pragma unroll
                for (int a = 0; a < M; ++a)
                    if (b - KS == a) ya = -(y[a].hi + y[a].lo);
                v = ya;
            }
            res[r] = v;
        }
    }

    // Certify the basis against the exact problem; repair if needed.
    // Returns 0 optimal, 1 infeasible, 3 not certified.  x gets the basic values.
    __device__ int certify(const Col (&col)[SS], const LaunchParams& P, df (&x)[M], int& piv)
    {
        for (int round = 0; round < kMaxCert; ++round) {
            // basic solution with two refinement steps
            float b0[M], t[M];
#pragma unroll
            for (int r = 0; r < M; ++r) b0[r] = rhs_df(r, P).hi;
            binv_apply(b0, t);
#pragma unroll
            for (int r = 0; r < M; ++r) x[r] = {t[r], 0.0f};
            // refine until the correction is below 2^-30 of the solution (the
            // tableau's B^-1 drifts over many FP32 pivots, so allow several steps)
            for (int it = 0; it < kMaxRefine; ++it) {
                float res[M], dx[M];
                primal_residual(col, x, P, res);
                binv_apply(res, dx);
                float dmax = 0.0f, xmax = 0.0f;
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    x[r] = df_add(x[r], df{dx[r], 0.0f});
                    dmax = fmaxf(dmax, fabsf(dx[r]));
                    xmax = fmaxf(xmax, fabsf(x[r].hi));
                }
                if (dmax <= 9.313225746154785e-10f * xmax) break;
            }
            // prices y = B^-T c_B with two refinement steps
            float cb[M], yt[M];
#pragma unroll
            for (int r = 0; r < M; ++r) cb[r] = cB[r];
            binvT_apply(cb, yt);
            df y[M];
#pragma unroll
            for (int a = 0; a < M; ++a) y[a] = {yt[a], 0.0f};
            for (int it = 0; it < kMaxRefine; ++it) {
                float res[M], dy[M];
                dual_residual(col, y, res);
                binvT_apply(res, dy);
                float dmax = 0.0f, ymax = 0.0f;
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    y[a] = df_add(y[a], df{dy[a], 0.0f});
                    dmax = fmaxf(dmax, fabsf(dy[a]));
                    ymax = fmaxf(ymax, fabsf(y[a].hi));
                }
                if (dmax <= 9.313225746154785e-10f * ymax) break;
            }
            // primal check: the most negative basic structural value
            int lrow = -1;
            float xmin = -kCertX;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                float v = x[r].hi + x[r].lo;
                if (basis[r] < KS && v < xmin) {
                    xmin = v;
                    lrow = r;
                }
            }
            // exact reduced costs of own nonbasic columns
            float dj[SS];
            int mine = 0x7fffffff;
#pragma unroll
            for (int c = SS - 1; c >= 0; --c) {
                dj[c] = 0.0f;
                if (!col[c].valid || isb[c]) continue;
                df v[M];
                monomials_df<M>(col[c], v);
                df s{col[c].chi, col[c].clo};
                float sc = fabsf(col[c].chi);
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    df p = df_mul(v[a], y[a]);
                    s = df_add(s, df_neg(p));
                    sc += fabsf(p.hi);
                }
                dj[c] = s.hi + s.lo;
                if (dj[c] < -kCertD * sc) mine = col_id(c);
            }
            int e = oct_min_i(mine);
            if (lrow < 0 && e == 0x7fffffff) return 0;
            if (lrow >= 0) {
                // dual repair: row lrow leaves; entering by the dual ratio test
                float best = INFINITY;
                int bid = 0x7fffffff;
#pragma unroll
                for (int c = 0; c < SS; ++c) {
                    if (!col[c].valid || isb[c]) continue;
                    float w = 0.0f;
#pragma unroll
                    for (int r = 0; r < M; ++r) w = (r == lrow) ? T[c][r] : w;
                    if (w < -kTolPiv) {
                        float ratio = fmaxf(dj[c], 0.0f) / (-w);
                        int id = col_id(c);
                        if (ratio < best || (ratio == best && id < bid)) {
                            best = ratio;
                            bid = id;
                        }
                    }
                }
                // octet arg-min of (ratio, id)
                float bmin = best;
                bmin = fminf(bmin, __shfl_xor(bmin, 1, VRM_WAVE));
                bmin = fminf(bmin, __shfl_xor(bmin, 2, VRM_WAVE));
                bmin = fminf(bmin, __shfl_xor(bmin, 4, VRM_WAVE));
                int cand = (best == bmin) ? bid : 0x7fffffff;
                int ent = oct_min_i(cand);
                if (ent == 0x7fffffff || bmin == INFINITY) return 1;
                float alpha[M], ce;
                fetch_column(ent, col, alpha, ce);
                pivot(lrow, ent, alpha, ce);
                ++piv;
                continue;
            }
            // primal pivot with Bland's entering column and the exact basic values
            float alpha[M], ce;
            fetch_column(e, col, alpha, ce);
            float xf[M];
#pragma unroll
            for (int r = 0; r < M; ++r) xf[r] = x[r].hi + x[r].lo;
            int l = ratio_test(alpha, xf, true);
            if (l < 0) return 3;
            pivot(l, e, alpha, ce);
            ++piv;
        }
        return 3;
    }
};

// --------------------------------------------------------------- columns
__device__ __forceinline__ Col make_col(float xi, float yi, float xj, float yj, int id, int pidx,
                                        const LaunchParams& P, int q)
{
    Col c;
    df dx = two_sum(xj, -xi);
    df dy = two_sum(yj, -yi);
    c.rx = dx.hi * P.scale2e;
    c.rxl = dx.lo * P.scale2e;
    c.ry = dy.hi * P.scale2e;
    c.ryl = dy.lo * P.scale2e;
    df X{c.rx, c.rxl}, Y{c.ry, c.ryl};
    df d2 = df_add(df_mul(X, X), df_mul(Y, Y));
    df w = (q == 2) ? df_mul(d2, df_sqrt(d2)) : df_mul(d2, d2);
    w = df_mul(w, df{P.cs_hi, P.cs_lo});
    c.chi = w.hi;
    c.clo = w.lo;
    c.id = id;
    c.pidx = pidx;
    c.valid = true;
    return c;
}

// rank of each valid column's id among all valid columns of the octet's LP;
// adds 2^-10 rank to the cost (exact in FP32 at these magnitudes)
template <int SS>
__device__ void add_rank_cost(Col (&col)[SS])
{
    int rank[SS];
#pragma unroll
    for (int c = 0; c < SS; ++c) rank[c] = 0;
#pragma unroll
    for (int s = 0; s < SS; ++s) {
        for (int src = 0; src < 8; ++src) {
            int oid = oct_bcast_i(col[s].valid ? col[s].id : 0x7fffffff, src);
#pragma unroll
            for (int c = 0; c < SS; ++c) rank[c] += (oid < col[c].id) ? 1 : 0;
        }
    }
#pragma unroll
    for (int c = 0; c < SS; ++c) {
        df w = two_sum(col[c].chi, 0.0009765625f * (float)rank[c]);
        w.lo += col[c].clo;
        w = fast_two_sum(w.hi, w.lo);
        col[c].chi = w.hi;
        col[c].clo = w.lo;
    }
}

template <int M, int KS>
__device__ int solve_octet(Col (&col)[KS / 8], const LaunchParams& P, float (&f)[KS / 8], float& fii, int& piv,
                           int& certified)
{
    constexpr int SS = KS / 8;
    add_rank_cost<SS>(col);
    OctetLP<M, KS> lp;
    lp.init(col, P);
    int st = lp.simplex(col, piv);
    certified = 1;
    if (st == 1) return 1;
    df x[M];
    int cs = lp.certify(col, P, x, piv);
    if (cs == 1) return 1;
    certified = (cs == 0 && st == 0) ? 1 : 0;
    float sum = 0.0f;
#pragma unroll
    for (int c = 0; c < SS; ++c) {
        float v = 0.0f;
        if (lp.isb[c]) {
            int id = lp.col_id(c);
#pragma unroll
            for (int r = 0; r < M; ++r)
                if (lp.basis[r] == id) v = x[r].hi + x[r].lo;
        }
        f[c] = v > 0.0f ? v : 0.0f;
        sum += f[c];
    }
    // a basic value below 2^-30 of the stencil's sum is the round-off of a
    // degenerate vertex (zero in exact arithmetic): make it zero
    float tiny = 9.313225746154785e-10f * oct_sum(sum);
    sum = 0.0f;
#pragma unroll
    for (int c = 0; c < SS; ++c) {
        f[c] = f[c] < tiny ? 0.0f : f[c];
        sum += f[c];
    }
    fii = -oct_sum(sum);
    return 0;
}

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

// Small-neighbourhood LPs (m = 5 rows, 8 columns), one octet per particle.
__global__ __launch_bounds__(256) void k_lp_small(const int32_t* __restrict__ perm, const float* __restrict__ xs,
                                                  const float* __restrict__ ys, const int32_t* __restrict__ ids,
                                                  const int32_t* __restrict__ small_slot,
                                                  const int32_t* __restrict__ q_small, Queues* qs,
                                                  int32_t* q_full, const float* __restrict__ gamma,
                                                  float* acc, LaunchParams P, StencilOut out, int apply,
                                                  vrm_counters* cnt)
{
    const int l8 = lane_id() & 7;
    const int oct = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int noct = (gridDim.x * blockDim.x) >> 3;
    const int nitems = qs->n_small;
    int loops = (nitems + noct - 1) / noct;
    for (int it = 0; it < loops; ++it) {
        int item = oct + it * noct;
        bool live = item < nitems;
        int t = live ? q_small[item] : 0;
        int i = live ? perm[t] : 0;
        float xi = xs[t], yi = ys[t];
        int u = live ? small_slot[(size_t)t * VRM_NSEG + l8] : -1;
        Col col[1];
        if (u >= 0) {
            col[0] = make_col(xi, yi, xs[u], ys[u], ids[u], perm[u], P, 2);
        } else {
            col[0] = Col{0, 0, 0, 0, 0, 0, 0x7fffffff, -1, false};
        }
        float f[1], fii = 0.0f;
        int piv = 0, certified = 1;
        int st = live ? solve_octet<5, 8>(col, P, f, fii, piv, certified) : 1;
        if (live && l8 == 0 && piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        bool ok = live && st == 0;
        if (ok) {
            float g = gamma[i];
            if (apply) {
                if (col[0].valid && f[0] != 0.0f) atomicAdd(&acc[col[0].pidx], f[0] * g);
                if (l8 == 0) atomicAdd(&acc[i], fii * g);
            }
            if (out.small_f) {
                out.small_idx[(size_t)i * VRM_NSEG + l8] = col[0].valid ? col[0].pidx : -1;
                out.small_f[(size_t)i * VRM_NSEG + l8] = col[0].valid ? f[0] : 0.0f;
                if (l8 == 0) {
                    out.fii[i] = fii;
                    out.status[i] = VRM_ST_SMALL;
                }
            }
        }
        bool lead = l8 == 0;
        count_add(&cnt->n_small, lead && ok);
        count_add(&cnt->n_uncertified, lead && ok && !certified);
        if (apply) {
            uint64_t m = __ballot(lead && ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
        bool fail = live && lead && st != 0;
        int p = wave_append(&qs->n_full, fail);
        if (fail) q_full[p] = t;
    }
}

// Complete-neighbourhood LPs (Sec. 4.3 fallback), one octet per particle.
template <int M>
__global__ __launch_bounds__(256) void k_lp_full(const int32_t* __restrict__ perm, const float* __restrict__ xs,
                                                 const float* __restrict__ ys, const int32_t* __restrict__ ids,
                                                 const int32_t* __restrict__ cell_start, const GridState* gs,
                                                 const int32_t* __restrict__ q_full, const Queues* qs,
                                                 const float* __restrict__ gamma, float* acc, LaunchParams P,
                                                 StencilOut out, int apply, vrm_counters* cnt)
{
    constexpr int KS = VRM_KMAX;
    constexpr int SS = KS / 8;
    constexpr int CAP = 128;   // member buffer per octet
    __shared__ int s_slot[32][CAP];
    __shared__ float s_d2[32][CAP];
    __shared__ int s_sel[32][KS];
    const int l8 = lane_id() & 7;
    const int loct = threadIdx.x >> 3;
    const int oct = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int noct = (gridDim.x * blockDim.x) >> 3;
    const int nitems = qs->n_full;
    const GridState g = *gs;
    int loops = (nitems + noct - 1) / noct;
    for (int it = 0; it < loops; ++it) {
        int item = oct + it * noct;
        bool live = item < nitems;
        int t = live ? q_full[item] : 0;
        int i = live ? perm[t] : 0;
        float xi = xs[t], yi = ys[t];
        int cnt_m = 0;   // members found (uniform in the octet)
        if (live) {
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
                    for (int ub = u0; ub < u1; ub += 8) {
                        int u = ub + l8;
                        bool in = false;
                        float d2 = 0.0f;
                        if (u < u1 && u != t) {
                            float dx = xs[u] - xi;
                            float dy = ys[u] - yi;
                            d2 = d2_f32(dx, dy);
                            in = d2 >= P.lo2f && d2 <= P.hi2f;
                        }
                        uint64_t m = __ballot(in);
                        uint32_t mo = (uint32_t)(m >> (lane_id() & ~7)) & 0xffu;
                        int before = __popc(mo & ((1u << l8) - 1u));
                        if (in && cnt_m + before < CAP) {
                            s_slot[loct][cnt_m + before] = u;
                            s_d2[loct][cnt_m + before] = d2;
                        }
                        cnt_m += __popc(mo);
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int k = cnt_m < CAP ? cnt_m : CAP;
        bool truncated = cnt_m > KS;
        // keep the KS nearest members by (d2, id): a member's rank among all members
        Col col[SS];
#pragma unroll
        for (int c = 0; c < SS; ++c) col[c] = Col{0, 0, 0, 0, 0, 0, 0x7fffffff, -1, false};
        if (!truncated) {
#pragma unroll
            for (int c = 0; c < SS; ++c) {
                int mi = c * 8 + l8;
                if (mi < k) {
                    int u = s_slot[loct][mi];
                    col[c] = make_col(xi, yi, xs[u], ys[u], ids[u], perm[u], P, M == 5 ? 2 : 3);
                }
            }
        } else {
            // rare: keep the KS nearest members by (d2, id), placed by rank
            for (int mi = l8; mi < k; mi += 8) {
                float d = s_d2[loct][mi];
                int u = s_slot[loct][mi];
                int idu = ids[u];
                int r = 0;
                for (int o = 0; o < k; ++o) {
                    float d_o = s_d2[loct][o];
                    int id_o = ids[s_slot[loct][o]];
                    r += (d_o < d || (d_o == d && id_o < idu)) ? 1 : 0;
                }
                if (r < KS) s_sel[loct][r] = u;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int c = 0; c < SS; ++c) {
                int u = s_sel[loct][c * 8 + l8];
                col[c] = make_col(xi, yi, xs[u], ys[u], ids[u], perm[u], P, M == 5 ? 2 : 3);
            }
            k = KS;
        }
        float f[SS], fii = 0.0f;
        int piv = 0, certified = 1;
        int st = (live && k > 0) ? solve_octet<M, KS>(col, P, f, fii, piv, certified) : 1;
        if (live && l8 == 0 && piv) atomicAdd((unsigned long long*)&cnt->pivots, (unsigned long long)piv);
        bool ok = live && st == 0;
        if (ok) {
            float gi = gamma[i];
            if (apply) {
#pragma unroll
                for (int c = 0; c < SS; ++c)
                    if (col[c].valid && f[c] != 0.0f) atomicAdd(&acc[col[c].pidx], f[c] * gi);
                if (l8 == 0) atomicAdd(&acc[i], fii * gi);
            }
            if (out.full_k) {
                if (l8 == 0) {
                    out.full_k[i] = k;
                    out.fii[i] = fii;
                    out.status[i] = VRM_ST_FULL;
                }
                if (out.full_idx) {
#pragma unroll
                    for (int c = 0; c < SS; ++c) {
                        int mi = c * 8 + l8;
                        if (mi < VRM_KMAX) {
                            out.full_idx[(size_t)i * VRM_KMAX + mi] = col[c].valid ? col[c].pidx : -1;
                            out.full_f[(size_t)i * VRM_KMAX + mi] = col[c].valid ? f[c] : 0.0f;
                        }
                    }
                }
            }
        } else if (live && out.status && l8 == 0) {
            out.status[i] = VRM_ST_INFEASIBLE;
        }
        bool lead = l8 == 0;
        count_add(&cnt->n_full, lead && ok);
        count_add(&cnt->n_infeasible, lead && live && !ok);
        count_add(&cnt->n_uncertified, lead && ok && !certified);
        count_add(&cnt->n_truncated, lead && live && truncated);
        if (apply) {
            uint64_t m = __ballot(lead && ok);
            if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
                atomicAdd((unsigned long long*)&cnt->redistributions, (unsigned long long)__popcll(m));
        }
        __builtin_amdgcn_wave_barrier();
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

int lp_grid()
{
    return 256 * 8;   // persistent: 8 blocks of 256 threads per CU
}

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
    hipLaunchKernelGGL(k_small_nbhd, dim3(nb), dim3(256), 0, c->stream, n, c->perm, c->xs, c->ys, c->ids,
                       c->cell_start, c->diffused, c->grid, lp, c->small_slot, c->q_small, c->q_full, c->queues,
                       (int32_t*)nullptr, (int32_t*)nullptr, 0);
    VRM_HIP(hipGetLastError());
    int grid = lp_grid();
    if (lp.m == 5) {
        hipLaunchKernelGGL(k_lp_small, dim3(grid), dim3(256), 0, c->stream, c->perm, c->xs, c->ys, c->ids,
                           c->small_slot, c->q_small, c->queues, c->q_full, cl->gamma_dev, c->acc, lp, out, apply,
                           c->counters);
        VRM_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_lp_full<5>, dim3(grid), dim3(256), 0, c->stream, c->perm, c->xs, c->ys, c->ids,
                           c->cell_start, c->grid, c->q_full, c->queues, cl->gamma_dev, c->acc, lp, out, apply,
                           c->counters);
    } else {
        hipLaunchKernelGGL(k_lp_full<9>, dim3(grid), dim3(256), 0, c->stream, c->perm, c->xs, c->ys, c->ids,
                           c->cell_start, c->grid, c->q_full, c->queues, cl->gamma_dev, c->acc, lp, out, apply,
                           c->counters);
    }
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}
