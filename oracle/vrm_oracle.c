/*
 * vrm_oracle.c -- plain, slow, obviously-correct FP64 reference of the
 * splitting-free vorticity redistribution step (Kirchhart & Obi,
 * "A Splitting-free Vorticity Redistribution Method").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP library: it is written separately from the paper's definitions.
 *
 * What it computes, and where the paper defines it:
 *   diffused set      Sec. 3.5 "Reducing the Number of Diffused Particles",
 *                     bound eq. (reduced_bound): skip the smallest |Gamma| while
 *                     their l1 norm stays <= C_diff h^(q+1) ||Gamma||_1
 *   neighbourhood     Sec. 2, eq. (neighbourhood): r h <= |x_i - x_j| <= R h
 *   segments          Sec. 4.2: eight 45-degree segments of the neighbourhood
 *   small nbhd        Sec. 4.3: the closest particle of every segment
 *   insertion         Sec. 4.2: a Gamma = 0 particle on the centre line of an
 *                     empty segment at radius 1.5 h
 *   moment LP         Sec. 2 eqs. (cond_two), (cond_alpha), (fii), (momcondmv);
 *                     Sec. 4.1: dense simplex on V f = b, f >= 0
 *   NNLS              Sec. 4.1: the alternative min_{f >= 0} |V f - b|^2 by
 *                     Lawson and Hanson's active-set method
 *   operator apply    Sec. 3.4 eq. (nsode): dGamma_i/dt = nu sum_j f_ji Gamma_j
 *   time stepping     Sec. 3.3: Euler steps; SSP Runge-Kutta schemes are convex
 *                     combinations of Euler steps (Shu-Osher SSP-RK3 here)
 *   removal           Sec. 6 (Outlook): the identity operator approximated by
 *                     a particle's neighbours, its circulation given to them
 *
 * Readings where the paper is silent (the same readings bind the GPU path):
 *   - q is the highest moment order matched: q = 2 -> 5 rows (paper n = 1),
 *     q = 3 -> 9 rows (paper n = 2).
 *   - Canonical stencil: among all non-negative solutions, the minimiser of
 *     sum_j c_j f_j with c_j = |r_j/h|^(q+1) + 2^-10 * rank_j, where rank_j is
 *     the rank of particle j's id among the LP's columns.  |r|^(q+1) is the
 *     remainder weight of the consistency proof (Theorem "Consistency"); the
 *     small rank term makes the optimum unique on symmetric clouds.
 *   - Decisions that pick integers (annulus membership, segment, closest
 *     particle, insertion position and conflicts) are taken in FP32 with the
 *     exact operation sequence written below (no fused multiply-add); the
 *     arithmetic of the method itself (moments, LP, apply, RK) is FP64.
 *   - Segments are centred on s*45 degrees, s = 0..7 counter-clockwise from +x;
 *     a point is "near the x axis" iff |dy| < t|dx|, "near the y axis" iff
 *     |dx| < t|dy| (t = fl32(tan 22.5 deg)), else diagonal.
 *   - Annulus bounds carry a relative slack of 2^-20 on the squared radii.
 *   - The small LP is attempted only when the small neighbourhood has at least
 *     m columns; otherwise, or when it is infeasible, the complete
 *     neighbourhood within R_full h is used (at most KMAX nearest columns).
 *   - Insertion: once per step, only diffused particles trigger it; candidates
 *     are taken greedily in (id, segment) order and rejected when closer than
 *     0.5 h to an already accepted candidate; accepted ones get ids N, N+1, ...
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_KMAX 48      /* max LP columns of a complete neighbourhood */
#define ORC_MMAX 9       /* max moment rows */
#define ORC_NSEG 8

/* ---------------------------------------------------------------- params */
typedef struct {
    double h, nu, r, R, R_full, c_diff, dt;
    int q;
    int solver;   /* 0: the canonical LP (Sec. 4.1 simplex); 1: non-negative least squares (Lawson-Hanson) */
} orc_params;

static int rows_for_q(int q) { return q == 2 ? 5 : 9; }

/* ------------------------------------------- FP32 decision arithmetic */
static const float ORC_TAN225 = 0.41421356237309503f;  /* tan(pi/8) */
static const float ORC_C45 = 0.70710678118654752f;     /* cos(pi/4) */

static float f32_d2(float dx, float dy)
{
    float a = dx * dx;
    float b = dy * dy;
    return a + b;
}

static int f32_segment(float dx, float dy)
{
    float ax = fabsf(dx), ay = fabsf(dy);
    float tx = ORC_TAN225 * ax, ty = ORC_TAN225 * ay;
    if (ay < tx) return dx > 0.0f ? 0 : 4;
    if (ax < ty) return dy > 0.0f ? 2 : 6;
    if (dx > 0.0f) return dy > 0.0f ? 1 : 7;
    return dy > 0.0f ? 3 : 5;
}

static void annulus_bounds(double h, double rin, double rout, float* lo2, float* hi2)
{
    *lo2 = (float)(rin * rin * h * h * (1.0 - 0x1p-20));
    *hi2 = (float)(rout * rout * h * h * (1.0 + 0x1p-20));
}

/* candidate position for segment s of a particle at (xi, yi) (FP32) */
static void f32_candidate(float xi, float yi, double h, int s, float* xc, float* yc)
{
    static const float cs[8] = {1.0f, 0.70710678118654752f, 0.0f, -0.70710678118654752f,
                                -1.0f, -0.70710678118654752f, 0.0f, 0.70710678118654752f};
    static const float sn[8] = {0.0f, 0.70710678118654752f, 1.0f, 0.70710678118654752f,
                                0.0f, -0.70710678118654752f, -1.0f, -0.70710678118654752f};
    (void)ORC_C45;
    float rad = (float)(1.5 * h);
    float ox = rad * cs[s];
    float oy = rad * sn[s];
    *xc = xi + ox;
    *yc = yi + oy;
}

/* ------------------------------------------------------- uniform grid */
/* A plain bucket grid over the bounding box, only used to find candidates.
 * Membership is decided by the FP32 distance test alone. */
typedef struct {
    double x0, y0, cs;
    int nx, ny;
    int* start;  /* nx*ny + 1 */
    int* items;  /* n */
} orc_grid;

static int grid_cell(const orc_grid* g, double x, double y, int* cx, int* cy)
{
    int ix = (int)floor((x - g->x0) / g->cs);
    int iy = (int)floor((y - g->y0) / g->cs);
    if (ix < 0) ix = 0;
    if (iy < 0) iy = 0;
    if (ix >= g->nx) ix = g->nx - 1;
    if (iy >= g->ny) iy = g->ny - 1;
    *cx = ix;
    *cy = iy;
    return iy * g->nx + ix;
}

static int grid_build(orc_grid* g, int n, const double* x, const double* y, double cs)
{
    double xmin = 0, xmax = 0, ymin = 0, ymax = 0;
    for (int i = 0; i < n; ++i) {
        if (i == 0 || x[i] < xmin) xmin = x[i];
        if (i == 0 || x[i] > xmax) xmax = x[i];
        if (i == 0 || y[i] < ymin) ymin = y[i];
        if (i == 0 || y[i] > ymax) ymax = y[i];
    }
    g->cs = cs;
    g->x0 = xmin - cs;
    g->y0 = ymin - cs;
    g->nx = (int)((xmax - g->x0) / cs) + 2;
    g->ny = (int)((ymax - g->y0) / cs) + 2;
    long long ncell = (long long)g->nx * g->ny;
    if (ncell > 200000000LL) return -1;
    g->start = (int*)calloc((size_t)ncell + 1, sizeof(int));
    g->items = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int* cell = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!g->start || !g->items || !cell) return -2;
    for (int i = 0; i < n; ++i) {
        int cx, cy;
        cell[i] = grid_cell(g, x[i], y[i], &cx, &cy);
        g->start[cell[i] + 1]++;
    }
    for (long long c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    int* fill = (int*)malloc(sizeof(int) * (size_t)ncell);
    memcpy(fill, g->start, sizeof(int) * (size_t)ncell);
    for (int i = 0; i < n; ++i) g->items[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
    return 0;
}

static void grid_free(orc_grid* g)
{
    free(g->start);
    free(g->items);
    g->start = g->items = NULL;
}

/* ------------------------------------------------ diffused-set selection */
typedef struct { double a, v; int id; int idx; } orc_key;

/* Ranking key of a particle for the reduced operator: |Gamma| rounded to FP32,
 * the precision the circulations are held in on the device.  Sec. 3.5 ranks
 * the particles by their individual circulation; particles whose keys are
 * exactly equal form one group and are left out together. */
static double selection_key(double g)
{
    return (double)(float)fabs(g);
}

/* Circulations that are equal in exact arithmetic (a symmetric cloud) differ
 * by round-off once computed, so the particle that reaches the bound is
 * diffused together with every particle whose key lies within a relative
 * 2^-16 below its key (the band covers the stated 1e-5 bound on per-value
 * GPU-vs-oracle differences and the random-walk round-off of FP32
 * circulations over 10^2 SSP-RK3 steps, sqrt(300) x ~14 roundings x 2^-24).
 * The band limit is formed in FP32: fl32(T * (1 - 2^-16)). */
static const float ORC_TIE_BAND = 0.9999847412109375f;   /* 1 - 2^-16 */

static int key_cmp(const void* pa, const void* pb)
{
    const orc_key* a = (const orc_key*)pa;
    const orc_key* b = (const orc_key*)pb;
    if (a->a < b->a) return -1;
    if (a->a > b->a) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* Sec. 3.5: leave out the particles of smallest |Gamma| (whole groups of equal
 * ranking key, see selection_key) while the l1 norm of the left-out set stays
 * <= c_diff h^(q+1) ||Gamma||_1; then diffuse again the left-out particles in
 * the band below the first key that does not fit (ORC_TIE_BAND), so the
 * left-out set only shrinks and the bound still holds.
 * diffused[i] = 1 for the particles that are diffused.  Returns the count
 * diffused; *norm1 = ||Gamma||_1 and *bound = the right-hand side. */
int orc_diffused(int n, const double* gamma, const int32_t* id, double h, int q, double c_diff,
                 uint8_t* diffused, double* norm1, double* bound)
{
    orc_key* k = (orc_key*)malloc(sizeof(orc_key) * (size_t)(n > 0 ? n : 1));
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        k[i].a = selection_key(gamma[i]);
        k[i].v = fabs(gamma[i]);
        k[i].id = id[i];
        k[i].idx = i;
        s += k[i].v;
    }
    double b = c_diff * pow(h, q + 1) * s;
    qsort(k, (size_t)n, sizeof(orc_key), key_cmp);
    for (int i = 0; i < n; ++i) diffused[i] = 1;
    double prefix = 0.0;
    int i = 0;
    while (i < n) {
        int j = i;
        double grp = 0.0;
        while (j < n && k[j].a == k[i].a) grp += k[j++].v;
        if (prefix + grp <= b) {
            prefix += grp;
            for (int t = i; t < j; ++t) diffused[k[t].idx] = 0;
            i = j;
        } else {
            break;
        }
    }
    if (i < n) {
        /* k[i].a is the first key that does not fit */
        double band = (double)((float)k[i].a * ORC_TIE_BAND);
        for (int t = i - 1; t >= 0 && k[t].a >= band; --t) diffused[k[t].idx] = 1;
    }
    int cnt = 0;
    for (int t = 0; t < n; ++t) cnt += diffused[t];
    if (norm1) *norm1 = s;
    if (bound) *bound = b;
    free(k);
    return cnt;
}

/* ---------------------------------------------------- neighbourhoods */
typedef struct { float d2; int id; int idx; int seg; } orc_nb;

static int nb_cmp_dist(const void* pa, const void* pb)
{
    const orc_nb* a = (const orc_nb*)pa;
    const orc_nb* b = (const orc_nb*)pb;
    if (a->d2 < b->d2) return -1;
    if (a->d2 > b->d2) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* All j != i with lo2 <= d2 <= hi2 (FP32), written to out (capacity cap).
 * Returns the true count (may exceed cap). */
static int annulus_members(const orc_grid* g, const double* x, const double* y, const int32_t* id,
                           int i, float lo2, float hi2, orc_nb* out, int cap)
{
    float xi = (float)x[i], yi = (float)y[i];
    int cx, cy;
    grid_cell(g, x[i], y[i], &cx, &cy);
    int cnt = 0;
    for (int oy = -1; oy <= 1; ++oy) {
        int yy = cy + oy;
        if (yy < 0 || yy >= g->ny) continue;
        for (int ox = -1; ox <= 1; ++ox) {
            int xx = cx + ox;
            if (xx < 0 || xx >= g->nx) continue;
            int c = yy * g->nx + xx;
            for (int t = g->start[c]; t < g->start[c + 1]; ++t) {
                int j = g->items[t];
                if (j == i) continue;
                float dx = (float)x[j] - xi;
                float dy = (float)y[j] - yi;
                float d2 = f32_d2(dx, dy);
                if (d2 < lo2 || d2 > hi2) continue;
                if (cnt < cap) {
                    out[cnt].d2 = d2;
                    out[cnt].id = id[j];
                    out[cnt].idx = j;
                    out[cnt].seg = f32_segment(dx, dy);
                }
                ++cnt;
            }
        }
    }
    return cnt;
}

/* Small neighbourhood (Sec. 4.3): the closest particle of each segment, ties
 * by smaller id; small[s] = particle index or -1 if segment s is empty. */
static void small_from_members(const orc_nb* m, int cnt, int small[ORC_NSEG], float best[ORC_NSEG],
                               int bid[ORC_NSEG])
{
    for (int s = 0; s < ORC_NSEG; ++s) {
        small[s] = -1;
        best[s] = INFINITY;
        bid[s] = 0;
    }
    for (int t = 0; t < cnt; ++t) {
        int s = m[t].seg;
        if (small[s] < 0 || m[t].d2 < best[s] || (m[t].d2 == best[s] && m[t].id < bid[s])) {
            small[s] = m[t].idx;
            best[s] = m[t].d2;
            bid[s] = m[t].id;
        }
    }
}

/* --------------------------------------------------------- the LP */
/* minimise c^T f subject to A f = b, f >= 0, with A (m x k, row-major) and b >= 0.
 * Simplex method as Sec. 4.1 describes it: every iteration solves m x m systems
 * built from the current set of basic columns of A by an LU decomposition
 * (Gaussian elimination with partial pivoting), from the original data, so no
 * rounding error is carried from one iteration to the next.  Phase I starts
 * from the artificial basis (unit columns) and minimises the sum of the
 * artificials; phase II minimises c^T f.  Bland's rule (lowest index enters,
 * lowest basic index leaves on ratio ties) prevents cycling.  FP64.
 * Returns 0 = optimal (f filled), 1 = infeasible, 2 = iteration limit / singular,
 * 3 = the final basis is not feasible for the unperturbed right-hand side.
 * basis_out (optional, m entries) gets the structural basic columns or -1. */
#define LP_EPS_PIV 1e-9   /* relative to max(1, max |B^-1 a_e|) */
#define LP_EPS_OPT 1e-9   /* relative to |c_j| + sum_i |y_i a_ij| */
#define LP_EPS_FEAS 1e-10
#define LP_MAXIT 2000

/* Solve M z = rhs (n x n, row-major, copied) by Gaussian elimination with
 * partial pivoting; if trans, solve M^T z = rhs.  Returns 0, or 1 if singular. */
static int dense_solve(int n, const double* M, int trans, const double* rhs, double* z)
{
    double a[ORC_MMAX][ORC_MMAX + 1];
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) a[r][c] = trans ? M[c * n + r] : M[r * n + c];
        a[r][n] = rhs[r];
    }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r][c]) > fabs(a[p][c])) p = r;
        if (a[p][c] == 0.0) return 1;
        if (p != c)
            for (int t = 0; t <= n; ++t) { double u = a[c][t]; a[c][t] = a[p][t]; a[p][t] = u; }
        for (int r = c + 1; r < n; ++r) {
            double fct = a[r][c] / a[c][c];
            for (int t = c; t <= n; ++t) a[r][t] -= fct * a[c][t];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = a[r][n];
        for (int t = r + 1; t < n; ++t) s -= a[r][t] * z[t];
        z[r] = s / a[r][r];
    }
    return 0;
}

/* column j of [A | I] */
static void lp_column(int m, int k, const double* A, int j, double* col)
{
    for (int i = 0; i < m; ++i) col[i] = j < k ? A[i * k + j] : (j - k == i ? 1.0 : 0.0);
}

static int lp_run(int m, int k, const double* A, const double* b_in, const double* c, double* f,
                  int* basis_out, int* pivots_out, double perturb)
{
    int basis[ORC_MMAX];
    double B[ORC_MMAX * ORC_MMAX], xB[ORC_MMAX], y[ORC_MMAX], cB[ORC_MMAX], col[ORC_MMAX],
        alpha[ORC_MMAX], b[ORC_MMAX];
    int piv = 0, status = 0;
    /* Anti-degeneracy: the iterations run on a right-hand side perturbed by
     * distinct small amounts (the classical perturbation method); the basis
     * they end with is then evaluated on the exact right-hand side. */
    double bmax = 0.0;
    for (int i = 0; i < m; ++i) bmax = fabs(b_in[i]) > bmax ? fabs(b_in[i]) : bmax;
    for (int i = 0; i < m; ++i) b[i] = b_in[i] + perturb * (bmax > 0 ? bmax : 1.0) * (1.0 + 0.618 * i);
    for (int i = 0; i < m; ++i) basis[i] = k + i;
    for (int phase = 1; phase <= 2 && status == 0; ++phase) {
        int it;
        for (it = 0; it < LP_MAXIT; ++it) {
            /* basis matrix and basic solution */
            for (int t = 0; t < m; ++t) {
                lp_column(m, k, A, basis[t], col);
                for (int i = 0; i < m; ++i) B[i * m + t] = col[i];
            }
            if (dense_solve(m, B, 0, b, xB)) { status = 2; break; }
            /* prices: B^T y = c_B */
            for (int t = 0; t < m; ++t) {
                int j = basis[t];
                cB[t] = phase == 1 ? (j >= k ? 1.0 : 0.0) : (j < k ? c[j] : 0.0);
            }
            if (dense_solve(m, B, 1, cB, y)) { status = 2; break; }
            /* entering column: lowest index with negative reduced cost */
            int e = -1;
            for (int j = 0; j < k && e < 0; ++j) {
                int basic = 0;
                for (int t = 0; t < m; ++t) basic |= basis[t] == j;
                if (basic) continue;
                double d = phase == 1 ? 0.0 : c[j];
                double scale = fabs(d);
                for (int i = 0; i < m; ++i) {
                    d -= y[i] * A[i * k + j];
                    scale += fabs(y[i] * A[i * k + j]);
                }
                if (d < -LP_EPS_OPT * scale) {
                    lp_column(m, k, A, j, col);
                    dense_solve(m, B, 0, col, alpha);
                    double amax = 1.0;
                    for (int t = 0; t < m; ++t) amax = fabs(alpha[t]) > amax ? fabs(alpha[t]) : amax;
                    int ok = 0;
                    for (int t = 0; t < m; ++t) ok |= alpha[t] > LP_EPS_PIV * amax;
                    if (ok) e = j;   /* a column with no positive entry cannot move */
                }
            }
            if (e < 0) break;
            double amax = 1.0;
            for (int t = 0; t < m; ++t) amax = fabs(alpha[t]) > amax ? fabs(alpha[t]) : amax;
            /* ratio test; ties -> lowest basic index */
            int l = -1;
            double best = 0.0;
            for (int t = 0; t < m; ++t) {
                if (alpha[t] <= LP_EPS_PIV * amax) continue;
                double xt = xB[t] > 0.0 ? xB[t] : 0.0;
                double ratio = xt / alpha[t];
                if (l < 0 || ratio < best || (ratio == best && basis[t] < basis[l])) {
                    l = t;
                    best = ratio;
                }
            }
            basis[l] = e;
            ++piv;
        }
        if (it == LP_MAXIT) status = 2;
        if (status) break;
        if (phase == 1) {
            double art = 0.0;
            for (int t = 0; t < m; ++t)
                if (basis[t] >= k) art += fabs(xB[t]);
            if (art > LP_EPS_FEAS) { status = 1; break; }
            /* drive zero-level artificials out where a structural column can replace them */
            for (int t = 0; t < m; ++t) {
                if (basis[t] < k) continue;
                for (int u = 0; u < m; ++u) {
                    lp_column(m, k, A, basis[u], col);
                    for (int i = 0; i < m; ++i) B[i * m + u] = col[i];
                }
                for (int j = 0; j < k; ++j) {
                    int basic = 0;
                    for (int u = 0; u < m; ++u) basic |= basis[u] == j;
                    if (basic) continue;
                    lp_column(m, k, A, j, col);
                    if (dense_solve(m, B, 0, col, alpha)) break;
                    if (fabs(alpha[t]) > 1e-7) { basis[t] = j; ++piv; break; }
                }
            }
        }
    }
    if (status == 0) {
        for (int t = 0; t < m; ++t) {
            lp_column(m, k, A, basis[t], col);
            for (int i = 0; i < m; ++i) B[i * m + t] = col[i];
        }
        if (dense_solve(m, B, 0, b_in, xB)) status = 2;
        for (int t = 0; t < m && status == 0; ++t)
            if (xB[t] < -1e-9) status = 3;   /* perturbation changed the optimal basis */
    }
    if (status == 0) {
        for (int j = 0; j < k; ++j) f[j] = 0.0;
        double fsum = 0.0;
        for (int t = 0; t < m; ++t)
            if (basis[t] < k) {
                f[basis[t]] = xB[t] > 0.0 ? xB[t] : 0.0;
                fsum += f[basis[t]];
            }
        /* a basic value below 2^-30 of the stencil's sum is the round-off of a
         * degenerate vertex (exactly zero in exact arithmetic): make it zero */
        for (int j = 0; j < k; ++j)
            if (f[j] < 0x1p-30 * fsum) f[j] = 0.0;
        if (basis_out)
            for (int t = 0; t < m; ++t) basis_out[t] = basis[t] < k ? basis[t] : -1;
    }
    if (pivots_out) *pivots_out = piv;
    return status;
}

int orc_lp(int m, int k, const double* A, const double* b, const double* c, double* f,
           int* basis_out, int* pivots_out)
{
    /* perturbations tried in turn; 0 is the plain method */
    static const double pert[4] = {1e-7, 1e-9, 1e-11, 0.0};
    int st = 2, tot = 0;
    for (int t = 0; t < 4; ++t) {
        int piv = 0;
        st = lp_run(m, k, A, b, c, f, basis_out, &piv, pert[t]);
        tot += piv;
        if (st <= 1) break;
    }
    if (pivots_out) *pivots_out = tot;
    return st;
}

/* ---------------------------------------- moment system of one particle */
/* Rows: alpha with 1 <= |alpha| <= q in the order (1,0),(0,1),(2,0),(1,1),(0,2),
 * (3,0),(2,1),(1,2),(0,3).  b = 2 at (2,0) and (0,2) (eq. cond_two). */
static void moment_column(double rx, double ry, int q, double* col)
{
    col[0] = rx;
    col[1] = ry;
    col[2] = rx * rx;
    col[3] = rx * ry;
    col[4] = ry * ry;
    if (q >= 3) {
        col[5] = rx * rx * rx;
        col[6] = rx * rx * ry;
        col[7] = rx * ry * ry;
        col[8] = ry * ry * ry;
    }
}

void orc_moment_rhs(int q, double* b)
{
    int m = rows_for_q(q);
    for (int i = 0; i < m; ++i) b[i] = 0.0;
    b[2] = 2.0;
    b[4] = 2.0;
}

/* Solve the canonical LP over the given columns (particle indices cols[0..k)).
 * Returns LP status; f (k entries) normalised fractions. */
/* ------------------------------------------------------------- NNLS */
/* Least squares on the columns in set[0..p): z = argmin |A_set z - b| by Householder
 * QR (m rows, p <= m columns).  Returns 0, or -1 if A_set is rank deficient. */
static int ls_solve(int m, int k, const double* A, const double* b, const int* set, int p, double* z)
{
    double Q[ORC_MMAX][ORC_MMAX], c[ORC_MMAX];
    if (p > m) return -1;
    for (int a = 0; a < m; ++a) {
        c[a] = b[a];
        for (int t = 0; t < p; ++t) Q[a][t] = A[a * k + set[t]];
    }
    double scale = 0.0;
    for (int a = 0; a < m; ++a)
        for (int t = 0; t < p; ++t) scale = fmax(scale, fabs(Q[a][t]));
    for (int t = 0; t < p; ++t) {
        /* reflect column t below the diagonal onto e_t */
        double nrm = 0.0;
        for (int a = t; a < m; ++a) nrm += Q[a][t] * Q[a][t];
        nrm = sqrt(nrm);
        if (nrm <= 1e-13 * scale) return -1;
        double alpha = Q[t][t] > 0.0 ? -nrm : nrm;
        double v[ORC_MMAX];
        for (int a = 0; a < m; ++a) v[a] = a < t ? 0.0 : Q[a][t];
        v[t] -= alpha;
        double vv = 0.0;
        for (int a = t; a < m; ++a) vv += v[a] * v[a];
        for (int u = t; u < p; ++u) {
            double s = 0.0;
            for (int a = t; a < m; ++a) s += v[a] * Q[a][u];
            s = 2.0 * s / vv;
            for (int a = t; a < m; ++a) Q[a][u] -= s * v[a];
        }
        double s = 0.0;
        for (int a = t; a < m; ++a) s += v[a] * c[a];
        s = 2.0 * s / vv;
        for (int a = t; a < m; ++a) c[a] -= s * v[a];
    }
    for (int t = p - 1; t >= 0; --t) {
        double s = c[t];
        for (int u = t + 1; u < p; ++u) s -= Q[t][u] * z[u];
        z[t] = s / Q[t][t];
    }
    return 0;
}

/* Non-negative least squares min_{f >= 0} |A f - b|^2 (the alternative of Sec. 4.1,
 * solved as Lawson and Hanson do): start with every column at zero; repeatedly
 * free the column whose negative gradient w_j = a_j . (b - A f) is largest (the
 * lowest index among equal ones), solve the unconstrained least-squares problem on
 * the free columns, and while that solution has a non-positive entry step back
 * from the current point towards it until the first entry reaches zero and fix
 * the entries at zero again.  Stops when no fixed column has w_j above a relative
 * 1e-12.  Returns the number of free-column additions, or -1 on a rank-deficient
 * subproblem. */
int orc_nnls(int m, int k, const double* A, const double* b, double* f)
{
    int set[ORC_MMAX + 1], p = 0;
    int inset[ORC_KMAX];
    double z[ORC_MMAX + 1], xs[ORC_MMAX + 1];
    double anorm = 0.0, bnorm = 0.0;
    for (int j = 0; j < k; ++j) {
        f[j] = 0.0;
        inset[j] = 0;
        for (int a = 0; a < m; ++a) anorm = fmax(anorm, fabs(A[a * k + j]));
    }
    for (int a = 0; a < m; ++a) bnorm = fmax(bnorm, fabs(b[a]));
    const double tol = 1e-12 * anorm * bnorm * m;
    int adds = 0;
    for (int outer = 0; outer < 4 * k + 16; ++outer) {
        double r[ORC_MMAX];
        for (int a = 0; a < m; ++a) {
            double s = b[a];
            for (int t = 0; t < p; ++t) s -= A[a * k + set[t]] * f[set[t]];
            r[a] = s;
        }
        int best = -1;
        double wbest = tol;
        for (int j = 0; j < k; ++j) {
            if (inset[j]) continue;
            double w = 0.0;
            for (int a = 0; a < m; ++a) w += A[a * k + j] * r[a];
            if (w > wbest) {
                wbest = w;
                best = j;
            }
        }
        if (best < 0 || p == m) return adds;
        set[p++] = best;
        inset[best] = 1;
        ++adds;
        for (;;) {
            if (ls_solve(m, k, A, b, set, p, z) != 0) return -1;
            int allpos = 1;
            for (int t = 0; t < p; ++t) allpos = allpos && z[t] > 0.0;
            if (allpos) {
                for (int t = 0; t < p; ++t) f[set[t]] = z[t];
                break;
            }
            double alpha = 1.0;
            for (int t = 0; t < p; ++t) {
                xs[t] = f[set[t]];
                if (z[t] <= 0.0) {
                    double q = xs[t] / (xs[t] - z[t]);
                    if (q < alpha) alpha = q;
                }
            }
            int q2 = 0;
            for (int t = 0; t < p; ++t) {
                double v = xs[t] + alpha * (z[t] - xs[t]);
                if (v <= 1e-15 * bnorm) {
                    f[set[t]] = 0.0;
                    inset[set[t]] = 0;
                } else {
                    f[set[t]] = v;
                    set[q2++] = set[t];
                }
            }
            p = q2;
            if (p == 0) break;
        }
    }
    return adds;
}

static int solve_columns(const double* x, const double* y, const int32_t* id, int i, const int* cols,
                         int k, const orc_params* P, double* f, int* pivots)
{
    int m = rows_for_q(P->q);
    double A[ORC_MMAX * ORC_KMAX], b[ORC_MMAX], c[ORC_KMAX];
    double col[ORC_MMAX];
    for (int t = 0; t < k; ++t) {
        int j = cols[t];
        double rx = (x[j] - x[i]) / P->h;
        double ry = (y[j] - y[i]) / P->h;
        moment_column(rx, ry, P->q, col);
        for (int a = 0; a < m; ++a) A[a * k + t] = col[a];
        double d = sqrt(rx * rx + ry * ry);
        int rank = 0;
        for (int u = 0; u < k; ++u)
            if (id[cols[u]] < id[j]) ++rank;
        c[t] = pow(d, P->q + 1) + 0x1p-10 * rank;
    }
    orc_moment_rhs(P->q, b);
    if (P->solver == 1) {
        /* NNLS: a stencil when the least-squares residual vanishes (moments to 1e-10 of b) */
        int adds = orc_nnls(m, k, A, b, f);
        if (pivots) *pivots = adds > 0 ? adds : 0;
        if (adds < 0) return 1;
        double res = 0.0;
        for (int a = 0; a < m; ++a) {
            double s = -b[a];
            for (int t = 0; t < k; ++t) s += A[a * k + t] * f[t];
            res = fmax(res, fabs(s));
        }
        return res <= 2e-10 ? 0 : 1;
    }
    return orc_lp(m, k, A, b, c, f, NULL, pivots);
}

/* ------------------------------------------------ stencils of all particles */
/* For every particle with diffused[i] != 0: small neighbourhood LP, else the
 * complete one.  Outputs (n entries each; KMAX columns per particle):
 *   kcol[i]   number of columns (0 if not diffused / infeasible)
 *   cols[i*KMAX + t]  particle index of column t
 *   f[i*KMAX + t]     normalised fraction (f_ij = f / h^2)
 *   fii[i]    -sum_t f   (eq. fii)
 *   status[i] 0 small ok, 1 complete ok, 2 infeasible, 3 not diffused
 *   small[i*8 + s]  small-neighbourhood member of segment s or -1
 *   kfull[i]  number of complete-neighbourhood members (within R_full)
 * Returns 0 or a negative error. */
int orc_stencils(int n, const double* x, const double* y, const int32_t* id, const uint8_t* diffused,
                 const orc_params* P, int32_t* kcol, int32_t* cols, double* f, double* fii,
                 uint8_t* status, int32_t* small, int32_t* kfull, int64_t* pivots_total)
{
    int m = rows_for_q(P->q);
    double Rmax = P->R_full > P->R ? P->R_full : P->R;
    orc_grid g;
    if (grid_build(&g, n, x, y, Rmax * P->h * 1.01) != 0) return -1;
    float lo2, hi2, lo2f, hi2f;
    annulus_bounds(P->h, P->r, P->R, &lo2, &hi2);
    annulus_bounds(P->h, P->r, P->R_full, &lo2f, &hi2f);
    int64_t piv_sum = 0;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : piv_sum)
    for (int i = 0; i < n; ++i) {
        orc_nb mem[512];
        int sm[ORC_NSEG], bid[ORC_NSEG];
        float best[ORC_NSEG];
        double fl[ORC_KMAX];
        int cl[ORC_KMAX];
        kcol[i] = 0;
        fii[i] = 0.0;
        status[i] = 3;
        for (int s = 0; s < ORC_NSEG; ++s) small[(size_t)i * ORC_NSEG + s] = -1;
        kfull[i] = 0;
        if (!diffused[i]) continue;
        int cnt = annulus_members(&g, x, y, id, i, lo2, hi2, mem, 512);
        if (cnt > 512) { err = -3; continue; }
        small_from_members(mem, cnt, sm, best, bid);
        int k = 0;
        for (int s = 0; s < ORC_NSEG; ++s) {
            small[(size_t)i * ORC_NSEG + s] = sm[s];
            if (sm[s] >= 0) cl[k++] = sm[s];
        }
        int piv = 0, st = 1;
        if (k >= m) {
            st = solve_columns(x, y, id, i, cl, k, P, fl, &piv);
            piv_sum += piv;
        }
        if (st == 0) {
            status[i] = 0;
        } else {
            /* complete neighbourhood within R_full: KMAX nearest, nearest first by (d2, id) */
            int cf = annulus_members(&g, x, y, id, i, lo2f, hi2f, mem, 512);
            if (cf > 512) { err = -3; continue; }
            kfull[i] = cf;
            qsort(mem, (size_t)cf, sizeof(orc_nb), nb_cmp_dist);
            k = cf < ORC_KMAX ? cf : ORC_KMAX;
            for (int t = 0; t < k; ++t) cl[t] = mem[t].idx;
            st = k >= 1 ? solve_columns(x, y, id, i, cl, k, P, fl, &piv) : 1;
            piv_sum += piv;
            status[i] = st == 0 ? 1 : 2;
        }
        if (status[i] <= 1) {
            double s = 0.0;
            kcol[i] = k;
            for (int t = 0; t < k; ++t) {
                cols[(size_t)i * ORC_KMAX + t] = cl[t];
                f[(size_t)i * ORC_KMAX + t] = fl[t];
                s += fl[t];
            }
            fii[i] = -s;
        }
        if (kfull[i] == 0) {
            /* count the complete neighbourhood for reporting */
            kfull[i] = annulus_members(&g, x, y, id, i, lo2f, hi2f, mem, 0);
        }
    }
    grid_free(&g);
    if (pivots_total) *pivots_total = piv_sum;
    return err;
}

/* ----------------------------------------------------- operator apply */
/* dgamma_i = (nu / h^2) sum_j f_ji Gamma_j  (eq. nsode), serial scatter in index order */
void orc_apply(int n, const int32_t* kcol, const int32_t* cols, const double* f, const double* fii,
               const uint8_t* status, const double* gamma, const orc_params* P, double* dgamma)
{
    double s = P->nu / (P->h * P->h);
    for (int i = 0; i < n; ++i) dgamma[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        if (status[j] > 1) continue;
        double g = gamma[j];
        for (int t = 0; t < kcol[j]; ++t) dgamma[cols[(size_t)j * ORC_KMAX + t]] += s * f[(size_t)j * ORC_KMAX + t] * g;
        dgamma[j] += s * fii[j] * g;
    }
}

/* ------------------------------------------------------------ insertion */
typedef struct { int id; int s; int src; float x, y; } orc_cand;

static int cand_cmp(const void* pa, const void* pb)
{
    const orc_cand* a = (const orc_cand*)pa;
    const orc_cand* b = (const orc_cand*)pb;
    if (a->id != b->id) return (a->id > b->id) - (a->id < b->id);
    return a->s - b->s;
}

/* Sec. 4.2: for every diffused particle and every empty segment of its
 * neighbourhood, a candidate at radius 1.5 h on the segment's centre line.
 * Greedy in (id, segment) order; a candidate closer than 0.5 h to an accepted
 * one is rejected.  Accepted particles are appended at n, n+1, ... with Gamma = 0
 * and ids next_id, next_id + 1, ...  Returns the new count, or -1 if it would
 * exceed cap (nothing appended).  Emptiness uses the annulus [r h, R h]. */
int orc_insert(int n, int cap, double* x, double* y, double* gamma, int32_t* id, const uint8_t* diffused,
               const orc_params* P, int32_t next_id, int32_t* n_candidates)
{
    orc_grid g;
    if (grid_build(&g, n, x, y, P->R * P->h * 1.01) != 0) return -2;
    float lo2, hi2;
    annulus_bounds(P->h, P->r, P->R, &lo2, &hi2);
    int ncand = 0, capc = 1024;
    orc_cand* c = (orc_cand*)malloc(sizeof(orc_cand) * (size_t)capc);
    orc_nb mem[512];
    for (int i = 0; i < n; ++i) {
        if (!diffused[i]) continue;
        int cnt = annulus_members(&g, x, y, id, i, lo2, hi2, mem, 512);
        if (cnt > 512) { free(c); grid_free(&g); return -3; }
        int occupied[ORC_NSEG] = {0};
        for (int t = 0; t < cnt; ++t) occupied[mem[t].seg] = 1;
        for (int s = 0; s < ORC_NSEG; ++s) {
            if (occupied[s]) continue;
            if (ncand == capc) {
                capc *= 2;
                c = (orc_cand*)realloc(c, sizeof(orc_cand) * (size_t)capc);
            }
            c[ncand].id = id[i];
            c[ncand].s = s;
            c[ncand].src = i;
            f32_candidate((float)x[i], (float)y[i], P->h, s, &c[ncand].x, &c[ncand].y);
            ++ncand;
        }
    }
    grid_free(&g);
    if (n_candidates) *n_candidates = ncand;
    qsort(c, (size_t)ncand, sizeof(orc_cand), cand_cmp);
    float ex2 = (float)(0.25 * P->h * P->h);
    int* acc = (int*)malloc(sizeof(int) * (size_t)(ncand > 0 ? ncand : 1));
    int na = 0;
    /* accepted candidates are bucketed in cells of edge 0.5 h (a search aid only:
     * every candidate closer than 0.5 h lies in the 3 x 3 surrounding cells) */
    double bx0 = 0, by0 = 0, bx1 = 0, by1 = 0;
    for (int t = 0; t < ncand; ++t) {
        if (t == 0 || c[t].x < bx0) bx0 = c[t].x;
        if (t == 0 || c[t].y < by0) by0 = c[t].y;
        if (t == 0 || c[t].x > bx1) bx1 = c[t].x;
        if (t == 0 || c[t].y > by1) by1 = c[t].y;
    }
    /* any cell edge >= 0.5 h keeps the 3 x 3 search exact: widen the cells until
     * the bucket array stays below 50M entries */
    double ce = 0.5 * P->h * 1.001;
    long long gnx, gny;
    for (;;) {
        gnx = (long long)((bx1 - bx0) / ce) + 3;
        gny = (long long)((by1 - by0) / ce) + 3;
        if (gnx * gny <= 50000000LL) break;
        ce *= 1.25;
    }
    int* head = (int*)malloc(sizeof(int) * (size_t)(gnx * gny));
    int* next = (int*)malloc(sizeof(int) * (size_t)(ncand > 0 ? ncand : 1));
    for (long long q = 0; q < gnx * gny; ++q) head[q] = -1;
    for (int t = 0; t < ncand; ++t) {
        long long cxq = (long long)((c[t].x - bx0) / ce) + 1;
        long long cyq = (long long)((c[t].y - by0) / ce) + 1;
        int ok = 1;
        for (long long oy = -1; oy <= 1 && ok; ++oy) {
            long long yy = cyq + oy;
            if (yy < 0 || yy >= gny) continue;
            for (long long ox = -1; ox <= 1 && ok; ++ox) {
                long long xx = cxq + ox;
                if (xx < 0 || xx >= gnx) continue;
                for (int u = head[yy * gnx + xx]; u >= 0; u = next[u]) {
                    float dx = c[u].x - c[t].x;
                    float dy = c[u].y - c[t].y;
                    if (f32_d2(dx, dy) < ex2) { ok = 0; break; }
                }
            }
        }
        if (ok) {
            acc[na++] = t;
            long long q = cyq * gnx + cxq;
            next[t] = head[q];
            head[q] = t;
        }
    }
    free(head);
    free(next);
    if (n + na > cap) { free(acc); free(c); return -1; }
    for (int u = 0; u < na; ++u) {
        x[n + u] = c[acc[u]].x;
        y[n + u] = c[acc[u]].y;
        gamma[n + u] = 0.0;
        id[n + u] = next_id + u;
    }
    free(acc);
    free(c);
    return n + na;
}

/* ------------------------------------------------------ particle removal */
/* Particle removal (Sec. 6 "Outlook"): the same moment method, applied to the
 * identity operator instead of the Laplacian, gives a particle's circulation
 * to its neighbours so that the particle itself can be dropped.
 *
 * Readings (the passage gives the idea only):
 *   - With non-negative fractions the identity can be matched to first order
 *     only (a second moment sum_j g_j |r_j|^2 is positive), so the conditions
 *     are sum_j g_j = 1 and sum_j g_j r_j = 0 (three rows: 1, x, y), g >= 0.
 *     They keep I0 and I1 exactly; I2 grows by Gamma_i sum_j g_j |r_j|^2.
 *   - Among those g, the one minimising sum_j c_j g_j with
 *     c_j = |r_j/h|^2 + 2^-16 rank_j^2: the I2 change plus a tie-break.  The
 *     tie-break is convex in the rank: on a lattice the ids of opposite
 *     neighbours are symmetric about i, so every opposite pair has the same
 *     rank sum and a tie-break linear in the rank would leave them tied.
 *   - Columns: the complete neighbourhood r h <= |r_j| <= R_full h (its KMAX
 *     nearest by (d2, id)).
 *   - Candidates are particles closer than r h to another particle (the ones
 *     the neighbourhood definition leaves out).  They are taken greedily in
 *     id order; one is rejected when it lies within R_full h of a candidate
 *     already taken, so that no removed particle receives circulation from
 *     another.  A taken candidate whose LP is infeasible stays.
 *   - Distances are decided in FP32 as for the neighbourhoods.
 * Outputs: removed[i] = 1 for removed particles; gamma of the receivers is
 * updated in place (removed entries keep their value; the caller drops them);
 * for removed particles kcol/cols/g hold the columns and fractions (KMAX per
 * particle).  Returns the number removed, or a negative error. */
typedef struct { int32_t id; int idx; } orc_idk;

static int idk_cmp(const void* pa, const void* pb)
{
    const orc_idk* a = (const orc_idk*)pa;
    const orc_idk* b = (const orc_idk*)pb;
    return (a->id > b->id) - (a->id < b->id);
}

int orc_remove(int n, const double* x, const double* y, double* gamma, const int32_t* id, const orc_params* P,
               uint8_t* removed, int32_t* kcol, int32_t* cols, double* g, int32_t* n_candidates)
{
    orc_grid gr;
    if (grid_build(&gr, n, x, y, P->R_full * P->h * 1.01) != 0) return -1;
    float lo2, hi2;
    annulus_bounds(P->h, P->r, P->R_full, &lo2, &hi2);
    /* candidates: another particle closer than r h */
    orc_idk* cand = (orc_idk*)malloc(sizeof(orc_idk) * (size_t)(n > 0 ? n : 1));
    uint8_t* taken = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    double* delta = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int nc = 0;
    for (int i = 0; i < n; ++i) {
        removed[i] = 0;
        kcol[i] = 0;
        float xi = (float)x[i], yi = (float)y[i];
        int cx, cy, close = 0;
        grid_cell(&gr, x[i], y[i], &cx, &cy);
        for (int oy = -1; oy <= 1 && !close; ++oy)
            for (int ox = -1; ox <= 1 && !close; ++ox) {
                int xx = cx + ox, yy = cy + oy;
                if (xx < 0 || yy < 0 || xx >= gr.nx || yy >= gr.ny) continue;
                int c = yy * gr.nx + xx;
                for (int t = gr.start[c]; t < gr.start[c + 1]; ++t) {
                    int j = gr.items[t];
                    if (j != i && f32_d2((float)x[j] - xi, (float)y[j] - yi) < lo2) {
                        close = 1;
                        break;
                    }
                }
            }
        if (close) {
            cand[nc].id = id[i];
            cand[nc].idx = i;
            ++nc;
        }
    }
    if (n_candidates) *n_candidates = nc;
    /* greedy in id order, exclusion radius R_full h */
    qsort(cand, (size_t)nc, sizeof(orc_idk), idk_cmp);
    for (int a = 0; a < nc; ++a) {
        int i = cand[a].idx;
        float xi = (float)x[i], yi = (float)y[i];
        int cx, cy, clash = 0;
        grid_cell(&gr, x[i], y[i], &cx, &cy);
        for (int oy = -1; oy <= 1 && !clash; ++oy)
            for (int ox = -1; ox <= 1 && !clash; ++ox) {
                int xx = cx + ox, yy = cy + oy;
                if (xx < 0 || yy < 0 || xx >= gr.nx || yy >= gr.ny) continue;
                int c = yy * gr.nx + xx;
                for (int t = gr.start[c]; t < gr.start[c + 1]; ++t) {
                    int j = gr.items[t];
                    if (j != i && taken[j] && f32_d2((float)x[j] - xi, (float)y[j] - yi) <= hi2) {
                        clash = 1;
                        break;
                    }
                }
            }
        if (!clash) taken[i] = 1;
    }
    /* the identity LP of every taken candidate */
    int nrem = 0;
    for (int i = 0; i < n; ++i) {
        if (!taken[i]) continue;
        orc_nb mem[512];
        int cf = annulus_members(&gr, x, y, id, i, lo2, hi2, mem, 512);
        if (cf > 512) { nrem = -3; break; }
        qsort(mem, (size_t)cf, sizeof(orc_nb), nb_cmp_dist);
        int k = cf < ORC_KMAX ? cf : ORC_KMAX;
        if (k == 0) continue;
        double A[3 * ORC_KMAX], b[3] = {1.0, 0.0, 0.0}, c[ORC_KMAX], f[ORC_KMAX];
        for (int t = 0; t < k; ++t) {
            int j = mem[t].idx;
            double rx = (x[j] - x[i]) / P->h;
            double ry = (y[j] - y[i]) / P->h;
            int rank = 0;
            for (int u = 0; u < k; ++u)
                if (mem[u].id < mem[t].id) ++rank;
            A[0 * k + t] = 1.0;
            A[1 * k + t] = rx;
            A[2 * k + t] = ry;
            c[t] = rx * rx + ry * ry + 0x1p-16 * rank * rank;
        }
        if (orc_lp(3, k, A, b, c, f, NULL, NULL) != 0) continue;
        removed[i] = 1;
        kcol[i] = k;
        for (int t = 0; t < k; ++t) {
            cols[(size_t)i * ORC_KMAX + t] = mem[t].idx;
            g[(size_t)i * ORC_KMAX + t] = f[t];
            delta[mem[t].idx] += f[t] * gamma[i];
        }
        ++nrem;
    }
    if (nrem >= 0)
        for (int i = 0; i < n; ++i) gamma[i] += delta[i];
    free(cand);
    free(taken);
    free(delta);
    grid_free(&gr);
    return nrem;
}

int orc_kmax(void) { return ORC_KMAX; }
