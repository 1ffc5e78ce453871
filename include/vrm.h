/*
 * vrm.h -- C ABI of the MI355X (gfx950) vorticity redistribution library.
 *
 * Splitting-free vorticity redistribution (Kirchhart & Obi): every particle
 * i carries a circulation Gamma_i at x_i (Sec. 1, eq. vfield).  The library
 * computes, for every diffused particle, non-negative fractions f_ij over its
 * neighbourhood that satisfy the moment conditions (Sec. 2, eqs. cond_two,
 * cond_alpha, fii, momcondmv), inserts Gamma = 0 particles where a
 * neighbourhood has an empty 45-degree segment (Sec. 4.2), and applies
 * dGamma_i/dt = nu sum_j f_ji Gamma_j (Sec. 3.4, eq. nsode) inside the stages
 * of an SSP Runge-Kutta scheme (Sec. 3.3).
 *
 * Conventions for every entry point
 *   - Pointers named *_dev are device pointers on the context's device; the
 *     caller owns them and keeps them alive until the stream has drained.
 *     Host pointers are named *_host.
 *   - Every call enqueues work on the context's stream and returns without
 *     waiting, except where "synchronises" is stated.
 *   - Return value: VRM_OK (0) or a negative VRM_E_* code; vrm_last_error()
 *     then describes the failure (thread-local).  Argument errors are found
 *     before anything is enqueued and leave all buffers untouched.
 *   - Fractions are normalised: f_ij = fhat_ij / h^2 (Sec. 2, last paragraph).
 *   - Floating point: FP32 state and fractions; FP64 only in the verification
 *     sums (moment residual, circulation).
 *   - Non-finite input: the first kernel that reads the positions (the cell
 *     list's bounding box) or the circulations (the diffused-set selection,
 *     the stage-0 copy of vrm_rk_stage, the removal's candidate scan) flags a
 *     NaN or infinite value on the device.  From then on no cell index is
 *     formed from it and no kernel changes the cloud: the calls of the step
 *     become no-ops.  The next synchronising call (vrm_insert_particles,
 *     vrm_step, vrm_remove_particles, vrm_read_counters) returns
 *     VRM_E_NONFINITE, clears the flag and drops the context's cached cell
 *     list and diffused set.
 */
#ifndef VRM_H
#define VRM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VRM_OK 0
#define VRM_E_ARG (-1)        /* bad argument (null, sizes, parameters) */
#define VRM_E_CAPACITY (-2)   /* insertion would exceed cloud capacity; nothing appended */
#define VRM_E_HIP (-3)        /* a HIP runtime call failed */
#define VRM_E_STATE (-4)      /* call order violated (e.g. no diffused set yet) */
#define VRM_E_NONFINITE (-5)  /* a position or circulation is NaN or infinite; the cloud is unchanged */

#define VRM_NSEG 8            /* 45-degree segments of a neighbourhood (Sec. 4.2) */
#define VRM_KMAX 48           /* max columns of a complete-neighbourhood LP */

/* per-particle status written by vrm_solve_fractions (Sec. 4.3) */
#define VRM_ST_SMALL 0        /* small neighbourhood LP solved */
#define VRM_ST_FULL 1         /* complete neighbourhood LP solved (fallback) */
#define VRM_ST_INFEASIBLE 2   /* no non-negative stencil: not diffused this stage */
#define VRM_ST_SKIPPED 3      /* not in the diffused set (Sec. 3.5) */
#define VRM_ST_WARM 4         /* solved from the warm start's basis (vrm_set_warm_start), certified like
                                 the cold solve: the same stencil; full_k_dev > 0 marks a complete
                                 neighbourhood */

typedef struct vrm_ctx vrm_ctx;

/* Particle cloud (Sec. 1, eq. vfield), structure of arrays, all device
 * pointers of `capacity` entries.  n_dev points to one int32 in device memory
 * holding the current count N; insertion increases it on the device.
 * vrm_insert_particles permutes the arrays (id travels with its particle);
 * vrm_remove_particles drops entries and closes the gaps in order. */
typedef struct {
    float* x_dev;
    float* y_dev;
    float* gamma_dev;
    int32_t* id_dev;
    int32_t* n_dev;
    int32_t capacity;
} vrm_cloud;

/* Method parameters.
 *   h       average particle spacing (> 0)
 *   nu      kinematic viscosity (>= 0)
 *   r, R    neighbourhood annulus r h <= |x_i - x_j| <= R h, R > r > 0
 *           (Sec. 2, eq. neighbourhood; the paper uses r = 1/2, R = 2)
 *   R_full  radius of the complete neighbourhood used when the small one fails
 *   c_diff  reduced-operator constant (Sec. 3.5, eq. reduced_bound)
 *   dt      time step of vrm_rk_stage
 *   q       highest moment order matched: 2 (5 conditions, paper n = 1) or
 *           3 (9 conditions, paper n = 2)
 *   deterministic  0: the update sum_j f_ji Gamma_j is accumulated with FP32
 *           atomics (fastest; the last bits depend on their order).  1: each
 *           contribution is rounded to a multiple of 2^(e - 46), max|Gamma^n| <
 *           2^e, and summed as a 64-bit integer: results are bit-reproducible
 *           whatever the launch shapes and the order of the atomics. */
typedef struct {
    double h, nu, r, R, R_full, c_diff, dt;
    int32_t q;
    int32_t deterministic;
} vrm_params;

/* Stencil output of vrm_solve_fractions, device arrays indexed by particle
 * index (capacity entries).  Unused slots hold -1 / 0. */
typedef struct {
    int32_t* small_idx_dev;   /* [capacity][8]: small-neighbourhood member per segment, or -1 */
    float* small_f_dev;       /* [capacity][8]: fhat for those members */
    float* fii_dev;           /* [capacity]:    fhat_ii = -sum_j fhat_ij (eq. fii) */
    uint8_t* status_dev;      /* [capacity]:    VRM_ST_* */
    int32_t* full_k_dev;      /* [capacity]:    number of complete-neighbourhood columns */
    int32_t* full_idx_dev;    /* [capacity][VRM_KMAX] (may be NULL: then not written) */
    float* full_f_dev;        /* [capacity][VRM_KMAX] (may be NULL together with full_idx_dev) */
} vrm_stencils;

/* Device-side counters, read with vrm_read_counters. */
typedef struct {
    int32_t n;                /* current particle count */
    int32_t n_diffused;       /* size of the diffused set of the step */
    int32_t n_candidates;     /* insertion candidates of the last insertion */
    int32_t n_inserted;       /* particles appended by the last insertion */
    int64_t n_small;          /* LPs solved on the small neighbourhood (cumulative) */
    int64_t n_full;           /* LPs solved on the complete neighbourhood (cumulative) */
    int64_t n_infeasible;     /* particles without a stencil (cumulative) */
    int64_t n_uncertified;    /* LPs whose optimality could not be certified (cumulative) */
    int64_t n_truncated;      /* complete neighbourhoods cut to VRM_KMAX (cumulative) */
    int32_t n_grid_clamped;   /* cell grids that hit their size limit (cumulative) */
    int32_t reserved0;
    int64_t pivots;           /* simplex pivots (cumulative) */
    int64_t redistributions;  /* stencils applied by vrm_rk_stage (cumulative) */
    int32_t capacity_needed;  /* set when an insertion failed for capacity */
    int32_t mis_rounds;       /* rounds of the last insertion's parallel conflict resolution; 0 when at most 1024
                                 candidates were resolved greedily in one workgroup (same result) */
    int64_t full_cols;        /* sum of the column counts of complete-neighbourhood LPs (cumulative) */
    int64_t warm_hit;         /* warm-started LPs whose predicted basis was optimal (cumulative) */
    int64_t warm_phase2;      /* warm-started LPs that needed phase-II pivots from the predicted basis */
    int64_t warm_cold;        /* predictions given up by the warm pass (rejected crash basis or more than a
                                 few phase-II pivots): solved by the cold pass (cumulative) */
    int64_t graph_replays;    /* vrm_step stage sequences replayed from the recorded graph (cumulative; host count) */
    int64_t cert_rounds;      /* certification rounds of the solved LPs (cumulative; 1 per LP when the first
                                 refinement already proves optimality) */
    int64_t cert_exact;       /* LPs whose certification needed the double-float dual check (cumulative) */
} vrm_counters;

/* Create a context on `device` that enqueues on `stream` (a hipStream_t; NULL
 * = the null stream) for clouds of up to `capacity` particles (at most 2^26).  The context
 * owns all scratch memory (about 250 bytes per particle of capacity) and
 * frees it in vrm_destroy.  Synchronises. */
int vrm_create(vrm_ctx** out, int device, void* stream, int32_t capacity);
int vrm_destroy(vrm_ctx* ctx);

/* Sec. 3.5, eq. reduced_bound: choose the diffused set of the step from the
 * current circulations: leave out the particles of smallest |Gamma| while the
 * l1 norm of the left-out ones stays <= c_diff h^(q+1) ||Gamma||_1.  Particles
 * are ranked by their FP32 |Gamma| (the whole 32-bit key; equal keys are left out
 * together or not at all); the sums are exact FP64 sums of |Gamma|.  With T the
 * first |Gamma| that does not fit, every particle with |Gamma| >= fl32(T (1 -
 * 2^-16)) is diffused: circulations equal in exact arithmetic but apart by
 * round-off stay together (the left-out set only shrinks, so the bound holds).
 * Kept in the context (and written to mask_dev[N] as 0/1 when mask_dev != NULL). */
int vrm_select_diffused(vrm_ctx* ctx, const vrm_cloud* cloud, const vrm_params* p, uint8_t* mask_dev);

/* Replace the context's diffused set with mask_dev[N] (0/1), e.g. to solve
 * for an externally chosen set. */
int vrm_set_diffused(vrm_ctx* ctx, const vrm_cloud* cloud, const uint8_t* mask_dev);

/* Sec. 2 eq. neighbourhood, Sec. 4.2-4.3: build the cell list at the
 * current positions and, for every diffused particle, the small
 * neighbourhood (closest member of each 45-degree segment of the annulus
 * r h <= d <= R h; ties by smaller id) and the size of the complete
 * neighbourhood within R_full h.  small_idx_dev[N][8] gets particle indices
 * (-1 for an empty segment); kfull_dev[N] the complete count (either may be
 * NULL).  Non-diffused particles get -1 / 0. */
int vrm_build_neighbourhoods(vrm_ctx* ctx, const vrm_cloud* cloud, const vrm_params* p,
                             int32_t* small_idx_dev, int32_t* kfull_dev);

/* Sec. 4.2: once per step.  Selects the diffused set (as
 * vrm_select_diffused), inserts a Gamma = 0 particle on the centre line of
 * every empty segment of every diffused particle at radius 1.5 h, resolving
 * conflicts between candidates closer than 0.5 h greedily in (id, segment)
 * order, appends the new particles with ids M+1, M+2, ... in that order, where
 * M is the largest id of the cloud (ids must be distinct and non-negative),
 * and reorders the whole cloud by cell.  On VRM_E_CAPACITY (detected on the
 * device; reported by the next vrm_read_counters as capacity_needed) or
 * VRM_E_NONFINITE the cloud is left unchanged.  Synchronises once. */
int vrm_insert_particles(vrm_ctx* ctx, vrm_cloud* cloud, const vrm_params* p);

/* Sec. 6 (outlook): particle removal.  The moment method applied to the
 * identity operator instead of the Laplacian gives a particle's circulation
 * to its neighbours, after which the particle is dropped.  A particle is a
 * candidate when another one lies closer than r h (inside the annulus the
 * neighbourhoods leave out).  Candidates are taken greedily in id order,
 * skipping any within R_full h of one already taken, so no removed particle
 * receives circulation.  A taken particle i solves, over its complete
 * neighbourhood r h <= |r_ij| <= R_full h (its VRM_KMAX nearest members),
 *   sum_j g_j = 1,  sum_j g_j r_ij = 0,  g >= 0   (first order: with g >= 0 no
 *   second moment can vanish), minimising sum_j g_j (|r_ij/h|^2 + 2^-16 rank(id_j)^2);
 * then Gamma_j += g_j Gamma_i and i is removed.  A particle whose LP is
 * infeasible stays.  I0 and I1 are kept; I2 grows by Gamma_i sum_j g_j |r_ij|^2.
 * The kept particles keep their order; *n_dev is updated.  Synchronises.
 * n_removed, n_candidates: host pointers (may be NULL) for the counts. */
int vrm_remove_particles(vrm_ctx* ctx, vrm_cloud* cloud, const vrm_params* p, int32_t* n_removed,
                         int32_t* n_candidates);

/* Sec. 2 and 4.1-4.3: stencils of all diffused particles at the current
 * positions.  The small-neighbourhood LP is tried when it has at least as many
 * columns as conditions; otherwise, or if it is infeasible, the complete
 * neighbourhood within R_full h (its VRM_KMAX nearest members).  Among all
 * non-negative solutions the one minimising sum_j c_j fhat_j with
 * c_j = |r_ij / h|^(q+1) + 2^-10 rank(id_j) is returned. */
int vrm_solve_fractions(vrm_ctx* ctx, const vrm_cloud* cloud, const vrm_params* p, vrm_stencils* out);

/* Sec. 3.3-3.4: one stage (0, 1, 2) of the Shu-Osher SSP-RK3 scheme,
 *   y^(s) = a_s y^n + b_s (y^(s-1) + dt L(y^(s-1))),  (a, b) = (0,1), (3/4,1/4), (1/3,2/3),
 * with L = (u, v, nu sum_j f_ji Gamma_j) evaluated at the current state.
 * u_dev, v_dev [N]: caller-supplied velocity at the current positions (NULL
 * for zero velocity).  Stage 0 records y^n.  Uses the diffused set of the
 * step. */
int vrm_rk_stage(vrm_ctx* ctx, vrm_cloud* cloud, const float* u_dev, const float* v_dev,
                 const vrm_params* p, int stage);

/* One whole SSP-RK3 step: vrm_insert_particles, then stages 0, 1, 2 of
 * vrm_rk_stage.  With n_vort > 0 each stage's velocity is the prescribed
 * vortex field of vrm_vortex_velocity at the stage time (t, t + dt, t + dt/2);
 * otherwise zero.  The context caches the cell list and the cell order of the
 * cloud between calls: a caller that changes positions or the count itself
 * must not rely on that cache (a different cloud or count resets it).
 * The three stages are recorded once as a HIP graph (on a stream of the
 * context's own) and replayed on the context's stream at every later call
 * with the same cloud, parameters, vortex table and warm-start and timing
 * settings; the stage kernels read N on the device, and the graph is
 * recorded again when N outgrows the bound its launches were sized for.
 * Results are those of the direct launches (up to the order of the
 * floating-point atomic sums).  Synchronises once (insertion). */
int vrm_step(vrm_ctx* ctx, vrm_cloud* cloud, const vrm_params* p, const float* vort_dev, int32_t n_vort, double t);

/* Sec. 4.1: which non-negative solution of the moment conditions a stencil is.
 * 0 (default): the canonical stencil, the minimiser of sum_j c_j f_j with
 * c_j = |r_j/h|^(q+1) + 2^-10 rank(id_j) (both phases, exact certificate; the
 * same result as any correct solver).  1: the first feasible vertex, as the
 * paper's method stops after phase I (fewer pivots; the stencil depends on the
 * pivoting rules, so results are checked by their moments, sign and
 * conservation, not against another solver).  A phase-I basis whose refined
 * values are not exactly feasible continues to the canonical stencil.
 * 2: non-negative least squares, min_{f >= 0} |V f - b|^2 (the alternative the
 * paper discusses and sets aside in Sec. 4.1), by Lawson and Hanson's
 * active-set method in FP32; the support it ends on gets its exact values from
 * the same double-float refinement as a simplex basis, and a stencil whose
 * refined values are not a non-negative solution of the moment conditions is
 * reported infeasible.  Another non-negative solution than the canonical one
 * (the method's path decides which).  Modes 1 and 2 leave counters' pivots as
 * pivots or freed columns.  Mode 2 excludes warm starts (VRM_E_STATE from
 * either setter while the other is on).  Errors: VRM_E_ARG for another mode. */
int vrm_set_lp_objective(vrm_ctx* ctx, int mode);

/* Launch shapes (performance only; results do not depend on them).  A zero
 * field keeps the library's default.  The values are device-independent
 * numbers of workgroups; an autotuner (paper_1508_06379_amd/autotune.py)
 * picks them per workload by timing steps. */
typedef struct vrm_tuning {
    int32_t lp_small_blocks;     /* most workgroups (256 threads) of the small-LP launch; default 2048 */
    int32_t lp_full_blocks;      /* most workgroups (64 threads) of the complete-LP launches; default 2048 */
    int32_t full_stored_cost_n;  /* clouds with N up to this keep complete-LP costs in LDS; default 200000;
                                    -1: never */
    int32_t infer_blocks;        /* most workgroups (256 threads) of the network's inference; default 768 */
    int32_t lp_small_lanes;      /* small LPs per wave of the small-LP launch (1, 2, 4, ..., 64); default 64 */
    int32_t lp_small_coop;       /* 1: the plain and phase-I small-LP passes give each LP eight lanes, one
                                    column each (shorter chains for latency-bound launches); 0 (default):
                                    one thread per LP.  Warm-start and training-collection passes always use
                                    one thread per LP.  Results are the same either way. */
    int32_t cert_rounds;         /* test hook, not a launch shape: repair rounds of an LP's exact
                                    certification (default 8, at most 64).  An LP still not certified
                                    after them keeps its basis only if the basis's exact values satisfy
                                    the moment and sign conditions (counted in n_uncertified); otherwise
                                    it is handled as infeasible. */
    int32_t reserved;
} vrm_tuning;
/* Set (t = NULL: restore the defaults) or read the launch shapes. */
int vrm_set_tuning(vrm_ctx* ctx, const vrm_tuning* t);
int vrm_get_tuning(vrm_ctx* ctx, vrm_tuning* out);

/* Enable (default) or disable the graph replay of vrm_step's stages; with it
 * disabled every stage kernel is launched directly.  Disabling synchronises
 * the stream and releases the recorded graph. */
int vrm_set_graph(vrm_ctx* ctx, int enable);

/* Sec. 2 eqs. cond_two/cond_alpha, Sec. 3.4: FP64 checks of a stencil set.
 * Writes, to report_dev[4] (device doubles): the maximum over particles of
 * max_alpha |sum_j fhat_ij r_ij^alpha / h^|alpha| - b_alpha| / 2, the circulation
 * sum_i Gamma_i, sum_i |Gamma_i|, and the largest sum_{j != i} fhat_ij. */
int vrm_verify(vrm_ctx* ctx, const vrm_cloud* cloud, const vrm_params* p, const vrm_stencils* st,
               double* report_dev);

/* Copy the device counters to *out_host.  Synchronises the stream.  Returns
 * VRM_E_NONFINITE (after filling *out_host) if a non-finite value was flagged. */
int vrm_read_counters(vrm_ctx* ctx, vrm_counters* out_host);

/* Sec. 3.4 eq. (nsode) with the regularised kernel of Sec. 5: the velocity
 * the particles induce on themselves,
 *   u_i = sum_j Gamma_j K_eps(x_i - x_j),
 *   K_eps(d) = (-d_y, d_x) (1 - exp(-|d|^2 / eps^2)) / (2 pi |d|^2),  K_eps(0) = 0,
 * by a direct sum over all N^2 pairs in FP32 (the paper evaluates it with a
 * fast multipole method; the direct sum suits clouds up to ~10^5 particles).
 * u_dev, v_dev: device floats [capacity], caller-owned; the first N entries
 * are overwritten.  eps > 0 (the paper: eps = 3h).  Enqueued on the context's
 * stream; no synchronisation. */
int vrm_biot_savart(vrm_ctx* ctx, const vrm_cloud* cloud, double eps, float* u_dev, float* v_dev);

/* Prescribed velocity of a sum of spreading Gaussian (Lamb-Oseen) vortices
 * at the current positions (test and benchmark harness, not part of the
 * method): for vortex k with centre (cx, cy), core sigma and strength G,
 *   u_theta = G / (2 pi r) (1 - exp(-r^2 / (sigma^2 + 4 nu t))), counter-clockwise.
 * vort_dev = device floats [n_vort][4] (cx, cy, sigma, G). */
int vrm_vortex_velocity(vrm_ctx* ctx, const vrm_cloud* cloud, const float* vort_dev, int32_t n_vort,
                        double nu, double t, float* u_dev, float* v_dev);

/* ---- Learned warm start (build component; not in the paper) ------------
 * A small network predicts, from the offsets of an LP's columns, which
 * columns form the optimal basis.  Input row (BF16, VRM_MLP_IN values): for
 * slots j < 32, (dx_j / h, dy_j / h) at [2j, 2j+1] and a 0/1 mask at [64 + j];
 * q - 2 at [96]; zeros elsewhere.  Slots are the small-neighbourhood columns by
 * segment (q = 2) or the complete-neighbourhood columns nearest first by
 * (distance, id) (q = 3).  Output row (FP32, VRM_MLP_OUT): 32 basis logits,
 * 32 fractions.  Layers 128 -> 128 (GELU) -> 128 (GELU) -> 64, BF16 matrix
 * products with FP32 accumulation.  Parameters (FP32, VRM_MLP_PARAMS values):
 * W1[128][128], b1[128], W2[128][128], b2[128], W3[128][64], b3[64].
 * The warm start never changes results: the predicted basis only seeds the
 * simplex, whose answer is certified exactly as without it. */
#define VRM_MLP_IN 128
#define VRM_MLP_OUT 64
#define VRM_MLP_PARAMS 41280
/* Copy parameters in (device FP32) / out. */
int vrm_mlp_load(vrm_ctx* ctx, const float* params_dev);
int vrm_mlp_read(vrm_ctx* ctx, float* params_dev);
/* Warm start of vrm_solve_fractions / vrm_rk_stage / vrm_step:
 *   0  off (every LP starts from the artificial basis);
 *   1  from the network's predicted basis (needs loaded parameters; allocates
 *      512 bytes per particle of capacity);
 *   2  from the basis of the particle's previous stencil (matched by column
 *      ids; allocates 36 bytes per particle of capacity).
 * In modes 1 and 2 a first LP pass starts from the predicted basis and a
 * second, cold pass solves what the first could not settle with a few
 * pivots; every accepted basis is certified exactly, so the stencils are
 * those of mode 0. */
int vrm_set_warm_start(vrm_ctx* ctx, int enable);
/* Training data from the plain solver at the current positions and diffused
 * set: for the LPs queued first (small ones for q = 2, complete ones for
 * q = 3), input rows x_dev[max_rows][128] (BF16) and targets y_dev[max_rows][64]
 * (32 basis indicators of the optimal stencil's non-zero fractions, 32
 * fractions).  *rows_host = rows written.  Synchronises. */
int vrm_collect_training(vrm_ctx* ctx, const vrm_cloud* cloud, const vrm_params* p, uint16_t* x_dev, float* y_dev,
                         int32_t max_rows, int32_t* rows_host);
/* One AdamW step (lr, weight decay; beta 0.9 / 0.999) on the mean over rows of
 * masked BCE-with-logits on the indicators plus frac_weight times the masked
 * squared error of the fractions.  loss_dev (one double) and grad_dev
 * (VRM_MLP_PARAMS floats, before the step) may be NULL.  lr = 0 computes the
 * loss and gradient only. */
int vrm_mlp_train_step(vrm_ctx* ctx, const uint16_t* x_dev, const float* y_dev, int32_t rows, float lr,
                       float weight_decay, float frac_weight, double* loss_dev, float* grad_dev);
/* Test hook of the learned warm start: the network outputs the warm pass would use
 * for the LPs queued at the current positions and diffused set (small LPs for
 * q = 2: their 8 logits in columns 0..7, zeros after; complete LPs for q = 3: the
 * 32 basis logits in columns 0..31, zeros after), computed by the kernels of the
 * LP path (input rows built on the device from the LPs' column lists).  out_dev[max_rows][64] FP32, particle_dev[max_rows]: the
 * cloud index of each row's particle; *rows_host = rows written.  Needs
 * vrm_set_warm_start(ctx, 1).  Synchronises. */
int vrm_warm_predictions(vrm_ctx* ctx, const vrm_cloud* cloud, const vrm_params* p, float* out_dev,
                         int32_t* particle_dev, int32_t max_rows, int32_t* rows_host);
/* Forward pass: y_dev[rows][64] from x_dev[rows][128]. */
int vrm_mlp_infer(vrm_ctx* ctx, const uint16_t* x_dev, int32_t rows, float* y_dev);
/* Matrix product on the BF16 matrix cores (test hook): C[M][N] (FP32, zeroed
 * by the caller) += op(A) op(B) with A[M][K] (or [K][M] if transA) and B[K][N]
 * (or [N][K] if transB), BF16 row-major. */
int vrm_gemm_bf16(vrm_ctx* ctx, const uint16_t* a_dev, const uint16_t* b_dev, float* c_dev, int32_t M, int32_t N,
                  int32_t K, int transA, int transB);

/* Kernel timers (profiling).  While enabled, every launch of the kernel
 * groups below is bracketed by HIP events recorded on the context's stream
 * (a few microseconds of overhead per launch).  vrm_read_timing synchronises,
 * adds the elapsed times per group into ms_host[VRM_NTIMER] and the launch
 * counts into launches_host[VRM_NTIMER] (either may be NULL), and starts a new
 * interval.  At most 8192 launches are timed per interval; later ones are
 * counted in launches_host but not timed (the return value is then 1). */
#define VRM_T_SELECT 0      /* reduced-operator selection (Sec. 3.5) */
#define VRM_T_CELLS 1       /* cell list build */
#define VRM_T_NBHD 2        /* small neighbourhoods (Sec. 4.3) */
#define VRM_T_LP_SMALL 3    /* small-neighbourhood LPs + apply */
#define VRM_T_LP_FULL 4     /* complete-neighbourhood LPs + apply */
#define VRM_T_INSERT 5      /* insertion (Sec. 4.2), including its host synchronisations */
#define VRM_T_COMBINE 6     /* Runge-Kutta stage combination */
#define VRM_T_MLP 7         /* warm-start network */
#define VRM_T_FULL_COLS 8   /* complete-neighbourhood column lists and their size bins (q = 3) */
#define VRM_NTIMER 9
int vrm_timing(vrm_ctx* ctx, int enable);
/* The same for the groups whose bit (1 << VRM_T_*) is set in `groups` only:
 * the other groups launch without events (0: timers off). */
int vrm_timing_groups(vrm_ctx* ctx, uint32_t groups);
int vrm_read_timing(vrm_ctx* ctx, double* ms_host, int64_t* launches_host);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the diffused-set selection
 * of vrm_select_diffused (Sec. 3.5, eq. reduced_bound; the same ranking, bound,
 * round-off band and result) without a context.  gamma_dev[n] (device FP32,
 * caller-owned) in; mask_dev[n] (device uint8, caller-owned) out, 1 = diffused;
 * nonfinite_dev (device int32, may be NULL) receives 2 if a circulation is NaN or
 * infinite, else 0.  h, q (2 or 3), c_diff as in vrm_params.  Runs on the current
 * device, enqueued on `stream` (a hipStream_t of that device; NULL = the null
 * stream), without synchronising.  Its working state (histogram bins, threshold,
 * flag: about 3 KB) lives in one fixed device array per GPU, kept until the
 * process ends; the call allocates nothing and clears that state itself.  Every
 * call on a GPU shares its array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  n up to 2^26;
 * VRM_E_ARG for larger n, NULL pointers or bad parameters. */
int vrm_select_diffused_static(const float* gamma_dev, int32_t n, double h, int32_t q, double c_diff,
                               uint8_t* mask_dev, int32_t* nonfinite_dev, void* stream);

const char* vrm_last_error(void);
const char* vrm_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* VRM_H */
