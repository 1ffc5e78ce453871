// Internal state of a libvrm context and the kernel launchers shared by the
// translation units.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vrm.h"
#include "vrm_mlp.h"

namespace vrm {

// The device counters live in kCounterStripes copies, one per 256-byte line.
// Accumulating kernels add to the copy of their workgroup, so that the waves of
// a large launch do not queue on one address; vrm_read_counters sums the
// copies.  Fields that are assigned (not accumulated) live in copy 0.
constexpr int kCounterStripes = 64;
constexpr size_t kCounterStride = (sizeof(vrm_counters) + 255) / 256 * 256;

// Append `want` entries per thread to a queue whose tail is *counter: positions
// follow the thread order of the workgroup, with one atomic per workgroup (a
// large launch then does not queue on one address).  Every thread of the
// workgroup must call it; s_tmp is __shared__ int[17].
__device__ __forceinline__ int block_append_n(int* counter, int want, int* s_tmp)
{
    const int lane = __lane_id(), w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int incl = want;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_tmp[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < nw; ++k) {
            const int c = s_tmp[k];
            s_tmp[k] = tot;
            tot += c;
        }
        s_tmp[16] = tot ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    const int pos = s_tmp[16] + s_tmp[w] + incl - want;
    __syncthreads();
    return pos;
}

__device__ __forceinline__ vrm_counters* counter_stripe(vrm_counters* base)
{
    return reinterpret_cast<vrm_counters*>(reinterpret_cast<char*>(base) +
                                           (size_t)(blockIdx.x % kCounterStripes) * kCounterStride);
}

// Grid of square cells over the bounding box of the cloud (device side).
struct GridState {
    uint32_t bbox[4];      // ordered keys: min x, min y, max x, max y
    float x0, y0, cs, inv_cs;
    int32_t nx, ny, ncells, clamped;
    // kBadPos: a position the last cell build read was not finite; kBadGamma: a
    // circulation the last selection or stage-0 copy read was not finite.  While
    // either bit is set no cell index is formed and no kernel changes the cloud.
    int32_t bad;
    // bits of max |Gamma^n| (stage 0): scale of the fixed-point accumulation
    uint32_t gmax_bits;
};
constexpr int32_t kBadPos = 1;
constexpr int32_t kBadGamma = 2;

// Queue counters of a stage (device side).
struct Queues {
    int32_t n_small;       // items in the small-LP queue
    int32_t n_full;        // items in the complete-LP queue
    int32_t n_cand;        // insertion candidates
    int32_t n_undecided;   // non-zero while insertion candidates are undecided
    int32_t n_accepted;    // accepted insertion candidates
    int32_t small_state;   // single-workgroup insertion: 0 not taken, 1 done, 2 capacity exceeded
    int32_t n_retry;       // LPs left by the warm pass for a cold solve
    int32_t blocks_done;   // blocks of the last LP launch that have finished
    int32_t last_small;    // n_small and n_full of the last stencil run (the queues
    int32_t last_full;     // themselves are zero between runs)
    int32_t n_removed;     // particle removal: particles removed by the last call
    int32_t n_rm_uncertified;   // ... of which optimality was not certified
    int32_t nonfinite;     // copy of GridState::bad taken when the record is published
    int32_t n_defer;       // complete LPs whose certification was deferred to a second launch
};

// Queue record published to pinned, coherent host memory: the kernel writes q,
// then seq last with a system-scope release; the host reads q once it sees the
// sequence number it asked for.
struct HostQueues {
    Queues q;
    int32_t seq;
};

// Column records of the queued small-neighbourhood LPs, in queue order and
// plane-major (plane p of item r at p * cap + r) so that the LP and network
// kernels read them coalesced instead of gathering neighbours.
struct SmallRec {
    int32_t cap;     // plane stride
    int32_t* i;      // [cap] cloud index of the particle
    int32_t* rank;   // [cap] id ranks of its 8 columns, 3 bits each (segment s at bit 3 s)
    int32_t* pj;     // [8][cap] cloud index of the column of segment s, -1 if the segment is empty
    float* off;      // [32][cap] exact scaled offset of segment s: planes 4s..4s+3 = X.hi, X.lo, Y.hi, Y.lo
};

// Column records of the queued complete LPs, as the network's inference reads them.
struct FullRec {
    const int32_t* rec;      // [item][row] (slot << 6) | id rank per column, nearest first
    int32_t row;             // record row stride
    const int32_t* kcol;     // [item] column count; -1: the list is left for the one-thread kernel
    const int32_t* q_full;   // [item] sorted-cloud index of the particle
    const float* xs;         // sorted positions
    const float* ys;
    float scale2e, sc;       // ((x_j - x_i) scale2e) sc is column j's offset over h
    int q;
};

// Reduced-operator selection state (device side).
struct SelectState {
    double norm1, bound, prefix;
    uint32_t key_prefix;   // resolved high bits of the threshold key
    uint32_t done;         // 1 once the threshold is known
    uint32_t threshold;    // particles with key < threshold are left out
    int32_t max_id;        // largest id of the cloud (new particles get max_id + 1, ...)
    double bin_sum[256];
    uint32_t bin_cnt[256];
};

struct LaunchParams {
    float h, lo2, hi2, lo2f, hi2f;      // annulus bounds (FP32, squared, unnormalised)
    float rad, ex2;                      // insertion radius 1.5 h and exclusion (0.5 h)^2
    float scale2e;                       // 2^-e with 2^e >= h: exact offset scaling
    float bt_hi, bt_lo;                  // rhs 2 h^2 / 4^e of the (2,0), (0,2) rows (double-float)
    float cs_hi, cs_lo;                  // (2^e / h)^(q+1): cost scale (double-float)
    float lam;                           // nu / h^2
    float sc;                            // 2^e / h: scaled offset -> offset / h
    int q, m;
    int phase1;                          // 1: stop at the first feasible vertex (phase I only)
    int det;                             // 1: order-independent fixed-point accumulation of the update
    int max_cert;                        // certification rounds of one LP (kMaxCert unless tuned)
};
constexpr int kMaxCert = 8;              // certification rounds: primal / dual repairs of one LP

// Fixed-point accumulation (deterministic mode): every contribution f Gamma is
// rounded to a multiple of 2^(e - 46), where max |Gamma^n| < 2^e, and summed as
// a 64-bit integer, so the sum does not depend on the order of the atomics and
// particles with equal contributions get bit-identical sums.  A fraction is at
// most 16 (Sec. 3.2 lemma: sum_{j != i} fhat_ij <= 4 / r^2), a stage value at
// most 4 max|Gamma^n|, and a particle receives at most 2^10 contributions, so
// every scaled sum stays below 2^62 in magnitude.
__device__ __forceinline__ double det_scale(uint32_t gmax_bits)
{
    const int e = (int)((gmax_bits >> 23) & 255u) - 126;   // max|Gamma| < 2^e
    return __builtin_ldexp(1.0, 46 - e);
}
__device__ __forceinline__ void acc_add(float* acc, int j, float f, float g, double dsc)
{
    if (dsc != 0.0)
        atomicAdd(reinterpret_cast<unsigned long long*>(acc) + j,
                  (unsigned long long)(long long)__builtin_rint((double)f * (double)g * dsc));
    else
        atomicAdd(acc + j, f * g);
}

}  // namespace vrm

struct vrm_ctx {
    int device;
    hipStream_t stream;
    int32_t capacity;
    int32_t ncell_cap;
    // cached count for the cloud last seen (host)
    const int32_t* n_ptr;
    int32_t n;
    int32_t n_diffused_valid;   // the diffused set matches the cloud
    int32_t cells_valid;        // cell list matches the current positions
    int32_t base_valid;         // y^n recorded (stage 0 done)
    int32_t sorted;             // cloud in cell order of the current cell list (perm is the identity)
    const float* cloud_x;       // cloud seen last (cached state belongs to it)
    float* u_tmp;               // [cap] stage velocity (vrm_step with prescribed vortices)
    float* v_tmp;
    // device buffers
    vrm::GridState* grid;
    vrm::Queues* queues;
    vrm::HostQueues* q_host;    // pinned, coherent host copy of *queues (vrm_read_queues)
    int32_t q_seq;              // last sequence number asked of it
    vrm::SelectState* sel;
    vrm_counters* counters;
    int32_t* cell_of;     // [cap] cell of particle
    int32_t* rank;        // [cap] rank within its cell
    int32_t* cell_start;  // [ncell_cap + 1]
    int32_t* scan_part;   // [1024]
    int32_t* perm;        // [cap] slot -> particle
    float* xs;            // [cap] positions in slot order
    float* ys;
    int32_t* ids;         // [cap] ids in slot order
    uint8_t* diffused;    // [cap] per particle
    float* acc;           // [2 cap] sum_j fhat_ji Gamma_j (FP32, or int64 fixed point when deterministic)
    float* x0;            // [cap] stage-0 state
    float* y0;
    float* g0;
    int32_t* q_small;     // [cap] slots queued for the small LP
    int32_t* q_full;      // [cap] slots queued for the complete LP
    int32_t* q_retry;     // [cap] slots the warm pass leaves for a cold solve
    vrm::SmallRec srec;   // column records of the queued small LPs
    // insertion
    float* cx;            // [2 cap] candidate positions
    float* cy;
    uint64_t* ckey;       // [2 cap] (id << 3) | segment
    uint8_t* cstate;      // [2 cap] 0 undecided, 1 in, 2 out
    int32_t* ccell;       // [2 cap]
    int32_t* crank;
    int32_t* cstart;      // [ncell_cap + 1]
    int32_t* cperm;       // [2 cap]
    uint64_t* akey;       // [2 cap] accepted keys / sort scratch
    int32_t* aidx;
    void* sort_tmp;
    size_t sort_tmp_bytes;
    // reorder scratch
    float* tmp_f;         // [3 cap]
    int32_t* tmp_i;       // [cap]
    uint8_t* tmp_u8;      // [cap]
    double* verify_buf;   // [8]
    int lp_objective;     // 0 canonical stencil (phase II), 1 first feasible vertex (phase I only)
    // kernel timers
    int timing;
    uint32_t timing_groups;   // bit g: group g is timed
    int ntimed;
    hipEvent_t* ev_start; // [kMaxTimed]
    hipEvent_t* ev_stop;
    int* ev_group;
    int64_t launches[VRM_NTIMER];
    double acc_ms[VRM_NTIMER];   // timings accumulated from graph replays
    int64_t acc_n[VRM_NTIMER];
    // the three stages of vrm_step as one HIP graph
    int capturing;               // the stream is being captured: timers take graph slots
    int graph_enabled;
    int64_t graph_replays;
    int graph_failed[2];         // capture failed (without / with timers): launch directly
    int graph_slots;             // timer slots used by the graph
    int graph_pending;           // a replay whose timer events are not yet accumulated
    int graph_nb;                // particle bound the graph's grids are sized for
    int graph_flags[3];          // cells_valid, sorted, base_valid after the stages
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    unsigned char graph_key[256];
    double* t_dev;               // step start time read by the graph's velocity kernels
    int32_t* prev;               // [cap][9] basis (column ids) of each particle's last stencil, by id
    uint64_t* pmask;             // [cap] crash basis (previous or predicted) as a column mask per complete LP
    int32_t* lkey;               // [cap] bin of each complete LP for the counting sort (pivot history or doubt)
    int32_t* q_defer;            // [cap] queue items the LP launch deferred (bit 31: settled warm; bit 30: solve cold)
    uint8_t* pivhist;            // [cap] by particle id: pivots of its last complete LP (255: none yet)
    vrm_tuning tuning;           // launch shapes in force (defaults filled in)
    hipStream_t cap_stream;      // stream the graph is captured on (the context's may be the null stream)
    // warm-start network (allocated on first use)
    vrm::MlpState* mlp;
    int warm;             // LP solves use the network's basis prediction
    uint16_t* feat;       // [cap][128] feature rows of the queued LPs (warm start / collection)
    float* pred;          // [cap][64] network outputs
    float* labels;        // [cap][64] collection targets
    int32_t* full_cols;   // [cap][48] complete-neighbourhood columns nearest first: (slot << 6) | id rank
    int32_t* full_k;      // [cap] their counts, by queue item
    int32_t* full_order;  // [cap] queue items grouped by decreasing count
    int32_t* khist;       // [2 (VRM_KMAX + 1)] histogram of the counts, then the bins' fill pointers
    int32_t feat_cap;
};

namespace vrm {
constexpr int kMaxTimed = 8192;
constexpr int kGraphTimed = 64;   // the last kGraphTimed event pairs belong to the step graph
// Bracket a group of launches with events when timing is on.
struct ScopedTimer {
    vrm_ctx* c;
    int slot;
    ScopedTimer(vrm_ctx* ctx, int group) : c(ctx), slot(-1)
    {
        if (!c->timing || !((c->timing_groups >> group) & 1u)) return;
        if (c->capturing) {
            // an event-record node of the step graph; counted when a replay is accumulated
            if (c->graph_slots >= kGraphTimed) return;
            slot = kMaxTimed - kGraphTimed + c->graph_slots++;
        } else {
            c->launches[group] += 1;
            if (c->ntimed >= kMaxTimed - kGraphTimed) return;
            slot = c->ntimed++;
        }
        c->ev_group[slot] = group;
        (void)hipEventRecord(c->ev_start[slot], c->stream);
    }
    ~ScopedTimer()
    {
        if (slot >= 0) (void)hipEventRecord(c->ev_stop[slot], c->stream);
    }
};
}  // namespace vrm

// launchers (vrm_cells.hip)
int vrm_build_cells(vrm_ctx* c, const float* x, const float* y, const int32_t* id, int32_t n,
                    const vrm::LaunchParams& lp, const int32_t* n_dev = nullptr);
int vrm_select_run(vrm_ctx* c, const float* gamma, const int32_t* ids, int32_t n, double bound_factor);
int vrm_insert_run(vrm_ctx* c, vrm_cloud* cl, int32_t n, const vrm::LaunchParams& lp);
// the queue record after the work enqueued so far on the context's stream,
// read from the pinned host copy (no stream synchronisation)
int vrm_read_queues(vrm_ctx* c, vrm::Queues& q);
int vrm_reorder_cloud(vrm_ctx* c, vrm_cloud* cl, int32_t n);
int vrm_remove_run(vrm_ctx* c, vrm_cloud* cl, int32_t n, const vrm::LaunchParams& lp, int32_t* n_candidates);
size_t vrm_remove_tmp_bytes(int32_t cap);
// launchers (vrm_lp.hip)
int vrm_stencil_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const vrm::LaunchParams& lp,
                    const vrm_stencils* out, int apply, uint16_t* feat_out = nullptr, float* label_out = nullptr,
                    int max_rows = 0);
int vrm_small_nbhd_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const vrm::LaunchParams& lp,
                       int32_t* small_idx, int32_t* kfull);
int vrm_warm_predict_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const vrm::LaunchParams& lp, float* out,
                         int32_t* particle, int max_rows);
// launchers (vrm_stage.hip)
int vrm_combine_run(vrm_ctx* c, vrm_cloud* cl, int32_t n, const float* u, const float* v, double dt,
                    float lam, int stage, int det);
int vrm_save_base_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, int det);
int vrm_biot_savart_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, double eps, float* u, float* v);
int vrm_verify_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const vrm::LaunchParams& lp, double h,
                   const vrm_stencils* st, double* report);
int vrm_velocity_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const float* vort, int32_t nv, double nu,
                     double t, float* u, float* v, const double* t_dev = nullptr);

// launchers (vrm_mlp.hip)
int vrm_mlp_alloc(vrm_ctx* c, int max_rows);
void vrm_mlp_free(vrm_ctx* c);
int vrm_mlp_set_weights(vrm_ctx* c, const float* w_dev);
int vrm_mlp_forward(vrm_ctx* c, const uint16_t* X, int rows, float* Y, const int* rows_dev);
int vrm_mlp_read_weights(vrm_ctx* c, float* w_dev);
int vrm_mlp_infer_run(vrm_ctx* c, const uint16_t* X, int rows, float* Y, const int* rows_dev);
// warm-start logits (8 per queued small LP) with the network input built from the positions
int vrm_mlp_infer_full_run(vrm_ctx* c, int rows, const int* rows_dev, const vrm::FullRec& fr, float* L);
int vrm_mlp_infer_small_run(vrm_ctx* c, int rows, const int* rows_dev, const vrm::SmallRec& rec, float sc, int q,
                            float* L);
int vrm_mlp_train(vrm_ctx* c, const uint16_t* X, const float* T, int rows, float lr, float wd, float wf,
                  double* loss_out, float* grad_out);
int vrm_gemm_test(vrm_ctx* c, const uint16_t* A, const uint16_t* B, float* C, int M, int N, int K, int transA,
                  int transB);

// error helpers (vrm_api.cpp)
int vrm_fail(int code, const char* fmt, ...);
// report a non-finite input (GridState::bad bits): clears the device flag and
// drops the context's cached cell list and diffused set; returns VRM_E_NONFINITE
int vrm_nonfinite(vrm_ctx* c, int32_t bits);
int vrm_hip_check(hipError_t e, const char* what);
#define VRM_HIP(call)                                                    \
    do {                                                                 \
        hipError_t _e = (call);                                          \
        if (_e != hipSuccess) return vrm_hip_check(_e, #call);           \
    } while (0)
