// Runge-Kutta stage combination, FP64 verification and the prescribed
// velocity harness of libvrm.
//
// Stage update: Sec. 3.3 (Euler steps; SSP Runge-Kutta schemes are convex
// combinations of them) with the Shu-Osher SSP-RK3 weights, applied to
// Gamma with dGamma_i/dt = nu sum_j f_ji Gamma_j (Sec. 3.4, eq. nsode) and to
// the positions with the caller's velocity.
#include <hip/hip_runtime.h>

#include "vrm_device.h"
#include "vrm_internal.h"

using namespace vrm;

namespace {

// n_dev (optional): the particle count read on the device (graph replays), else n.
// det: the accumulator holds 64-bit fixed-point sums (scale det_scale).  While a
// non-finite value is flagged the accumulator is cleared and the cloud is left
// as it is.
__global__ __launch_bounds__(256) void k_combine(int n, const int32_t* __restrict__ n_dev, float a, float b, float dt,
                                                 float lam, const float* __restrict__ x0, const float* __restrict__ y0,
                                                 const float* __restrict__ g0, float* x, float* y, float* g,
                                                 const float* __restrict__ u, const float* __restrict__ v, float* acc,
                                                 const GridState* gs, int det)
{
    if (n_dev) n = *n_dev;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float sum;
    if (det) {
        unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(acc);
        const long long w = (long long)acc64[i];
        acc64[i] = 0ull;
        sum = (float)((double)w * (1.0 / det_scale(gs->gmax_bits)));
    } else {
        sum = acc[i];
        acc[i] = 0.0f;
    }
    if (gs->bad) return;
    float dg = lam * sum;
    float gn = __builtin_fmaf(dt, dg, g[i]);
    float gst = b * gn;
    if (a != 0.0f) gst = __builtin_fmaf(a, g0[i], gst);
    g[i] = gst;
    if (u) {
        float xn = __builtin_fmaf(dt, u[i], x[i]);
        float yn = __builtin_fmaf(dt, v[i], y[i]);
        float xs = b * xn, ys = b * yn;
        if (a != 0.0f) {
            xs = __builtin_fmaf(a, x0[i], xs);
            ys = __builtin_fmaf(a, y0[i], ys);
        }
        x[i] = xs;
        y[i] = ys;
    } else if (a != 0.0f) {
        // zero velocity: positions stay exactly y^n (the convex combination is the identity)
        x[i] = x0[i];
        y[i] = y0[i];
    }
}

// FP64 moment residual of each stencil (rows 1 <= |alpha| <= q, relative to
// b = 2), circulation and l1 norm, and the largest sum_j fhat_ij.
__global__ __launch_bounds__(256) void k_verify(int n, const float* __restrict__ x, const float* __restrict__ y,
                                                const float* __restrict__ g, double h, int q,
                                                const int32_t* __restrict__ sidx, const float* __restrict__ sf,
                                                const uint8_t* __restrict__ status, const int32_t* __restrict__ fk,
                                                const int32_t* __restrict__ fidx, const float* __restrict__ ff,
                                                unsigned long long* out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double res = 0.0, i0 = 0.0, l1 = 0.0, fsum = 0.0;
    if (i < n) {
        double gi = (double)g[i];
        i0 = gi;
        l1 = fabs(gi);
        int st = status ? status[i] : 3;
        if (st == VRM_ST_WARM) st = (fk && fk[i] > 0) ? 1 : 0;   // warm-started: small or complete
        if (st <= 1) {
            double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            double xi = (double)x[i], yi = (double)y[i];
            int k = st == 0 ? VRM_NSEG : fk[i];
            for (int t = 0; t < k; ++t) {
                int j;
                double f;
                if (st == 0) {
                    j = sidx[(size_t)i * VRM_NSEG + t];
                    f = (double)sf[(size_t)i * VRM_NSEG + t];
                } else {
                    j = fidx[(size_t)i * VRM_KMAX + t];
                    f = (double)ff[(size_t)i * VRM_KMAX + t];
                }
                if (j < 0) continue;
                double rx = ((double)x[j] - xi) / h, ry = ((double)y[j] - yi) / h;
                m[0] += f * rx;
                m[1] += f * ry;
                m[2] += f * rx * rx;
                m[3] += f * rx * ry;
                m[4] += f * ry * ry;
                m[5] += f * rx * rx * rx;
                m[6] += f * rx * rx * ry;
                m[7] += f * rx * ry * ry;
                m[8] += f * ry * ry * ry;
                fsum += f;
            }
            m[2] -= 2.0;
            m[4] -= 2.0;
            int rows = q == 2 ? 5 : 9;
            for (int a = 0; a < rows; ++a) res = fmax(res, fabs(m[a]) / 2.0);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        res = fmax(res, __shfl_xor(res, o, VRM_WAVE));
        fsum = fmax(fsum, __shfl_xor(fsum, o, VRM_WAVE));
        i0 += __shfl_xor(i0, o, VRM_WAVE);
        l1 += __shfl_xor(l1, o, VRM_WAVE);
    }
    if (lane_id() == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(res));
        atomicAdd((double*)&out[1], i0);
        atomicAdd((double*)&out[2], l1);
        atomicMax(&out[3], (unsigned long long)__double_as_longlong(fsum));
    }
}

// y^n of the step; also flags a non-finite circulation (kBadGamma) and, for the
// fixed-point accumulation (det), finds max |Gamma^n| (k_gmax_reset first)
__global__ __launch_bounds__(256) void k_save_base(int n, const int32_t* __restrict__ n_dev,
                                                   const float* __restrict__ x, const float* __restrict__ y,
                                                   const float* __restrict__ g, float* x0, float* y0, float* g0,
                                                   GridState* gs, int det)
{
    if (n_dev) n = *n_dev;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t bits = 0u;
    if (i < n) {
        const float gi = g[i];
        x0[i] = x[i];
        y0[i] = y[i];
        g0[i] = gi;
        bits = __float_as_uint(fabsf(gi));
    }
    if (__any(bits >= 0x7f800000u) && lane_id() == 0) atomicOr(&gs->bad, kBadGamma);
    if (det) {
        for (int o = 32; o > 0; o >>= 1) bits = max(bits, (uint32_t)__shfl_xor((int)bits, o, VRM_WAVE));
        if (lane_id() == 0 && bits < 0x7f800000u) atomicMax(&gs->gmax_bits, bits);
    }
}

__global__ void k_gmax_reset(GridState* gs) { gs->gmax_bits = 0u; }

__global__ void k_verify_init(unsigned long long* out)
{
    out[0] = 0ull;
    out[1] = 0ull;
    out[2] = 0ull;
    out[3] = 0ull;
}

// Prescribed velocity of Lamb-Oseen vortices (centre, core sigma, circulation G):
// u(x) = sum_k G_k (-d_y, d_x) (1 - exp(-|d|^2 / (sigma_k^2 + 4 nu t))) / (2 pi |d|^2),
// d = x - centre_k, and 0 at a centre.  Time = t, or *t_dev + t when t_dev is
// given (graph replays).  Each thread holds kVelT targets, so the per-vortex
// constants a = G / (2 pi) and b = log2(e) / (sigma^2 + 4 nu t) (one hardware
// reciprocal) are paid once per kVelT pairs; a pair costs two differences, two
// FMAs for |d|^2, exp2(-b |d|^2), a reciprocal of |d|^2, one product, one FMA
// for t - t e, a select and two accumulating FMAs, with no IEEE division.
// A pair with |d|^2 <= 1e-30 (a target on a centre) contributes 0.
constexpr int kVelT = 4;

__global__ __launch_bounds__(256) void k_velocity(int n, const int32_t* __restrict__ n_dev,
                                                  const float* __restrict__ x, const float* __restrict__ y,
                                                  const float* __restrict__ vort, int nv, double nu, double t,
                                                  const double* __restrict__ t_dev, float* u, float* v)
{
    if (n_dev) n = *n_dev;
    const int base = blockIdx.x * (256 * kVelT) + threadIdx.x;
    if (base >= n) return;
    const double tt = t_dev ? *t_dev + t : t;
    const float four_nu_t = (float)(4.0 * nu * tt);
    const float inv2pi = 0.15915494309189535f, log2e = 1.4426950408889634f;
    float xi[kVelT], yi[kVelT], su[kVelT], sv[kVelT];
#pragma unroll
    for (int j = 0; j < kVelT; ++j) {
        const int i = min(base + 256 * j, n - 1);
        xi[j] = x[i];
        yi[j] = y[i];
        su[j] = 0.0f;
        sv[j] = 0.0f;
    }
    for (int k = 0; k < nv; ++k) {
        const float cx = vort[4 * k], cy = vort[4 * k + 1], s = vort[4 * k + 2];
        const float a = vort[4 * k + 3] * inv2pi;
        const float b = -log2e * __builtin_amdgcn_rcpf(__builtin_fmaf(s, s, four_nu_t));
#pragma unroll
        for (int j = 0; j < kVelT; ++j) {
            const float dx = xi[j] - cx, dy = yi[j] - cy;
            const float r2 = __builtin_fmaf(dx, dx, dy * dy);
            const float ex = __builtin_amdgcn_exp2f(b * r2);
            const float tr = __builtin_amdgcn_rcpf(r2) * a;
            const float f = r2 > 1e-30f ? __builtin_fmaf(-tr, ex, tr) : 0.0f;
            su[j] = __builtin_fmaf(-f, dy, su[j]);
            sv[j] = __builtin_fmaf(f, dx, sv[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < kVelT; ++j) {
        const int i = base + 256 * j;
        if (i < n) {
            u[i] = su[j];
            v[i] = sv[j];
        }
    }
}

int blocks_for(int n) { return n > 0 ? (n + 255) / 256 : 1; }

// ------------------------------------------------------------ Biot-Savart (direct sum)
// u(x_i) = sum_j Gamma_j K_eps(x_i - x_j) with K_eps(d) = (-d_y, d_x) (1 - exp(-|d|^2 / eps^2))
// / (2 pi |d|^2) and K_eps(0) = 0 (Sec. 3.4 eq. nsode, the regularised kernel of Sec. 5).
// Each thread accumulates kBsT targets; a workgroup streams one chunk of the
// sources (blockIdx.y) through LDS in tiles of kBsTile, and the chunks' partial
// sums meet in u, v by atomics (distinct addresses: no contention).
// Positions are scaled by s = sqrt(log2 e) / eps, so that with D = s d the
// exponential is exp2(-|D|^2) and the pair term is s Gamma_j (-D_y, D_x)
// (1 - 2^-|D|^2) / (2 pi |D|^2): per pair two differences, two FMAs for |D|^2,
// exp2, a reciprocal, one product, one FMA for t - t e and two accumulating
// FMAs; s multiplies the sums once.  The 1e-30 added to |D|^2 makes the self
// term 0 * finite instead of a branch.
constexpr int kBsBlock = 256;
constexpr int kBsT = 2;
constexpr int kBsTile = 512;

__global__ __launch_bounds__(kBsBlock) void k_biot_savart(const int32_t* __restrict__ n_dev,
                                                          const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ g, float sc, int chunk,
                                                          float* u, float* v)
{
    __shared__ float4 s_src[kBsTile];
    const int n = *n_dev;
    const int tid = threadIdx.x;
    float xt[kBsT], yt[kBsT], su[kBsT], sv[kBsT];
#pragma unroll
    for (int k = 0; k < kBsT; ++k) {
        const int a = blockIdx.x * (kBsBlock * kBsT) + k * kBsBlock + tid;
        xt[k] = a < n ? x[a] * sc : 0.0f;
        yt[k] = a < n ? y[a] * sc : 0.0f;
        su[k] = 0.0f;
        sv[k] = 0.0f;
    }
    const float inv2pi = 0.15915494309189535f;
    const int j0 = blockIdx.y * chunk, j1 = min(j0 + chunk, n);
    for (int base = j0; base < j1; base += kBsTile) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kBsTile / kBsBlock; ++q) {
            const int e = q * kBsBlock + tid, j = base + e;
            s_src[e] = j < j1 ? make_float4(x[j] * sc, y[j] * sc, g[j] * inv2pi, 0.0f)
                              : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        __syncthreads();
#pragma unroll 4
        for (int e = 0; e < kBsTile; ++e) {
            const float4 s = s_src[e];
#pragma unroll
            for (int k = 0; k < kBsT; ++k) {
                const float dx = xt[k] - s.x, dy = yt[k] - s.y;
                const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, 1e-30f));
                const float ex = __builtin_amdgcn_exp2f(-r2);
                const float t = __builtin_amdgcn_rcpf(r2) * s.z;
                const float f = __builtin_fmaf(-t, ex, t);
                su[k] = __builtin_fmaf(-dy, f, su[k]);
                sv[k] = __builtin_fmaf(dx, f, sv[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kBsT; ++k) {
        const int a = blockIdx.x * (kBsBlock * kBsT) + k * kBsBlock + tid;
        if (a < n) {
            atomicAdd(&u[a], su[k] * sc);
            atomicAdd(&v[a], sv[k] * sc);
        }
    }
}

__global__ void k_zero_uv(const int32_t* __restrict__ n_dev, float* u, float* v)
{
    const int n = *n_dev;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        u[i] = 0.0f;
        v[i] = 0.0f;
    }
}

}  // namespace

int vrm_biot_savart_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, double eps, float* u, float* v)
{
    if (n <= 0) return VRM_OK;
    hipLaunchKernelGGL(k_zero_uv, dim3(min(blocks_for(n), 1024)), dim3(256), 0, c->stream, cl->n_dev, u, v);
    const int tx = (n + kBsBlock * kBsT - 1) / (kBsBlock * kBsT);
    // source chunks: enough workgroups to fill the chip (>= 2048), whole tiles each
    const int tiles = (n + kBsTile - 1) / kBsTile;
    const int sy = max(1, min(tiles, (2048 + tx - 1) / tx));
    const int chunk = ((tiles + sy - 1) / sy) * kBsTile;
    const int ny = (n + chunk - 1) / chunk;
    const float sc = (float)(sqrt(1.4426950408889634) / eps);
    hipLaunchKernelGGL(k_biot_savart, dim3(tx, ny), dim3(kBsBlock), 0, c->stream, cl->n_dev, cl->x_dev, cl->y_dev,
                       cl->gamma_dev, sc, chunk, u, v);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_combine_run(vrm_ctx* c, vrm_cloud* cl, int32_t n, const float* u, const float* v, double dt, float lam,
                    int stage, int det)
{
    static const float A[3] = {0.0f, 0.75f, 1.0f / 3.0f};
    static const float B[3] = {1.0f, 0.25f, 2.0f / 3.0f};
    if (n <= 0) return VRM_OK;
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(256), 0, c->stream, n, cl->n_dev, A[stage], B[stage],
                       (float)dt, lam, c->x0, c->y0, c->g0, cl->x_dev, cl->y_dev, cl->gamma_dev, u, v, c->acc, c->grid,
                       det);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_save_base_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, int det)
{
    if (n <= 0) return VRM_OK;
    if (det) hipLaunchKernelGGL(k_gmax_reset, dim3(1), dim3(1), 0, c->stream, c->grid);
    hipLaunchKernelGGL(k_save_base, dim3(blocks_for(n)), dim3(256), 0, c->stream, n, cl->n_dev, cl->x_dev, cl->y_dev,
                       cl->gamma_dev, c->x0, c->y0, c->g0, c->grid, det);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_verify_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const LaunchParams& lp, double h,
                   const vrm_stencils* st, double* report)
{
    unsigned long long* out = reinterpret_cast<unsigned long long*>(report);
    hipLaunchKernelGGL(k_verify_init, dim3(1), dim3(1), 0, c->stream, out);
    if (n > 0) {
        hipLaunchKernelGGL(k_verify, dim3(blocks_for(n)), dim3(256), 0, c->stream, n, cl->x_dev, cl->y_dev,
                           cl->gamma_dev, h, lp.q, st ? st->small_idx_dev : nullptr,
                           st ? st->small_f_dev : nullptr, st ? st->status_dev : nullptr,
                           st ? st->full_k_dev : nullptr, st ? st->full_idx_dev : nullptr,
                           st ? st->full_f_dev : nullptr, out);
    }
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_velocity_run(vrm_ctx* c, const vrm_cloud* cl, int32_t n, const float* vort, int32_t nv, double nu, double t,
                     float* u, float* v, const double* t_dev)
{
    if (n <= 0) return VRM_OK;
    hipLaunchKernelGGL(k_velocity, dim3((n + 256 * kVelT - 1) / (256 * kVelT)), dim3(256), 0, c->stream, n, cl->n_dev, cl->x_dev, cl->y_dev,
                       vort, nv, nu, t, t_dev, u, v);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}
