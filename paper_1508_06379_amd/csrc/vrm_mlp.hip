// Warm-start network of libvrm: a small MLP that predicts, from the offsets of
// an LP's columns, which columns form the optimal basis and their fractions.
//
//   x[128] (32 slots x (dx/h, dy/h), 32 slot masks, q - 2, zero padding)
//     -> 128 (GELU) -> 128 (GELU) -> 64 (32 basis logits, 32 fractions)
//
// Every matrix product runs on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation) in one generic tiled kernel with fused epilogues; the
// backward pass uses the same kernel with transposed operand strides and
// split-K atomics for the weight gradients.  Master weights and AdamW state
// are FP32; the products read BF16 copies.
#include <hip/hip_runtime.h>

#include "vrm_device.h"
#include "vrm_internal.h"
#include "vrm_mlp.h"

using namespace vrm;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 to BF16, round to nearest even (the conversion instruction of gfx950)
__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU in its tanh form: z sigma(2u) with u = sqrt(2/pi) (z + 0.044715 z^3)
// (0.5 z (1 + tanh u)); one exponential and one reciprocal
constexpr float kGeluK1 = -2.302208198144325f;    // -2 log2(e) sqrt(2/pi)
constexpr float kGeluK2 = -0.1029432395800235f;   // kGeluK1 * 0.044715
__device__ __forceinline__ float gelu_sigma(float z, float z2)
{
    // exp(-2u) = 2^(z (K1 + K2 z^2)): the factor -2 log2(e) folded into the constants
    const float a = z * __builtin_fmaf(z2, kGeluK2, kGeluK1);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a));   // (1 + tanh u) / 2
}
__device__ __forceinline__ float gelu(float z) { return z * gelu_sigma(z, z * z); }
__device__ __forceinline__ float gelu_grad(float z)
{
    const float z2 = z * z;
    const float s = gelu_sigma(z, z2);
    const float du = 0.7978845608028654f + 0.1070322244089003f * z2;
    return s + 2.0f * z * s * (1.0f - s) * du;
}

constexpr int TM = 64, TN = 64, TK = 32, KPAD = 8;

// One 64 x 32 operand tile into LDS as T[i][kk] (i: row of A or column of B, kk
// the k offset), from P(i, k) = P[i * si + k * sk], zeros outside i < ni,
// k < ke.  An operand contiguous in k or in i is read eight elements (16
// bytes) per thread: a run inside the bounds and 16-byte aligned by one
// vector load, else element by element.  Any other layout: one element per load.
__device__ __forceinline__ void stage_tile(uint16_t (*T)[TK + KPAD], const uint16_t* __restrict__ P, long si, long sk,
                                           int i0, int ni, int k0, int ke, int tid)
{
    if (sk == 1) {
        // thread: row tid / 4, k run 8 (tid % 4)
        const int r = tid >> 2, kk = (tid & 3) * 8;
        const int i = i0 + r, k = k0 + kk;
        const uint16_t* src = P + (long)i * si + k;
        uint4 v = {0u, 0u, 0u, 0u};
        if (i < ni && k + 7 < ke && ((uintptr_t)src & 15) == 0) {
            v = *reinterpret_cast<const uint4*>(src);
        } else if (i < ni) {
            uint16_t e[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) e[u] = k + u < ke ? src[u] : (uint16_t)0;
            v = uint4{e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16), e[4] | ((uint32_t)e[5] << 16),
                      e[6] | ((uint32_t)e[7] << 16)};
        }
        *reinterpret_cast<uint4*>(&T[r][kk]) = v;
    } else if (si == 1) {
        // thread: k offset tid / 8, rows 8 (tid % 8) .. + 7
        const int kk = tid >> 3, r0 = (tid & 7) * 8;
        const int i = i0 + r0, k = k0 + kk;
        const uint16_t* src = P + (long)k * sk + i;
        uint16_t e[8];
        if (k < ke && i + 7 < ni && ((uintptr_t)src & 15) == 0) {
            const uint4 v = *reinterpret_cast<const uint4*>(src);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                e[2 * u] = (uint16_t)w[u];
                e[2 * u + 1] = (uint16_t)(w[u] >> 16);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) e[u] = (k < ke && i + u < ni) ? src[u] : (uint16_t)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) T[r0 + u][kk] = e[u];
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + e * 256;
            const int r = idx >> 5, kk = idx & 31;
            const int i = i0 + r, k = k0 + kk;
            T[r][kk] = (i < ni && k < ke) ? P[(long)i * si + (long)k * sk] : (uint16_t)0;
        }
    }
}

// C(m, n) = epi(sum_k A(m, k) B(k, n));  A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn].
// Tile 64 x 64 per block of 4 waves (each 32 x 32 = 2 x 2 MFMA blocks); K in steps of 32.
// gridDim.z > 1 splits K; the partial sums are added atomically (EPI_ACC only).
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t* __restrict__ A, long sam, long sak,
                                              const uint16_t* __restrict__ B, long sbk, long sbn, float* C, long ldc,
                                              const float* __restrict__ bias, uint16_t* Cbf, const float* Zaux,
                                              int kchunk, const int* Mdev)
{
    if (Mdev) M = *Mdev;
    if ((int)blockIdx.y * TM >= M) return;
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][TK + KPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][TK + KPAD];   // stored [n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kb; k0 < ke; k0 += TK) {
        // stage A (64 x 32) and B (32 x 64, stored [n][k]): 8 elements per thread each
        stage_tile(As, A, sam, sak, m0, M, k0, ke, tid);
        stage_tile(Bs, B, sbn, sbk, n0, N, k0, ke, tid);
        __syncthreads();
        const int row = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm + i * 16 + row][kq]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn + j * 16 + row][kq]);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // epilogue: lane holds rows 4 * (lane / 16) + v, column lane % 16 of each 16 x 16 block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int m = m0 + wm + i * 16 + (lane >> 4) * 4 + v;
                int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= M || n >= N) continue;
                float s = acc[i][j][v];
                long o = (long)m * ldc + n;
                if constexpr (EPI == kEpiAcc) {
                    if (gridDim.z > 1)
                        atomicAdd(&C[o], s);
                    else
                        C[o] = s;
                } else if constexpr (EPI == kEpiBias) {
                    C[o] = s + bias[n];
                } else if constexpr (EPI == kEpiBiasGelu) {
                    float z = s + bias[n];
                    C[o] = z;                  // pre-activation, kept for the backward pass
                    Cbf[o] = to_bf16(gelu(z));
                } else if constexpr (EPI == kEpiGeluBwd) {
                    float d = s * gelu_grad(Zaux[o]);
                    C[o] = d;
                    Cbf[o] = to_bf16(d);
                }
            }
}

// Masked loss: BCE-with-logits on the basis indicators and squared error on the
// fractions, averaged over rows.  dY (BF16) = d loss / d Y.
__global__ __launch_bounds__(256) void k_loss(int rows, const float* __restrict__ Y, const float* __restrict__ T,
                                              const uint16_t* __restrict__ X, float wf, uint16_t* dY, float* dYf,
                                              double* loss)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (idx < rows * kMlpSlots) {
        int r = idx / kMlpSlots, s = idx % kMlpSlots;
        float mask = from_bf16(X[(long)r * kMlpIn + 2 * kMlpSlots + s]);
        float z = Y[(long)r * kMlpOut + s], y = T[(long)r * kMlpOut + s];
        float p = Y[(long)r * kMlpOut + kMlpSlots + s], f = T[(long)r * kMlpOut + kMlpSlots + s];
        float inv = 1.0f / (float)rows;
        float sp = fmaxf(z, 0.0f) + log1pf(__expf(-fabsf(z)));   // softplus
        float sig = 1.0f / (1.0f + __expf(-z));
        l = mask * ((sp - y * z) + wf * (p - f) * (p - f)) * inv;
        float gz = mask * (sig - y) * inv;
        float gp = mask * wf * 2.0f * (p - f) * inv;
        dY[(long)r * kMlpOut + s] = to_bf16(gz);
        dY[(long)r * kMlpOut + kMlpSlots + s] = to_bf16(gp);
        if (dYf) {
            dYf[(long)r * kMlpOut + s] = gz;
            dYf[(long)r * kMlpOut + kMlpSlots + s] = gp;
        }
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, VRM_WAVE);
    if (lane_id() == 0 && l != 0.0) atomicAdd(loss, l);
}

// column sums of G[rows][n] (bias gradients), accumulated atomically
__global__ __launch_bounds__(256) void k_colsum(int rows, int n, const float* __restrict__ G, float* out)
{
    int c = threadIdx.x % n;
    int lanes_per_col = blockDim.x / n;
    int part = threadIdx.x / n;
    float s = 0.0f;
    for (int r = blockIdx.x * lanes_per_col + part; r < rows; r += gridDim.x * lanes_per_col) s += G[(long)r * n + c];
    atomicAdd(&out[c], s);
}

__global__ __launch_bounds__(256) void k_adamw(int n, float* w, const float* g, float* m, float* v, float lr, float b1,
                                               float b2, float eps, float wd, float c1, float c2, uint16_t* wbf)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / c1, vh = vi / c2;
    float wi = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
    w[i] = wi;
    wbf[i] = to_bf16(wi);
}

__global__ __launch_bounds__(256) void k_to_bf16(int n, const float* __restrict__ in, uint16_t* out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = to_bf16(in[i]);
}

__global__ void k_zero_f(int n, float* p)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

int nblk(long n) { return (int)((n + 255) / 256); }

// BF16 weights transposed to [n][k] (the B-operand layout of the fused kernel)
constexpr int kOffT1 = 0, kOffT2 = kMlpIn * kMlpHid, kOffT3 = kOffT2 + kMlpHid * kMlpHid;
constexpr int kWtSize = kOffT3 + kMlpHid * kMlpOut;

__global__ __launch_bounds__(256) void k_transpose_w(const uint16_t* __restrict__ wbf, uint16_t* wt)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kMlpIn * kMlpHid) {
        int k = e / kMlpHid, n = e % kMlpHid;
        wt[kOffT1 + n * kMlpIn + k] = wbf[kOffW1 + e];
        wt[kOffT2 + n * kMlpHid + k] = wbf[kOffW2 + e];
    }
    if (e < kMlpHid * kMlpOut) {
        int k = e / kMlpOut, n = e % kMlpOut;
        wt[kOffT3 + n * kMlpHid + k] = wbf[kOffW3 + e];
    }
}

// Fused inference: each block runs all three layers on tiles of 64 rows; the
// activations stay in LDS and the (L2-resident) transposed weights are read
// from memory as MFMA B operands.  Persistent: blocks loop over tiles; the row
// count may be read on the device.  The inference kernels ask for three waves per SIMD
// (at most 168 VGPRs, no spills): one more wave than the default allocation
// gives hides more of the epilogue's and the loads' latency.
constexpr int FR = 64;               // rows per tile
constexpr int FKP = kMlpHid + 8;     // padded LDS row (bank spread)

// The two hidden layers on the tile in Ta: Ta -> Tb -> Ta (GELU, BF16).
// Wave wv computes all 64 rows x columns [32 wv, 32 wv + 32).
__device__ __forceinline__ void mlp_hidden(uint16_t* Ta, uint16_t* Tb, const uint16_t* __restrict__ wt,
                                           const float* __restrict__ w, int tid)
{
    const int lane = tid & 63, wv = tid >> 6;
    const int row = lane & 15, kq = (lane >> 4) * 8;
    for (int layer = 0; layer < 2; ++layer) {
        const uint16_t* A = layer == 0 ? Ta : Tb;
        uint16_t* O = layer == 0 ? Tb : Ta;
        const uint16_t* Wt = wt + (layer == 0 ? kOffT1 : kOffT2);
        const float* bias = w + (layer == 0 ? kOffB1 : kOffB2);
        f32x4 acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k0 = 0; k0 < kMlpHid; k0 += 32) {
            bf16x8 b[2];
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&Wt[(wv * 32 + j * 16 + row) * kMlpHid + k0 + kq]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bf16x8 a = *reinterpret_cast<const bf16x8*>(&A[(i * 16 + row) * FKP + k0 + kq]);
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int m = i * 16 + (lane >> 4) * 4 + v;
                    int n = wv * 32 + j * 16 + (lane & 15);
                    O[m * FKP + n] = to_bf16(gelu(acc[i][j][v] + bias[n]));
                }
        __syncthreads();
    }
}

// Output columns [n0, n0 + 16) of the last layer for the 64 rows of the tile
// in Ta: lane holds rows i * 16 + 4 (lane / 16) + v, column n0 + lane % 16.
__device__ __forceinline__ void mlp_out16(const uint16_t* Ta, const uint16_t* __restrict__ wt, int n0, int lane,
                                          f32x4 (&acc)[4])
{
    const int row = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < kMlpHid; k0 += 32) {
        bf16x8 b = *reinterpret_cast<const bf16x8*>(&wt[kOffT3 + (n0 + row) * kMlpHid + k0 + kq]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bf16x8 a = *reinterpret_cast<const bf16x8*>(&Ta[(i * 16 + row) * FKP + k0 + kq]);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_infer(int rows, const int* rows_dev, const uint16_t* __restrict__ X,
                                                   const uint16_t* __restrict__ wt, const float* __restrict__ w,
                                                   float* __restrict__ Y)
{
    __shared__ __attribute__((aligned(16))) uint16_t Ta[FR * FKP];
    __shared__ __attribute__((aligned(16))) uint16_t Tb[FR * FKP];
    if (rows_dev) rows = *rows_dev;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int r0 = blockIdx.x * FR; r0 < rows; r0 += gridDim.x * FR) {
        for (int e = tid; e < FR * kMlpIn / 8; e += 256) {
            int r = e / (kMlpIn / 8), c8 = (e % (kMlpIn / 8)) * 8;
            uint4 v = {0u, 0u, 0u, 0u};
            if (r0 + r < rows) v = *reinterpret_cast<const uint4*>(&X[(long)(r0 + r) * kMlpIn + c8]);
            *reinterpret_cast<uint4*>(&Ta[r * FKP + c8]) = v;
        }
        __syncthreads();
        mlp_hidden(Ta, Tb, wt, w, tid);
        // output layer: wave wv computes columns [16 wv, 16 wv + 16)
        f32x4 acc[4];
        mlp_out16(Ta, wt, wv * 16, lane, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int m = r0 + i * 16 + (lane >> 4) * 4 + v;
                int n = wv * 16 + (lane & 15);
                if (m < rows) Y[(long)m * kMlpOut + n] = acc[i][v] + w[kOffB3 + n];
            }
        __syncthreads();
    }
}

// Inference for the queued small-neighbourhood LPs, with the network input
// built in LDS from their column records (slot s = segment s: exact offset /
// h and mask; q - 2), and only the logits of the eight columns written:
// L[item][8].
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_infer_small(const int* rows_dev, SmallRec rec, float sc, int q,
                                                         const uint16_t* __restrict__ wt, const float* __restrict__ w,
                                                         float* __restrict__ L)
{
    __shared__ __attribute__((aligned(16))) uint16_t Ta[FR * FKP];
    __shared__ __attribute__((aligned(16))) uint16_t Tb[FR * FKP];
    const int rows = *rows_dev;
    const size_t cap = (size_t)rec.cap;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int r0 = blockIdx.x * FR; r0 < rows; r0 += gridDim.x * FR) {
        for (int e = tid; e < FR * kMlpIn / 8; e += 256) {
            int r = e / (kMlpIn / 8), c8 = (e % (kMlpIn / 8)) * 8;
            *reinterpret_cast<uint4*>(&Ta[r * FKP + c8]) = uint4{0u, 0u, 0u, 0u};
        }
        __syncthreads();
        for (int e = tid; e < FR * VRM_NSEG; e += 256) {
            // consecutive threads take consecutive rows of one segment plane
            const int s = e / FR, r = e % FR;
            const int item = r0 + r;
            if (item < rows) {
                if (rec.pj[s * cap + item] >= 0) {
                    Ta[r * FKP + 2 * s] = to_bf16(rec.off[(4 * s + 0) * cap + item] * sc);
                    Ta[r * FKP + 2 * s + 1] = to_bf16(rec.off[(4 * s + 2) * cap + item] * sc);
                    Ta[r * FKP + 2 * kMlpSlots + s] = 0x3f80;   // 1.0
                }
                if (s == 0) Ta[r * FKP + 3 * kMlpSlots] = q == 3 ? 0x3f80 : 0;
            }
        }
        __syncthreads();
        mlp_hidden(Ta, Tb, wt, w, tid);
        if (wv == 0) {
            f32x4 acc[4];
            mlp_out16(Ta, wt, 0, lane, acc);
            const int n = lane & 15;
            if (n < VRM_NSEG) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int m = r0 + i * 16 + (lane >> 4) * 4 + v;
                        if (m < rows) L[(long)m * VRM_NSEG + n] = acc[i][v] + w[kOffB3 + n];
                    }
            }
        }
        __syncthreads();
    }
}

// Inference for the queued complete LPs from their column records: the input
// row is built in LDS from the record (slot j < 32 of the nearest-first list:
// offset / h and mask; q - 2), four threads per row, and only the 32 basis
// logits are computed and written: L[item][kMlpSlots].  (Choosing the m
// largest here, at this kernel's occupancy, costs more than a separate pass.)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_infer_full(const int* rows_dev, FullRec fr,
                                                        const uint16_t* __restrict__ wt, const float* __restrict__ w,
                                                        float* __restrict__ Lout)
{
    __shared__ __attribute__((aligned(16))) uint16_t Ta[FR * FKP];
    __shared__ __attribute__((aligned(16))) uint16_t Tb[FR * FKP];
    constexpr int LS = kMlpSlots + 1;   // row stride of the logits (staged in Tb)
    static_assert(FR * LS * sizeof(float) <= sizeof(Tb), "the logits fit in the second tile");
    const int rows = *rows_dev;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rr = tid >> 2, part = tid & 3;   // this thread's row of the tile, its quarter of the slots
    for (int r0 = blockIdx.x * FR; r0 < rows; r0 += gridDim.x * FR) {
        const int r = r0 + rr;
        const int k = r < rows ? fr.kcol[r] : -1;
        {
            float xi = 0.0f, yi = 0.0f;
            if (k > 0) {
                const int t = fr.q_full[r];
                xi = fr.xs[t];
                yi = fr.ys[t];
            }
            const int32_t* rrow = fr.rec + (size_t)r * fr.row;
            uint32_t off[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int j = 8 * part + i;
                uint32_t pr = 0;
                if (j < k) {
                    const int u = (int)((unsigned)rrow[j] >> 6);
                    pr = (uint32_t)to_bf16(((fr.xs[u] - xi) * fr.scale2e) * fr.sc) |
                         ((uint32_t)to_bf16(((fr.ys[u] - yi) * fr.scale2e) * fr.sc) << 16);
                }
                off[i] = pr;
            }
            uint16_t* row = Ta + rr * FKP;
            // elements 16 part .. 16 part + 15: the offset pairs of slots 8 part .. 8 part + 7
            *reinterpret_cast<uint4*>(row + 16 * part) = uint4{off[0], off[1], off[2], off[3]};
            *reinterpret_cast<uint4*>(row + 16 * part + 8) = uint4{off[4], off[5], off[6], off[7]};
            // their masks, then q - 2 (element 3 kMlpSlots) and zero padding
            uint32_t mk[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 8 * part + 2 * i;
                mk[i] = (j < k ? 0x3f80u : 0u) | ((j + 1 < k ? 0x3f80u : 0u) << 16);
            }
            *reinterpret_cast<uint4*>(row + 2 * kMlpSlots + 8 * part) = uint4{mk[0], mk[1], mk[2], mk[3]};
            *reinterpret_cast<uint4*>(row + 3 * kMlpSlots + 8 * part) =
                uint4{part == 0 && fr.q == 3 ? 0x3f80u : 0u, 0u, 0u, 0u};
        }
        __syncthreads();
        mlp_hidden(Ta, Tb, wt, w, tid);
        // the logits: waves 0 and 1 compute columns [16 wv, 16 wv + 16) of the 64 rows
        float* L = reinterpret_cast<float*>(Tb);
        if (wv < 2) {
            f32x4 acc[4];
            mlp_out16(Ta, wt, wv * 16, lane, acc);
            const int n = wv * 16 + (lane & 15);
            const float b = w[kOffB3 + n];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) L[(i * 16 + (lane >> 4) * 4 + v) * LS + n] = acc[i][v] + b;
        }
        __syncthreads();
        if (r < rows) {
            float4* dst = reinterpret_cast<float4*>(Lout + (size_t)r * kMlpSlots + 8 * part);
            // LS is odd: the row start is not 16-byte aligned in LDS, so the values are read one by one
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = L[rr * LS + 8 * part + i];
            dst[0] = float4{v[0], v[1], v[2], v[3]};
            dst[1] = float4{v[4], v[5], v[6], v[7]};
        }
        __syncthreads();
    }
}

template <int EPI>
int gemm(hipStream_t s, int M, int N, int K, const uint16_t* A, long sam, long sak, const uint16_t* B, long sbk,
         long sbn, float* C, long ldc, const float* bias, uint16_t* Cbf, const float* Zaux, int splitk,
         const int* Mdev = nullptr)
{
    if (M <= 0) return VRM_OK;
    int kchunk = K;
    if (splitk > 1) kchunk = ((K + splitk - 1) / splitk + TK - 1) / TK * TK;
    int gz = (K + kchunk - 1) / kchunk;
    dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, gz);
    hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, Cbf, Zaux,
                       kchunk, Mdev);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

}  // namespace

// ----------------------------------------------------------------- host
int vrm_mlp_read_weights(vrm_ctx* c, float* w_dev)
{
    VRM_HIP(hipMemcpyAsync(w_dev, c->mlp->w, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, c->stream));
    return VRM_OK;
}

int vrm_mlp_alloc(vrm_ctx* c, int max_rows)
{
    if (c->mlp && c->mlp->max_rows >= max_rows) return VRM_OK;
    MlpState* m = c->mlp;
    void* p;
#define AL(field, bytes)                            \
    VRM_HIP(hipMalloc(&p, (bytes) + 64));           \
    m->field = reinterpret_cast<decltype(m->field)>(p);
    if (!m) {
        m = new MlpState();
        std::memset(m, 0, sizeof(*m));
        AL(w, sizeof(float) * kMlpParams);
        AL(g, sizeof(float) * kMlpParams);
        AL(am, sizeof(float) * kMlpParams);
        AL(av, sizeof(float) * kMlpParams);
        AL(wbf, sizeof(uint16_t) * kMlpParams);
        AL(wt, sizeof(uint16_t) * kWtSize);
        AL(loss, sizeof(double) * 2);
        VRM_HIP(hipMemsetAsync(m->w, 0, sizeof(float) * kMlpParams, c->stream));
        VRM_HIP(hipMemsetAsync(m->wbf, 0, sizeof(uint16_t) * kMlpParams, c->stream));
        VRM_HIP(hipMemsetAsync(m->am, 0, sizeof(float) * kMlpParams, c->stream));
        VRM_HIP(hipMemsetAsync(m->av, 0, sizeof(float) * kMlpParams, c->stream));
        c->mlp = m;
    }
    if (max_rows > m->max_rows) {
        void* old[] = {m->z1, m->z2, m->h1, m->h2, m->y, m->dy, m->dyf, m->dz, m->dzb, m->dzb2};
        VRM_HIP(hipStreamSynchronize(c->stream));
        for (void* q : old)
            if (q) (void)hipFree(q);
        size_t R = (size_t)max_rows;
        AL(z1, sizeof(float) * R * kMlpHid);
        AL(z2, sizeof(float) * R * kMlpHid);
        AL(h1, sizeof(uint16_t) * R * kMlpHid);
        AL(h2, sizeof(uint16_t) * R * kMlpHid);
        AL(y, sizeof(float) * R * kMlpOut);
        AL(dy, sizeof(uint16_t) * R * kMlpOut);
        AL(dyf, sizeof(float) * R * kMlpOut);
        AL(dz, sizeof(float) * R * kMlpHid);
        AL(dzb, sizeof(uint16_t) * R * kMlpHid);
        AL(dzb2, sizeof(uint16_t) * R * kMlpHid);
        m->max_rows = max_rows;
    }
#undef AL
    return VRM_OK;
}

void vrm_mlp_free(vrm_ctx* c)
{
    if (!c->mlp) return;
    MlpState* m = c->mlp;
    void* ptrs[] = {m->w, m->g, m->am, m->av, m->wbf, m->wt, m->z1, m->z2, m->h1, m->h2, m->y, m->dy, m->dyf, m->dz, m->dzb,
                    m->dzb2, m->loss};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
    c->mlp = nullptr;
}

int vrm_mlp_set_weights(vrm_ctx* c, const float* w_dev)
{
    MlpState* m = c->mlp;
    VRM_HIP(hipMemcpyAsync(m->w, w_dev, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(kMlpParams)), dim3(256), 0, c->stream, kMlpParams, m->w, m->wbf);
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk(kMlpIn * kMlpHid)), dim3(256), 0, c->stream, m->wbf, m->wt);
    VRM_HIP(hipGetLastError());
    VRM_HIP(hipMemsetAsync(m->am, 0, sizeof(float) * kMlpParams, c->stream));
    VRM_HIP(hipMemsetAsync(m->av, 0, sizeof(float) * kMlpParams, c->stream));
    m->step = 0;
    m->loaded = 1;
    return VRM_OK;
}

// forward pass over `rows` feature rows X (BF16); Y (FP32, rows x 64).  With
// rows_dev the row count is read on the device (rows is then an upper bound).
int vrm_mlp_forward(vrm_ctx* c, const uint16_t* X, int rows, float* Y, const int* rows_dev)
{
    MlpState* m = c->mlp;
    hipStream_t s = c->stream;
    const uint16_t* W1 = m->wbf + kOffW1;
    const uint16_t* W2 = m->wbf + kOffW2;
    const uint16_t* W3 = m->wbf + kOffW3;
    int r = gemm<kEpiBiasGelu>(s, rows, kMlpHid, kMlpIn, X, kMlpIn, 1, W1, kMlpHid, 1, m->z1, kMlpHid, m->w + kOffB1,
                               m->h1, nullptr, 1, rows_dev);
    if (!r)
        r = gemm<kEpiBiasGelu>(s, rows, kMlpHid, kMlpHid, m->h1, kMlpHid, 1, W2, kMlpHid, 1, m->z2, kMlpHid,
                               m->w + kOffB2, m->h2, nullptr, 1, rows_dev);
    if (!r)
        r = gemm<kEpiBias>(s, rows, kMlpOut, kMlpHid, m->h2, kMlpHid, 1, W3, kMlpOut, 1, Y, kMlpOut, m->w + kOffB3,
                           nullptr, nullptr, 1, rows_dev);
    return r;
}

// fused forward for inference (no intermediate buffers); rows may be an upper bound with rows_dev
int vrm_mlp_infer_small_run(vrm_ctx* c, int rows, const int* rows_dev, const SmallRec& rec, float sc, int q, float* L)
{
    if (rows <= 0) return VRM_OK;
    MlpState* m = c->mlp;
    int tiles = (rows + FR - 1) / FR;
    int grid = tiles < c->tuning.infer_blocks ? tiles : c->tuning.infer_blocks;
    hipLaunchKernelGGL(k_mlp_infer_small, dim3(grid), dim3(256), 0, c->stream, rows_dev, rec, sc, q, m->wt, m->w, L);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_mlp_infer_full_run(vrm_ctx* c, int rows, const int* rows_dev, const FullRec& fr, float* L)
{
    if (rows <= 0) return VRM_OK;
    MlpState* m = c->mlp;
    int tiles = (rows + FR - 1) / FR;
    int grid = tiles < c->tuning.infer_blocks ? tiles : c->tuning.infer_blocks;
    hipLaunchKernelGGL(k_mlp_infer_full, dim3(grid), dim3(256), 0, c->stream, rows_dev, fr, m->wt, m->w, L);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

int vrm_mlp_infer_run(vrm_ctx* c, const uint16_t* X, int rows, float* Y, const int* rows_dev)
{
    if (rows <= 0) return VRM_OK;
    MlpState* m = c->mlp;
    int tiles = (rows + FR - 1) / FR;
    int grid = tiles < c->tuning.infer_blocks ? tiles : c->tuning.infer_blocks;
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), 0, c->stream, rows, rows_dev, X, m->wt, m->w, Y);
    VRM_HIP(hipGetLastError());
    return VRM_OK;
}

// one AdamW step on the masked BCE + MSE loss of a batch (X, T)
int vrm_mlp_train(vrm_ctx* c, const uint16_t* X, const float* T, int rows, float lr, float wd, float wf,
                  double* loss_out, float* grad_out)
{
    MlpState* m = c->mlp;
    hipStream_t s = c->stream;
    int r = vrm_mlp_forward(c, X, rows, m->y, nullptr);
    if (r) return r;
    VRM_HIP(hipMemsetAsync(m->loss, 0, sizeof(double), s));
    VRM_HIP(hipMemsetAsync(m->g, 0, sizeof(float) * kMlpParams, s));
    hipLaunchKernelGGL(k_loss, dim3(nblk((long)rows * kMlpSlots)), dim3(256), 0, s, rows, m->y, T, X, wf, m->dy, m->dyf,
                       m->loss);
    VRM_HIP(hipGetLastError());
    const uint16_t* W2 = m->wbf + kOffW2;
    const uint16_t* W3 = m->wbf + kOffW3;
    int split = rows >= 4096 ? 16 : 1;
    // layer 3: dW3 = H2^T dY, db3 = colsum dY, dZ2 = (dY W3^T) * gelu'(Z2)
    r = gemm<kEpiAcc>(s, kMlpHid, kMlpOut, rows, m->h2, 1, kMlpHid, m->dy, kMlpOut, 1, m->g + kOffW3, kMlpOut, nullptr,
                      nullptr, nullptr, split);
    if (r) return r;
    hipLaunchKernelGGL(k_colsum, dim3(64), dim3(256), 0, s, rows, kMlpOut, m->dyf, m->g + kOffB3);
    r = gemm<kEpiGeluBwd>(s, rows, kMlpHid, kMlpOut, m->dy, kMlpOut, 1, W3, 1, kMlpOut, m->dz, kMlpHid, nullptr, m->dzb,
                          m->z2, 1);
    if (r) return r;
    // layer 2
    r = gemm<kEpiAcc>(s, kMlpHid, kMlpHid, rows, m->h1, 1, kMlpHid, m->dzb, kMlpHid, 1, m->g + kOffW2, kMlpHid, nullptr,
                      nullptr, nullptr, split);
    if (r) return r;
    hipLaunchKernelGGL(k_colsum, dim3(64), dim3(256), 0, s, rows, kMlpHid, m->dz, m->g + kOffB2);
    r = gemm<kEpiGeluBwd>(s, rows, kMlpHid, kMlpHid, m->dzb, kMlpHid, 1, W2, 1, kMlpHid, m->dz, kMlpHid, nullptr,
                          m->dzb2, m->z1, 1);
    if (r) return r;
    // layer 1
    r = gemm<kEpiAcc>(s, kMlpIn, kMlpHid, rows, X, 1, kMlpIn, m->dzb2, kMlpHid, 1, m->g + kOffW1, kMlpHid, nullptr,
                      nullptr, nullptr, split);
    if (r) return r;
    hipLaunchKernelGGL(k_colsum, dim3(64), dim3(256), 0, s, rows, kMlpHid, m->dz, m->g + kOffB1);
    VRM_HIP(hipGetLastError());
    if (grad_out) VRM_HIP(hipMemcpyAsync(grad_out, m->g, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, s));
    if (loss_out) VRM_HIP(hipMemcpyAsync(loss_out, m->loss, sizeof(double), hipMemcpyDeviceToDevice, s));
    if (lr > 0.0f) {
        m->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        float c1 = 1.0f - powf(b1, (float)m->step), c2 = 1.0f - powf(b2, (float)m->step);
        hipLaunchKernelGGL(k_adamw, dim3(nblk(kMlpParams)), dim3(256), 0, s, kMlpParams, m->w, m->g, m->am, m->av, lr, b1,
                           b2, 1e-8f, wd, c1, c2, m->wbf);
        hipLaunchKernelGGL(k_transpose_w, dim3(nblk(kMlpIn * kMlpHid)), dim3(256), 0, s, m->wbf, m->wt);
        VRM_HIP(hipGetLastError());
    }
    return VRM_OK;
}

// plain product for tests: C (FP32, M x N) = A (BF16, M x K, row-major) * B (BF16, K x N, row-major)
int vrm_gemm_test(vrm_ctx* c, const uint16_t* A, const uint16_t* B, float* C, int M, int N, int K, int transA,
                  int transB)
{
    long sam = transA ? 1 : K, sak = transA ? M : 1;
    long sbk = transB ? 1 : N, sbn = transB ? K : 1;
    return gemm<kEpiAcc>(c->stream, M, N, K, A, sam, sak, B, sbk, sbn, C, N, nullptr, nullptr, nullptr,
                         K >= 1024 ? 8 : 1);
}
