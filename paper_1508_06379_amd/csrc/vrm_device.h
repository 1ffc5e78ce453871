// Device helpers shared by the HIP kernels of libvrm (gfx950, wave64).
//
// Decision arithmetic (annulus membership, segment, insertion positions and
// conflicts) is FP32 with a fixed operation order.  The library is compiled
// with -ffp-contract=off so that x*x + y*y is two roundings, never an FMA;
// FMAs are written explicitly where they are wanted.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define VRM_NSEG 8
#define VRM_KMAX 48
#define VRM_WAVE 64

namespace vrm {

// ------------------------------------------------------------- decisions
// tan(22.5 deg) rounded to FP32: segment boundaries sit at 22.5 + s * 45 deg.
__device__ __forceinline__ float tan_pi8() { return 0.41421356237309503f; }

__device__ __forceinline__ float d2_f32(float dx, float dy)
{
    float a = dx * dx;
    float b = dy * dy;
    return a + b;
}

// Eight 45-degree segments centred on s * 45 deg, counter-clockwise from +x:
// near the x axis iff |dy| < t |dx|, near the y axis iff |dx| < t |dy|.
__device__ __forceinline__ int segment_f32(float dx, float dy)
{
    float ax = fabsf(dx), ay = fabsf(dy);
    float tx = tan_pi8() * ax, ty = tan_pi8() * ay;
    if (ay < tx) return dx > 0.0f ? 0 : 4;
    if (ax < ty) return dy > 0.0f ? 2 : 6;
    if (dx > 0.0f) return dy > 0.0f ? 1 : 7;
    return dy > 0.0f ? 3 : 5;
}

// Insertion candidate on the centre line of segment s at radius rad = fl32(1.5 h).
__device__ __forceinline__ void candidate_f32(float xi, float yi, float rad, int s, float& xc, float& yc)
{
    const float c45 = 0.70710678118654752f;
    float cs = (s == 0) ? 1.0f : (s == 4) ? -1.0f : (s == 2 || s == 6) ? 0.0f : (s == 1 || s == 7) ? c45 : -c45;
    float sn = (s == 2) ? 1.0f : (s == 6) ? -1.0f : (s == 0 || s == 4) ? 0.0f : (s == 1 || s == 3) ? c45 : -c45;
    float ox = rad * cs;
    float oy = rad * sn;
    xc = xi + ox;
    yc = yi + oy;
}

// Monotone map of a float to uint32 (total order of finite values).
__device__ __forceinline__ uint32_t ordered_key(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ordered_key_inv(uint32_t k)
{
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

// ------------------------------------------------------- double-float
// Unevaluated sums hi + lo with |lo| <= ulp(hi)/2 (Dekker / Knuth).
struct df {
    float hi, lo;
};

__device__ __forceinline__ df two_sum(float a, float b)
{
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ df fast_two_sum(float a, float b)
{
    float s = a + b;
    float e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ df two_prod(float a, float b)
{
    float p = a * b;
    float e = __builtin_fmaf(a, b, -p);
    return {p, e};
}
__device__ __forceinline__ df df_add(df a, df b)
{
    df s = two_sum(a.hi, b.hi);
    df t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ df df_mul(df a, df b)
{
    df p = two_prod(a.hi, b.hi);
    p.lo = __builtin_fmaf(a.hi, b.lo, p.lo);
    p.lo = __builtin_fmaf(a.lo, b.hi, p.lo);
    return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ df df_mul_f(df a, float b)
{
    df p = two_prod(a.hi, b);
    p.lo = __builtin_fmaf(a.lo, b, p.lo);
    return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ df df_neg(df a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ df df_sqrt(df a)
{
    if (a.hi <= 0.0f) return {0.0f, 0.0f};
    float t = __builtin_sqrtf(a.hi);
    float e = __builtin_fmaf(-t, t, a.hi);
    float c = (e + a.lo) / (2.0f * t);
    return fast_two_sum(t, c);
}

// ------------------------------------------------------------ octets
// An octet is 8 consecutive lanes of a wave cooperating on one LP.
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ float oct_bcast(float v, int src8)
{
    int base = lane_id() & ~7;
    return __shfl(v, base + src8, VRM_WAVE);
}
__device__ __forceinline__ int oct_bcast_i(int v, int src8)
{
    int base = lane_id() & ~7;
    return __shfl(v, base + src8, VRM_WAVE);
}
__device__ __forceinline__ float oct_sum(float v)
{
    v += __shfl_xor(v, 1, VRM_WAVE);
    v += __shfl_xor(v, 2, VRM_WAVE);
    v += __shfl_xor(v, 4, VRM_WAVE);
    return v;
}
__device__ __forceinline__ int oct_min_i(int v)
{
    v = min(v, __shfl_xor(v, 1, VRM_WAVE));
    v = min(v, __shfl_xor(v, 2, VRM_WAVE));
    v = min(v, __shfl_xor(v, 4, VRM_WAVE));
    return v;
}
__device__ __forceinline__ int oct_max_i(int v)
{
    v = max(v, __shfl_xor(v, 1, VRM_WAVE));
    v = max(v, __shfl_xor(v, 2, VRM_WAVE));
    v = max(v, __shfl_xor(v, 4, VRM_WAVE));
    return v;
}
// Exact octet sum of double-floats (error-free tree with renormalisation).
__device__ __forceinline__ df oct_sum_df(df v)
{
    for (int o = 1; o < 8; o <<= 1) {
        df w{__shfl_xor(v.hi, o, VRM_WAVE), __shfl_xor(v.lo, o, VRM_WAVE)};
        v = df_add(v, w);
    }
    return v;
}

}  // namespace vrm
