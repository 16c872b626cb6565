// device.h -- small device helpers shared by the libmd kernels (gfx950, wave64).
//
// Reciprocal and reciprocal square root: the hardware approximations
// (v_rcp_f32/v_rsq_f32 are accurate to about 1 ulp of FP32; the FP64 forms are
// only a seed of about 24 bits) refined to FP64 by a second-order correction.
// Reductions: fixed butterfly orders inside a wavefront and a fixed serial order
// across the wavefronts of a block, so every sum is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md_internal.h"

namespace md {

__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq32(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/x in FP64.  The hardware seed y0 has a relative error e = 1 - x*y0 with
// |e| < 2^-24 (measured on gfx950: 2^-24.4), so 1/x = y0 / (1 - e) = y0 (1 + e + e^2)
// + O(e^3): three FMAs, one rounding of the final result (about 1 ulp).
__device__ __forceinline__ double rcp64(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, __builtin_fma(e, e, e), y);
}

// 1/sqrt(x) in FP64.  With e = 1 - x*y0^2 (|e| < 2^-23), 1/sqrt(x) = y0 (1 - e)^(-1/2)
// = y0 (1 + e/2 + 3e^2/8) + O(e^3).
__device__ __forceinline__ double rsq64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y, y, 1.0);
    return __builtin_fma(y, e * __builtin_fma(e, 0.375, 0.5), y);
}

// sin and cos together (Cody and Waite's argument reduction followed by Taylor
// polynomials).  x = k pi/2 + r with k = rint(x 2/pi); pi/2 is split into a
// double and a correction (pi/2 = P1 + P2 to about 1e-33), and the two FMA steps
// r = (x - k P1) - k P2 leave |r| <= pi/4 with an absolute error near 1e-16 for
// |x| < 2^30.  On |r| <= pi/4 the Taylor series of sin to r^17 and of cos to r^16
// are exact to 1e-19.  The quadrant k mod 4 permutes and negates the pair.
// Larger |x| (never reached by the dynamics here) falls back to the library.
constexpr double kSincosMaxArg = 1073741824.0;  // 2^30: the reduction's range

// sincos64 without the fallback: valid for |x| < kSincosMaxArg, no branch.
__device__ __forceinline__ void sincos64_reduced(double x, double *sp, double *cp)
{
    const double P1 = 1.5707963267948966;      // pi/2 rounded to double
    const double P2 = 6.123233995736766e-17;   // pi/2 - P1
    const double k = __builtin_rint(x * 0.6366197723675814);
    double r = __builtin_fma(-k, P1, x);
    r = __builtin_fma(-k, P2, r);
    const double z = r * r;
    double ps = -1.0 / 355687428096000.0;       // -1/17!
    ps = __builtin_fma(ps, z, 1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, z, -1.0 / 6227020800.0);
    ps = __builtin_fma(ps, z, 1.0 / 39916800.0);
    ps = __builtin_fma(ps, z, -1.0 / 362880.0);
    ps = __builtin_fma(ps, z, 1.0 / 5040.0);
    ps = __builtin_fma(ps, z, -1.0 / 120.0);
    ps = __builtin_fma(ps, z, 1.0 / 6.0);
    double pc = 1.0 / 20922789888000.0;         // 1/16!
    pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);
    pc = __builtin_fma(pc, z, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, z, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, z, 1.0 / 40320.0);
    pc = __builtin_fma(pc, z, -1.0 / 720.0);
    pc = __builtin_fma(pc, z, 1.0 / 24.0);
    pc = __builtin_fma(pc, z, -0.5);
    const double sr = __builtin_fma(-r * z, ps, r);   // r - r^3/6 + ...  (ps holds +1/6 - ...)
    const double cr = __builtin_fma(z, pc, 1.0);
    const int q = (int)k;
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    *sp = (q & 2) ? -a : a;
    *cp = ((q + 1) & 2) ? -b : b;
}

__device__ __forceinline__ void sincos64(double x, double *sp, double *cp)
{
    if (!(fabs(x) < kSincosMaxArg)) {
        sincos(x, sp, cp);
        return;
    }
    sincos64_reduced(x, sp, cp);
}

// FP32 counterpart (the FP32-state HMF path keeps |x| <= pi): Taylor to r^11 / r^12.
__device__ __forceinline__ void sincos32(float x, float *sp, float *cp)
{
    const float P1 = 1.57079637f;        // pi/2 rounded to float
    const float P2 = -4.37113883e-8f;    // pi/2 - P1
    const float k = __builtin_rintf(x * 0.636619772f);
    float r = __builtin_fmaf(-k, P1, x);
    r = __builtin_fmaf(-k, P2, r);
    const float z = r * r;
    float ps = -1.0f / 39916800.0f;
    ps = __builtin_fmaf(ps, z, 1.0f / 362880.0f);
    ps = __builtin_fmaf(ps, z, -1.0f / 5040.0f);
    ps = __builtin_fmaf(ps, z, 1.0f / 120.0f);
    ps = __builtin_fmaf(ps, z, -1.0f / 6.0f);
    float pc = 1.0f / 479001600.0f;
    pc = __builtin_fmaf(pc, z, -1.0f / 3628800.0f);
    pc = __builtin_fmaf(pc, z, 1.0f / 40320.0f);
    pc = __builtin_fmaf(pc, z, -1.0f / 720.0f);
    pc = __builtin_fmaf(pc, z, 1.0f / 24.0f);
    pc = __builtin_fmaf(pc, z, -0.5f);
    const float sr = __builtin_fmaf(r * z, ps, r);
    const float cr = __builtin_fmaf(z, pc, 1.0f);
    const int q = (int)k;
    const float a = (q & 1) ? cr : sr;
    const float b = (q & 1) ? sr : cr;
    *sp = (q & 2) ? -a : a;
    *cp = ((q + 1) & 2) ? -b : b;
}

// Sum over the 64 lanes of a wavefront (xor butterfly; every lane gets the total).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// Sum over a block of up to 1024 threads (blockDim.x a multiple of 64).  `lds` must
// hold blockDim.x/64 doubles.  The result is valid in thread 0 only.  Contains a
// __syncthreads(): every thread of the block must call it.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x / kWave;
        for (int w = 0; w < nw; ++w) t += lds[w];
    }
    return t;
}

// The fixed order in which every launch form adds the S partials (slots) of a
// particle, b = 0 .. S-1: blocks of kSlotBlock = 8 consecutive slots, each added as
// a balanced tree, ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)); the block
// sums added in order of the block, starting from 0; then the S mod 8 slots past
// the last block one by one.  All in FP64 (FP32 slots widened first).  The trees
// keep the dependent adds per particle to S / 8 + 3 + S mod 8: the fused stage
// sums up to 128 partials per particle inside one block, where a chain of S
// dependent adds was the longest phase after the pair loop.
constexpr int kSlotBlock = 8;

template <typename V>
__device__ __forceinline__ double tree8(const V (&v)[kSlotBlock])
{
    return (((double)v[0] + (double)v[1]) + ((double)v[2] + (double)v[3])) +
           (((double)v[4] + (double)v[5]) + ((double)v[6] + (double)v[7]));
}

// The sum of part[(b D + d) npad + i] over b in the order above.  The loads go out
// 16 at a time: one load, wait and add per slot leaves the update kernels bound by
// the memory latency (the symmetric 2D form at N = 262,144 adds 256 slots per
// coordinate).
template <int D>
__device__ __forceinline__ double slot_sum(const double *__restrict__ part, int S, int d, int npad, int i)
{
    double s = 0.0;
    int b = 0;
    for (; b + 2 * kSlotBlock <= S; b += 2 * kSlotBlock) {
        double v[2][kSlotBlock];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < kSlotBlock; ++u) v[h][u] = part[(size_t)((b + h * kSlotBlock + u) * D + d) * npad + i];
        s += tree8(v[0]);
        s += tree8(v[1]);
    }
    if (b + kSlotBlock <= S) {
        double v[kSlotBlock];
#pragma unroll
        for (int u = 0; u < kSlotBlock; ++u) v[u] = part[(size_t)((b + u) * D + d) * npad + i];
        s += tree8(v);
        b += kSlotBlock;
    }
    for (; b < S; ++b) s += part[(size_t)(b * D + d) * npad + i];
    return s;
}

// slot_sum for every coordinate d < D at once: the loads of all coordinates go
// out together (16 D in flight).  Slots of FP32 (the symmetric form's MD_MIXED
// slots) or FP64.
template <int D, typename SlotT = double>
__device__ __forceinline__ void slot_sums(const SlotT *__restrict__ part, int S, int npad, int i, double (&s)[D])
{
#pragma unroll
    for (int d = 0; d < D; ++d) s[d] = 0.0;
    int b = 0;
    for (; b + 2 * kSlotBlock <= S; b += 2 * kSlotBlock) {
        SlotT v[D][2][kSlotBlock];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < kSlotBlock; ++u)
#pragma unroll
                for (int d = 0; d < D; ++d)
                    v[d][h][u] = part[(size_t)((b + h * kSlotBlock + u) * D + d) * npad + i];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            s[d] += tree8(v[d][0]);
            s[d] += tree8(v[d][1]);
        }
    }
    if (b + kSlotBlock <= S) {
        SlotT v[D][kSlotBlock];
#pragma unroll
        for (int u = 0; u < kSlotBlock; ++u)
#pragma unroll
            for (int d = 0; d < D; ++d) v[d][u] = part[(size_t)((b + u) * D + d) * npad + i];
#pragma unroll
        for (int d = 0; d < D; ++d) s[d] += tree8(v[d]);
        b += kSlotBlock;
    }
    for (; b < S; ++b)
#pragma unroll
        for (int d = 0; d < D; ++d) s[d] += (double)part[(size_t)(b * D + d) * npad + i];
}

}  // namespace md
