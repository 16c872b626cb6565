// device.h -- small device helpers shared by the libmd kernels (gfx950, wave64).
//
// Reciprocal and reciprocal square root: the hardware approximations
// (v_rcp_f32/v_rsq_f32 are accurate to about 1 ulp of FP32; the FP64 forms are
// only a seed) refined by Newton's iteration where FP64 accuracy is needed.
// Reductions: fixed butterfly orders inside a wavefront and a fixed serial order
// across the wavefronts of a block, so every sum is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md_internal.h"

namespace md {

__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq32(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/x in FP64: hardware seed, then two Newton steps y <- y + y (1 - x y).
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}

// 1/sqrt(x) in FP64: hardware seed, then two Newton steps y <- y (3/2 - x y^2 / 2).
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = __builtin_fma(-h * y, y, 0.5);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-h * y, y, 0.5);
    return __builtin_fma(y, e, y);
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

}  // namespace md
