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
