// energy.hip -- diagnostic energies, always FP64 arithmetic and FP64 sums:
// K = (1/2) sum p^2; V of eq. 1 (Ring) and eq. 3 (2D) as the sum over pairs
// i < j; V of the HMF model through the magnetization (eq. 5).  The relative
// energy error |E - E0| / |E0| of Sec. 4 is formed from these on the host.
//
// Every sum is a per-thread FP64 partial over a fixed index set, a fixed
// block tree, and a one-block finalize in a fixed order: bitwise reproducible.
#include "device.h"
#include "md_internal.h"

namespace md {
namespace {

constexpr int kKinGrid = 1024;

// Pair partial sums of the potential over i < j.  Block (bx, by) covers the 256
// particles i of block bx against j in the by-th j range; red[by*gx + bx].
// Ring term: 1/sqrt(2 sin^2((ti - tj)/2) + eps) (= 1/sqrt(1 - cos(ti - tj) + eps)).
// 2D term: log(|r_i - r_j|^2 + eps).
template <int MODEL>
__global__ __launch_bounds__(kEnergyBlock) void k_energy_pairs(const double *__restrict__ q, int n, int jlen,
                                                               double eps, double *__restrict__ red)
{
    __shared__ double lds[kEnergyBlock / kWave];
    const int ib = blockIdx.x * kEnergyBlock;
    const int i = ib + threadIdx.x;
    const int j0 = max((int)blockIdx.y * jlen, ib + 1);
    const int j1 = min(n, ((int)blockIdx.y + 1) * jlen);
    double acc = 0.0;
    if (i < n) {
        if (MODEL == MD_GRAV2D) {
            const double xi = q[i], yi = q[n + i];
            for (int j = j0; j < j1; ++j) {
                const double dx = xi - q[j];
                const double dy = yi - q[n + j];
                if (j > i) acc += log(dx * dx + dy * dy + eps);
            }
        } else {
            const double ti = q[i];
            for (int j = j0; j < j1; ++j) {
                const double h = sin(0.5 * (ti - q[j]));
                if (j > i) acc += 1.0 / sqrt(2.0 * h * h + eps);
            }
        }
    }
    const double b = block_sum(acc, lds);
    if (threadIdx.x == 0) red[blockIdx.y * gridDim.x + blockIdx.x] = b;
}

// Block partials of sum p^2 over len values (grid-stride, fixed grid).
__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ p, int64_t len,
                                               double *__restrict__ red)
{
    __shared__ double lds[4];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += stride) acc += p[k] * p[k];
    const double b = block_sum(acc, lds);
    if (threadIdx.x == 0) red[blockIdx.x] = b;
}

// Sum of red[0 .. m) in a fixed order (valid in thread 0).
__device__ double ordered_sum(const double *__restrict__ red, int m, int stride, double *lds)
{
    double acc = 0.0;
    for (int b = threadIdx.x; b < m; b += blockDim.x) acc += red[(size_t)b * stride];
    return block_sum(acc, lds);
}

// out = {K, V, K + V}.  redV: nv pair partials (Ring, 2D) or hmf_grid pairs of
// (sum cos, sum sin) (HMF).  redK: nk partials of sum p^2.
__global__ __launch_bounds__(256) void k_energy_finalize(const double *__restrict__ redV, int nv,
                                                         const double *__restrict__ redK, int nk, int model,
                                                         int n, double *__restrict__ out)
{
    __shared__ double lds[3][4];
    const double k2 = ordered_sum(redK, nk, 1, lds[0]);
    double v;
    if (model == MD_HMF) {
        const double sc = ordered_sum(redV, nv, 2, lds[1]);
        const double ss = ordered_sum(redV + 1, nv, 2, lds[2]);
        const double mx = sc / (double)n, my = ss / (double)n;
        v = 0.5 * (double)n * (1.0 - mx * mx - my * my);
    } else {
        const double sv = ordered_sum(redV, nv, 1, lds[1]);
        v = model == MD_GRAV2D ? sv / (double)n : -sv / (sqrt(2.0) * (double)n);
    }
    if (threadIdx.x == 0) {
        const double kin = 0.5 * k2;
        out[0] = kin;
        out[1] = v;
        out[2] = kin + v;
    }
}

// flag = 1 if any of v[0 .. count) is not finite, else 0 (one block).
__global__ __launch_bounds__(256) void k_finite_flag(const double *__restrict__ v, int count,
                                                     unsigned *__restrict__ flag)
{
    int bad = 0;
    for (int k = threadIdx.x; k < count; k += blockDim.x) bad |= !isfinite(v[k]);
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) *flag = bad ? 1u : 0u;
}

}  // namespace

hipError_t launch_finite_flag(md_ctx *c, const double *vals, int count)
{
    hipLaunchKernelGGL(k_finite_flag, dim3(1), dim3(256), 0, c->stream, vals, count, finite_flag(c));
    return hipGetLastError();
}

// Layout of the reduction scratch: [0, kRedSlots/2) potential partials,
// [kRedSlots/2, kRedSlots/2 + kKinGrid) kinetic partials.
int energy_jsplit(int64_t n)
{
    const int64_t ib = (n + kEnergyBlock - 1) / kEnergyBlock;
    int64_t s = 8;
    while (s > 1 && ib * s > kRedSlots / 2) s >>= 1;
    return (int)s;
}

hipError_t launch_energy(md_ctx *c, const double *q, const double *p, double *out3)
{
    const int n = (int)c->n;
    const int d = dims(c->model);
    double *redV = c->red;
    double *redK = c->red + kRedSlots / 2;
    int nv;
    if (c->model == MD_HMF) {
        // block partials of sum cos, sum sin of q (added here in FP64, in a fixed order; the pass's
        // fixed-point sums are not read)
        hipError_t e = launch_hmf_pass(c, 0, HMF_REDUCE, 0.0, 0.0, 0.0, const_cast<double *>(q), nullptr, nullptr,
                                       nullptr, false);
        if (e != hipSuccess) return e;
        nv = hmf_grid(c->n);
        redV = const_cast<double *>(hmf_partials(c));
    } else {
        const int gx = (n + kEnergyBlock - 1) / kEnergyBlock;
        const int s = energy_jsplit(c->n);
        const int jlen = (n + s - 1) / s;
        const dim3 grid((unsigned)gx, (unsigned)s);
        if (c->model == MD_GRAV2D)
            hipLaunchKernelGGL(k_energy_pairs<MD_GRAV2D>, grid, dim3(kEnergyBlock), 0, c->stream, q, n, jlen,
                               c->eps, redV);
        else
            hipLaunchKernelGGL(k_energy_pairs<MD_RING>, grid, dim3(kEnergyBlock), 0, c->stream, q, n, jlen,
                               c->eps, redV);
        nv = gx * s;
    }
    hipLaunchKernelGGL(k_sumsq, dim3(kKinGrid), dim3(256), 0, c->stream, p, (int64_t)d * n, redK);
    hipLaunchKernelGGL(k_energy_finalize, dim3(1), dim3(256), 0, c->stream, redV, nv, redK, kKinGrid, c->model,
                       n, out3);
    return hipGetLastError();
}

hipError_t launch_magnetization(md_ctx *c, const double *q, double *out2)
{
    hipError_t e = launch_hmf_begin(c);
    if (e == hipSuccess)
        e = launch_hmf_pass(c, 0, HMF_REDUCE, 0.0, 0.0, 0.0, const_cast<double *>(q), nullptr, nullptr, nullptr,
                            false);
    if (e != hipSuccess) return e;
    return launch_hmf_magnetization(c, out2);
}

}  // namespace md
