// hmf.hip -- the Hamiltonian Mean Field model in O(N) (Sec. 3.1): the force
// f_i = cos(t_i) My - sin(t_i) Mx (eq. 6) from the magnetization
// (Mx, My) = (1/N) sum_i (cos t_i, sin t_i) (eq. 7).
//
// Unlike the paper's kernels, the cosines and sines are not stored: one pass
// over the particles reads (t, p) once, kicks with the current magnetization
// (recomputing sincos of the old angle), drifts, takes sincos of the new angle
// for the next magnetization, and writes (t, p) back.  Stored sines/cosines
// would add 32 B of HBM traffic per particle per stage to a bandwidth-bound
// pass; two sincos evaluations cost less.  The magnetization is a grid-wide
// dependency, so each pass ends with FP64 block partials (wavefront butterfly,
// then a fixed serial order over wavefronts) and a one-block finalize kernel sums
// them in a fixed order: deterministic, no atomics.
#include "device.h"
#include "md_internal.h"

namespace md {
namespace {

__device__ __forceinline__ void sincos_(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_(float x, float *s, float *c) { sincosf(x, s, c); }

// Map an FP32 angle into [-pi, pi).
__device__ __forceinline__ float wrap_pi(float t)
{
    const float two_pi = 6.28318530717958647692f;
    const float k = rintf(t * 0.159154943091895335769f);
    t = __builtin_fmaf(-k, two_pi, t);
    if (t >= 3.14159265358979323846f) t -= two_pi;
    if (t < -3.14159265358979323846f) t += two_pi;
    return t;
}

// One kick/drift/reduce pass over all particles (grid-stride; the grid size is
// fixed per n, so the partial sums are reproducible).  T is the state type.
template <typename T>
__global__ __launch_bounds__(256) void k_hmf_pass(T *__restrict__ th, T *__restrict__ p,
                                                  const double *__restrict__ f_in,
                                                  const double *__restrict__ M, double *__restrict__ f_out,
                                                  T kick1, T kick2, T drift, int flags, int n,
                                                  double *__restrict__ red)
{
    __shared__ double lds[2][4];
    T mx = 0, my = 0;
    if (flags & (HMF_KICK_M | HMF_STORE_F)) {
        mx = (T)M[0];
        my = (T)M[1];
    }
    double sc = 0.0, ss = 0.0;
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        T t = th[i];
        T pp = 0;
        if (flags & (HMF_KICK_F | HMF_KICK_M | HMF_DRIFT)) pp = p[i];
        if (flags & (HMF_KICK_M | HMF_STORE_F)) {
            T s, c;
            sincos_(t, &s, &c);
            const T f = c * my - s * mx;
            if (flags & HMF_STORE_F) f_out[i] = (double)f;
            if (flags & HMF_KICK_M) {
                pp += kick1 * f;
                if (flags & HMF_KICK2) pp += kick2 * f;
            }
        } else if (flags & HMF_KICK_F) {
            pp += kick1 * (T)f_in[i];
        }
        if (flags & HMF_DRIFT) {
            t += drift * pp;
            if constexpr (sizeof(T) == 4) t = wrap_pi(t);
        }
        if (flags & HMF_WRITE) {
            th[i] = t;
            p[i] = pp;
        }
        if (flags & HMF_REDUCE) {
            T s, c;
            sincos_(t, &s, &c);
            sc += (double)c;
            ss += (double)s;
        }
    }
    if (flags & HMF_REDUCE) {
        const double bc = block_sum(sc, lds[0]);
        const double bs = block_sum(ss, lds[1]);
        if (threadIdx.x == 0) {
            red[2 * blockIdx.x] = bc;
            red[2 * blockIdx.x + 1] = bs;
        }
    }
}

// M[0..1] = (sum of the nblk partial pairs) / n, in a fixed order.
__global__ __launch_bounds__(256) void k_hmf_finalize(const double *__restrict__ red, int nblk, int n,
                                                      double *__restrict__ M)
{
    __shared__ double lds[2][4];
    double sc = 0.0, ss = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        sc += red[2 * b];
        ss += red[2 * b + 1];
    }
    sc = block_sum(sc, lds[0]);
    ss = block_sum(ss, lds[1]);
    if (threadIdx.x == 0) {
        M[0] = sc / (double)n;
        M[1] = ss / (double)n;
    }
}

// FP64 state <-> FP32 state (angles wrapped to [-pi, pi) on the way in).
__global__ __launch_bounds__(256) void k_hmf_convert(double *__restrict__ th, double *__restrict__ p,
                                                     float *__restrict__ th32, float *__restrict__ p32,
                                                     int n, int to_f32)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (to_f32) {
        th32[i] = wrap_pi((float)th[i]);
        p32[i] = (float)p[i];
    } else {
        th[i] = (double)th32[i];
        p[i] = (double)p32[i];
    }
}

}  // namespace

int hmf_grid(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int)(b < kHmfGrid ? (b < 1 ? 1 : b) : kHmfGrid);
}

hipError_t launch_hmf_pass(md_ctx *c, int flags, double kick1, double kick2, double drift, double *th,
                           double *p, const double *f_in, double *f_out, bool f32state)
{
    const int n = (int)c->n;
    const int g = hmf_grid(c->n);
    if (f32state) {
        hipLaunchKernelGGL((k_hmf_pass<float>), dim3(g), dim3(256), 0, c->stream, c->th32, c->p32, f_in,
                           c->scal, f_out, (float)kick1, (float)kick2, (float)drift, flags, n, c->red);
    } else {
        hipLaunchKernelGGL((k_hmf_pass<double>), dim3(g), dim3(256), 0, c->stream, th, p, f_in, c->scal,
                           f_out, kick1, kick2, drift, flags, n, c->red);
    }
    return hipGetLastError();
}

hipError_t launch_hmf_finalize(md_ctx *c)
{
    hipLaunchKernelGGL(k_hmf_finalize, dim3(1), dim3(256), 0, c->stream, c->red, hmf_grid(c->n), (int)c->n,
                       c->scal);
    return hipGetLastError();
}

hipError_t launch_hmf_convert(md_ctx *c, double *th, double *p, bool to_f32)
{
    const int n = (int)c->n;
    hipLaunchKernelGGL(k_hmf_convert, dim3((n + 255) / 256), dim3(256), 0, c->stream, th, p, c->th32, c->p32,
                       n, to_f32 ? 1 : 0);
    return hipGetLastError();
}

}  // namespace md
