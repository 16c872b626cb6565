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
// dependency: each pass ends with FP64 block partials (wavefront butterfly, then
// a fixed serial order over wavefronts), which every block adds in fixed point
// (limbs of 2^-32 and 2^-64, 64-bit integer atomics into kMSlots slots) to one of
// three buffers, and every block of the next pass sums the slots exactly, in
// integers, and converts the total once to FP64 (no launch between passes).
// Integer sums do not depend on the order of the atomics, so M is reproducible,
// and it is the exact sum of the FP64 block partials rounded once.  That is for
// grids of at most kHmfInPassM blocks (N <= 2.1e6); on larger ones every block
// re-deriving M costs more than a launch, so a one-block kernel sums the FP64
// block partials in a fixed order instead (M then differs in its last bits from
// the fixed-point total; either way it is fixed per N, so runs are
// reproducible).  The kernel boundary is the only synchronisation: no
// device-wide fences (on this GPU a device-scope release writes back the L2 of
// the issuing XCD).  The FP64 block partials are always stored (the energy sums
// them in its own fixed order).
//
// Memory access: each lane moves W consecutive elements (16-byte vector loads and
// stores: W = 2 in FP64, 4 in FP32), U vectors per grid-stride iteration, over a
// grid of one block per 2048 particles (at most 32768 blocks).  Pointers that are
// not 16-byte aligned take W = 1.
//
// Also here: the O(N) Hessian-vector product of the HMF potential (the mean-field
// form of eqs. 6-7) and the elementwise stage of its reverse sweep.
#include "device.h"
#include "md_internal.h"

namespace md {
namespace {

constexpr int kUnroll = 2;  // vectors per thread per grid-stride iteration

// sincos of E angles, each step over all of them before the next, so that their
// chains interleave.  FP64: the branch-free reduced form for all, then the library
// for any angle beyond its range (never, for the dynamics here).
template <int E>
__device__ __forceinline__ void sincos_n(const double (&x)[E], double (&s)[E], double (&c)[E])
{
    bool big = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        sincos64_reduced(x[e], &s[e], &c[e]);
        big |= !(fabs(x[e]) < kSincosMaxArg);
    }
    if (big) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (!(fabs(x[e]) < kSincosMaxArg)) sincos(x[e], &s[e], &c[e]);
    }
}
template <int E>
__device__ __forceinline__ void sincos_n(const float (&x)[E], float (&s)[E], float (&c)[E])
{
#pragma unroll
    for (int e = 0; e < E; ++e) sincos32(x[e], &s[e], &c[e]);
}

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

// W consecutive values, aligned to their size (one vector load/store when W > 1).
template <typename T, int W>
struct alignas(sizeof(T) * W) Vec {
    T x[W];
};

struct PassArgs {
    double kick1, kick2, drift;
    int flags;
};

// The work of one stage on E particles: kick (with f from f_in or from M), drift,
// and the sincos of the new angle into the partial sums (of the particles with
// ok[e]; in the order of e).  Each step runs over all E particles before the next,
// with no branch between them.
template <typename T, int E>
__device__ __forceinline__ void stage_n(T (&t)[E], T (&p)[E], const double (&fin)[E], double (&fout)[E],
                                        const bool (&ok)[E], T mx, T my, T k1, T k2, T dr, int flags, double &sc,
                                        double &ss)
{
    if (flags & (HMF_KICK_M | HMF_STORE_F)) {
        T s[E], c[E], f[E];
        sincos_n(t, s, c);
#pragma unroll
        for (int e = 0; e < E; ++e) f[e] = c[e] * my - s[e] * mx;
        if (flags & HMF_STORE_F) {
#pragma unroll
            for (int e = 0; e < E; ++e) fout[e] = (double)f[e];
        }
        if (flags & HMF_KICK_M) {
#pragma unroll
            for (int e = 0; e < E; ++e) p[e] += k1 * f[e];
            if (flags & HMF_KICK2) {
#pragma unroll
                for (int e = 0; e < E; ++e) p[e] += k2 * f[e];
            }
        }
    } else if (flags & HMF_KICK_F) {
#pragma unroll
        for (int e = 0; e < E; ++e) p[e] += k1 * (T)fin[e];
    }
    if (flags & HMF_DRIFT) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            t[e] += dr * p[e];
            if constexpr (sizeof(T) == 4) t[e] = wrap_pi(t[e]);
        }
    }
    if (flags & HMF_REDUCE) {
        T s[E], c[E];
        sincos_n(t, s, c);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (ok[e]) {
                sc += (double)c[e];
                ss += (double)s[e];
            }
        }
    }
}

static_assert(kMSlots * kMLimbs == 256, "the 256 limb words: one per thread of a pass block");
static_assert(kMSlots == kWave, "one slot per lane of the wavefront that converts the sums");

// x = (hi + lo 2^-32) 2^-32, hi = floor(x 2^32), 0 <= lo <= 2^32: exact for |x| < 2^20
// down to 2^-64 (the bits below are rounded).
__device__ __forceinline__ void to_limbs(double x, long long &hi, long long &lo)
{
    const double y = x * 0x1p32;
    const double h = floor(y);
    hi = (long long)h;
    lo = (long long)rint((y - h) * 0x1p32);
}

// M = (the total of the limb sums) / n, by a wavefront whose lane l holds the limbs
// of slot l: a butterfly adds the slots in 64-bit integers (exact, so every lane
// ends with the same total, in any order).
__device__ __forceinline__ void limbs_sum(long long (&v)[kMLimbs], int n, double &mx, double &my)
{
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1)
#pragma unroll
        for (int l = 0; l < kMLimbs; ++l) v[l] += __shfl_xor(v[l], m);
    mx = ((double)v[0] * 0x1p-32 + (double)v[1] * 0x1p-64) / (double)n;
    my = ((double)v[2] * 0x1p-32 + (double)v[3] * 0x1p-64) / (double)n;
}

// The same total by the 256 threads of a block: one word each, then four threads
// add the 64 slots of one limb (a barrier before and after).
__device__ __forceinline__ void limbs_sum_block(const long long *__restrict__ acc, int n, long long *lds, double &mx,
                                                double &my)
{
    const int t = threadIdx.x;
    lds[t] = acc[t];
    __syncthreads();
    if (t < kMLimbs) {
        long long v = 0;
        for (int k = 0; k < kMSlots; ++k) v += lds[k * kMLimbs + t];
        lds[kMSlots * kMLimbs + t] = v;
    }
    __syncthreads();
    const long long *L = lds + kMSlots * kMLimbs;
    mx = ((double)L[0] * 0x1p-32 + (double)L[1] * 0x1p-64) / (double)n;
    my = ((double)L[2] * 0x1p-32 + (double)L[3] * 0x1p-64) / (double)n;
}

// One kick/drift/reduce pass over all particles (grid-stride over a grid fixed
// per n, so every partial sum is reproducible).  T: state type; W: elements per
// vector access.  HMF_REDUCE writes the block partials (sum cos, sum sin) to
// red[2b], red[2b+1].  LIMBS (small grids): HMF_KICK_M / HMF_STORE_F take the
// magnetization from the limb sums mrd (block 0 also stores it to M), HMF_REDUCE
// adds the partials' limbs to mwr, and block 0 zeroes mzero for a later pass.
// Without LIMBS the kernel reads M[0..1] and leaves the partials to the one-block
// kernel (no code of the limbs).  Launched with 256 threads.
template <typename T, int W, bool LIMBS>
__global__ __launch_bounds__(256) void k_hmf_pass(T *__restrict__ th, T *__restrict__ p,
                                                  const double *__restrict__ f_in, double *__restrict__ f_out,
                                                  const long long *__restrict__ mrd, long long *__restrict__ mwr,
                                                  long long *__restrict__ mzero, double *__restrict__ M,
                                                  PassArgs a, int n, double *__restrict__ red, T *__restrict__ snap)
{
    __shared__ double lds[2][4];
    __shared__ long long mlds[LIMBS ? kMSlots * kMLimbs + kMLimbs : 1];
    const int flags = a.flags;
    const T k1 = (T)a.kick1, k2 = (T)a.kick2, dr = (T)a.drift;
    T mx = 0, my = 0;
    if (flags & (HMF_KICK_M | HMF_STORE_F)) {
        if constexpr (LIMBS) {
            double dmx, dmy;
            limbs_sum_block(mrd, n, mlds, dmx, dmy);
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                M[0] = dmx;
                M[1] = dmy;
            }
            mx = (T)dmx;
            my = (T)dmy;
        } else {
            mx = (T)M[0];
            my = (T)M[1];
        }
    }
    if (LIMBS && blockIdx.x == 0) mzero[threadIdx.x] = 0;
    const bool need_p = flags & (HMF_KICK_F | HMF_KICK_M | HMF_DRIFT);
    const bool write = flags & HMF_WRITE;
    double sc = 0.0, ss = 0.0;
    const int nvec = n / W;
    const int stride = gridDim.x * blockDim.x;
    using VT = Vec<T, W>;
    using VD = Vec<double, W>;
    constexpr int E = kUnroll * W;  // particles per thread and iteration: e = u W + w
    for (int base = blockIdx.x * blockDim.x + threadIdx.x; base < nvec; base += stride * kUnroll) {
        VT t[kUnroll], q[kUnroll];
        VD fi[kUnroll];
        bool ok[E];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int v = base + u * stride;
            t[u] = VT{};
            q[u] = VT{};
            fi[u] = VD{};
            if (v < nvec) {
                t[u] = reinterpret_cast<const VT *>(th)[v];
                if (need_p) q[u] = reinterpret_cast<const VT *>(p)[v];
                if (flags & HMF_KICK_F) fi[u] = reinterpret_cast<const VD *>(f_in)[v];
            }
#pragma unroll
            for (int w = 0; w < W; ++w) ok[u * W + w] = v < nvec;
        }
        T te[E], pe[E];
        double fe[E], fo[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            te[e] = t[e / W].x[e % W];
            pe[e] = q[e / W].x[e % W];
            fe[e] = fi[e / W].x[e % W];
            fo[e] = 0.0;
        }
        stage_n(te, pe, fe, fo, ok, mx, my, k1, k2, dr, flags, sc, ss);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int v = base + u * stride;
            if (v >= nvec) continue;
            VT to, po;
            VD ff;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                to.x[w] = te[u * W + w];
                po.x[w] = pe[u * W + w];
                ff.x[w] = fo[u * W + w];
            }
            if (flags & HMF_STORE_F) reinterpret_cast<VD *>(f_out)[v] = ff;
            if (write) {
                reinterpret_cast<VT *>(th)[v] = to;
                if (need_p) reinterpret_cast<VT *>(p)[v] = po;
            }
            if (snap && (flags & HMF_DRIFT)) {
#pragma unroll
                for (int w = 0; w < W; ++w) snap[v * W + w] = to.x[w];
            }
        }
    }
    // the n mod W particles past the last full vector: block 0
    if (W > 1 && blockIdx.x == 0 && (int)threadIdx.x < n - nvec * W) {
        const int i = nvec * W + threadIdx.x;
        T t1[1] = {th[i]};
        T p1[1] = {need_p ? p[i] : T(0)};
        const double f1[1] = {(flags & HMF_KICK_F) ? f_in[i] : 0.0};
        double fo1[1] = {0.0};
        const bool ok1[1] = {true};
        stage_n(t1, p1, f1, fo1, ok1, mx, my, k1, k2, dr, flags, sc, ss);
        if (flags & HMF_STORE_F) f_out[i] = fo1[0];
        if (write) {
            th[i] = t1[0];
            if (need_p) p[i] = p1[0];
        }
        if (snap && (flags & HMF_DRIFT)) snap[i] = t1[0];
    }
    if (flags & HMF_REDUCE) {
        const double bc = block_sum(sc, lds[0]);
        const double bs = block_sum(ss, lds[1]);
        if (threadIdx.x == 0) {
            red[2 * blockIdx.x] = bc;
            red[2 * blockIdx.x + 1] = bs;
        }
        if (LIMBS && threadIdx.x == 0) {
            unsigned long long *w = reinterpret_cast<unsigned long long *>(mwr + (blockIdx.x % kMSlots) * kMLimbs);
            long long hi, lo;
            to_limbs(bc, hi, lo);
            atomicAdd(w, (unsigned long long)hi);  // two's complement: the signed sum, exactly
            atomicAdd(w + 1, (unsigned long long)lo);
            to_limbs(bs, hi, lo);
            atomicAdd(w + 2, (unsigned long long)hi);
            atomicAdd(w + 3, (unsigned long long)lo);
        }
    }
}

// Zeroes one limb buffer (the first of a call's passes adds into it).
__global__ __launch_bounds__(256) void k_hmf_zero_limbs(long long *__restrict__ acc) { acc[threadIdx.x] = 0; }

// M from the limb sums of one buffer (one wavefront, lane l loads slot l), to
// M[0..1] and (if given) out[0..1].
__global__ __launch_bounds__(64) void k_hmf_limbs_to_m(const long long *__restrict__ acc, int n,
                                                       double *__restrict__ out, double *__restrict__ M)
{
    double mx, my;
    long long v[kMLimbs];
#pragma unroll
    for (int l = 0; l < kMLimbs; ++l) v[l] = acc[threadIdx.x * kMLimbs + l];
    limbs_sum(v, n, mx, my);
    if (threadIdx.x == 0) {
        if (out) {
            out[0] = mx;
            out[1] = my;
        }
        M[0] = mx;
        M[1] = my;
    }
}

// M[0..1] = (sum of the g partial pairs) / n, in a fixed order (one block of
// 1024 threads; thread t adds partials t, t + 1024, ... in that order).  Loads go
// out kFinBatch per thread at a time, which keeps the kernel in registers (no
// private segment) at 1024 threads; g <= kHmfGrid takes at most 4 batches.
constexpr int kFinBatch = 8;

__global__ __launch_bounds__(1024) void k_hmf_finalize(const double *__restrict__ red, int g, int n,
                                                       double *__restrict__ M)
{
    __shared__ double lds[2][16];
    double c = 0.0, s = 0.0;
    for (int b0 = 0; b0 < g; b0 += 1024 * kFinBatch) {
        double vc[kFinBatch], vs[kFinBatch];
#pragma unroll
        for (int k = 0; k < kFinBatch; ++k) {
            const int b = b0 + threadIdx.x + 1024 * k;
            vc[k] = b < g ? red[2 * b] : 0.0;
            vs[k] = b < g ? red[2 * b + 1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kFinBatch; ++k) {
            c += vc[k];
            s += vs[k];
        }
    }
    c = block_sum(c, lds[0]);
    s = block_sum(s, lds[1]);
    if (threadIdx.x == 0) {
        M[0] = c / (double)n;
        M[1] = s / (double)n;
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

// ------------------------------------------------------------------- adjoint --
// HMF Hessian-vector product, O(N): phi''(d) = cos(d)/N gives
//   (H w)_i = w_i (c_i Mx + s_i My) - (c_i Cw + s_i Sw),
// Mx, My the magnetization (eq. 7), Cw = (1/N) sum c_j w_j, Sw = (1/N) sum s_j w_j.

// Block partials of sum c, sum s, sum c w, sum s w (grid-stride, fixed grid).
__global__ __launch_bounds__(256) void k_hmf_hvp_sums(const double *__restrict__ th, const double *__restrict__ w,
                                                      int n, double *__restrict__ red)
{
    __shared__ double lds[4][4];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double s, c;
        sincos64(th[i], &s, &c);
        const double wi = w[i];
        a[0] += c;
        a[1] += s;
        a[2] += c * wi;
        a[3] += s * wi;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double b = block_sum(a[k], lds[k]);
        if (threadIdx.x == 0) red[4 * blockIdx.x + k] = b;
    }
}

// sums[0..3] = (Mx, My, Cw, Sw): the g partial quadruples added in a fixed order.
__global__ __launch_bounds__(256) void k_hmf_hvp_finalize(const double *__restrict__ red, int g, int n,
                                                          double *__restrict__ sums)
{
    __shared__ double lds[4][4];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < g; b += blockDim.x)
        for (int k = 0; k < 4; ++k) a[k] += red[4 * b + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = block_sum(a[k], lds[k]);
        if (threadIdx.x == 0) sums[k] = t / (double)n;
    }
}

// Elementwise, with the sums of H(th) lp: hw = (H lp)_i; out = hw; lq -= h hw
// [; lq -= h2 hw]; lp += a lq.  Flags as the pair-model adjoint update.
__global__ __launch_bounds__(256) void k_hmf_adj_update(const double *__restrict__ th, const double *__restrict__ sums,
                                                        int flags, double h, double h2, double a, int n,
                                                        double *__restrict__ lq, double *__restrict__ lp,
                                                        double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (flags & (ADJ_OUT | ADJ_KICK)) {
        double s, c;
        sincos64(th[i], &s, &c);
        const double w = lp[i];
        const double hw = w * (c * sums[0] + s * sums[1]) - (c * sums[2] + s * sums[3]);
        if (flags & ADJ_OUT) out[i] = hw;
        if (flags & ADJ_KICK) {
            double l = lq[i] - h * hw;
            if (flags & ADJ_KICK2) l -= h2 * hw;
            lq[i] = l;
        }
    }
    if (flags & ADJ_DRIFT) lp[i] += a * lq[i];
}

}  // namespace

// Vector width of the accesses for this context (1 when a pointer is not 16-byte aligned).
static int vec_width(bool f32, const void *a, const void *b, const void *c, const void *d)
{
    const uintptr_t m = (uintptr_t)a | (uintptr_t)b | (uintptr_t)c | (uintptr_t)d;
    if (m & 15u) return 1;
    return f32 ? 4 : 2;
}

// Blocks of an HMF pass: 2048 particles per block (two grid-stride iterations of
// W = 2 at kUnroll = 2); measured at N = 1e7 against 1024 (7% slower: each block's
// closing reduction is amortised over fewer particles) and 4096 (2% slower).  At
// most kHmfGrid blocks (N = 6.7e7); above that the grid strides.  Capping at 16384
// instead made N = 5e7 8% slower.
int hmf_grid(int64_t n)
{
    const int64_t per_block = 256 * kUnroll * 2 * 2;
    const int64_t b = (n + per_block - 1) / per_block;
    return (int)(b < kHmfGrid ? (b < 1 ? 1 : b) : kHmfGrid);
}

const double *hmf_partials(const md_ctx *c) { return c->red; }

// The passes of this context sum M in fixed point (small grids) rather than
// through the one-block kernel over the FP64 partials.
static bool hmf_in_pass(const md_ctx *c) { return hmf_grid(c->n) <= kHmfInPassM; }

hipError_t launch_hmf_begin(md_ctx *c)
{
    if (!hmf_in_pass(c)) return hipSuccess;
    hipLaunchKernelGGL(k_hmf_zero_limbs, dim3(1), dim3(kMSlots * kMLimbs), 0, c->stream, c->macc);
    return hipGetLastError();
}

hipError_t launch_hmf_pass(md_ctx *c, int k, int flags, double kick1, double kick2, double drift, double *th,
                           double *p, const double *f_in, double *f_out, bool f32state, double *snap)
{
    const int n = (int)c->n;
    const int g = hmf_grid(c->n);
    const PassArgs a{kick1, kick2, drift, flags};
    constexpr int B = kMSlots * kMLimbs;  // words per limb buffer
    // Small grids: M from the limb sums inside the pass, no other launch.  Large
    // ones: the one-block kernel over the FP64 partials after a reducing pass, and
    // M read from c->scal.
    const bool in_pass = hmf_in_pass(c);
    const long long *mrd = in_pass ? c->macc + (size_t)((k + 2) % 3) * B : nullptr;
    long long *mwr = in_pass ? c->macc + (size_t)(k % 3) * B : nullptr;
    long long *mzero = in_pass ? c->macc + (size_t)((k + 1) % 3) * B : nullptr;
    const int ts = timed_begin(c, "k_hmf_pass");
#define MD_HMF_PASS(T_, W_, TH_, P_, SNAP_)                                                                          \
    do {                                                                                                         \
        if (in_pass)                                                                                             \
            hipLaunchKernelGGL((k_hmf_pass<T_, W_, true>), dim3(g), dim3(256), 0, c->stream, TH_, P_, f_in, f_out, \
                               mrd, mwr, mzero, c->scal, a, n, c->red, SNAP_);                                   \
        else                                                                                                     \
            hipLaunchKernelGGL((k_hmf_pass<T_, W_, false>), dim3(g), dim3(256), 0, c->stream, TH_, P_, f_in,      \
                               f_out, mrd, mwr, mzero, c->scal, a, n, c->red, SNAP_);                            \
    } while (0)
    if (f32state) {
        if (vec_width(true, c->th32, c->p32, f_in, f_out) == 4) MD_HMF_PASS(float, 4, c->th32, c->p32, (float *)nullptr);
        else MD_HMF_PASS(float, 1, c->th32, c->p32, (float *)nullptr);
    } else {
        // snap: element stores, any alignment
        if (vec_width(false, th, p, f_in, f_out) == 2) MD_HMF_PASS(double, 2, th, p, snap);
        else MD_HMF_PASS(double, 1, th, p, snap);
    }
#undef MD_HMF_PASS
    hipError_t e = hipGetLastError();
    timed_end(c, ts);
    if (e == hipSuccess && !in_pass && (flags & HMF_REDUCE)) {
        hipLaunchKernelGGL(k_hmf_finalize, dim3(1), dim3(1024), 0, c->stream, c->red, g, n, c->scal);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_hmf_magnetization(md_ctx *c, double *out2)
{
    if (!hmf_in_pass(c))  // the reducing pass's one-block kernel left M in c->scal
        return hipMemcpyAsync(out2, c->scal, 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    hipLaunchKernelGGL(k_hmf_limbs_to_m, dim3(1), dim3(kWave), 0, c->stream, c->macc, (int)c->n, out2, c->scal);
    return hipGetLastError();
}

hipError_t launch_hmf_convert(md_ctx *c, double *th, double *p, bool to_f32)
{
    const int n = (int)c->n;
    hipLaunchKernelGGL(k_hmf_convert, dim3((n + 255) / 256), dim3(256), 0, c->stream, th, p, c->th32, c->p32,
                       n, to_f32 ? 1 : 0);
    return hipGetLastError();
}

// Sums (Mx, My, Cw, Sw) of H(th) w into the context scalars c->scal[4..7].
hipError_t launch_hmf_hvp_sums(md_ctx *c, const double *th, const double *w)
{
    const int n = (int)c->n;
    int g = (int)((c->n + 255) / 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_hmf_hvp_sums, dim3(g), dim3(256), 0, c->stream, th, w, n, c->red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hmf_hvp_finalize, dim3(1), dim3(256), 0, c->stream, c->red, g, n, c->scal + 4);
    return hipGetLastError();
}

hipError_t launch_hmf_adj_update(md_ctx *c, const double *th, int flags, double h, double h2, double a, double *lq,
                                 double *lp, double *out)
{
    const int n = (int)c->n;
    hipLaunchKernelGGL(k_hmf_adj_update, dim3((n + 255) / 256), dim3(256), 0, c->stream, th, c->scal + 4, flags, h, h2,
                       a, n, lq, lp, out);
    return hipGetLastError();
}

}  // namespace md
