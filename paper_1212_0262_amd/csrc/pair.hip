// pair.hip -- the O(N^2) all-pairs forces of the Ring model (eqs. 8-9) and the
// 2D self-gravitating model (gradient of eq. 3), and the O(N) kick/drift stages
// of the Yoshida composition (eq. 4) that surround them.
//
// Staged pair kernel design (gfx950, wave64):
//   * i-tile in registers: each lane owns i_per_lane particles i, 64 apart.
//   * j-stream broadcast: every lane of a wavefront walks the same j, so the j
//     operands are wave-uniform loads that the compiler places in scalar
//     registers (s_load through the scalar cache); they feed the VALU directly as
//     the one scalar operand an instruction may take.  No LDS, no barriers.
//   * j-split: the j range is cut into j_split pieces computed by different
//     blocks (grid.y) so that small N still fills 256 CUs; the partial sums are
//     added in a fixed order by the update kernel (deterministic).
// The fused small-N stage (k_fused, below) keeps the same j ranges and order but
// moves them into one block per i tile, streams j through LDS, and adds the
// partials and runs the update in the same launch.
//   * self pair: contributes exactly zero (2D: dx = dy = 0; Ring: the numerator
//     sin(ti)cos(tj) - cos(ti)sin(tj) is formed from rounded products, without
//     fused multiply-add, so it is exactly 0 at j = i), so no mask is needed.
//   * ragged N: the j loop bound is uniform; lanes with i >= N load particle
//     N-1 and do not store.
// Accumulation policies (md_prec): FP32 partial per j-tile folded into FP64;
// Kahan-compensated FP32 per pair; FP64 add per pair; plain FP64.
#include "device.h"
#include "md_internal.h"
#include "pair_terms.h"

#include <type_traits>

namespace md {
namespace {

using namespace pairs;

// ---------------------------------------------------------------- pair kernels --

// part[(s*2 + c)*npad + i] = sum over j in the s-th j range of the 2D pair term.
template <typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_pair_2d(const T *__restrict__ xs, const T *__restrict__ ys,
                                                 int n, int npad, int jlen, int jtile, T eps,
                                                 double *__restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = (blockIdx.x * (blockDim.x / kWave) + wave) * (kWave * IPL) + lane;
    const int s = blockIdx.y;
    const int j0 = s * jlen;
    const int j1 = min(n, j0 + jlen);

    T xi[IPL], yi[IPL];
    A ax[IPL], ay[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, n - 1);
        xi[k] = xs[i];
        yi[k] = ys[i];
    }
    grav_j_range<T, A, IPL>(xs, ys, j0, j1, jtile, eps, xi, yi, ax, ay);
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < n) {
            part[(size_t)(2 * s) * npad + i] = ax[k].get();
            part[(size_t)(2 * s + 1) * npad + i] = ay[k].get();
        }
    }
}

// Adds the Ring pair terms of j in [j0, j1) to each lane's IPL accumulators, in
// the order every Ring kernel shares (j ascending, folds every jtile j).
// cc, ss: the j operand rows (wave-uniform).
template <typename T, typename A, int IPL>
__device__ __forceinline__ void ring_range(const T *__restrict__ cc, const T *__restrict__ ss, int j0, int j1,
                                           int jtile, T one_eps, const T (&ci)[IPL], const T (&si)[IPL],
                                           A (&a)[IPL])
{
    for (int jt = j0; jt < j1; jt += jtile) {
        const int je = min(j1, jt + jtile);
        int j = jt;
        for (; j + 8 <= je; j += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const T cj = cc[j + u];
                const T sj = ss[j + u];
#pragma unroll
                for (int k = 0; k < IPL; ++k) ring_term(ci[k], si[k], cj, sj, one_eps, a[k]);
            }
        }
        for (; j < je; ++j) {
            const T cj = cc[j];
            const T sj = ss[j];
#pragma unroll
            for (int k = 0; k < IPL; ++k) ring_term(ci[k], si[k], cj, sj, one_eps, a[k]);
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k) a[k].fold();
    }
}

// part[s*npad + i] = sum over j in the s-th j range of the Ring pair term.
// cs = two rows of npad: [cos t | sin t] (FP64) or sqrt2 [cos(t/2) | sin(t/2)] (FP32).
template <typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_pair_ring(const T *__restrict__ cs, int n, int npad, int jlen,
                                                   int jtile, T one_eps, double *__restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = (blockIdx.x * (blockDim.x / kWave) + wave) * (kWave * IPL) + lane;
    const int s = blockIdx.y;
    const int j0 = s * jlen;
    const int j1 = min(n, j0 + jlen);
    const T *__restrict__ cc = cs;
    const T *__restrict__ ss = cs + npad;

    T ci[IPL], si[IPL];
    A a[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, n - 1);
        ci[k] = cc[i];
        si[k] = ss[i];
    }
    ring_range<T, A, IPL>(cc, ss, j0, j1, jtile, one_eps, ci, si, a);
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < n) part[(size_t)s * npad + i] = a[k].get();
    }
}

// Staged pair kernel with the j operands in a block-shared LDS window (coalesced
// vector loads, one barrier pair per window) instead of wave-uniform scalar loads:
// at mid-range N too few wavefronts share a SIMD to hide the scalar loads' latency
// (they return out of order, so each wait is for all of them), while vector loads
// pipeline.  Same j ranges, order and folds as k_pair_2d / k_pair_ring, so the same
// partials bit for bit.  r0, r1: the two operand rows.
constexpr int kWinJ = 512;  // j per window
// The Ring FP32 (half-angle) forms take this kernel at every N: measured 7-10%
// faster than the scalar-load kernel with the per-tile fold and 13-14% with Kahan
// (N = 10240 .. 512000).  Both j operands enter the same instructions there, and
// the VALU takes few scalar operands, so scalar j operands cost extra moves; from
// LDS they arrive in vector registers.  The FP64 forms (8-byte operands) and the
// 2D forms measured 2-11% slower with the window.

template <int MODEL, typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_pair_win(const T *__restrict__ r0, const T *__restrict__ r1, int n,
                                                  int npad, int jlen, int jtile, T e, double *__restrict__ part)
{
    __shared__ T win[2][kWinJ];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = (blockIdx.x * (blockDim.x / kWave) + wave) * (kWave * IPL) + lane;
    const int s = blockIdx.y;
    const int j0 = s * jlen;
    const int j1 = min(n, j0 + jlen);
    T a0[IPL], a1[IPL];
    A acc0[IPL], acc1[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, n - 1);
        a0[k] = r0[i];
        a1[k] = r1[i];
    }
    auto term = [&](T x, T y) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            if constexpr (MODEL == MD_GRAV2D) pair_2d(a0[k], a1[k], x, y, e, acc0[k], acc1[k]);
            else ring_term(a0[k], a1[k], x, y, e, acc0[k]);
        }
    };
    window_stream<kWinJ>(r0, r1, j0, j1, jtile, win, term, [&]() {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            acc0[k].fold();
            if constexpr (MODEL == MD_GRAV2D) acc1[k].fold();
        }
    });
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < n) {
            if constexpr (MODEL == MD_GRAV2D) {
                part[(size_t)(2 * s) * npad + i] = acc0[k].get();
                part[(size_t)(2 * s + 1) * npad + i] = acc1[k].get();
            } else {
                part[(size_t)s * npad + i] = acc0[k].get();
            }
        }
    }
}

// ------------------------------------------------------- symmetric kernels --

// One launch of k_sym<MODEL, T, A> per force evaluation takes the diagonal tiles
// (a, a): every ordered pair of the tile, i side only; and every tile pair (a, b),
// a < b, of a single system (the scheme of sym_tile in pair_terms.h):
//   i side: the tile's sum goes to slot b of the i particles (MD_MIXED: partials
//     over 128 j folded into FP64);
//   j side: the sum over the 256 i of a wavefront, the 4 wavefronts added in
//     FP64 in a fixed order at the end of the tile (MD_MIXED, FP32 wavefront
//     sums) or after every 64-j block through a small LDS buffer (the other
//     accumulations), into slot a of the j particles.
// Each particle thus receives one slot per tile and the update kernel adds them
// in FP64 in the fixed order of slot_sums (device.h): no atomics.  The slots of
// MD_MIXED are FP32 (the tile's sum rounded once: half the bytes the update reads
// back, for a rounding below that of the FP32 partials themselves); the others
// are FP64.  The tile pairs are numbered by sym_tile_pair (pair_terms.h).
// Pad particles (n .. npad - 1) contribute nothing:
//   2D FP32: at (1e30, 1e30): r^2 overflows to +inf for any pair with a pad
//     particle, the reciprocal is 0 and both terms are exactly zero (a pad-pad
//     pair has dx = dy = 0);
//   2D FP64: at (1e150, 1e150): r^2 is about 2e300 (finite: the refined FP64
//     reciprocal of +inf would be NaN), so a term with a pad particle is about
//     5e-151, below the last bit of any force sum larger than 1e-135;
//   Ring: operands (0, 0): the numerator p is exactly 0 and q finite.

// Slot type of the symmetric form with accumulator A.
template <typename A>
using sym_slot_t = std::conditional_t<std::is_same_v<A, AccTile>, float, double>;

// JW32 (MD_MIXED): the wavefronts' FP32 j-side sums of the whole tile, added at
// its end; otherwise (Kahan, per-pair FP64, FP64) their FP64 values after every
// 64-j block (a Kahan sum's value carries its compensation: FP32 would drop it).
template <typename A>
constexpr bool kJW32 = std::is_same_v<A, AccTile>;
// The block's LDS for the j-side sums of a tile pair of W wavefronts (one of the
// two arrays is in use: a union, so the unused one adds no bytes to the block's
// LDS, which sets how many blocks a CU holds).
template <int D, typename A, int W>
union SymLds {
    float jw32[kJW32<A> ? W : 1][D][kJW32<A> ? W * kWave * kSymIpl : 1];
    double jw64[kJW32<A> ? 1 : W][D][kJW32<A> ? 1 : kWave];
};

// One block's share of a symmetric force evaluation: the tile pair (a, b), a < b
// (SYM), or the diagonal tile a = b, of tiles of W x 64 x 4 particles (W = 4: the
// 1024 of kSymTile; W = 2: 512 for smaller n, sym_tile_n in api.hip).  r0, r1: the operand rows ([2][npad],
// padded); part: slots [ntile][D][npad] of sym_slot_t<A>.
template <int MODEL, typename T, typename A, bool SYM, int W>
__device__ __forceinline__ void sym_block(const T *__restrict__ r0, const T *__restrict__ r1, int n, int npad,
                                          T e, sym_slot_t<A> *__restrict__ part, int a, int b,
                                          SymLds<MODEL == MD_GRAV2D ? 2 : 1, A, W> &lds)
{
    constexpr bool JW32 = kJW32<A>;
    constexpr int D = MODEL == MD_GRAV2D ? 2 : 1;
    constexpr int TILE = W * kWave * kSymIpl;
    auto &jw32 = lds.jw32;
    auto &jw64 = lds.jw64;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int i0 = a * TILE + wave * kWave * kSymIpl + lane;
    T u0[kSymIpl], u1[kSymIpl];
    A acc[D][kSymIpl];
#pragma unroll
    for (int k = 0; k < kSymIpl; ++k) {
        u0[k] = r0[i0 + k * kWave];
        u1[k] = r1[i0 + k * kWave];
    }
    const int jl = b * TILE + lane;
    auto load = [&](int blk, T &v0, T &v1) {
        v0 = r0[jl + blk * kWave];
        v1 = r1[jl + blk * kWave];
    };
    auto jsum = [&](int blk, int m, A (&sj)[D]) {
        if constexpr (JW32) {
#pragma unroll
            for (int d = 0; d < D; ++d) jw32[wave][d][blk * kWave + m] = (float)sj[d].get();
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) jw64[wave][d][m] = sj[d].get();
            __syncthreads();
            for (int x = threadIdx.x; x < D * kWave; x += W * kWave) {  // W = 1: a thread per (d, j) in turn
                const int d = x / kWave, mm = x & (kWave - 1);
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < W; ++w) t += jw64[w][d][mm];
                part[(size_t)(D * a + d) * npad + b * TILE + blk * kWave + mm] = (sym_slot_t<A>)t;
            }
            __syncthreads();
        }
    };
    // 2D FP64: one reciprocal for a lane's four i against each j (SHARE), except in
    // a j tile that holds pads (b is never below a).  Measured at N = 262,144, per
    // force evaluation: 16.36 -> 14.76 ms with one reciprocal for two i, and 4% less
    // again with one for four.  The FP32 forms keep one reciprocal a pair: there the
    // shared form measured 1.5% slower (7.35 -> 7.45 ms), its multiplies costing
    // about what the FP32 reciprocal does
    constexpr bool kShare = MODEL == MD_GRAV2D && sizeof(T) == 8;
    if (!kShare || (b + 1) * TILE > n)
        sym_tile<MODEL, T, A, SYM, false>(u0, u1, e, lane, TILE / kWave, load, jsum, acc);
    else
        sym_tile<MODEL, T, A, SYM, kShare>(u0, u1, e, lane, TILE / kWave, load, jsum, acc);
#pragma unroll
    for (int k = 0; k < kSymIpl; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) part[(size_t)(D * b + d) * npad + i0 + k * kWave] = (sym_slot_t<A>)acc[d][k].get();
    if constexpr (SYM && JW32) {
        __syncthreads();
        for (int m = threadIdx.x; m < TILE; m += W * kWave) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < W; ++w) t += (double)jw32[w][d][m];
                part[(size_t)(D * a + d) * npad + b * TILE + m] = (sym_slot_t<A>)t;
            }
        }
    }
}

// One launch per force evaluation: the tile pairs a < b in row-major order, then
// the diagonal tiles, the cheaper blocks at the end of the grid, where they fill
// the last round.  Measured against two launches (tile pairs, then diagonal
// tiles), 2D mixed: 7.28 -> 7.24 ms at N = 262,144 and 0.652 -> 0.613 ms at 65,536
// (the diagonal tiles' separate launch was one latency-bound round of T blocks).
template <int MODEL, typename T, typename A, int W>
__global__ __launch_bounds__(W * kWave) void k_sym(const T *__restrict__ r0, const T *__restrict__ r1, int n, int npad,
                                                   int ntile, T e, sym_slot_t<A> *__restrict__ part)
{
    __shared__ SymLds<MODEL == MD_GRAV2D ? 2 : 1, A, W> lds;
    const int t = (int)blockIdx.x, noff = ntile * (ntile - 1) / 2;
    if (t < noff) {
        int a, b;
        sym_tile_pair(t, ntile, a, b);
        sym_block<MODEL, T, A, true, W>(r0, r1, n, npad, e, part, a, b, lds);
    } else {
        sym_block<MODEL, T, A, false, W>(r0, r1, n, npad, e, part, t - noff, t - noff, lds);
    }
}

// The pads (particles n .. npad - 1) hold sym_pad's operands: every operand refresh
// (UPD_PREP in k_update) writes them, so they are in place before any pair launch
// of the same call, also inside a captured graph.
template <int MODEL, typename T, typename A>
hipError_t sym_launch(md_ctx *c)
{
    const int npad = (int)c->npad, tile = sym_tile_n(c->model, c->prec, c->n), ntile = npad / tile;
    const T *ops = static_cast<const T *>(c->ops);
    const T e = MODEL == MD_GRAV2D ? (T)c->eps : sizeof(T) == 4 ? (T)(2.0 * c->eps) : (T)(1.0 + c->eps);
    const int nblk = ntile * (ntile - 1) / 2 + ntile;  // tile pairs, then diagonal tiles
    sym_slot_t<A> *slots = reinterpret_cast<sym_slot_t<A> *>(c->part);
    const int ts = timed_begin(c, MODEL == MD_GRAV2D ? "k_sym (2D)" : "k_sym (Ring)");
    if (tile == kSymTile)
        hipLaunchKernelGGL((k_sym<MODEL, T, A, 4>), dim3((unsigned)nblk), dim3(4 * kWave), 0, c->stream, ops,
                           ops + npad, (int)c->n, npad, ntile, e, slots);
    else if (tile == kSymTileSmall)
        hipLaunchKernelGGL((k_sym<MODEL, T, A, 2>), dim3((unsigned)nblk), dim3(2 * kWave), 0, c->stream, ops,
                           ops + npad, (int)c->n, npad, ntile, e, slots);
    else
        hipLaunchKernelGGL((k_sym<MODEL, T, A, 1>), dim3((unsigned)nblk), dim3(kWave), 0, c->stream, ops,
                           ops + npad, (int)c->n, npad, ntile, e, slots);
    const hipError_t err = hipGetLastError();
    timed_end(c, ts);
    return err;
}

// --------------------------------------------------------------- update kernel --

// Operand refresh after a drift.  COPY64: an FP64 copy of q (2D FP64 operands of
// the fused stage, which cannot read q while other blocks drift it).
enum Prep { PREP_NONE = 0, PREP_CAST32 = 1, PREP_HALF32 = 2, PREP_SINCOS64 = 3, PREP_COPY64 = 4 };

// Which of q, p a stage reads.
__host__ __device__ constexpr bool stage_reads_q(int flags) { return flags & (UPD_DRIFT | UPD_PREP); }
__host__ __device__ constexpr bool stage_reads_p(int flags) { return flags & (UPD_KICK1 | UPD_KICK2 | UPD_DRIFT); }

// The stage's work on coordinate d of particle i, given its force component fd
// and its current q, p (read by the caller when the flags need them): store f,
// p += kick * f, q += drift * p, then the pair operands of the new q.
template <int PREP>
__device__ __forceinline__ void stage_elem_v(int d, int i, int n, int npad, double fd, double qd, double pd,
                                             int flags, double *__restrict__ f, double *__restrict__ p,
                                             double *__restrict__ q, void *__restrict__ ops, double kick1,
                                             double kick2, double drift, double *__restrict__ snap)
{
    const size_t k = (size_t)d * n + i;
    if (flags & UPD_STORE_F) f[k] = fd;
    if (stage_reads_p(flags)) {
        if (flags & UPD_KICK1) pd += kick1 * fd;
        if (flags & UPD_KICK2) pd += kick2 * fd;
        if (flags & (UPD_KICK1 | UPD_KICK2)) p[k] = pd;
        if (flags & UPD_DRIFT) {
            qd += drift * pd;
            q[k] = qd;
            if (snap) snap[k] = qd;
        }
    }
    if (flags & UPD_PREP) {
        if (PREP == PREP_CAST32) {
            static_cast<float *>(ops)[(size_t)d * npad + i] = (float)qd;
        } else if (PREP == PREP_COPY64) {
            static_cast<double *>(ops)[(size_t)d * npad + i] = qd;
        } else if (PREP == PREP_HALF32) {
            double sn, cn;
            sincos64(0.5 * qd, &sn, &cn);
            static_cast<float *>(ops)[i] = (float)(1.4142135623730951 * cn);
            static_cast<float *>(ops)[npad + i] = (float)(1.4142135623730951 * sn);
        } else if (PREP == PREP_SINCOS64) {
            double sn, cn;
            sincos64(qd, &sn, &cn);
            static_cast<double *>(ops)[i] = cn;
            static_cast<double *>(ops)[npad + i] = sn;
        }
    }
}

template <int PREP>
__device__ __forceinline__ void stage_elem(int d, int i, int n, int npad, double fd, int flags,
                                           double *__restrict__ f, double *__restrict__ p, double *__restrict__ q,
                                           void *__restrict__ ops, double kick1, double kick2, double drift,
                                           double *__restrict__ snap)
{
    const size_t k = (size_t)d * n + i;
    const double qd = stage_reads_q(flags) ? q[k] : 0.0;
    const double pd = stage_reads_p(flags) ? p[k] : 0.0;
    stage_elem_v<PREP>(d, i, n, npad, fd, qd, pd, flags, f, p, q, ops, kick1, kick2, drift, snap);
}

// One kick-drift stage, elementwise over particles (eq. 4 and the step list of
// Sec. 3): f from the pair partials (times the model prefactor), p += kick * f,
// q += drift * p, then the pair operands of the new q.
// The pad operand of particle i in [n, npad) (the symmetric form's padding; the
// other forms never read past n).
template <int PREP>
__device__ __forceinline__ void stage_pad(int i, int npad, void *__restrict__ ops)
{
    if (PREP == PREP_CAST32) {
        static_cast<float *>(ops)[i] = static_cast<float *>(ops)[npad + i] = sym_pad<MD_GRAV2D, float>();
    } else if (PREP == PREP_COPY64) {
        static_cast<double *>(ops)[i] = static_cast<double *>(ops)[npad + i] = sym_pad<MD_GRAV2D, double>();
    } else if (PREP == PREP_HALF32) {
        static_cast<float *>(ops)[i] = static_cast<float *>(ops)[npad + i] = sym_pad<MD_RING, float>();
    } else if (PREP == PREP_SINCOS64) {
        static_cast<double *>(ops)[i] = static_cast<double *>(ops)[npad + i] = sym_pad<MD_RING, double>();
    }
}

// part: the pair partials, S slots [S][D][npad] of SlotT (FP32 for the symmetric
// form's MD_MIXED slots, else FP64).
template <int D, int PREP, typename SlotT>
__global__ __launch_bounds__(256) void k_update(const SlotT *__restrict__ part, int S, int n, int npad,
                                                double pref, double *__restrict__ f,
                                                double *__restrict__ p, double *__restrict__ q,
                                                void *__restrict__ ops, double kick1, double kick2,
                                                double drift, int flags, double *__restrict__ snap)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) {  // with UPD_PREP the grid covers the pads too
        if ((flags & UPD_PREP) && i < npad) stage_pad<PREP>(i, npad, ops);
        return;
    }
    double fs[D];
    if (flags & UPD_F_FROM_PART) slot_sums<D, SlotT>(part, S, npad, i, fs);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double fd = 0.0;
        if (flags & UPD_F_FROM_PART) {
            fd = pref * fs[d];
        } else if (flags & (UPD_KICK1 | UPD_KICK2 | UPD_STORE_F)) {
            fd = f[(size_t)d * n + i];
        }
        stage_elem<PREP>(d, i, n, npad, fd, flags, f, p, q, ops, kick1, kick2, drift, snap);
    }
}

// k_update for VW consecutive particles per thread (the symmetric form's slots,
// large n): each slot row is read with one 16-byte load per lane (float4 of FP32
// slots, double2 of FP64 ones) instead of VW 4- or 8-byte ones, the slots of each
// particle still added in the order of slot_sums (device.h), so the sums are
// those of k_update bit for bit.  Measured on the 2D slot sum at N = 262,144 (256 FP32 slots a coordinate):
// 102 -> 93 us.  The grid covers (UPD_PREP ? npad : n) / VW threads; npad is a
// multiple of 1024, so every load of a thread's VW particles is in the slots.
template <typename SlotT, int VW>
struct SlotVec;
template <>
struct SlotVec<float, 4> {
    using T = float4;
};
template <>
struct SlotVec<double, 2> {
    using T = double2;
};

template <int D, int PREP, typename SlotT, int VW>
__global__ __launch_bounds__(64) void k_update_vec(const SlotT *__restrict__ part, int S, int n, int npad,
                                                   double pref, double *__restrict__ f, double *__restrict__ p,
                                                   double *__restrict__ q, void *__restrict__ ops, double kick1,
                                                   double kick2, double drift, int flags, double *__restrict__ snap)
{
    using V = typename SlotVec<SlotT, VW>::T;
    constexpr int U = kSlotBlock;
    const int i0 = VW * (blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= npad) return;
    double fs[VW][D];
#pragma unroll
    for (int k = 0; k < VW; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) fs[k][d] = 0.0;
    // q and p of the thread's particles go out before the slot loads: their
    // latency then hides under the slot sum instead of following it
    double qv[VW][D], pv[VW][D];
#pragma unroll
    for (int k = 0; k < VW; ++k)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int i = i0 + k;
            const size_t e = (size_t)d * n + i;
            qv[k][d] = (i < n && stage_reads_q(flags)) ? q[e] : 0.0;
            pv[k][d] = (i < n && stage_reads_p(flags)) ? p[e] : 0.0;
        }
    if (flags & UPD_F_FROM_PART) {  // the slot order of slot_sums (device.h)
        int b = 0;
        for (; b + U <= S; b += U) {
            V v[D][U];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int d = 0; d < D; ++d)
                    v[d][u] = *reinterpret_cast<const V *>(part + (size_t)((b + u) * D + d) * npad + i0);
#pragma unroll
            for (int d = 0; d < D; ++d)
#pragma unroll
                for (int k = 0; k < VW; ++k) {
                    SlotT e[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) e[u] = reinterpret_cast<const SlotT *>(&v[d][u])[k];
                    fs[k][d] += tree8(e);
                }
        }
        for (; b < S; ++b)
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const V v = *reinterpret_cast<const V *>(part + (size_t)(b * D + d) * npad + i0);
                const SlotT *e = reinterpret_cast<const SlotT *>(&v);
#pragma unroll
                for (int k = 0; k < VW; ++k) fs[k][d] += (double)e[k];
            }
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        const int i = i0 + k;
        if (i >= n) {  // with UPD_PREP the grid covers the pads too
            if (flags & UPD_PREP) stage_pad<PREP>(i, npad, ops);
            continue;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double fd = 0.0;
            if (flags & UPD_F_FROM_PART) {
                fd = pref * fs[k][d];
            } else if (flags & (UPD_KICK1 | UPD_KICK2 | UPD_STORE_F)) {
                fd = f[(size_t)d * n + i];
            }
            stage_elem_v<PREP>(d, i, n, npad, fd, qv[k][d], pv[k][d], flags, f, p, q, ops, kick1, kick2, drift,
                               snap);
        }
    }
}

// ------------------------------------------------------------- fused stage --

// Makes a wavefront's LDS writes visible to all its lanes' later reads.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Small N: one launch per force evaluation.  A block owns an i tile and all of
// its j ranges: S wavefronts, each split into L lane groups of 64 / L lanes; lane
// (group g, slot il) of wavefront w holds the IPL particles i0 + il + k 64/L and
// sums the pair terms of j range b = w L + g (the staged path's range b: same
// jlen, j ascending, folds every jtile j from the range start).  The j operands
// stream through a private LDS window per wavefront (coalesced vector loads, one
// round trip per window, then reads broadcast within each group; at small N too
// few wavefronts share a SIMD to hide the latency of the pair kernels'
// wave-uniform scalar loads).  The window's slice then holds the wavefront's
// partials; the block adds the S L partials of each particle in the staged
// order and runs the stage on its own particles: bit for bit the staged pair +
// update launches.  The j operands come from `in`; the refreshed ones go to
// `out` (another buffer: other blocks still read `in`), so the two alternate.
template <int MODEL, typename T, typename A, int IPL, int PREP, int L>
__global__ __launch_bounds__(1024) void k_fused(const T *__restrict__ in, void *__restrict__ out, int n, int npad,
                                                int jlen, int jtile, T e, double pref, double *__restrict__ f,
                                                double *__restrict__ p, double *__restrict__ q, double kick1,
                                                double kick2, double drift, int flags, double *__restrict__ snap)
{
    constexpr int D = MODEL == MD_GRAV2D ? 2 : 1;
    constexpr int IL = kWave / L;          // i slots per lane group
    constexpr int PAD = L > 1 ? 1 : 0;     // group windows one element apart: no LDS bank conflicts
    extern __shared__ double lds[];
    const int S = blockDim.x / kWave;
    const int slice_bytes = kFusedLdsBytes / S;
    const int CHL = ((slice_bytes / (2 * (int)sizeof(T) * L)) - PAD) / 16 * 16;  // j per group per window
    const int WS = CHL + PAD;              // window row stride per group
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int g = lane / IL, il = lane % IL;
    char *slice = reinterpret_cast<char *>(lds) + (size_t)w * slice_bytes;
    T *win = reinterpret_cast<T *>(slice);  // [2][L][WS]
    const int i0 = blockIdx.x * (IL * IPL);
    const int b = w * L + g;
    const int j0 = b * jlen;
    const int len = max(0, min(n - j0, jlen));                 // this lane's range length
    const int wlen = max(0, min(n - w * L * jlen, jlen));      // the wavefront's longest (its group 0)
    const T *__restrict__ r0 = in;
    const T *__restrict__ r1 = in + npad;
    T a0[IPL], a1[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(i0 + IL * k + il, n - 1);
        a0[k] = r0[i];
        a1[k] = r1[i];
    }
    // The stage's own q, p, fetched now so that their latency hides under the pair
    // loop (the block owns these particles: nothing else writes them meanwhile).
    const bool one_pass = IPL * D * IL <= (int)blockDim.x;
    double q_pre = 0.0, p_pre = 0.0;
    if (one_pass && (int)threadIdx.x < IPL * D * IL) {
        const int it = threadIdx.x, s2 = it % IL, kd = it / IL;
        const int i = i0 + IL * (kd / D) + s2;
        if (i < n) {
            const size_t kk = (size_t)(kd % D) * n + i;
            if (stage_reads_q(flags)) q_pre = q[kk];
            if (stage_reads_p(flags)) p_pre = p[kk];
        }
    }
    A acc0[IPL], acc1[IPL];
    auto term = [&](T x, T y) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            if constexpr (MODEL == MD_GRAV2D) pair_2d(a0[k], a1[k], x, y, e, acc0[k], acc1[k]);
            else ring_term(a0[k], a1[k], x, y, e, acc0[k]);
        }
    };
    // 2D FP64: the j in fours from the start of each jtile, then a last two and a
    // last one, as the staged kernel (grav_j_range)
    constexpr bool SHARE = MODEL == MD_GRAV2D && kPairShare<T>;
    auto term4 = [&](const T *x, const T *y) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) pair_2d_four(a0[k], a1[k], x, y, e, acc0[k], acc1[k]);
    };
    auto term2 = [&](T xa, T ya, T xb, T yb) {
#pragma unroll
        for (int k = 0; k < IPL; ++k) pair_2d_two(a0[k], a1[k], xa, ya, xb, yb, e, acc0[k], acc1[k]);
    };
    for (int t = 0; t < wlen; t += 16) {
        const int off = t % CHL;
        if (off == 0) {
            wave_sync();  // the previous window's reads are done
            // The window's cnt j per group (none past the wavefront's longest range):
            // FB 64-j columns of every group are loaded (addresses clamped in
            // bounds) before the first LDS write, so a window of up to FB * 64 j per
            // group costs one memory round trip.  Measured at N = 2048 (Ring), from
            // the kernel's start to the first window in LDS, against one load and
            // its LDS write per loop trip: 2.2 -> 1.9 us (FP64), 3.3 -> 1.6 us (FP32,
            // whose windows are twice as long); a step 23.7 -> 22.7 us (FP64) and
            // 24.1 -> 17.7 us (mixed).
            constexpr int FB = 8 / L;
            const int cnt = min(CHL, wlen - t);
            for (int e0 = 0; e0 < cnt; e0 += FB * kWave) {
                T x0[FB][L], x1[FB][L];
#pragma unroll
                for (int m = 0; m < FB; ++m)
#pragma unroll
                    for (int gg = 0; gg < L; ++gg) {
                        const int ee = e0 + m * kWave + lane;
                        const int j = (w * L + gg) * jlen + t + ee;
                        const int jc = ee < cnt && j < n ? j : 0;
                        x0[m][gg] = r0[jc];
                        x1[m][gg] = r1[jc];
                    }
#pragma unroll
                for (int m = 0; m < FB; ++m)
#pragma unroll
                    for (int gg = 0; gg < L; ++gg) {
                        const int ee = e0 + m * kWave + lane;
                        const int j = (w * L + gg) * jlen + t + ee;
                        if (ee < cnt && j < n) {
                            win[gg * WS + ee] = x0[m][gg];
                            win[(L + gg) * WS + ee] = x1[m][gg];
                        }
                    }
            }
            wave_sync();
        }
        const T *w0 = win + g * WS + off;
        const T *w1 = win + (L + g) * WS + off;
        if (t + 16 <= len) {
            if constexpr (SHARE) {
#pragma unroll
                for (int u = 0; u < 16; u += 4) {
                    const T xq[4] = {w0[u], w0[u + 1], w0[u + 2], w0[u + 3]};
                    const T yq[4] = {w1[u], w1[u + 1], w1[u + 2], w1[u + 3]};
                    term4(xq, yq);
                }
            } else {
#pragma unroll
                for (int u = 0; u < 16; ++u) term(w0[u], w1[u]);
            }
        } else {
            int u = 0;
            if constexpr (SHARE) {
                for (; u + 4 <= len - t; u += 4) {
                    const T xq[4] = {w0[u], w0[u + 1], w0[u + 2], w0[u + 3]};
                    const T yq[4] = {w1[u], w1[u + 1], w1[u + 2], w1[u + 3]};
                    term4(xq, yq);
                }
                if (u + 2 <= len - t) {
                    term2(w0[u], w1[u], w0[u + 1], w1[u + 1]);
                    u += 2;
                }
            }
            for (; u < len - t; ++u) term(w0[u], w1[u]);
        }
        if (t < len && ((t + 16) % jtile == 0 || t + 16 >= len)) {
#pragma unroll
            for (int k = 0; k < IPL; ++k) {
                acc0[k].fold();
                if constexpr (MODEL == MD_GRAV2D) acc1[k].fold();
            }
        }
    }
    wave_sync();  // window reads done before the slice takes the partials
    double *part = reinterpret_cast<double *>(slice);  // [L][IPL * D][IL]
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        part[(g * IPL * D + k * D) * IL + il] = acc0[k].get();
        if constexpr (MODEL == MD_GRAV2D) part[(g * IPL * D + k * D + 1) * IL + il] = acc1[k].get();
    }
    __syncthreads();
    // The partials of range bb (of S L) for coordinate kd of i slot s2 (the order of
    // slot_sums in device.h, range 0 first).  First the blocks of kSlotBlock ranges,
    // a thread per block: its tree sum replaces the block's first partial (each
    // partial is read by one thread only); then a thread per particle adds them.
    auto fpart = [&](int bb, int kd, int s2) {
        return reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + (size_t)(bb / L) * slice_bytes) +
               ((bb % L) * IPL * D + kd) * IL + s2;
    };
    const int nblk = S * L / kSlotBlock;
    if (flags & UPD_F_FROM_PART) {
        // wavefront k takes block k (and k + S, ...), its lanes the particles: with 8
        // lane groups the block is one wavefront's slice, and the lanes of each LDS
        // read take consecutive words
        for (int k = w; k < nblk; k += S) {
            for (int it = lane; it < IPL * D * IL; it += kWave) {
                const int bb = k * kSlotBlock, s2 = it % IL, kd = it / IL;
                double v[kSlotBlock];
#pragma unroll
                for (int u = 0; u < kSlotBlock; ++u) v[u] = *fpart(bb + u, kd, s2);
                *fpart(bb, kd, s2) = tree8(v);
            }
        }
        __syncthreads();
    }
    for (int it = threadIdx.x; it < IPL * D * IL; it += blockDim.x) {
        const int s2 = it % IL, kd = it / IL;
        const int k = kd / D, d = kd % D;
        const int i = i0 + IL * k + s2;
        if (i < n) {
            double fd = 0.0;
            if (flags & UPD_F_FROM_PART) {  // the block sums above, then the rest
                constexpr int kMaxBlk = kFusedMaxWaves * 8 / kSlotBlock;  // S <= 16 wavefronts, L <= 8
                double bs[kMaxBlk];
#pragma unroll
                for (int k = 0; k < kMaxBlk; ++k) bs[k] = k < nblk ? *fpart(k * kSlotBlock, kd, s2) : 0.0;
                double sum = 0.0;
#pragma unroll
                for (int k = 0; k < kMaxBlk; ++k)
                    if (k < nblk) sum += bs[k];
                for (int bb = nblk * kSlotBlock; bb < S * L; ++bb) sum += *fpart(bb, kd, s2);
                fd = pref * sum;
            } else if (flags & (UPD_KICK1 | UPD_KICK2 | UPD_STORE_F)) {
                fd = f[(size_t)d * n + i];
            }
            if (one_pass)
                stage_elem_v<PREP>(d, i, n, npad, fd, q_pre, p_pre, flags, f, p, q, out, kick1, kick2, drift, snap);
            else
                stage_elem<PREP>(d, i, n, npad, fd, flags, f, p, q, out, kick1, kick2, drift, snap);
        }
    }
}

// ------------------------------------------------------------------ launchers --

int prep_kind(const md_ctx *c, bool fused)
{
    if (c->model == MD_GRAV2D) {
        if (c->prec != MD_FP64) return PREP_CAST32;
        // FP64: the fused stage and the symmetric form read a padded copy; the staged kernel reads q
        return fused || launch_form(c) == MD_LAUNCH_SYMMETRIC ? PREP_COPY64 : PREP_NONE;
    }
    return c->prec == MD_FP64 ? PREP_SINCOS64 : PREP_HALF32;
}

// ops: where UPD_PREP writes the operands (c->ops for the staged path).
hipError_t update(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                  double *f, double *snap, void *ops, bool fused)
{
    const int n = (int)c->n;
    const double pref = force_prefactor(c->model, c->prec, n);
    const bool sym = !fused && launch_form(c) == MD_LAUNCH_SYMMETRIC;
    const int S = sym ? (int)(c->npad / sym_tile_n(c->model, c->prec, c->n)) : c->tiles.jsplit;
    const bool slots32 = sym && c->prec == MD_MIXED;  // the symmetric form's FP32 slots (sym_slot_t)
    const int npad = (int)c->npad;
    const int pk = prep_kind(c, fused);
    if (pk == PREP_NONE) flags &= ~UPD_PREP;
    const int nthreads = (flags & UPD_PREP) ? npad : n;  // an operand refresh also writes the pads
    const dim3 block(256), grid((unsigned)((nthreads + 255) / 256));
    // the symmetric form's slot sums with 16-byte loads where VW particles a thread
    // still leave at least 1024 blocks of one wavefront
    const int vw = slots32 ? 4 : 2;
    const bool vec = sym && (flags & UPD_F_FROM_PART) && npad / vw / kWave >= 1024;
    const dim3 vblock(kWave), vgrid((unsigned)((nthreads + vw * kWave - 1) / (vw * kWave)));
#define MD_UPD(D_, P_)                                                                                              \
    do {                                                                                                            \
        if (vec && slots32)                                                                                         \
            hipLaunchKernelGGL((k_update_vec<D_, P_, float, 4>), vgrid, vblock, 0, c->stream,                       \
                               reinterpret_cast<const float *>(c->part), S, n, npad, pref, f, p, q, ops, kick1, kick2, \
                               drift, flags, snap);                                                                 \
        else if (vec)                                                                                               \
            hipLaunchKernelGGL((k_update_vec<D_, P_, double, 2>), vgrid, vblock, 0, c->stream, c->part, S, n, npad, \
                               pref, f, p, q, ops, kick1, kick2, drift, flags, snap);                               \
        else if (slots32)                                                                                           \
            hipLaunchKernelGGL((k_update<D_, P_, float>), grid, block, 0, c->stream,                                \
                               reinterpret_cast<const float *>(c->part), S, n, npad, pref, f, p, q, ops, kick1, kick2, \
                               drift, flags, snap);                                                                 \
        else                                                                                                        \
            hipLaunchKernelGGL((k_update<D_, P_, double>), grid, block, 0, c->stream, c->part, S, n, npad, pref, f, \
                               p, q, ops, kick1, kick2, drift, flags, snap);                                        \
    } while (0)
    if (c->model == MD_GRAV2D) {
        if (pk == PREP_CAST32) MD_UPD(2, PREP_CAST32);
        else if (pk == PREP_COPY64) MD_UPD(2, PREP_COPY64);
        else MD_UPD(2, PREP_NONE);
    } else {
        if (pk == PREP_HALF32) MD_UPD(1, PREP_HALF32);
        else MD_UPD(1, PREP_SINCOS64);
    }
#undef MD_UPD
    return hipGetLastError();
}

template <int MODEL, typename T, typename A, int PREP>
hipError_t fused_ipl(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                     double *f, const void *in, void *out, double *snap, T e)
{
    const Tiles &t = c->tiles;
    const int n = (int)c->n, npad = (int)c->npad, js = t.jsplit;
    const int L = fused_groups(js), S = js / L;
    int jlen = (n + js - 1) / js;
    jlen = (jlen + 15) / 16 * 16;
    const double pref = force_prefactor(c->model, c->prec, n);
    const int itile = kWave / L * t.ipl;
    const dim3 block((unsigned)(kWave * S));
    const dim3 grid((unsigned)((n + itile - 1) / itile));
    const size_t lds = (size_t)(kFusedLdsBytes / S) * S;
    const T *src = static_cast<const T *>(in);
#define MD_FUSED(I_, L_)                                                                                              \
    hipLaunchKernelGGL((k_fused<MODEL, T, A, I_, PREP, L_>), grid, block, lds, c->stream, src, out, n, npad, jlen, \
                       t.jtile, e, pref, f, p, q, kick1, kick2, drift, flags, snap)
#define MD_FUSED_L(I_)                          \
    switch (L) {                                \
    case 1: MD_FUSED(I_, 1); break;             \
    case 2: MD_FUSED(I_, 2); break;             \
    case 4: MD_FUSED(I_, 4); break;             \
    default: MD_FUSED(I_, 8); break;            \
    }
    const int ts = timed_begin(c, "k_fused");
    switch (t.ipl) {
    case 1: MD_FUSED_L(1); break;
    case 2: MD_FUSED_L(2); break;
    default: MD_FUSED_L(4); break;
    }
#undef MD_FUSED_L
#undef MD_FUSED
    const hipError_t err = hipGetLastError();
    timed_end(c, ts);
    return err;
}

template <typename T, typename A>
hipError_t pair_ipl(md_ctx *c, const void *src, dim3 grid, dim3 block, int jlen)
{
    const int n = (int)c->n, npad = (int)c->npad, jt = c->tiles.jtile;
    const int ts = timed_begin(c, c->model == MD_GRAV2D ? "k_pair_2d" : sizeof(T) == 4 ? "k_pair_win" : "k_pair_ring");
    if (c->model == MD_GRAV2D) {
        const T *x = static_cast<const T *>(src);
        const T *y = x + (src == c->ops ? npad : n);
        const T eps = (T)c->eps;
        switch (c->tiles.ipl) {
        case 1: hipLaunchKernelGGL((k_pair_2d<T, A, 1>), grid, block, 0, c->stream, x, y, n, npad, jlen, jt, eps, c->part); break;
        case 2: hipLaunchKernelGGL((k_pair_2d<T, A, 2>), grid, block, 0, c->stream, x, y, n, npad, jlen, jt, eps, c->part); break;
        default: hipLaunchKernelGGL((k_pair_2d<T, A, 4>), grid, block, 0, c->stream, x, y, n, npad, jlen, jt, eps, c->part); break;
        }
    } else if constexpr (sizeof(T) == 4) {
        // Ring FP32 forms: the LDS-window kernel
        const T *r0 = static_cast<const T *>(src);
        const T e = (T)(2.0 * c->eps);  // half-angle form: 2 eps
#define MD_WIN(I_)                                                                                                 \
    hipLaunchKernelGGL((k_pair_win<MD_RING, T, A, I_>), grid, block, 0, c->stream, r0, r0 + npad, n, npad, jlen, jt, \
                       e, c->part)
        switch (c->tiles.ipl) {
        case 1: MD_WIN(1); break;
        case 2: MD_WIN(2); break;
        default: MD_WIN(4); break;
        }
#undef MD_WIN
    } else {
        const T *cs = static_cast<const T *>(src);
        const T one_eps = (T)(1.0 + c->eps);
        switch (c->tiles.ipl) {
        case 1: hipLaunchKernelGGL((k_pair_ring<T, A, 1>), grid, block, 0, c->stream, cs, n, npad, jlen, jt, one_eps, c->part); break;
        case 2: hipLaunchKernelGGL((k_pair_ring<T, A, 2>), grid, block, 0, c->stream, cs, n, npad, jlen, jt, one_eps, c->part); break;
        default: hipLaunchKernelGGL((k_pair_ring<T, A, 4>), grid, block, 0, c->stream, cs, n, npad, jlen, jt, one_eps, c->part); break;
        }
    }
    const hipError_t err = hipGetLastError();
    timed_end(c, ts);
    return err;
}

}  // namespace

hipError_t launch_update(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                         double *f, double *snap)
{
    return update(c, flags, kick1, kick2, drift, q, p, f, snap, c->ops, false);
}

hipError_t launch_update_fused(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                               double *f, void *ops, double *snap)
{
    return update(c, flags, kick1, kick2, drift, q, p, f, snap, ops, true);
}

hipError_t launch_fused(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                        double *f, const void *in, void *out, double *snap)
{
    const double eps = c->eps;
    if (c->model == MD_GRAV2D) {
        switch (c->prec) {
        case MD_FP64:
            return fused_ipl<MD_GRAV2D, double, AccF64, PREP_COPY64>(c, flags, kick1, kick2, drift, q, p, f, in, out,
                                                                     snap, eps);
        case MD_MIXED:
            return fused_ipl<MD_GRAV2D, float, AccTile, PREP_CAST32>(c, flags, kick1, kick2, drift, q, p, f, in, out,
                                                                     snap, (float)eps);
        case MD_MIXED_KAHAN:
            return fused_ipl<MD_GRAV2D, float, AccKahan, PREP_CAST32>(c, flags, kick1, kick2, drift, q, p, f, in,
                                                                      out, snap, (float)eps);
        default:
            return fused_ipl<MD_GRAV2D, float, AccPair64, PREP_CAST32>(c, flags, kick1, kick2, drift, q, p, f, in,
                                                                       out, snap, (float)eps);
        }
    }
    switch (c->prec) {
    case MD_FP64:
        return fused_ipl<MD_RING, double, AccF64, PREP_SINCOS64>(c, flags, kick1, kick2, drift, q, p, f, in, out,
                                                                 snap, 1.0 + eps);
    case MD_MIXED:
        return fused_ipl<MD_RING, float, AccTile, PREP_HALF32>(c, flags, kick1, kick2, drift, q, p, f, in, out, snap,
                                                               (float)(2.0 * eps));
    case MD_MIXED_KAHAN:
        return fused_ipl<MD_RING, float, AccKahan, PREP_HALF32>(c, flags, kick1, kick2, drift, q, p, f, in, out,
                                                                snap, (float)(2.0 * eps));
    default:
        return fused_ipl<MD_RING, float, AccPair64, PREP_HALF32>(c, flags, kick1, kick2, drift, q, p, f, in, out,
                                                                 snap, (float)(2.0 * eps));
    }
}

// Pair partials of the current operands.  For FP64 2D the operands are q itself.
hipError_t launch_pair(md_ctx *c, const double *q)
{
    if (launch_form(c) == MD_LAUNCH_SYMMETRIC) {
        if (c->model == MD_GRAV2D) {
            switch (c->prec) {
            case MD_FP64: return sym_launch<MD_GRAV2D, double, AccF64>(c);
            case MD_MIXED: return sym_launch<MD_GRAV2D, float, AccTile>(c);
            case MD_MIXED_KAHAN: return sym_launch<MD_GRAV2D, float, AccKahan>(c);
            default: return sym_launch<MD_GRAV2D, float, AccPair64>(c);
            }
        }
        switch (c->prec) {
        case MD_FP64: return sym_launch<MD_RING, double, AccF64>(c);
        case MD_MIXED: return sym_launch<MD_RING, float, AccTile>(c);
        case MD_MIXED_KAHAN: return sym_launch<MD_RING, float, AccKahan>(c);
        default: return sym_launch<MD_RING, float, AccPair64>(c);
        }
    }
    const Tiles &t = c->tiles;
    const int n = (int)c->n;
    const int per_block = kWave * t.ipl * t.waves;
    const dim3 block((unsigned)(kWave * t.waves));
    const dim3 grid((unsigned)((n + per_block - 1) / per_block), (unsigned)t.jsplit);
    int jlen = (n + t.jsplit - 1) / t.jsplit;
    jlen = (jlen + 15) / 16 * 16;
    const void *src = (c->model == MD_GRAV2D && c->prec == MD_FP64) ? (const void *)q : (const void *)c->ops;
    switch (c->prec) {
    case MD_FP64: return pair_ipl<double, AccF64>(c, src, grid, block, jlen);
    case MD_MIXED: return pair_ipl<float, AccTile>(c, src, grid, block, jlen);
    case MD_MIXED_KAHAN: return pair_ipl<float, AccKahan>(c, src, grid, block, jlen);
    default: return pair_ipl<float, AccPair64>(c, src, grid, block, jlen);
    }
}

}  // namespace md
