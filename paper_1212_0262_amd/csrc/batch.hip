// batch.hip -- many independent systems of uneven size advanced together: an
// ensemble of realizations of one model (each with its own N_b and eps_b), as
// used for ensemble averages of quasi-stationary states.  Every realization is
// exactly the single-system computation of pair.hip (the same pair terms and
// accumulators from pair_terms.h); batching only changes how the work is
// scheduled.
//
// Layout: the realizations are concatenated, [d][ntot] FP64 structure of arrays
// with CSR offsets off[b] .. off[b+1].
//
// Scheduling (staged form): one launch per stage for the whole ensemble.  The host cuts every
// realization into (i-block, j-chunk) work items -- an i-block of
// 64 * i_per_lane * waves particles against a j-chunk of one realization's own
// particles -- and sorts them by cost, largest first, so that the 260x spread of
// N_b^2 does not leave a tail.  Each item writes its own slot of the partial
// buffer; the update kernel adds a particle's slots in chunk order, so results
// do not depend on the schedule (bitwise reproducible).  The symmetric form
// (k_batch_sym) instead takes tile pairs within each realization, each pair of
// particles evaluated once.
#include "device.h"
#include "md_internal.h"
#include "pair_terms.h"

namespace md {
namespace {

using namespace pairs;

// Pair work item: a = (b, i0, i1, slot), c = (j0, j1, 0, 0); global indices.
struct alignas(32) PairItem {
    int b, i0, i1, slot, j0, j1, slot_j, pad;  // slot_j: the symmetric form's j-side slot
};

template <typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_batch_pair_2d(const PairItem *__restrict__ items,
                                                       const T *__restrict__ xs, const T *__restrict__ ys,
                                                       const double *__restrict__ beps, int npad, int jtile,
                                                       double *__restrict__ part)
{
    const PairItem it = items[blockIdx.x];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = it.i0 + wave * (kWave * IPL) + lane;
    const T eps = (T)beps[it.b];
    T xi[IPL], yi[IPL];
    A ax[IPL], ay[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, it.i1 - 1);
        xi[k] = xs[i];
        yi[k] = ys[i];
    }
    grav_j_range<T, A, IPL>(xs, ys, it.j0, it.j1, jtile, eps, xi, yi, ax, ay);
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < it.i1) {
            part[(size_t)(2 * it.slot) * npad + i] = ax[k].get();
            part[(size_t)(2 * it.slot + 1) * npad + i] = ay[k].get();
        }
    }
}


template <typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_batch_pair_ring(const PairItem *__restrict__ items, const T *__restrict__ cs,
                                                         const double *__restrict__ beps, int npad, int jtile,
                                                         double *__restrict__ part)
{
    const PairItem it = items[blockIdx.x];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = it.i0 + wave * (kWave * IPL) + lane;
    const T one_eps = sizeof(T) == 8 ? (T)(1.0 + beps[it.b]) : (T)(2.0 * beps[it.b]);  // FP32 half-angle form: 2 eps
    const T *__restrict__ cc = cs;
    const T *__restrict__ ss = cs + npad;
    T ci[IPL], si[IPL];
    A a[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, it.i1 - 1);
        ci[k] = cc[i];
        si[k] = ss[i];
    }
    for (int jt = it.j0; jt < it.j1; jt += jtile) {
        const int je = min(it.j1, jt + jtile);
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
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < it.i1) part[(size_t)it.slot * npad + i] = a[k].get();
    }
}

enum Prep { PREP_NONE = 0, PREP_CAST32 = 1, PREP_HALF32 = 2, PREP_SINCOS64 = 3 };

// One kick-drift stage for the particles [i0, i1) of realization b (one block per
// row item, up to 256 particles): f = pref_b * (chunk partials added in order),
// kick(s), drift, refresh of the pair operands.  rows[k] = (b, i0, i1, S_b);
// bpref[b] is the realization's force prefactor (1/N_b coupling).
template <int D, int PREP>
__global__ __launch_bounds__(256) void k_batch_update(const int4 *__restrict__ rows,
                                                      const double *__restrict__ bpref,
                                                      const double *__restrict__ part, int npad, int ntot,
                                                      double *__restrict__ f, double *__restrict__ p,
                                                      double *__restrict__ q, void *__restrict__ ops, double kick1,
                                                      double kick2, double drift, int flags)
{
    const int4 r = rows[blockIdx.x];
    const int i = r.y + threadIdx.x;
    if (i >= r.z) return;
    const double pref = bpref[r.x];
    const int S = r.w;
    const bool need_p = flags & (UPD_KICK1 | UPD_KICK2 | UPD_DRIFT);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const size_t k = (size_t)d * ntot + i;
        double fd = 0.0;
        if (flags & UPD_F_FROM_PART) {
            fd = pref * slot_sum<D>(part, S, d, npad, i);
        } else if (flags & (UPD_KICK1 | UPD_KICK2 | UPD_STORE_F)) {
            fd = f[k];
        }
        if (flags & UPD_STORE_F) f[k] = fd;
        double qd = 0.0;
        if (flags & (UPD_DRIFT | UPD_PREP)) qd = q[k];
        if (need_p) {
            double pd = p[k];
            if (flags & UPD_KICK1) pd += kick1 * fd;
            if (flags & UPD_KICK2) pd += kick2 * fd;
            if (flags & (UPD_KICK1 | UPD_KICK2)) p[k] = pd;
            if (flags & UPD_DRIFT) {
                qd += drift * pd;
                q[k] = qd;
            }
        }
        if (flags & UPD_PREP) {
            if (PREP == PREP_CAST32) {
                static_cast<float *>(ops)[(size_t)d * npad + i] = (float)qd;
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
}

// Energy work item (b, i0, i1, j0) + j1: pairs i < j with i in [i0, i1), j in [j0, j1).
template <int MODEL>
__global__ __launch_bounds__(256) void k_batch_energy_pairs(const PairItem *__restrict__ items,
                                                            const double *__restrict__ q,
                                                            const double *__restrict__ beps, int ntot,
                                                            double *__restrict__ red)
{
    __shared__ double lds[4];
    const PairItem it = items[blockIdx.x];
    const int i = it.i0 + threadIdx.x;
    const double eps = beps[it.b];
    double acc = 0.0;
    if (i < it.i1) {
        const int j0 = max(it.j0, i + 1);
        if (MODEL == MD_GRAV2D) {
            const double xi = q[i], yi = q[ntot + i];
            for (int j = j0; j < it.j1; ++j) {
                const double dx = xi - q[j];
                const double dy = yi - q[ntot + j];
                acc += log(dx * dx + dy * dy + eps);
            }
        } else {
            const double ti = q[i];
            for (int j = j0; j < it.j1; ++j) {
                const double h = sin(0.5 * (ti - q[j]));
                acc += 1.0 / sqrt(2.0 * h * h + eps);
            }
        }
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// Per row item: sum of p^2 over its particles (all D rows).
template <int D>
__global__ __launch_bounds__(256) void k_batch_sumsq(const int4 *__restrict__ rows, const double *__restrict__ p,
                                                     int ntot, double *__restrict__ red)
{
    __shared__ double lds[4];
    const int4 r = rows[blockIdx.x];
    const int i = r.y + threadIdx.x;
    double acc = 0.0;
    if (i < r.z) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double v = p[(size_t)d * ntot + i];
            acc += v * v;
        }
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// One block per realization: out[3b..3b+2] = {K, V, K + V} from its item partials
// (energy items eoff[b] .. eoff[b+1], row items roff[b] .. roff[b+1]), fixed order.
__global__ __launch_bounds__(256) void k_batch_energy_finalize(const double *__restrict__ ered,
                                                               const int *__restrict__ eoff,
                                                               const double *__restrict__ kred,
                                                               const int *__restrict__ roff,
                                                               const int64_t *__restrict__ off, int model,
                                                               double *__restrict__ out)
{
    __shared__ double lds[2][4];
    const int b = blockIdx.x;
    double v = 0.0, k2 = 0.0;
    for (int e = eoff[b] + (int)threadIdx.x; e < eoff[b + 1]; e += blockDim.x) v += ered[e];
    for (int r = roff[b] + (int)threadIdx.x; r < roff[b + 1]; r += blockDim.x) k2 += kred[r];
    v = block_sum(v, lds[0]);
    k2 = block_sum(k2, lds[1]);
    if (threadIdx.x == 0) {
        const double n = (double)(off[b + 1] - off[b]);
        const double pot = model == MD_GRAV2D ? v / n : -v / (sqrt(2.0) * n);
        const double kin = 0.5 * k2;
        out[3 * b] = kin;
        out[3 * b + 1] = pot;
        out[3 * b + 2] = kin + pot;
    }
}

// Ring FP32 forms: the work item's j chunk through a block-shared LDS window (see
// window_stream; the same terms in the same order as k_batch_pair_ring).
constexpr int kWinJ = 512;

template <typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_batch_pair_ring_win(const PairItem *__restrict__ items,
                                                             const T *__restrict__ cs,
                                                             const double *__restrict__ beps, int npad, int jtile,
                                                             double *__restrict__ part)
{
    __shared__ T win[2][kWinJ];
    const PairItem it = items[blockIdx.x];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = it.i0 + wave * (kWave * IPL) + lane;
    const T e = (T)(2.0 * beps[it.b]);  // half-angle form: 2 eps
    const T *__restrict__ cc = cs;
    const T *__restrict__ ss = cs + npad;
    T ci[IPL], si[IPL];
    A a[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, it.i1 - 1);
        ci[k] = cc[i];
        si[k] = ss[i];
    }
    window_stream<kWinJ>(
        cc, ss, it.j0, it.j1, jtile, win,
        [&](T cj, T sj) {
#pragma unroll
            for (int k = 0; k < IPL; ++k) ring_term(ci[k], si[k], cj, sj, e, a[k]);
        },
        [&]() {
#pragma unroll
            for (int k = 0; k < IPL; ++k) a[k].fold();
        });
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < it.i1) part[(size_t)it.slot * npad + i] = a[k].get();
    }
}

// Symmetric form (sym_tile in pair_terms.h): a work item is a tile pair
// (a, b), a < b, of one realization, or one of its diagonal tiles (SYM = false).
// it.i0, it.j0: the tiles' first particles; it.i1, it.j1: the realization's end.
// Particles past the end read their realization's last operand and replace it by
// the pad value, whose terms vanish.  The i side goes to slot it.slot of the i
// particles, the j side (the wavefronts' sums added in FP64, fixed order, after
// every 64-j block) to slot it.slot_j of the j particles.
template <int MODEL, typename T, typename A, bool SYM, int W>
__device__ __forceinline__ void batch_sym_item(const PairItem &it, const T *__restrict__ r0,
                                               const T *__restrict__ r1, const double *__restrict__ beps, int npad,
                                               double *__restrict__ part,
                                               double (&jw)[W][MODEL == MD_GRAV2D ? 2 : 1][kWave])
{
    constexpr int D = MODEL == MD_GRAV2D ? 2 : 1;
    constexpr int TILE = W * kWave * kSymIpl;
    const double eb = beps[it.b];
    const T e = MODEL == MD_GRAV2D ? (T)eb : sizeof(T) == 4 ? (T)(2.0 * eb) : (T)(1.0 + eb);
    const T pad = sym_pad<MODEL, T>();
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int ib = it.i0 + wave * kWave * kSymIpl + lane;
    // A diagonal tile's wavefront whose i are all past the realization's end has no
    // work (no barriers without SYM).  The j tile stops after its last 64-j block
    // that holds a particle: the pads' terms are zero.
    if (!SYM && it.i0 + wave * kWave * kSymIpl >= it.i1) return;
    // (j1 is the realization's end: only its last tile is shorter than TILE)
    const int nblk = min(TILE / kWave, (it.j1 - it.j0 + kWave - 1) / kWave);
    T u0[kSymIpl], u1[kSymIpl];
    A acc[D][kSymIpl];
#pragma unroll
    for (int k = 0; k < kSymIpl; ++k) {
        const int i = ib + k * kWave;
        const int ic = min(i, it.i1 - 1);
        u0[k] = i < it.i1 ? r0[ic] : pad;
        u1[k] = i < it.i1 ? r1[ic] : pad;
    }
    sym_tile<MODEL, T, A, SYM>(
        u0, u1, e, lane, nblk,
        [&](int blk, T &v0, T &v1) {
            const int j = it.j0 + blk * kWave + lane;
            const int jc = min(j, it.j1 - 1);
            v0 = j < it.j1 ? r0[jc] : pad;
            v1 = j < it.j1 ? r1[jc] : pad;
        },
        [&](int blk, int m, A (&sj)[D]) {
#pragma unroll
            for (int d = 0; d < D; ++d) jw[wave][d][m] = sj[d].get();
            __syncthreads();
            for (int x = threadIdx.x; x < D * kWave; x += W * kWave) {  // W = 1: a thread per (d, j) in turn
                const int d = x / kWave, mm = x & (kWave - 1);
                const int j = it.j0 + blk * kWave + mm;
                if (j < it.j1) {
                    double t = 0.0;
#pragma unroll
                    for (int w = 0; w < W; ++w) t += jw[w][d][mm];
                    part[(size_t)(D * it.slot_j + d) * npad + j] = t;
                }
            }
            __syncthreads();
        },
        acc);
#pragma unroll
    for (int k = 0; k < kSymIpl; ++k) {
        const int i = ib + k * kWave;
        if (i < it.i1) {
#pragma unroll
            for (int d = 0; d < D; ++d) part[(size_t)(D * it.slot + d) * npad + i] = acc[d][k].get();
        }
    }
}

// One launch per force evaluation: the n_soff tile pairs of the work list (a
// block each), then its diagonal tiles, cheaper, at the end of the grid.
template <int MODEL, typename T, typename A, int W>
__global__ __launch_bounds__(W * kWave) void k_batch_sym(const PairItem *__restrict__ items, int n_soff,
                                                         const T *__restrict__ r0, const T *__restrict__ r1,
                                                         const double *__restrict__ beps, int npad,
                                                         double *__restrict__ part)
{
    __shared__ double jw[W][MODEL == MD_GRAV2D ? 2 : 1][kWave];
    const PairItem it = items[blockIdx.x];
    if ((int)blockIdx.x < n_soff)
        batch_sym_item<MODEL, T, A, true, W>(it, r0, r1, beps, npad, part, jw);
    else
        batch_sym_item<MODEL, T, A, false, W>(it, r0, r1, beps, npad, part, jw);
}

template <int MODEL, typename T, typename A>
hipError_t sym_launch(md_ctx *c)
{
    const Batch &B = *c->batch;
    const T *r0 = static_cast<const T *>(c->ops);
    const int npad = (int)c->npad;
    const PairItem *items = reinterpret_cast<const PairItem *>(B.d_sitems);
    constexpr int W = kBatchSymTile / (kWave * kSymIpl);
    const int ts = timed_begin(c, "k_batch_sym");
    hipLaunchKernelGGL((k_batch_sym<MODEL, T, A, W>), dim3((unsigned)(B.n_soff + B.n_sdiag)), dim3(W * kWave), 0,
                       c->stream, items, B.n_soff, r0, r0 + npad, B.d_eps, npad, c->part);
    const hipError_t err = hipGetLastError();
    timed_end(c, ts);
    return err;
}

int prep_kind(const md_ctx *c)
{
    if (c->model == MD_GRAV2D) return c->prec == MD_FP64 ? PREP_NONE : PREP_CAST32;
    return c->prec == MD_FP64 ? PREP_SINCOS64 : PREP_HALF32;
}

template <typename T, typename A>
hipError_t pair_launch(md_ctx *c, const void *src)
{
    const Batch &B = *c->batch;
    const int npad = (int)c->npad, jt = c->tiles.jtile;
    const dim3 grid((unsigned)B.n_items), block((unsigned)(kWave * c->tiles.waves));
    const PairItem *items = reinterpret_cast<const PairItem *>(B.d_items);
    const int ts = timed_begin(c, c->model == MD_GRAV2D ? "k_batch_pair_2d"
                                  : sizeof(T) == 4     ? "k_batch_pair_ring_win"
                                                       : "k_batch_pair_ring");
    if (c->model == MD_GRAV2D) {
        const T *x = static_cast<const T *>(src);
        const T *y = x + (src == c->ops ? npad : c->n);
        switch (c->tiles.ipl) {
        case 1: hipLaunchKernelGGL((k_batch_pair_2d<T, A, 1>), grid, block, 0, c->stream, items, x, y, B.d_eps, npad, jt, c->part); break;
        case 2: hipLaunchKernelGGL((k_batch_pair_2d<T, A, 2>), grid, block, 0, c->stream, items, x, y, B.d_eps, npad, jt, c->part); break;
        default: hipLaunchKernelGGL((k_batch_pair_2d<T, A, 4>), grid, block, 0, c->stream, items, x, y, B.d_eps, npad, jt, c->part); break;
        }
    } else if constexpr (sizeof(T) == 4) {
        const T *cs = static_cast<const T *>(src);
        switch (c->tiles.ipl) {
        case 1: hipLaunchKernelGGL((k_batch_pair_ring_win<T, A, 1>), grid, block, 0, c->stream, items, cs, B.d_eps, npad, jt, c->part); break;
        case 2: hipLaunchKernelGGL((k_batch_pair_ring_win<T, A, 2>), grid, block, 0, c->stream, items, cs, B.d_eps, npad, jt, c->part); break;
        default: hipLaunchKernelGGL((k_batch_pair_ring_win<T, A, 4>), grid, block, 0, c->stream, items, cs, B.d_eps, npad, jt, c->part); break;
        }
    } else {
        const T *cs = static_cast<const T *>(src);
        switch (c->tiles.ipl) {
        case 1: hipLaunchKernelGGL((k_batch_pair_ring<T, A, 1>), grid, block, 0, c->stream, items, cs, B.d_eps, npad, jt, c->part); break;
        case 2: hipLaunchKernelGGL((k_batch_pair_ring<T, A, 2>), grid, block, 0, c->stream, items, cs, B.d_eps, npad, jt, c->part); break;
        default: hipLaunchKernelGGL((k_batch_pair_ring<T, A, 4>), grid, block, 0, c->stream, items, cs, B.d_eps, npad, jt, c->part); break;
        }
    }
    const hipError_t err = hipGetLastError();
    timed_end(c, ts);
    return err;
}

}  // namespace

hipError_t batch_pair(md_ctx *c, const double *q)
{
    if (launch_form(c) == MD_LAUNCH_SYMMETRIC) {
        if (c->model == MD_GRAV2D)
            return c->prec == MD_MIXED_KAHAN ? sym_launch<MD_GRAV2D, float, AccKahan>(c)
                                             : sym_launch<MD_GRAV2D, float, AccTile>(c);
        if (c->prec == MD_FP64) return sym_launch<MD_RING, double, AccF64>(c);
        return c->prec == MD_MIXED_KAHAN ? sym_launch<MD_RING, float, AccKahan>(c) : sym_launch<MD_RING, float, AccTile>(c);
    }
    const void *src = (c->model == MD_GRAV2D && c->prec == MD_FP64) ? (const void *)q : (const void *)c->ops;
    switch (c->prec) {
    case MD_FP64: return pair_launch<double, AccF64>(c, src);
    case MD_MIXED: return pair_launch<float, AccTile>(c, src);
    case MD_MIXED_KAHAN: return pair_launch<float, AccKahan>(c, src);
    default: return pair_launch<float, AccPair64>(c, src);
    }
}

hipError_t batch_update(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                        double *f)
{
    const Batch &B = *c->batch;
    const int pk = prep_kind(c);
    if (pk == PREP_NONE) flags &= ~UPD_PREP;
    const dim3 grid((unsigned)B.n_rows), block(256);
    // the symmetric form's rows carry S_b = T_b tile slots
    const int4 *rows = reinterpret_cast<const int4 *>(launch_form(c) == MD_LAUNCH_SYMMETRIC ? B.d_srows : B.d_rows);
    const int npad = (int)c->npad, ntot = (int)c->n;
#define MD_BUPD(D_, P_)                                                                                         \
    hipLaunchKernelGGL((k_batch_update<D_, P_>), grid, block, 0, c->stream, rows, B.d_pref, c->part, npad, ntot, \
                       f, p, q, c->ops, kick1, kick2, drift, flags)
    if (c->model == MD_GRAV2D) {
        if (pk == PREP_CAST32) MD_BUPD(2, PREP_CAST32);
        else MD_BUPD(2, PREP_NONE);
    } else {
        if (pk == PREP_HALF32) MD_BUPD(1, PREP_HALF32);
        else MD_BUPD(1, PREP_SINCOS64);
    }
#undef MD_BUPD
    return hipGetLastError();
}

hipError_t batch_energy(md_ctx *c, const double *q, const double *p, double *out)
{
    const Batch &B = *c->batch;
    const int ntot = (int)c->n;
    const PairItem *eitems = reinterpret_cast<const PairItem *>(B.d_eitems);
    const int4 *rows = reinterpret_cast<const int4 *>(B.d_rows);
    if (B.n_eitems > 0) {
        if (c->model == MD_GRAV2D)
            hipLaunchKernelGGL(k_batch_energy_pairs<MD_GRAV2D>, dim3((unsigned)B.n_eitems), dim3(256), 0, c->stream,
                               eitems, q, B.d_eps, ntot, B.d_ered);
        else
            hipLaunchKernelGGL(k_batch_energy_pairs<MD_RING>, dim3((unsigned)B.n_eitems), dim3(256), 0, c->stream,
                               eitems, q, B.d_eps, ntot, B.d_ered);
    }
    if (c->model == MD_GRAV2D)
        hipLaunchKernelGGL(k_batch_sumsq<2>, dim3((unsigned)B.n_rows), dim3(256), 0, c->stream, rows, p, ntot, B.d_kred);
    else
        hipLaunchKernelGGL(k_batch_sumsq<1>, dim3((unsigned)B.n_rows), dim3(256), 0, c->stream, rows, p, ntot, B.d_kred);
    hipLaunchKernelGGL(k_batch_energy_finalize, dim3((unsigned)B.nb), dim3(256), 0, c->stream, B.d_ered, B.d_eoff,
                       B.d_kred, B.d_roff, B.d_off, c->model, out);
    return hipGetLastError();
}

}  // namespace md
