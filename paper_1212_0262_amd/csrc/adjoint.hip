// adjoint.hip -- Hessian-vector products of the pair potentials and the reverse
// sweep of the Yoshida step (eq. 4), for gradients of an observable of the final
// state with respect to the initial state.
//
// For V = sum_{i<j} phi(q_i - q_j) the product is (H w)_i = sum_j phi''(q_i - q_j)
// (w_i - w_j), with
//   2D (eq. 3):   phi''(r) = (2/N) [I/s - 2 r r^T / s^2],  s = |r|^2 + eps
//   Ring (eq. 1): phi''(d) = (1/(2 sqrt2 N)) u^{-3/2} [cos d - (3/2) sin^2 d / u],
//                 u = 1 - cos d + eps, from the cosines and sines of both angles
//                 (FP64) or from their half angles (FP32 forms, as the force)
// computed with the same j-broadcast, i-in-registers, j-split scheme as the force
// (pair.hip), in FP64 or with FP32 pair arithmetic and the same accumulators.
// The self pair contributes exactly zero (w_i - w_i = 0 and, in 2D, r = 0).
//
// Reverse sweep: a drift q += a p is undone by lp += a lq, a kick p += h F(q) by
// lq -= h H(q) lp (F = -grad V).  One fused elementwise kernel combines the
// Hessian-vector partials, applies the kick and the next drift in reverse order,
// and refreshes the operands of the next product.
#include "device.h"
#include "md_internal.h"
#include "pair_terms.h"

namespace md {
namespace {

using namespace pairs;

// 2D: adds (u - 2 r (r.u)/s)/s, u = w_i - w_j, r = r_i - r_j, to (ax, ay), given
// r and inv = 1/s.
template <typename T, typename A>
__device__ __forceinline__ void hvp_2d_add(T dx, T dy, T inv, T wxi, T wyi, T wxj, T wyj, A &ax, A &ay)
{
    const T ux = wxi - wxj, uy = wyi - wyj;
    const T t = fma_(dx, ux, dy * uy) * inv;
    const T c = (t + t) * inv;
    ax.add(inv, ux);
    ax.add(-c, dx);
    ay.add(inv, uy);
    ay.add(-c, dy);
}

template <typename T, typename A>
__device__ __forceinline__ void hvp_2d(T xi, T yi, T wxi, T wyi, T xj, T yj, T wxj, T wyj, T eps, A &ax, A &ay)
{
    const T dx = xi - xj, dy = yi - yj;
    hvp_2d_add(dx, dy, rcp_(fma_(dx, dx, fma_(dy, dy, eps))), wxi, wyi, wxj, wyj, ax, ay);
}

// The terms of four j with one reciprocal, the weights as the force's pair_2d_four
// (pair_terms.h: nine multiplies and one refined FP64 reciprocal in place of four;
// the product of the four |r_i - r_j|^2 + eps stays a normal number for the eps
// md_init takes and particles closer than about 1e38); added in the order of the j.
template <typename T, typename A>
__device__ __forceinline__ void hvp_2d_four(T xi, T yi, T wxi, T wyi, const T *xj, const T *yj, const T *wxj,
                                            const T *wyj, T eps, A &ax, A &ay)
{
    T dx[4], dy[4], s[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dx[k] = xi - xj[k];
        dy[k] = yi - yj[k];
        s[k] = fma_(dx[k], dx[k], fma_(dy[k], dy[k], eps));
    }
    const T p01 = s[0] * s[1], p23 = s[2] * s[3];
    const T r = rcp_(p01 * p23);
    const T r01 = r * p23, r23 = r * p01;
    const T inv[4] = {r01 * s[1], r01 * s[0], r23 * s[3], r23 * s[2]};
#pragma unroll
    for (int k = 0; k < 4; ++k) hvp_2d_add(dx[k], dy[k], inv[k], wxi, wyi, wxj[k], wyj[k], ax, ay);
}

// Ring: adds phi''(d) (w_i - w_j) / pref, d = ti - tj.
// FP64: from (cos t, sin t): u^{-3/2} [cos d - 1.5 sin^2 d / u], u = e - cos d,
//   e = 1 + eps; pref = 1/(2 sqrt2 N).
// FP32: from the half-angle operands sqrt2 (cos(t/2), sin(t/2)) of the force
//   (pair_terms.h): a = 2 sin(d/2), b = 2 cos(d/2), r' = (a^2 + 2 eps)^{-1/2}
//   (e = 2 eps): the same quantity is r'^3 [(1 - a^2/2) - (3/4) a^2 b^2 r'^2] with
//   pref = 1/N.
template <typename T, typename A>
__device__ __forceinline__ void hvp_ring(T ci, T si, T wi, T cj, T sj, T wj, T e, A &acc)
{
    if constexpr (sizeof(T) == 8) {
        const T cd = fma_(ci, cj, si * sj);
        const T sd = fma_(si, cj, -(ci * sj));
        const T r = rsq_(e - cd);
        const T r2 = r * r;
        const T h = r2 * r * fma_(T(-1.5) * sd * sd, r2, cd);
        acc.add(h, wi - wj);
    } else {
        T a;
        {
#pragma clang fp contract(off)
            a = si * cj - ci * sj;
        }
        const T b = fma_(ci, cj, si * sj);
        const T a2 = a * a;
        const T r = rsq_(a2 + e);
        const T r2 = r * r;
        const T h = r2 * r * fma_(T(-0.75) * a2 * b * b, r2, fma_(T(-0.5), a2, T(1)));
        acc.add(h, wi - wj);
    }
}

template <typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_hvp_2d(const T *__restrict__ xs, const T *__restrict__ ys,
                                                const T *__restrict__ wxs, const T *__restrict__ wys, int n,
                                                int npad, int jlen, int jtile, T eps, double *__restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = (blockIdx.x * (blockDim.x / kWave) + wave) * (kWave * IPL) + lane;
    const int s = blockIdx.y;
    const int j0 = s * jlen;
    const int j1 = min(n, j0 + jlen);
    T xi[IPL], yi[IPL], wxi[IPL], wyi[IPL];
    A ax[IPL], ay[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, n - 1);
        xi[k] = xs[i];
        yi[k] = ys[i];
        wxi[k] = wxs[i];
        wyi[k] = wys[i];
    }
    for (int jt = j0; jt < j1; jt += jtile) {
        const int je = min(j1, jt + jtile);
        int j = jt;
        for (; j + 4 <= je; j += 4) {
            if constexpr (sizeof(T) == 8) {
                // FP64: one reciprocal for four j (measured FP32: a shared form does
                // not pay, its multiplies costing what the FP32 reciprocal does)
                const T xq[4] = {xs[j], xs[j + 1], xs[j + 2], xs[j + 3]};
                const T yq[4] = {ys[j], ys[j + 1], ys[j + 2], ys[j + 3]};
                const T wxq[4] = {wxs[j], wxs[j + 1], wxs[j + 2], wxs[j + 3]};
                const T wyq[4] = {wys[j], wys[j + 1], wys[j + 2], wys[j + 3]};
#pragma unroll
                for (int k = 0; k < IPL; ++k)
                    hvp_2d_four(xi[k], yi[k], wxi[k], wyi[k], xq, yq, wxq, wyq, eps, ax[k], ay[k]);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const T xj = xs[j + u], yj = ys[j + u], wxj = wxs[j + u], wyj = wys[j + u];
#pragma unroll
                    for (int k = 0; k < IPL; ++k)
                        hvp_2d(xi[k], yi[k], wxi[k], wyi[k], xj, yj, wxj, wyj, eps, ax[k], ay[k]);
                }
            }
        }
        for (; j < je; ++j) {
            const T xj = xs[j], yj = ys[j], wxj = wxs[j], wyj = wys[j];
#pragma unroll
            for (int k = 0; k < IPL; ++k)
                hvp_2d(xi[k], yi[k], wxi[k], wyi[k], xj, yj, wxj, wyj, eps, ax[k], ay[k]);
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            ax[k].fold();
            ay[k].fold();
        }
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < n) {
            part[(size_t)(2 * s) * npad + i] = ax[k].get();
            part[(size_t)(2 * s + 1) * npad + i] = ay[k].get();
        }
    }
}

template <typename T, typename A, int IPL>
__global__ __launch_bounds__(256) void k_hvp_ring(const T *__restrict__ cs, const T *__restrict__ ws, int n,
                                                  int npad, int jlen, int jtile, T one_eps,
                                                  double *__restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int ibase = (blockIdx.x * (blockDim.x / kWave) + wave) * (kWave * IPL) + lane;
    const int s = blockIdx.y;
    const int j0 = s * jlen;
    const int j1 = min(n, j0 + jlen);
    const T *__restrict__ cc = cs;
    const T *__restrict__ ss = cs + npad;
    T ci[IPL], si[IPL], wi[IPL];
    A a[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = min(ibase + kWave * k, n - 1);
        ci[k] = cc[i];
        si[k] = ss[i];
        wi[k] = ws[i];
    }
    for (int jt = j0; jt < j1; jt += jtile) {
        const int je = min(j1, jt + jtile);
        int j = jt;
        for (; j + 8 <= je; j += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const T cj = cc[j + u], sj = ss[j + u], wj = ws[j + u];
#pragma unroll
                for (int k = 0; k < IPL; ++k) hvp_ring(ci[k], si[k], wi[k], cj, sj, wj, one_eps, a[k]);
            }
        }
        for (; j < je; ++j) {
            const T cj = cc[j], sj = ss[j], wj = ws[j];
#pragma unroll
            for (int k = 0; k < IPL; ++k) hvp_ring(ci[k], si[k], wi[k], cj, sj, wj, one_eps, a[k]);
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k) a[k].fold();
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int i = ibase + kWave * k;
        if (i < n) part[(size_t)s * npad + i] = a[k].get();
    }
}

// ------------------------------------------------------ symmetric product --

// The 2D term t(i, j) = phi''(r_i - r_j) (w_i - w_j) is odd under i <-> j (phi'' is
// even in r, w_i - w_j odd), so, as for the force (k_sym, pair.hip), one evaluation
// serves both particles: i adds t, j adds -t.  FP64, the force's tiles: a block
// takes a tile pair (a, b), a < b (SYM), or a diagonal tile (a, a), every ordered
// pair, i side only.  A wavefront holds 4 i per lane; tile b streams through in 16
// blocks of 64 j, and at step s lane l meets j = (l + s) mod 64: the j operands
// (x, y, wx, wy) and the j-side sums move one lane per step through ds_bpermute.
// The 4 i of a lane take one reciprocal (SHARE: the force's scheme, sym_tile in
// pair_terms.h), except where the tile holds pads, whose s would overflow the
// product.
//   x, y, wx, wy: this lane's 4 i;  e: eps;
//   load(blk, xj, yj, wxj, wyj): this lane's j of 64-j block blk (lane l: j = l);
//   jsum(blk, m, sj): the j-side sums of the block (sj belongs to j = m of it);
//   acc: the i-side sums, [component][i].
template <int TILE, bool SYM, bool SHARE, typename Load, typename JSum>
__device__ __forceinline__ void sym_tile_hvp(const double (&x)[kSymIpl], const double (&y)[kSymIpl],
                                             const double (&wx)[kSymIpl], const double (&wy)[kSymIpl], double e,
                                             int lane, Load &&load, JSum &&jsum, AccF64 (&acc)[2][kSymIpl])
{
    constexpr int nblk = TILE / kWave;
    const int next = ((lane + 1) & (kWave - 1)) * 4;  // ds_bpermute byte address of lane l + 1
    double n0, n1, n2, n3;
    load(0, n0, n1, n2, n3);
    for (int blk = 0; blk < nblk; ++blk) {
        double xj = n0, yj = n1, wxj = n2, wyj = n3;
        if (blk + 1 < nblk) load(blk + 1, n0, n1, n2, n3);
        AccF64 sj[2];
#pragma unroll 8
        for (int s = 0; s < kWave; ++s) {
            if (s) {
                xj = lane_next(next, xj);
                yj = lane_next(next, yj);
                wxj = lane_next(next, wxj);
                wyj = lane_next(next, wyj);
                if (SYM) {
                    sj[0].rotate(next);
                    sj[1].rotate(next);
                }
            }
            double dx[kSymIpl], dy[kSymIpl], inv[kSymIpl];
#pragma unroll
            for (int k = 0; k < kSymIpl; ++k) {
                dx[k] = x[k] - xj;
                dy[k] = y[k] - yj;
                inv[k] = fma_(dx[k], dx[k], fma_(dy[k], dy[k], e));
            }
            if constexpr (SHARE) {  // one reciprocal for the 4 i, as the force's (pair_terms.h)
                static_assert(kSymIpl == 4, "one reciprocal for the lane's 4 i");
                const double p01 = inv[0] * inv[1], p23 = inv[2] * inv[3];
                const double r = rcp_(p01 * p23);
                const double r01 = r * p23, r23 = r * p01;
                const double s0 = inv[0], s2 = inv[2];
                inv[0] = r01 * inv[1];
                inv[1] = r01 * s0;
                inv[2] = r23 * inv[3];
                inv[3] = r23 * s2;
            } else {
#pragma unroll
                for (int k = 0; k < kSymIpl; ++k) inv[k] = rcp_(inv[k]);
            }
#pragma unroll
            for (int k = 0; k < kSymIpl; ++k) {
                const double ux = wx[k] - wxj, uy = wy[k] - wyj;
                const double t = fma_(dx[k], ux, dy[k] * uy) * inv[k];
                const double c = (t + t) * inv[k];
                acc[0][k].add(inv[k], ux);
                acc[0][k].add(-c, dx[k]);
                acc[1][k].add(inv[k], uy);
                acc[1][k].add(-c, dy[k]);
                if (SYM) {
                    sj[0].add(-inv[k], ux);
                    sj[0].add(c, dx[k]);
                    sj[1].add(-inv[k], uy);
                    sj[1].add(c, dy[k]);
                }
            }
        }
        if (SYM) jsum(blk, (lane + kWave - 1) & (kWave - 1), sj);  // after step 63 lane l holds j = l - 1
    }
}

// One block's share of the symmetric product: tile pair (a, b) (SYM) or the diagonal
// tile a = b, tiles of W x 64 x 4 particles (the force's, sym_tile_n).  q, w:
// [2][npad] operand rows (padded); part: slots [ntile][2][npad], the i side to slot
// b of the i particles, the j side (the W wavefronts' sums added in FP64 in a
// fixed order after every 64-j block) to slot a of the j particles.
template <bool SYM, int W>
__device__ __forceinline__ void hvp_sym_block(const double *__restrict__ q, const double *__restrict__ w, int n,
                                              int npad, double e, double *__restrict__ part, int a, int b,
                                              double (&jw)[W][2][kWave])
{
    constexpr int TILE = W * kWave * kSymIpl;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int i0 = a * TILE + wave * kWave * kSymIpl + lane;
    double x[kSymIpl], y[kSymIpl], wx[kSymIpl], wy[kSymIpl];
#pragma unroll
    for (int k = 0; k < kSymIpl; ++k) {
        const int i = i0 + k * kWave;
        x[k] = q[i];
        y[k] = q[npad + i];
        wx[k] = w[i];
        wy[k] = w[npad + i];
    }
    const int jl = b * TILE + lane;
    auto load = [&](int blk, double &xj, double &yj, double &wxj, double &wyj) {
        const int j = jl + blk * kWave;
        xj = q[j];
        yj = q[npad + j];
        wxj = w[j];
        wyj = w[npad + j];
    };
    auto jsum = [&](int blk, int m, AccF64 (&sj)[2]) {
        jw[wave][0][m] = sj[0].get();
        jw[wave][1][m] = sj[1].get();
        __syncthreads();
        for (int x = threadIdx.x; x < 2 * kWave; x += W * kWave) {  // W = 1: a thread per (d, j) in turn
            const int d = x / kWave, mm = x & (kWave - 1);
            double t = 0.0;
#pragma unroll
            for (int v = 0; v < W; ++v) t += jw[v][d][mm];
            part[(size_t)(2 * a + d) * npad + b * TILE + blk * kWave + mm] = t;
        }
        __syncthreads();
    };
    AccF64 acc[2][kSymIpl];
    if ((b + 1) * TILE > n)  // a j tile with pads: one reciprocal a pair
        sym_tile_hvp<TILE, SYM, false>(x, y, wx, wy, e, lane, load, jsum, acc);
    else
        sym_tile_hvp<TILE, SYM, true>(x, y, wx, wy, e, lane, load, jsum, acc);
#pragma unroll
    for (int k = 0; k < kSymIpl; ++k)
#pragma unroll
        for (int d = 0; d < 2; ++d) part[(size_t)(2 * b + d) * npad + i0 + k * kWave] = acc[d][k].get();
}

// One launch per product: the tile pairs a < b in row-major order, then the diagonal
// tiles (the force's order, k_sym in pair.hip).
template <int W>
__global__ __launch_bounds__(W * kWave) void k_hvp_sym(const double *__restrict__ q, const double *__restrict__ w,
                                                       int n, int npad, int ntile, double e,
                                                       double *__restrict__ part)
{
    __shared__ double jw[W][2][kWave];
    const int t = (int)blockIdx.x, noff = ntile * (ntile - 1) / 2;
    if (t < noff) {
        int a, b;
        sym_tile_pair(t, ntile, a, b);
        hvp_sym_block<true, W>(q, w, n, npad, e, part, a, b, jw);
    } else {
        hvp_sym_block<false, W>(q, w, n, npad, e, part, t - noff, t - noff, jw);
    }
}

// PREP_COPY64: the symmetric product's padded FP64 rows (positions to ops, vector to wops).
enum Prep { PREP_NONE = 0, PREP_CAST32 = 1, PREP_HALF32 = 2, PREP_SINCOS64 = 3, PREP_COPY64 = 4 };

// Elementwise: hw = pref * (sum of the product partials, fixed order); out = hw;
// lq -= h hw; lp += a lq; operands of the next product (positions pos, vector lp).
// PREP_COPY64 (the symmetric product): the grid covers npad and writes the pads of
// the operand rows too, positions at sym_pad (1e150) and the vector at 0.
template <int D, int PREP>
__global__ __launch_bounds__(256) void k_adj_update(const double *__restrict__ part, int S, int n, int npad,
                                                    double pref, int flags, double h, double h2, double a,
                                                    double *__restrict__ lq, double *__restrict__ lp,
                                                    double *__restrict__ out, const double *__restrict__ pos,
                                                    void *__restrict__ ops, void *__restrict__ wops)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) {
        if constexpr (PREP == PREP_COPY64) {
            if (i < npad) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (flags & ADJ_PREPQ) static_cast<double *>(ops)[(size_t)d * npad + i] = sym_pad<MD_GRAV2D, double>();
                    if (flags & ADJ_PREPW) static_cast<double *>(wops)[(size_t)d * npad + i] = 0.0;
                }
            }
        }
        return;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const size_t k = (size_t)d * n + i;
        if (flags & (ADJ_OUT | ADJ_KICK)) {
            const double hw = pref * slot_sum<D>(part, S, d, npad, i);
            if (flags & ADJ_OUT) out[k] = hw;
            if (flags & ADJ_KICK) {
                double l = lq[k] - h * hw;
                if (flags & ADJ_KICK2) l -= h2 * hw;  // a second kick at the same positions
                lq[k] = l;
            }
        }
        if (flags & ADJ_DRIFT) lp[k] += a * lq[k];
        if (flags & ADJ_PREPW) {
            if (PREP == PREP_COPY64) static_cast<double *>(wops)[(size_t)d * npad + i] = lp[k];
            else static_cast<float *>(wops)[(size_t)d * npad + i] = (float)lp[k];
        }
        if ((flags & ADJ_PREPQ) && PREP != PREP_NONE) {
            const double qd = pos[k];
            if (PREP == PREP_COPY64) {
                static_cast<double *>(ops)[(size_t)d * npad + i] = qd;
            } else if (PREP == PREP_CAST32) {
                static_cast<float *>(ops)[(size_t)d * npad + i] = (float)qd;
            } else if (PREP == PREP_HALF32) {
                double sn, cn;
                sincos64(0.5 * qd, &sn, &cn);
                static_cast<float *>(ops)[i] = (float)(1.4142135623730951 * cn);
                static_cast<float *>(ops)[npad + i] = (float)(1.4142135623730951 * sn);
            } else {
                double sn, cn;
                sincos64(qd, &sn, &cn);
                static_cast<double *>(ops)[i] = cn;
                static_cast<double *>(ops)[npad + i] = sn;
            }
        }
    }
}

// The symmetric product (k_hvp_sym) where the force takes the symmetric form: 2D, FP64.
bool hvp_sym(const md_ctx *c)
{
    return c->model == MD_GRAV2D && c->prec == MD_FP64 && !c->batch && launch_form(c) == MD_LAUNCH_SYMMETRIC;
}

int prep_kind(const md_ctx *c)
{
    if (c->model == MD_GRAV2D) return c->prec != MD_FP64 ? PREP_CAST32 : hvp_sym(c) ? PREP_COPY64 : PREP_NONE;
    return c->prec == MD_FP64 ? PREP_SINCOS64 : PREP_HALF32;
}

template <typename T, typename A>
hipError_t hvp_launch(md_ctx *c, const void *qsrc, const void *wsrc, dim3 grid, dim3 block, int jlen)
{
    const int n = (int)c->n, npad = (int)c->npad, jt = c->tiles.jtile;
    const bool fp64 = c->prec == MD_FP64;
    const int ts = timed_begin(c, c->model == MD_GRAV2D ? "k_hvp_2d" : "k_hvp_ring");
    if (c->model == MD_GRAV2D) {
        const T *x = static_cast<const T *>(qsrc);
        const T *y = x + (fp64 ? n : npad);
        const T *wx = static_cast<const T *>(wsrc);
        const T *wy = wx + (fp64 ? n : npad);
        const T eps = (T)c->eps;
        switch (c->tiles.ipl) {
        case 1: hipLaunchKernelGGL((k_hvp_2d<T, A, 1>), grid, block, 0, c->stream, x, y, wx, wy, n, npad, jlen, jt, eps, c->part); break;
        case 2: hipLaunchKernelGGL((k_hvp_2d<T, A, 2>), grid, block, 0, c->stream, x, y, wx, wy, n, npad, jlen, jt, eps, c->part); break;
        default: hipLaunchKernelGGL((k_hvp_2d<T, A, 4>), grid, block, 0, c->stream, x, y, wx, wy, n, npad, jlen, jt, eps, c->part); break;
        }
    } else {
        const T *cs = static_cast<const T *>(qsrc);
        const T *w = static_cast<const T *>(wsrc);
        const T one_eps = sizeof(T) == 8 ? (T)(1.0 + c->eps) : (T)(2.0 * c->eps);  // FP32 half-angle form: 2 eps
        switch (c->tiles.ipl) {
        case 1: hipLaunchKernelGGL((k_hvp_ring<T, A, 1>), grid, block, 0, c->stream, cs, w, n, npad, jlen, jt, one_eps, c->part); break;
        case 2: hipLaunchKernelGGL((k_hvp_ring<T, A, 2>), grid, block, 0, c->stream, cs, w, n, npad, jlen, jt, one_eps, c->part); break;
        default: hipLaunchKernelGGL((k_hvp_ring<T, A, 4>), grid, block, 0, c->stream, cs, w, n, npad, jlen, jt, one_eps, c->part); break;
        }
    }
    const hipError_t err = hipGetLastError();
    timed_end(c, ts);
    return err;
}

}  // namespace

// Product partials of H(pos) w into c->part.  FP64 2D reads pos and w directly;
// every other form reads the operands prepared by launch_adj_update (ADJ_PREPQ,
// ADJ_PREPW), i.e. `pos` and `w` must be the arrays those operands came from.
hipError_t launch_hvp_pair(md_ctx *c, const double *pos, const double *w)
{
    if (hvp_sym(c)) {
        const int npad = (int)c->npad, tile = sym_tile_n(c->model, c->prec, c->n), ntile = npad / tile;
        const int nblocks = ntile * (ntile - 1) / 2 + ntile;
        const double *q = static_cast<const double *>(c->ops), *w = static_cast<const double *>(c->wops);
        const int ts = timed_begin(c, "k_hvp_sym");
        if (tile == kSymTile)
            hipLaunchKernelGGL(k_hvp_sym<4>, dim3((unsigned)nblocks), dim3(4 * kWave), 0, c->stream, q, w, (int)c->n,
                               npad, ntile, c->eps, c->part);
        else if (tile == kSymTileSmall)
            hipLaunchKernelGGL(k_hvp_sym<2>, dim3((unsigned)nblocks), dim3(2 * kWave), 0, c->stream, q, w, (int)c->n,
                               npad, ntile, c->eps, c->part);
        else
            hipLaunchKernelGGL(k_hvp_sym<1>, dim3((unsigned)nblocks), dim3(kWave), 0, c->stream, q, w, (int)c->n,
                               npad, ntile, c->eps, c->part);
        const hipError_t err = hipGetLastError();
        timed_end(c, ts);
        return err;
    }
    const Tiles &t = c->tiles;
    const int n = (int)c->n;
    const int per_block = kWave * t.ipl * t.waves;
    const dim3 block((unsigned)(kWave * t.waves));
    const dim3 grid((unsigned)((n + per_block - 1) / per_block), (unsigned)t.jsplit);
    int jlen = (n + t.jsplit - 1) / t.jsplit;
    jlen = (jlen + 15) / 16 * 16;
    const bool fp64 = c->prec == MD_FP64;
    const void *qsrc = (c->model == MD_GRAV2D && fp64) ? (const void *)pos : (const void *)c->ops;
    const void *wsrc = fp64 ? (const void *)w : (const void *)c->wops;
    switch (c->prec) {
    case MD_FP64: return hvp_launch<double, AccF64>(c, qsrc, wsrc, grid, block, jlen);
    case MD_MIXED: return hvp_launch<float, AccTile>(c, qsrc, wsrc, grid, block, jlen);
    case MD_MIXED_KAHAN: return hvp_launch<float, AccKahan>(c, qsrc, wsrc, grid, block, jlen);
    default: return hvp_launch<float, AccPair64>(c, qsrc, wsrc, grid, block, jlen);
    }
}

hipError_t launch_adj_update(md_ctx *c, int flags, double h, double h2, double a, double *lq, double *lp,
                             double *out, const double *pos)
{
    const int n = (int)c->n;
    const bool sym = hvp_sym(c);
    const int nthreads = sym && (flags & (ADJ_PREPQ | ADJ_PREPW)) ? (int)c->npad : n;  // the pads too
    const dim3 block(256), grid((unsigned)((nthreads + 255) / 256));
    // Hessian prefactors: 2/N (2D); 1/(2 sqrt2 N) (Ring, FP64 terms); 1/N (Ring, half-angle FP32 terms)
    const double pref = c->model == MD_GRAV2D ? 2.0 / (double)n
                        : c->prec == MD_FP64  ? 1.0 / (2.0 * 1.4142135623730951 * (double)n)
                                              : 1.0 / (double)n;
    const int pk = prep_kind(c);
    if (c->prec == MD_FP64 && !sym) flags &= ~ADJ_PREPW;
    if (pk == PREP_NONE) flags &= ~ADJ_PREPQ;
    const int npad = (int)c->npad, S = sym ? npad / sym_tile_n(c->model, c->prec, c->n) : c->tiles.jsplit;
#define MD_ADJ(D_, P_)                                                                                          \
    hipLaunchKernelGGL((k_adj_update<D_, P_>), grid, block, 0, c->stream, c->part, S, n, npad, pref, flags, h, h2, a, \
                       lq, lp, out, pos, c->ops, c->wops)
    if (c->model == MD_GRAV2D) {
        if (pk == PREP_CAST32) MD_ADJ(2, PREP_CAST32);
        else if (pk == PREP_COPY64) MD_ADJ(2, PREP_COPY64);
        else MD_ADJ(2, PREP_NONE);
    } else {
        if (pk == PREP_HALF32) MD_ADJ(1, PREP_HALF32);
        else MD_ADJ(1, PREP_SINCOS64);
    }
#undef MD_ADJ
    return hipGetLastError();
}

}  // namespace md
