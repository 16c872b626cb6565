// pair_terms.h -- the per-pair arithmetic of the Ring (eqs. 8-9) and 2D
// (gradient of eq. 3) forces and the per-particle accumulation policies, shared
// by the single-system kernels (pair.hip) and the batched-ensemble kernels
// (batch.hip) so both compute bit-identical pair terms.
#pragma once

#include "device.h"

namespace md {
namespace pairs {

// The value v of lane addr / 4 of the wavefront (ds_bpermute: the LDS crossbar,
// no LDS memory and no VALU issue).
__device__ __forceinline__ float lane_next(int addr, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_next(int addr, double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------- accumulators --
// rotate(addr): take the accumulator of lane addr / 4 (the symmetric kernels move
// the j-side sums with their j).

// FP32 partial over a j tile, folded into an FP64 total once per tile.
struct AccTile {
    float s = 0.f;
    double t = 0.0;
    __device__ __forceinline__ void add(float a, float b) { s = __builtin_fmaf(a, b, s); }
    __device__ __forceinline__ void fold() { t += (double)s; s = 0.f; }
    __device__ __forceinline__ double get() const { return t; }
    __device__ __forceinline__ void rotate(int addr) { s = lane_next(addr, s); }
};

// Kahan-compensated FP32 sum of every pair term; -c holds the lost low part.
struct AccKahan {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float a, float b)
    {
        const float y = a * b - c;
        const float u = s + y;
        c = (u - s) - y;
        s = u;
    }
    __device__ __forceinline__ void fold() {}
    __device__ __forceinline__ double get() const { return (double)s - (double)c; }
    __device__ __forceinline__ void rotate(int addr)
    {
        s = lane_next(addr, s);
        c = lane_next(addr, c);
    }
};

// Each FP32 pair term added into an FP64 accumulator.
struct AccPair64 {
    double t = 0.0;
    __device__ __forceinline__ void add(float a, float b) { t += (double)(a * b); }
    __device__ __forceinline__ void fold() {}
    __device__ __forceinline__ double get() const { return t; }
    __device__ __forceinline__ void rotate(int addr) { t = lane_next(addr, t); }
};

// Plain FP64.
struct AccF64 {
    double t = 0.0;
    __device__ __forceinline__ void add(double a, double b) { t = __builtin_fma(a, b, t); }
    __device__ __forceinline__ void fold() {}
    __device__ __forceinline__ double get() const { return t; }
    __device__ __forceinline__ void rotate(int addr) { t = lane_next(addr, t); }
};

__device__ __forceinline__ float rcp_(float x) { return rcp32(x); }
__device__ __forceinline__ double rcp_(double x) { return rcp64(x); }
__device__ __forceinline__ float rsq_(float x) { return rsq32(x); }
__device__ __forceinline__ double rsq_(double x) { return rsq64(x); }
// u^{-3/2}.  FP32: the hardware inverse square root, cubed.  FP64: with y the
// hardware seed of u^{-1/2} (relative error below 2^-23) and e = 1 - u y^2,
// u^{-3/2} = y^3 (1 - e)^{-3/2} = y^3 (1 + 3e/2 + 15e^2/8) + O(e^3): refined once
// in the cube, one FP64 operation fewer than refining u^{-1/2} and cubing it.
__device__ __forceinline__ float rsq3_(float u)
{
    const float r = rsq32(u);
    return r * r * r;
}
__device__ __forceinline__ double rsq3_(double u)
{
    const double y = __builtin_amdgcn_rsq(u);
    const double y2 = y * y;
    const double e = __builtin_fma(-u, y2, 1.0);
    const double y3 = y2 * y;
    return __builtin_fma(y3, e * __builtin_fma(e, 1.875, 1.5), y3);
}
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------------------ pair terms --

// 2D: adds (r_i - r_j) / (|r_i - r_j|^2 + eps) to (ax, ay).
template <typename T, typename A>
__device__ __forceinline__ void pair_2d(T xi, T yi, T xj, T yj, T eps, A &ax, A &ay)
{
    const T dx = xi - xj;
    const T dy = yi - yj;
    const T w = rcp_(fma_(dx, dx, fma_(dy, dy, eps)));
    ax.add(dx, w);
    ay.add(dy, w);
}

// 2D, two j (a, then b) against the same i with one reciprocal: with s_a, s_b the
// two |r_i - r_j|^2 + eps and R = 1/(s_a s_b), the weights are 1/s_a = R s_b and
// 1/s_b = R s_a (three multiplies in place of a reciprocal; each weight carries
// about 2 ulp instead of 1).  s_a s_b must be finite and nonzero.  The FP64 forms
// take it (the refined FP64 reciprocal is a quarter-rate seed and three FMAs); in
// FP32 the three multiplies cost about what the reciprocal does.
template <typename T, typename A>
__device__ __forceinline__ void pair_2d_two(T xi, T yi, T xa, T ya, T xb, T yb, T eps, A &ax, A &ay)
{
    const T dxa = xi - xa, dya = yi - ya, dxb = xi - xb, dyb = yi - yb;
    const T sa = fma_(dxa, dxa, fma_(dya, dya, eps));
    const T sb = fma_(dxb, dxb, fma_(dyb, dyb, eps));
    const T r = rcp_(sa * sb);
    const T wa = r * sb, wb = r * sa;
    ax.add(dxa, wa);
    ay.add(dya, wa);
    ax.add(dxb, wb);
    ay.add(dyb, wb);
}

// 2D, four j (a, b, c, d) against the same i with one reciprocal: with P = s_a s_b,
// Q = s_c s_d and R = 1/(P Q), the weights are 1/s_a = (R Q) s_b, 1/s_b = (R Q) s_a,
// 1/s_c = (R P) s_d and 1/s_d = (R P) s_c (nine multiplies and one reciprocal in
// place of four; each weight carries about 5 ulp).  The product of the four s must
// be a normal number: in FP64, eps in the range md_init takes and particles closer
// than about 1e38 to each other.  The terms are added in the order a, b, c, d.
template <typename T, typename A>
__device__ __forceinline__ void pair_2d_four(T xi, T yi, const T *xj, const T *yj, T eps, A &ax, A &ay)
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
    const T w[4] = {r01 * s[1], r01 * s[0], r23 * s[3], r23 * s[2]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ax.add(dx[k], w[k]);
        ay.add(dy[k], w[k]);
    }
}

// Whether the 2D terms of operand type T share reciprocals: the j in fours
// (pair_2d_four), then twos (pair_2d_two), then one by one.
template <typename T>
constexpr bool kPairShare = sizeof(T) == 8;

// The 2D terms of j in [j0, j1) for each lane's IPL i, j ascending, the
// accumulators folded every jtile j from j0 (jtile a multiple of 16).  The j
// operands are wave-uniform (scalar loads).  With kPairShare<T> the j of each
// jtile go in fours from its start (j + 4m), then a last two and a last one as
// they remain: the grouping every 2D staged, fused and batched kernel shares, so
// that they agree bit for bit.
template <typename T, typename A, int IPL>
__device__ __forceinline__ void grav_j_range(const T *__restrict__ xs, const T *__restrict__ ys, int j0, int j1,
                                             int jtile, T eps, const T (&xi)[IPL], const T (&yi)[IPL],
                                             A (&ax)[IPL], A (&ay)[IPL])
{
    for (int jt = j0; jt < j1; jt += jtile) {
        const int je = min(j1, jt + jtile);
        int j = jt;
        for (; j + 8 <= je; j += 8) {
            if constexpr (kPairShare<T>) {
#pragma unroll
                for (int u = 0; u < 8; u += 4) {
                    const T xq[4] = {xs[j + u], xs[j + u + 1], xs[j + u + 2], xs[j + u + 3]};
                    const T yq[4] = {ys[j + u], ys[j + u + 1], ys[j + u + 2], ys[j + u + 3]};
#pragma unroll
                    for (int k = 0; k < IPL; ++k) pair_2d_four(xi[k], yi[k], xq, yq, eps, ax[k], ay[k]);
                }
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const T xj = xs[j + u];
                    const T yj = ys[j + u];
#pragma unroll
                    for (int k = 0; k < IPL; ++k) pair_2d(xi[k], yi[k], xj, yj, eps, ax[k], ay[k]);
                }
            }
        }
        if constexpr (kPairShare<T>) {
            if (j + 4 <= je) {
                const T xq[4] = {xs[j], xs[j + 1], xs[j + 2], xs[j + 3]};
                const T yq[4] = {ys[j], ys[j + 1], ys[j + 2], ys[j + 3]};
#pragma unroll
                for (int k = 0; k < IPL; ++k) pair_2d_four(xi[k], yi[k], xq, yq, eps, ax[k], ay[k]);
                j += 4;
            }
            if (j + 2 <= je) {
                const T xa = xs[j], ya = ys[j], xb = xs[j + 1], yb = ys[j + 1];
#pragma unroll
                for (int k = 0; k < IPL; ++k) pair_2d_two(xi[k], yi[k], xa, ya, xb, yb, eps, ax[k], ay[k]);
                j += 2;
            }
        }
        for (; j < je; ++j) {
            const T xj = xs[j];
            const T yj = ys[j];
#pragma unroll
            for (int k = 0; k < IPL; ++k) pair_2d(xi[k], yi[k], xj, yj, eps, ax[k], ay[k]);
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            ax[k].fold();
            ay[k].fold();
        }
    }
}

// Ring (eq. 9): the term sin(ti - tj) / (1 - cos(ti - tj) + eps)^{3/2} as the
// factors p q, from the cosines and sines of both angles.  one_eps = 1 + eps.
// q is symmetric in i, j.  With EXACT the numerator p is two rounded products and
// a difference, so exactly antisymmetric (and exactly 0 for i = j): needed where a
// pair is evaluated once per ordered pair.  Without it p is one product and one
// FMA (one rounding fewer, one instruction fewer), for a pair evaluated once for
// both of its particles, never i with itself.
template <typename T, bool EXACT = true>
__device__ __forceinline__ void ring_factors_eq9(T ci, T si, T cj, T sj, T one_eps, T &p, T &q)
{
    T num;
    if constexpr (EXACT) {
#pragma clang fp contract(off)
        num = si * cj - ci * sj;
    } else {
        num = fma_(si, cj, -(ci * sj));
    }
    const T u = fma_(-ci, cj, fma_(-si, sj, one_eps));
    p = num;
    q = rsq3_(u);
}

// Ring, half-angle operands (the FP32 forms): A = sqrt2 sin(t/2), B = sqrt2 cos(t/2)
// of each angle.  With d = ti - tj:  a = A_i B_j - B_i A_j = 2 sin(d/2) (exactly
// antisymmetric: two rounded products) and b = B_i B_j + A_i A_j = 2 cos(d/2), so
// 1 - cos d = a^2/2 and sin d = a b/2.  With u' = a^2 + 2 eps = 2 (1 - cos d + eps)
// and r' = u'^{-1/2}, the term sin d / (1 - cos d + eps)^{3/2} is sqrt2 a b r'^3;
// the sqrt2 goes into the prefactor, and eps2 = 2 eps.  Unlike eq. 9's angle-sum
// form, 1 - cos d is formed without cancelling against 1: its rounding error
// scales with |d|, which matters in FP32 for close pairs.  Factors: p = a b
// (antisymmetric), q = r'^3 (symmetric).  EXACT as for eq. 9: without it a is one
// product and one FMA.
template <typename T, bool EXACT = true>
__device__ __forceinline__ void ring_factors_half(T ai, T bi, T aj, T bj, T eps2, T &p, T &q)
{
    T a;
    if constexpr (EXACT) {
#pragma clang fp contract(off)
        a = ai * bj - bi * aj;
    } else {
        a = fma_(ai, bj, -(bi * aj));
    }
    const T b = fma_(bi, bj, ai * aj);
    const T r = rsq_(fma_(a, a, eps2));
    p = a * b;
    q = r * r * r;
}

// The Ring pair term's factors in the context's precision: eq. 9 on (cos t, sin t)
// in FP64; the half-angle form on sqrt2 (cos(t/2), sin(t/2)) in FP32 (then e holds
// 2 eps, else 1 + eps).
template <typename T, bool EXACT = true>
__device__ __forceinline__ void ring_factors(T c0, T s0, T c1, T s1, T e, T &p, T &q)
{
    if constexpr (sizeof(T) == 8) ring_factors_eq9<T, EXACT>(c0, s0, c1, s1, e, p, q);
    else ring_factors_half<T, EXACT>(s0, c0, s1, c1, e, p, q);
}

// Adds the Ring pair term (i = 0, j = 1) to the accumulator a.
template <typename T, typename A>
__device__ __forceinline__ void ring_term(T c0, T s0, T c1, T s1, T e, A &a)
{
    T p, q;
    ring_factors(c0, s0, c1, s1, e, p, q);
    a.add(p, q);
}

// Streams the j operands (rows r0, r1) of j in [j0, j1) through a block-shared
// LDS window of WJ entries per row: the block loads each window with coalesced
// vector loads between two barriers, and every lane reads the entries broadcast.
// term(x, y) runs for every j in ascending order and fold() after every jtile j
// counted from j0 and at j1 (jtile a multiple of 16): the order of the
// scalar-load kernels, so the same sums bit for bit.  j0 and j1 must be uniform
// across the block (every thread reaches the barriers).
template <int WJ, typename T, typename Term, typename Fold>
__device__ __forceinline__ void window_stream(const T *__restrict__ r0, const T *__restrict__ r1, int j0, int j1,
                                              int jtile, T (*win)[WJ], Term &&term, Fold &&fold)
{
    for (int g = j0; g < j1; g += 16) {
        const int off = (g - j0) % WJ;
        if (off == 0) {
            __syncthreads();  // the previous window's reads are done
            for (int m = threadIdx.x; m < WJ; m += blockDim.x) {
                const int j = g + m;
                if (j < j1) {
                    win[0][m] = r0[j];
                    win[1][m] = r1[j];
                }
            }
            __syncthreads();
        }
        if (g + 16 <= j1) {
#pragma unroll
            for (int u = 0; u < 16; ++u) term(win[0][off + u], win[1][off + u]);
        } else {
            for (int u = 0; u < j1 - g; ++u) term(win[0][off + u], win[1][off + u]);
        }
        if ((g + 16 - j0) % jtile == 0 || g + 16 >= j1) fold();
    }
}


// ------------------------------------------------------- symmetric tile pass --

// The 2D pair term of the gradient of eq. 3 is odd in r_i - r_j, and the Ring term
// of eq. 9 is odd in ti - tj, so one evaluation serves both particles (Newton's
// third law).  A tile is kSymTile = 4 wavefronts x 64 lanes x 4 i.  For a tile
// pair (a, b) each wavefront holds its 256 i of tile a in registers and tile b
// streams through in 16 blocks of 64 j.  At step s of a 64-j block, lane l pairs
// its 4 i with j = (l + s) mod 64: the j operands and the j-side sums move one
// lane per step through ds_bpermute (no VALU issue; DPP lane moves measured 2-3x
// the cost of an FMA on gfx950), so every lane adds to a different j and no
// atomics are needed.
//   2D, per pair: 2 differences, r^2 + eps (2 FMA), 1 reciprocal; the i side adds
//     the staged form's term (r_i - r_j) w, the j side its negative.
//   Ring, per pair: the factors p q of the staged form's term (ring_factors; p is
//     exactly antisymmetric, q symmetric); the i side adds p q, the j side -p q.
// A is the accumulation policy of the precision form (AccTile: FP32, folded into
// FP64 every 128 j on the i side; AccKahan; AccF64).  SYM = false: a diagonal tile,
// every ordered pair, i side only.
//   u0, u1:   the wavefront's i operands (4 per lane);
//   e:        eps (2D), 1 + eps (Ring FP64) or 2 eps (Ring FP32);
//   load(blk, v0, v1): this lane's j operands of 64-j block blk (lane l: j = l);
//   jsum(blk, m, sj):  the j-side sums of the block; sj belongs to j = m of it;
//   acc:      the i-side accumulators, [component][i].
constexpr int kSymIpl = 4, kSymWaves = kSymTile / (kWave * kSymIpl);

// Tile pair (a, b), a < b, of linear index t in row-major order over a.
__device__ __forceinline__ void sym_tile_pair(int t, int ntile, int &a, int &b)
{
    auto row0 = [ntile](int r) { return r * (2 * ntile - r - 1) / 2; };  // first index of row r
    const double m = 2.0 * ntile - 1.0;
    int r = (int)((m - sqrt(m * m - 8.0 * t)) * 0.5);
    r = max(0, min(r, ntile - 2));
    while (r > 0 && row0(r) > t) --r;
    while (r + 1 <= ntile - 2 && row0(r + 1) <= t) ++r;
    a = r;
    b = r + 1 + (t - row0(r));
}

// Operand value of a pad particle (beyond the system's or realization's end): its
// pair terms vanish.  2D FP32: r^2 overflows to +inf, the reciprocal is 0 and the
// terms exactly 0.  2D FP64: r^2 about 2e300 (the refined FP64 reciprocal of +inf
// would be NaN), terms about 5e-151.  Ring: the numerator p is exactly 0.
template <int MODEL, typename T>
__host__ __device__ constexpr T sym_pad()
{
    if (MODEL == MD_RING) return T(0);
    return sizeof(T) == 4 ? T(1e30f) : T(1e150);
}

// nblk (1 .. kSymTile / kWave, uniform across the block): the 64-j blocks of the j
// tile to stream; a ragged tile stops after its last block that holds a particle.
// SHARE (2D): the lane's 4 i take one reciprocal against the same j: with s0 .. s3
// their |r_i - r_j|^2 + eps, P01 = s0 s1, P23 = s2 s3 and R = 1/(P01 P23), the
// weights are 1/s0 = (R P23) s1, 1/s1 = (R P23) s0, 1/s2 = (R P01) s3 and
// 1/s3 = (R P01) s2 (nine multiplies and one refined reciprocal in place of four;
// each weight carries about 5 ulp instead of 1).  Needs s0 s1 s2 s3 a normal FP64
// number (particles closer than about 1e38 to each other, eps in [1e-75, 1e75],
// the range md_init takes) and no pad particle among the operands (the pads' s
// would overflow the product), so blocks that hold pads take SHARE = false.
template <int MODEL, typename T, typename A, bool SYM, bool SHARE = false, typename Load, typename JSum>
__device__ __forceinline__ void sym_tile(const T (&u0)[kSymIpl], const T (&u1)[kSymIpl], T e, int lane, int nblk,
                                         Load &&load, JSum &&jsum, A (&acc)[MODEL == MD_GRAV2D ? 2 : 1][kSymIpl])
{
    constexpr int D = MODEL == MD_GRAV2D ? 2 : 1;
    const int next = ((lane + 1) & (kWave - 1)) * 4;  // ds_bpermute byte address of lane l + 1
    T v0n, v1n;
    load(0, v0n, v1n);
    for (int blk = 0; blk < nblk; ++blk) {
        T v0 = v0n, v1 = v1n;
        if (blk + 1 < nblk) load(blk + 1, v0n, v1n);
        A sj[D];  // j-side sums of the j this lane holds
#pragma unroll 16
        for (int s = 0; s < kWave; ++s) {
            if (s) {
                v0 = lane_next(next, v0);
                v1 = lane_next(next, v1);
                if (SYM) {
#pragma unroll
                    for (int d = 0; d < D; ++d) sj[d].rotate(next);
                }
            }
            if constexpr (MODEL == MD_GRAV2D && SHARE) {
                T dx[kSymIpl], dy[kSymIpl], w[kSymIpl];
#pragma unroll
                for (int k = 0; k < kSymIpl; ++k) {
                    dx[k] = v0 - u0[k];
                    dy[k] = v1 - u1[k];
                    w[k] = fma_(dx[k], dx[k], fma_(dy[k], dy[k], e));
                }
                static_assert(kSymIpl == 4, "one reciprocal for the lane's 4 i");
                {
                    const T p01 = w[0] * w[1], p23 = w[2] * w[3];
                    const T r = rcp_(p01 * p23);
                    const T r01 = r * p23, r23 = r * p01;
                    const T s0 = w[0], s2 = w[2];
                    w[0] = r01 * w[1];
                    w[1] = r01 * s0;
                    w[2] = r23 * w[3];
                    w[3] = r23 * s2;
                }
#pragma unroll
                for (int k = 0; k < kSymIpl; ++k) {
                    acc[0][k].add(-dx[k], w[k]);
                    acc[1][k].add(-dy[k], w[k]);
                    if (SYM) {
                        sj[0].add(dx[k], w[k]);
                        sj[1].add(dy[k], w[k]);
                    }
                }
                continue;
            }
#pragma unroll
            for (int k = 0; k < kSymIpl; ++k) {
                if constexpr (MODEL == MD_GRAV2D) {
                    const T dx = v0 - u0[k], dy = v1 - u1[k];
                    const T w = rcp_(fma_(dx, dx, fma_(dy, dy, e)));
                    acc[0][k].add(-dx, w);
                    acc[1][k].add(-dy, w);
                    if (SYM) {
                        sj[0].add(dx, w);
                        sj[1].add(dy, w);
                    }
                } else {
                    T p, q;  // a tile pair meets each pair once, never i with itself
                    ring_factors<T, !SYM>(u0[k], u1[k], v0, v1, e, p, q);
                    acc[0][k].add(p, q);
                    if (SYM) sj[0].add(-p, q);
                }
            }
        }
        if (SYM) {  // after step 63 lane l holds j = l - 1 (mod 64) of the block
#pragma unroll
            for (int d = 0; d < D; ++d) sj[d].fold();
            jsum(blk, (lane + kWave - 1) & (kWave - 1), sj);
        }
        if ((blk & 1) || blk + 1 == nblk) {  // every 128 j, and at the end
#pragma unroll
            for (int k = 0; k < kSymIpl; ++k)
#pragma unroll
                for (int d = 0; d < D; ++d) acc[d][k].fold();
        }
    }
}

}  // namespace pairs
}  // namespace md
