// api.hip -- the C ABI of libmd (md.h): argument validation, workspace carve-up,
// tile configuration and launch form (staged or fused), the driver of the
// fourth-order Yoshida composition (Sec. 3, eq. 4) that sequences the kernels of
// pair.hip and hmf.hip, its reverse sweep over adjoint.hip's products, and the
// batched-ensemble work lists of batch.hip.
//
// The Yoshida step (eq. 4 and the step list after it) as a kick-drift sequence,
// with the force at the new positions used for the final kick and carried into
// the next step (three force evaluations per step):
//     p += B0 dt f;  q += D0 dt p;  f = F(q)
//     p += B1 dt f;  q += D1 dt p;  f = F(q)
//     p += B1 dt f;  q += D0 dt p;  f = F(q)
//     p += B0 dt f
// The coefficients are not printed in the paper; they are those of Yoshida's
// triple-jump composition of the second-order leapfrog: with w1 = 1/(2 - 2^{1/3})
// and w0 = -2^{1/3}/(2 - 2^{1/3}), D0 = w1, D1 = w0, B0 = w1/2, B1 = (w0 + w1)/2.
// Inside one call the end kick of a step and the start kick of the next are
// applied by the same kernel (two separate adds, same result as two stages).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "md_internal.h"

namespace md {
namespace {

constexpr int64_t kMaxPairN = int64_t(1) << 23;  // O(N^2) models
constexpr int64_t kMaxHmfN = int64_t(1) << 30;   // O(N) model
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool prec_ok(int model, int prec)
{
    if (model == MD_HMF) return prec == MD_FP64 || prec == MD_MIXED_F32STATE;
    if (model == MD_RING || model == MD_GRAV2D) return prec >= MD_FP64 && prec <= MD_MIXED_PAIRF64;
    return false;
}

bool model_ok(int model) { return model == MD_HMF || model == MD_RING || model == MD_GRAV2D; }

// The softening each pair form takes without an overflow, a non-normal number or a
// negative square-root argument in its terms, for any positions: 2D FP64 adds up to
// four terms with one reciprocal of the product of their s >= eps, which has to
// stay a normal FP64 number; the FP32 forms round eps to FP32 and divide by it (2D) or raise
// 2 eps to the -3/2 (the Ring's half-angle form); eq. 9 in FP64 forms
// u = 1 + eps - cos d, which must stay positive for two particles at the same
// angle (1 + eps is rounded to 2^-53).  MD_HMF has no softening.
bool eps_ok(int model, int prec, double eps)
{
    if (model == MD_HMF) return true;
    if (!(eps > 0.0 && isfinite(eps))) return false;
    if (model == MD_GRAV2D)
        return prec == MD_FP64 ? (eps >= MD_EPS_MIN_2D_FP64 && eps <= MD_EPS_MAX_2D_FP64)
                               : (eps >= MD_EPS_MIN_2D_FP32 && eps <= MD_EPS_MAX_FP32);
    return prec == MD_FP64 ? eps >= MD_EPS_MIN_RING_FP64 : (eps >= MD_EPS_MIN_RING_FP32 && eps <= MD_EPS_MAX_FP32);
}

// Contexts that can take the symmetric form (and carry its partial slots): Ring
// and 2D in every precision form they accept.
bool sym_capable(int model, int prec, int64_t n)
{
    return (model == MD_GRAV2D || model == MD_RING) && prec >= MD_FP64 && prec <= MD_MIXED_PAIRF64 &&
           n >= kSymMinN && n <= kSymMaxN;
}

struct Layout {
    size_t red, scal, macc, ops, wops, part, th32, p32, fops0, fops1, total;
};

Layout layout(int model, int prec, int64_t n)
{
    Layout L{};
    const size_t npad = (size_t)pad_n(n);
    size_t off = 0;
    L.red = off;
    off = align_up(off + sizeof(double) * kRedSlots);
    L.scal = off;
    off = align_up(off + sizeof(double) * 32);
    L.macc = off;
    if (model == MD_HMF) off = align_up(off + sizeof(long long) * kMWords);
    L.ops = off;
    if (model == MD_RING) off = align_up(off + 2 * npad * (prec == MD_FP64 ? sizeof(double) : sizeof(float)));
    else if (model == MD_GRAV2D && prec != MD_FP64) off = align_up(off + 2 * npad * sizeof(float));
    else if (model == MD_GRAV2D && sym_capable(model, prec, n))
        off = align_up(off + 2 * npad * sizeof(double));  // 2D FP64: the symmetric form's padded copy
    L.wops = off;
    if (model != MD_HMF && prec != MD_FP64) off = align_up(off + (size_t)dims(model) * npad * sizeof(float));
    else if (model == MD_GRAV2D && sym_capable(model, prec, n))
        off = align_up(off + 2 * npad * sizeof(double));  // 2D FP64: the symmetric product's padded vector
    L.part = off;
    if (model != MD_HMF) {
        size_t slots = (size_t)max_j_split(n);
        if (sym_capable(model, prec, n)) slots = std::max(slots, npad / (size_t)sym_tile_n(model, prec, n));
        off = align_up(off + slots * dims(model) * npad * sizeof(double));
    }
    L.th32 = off;
    if (model == MD_HMF && prec == MD_MIXED_F32STATE) off = align_up(off + npad * sizeof(float));
    L.p32 = off;
    if (model == MD_HMF && prec == MD_MIXED_F32STATE) off = align_up(off + npad * sizeof(float));
    const bool fused = model != MD_HMF && n <= kFusedMaxN;
    L.fops0 = off;
    if (fused) off = align_up(off + 2 * npad * sizeof(double));
    L.fops1 = off;
    if (fused) off = align_up(off + 2 * npad * sizeof(double));
    L.total = off;
    return L;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

int fail(md_ctx *c, int status, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(md_ctx *c, int status, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return status;
}

int dev_fail(md_ctx *c, hipError_t e, const char *what)
{
    return fail(c, MD_EDEVICE, "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

// Makes the context's device current for the scope of one call.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void yoshida(double *b0, double *b1, double *d0, double *d1)
{
    const double cb = cbrt(2.0);
    const double w1 = 1.0 / (2.0 - cb);
    const double w0 = -cb / (2.0 - cb);
    *d0 = w1;
    *d1 = w0;
    *b0 = 0.5 * w1;
    *b1 = 0.5 * (w0 + w1);
}

#define MD_TRY(expr, what)                        \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return dev_fail(c, e_, what); \
    } while (0)

// Pair partials and update stage of a single system or a batched ensemble.
hipError_t pair_(md_ctx *c, const double *q) { return c->batch ? batch_pair(c, q) : launch_pair(c, q); }

// snap (single systems only): the positions after every drift are also written to
// consecutive [d][n] slots of snap, snap_stride doubles apart.
hipError_t update_(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p, double *f,
                   double *snap = nullptr)
{
    return c->batch ? batch_update(c, flags, kick1, kick2, drift, q, p, f)
                    : launch_update(c, flags, kick1, kick2, drift, q, p, f, snap);
}

// The fused stage applies: single system with its operand buffers, and tiles
// whose j ranges fit one block's wavefronts and LDS.
bool fused_ok(const md_ctx *c, const Tiles &t)
{
    if (c->batch || c->model == MD_HMF || !c->fops[0]) return false;
    const int S = t.jsplit / fused_groups(t.jsplit);
    // each wavefront's LDS slice holds its partials (i_per_lane * d * 64 doubles)
    return S <= kFusedMaxWaves && t.ipl * dims(c->model) * kWave * 8 <= kFusedLdsBytes / S;
}

bool sym_ok(const md_ctx *c) { return c->batch ? c->batch->sym : sym_capable(c->model, c->prec, c->n); }

// MD_LAUNCH_AUTO for an ensemble: the symmetric form when the realizations' tile
// pairs outnumber their diagonal tiles (small realizations gain nothing from it).
bool batch_sym_auto(const Batch &B) { return B.sym && B.n_soff >= B.n_sdiag; }

// MD_LAUNCH_AUTO takes the fused form up to this n.  Measured on MI355X, md_step
// staged (its built-in tiles) against fused (8 lane groups x 8 wavefronts), us per
// step: Ring FP64 46.8 / 46.7 at N = 4096, 72.2 / 79.3 at 5120; Ring mixed 34.8 /
// 29.6 and 48.2 / 48.9; 2D FP64 73.0 / 69.4 at 6144, 103.6 / 113.8 at 8192; 2D
// mixed 49.2 / 45.9 and 68.6 / 67.0 (the 2D forms' j terms are cheaper, so the
// fused stage's one block per 8 particles stays ahead longer).
int64_t fused_auto_n(int model) { return model == MD_GRAV2D ? kFusedAutoN2D : kFusedAutoN; }

// md_step's launch form for this context.
int form_of(const md_ctx *c)
{
    if (c->batch) {
        const bool s = c->launch == MD_LAUNCH_SYMMETRIC || (c->launch == MD_LAUNCH_AUTO && batch_sym_auto(*c->batch));
        return s && c->batch->sym ? MD_LAUNCH_SYMMETRIC : MD_LAUNCH_STAGED;
    }
    if (c->launch == MD_LAUNCH_SYMMETRIC || (c->launch == MD_LAUNCH_AUTO && c->n >= sym_auto_n(c->model, c->prec)))
        if (sym_ok(c)) return MD_LAUNCH_SYMMETRIC;
    if (c->launch == MD_LAUNCH_STAGED || c->launch == MD_LAUNCH_SYMMETRIC || !fused_ok(c, c->tiles))
        return MD_LAUNCH_STAGED;
    if (c->launch == MD_LAUNCH_FUSED || c->n <= fused_auto_n(c->model)) return MD_LAUNCH_FUSED;
    return MD_LAUNCH_STAGED;
}

int step_pairs(md_ctx *c, double *q, double *p, double *f, double dt, int64_t nsteps, double *snap = nullptr,
               size_t snap_stride = 0)
{
    double B0, B1, D0, D1;
    yoshida(&B0, &B1, &D0, &D1);
    const int stage = UPD_F_FROM_PART | UPD_STORE_F | UPD_KICK1 | UPD_DRIFT | UPD_PREP;
    int64_t slot = 0;
    auto next = [&]() { return snap ? snap + (size_t)(slot++) * snap_stride : nullptr; };
    if (form_of(c) == MD_LAUNCH_FUSED) {
        // the same stage sequence as below, pair kernel and update in one launch;
        // the operand buffers alternate
        void *const buf[2] = {c->fops[0], c->fops[1]};
        int cur = 0;
        auto fused = [&](int flags, double k1, double k2, double dr, double *sn) {
            hipError_t e = launch_fused(c, flags, k1, k2, dr, q, p, f, buf[cur], buf[cur ^ 1], sn);
            cur ^= 1;
            return e;
        };
        MD_TRY(launch_update_fused(c, UPD_KICK1 | UPD_DRIFT | UPD_PREP, B0 * dt, 0.0, D0 * dt, q, p, f, buf[0],
                                   next()),
               "step: first kick");
        for (int64_t s = 0; s < nsteps; ++s) {
            MD_TRY(fused(stage, B1 * dt, 0.0, D1 * dt, next()), "step: fused stage");
            MD_TRY(fused(stage, B1 * dt, 0.0, D0 * dt, next()), "step: fused stage");
            if (s + 1 < nsteps)
                MD_TRY(fused(stage | UPD_KICK2, B0 * dt, B0 * dt, D0 * dt, next()), "step: fused stage");
            else
                MD_TRY(fused(UPD_F_FROM_PART | UPD_STORE_F | UPD_KICK1, B0 * dt, 0.0, 0.0, nullptr),
                       "step: last kick");
        }
        return MD_OK;
    }
    MD_TRY(update_(c, UPD_KICK1 | UPD_DRIFT | UPD_PREP, B0 * dt, 0.0, D0 * dt, q, p, f, next()), "step: first kick");
    for (int64_t s = 0; s < nsteps; ++s) {
        MD_TRY(pair_(c, q), "step: pair kernel");
        MD_TRY(update_(c, stage, B1 * dt, 0.0, D1 * dt, q, p, f, next()), "step: update");
        MD_TRY(pair_(c, q), "step: pair kernel");
        MD_TRY(update_(c, stage, B1 * dt, 0.0, D0 * dt, q, p, f, next()), "step: update");
        MD_TRY(pair_(c, q), "step: pair kernel");
        if (s + 1 < nsteps)
            MD_TRY(update_(c, stage | UPD_KICK2, B0 * dt, B0 * dt, D0 * dt, q, p, f, next()), "step: update");
        else
            MD_TRY(update_(c, UPD_F_FROM_PART | UPD_STORE_F | UPD_KICK1, B0 * dt, 0.0, 0.0, q, p, f),
                   "step: last kick");
    }
    return MD_OK;
}

// Doubles per stage slot: d n rounded up to even, so a 16-byte aligned stage keeps
// every slot 16-byte aligned (the HMF pass then uses the same vector width, hence
// the same reduction order, as md_step on aligned arrays).
size_t vjp_slot(const md_ctx *c) { return ((size_t)dims(c->model) * (size_t)c->n + 1) & ~(size_t)1; }

// Reverse sweep over nsteps recorded steps: pos(m) are the positions at which the
// kicks evaluated the force (pos(0) = q0, then P_1 .. P_3n, slot doubles apart).
int reverse_pairs(md_ctx *c, const double *q0, const double *P, size_t slot, double dt, int64_t nsteps, double *lq,
                  double *lp)
{
    double B0, B1, D0, D1;
    yoshida(&B0, &B1, &D0, &D1);
    auto pos = [&](int64_t m) -> const double * { return m == 0 ? q0 : P + (size_t)(m - 1) * slot; };
    // pending product at P_3n, kick weight B0 dt
    const int prep = ADJ_PREPQ | ADJ_PREPW;
    MD_TRY(launch_adj_update(c, prep, 0.0, 0.0, 0.0, lq, lp, nullptr, pos(3 * nsteps)), "vjp: operands");
    MD_TRY(launch_hvp_pair(c, pos(3 * nsteps), lp), "vjp: hvp");
    int kick = ADJ_KICK;  // the pending product's kick(s)
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        MD_TRY(launch_adj_update(c, kick | ADJ_DRIFT | prep, B0 * dt, B0 * dt, D0 * dt, lq, lp, nullptr,
                                 pos(3 * s + 2)),
               "vjp: update");
        MD_TRY(launch_hvp_pair(c, pos(3 * s + 2), lp), "vjp: hvp");
        MD_TRY(launch_adj_update(c, ADJ_KICK | ADJ_DRIFT | prep, B1 * dt, 0.0, D1 * dt, lq, lp, nullptr,
                                 pos(3 * s + 1)),
               "vjp: update");
        MD_TRY(launch_hvp_pair(c, pos(3 * s + 1), lp), "vjp: hvp");
        MD_TRY(launch_adj_update(c, ADJ_KICK | ADJ_DRIFT | prep, B1 * dt, 0.0, D0 * dt, lq, lp, nullptr, pos(3 * s)),
               "vjp: update");
        MD_TRY(launch_hvp_pair(c, pos(3 * s), lp), "vjp: hvp");
        // the first kick of step s and the last kick of step s - 1 act at the same
        // positions with no drift between them: one product, applied as two kicks
        kick = s > 0 ? (ADJ_KICK | ADJ_KICK2) : ADJ_KICK;
    }
    MD_TRY(launch_adj_update(c, kick, B0 * dt, B0 * dt, 0.0, lq, lp, nullptr, nullptr), "vjp: last kick");
    return MD_OK;
}

// HMF reverse sweep: as reverse_pairs, with the O(N) product -- per kick one pass
// of sums over (P_m, lambda_p) and one elementwise pass that applies the kick and
// the preceding drift.
int reverse_hmf(md_ctx *c, const double *q0, const double *P, size_t slot, double dt, int64_t nsteps, double *lq,
                double *lp)
{
    double B0, B1, D0, D1;
    yoshida(&B0, &B1, &D0, &D1);
    auto pos = [&](int64_t m) -> const double * { return m == 0 ? q0 : P + (size_t)(m - 1) * slot; };
    MD_TRY(launch_hmf_hvp_sums(c, pos(3 * nsteps), lp), "vjp: sums");
    int kick = ADJ_KICK;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        MD_TRY(launch_hmf_adj_update(c, pos(3 * s + 3), kick | ADJ_DRIFT, B0 * dt, B0 * dt, D0 * dt, lq, lp, nullptr),
               "vjp: update");
        MD_TRY(launch_hmf_hvp_sums(c, pos(3 * s + 2), lp), "vjp: sums");
        MD_TRY(launch_hmf_adj_update(c, pos(3 * s + 2), ADJ_KICK | ADJ_DRIFT, B1 * dt, 0.0, D1 * dt, lq, lp, nullptr),
               "vjp: update");
        MD_TRY(launch_hmf_hvp_sums(c, pos(3 * s + 1), lp), "vjp: sums");
        MD_TRY(launch_hmf_adj_update(c, pos(3 * s + 1), ADJ_KICK | ADJ_DRIFT, B1 * dt, 0.0, D0 * dt, lq, lp, nullptr),
               "vjp: update");
        MD_TRY(launch_hmf_hvp_sums(c, pos(3 * s), lp), "vjp: sums");
        kick = s > 0 ? (ADJ_KICK | ADJ_KICK2) : ADJ_KICK;
    }
    MD_TRY(launch_hmf_adj_update(c, q0, kick, B0 * dt, B0 * dt, 0.0, lq, lp, nullptr), "vjp: last kick");
    return MD_OK;
}

// snap (FP64 state only): the angles after every drift are also written to
// consecutive slots of snap, snap_stride doubles apart.
int step_hmf(md_ctx *c, double *q, double *p, double *f, double dt, int64_t nsteps, double *snap = nullptr,
             size_t snap_stride = 0)
{
    double B0, B1, D0, D1;
    yoshida(&B0, &B1, &D0, &D1);
    const bool f32 = c->prec == MD_MIXED_F32STATE;
    const int stage = HMF_KICK_M | HMF_DRIFT | HMF_WRITE | HMF_REDUCE;
    int64_t slot = 0;
    auto next = [&]() { return snap ? snap + (size_t)(slot++) * snap_stride : nullptr; };
    if (f32) MD_TRY(launch_hmf_convert(c, q, p, true), "step: convert in");
    int k = 0;  // pass index: pass k reads the magnetization sums of pass k - 1
    MD_TRY(launch_hmf_begin(c), "step: magnetization sums");
    MD_TRY(launch_hmf_pass(c, k++, HMF_KICK_F | HMF_DRIFT | HMF_WRITE | HMF_REDUCE, B0 * dt, 0.0, D0 * dt, q, p, f,
                           nullptr, f32, next()),
           "step: first pass");
    for (int64_t s = 0; s < nsteps; ++s) {
        MD_TRY(launch_hmf_pass(c, k++, stage, B1 * dt, 0.0, D1 * dt, q, p, nullptr, nullptr, f32, next()),
               "step: pass");
        MD_TRY(launch_hmf_pass(c, k++, stage, B1 * dt, 0.0, D0 * dt, q, p, nullptr, nullptr, f32, next()),
               "step: pass");
        if (s + 1 < nsteps)
            MD_TRY(launch_hmf_pass(c, k++, stage | HMF_KICK2, B0 * dt, B0 * dt, D0 * dt, q, p, nullptr, nullptr,
                                   f32, next()),
                   "step: pass");
        else
            MD_TRY(launch_hmf_pass(c, k++, HMF_KICK_M | HMF_STORE_F | HMF_WRITE, B0 * dt, 0.0, 0.0, q, p, nullptr,
                                   f, f32),
                   "step: last pass");
    }
    if (f32) MD_TRY(launch_hmf_convert(c, q, p, false), "step: convert out");
    return MD_OK;
}

// md_step_vjp: recompute the steps from (q0, p0) into stage = [q | p | f | P_1 .. P_3n]
// (one slot each), then sweep back.
int step_vjp(md_ctx *c, const double *q0, const double *p0, double dt, int64_t nsteps, double *lq, double *lp,
             double *stage)
{
    const size_t len = (size_t)dims(c->model) * c->n, slot = vjp_slot(c);
    double *qw = stage, *pw = stage + slot, *fw = stage + 2 * slot, *P = stage + 3 * slot;
    MD_TRY(hipMemcpyAsync(qw, q0, len * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "vjp: copy q");
    MD_TRY(hipMemcpyAsync(pw, p0, len * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "vjp: copy p");
    int st;
    if (c->model == MD_HMF) {
        MD_TRY(launch_hmf_begin(c), "vjp: magnetization sums");
        MD_TRY(launch_hmf_pass(c, 0, HMF_REDUCE, 0.0, 0.0, 0.0, qw, nullptr, nullptr, nullptr, false),
               "vjp: reduce");
        MD_TRY(launch_hmf_pass(c, 1, HMF_STORE_F, 0.0, 0.0, 0.0, qw, nullptr, nullptr, fw, false), "vjp: force");
        st = step_hmf(c, qw, pw, fw, dt, nsteps, P, slot);
        if (st != MD_OK) return st;
        return reverse_hmf(c, q0, P, slot, dt, nsteps, lq, lp);
    }
    MD_TRY(update_(c, UPD_PREP, 0.0, 0.0, 0.0, qw, nullptr, nullptr), "vjp: operands");
    MD_TRY(pair_(c, qw), "vjp: pair kernel");
    MD_TRY(update_(c, UPD_F_FROM_PART | UPD_STORE_F, 0.0, 0.0, 0.0, qw, nullptr, fw), "vjp: force");
    st = step_pairs(c, qw, pw, fw, dt, nsteps, P, slot);
    if (st != MD_OK) return st;
    return reverse_pairs(c, q0, P, slot, dt, nsteps, lq, lp);
}

// ------------------------------------------------------------ batched ensembles --

constexpr int64_t kMaxBatchTotal = int64_t(1) << 24;  // particles over all realizations
constexpr int kBatchMaxSplit = 32;
constexpr int kERowsI = 256;    // energy items: i rows per block
constexpr int kEChunk = 2048;   // energy items: j per block

int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// j-chunk length for j_split pieces of the largest realization (a multiple of 64).
int64_t batch_chunk(const Batch &B, int jsplit) { return div_up(div_up(B.nmax, jsplit), 64) * 64; }

// Validates the ensemble description and fills the tile-independent parts of B.
int make_batch(int model, int prec, int nb, const int64_t *off, const double *eps, Batch &B)
{
    if (nb < 1 || !off || !eps) return MD_EINVAL;
    if (off[0] != 0) return MD_EINVAL;
    B.nb = nb;
    B.off.assign(off, off + nb + 1);
    B.eps.assign(eps, eps + nb);
    B.pref.resize(nb);
    B.nmax = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t n = off[b + 1] - off[b];
        if (n < 1 || off[b + 1] > kMaxBatchTotal) return MD_EINVAL;
        if (!eps_ok(model, prec, eps[b])) return MD_EINVAL;
        if (n > B.nmax) B.nmax = n;
        B.pref[b] = force_prefactor(model, prec, n);
    }
    int64_t sm = B.nmax / 64;
    B.smax = (int)(sm < 1 ? 1 : (sm > kBatchMaxSplit ? kBatchMaxSplit : sm));
    // rows (their S_b is set by build_lists), energy items and their ranges
    B.n_rows = 0;
    B.roff.assign(nb + 1, 0);
    B.eitems.clear();
    B.eoff.assign(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        B.roff[b] = B.n_rows;
        B.eoff[b] = (int)(B.eitems.size() / 8);
        const int64_t o = off[b], n = off[b + 1] - off[b];
        B.n_rows += (int)div_up(n, 256);
        for (int64_t i0 = o; i0 < o + n; i0 += kERowsI) {
            const int64_t i1 = i0 + kERowsI < o + n ? i0 + kERowsI : o + n;
            for (int64_t j0 = o; j0 < o + n; j0 += kEChunk) {
                const int64_t j1 = j0 + kEChunk < o + n ? j0 + kEChunk : o + n;
                if (j1 <= i0 + 1) continue;  // no pair with j > i
                const int it[8] = {b, (int)i0, (int)i1, 0, (int)j0, (int)j1, 0, 0};
                B.eitems.insert(B.eitems.end(), it, it + 8);
            }
        }
    }
    B.roff[nb] = B.n_rows;
    B.n_eitems = (int)(B.eitems.size() / 8);
    B.eoff[nb] = B.n_eitems;
    // symmetric form: every realization within the single-system limits, slots within 4 GiB
    const bool sym_prec = model == MD_RING ? (prec == MD_MIXED || prec == MD_MIXED_KAHAN || prec == MD_FP64)
                                           : (prec == MD_MIXED || prec == MD_MIXED_KAHAN);
    B.tmax = (int)div_up(B.nmax, kBatchSymTile);
    const size_t sym_slot_bytes = (size_t)B.tmax * dims(model) * (size_t)pad_n(off[nb]) * sizeof(double);
    B.sym = sym_prec && B.nmax <= kSymMaxN && sym_slot_bytes <= (size_t(1) << 32);
    B.sitems.clear();
    B.srows.clear();
    B.n_soff = B.n_sdiag = 0;
    if (B.sym) {
        std::vector<int> diag;
        for (int b = 0; b < nb; ++b) {
            const int64_t o = off[b], n = off[b + 1] - off[b];
            const int T = (int)div_up(n, kBatchSymTile);
            for (int ta = 0; ta < T; ++ta) {
                const int ia = (int)(o + (int64_t)ta * kBatchSymTile);
                for (int tb = ta + 1; tb < T; ++tb) {
                    const int it[8] = {b, ia, (int)(o + n), tb, (int)(o + (int64_t)tb * kBatchSymTile), (int)(o + n), ta, 0};
                    B.sitems.insert(B.sitems.end(), it, it + 8);
                }
                const int dg[8] = {b, ia, (int)(o + n), ta, ia, (int)(o + n), ta, 0};
                diag.insert(diag.end(), dg, dg + 8);
            }
            for (int64_t i0 = o; i0 < o + n; i0 += 256) {
                const int r[4] = {b, (int)i0, (int)(i0 + 256 < o + n ? i0 + 256 : o + n), T};
                B.srows.insert(B.srows.end(), r, r + 4);
            }
        }
        B.n_soff = (int)(B.sitems.size() / 8);
        B.n_sdiag = (int)(diag.size() / 8);
        B.sitems.insert(B.sitems.end(), diag.begin(), diag.end());
    }
    // largest pair-item count over all tile choices: 64-particle i blocks, smax pieces
    const int64_t cmin = batch_chunk(B, B.smax);
    int64_t mx = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t n = off[b + 1] - off[b];
        mx += div_up(n, 64) * div_up(n, cmin);
    }
    B.max_items = (int)mx;
    return MD_OK;
}

// Pair items for the current tiles (largest first) and the rows' chunk counts.
void build_lists(Batch &B, const Tiles &t)
{
    const int64_t chunk = batch_chunk(B, t.jsplit);
    const int64_t iblock = (int64_t)kWave * t.ipl * t.waves;
    struct Item {
        int64_t cost;
        int v[8];
    };
    std::vector<Item> items;
    B.rows.clear();
    for (int b = 0; b < B.nb; ++b) {
        const int64_t o = B.off[b], n = B.off[b + 1] - B.off[b];
        const int S = (int)div_up(n, chunk);
        for (int64_t i0 = o; i0 < o + n; i0 += 256) {
            const int r[4] = {b, (int)i0, (int)(i0 + 256 < o + n ? i0 + 256 : o + n), S};
            B.rows.insert(B.rows.end(), r, r + 4);
        }
        for (int64_t i0 = o; i0 < o + n; i0 += iblock) {
            const int64_t i1 = i0 + iblock < o + n ? i0 + iblock : o + n;
            for (int s = 0; s < S; ++s) {
                const int64_t j0 = o + s * chunk;
                const int64_t j1 = j0 + chunk < o + n ? j0 + chunk : o + n;
                items.push_back({(i1 - i0) * (j1 - j0), {b, (int)i0, (int)i1, s, (int)j0, (int)j1, 0, 0}});
            }
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
    B.items.resize(items.size() * 8);
    for (size_t k = 0; k < items.size(); ++k)
        for (int m = 0; m < 8; ++m) B.items[k * 8 + m] = items[k].v[m];
    B.n_items = (int)items.size();
}

struct BatchLayout {
    size_t scal, ops, part, items, rows, eitems, eps, pref, ered, kred, eoff, roff, off, sitems, srows, total;
};

BatchLayout batch_layout(int model, int prec, const Batch &B)
{
    BatchLayout L{};
    const size_t npad = (size_t)pad_n(B.off[B.nb]);
    const int d = dims(model);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.scal = take(sizeof(double) * 32);
    size_t ops = 0;
    if (model == MD_RING) ops = 2 * npad * (prec == MD_FP64 ? sizeof(double) : sizeof(float));
    else if (prec != MD_FP64) ops = 2 * npad * sizeof(float);
    L.ops = take(ops);
    L.part = take((size_t)std::max(B.smax, B.sym ? B.tmax : 0) * d * npad * sizeof(double));
    L.items = take((size_t)B.max_items * 8 * sizeof(int));
    L.rows = take((size_t)B.n_rows * 4 * sizeof(int));
    L.eitems = take((size_t)B.n_eitems * 8 * sizeof(int));
    L.eps = take(B.nb * sizeof(double));
    L.pref = take(B.nb * sizeof(double));
    L.ered = take((size_t)B.n_eitems * sizeof(double));
    L.kred = take((size_t)B.n_rows * sizeof(double));
    L.eoff = take((B.nb + 1) * sizeof(int));
    L.roff = take((B.nb + 1) * sizeof(int));
    L.off = take((B.nb + 1) * sizeof(int64_t));
    L.sitems = take(B.sitems.size() * sizeof(int));
    L.srows = take(B.srows.size() * sizeof(int));
    L.total = o;
    return L;
}

Tiles batch_default_tiles(const Batch &B)
{
    Tiles t;
    t.ipl = 1;
    t.waves = 4;
    t.jsplit = B.smax < 8 ? B.smax : 8;
    t.jtile = 128;
    return t;
}

// Uploads the tile-dependent lists (pair items, rows).
hipError_t upload_lists(md_ctx *c)
{
    Batch &B = *c->batch;
    hipError_t e = hipMemcpyAsync(B.d_items, B.items.data(), B.items.size() * sizeof(int), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.d_rows, B.rows.data(), B.rows.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    return e;
}

}  // namespace

int64_t pad_n(int64_t n) { return (n + kSymTile - 1) / kSymTile * kSymTile; }

// Smaller tiles in the symmetric form of single systems below a size: a block's
// tile pair is a serial unit of work (its wavefronts hold their i for the whole j
// tile), so with few tile pairs the launch is as long as a block's round.  Tiles
// of 256 (one wavefront a block) give 16 times the tile pairs of 1024-tiles at a
// sixteenth of the work each, tiles of 512 (two wavefronts) four times.  Measured
// md_step, us per step (MI355X), 256- / 512- / 1024-tiles where measured:
//   2D mixed: N = 32,768 419 / 480 / 562; 49,152 842 / 1005 / 933; 65,536 1434 /
//     1613 / 1509; 98,304 3195 / 3218 / 3174;
//   2D FP64: 32,768 788 / 821 / 931; 65,536 2930 / 2943 / 2978; 98,304 6639 / 6376 /
//     6392;
//   2D Kahan: 49,152 1586 / 1705 / 1780; 65,536 2747 / 2754 / 2800; 98,304 6227 / -
//     / 6009;
//   Ring mixed: 49,152 1001 / 1090 / 1154; 131,072 6563 / 6651 / 6710; 196,608
//     14,736 / - / 14,596;
//   Ring FP64: 65,536 3464 / 3532 / 3646; 98,304 7677 / 7649 / 7709; 131,072 13,597
//     / 13,459 / 13,403 (the 1024 figure from another box);
//   Ring Kahan: 65,536 2262 / 2319 / -; 131,072 8849 / 8741 / -.
int sym_tile_n(int model, int prec, int64_t n)
{
    (void)prec;
    if (n <= 65536) return 256;
    return model == MD_RING && n <= 131072 ? kSymTileSmall : kSymTile;
}

int launch_form(const md_ctx *c) { return form_of(c); }

int dims(int model) { return model == MD_GRAV2D ? 2 : 1; }

int max_j_split(int64_t n)
{
    if (n < 1) return 1;
    int64_t s = (int64_t(1) << 22) / n;
    if (s > kMaxJSplit) s = kMaxJSplit;
    return s < 1 ? 1 : (int)s;
}

// Built-in tile choice (measured on MI355X, md_step at N = 512 .. 262144): the
// pair kernels are VALU-issue bound at large N, so the aim there is enough
// independent wavefronts (several rounds of 8 per SIMD over 1024 SIMDs, which
// evens out the tail) while each block keeps a j range long enough to amortise
// its i loads and its output; below that, fixed choices found by the autotuner.
Tiles default_tiles(int model, int prec, int64_t n)
{
    (void)prec;
    Tiles t;
    t.waves = 4;
    t.jtile = 128;
    if (n <= fused_auto_n(model)) {
        // the automatic fused launch: the most j ranges (8 lane groups x 8 wavefronts
        // per block) measured fastest from N = 512 to 4096 (above fused_auto_n the
        // staged form with the tiles below is faster)
        t.ipl = 1;
        t.jsplit = max_j_split(n) < 64 ? max_j_split(n) : 64;
        return t;
    }
    t.ipl = n >= 65536 ? 2 : 1;
    if (n < 131072) {
        // staged, N = 4097 .. 131071: 32 j ranges measured best or within 3% for both
        // models and both precisions (autotuner at N = 51200, 102400; N = 4096 to 8192
        // against 16 and 64 j ranges and two i per lane); 64 j ranges measured 1.4-3.5%
        // faster at N = 10240 and 20480 and up to 2.6% faster (2D FP64 level) from 24576
        // to 40960, every model and precision, since the update adds the slots 16
        // loads at a time
        const int js = (n > 8192 && n <= 40960) ? 64 : 32;
        t.jsplit = max_j_split(n) < js ? max_j_split(n) : js;
        return t;
    }
    const int64_t wi = (n + kWave * t.ipl - 1) / (kWave * t.ipl);
    const int64_t target = n >= 65536 ? 32768 : 16384;
    int64_t s = target / wi;
    int64_t cap = n > 2048 ? n / 128 : n / 64;
    if (cap > max_j_split(n)) cap = max_j_split(n);
    if (s > cap) s = cap;
    int64_t p2 = 1;
    while (p2 * 2 <= s) p2 *= 2;
    t.jsplit = (int)p2;
    return t;
}

Timing::~Timing()
{
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
}

int timed_begin(md_ctx *c, const char *kernel)
{
    Timing *t = c->timing;
    if (!t || 2 * (size_t)(t->used + 1) > t->ev.size()) return -1;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->stream, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return -1;
    if (hipEventRecord(t->ev[2 * (size_t)t->used], c->stream) != hipSuccess) return -1;
    t->kernel = kernel;
    return t->used++;
}

void timed_end(md_ctx *c, int slot)
{
    if (slot >= 0 && c->timing) (void)hipEventRecord(c->timing->ev[2 * (size_t)slot + 1], c->stream);
}

// ---- the force without a caller's workspace (md_force_noalloc) ----
//
// The workspace lives in `scratch`, a file-scope device array: every GPU the
// library runs on holds its own copy, at its own address, from module load to
// process end.  In host code the array's name is only a stand-in for that
// address, so host code never passes it: the first md_force_noalloc call on a
// device looks the device's address up (hipGetSymbolAddress, with that device
// current) and keeps it; every later call on the device uses the kept address.
static __device__ __align__(256) char scratch[MD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device, once looked up

// The address of the current device's `scratch` (dev = the current device).
hipError_t scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr || ((uintptr_t)ptr % kAlign) != 0) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// What md_force reads and writes besides q and f, in the staged form with
// `jsplit` j ranges: the context's carve-up without the symmetric form's slots,
// the fused stage's operand buffers, the HVP vector and the HMF FP32 state,
// which md_force does not touch.
struct ForceLayout {
    size_t red, scal, macc, ops, part, total;
};

ForceLayout force_layout(int model, int prec, int64_t n, int jsplit)
{
    ForceLayout L{};
    const size_t npad = (size_t)pad_n(n);
    size_t off = 0;
    L.red = off;
    off = align_up(off + sizeof(double) * kRedSlots);
    L.scal = off;
    off = align_up(off + sizeof(double) * 32);
    L.macc = off;
    if (model == MD_HMF) off = align_up(off + sizeof(long long) * kMWords);
    L.ops = off;
    if (model == MD_RING) off = align_up(off + 2 * npad * (prec == MD_FP64 ? sizeof(double) : sizeof(float)));
    else if (model == MD_GRAV2D && prec != MD_FP64) off = align_up(off + 2 * npad * sizeof(float));
    L.part = off;
    if (model != MD_HMF) off = align_up(off + (size_t)jsplit * dims(model) * npad * sizeof(double));
    L.total = off;
    return L;
}

}  // namespace
}  // namespace md

using namespace md;

extern "C" {

size_t md_workspace_bytes(int model, int prec, int64_t n)
{
    if (!model_ok(model) || !prec_ok(model, prec) || n < 1) return 0;
    if (n > (model == MD_HMF ? kMaxHmfN : kMaxPairN)) return 0;
    return layout(model, prec, n).total;
}

int md_max_j_split(int64_t n) { return max_j_split(n); }

int md_init(md_ctx **out, int model, int prec, int64_t n, double eps, void *hip_stream, void *workspace,
            size_t workspace_bytes)
{
    if (!out) return MD_EINVAL;
    *out = nullptr;
    if (!model_ok(model) || n < 1 || n > (model == MD_HMF ? kMaxHmfN : kMaxPairN)) return MD_EINVAL;
    if (!prec_ok(model, prec)) return MD_EUNSUPPORTED;
    if (!eps_ok(model, prec, eps)) return MD_EINVAL;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return MD_EINVAL;
    const Layout L = layout(model, prec, n);
    if (workspace_bytes < L.total) return MD_ENOMEM;

    md_ctx *c = new (std::nothrow) md_ctx();
    if (!c) return MD_ENOMEM;
    c->model = model;
    c->prec = prec;
    c->n = n;
    c->npad = pad_n(n);
    c->eps = model == MD_HMF ? 0.0 : eps;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char *>(workspace);
    c->ws_bytes = workspace_bytes;
    c->red = reinterpret_cast<double *>(c->ws + L.red);
    c->scal = reinterpret_cast<double *>(c->ws + L.scal);
    c->macc = (L.ops > L.macc) ? reinterpret_cast<long long *>(c->ws + L.macc) : nullptr;
    c->ops = (L.wops > L.ops) ? static_cast<void *>(c->ws + L.ops) : nullptr;
    c->wops = (L.part > L.wops) ? static_cast<void *>(c->ws + L.wops) : nullptr;
    c->part = (L.th32 > L.part) ? reinterpret_cast<double *>(c->ws + L.part) : nullptr;
    c->th32 = (L.p32 > L.th32) ? reinterpret_cast<float *>(c->ws + L.th32) : nullptr;
    c->p32 = (L.fops0 > L.p32) ? reinterpret_cast<float *>(c->ws + L.p32) : nullptr;
    if (L.total > L.fops0) {
        c->fops[0] = c->ws + L.fops0;
        c->fops[1] = c->ws + L.fops1;
    }
    c->tiles = default_tiles(model, prec, n);
    hipError_t e = hipGetDevice(&c->dev);
    if (e != hipSuccess) {
        delete c;
        return MD_EDEVICE;
    }
    *out = c;
    return MD_OK;
}

size_t md_batch_workspace_bytes(int model, int prec, int nb, const int64_t *offsets, const double *eps)
{
    if (!(model == MD_RING || model == MD_GRAV2D) || !prec_ok(model, prec)) return 0;
    Batch B;
    if (make_batch(model, prec, nb, offsets, eps, B) != MD_OK) return 0;
    return batch_layout(model, prec, B).total;
}

int md_batch_init(md_ctx **out, int model, int prec, int nb, const int64_t *offsets, const double *eps,
                  void *hip_stream, void *workspace, size_t workspace_bytes)
{
    if (!out) return MD_EINVAL;
    *out = nullptr;
    if (!model_ok(model)) return MD_EINVAL;
    if (model == MD_HMF || !prec_ok(model, prec)) return MD_EUNSUPPORTED;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return MD_EINVAL;
    Batch *B = new (std::nothrow) Batch();
    if (!B) return MD_ENOMEM;
    int st = make_batch(model, prec, nb, offsets, eps, *B);
    if (st != MD_OK) {
        delete B;
        return st;
    }
    const BatchLayout L = batch_layout(model, prec, *B);
    if (workspace_bytes < L.total) {
        delete B;
        return MD_ENOMEM;
    }
    md_ctx *c = new (std::nothrow) md_ctx();
    if (!c) {
        delete B;
        return MD_ENOMEM;
    }
    c->batch = B;
    c->model = model;
    c->prec = prec;
    c->n = B->off[nb];
    c->npad = pad_n(c->n);
    c->eps = B->eps[0];
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char *>(workspace);
    c->ws_bytes = workspace_bytes;
    c->scal = reinterpret_cast<double *>(c->ws + L.scal);
    c->ops = L.part > L.ops ? static_cast<void *>(c->ws + L.ops) : nullptr;
    c->part = reinterpret_cast<double *>(c->ws + L.part);
    B->d_items = c->ws + L.items;
    B->d_rows = c->ws + L.rows;
    B->d_eitems = c->ws + L.eitems;
    B->d_eps = reinterpret_cast<double *>(c->ws + L.eps);
    B->d_pref = reinterpret_cast<double *>(c->ws + L.pref);
    B->d_ered = reinterpret_cast<double *>(c->ws + L.ered);
    B->d_kred = reinterpret_cast<double *>(c->ws + L.kred);
    B->d_eoff = reinterpret_cast<int *>(c->ws + L.eoff);
    B->d_roff = reinterpret_cast<int *>(c->ws + L.roff);
    B->d_off = reinterpret_cast<int64_t *>(c->ws + L.off);
    B->d_sitems = c->ws + L.sitems;
    B->d_srows = c->ws + L.srows;
    c->tiles = batch_default_tiles(*B);
    build_lists(*B, c->tiles);
    hipError_t e = hipGetDevice(&c->dev);
    const hipMemcpyKind h2d = hipMemcpyHostToDevice;
    if (e == hipSuccess) e = upload_lists(c);
    if (e == hipSuccess && B->n_eitems > 0)
        e = hipMemcpyAsync(B->d_eitems, B->eitems.data(), B->eitems.size() * sizeof(int), h2d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B->d_eps, B->eps.data(), nb * sizeof(double), h2d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B->d_pref, B->pref.data(), nb * sizeof(double), h2d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B->d_eoff, B->eoff.data(), (nb + 1) * sizeof(int), h2d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B->d_roff, B->roff.data(), (nb + 1) * sizeof(int), h2d, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(B->d_off, B->off.data(), (nb + 1) * sizeof(int64_t), h2d, c->stream);
    if (e == hipSuccess && !B->sitems.empty())
        e = hipMemcpyAsync(B->d_sitems, B->sitems.data(), B->sitems.size() * sizeof(int), h2d, c->stream);
    if (e == hipSuccess && !B->srows.empty())
        e = hipMemcpyAsync(B->d_srows, B->srows.data(), B->srows.size() * sizeof(int), h2d, c->stream);
    if (e != hipSuccess) {
        delete c;
        return MD_EDEVICE;
    }
    *out = c;
    return MD_OK;
}

int md_batch_size(const md_ctx *c) { return c ? (c->batch ? c->batch->nb : 1) : 0; }

int md_set_stream(md_ctx *c, void *hip_stream)
{
    if (!c) return MD_EINVAL;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return MD_OK;
}

int md_set_tiles(md_ctx *c, int i_per_lane, int waves, int j_split, int j_tile)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    const Tiles d = c->batch ? batch_default_tiles(*c->batch) : default_tiles(c->model, c->prec, c->n);
    const int smax = c->batch ? c->batch->smax : max_j_split(c->n);
    Tiles t;
    t.ipl = i_per_lane ? i_per_lane : d.ipl;
    t.waves = waves ? waves : d.waves;
    t.jsplit = j_split ? j_split : d.jsplit;
    t.jtile = j_tile ? j_tile : d.jtile;
    if (t.ipl != 1 && t.ipl != 2 && t.ipl != 4)
        return fail(c, MD_EUNSUPPORTED, "i_per_lane must be 1, 2 or 4 (got %d)", t.ipl);
    if (t.waves != 1 && t.waves != 2 && t.waves != 4)
        return fail(c, MD_EUNSUPPORTED, "waves must be 1, 2 or 4 (got %d)", t.waves);
    if (t.jsplit < 1 || t.jsplit > smax)
        return fail(c, MD_EINVAL, "j_split must be in [1, %d] (got %d)", smax, t.jsplit);
    if (t.jtile < 16 || t.jtile > 4096 || t.jtile % 16)
        return fail(c, MD_EINVAL, "j_tile must be a multiple of 16 in [16, 4096] (got %d)", t.jtile);
    if (c->launch == MD_LAUNCH_FUSED && !fused_ok(c, t))
        return fail(c, MD_EUNSUPPORTED, "the fused launch needs j_split / (lane groups) <= %d wavefronts and "
                    "i_per_lane * d * 512 <= %d / wavefronts LDS bytes", kFusedMaxWaves, kFusedLdsBytes);
    c->tiles = t;
    if (c->batch) {
        build_lists(*c->batch, t);
        DeviceGuard g(c->dev);
        if (g.err != hipSuccess) return dev_fail(c, g.err, "md_set_tiles: set device");
        MD_TRY(upload_lists(c), "md_set_tiles: upload work lists");
    }
    return MD_OK;
}

int md_set_launch(md_ctx *c, int mode)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (mode != MD_LAUNCH_AUTO && mode != MD_LAUNCH_STAGED && mode != MD_LAUNCH_FUSED &&
        mode != MD_LAUNCH_SYMMETRIC)
        return fail(c, MD_EINVAL, "md_set_launch: unknown mode %d", mode);
    if (mode == MD_LAUNCH_SYMMETRIC && !sym_ok(c))
        return fail(c, MD_EUNSUPPORTED,
                    "md_set_launch: the symmetric launch needs a 2D or Ring system, %lld <= n <= %lld (ensembles: "
                    "MD_MIXED, MD_MIXED_KAHAN, Ring MD_FP64, every N_b <= %lld)",
                    (long long)kSymMinN, (long long)kSymMaxN, (long long)kSymMaxN);
    if (mode == MD_LAUNCH_FUSED && !fused_ok(c, c->tiles))
        return fail(c, MD_EUNSUPPORTED,
                    "md_set_launch: the fused launch needs a single Ring or 2D system with n <= %lld and tiles it "
                    "can hold (j_split / lane groups <= %d wavefronts, their partials within %d LDS bytes)",
                    (long long)kFusedMaxN, kFusedMaxWaves, kFusedLdsBytes);
    c->launch = mode;
    return MD_OK;
}

int md_get_launch(const md_ctx *c)
{
    if (!c) return MD_EINVAL;
    if (c->model == MD_HMF) return MD_LAUNCH_STAGED;
    return form_of(c);
}

int md_get_sym_tile(const md_ctx *c)
{
    if (!c) return MD_EINVAL;
    if (c->model == MD_HMF || form_of(c) != MD_LAUNCH_SYMMETRIC) return 0;
    return c->batch ? kBatchSymTile : sym_tile_n(c->model, c->prec, c->n);
}

int md_get_tiles(const md_ctx *c, int *out4)
{
    if (!c || !out4) return MD_EINVAL;
    out4[0] = c->tiles.ipl;
    out4[1] = c->tiles.waves;
    out4[2] = c->tiles.jsplit;
    out4[3] = c->tiles.jtile;
    return MD_OK;
}

int md_force(md_ctx *c, const double *q, double *f)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (!q || !f || !aligned8(q) || !aligned8(f)) return fail(c, MD_EINVAL, "md_force: null or misaligned pointer");
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_force: set device");
    double *qm = const_cast<double *>(q);
    if (c->model == MD_HMF) {
        MD_TRY(launch_hmf_begin(c), "force: magnetization sums");
        MD_TRY(launch_hmf_pass(c, 0, HMF_REDUCE, 0.0, 0.0, 0.0, qm, nullptr, nullptr, nullptr, false),
               "force: reduce");
        MD_TRY(launch_hmf_pass(c, 1, HMF_STORE_F, 0.0, 0.0, 0.0, qm, nullptr, nullptr, f, false), "force: store");
        c->forced = true;
        return MD_OK;
    }
    MD_TRY(update_(c, UPD_PREP, 0.0, 0.0, 0.0, qm, nullptr, nullptr), "force: operands");
    MD_TRY(pair_(c, q), "force: pair kernel");
    MD_TRY(update_(c, UPD_F_FROM_PART | UPD_STORE_F, 0.0, 0.0, 0.0, qm, nullptr, f), "force: combine");
    c->forced = true;
    return MD_OK;
}

int md_step(md_ctx *c, double *q, double *p, double *f, double dt, int64_t nsteps)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (!q || !p || !f || !aligned8(q) || !aligned8(p) || !aligned8(f))
        return fail(c, MD_EINVAL, "md_step: null or misaligned pointer");
    if (!isfinite(dt)) return fail(c, MD_EINVAL, "md_step: dt must be finite");
    if (nsteps < 0) return fail(c, MD_EINVAL, "md_step: nsteps must be >= 0");
    if (nsteps == 0) return MD_OK;
    if (!c->forced) return fail(c, MD_ESTATE, "md_step: f must hold force(q): call md_force on this context first");
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_step: set device");
    return c->model == MD_HMF ? step_hmf(c, q, p, f, dt, nsteps) : step_pairs(c, q, p, f, dt, nsteps);
}

int md_energy(md_ctx *c, const double *q, const double *p, double *out_dev3)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (!q || !p || !out_dev3 || !aligned8(q) || !aligned8(p) || !aligned8(out_dev3))
        return fail(c, MD_EINVAL, "md_energy: null or misaligned pointer");
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_energy: set device");
    MD_TRY(c->batch ? batch_energy(c, q, p, out_dev3) : launch_energy(c, q, p, out_dev3), "energy");
    MD_TRY(launch_finite_flag(c, out_dev3, 3 * (c->batch ? c->batch->nb : 1)), "energy: finiteness");
    c->checkable = true;
    return MD_OK;
}

int md_magnetization(md_ctx *c, const double *q, double *out_dev2)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (c->model != MD_HMF) return fail(c, MD_EUNSUPPORTED, "md_magnetization: HMF contexts only");
    if (!q || !out_dev2 || !aligned8(q) || !aligned8(out_dev2))
        return fail(c, MD_EINVAL, "md_magnetization: null or misaligned pointer");
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_magnetization: set device");
    MD_TRY(launch_magnetization(c, q, out_dev2), "magnetization");
    // M is finite exactly when the pass's FP64 block partials are: the fixed-point
    // sums of small grids turn a NaN partial into some finite integer, so the
    // partials, not the output, decide
    MD_TRY(launch_finite_flag(c, hmf_partials(c), 2 * hmf_grid(c->n)), "magnetization: finiteness");
    c->checkable = true;
    return MD_OK;
}

int md_check(md_ctx *c)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (!c->checkable) return fail(c, MD_ESTATE, "md_check: no md_energy or md_magnetization on this context yet");
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_check: set device");
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    MD_TRY(hipStreamIsCapturing(c->stream, &st), "md_check: capture status");
    if (st != hipStreamCaptureStatusNone) return fail(c, MD_ESTATE, "md_check: the stream is being captured");
    unsigned flag = 0;
    MD_TRY(hipMemcpyAsync(&flag, finite_flag(c), sizeof flag, hipMemcpyDeviceToHost, c->stream), "md_check: read");
    MD_TRY(hipStreamSynchronize(c->stream), "md_check: wait");
    if (flag) return fail(c, MD_ENONFINITE, "md_check: the last energies or magnetization were not finite");
    return MD_OK;
}

int md_hvp(md_ctx *c, const double *q, const double *w, double *out)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (c->batch) return fail(c, MD_EUNSUPPORTED, "md_hvp: single systems only");
    if (!q || !w || !out || !aligned8(q) || !aligned8(w) || !aligned8(out))
        return fail(c, MD_EINVAL, "md_hvp: null or misaligned pointer");
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_hvp: set device");
    double *wm = const_cast<double *>(w);
    if (c->model == MD_HMF) {
        MD_TRY(launch_hmf_hvp_sums(c, q, w), "hvp: sums");
        MD_TRY(launch_hmf_adj_update(c, q, ADJ_OUT, 0.0, 0.0, 0.0, nullptr, wm, out), "hvp: product");
        return MD_OK;
    }
    MD_TRY(launch_adj_update(c, ADJ_PREPQ | ADJ_PREPW, 0.0, 0.0, 0.0, nullptr, wm, nullptr, q), "hvp: operands");
    MD_TRY(launch_hvp_pair(c, q, w), "hvp: pair kernel");
    MD_TRY(launch_adj_update(c, ADJ_OUT, 0.0, 0.0, 0.0, nullptr, nullptr, out, nullptr), "hvp: combine");
    return MD_OK;
}

size_t md_vjp_stage_bytes(const md_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0) return 0;
    return (size_t)(3 * nsteps + 3) * vjp_slot(c) * sizeof(double);
}

int md_step_vjp(md_ctx *c, const double *q0, const double *p0, double dt, int64_t nsteps, double *lam_q,
                double *lam_p, double *stage, size_t stage_bytes)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (c->batch) return fail(c, MD_EUNSUPPORTED, "md_step_vjp: single systems only");
    if (c->model == MD_HMF && c->prec != MD_FP64)
        return fail(c, MD_EUNSUPPORTED, "md_step_vjp: HMF needs an FP64-state context");
    if (!q0 || !p0 || !lam_q || !lam_p || !stage || !aligned8(q0) || !aligned8(p0) || !aligned8(lam_q) ||
        !aligned8(lam_p) || !aligned8(stage))
        return fail(c, MD_EINVAL, "md_step_vjp: null or misaligned pointer");
    if (!isfinite(dt)) return fail(c, MD_EINVAL, "md_step_vjp: dt must be finite");
    if (nsteps < 0) return fail(c, MD_EINVAL, "md_step_vjp: nsteps must be >= 0");
    if (stage_bytes < md_vjp_stage_bytes(c, nsteps))
        return fail(c, MD_ENOMEM, "md_step_vjp: stage buffer needs %zu bytes", md_vjp_stage_bytes(c, nsteps));
    if (nsteps == 0) return MD_OK;
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_step_vjp: set device");
    return step_vjp(c, q0, p0, dt, nsteps, lam_q, lam_p, stage);
}

size_t md_record_stage_bytes(const md_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0) return 0;
    return (size_t)(3 * nsteps) * vjp_slot(c) * sizeof(double);
}

int md_step_record(md_ctx *c, double *q, double *p, double *f, double dt, int64_t nsteps, double *stage,
                   size_t stage_bytes)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (c->batch) return fail(c, MD_EUNSUPPORTED, "md_step_record: single systems only");
    if (c->model == MD_HMF && c->prec != MD_FP64)
        return fail(c, MD_EUNSUPPORTED, "md_step_record: HMF needs an FP64-state context");
    if (!q || !p || !f || !stage || !aligned8(q) || !aligned8(p) || !aligned8(f) || !aligned8(stage))
        return fail(c, MD_EINVAL, "md_step_record: null or misaligned pointer");
    if (!isfinite(dt)) return fail(c, MD_EINVAL, "md_step_record: dt must be finite");
    if (nsteps < 0) return fail(c, MD_EINVAL, "md_step_record: nsteps must be >= 0");
    if (stage_bytes < md_record_stage_bytes(c, nsteps))
        return fail(c, MD_ENOMEM, "md_step_record: stage buffer needs %zu bytes", md_record_stage_bytes(c, nsteps));
    if (nsteps == 0) return MD_OK;
    if (!c->forced)
        return fail(c, MD_ESTATE, "md_step_record: f must hold force(q): call md_force on this context first");
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_step_record: set device");
    const size_t slot = vjp_slot(c);
    return c->model == MD_HMF ? step_hmf(c, q, p, f, dt, nsteps, stage, slot)
                              : step_pairs(c, q, p, f, dt, nsteps, stage, slot);
}

int md_step_vjp_recorded(md_ctx *c, const double *q0, double dt, int64_t nsteps, double *lam_q, double *lam_p,
                         const double *stage, size_t stage_bytes)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (c->batch) return fail(c, MD_EUNSUPPORTED, "md_step_vjp_recorded: single systems only");
    if (!q0 || !lam_q || !lam_p || !stage || !aligned8(q0) || !aligned8(lam_q) || !aligned8(lam_p) ||
        !aligned8(stage))
        return fail(c, MD_EINVAL, "md_step_vjp_recorded: null or misaligned pointer");
    if (!isfinite(dt)) return fail(c, MD_EINVAL, "md_step_vjp_recorded: dt must be finite");
    if (nsteps < 0) return fail(c, MD_EINVAL, "md_step_vjp_recorded: nsteps must be >= 0");
    if (stage_bytes < md_record_stage_bytes(c, nsteps))
        return fail(c, MD_ENOMEM, "md_step_vjp_recorded: stage buffer needs %zu bytes",
                    md_record_stage_bytes(c, nsteps));
    if (nsteps == 0) return MD_OK;
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_step_vjp_recorded: set device");
    const size_t slot = vjp_slot(c);
    return c->model == MD_HMF ? reverse_hmf(c, q0, stage, slot, dt, nsteps, lam_q, lam_p)
                              : reverse_pairs(c, q0, stage, slot, dt, nsteps, lam_q, lam_p);
}

int md_timing_begin(md_ctx *c, int max_launches)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (max_launches < 1 || max_launches > 65536)
        return fail(c, MD_EINVAL, "md_timing_begin: max_launches = %d outside [1, 65536]", max_launches);
    DeviceGuard g(c->dev);
    if (g.err != hipSuccess) return dev_fail(c, g.err, "md_timing_begin: device");
    delete c->timing;
    c->timing = nullptr;
    Timing *t = new (std::nothrow) Timing;
    if (!t) return fail(c, MD_ENOMEM, "md_timing_begin: host allocation");
    t->ev.assign(2 * (size_t)max_launches, nullptr);
    for (hipEvent_t &e : t->ev) {
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            delete t;
            return dev_fail(c, r, "md_timing_begin: hipEventCreate");
        }
    }
    c->timing = t;
    return MD_OK;
}

int md_timing_end(md_ctx *c, double *ms_total, int *launches, char *name, size_t name_bytes)
{
    if (!c) return MD_EINVAL;
    c->err.clear();
    if (!ms_total || !launches) return fail(c, MD_EINVAL, "md_timing_end: null output");
    if (!c->timing) return fail(c, MD_ESTATE, "md_timing_end: timing is not on (md_timing_begin)");
    DeviceGuard g(c->dev);
    Timing *t = c->timing;
    c->timing = nullptr;
    double total = 0.0;
    hipError_t e = g.err;
    for (int i = 0; e == hipSuccess && i < t->used; ++i) {
        float ms = 0.0f;
        e = hipEventSynchronize(t->ev[2 * (size_t)i + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t->ev[2 * (size_t)i], t->ev[2 * (size_t)i + 1]);
        total += ms;
    }
    const int used = t->used;
    if (name && name_bytes) snprintf(name, name_bytes, "%s", t->kernel);
    delete t;
    if (e != hipSuccess) return dev_fail(c, e, "md_timing_end");
    *ms_total = total;
    *launches = used;
    return MD_OK;
}

int md_destroy(md_ctx *c)
{
    delete c;
    return MD_OK;
}

const char *md_strerror(int status)
{
    switch (status) {
    case MD_OK: return "success";
    case MD_EINVAL: return "invalid argument";
    case MD_EDEVICE: return "HIP device or launch error";
    case MD_ENOMEM: return "workspace too small or host allocation failed";
    case MD_ESTATE: return "call out of order";
    case MD_ENONFINITE: return "non-finite result";
    case MD_EUNSUPPORTED: return "unsupported model, precision or tile configuration";
    default: return "unknown status";
    }
}

const char *md_last_error(const md_ctx *c) { return c ? c->err.c_str() : ""; }

const char *md_version(void) { return "libmd 0.1 (gfx950)"; }

int md_force_noalloc(int model, int prec, int64_t n, double eps, void *hip_stream, const double *q, double *f)
{
    if (!model_ok(model) || n < 1 || n > (model == MD_HMF ? kMaxHmfN : kMaxPairN)) return MD_EINVAL;
    if (!prec_ok(model, prec)) return MD_EUNSUPPORTED;
    if (!eps_ok(model, prec, eps)) return MD_EINVAL;
    if (!q || !f || !aligned8(q) || !aligned8(f)) return MD_EINVAL;
    // the built-in tiles, with the j split halved until its partials fit
    Tiles t = default_tiles(model, prec, n);
    while (t.jsplit > 1 && force_layout(model, prec, n, t.jsplit).total > MD_NOALLOC_SCRATCH_BYTES) t.jsplit /= 2;
    const ForceLayout L = force_layout(model, prec, n, t.jsplit);
    if (L.total > MD_NOALLOC_SCRATCH_BYTES) return MD_ENOMEM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MD_EDEVICE;
    void *base = nullptr;
    if (scratch_address(dev, &base) != hipSuccess) return MD_EDEVICE;

    // A context on the stack over the scratch (no host allocation either): the
    // same fields md_init sets for what md_force reads
    md_ctx c;
    c.model = model;
    c.prec = prec;
    c.n = n;
    c.npad = pad_n(n);
    c.eps = model == MD_HMF ? 0.0 : eps;
    c.stream = static_cast<hipStream_t>(hip_stream);
    c.dev = dev;
    c.ws = static_cast<char *>(base);
    c.ws_bytes = MD_NOALLOC_SCRATCH_BYTES;
    c.red = reinterpret_cast<double *>(c.ws + L.red);
    c.scal = reinterpret_cast<double *>(c.ws + L.scal);
    c.macc = L.ops > L.macc ? reinterpret_cast<long long *>(c.ws + L.macc) : nullptr;
    c.ops = L.part > L.ops ? static_cast<void *>(c.ws + L.ops) : nullptr;
    c.part = L.total > L.part ? reinterpret_cast<double *>(c.ws + L.part) : nullptr;
    c.launch = MD_LAUNCH_STAGED;
    c.tiles = t;
    double *qm = const_cast<double *>(q);
    hipError_t e = hipSuccess;
    if (model == MD_HMF) {
        // launch_hmf_begin zeroes the fixed-point sums the previous call left
        e = launch_hmf_begin(&c);
        if (e == hipSuccess) e = launch_hmf_pass(&c, 0, HMF_REDUCE, 0.0, 0.0, 0.0, qm, nullptr, nullptr, nullptr, false);
        if (e == hipSuccess) e = launch_hmf_pass(&c, 1, HMF_STORE_F, 0.0, 0.0, 0.0, qm, nullptr, nullptr, f, false);
    } else {
        // every slot the combine reads is written by the pair kernel first
        e = launch_update(&c, UPD_PREP, 0.0, 0.0, 0.0, qm, nullptr, nullptr);
        if (e == hipSuccess) e = launch_pair(&c, q);
        if (e == hipSuccess) e = launch_update(&c, UPD_F_FROM_PART | UPD_STORE_F, 0.0, 0.0, 0.0, qm, nullptr, f);
    }
    return e == hipSuccess ? MD_OK : MD_EDEVICE;
}

}  // extern "C"
