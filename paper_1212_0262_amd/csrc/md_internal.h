// md_internal.h -- host-side context of libmd and the kernel launchers each
// translation unit provides.  Not installed; the public interface is md.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "md.h"

namespace md {

// Update-kernel flags (one kick-drift stage of the Yoshida composition, eq. 4).
enum : int {
    UPD_F_FROM_PART = 1 << 0,  // f = prefactor * (sum of the pair-kernel partials), else read f
    UPD_STORE_F = 1 << 1,      // write f
    UPD_KICK1 = 1 << 2,        // p += kick1 * f
    UPD_KICK2 = 1 << 3,        // p += kick2 * f (end kick of a step merged with the next start)
    UPD_DRIFT = 1 << 4,        // q += drift * p
    UPD_PREP = 1 << 5,         // refresh the pair-kernel operands from q (FP32 copy / sincos)
};

// HMF pass flags.
enum : int {
    HMF_KICK_F = 1 << 0,    // p += kick1 * f_in[i]
    HMF_KICK_M = 1 << 1,    // p += (kick1 [+ kick2]) * (cos(t) My - sin(t) Mx)
    HMF_KICK2 = 1 << 2,     // second kick of the same force
    HMF_DRIFT = 1 << 3,     // t += drift * p
    HMF_REDUCE = 1 << 4,    // block partials of sum cos(t'), sum sin(t')
    HMF_STORE_F = 1 << 5,   // f_out = cos(t) My - sin(t) Mx  (no drift in the same pass)
    HMF_WRITE = 1 << 6,     // write t, p back
};

constexpr int kWave = 64;           // lanes per wavefront (CDNA)
constexpr int kMaxJSplit = 64;
constexpr int kRedSlots = 1 << 17;   // doubles of reduction scratch (HMF pass partials: first half)
constexpr int kHmfGrid = 32768;      // most blocks of an HMF pass (2 FP64 partials each)
// The HMF magnetization sums in fixed point (grids of at most kHmfInPassM blocks):
// each reducing block adds its partial sums of cos and sin, as limbs of 2^-32 and
// 2^-64, to slot (block mod kMSlots) with 64-bit integer atomics (exact, so the
// total does not depend on the order), in one of three buffers that rotate over
// the passes of a call.
constexpr int kMSlots = 64;
constexpr int kMLimbs = 4;  // sum cos: 2^-32 and 2^-64 limbs; sum sin: the same
constexpr int kMWords = 3 * kMSlots * kMLimbs;
constexpr int kHmfInPassM = 1024;  // grids of at most this many blocks use the fixed-point sums
constexpr int kEnergyBlock = 256;
constexpr int64_t kFusedMaxN = 65536;   // contexts up to this n carry the fused stage's operand buffers
constexpr int kFusedMaxWaves = 16;      // wavefronts per fused block
constexpr int kFusedLdsBytes = 49152;   // LDS per fused block (split evenly between its wavefronts)
constexpr int64_t kFusedAutoN = 4096;   // MD_LAUNCH_AUTO takes the fused form up to this n (Ring)
constexpr int64_t kFusedAutoN2D = 6144; // ... and up to this n for 2D gravity
constexpr int kSymTile = 1024;          // particles per tile of the symmetric form (4 waves x 64 x 4 i)
constexpr int kBatchSymTile = 512;     // tiles of the ensembles' symmetric form (2 waves x 64 x 4 i)
constexpr int kSymTileSmall = 512;      // ... for smaller n (2 waves x 64 x 4 i; sym_tile_n), and 256
                                        // (1 wave) for smaller n still
constexpr int64_t kSymMinN = 2048;      // the symmetric form needs two tiles at least
constexpr int64_t kSymMaxN = 1 << 20;   // and at most 1024 tiles (its partial slots: 8 d n^2 / 1024 bytes)
// MD_LAUNCH_AUTO takes the symmetric form from this n (measured crossovers)
inline int64_t sym_auto_n(int model, int prec)
{
    if (model != MD_RING)
        return prec == MD_MIXED_KAHAN || prec == MD_MIXED_PAIRF64 ? MD_SYMMETRIC_AUTO_N_COMP : MD_SYMMETRIC_AUTO_N;
    return prec == MD_FP64 ? MD_SYMMETRIC_AUTO_N_RING64 : MD_SYMMETRIC_AUTO_N_RING;
}

// Lane groups per wavefront of the fused stage for j_split j ranges: the largest
// power of two <= 8 dividing j_split (more, smaller i tiles: more blocks).
inline int fused_groups(int jsplit)
{
    int L = 1;
    while (L < 8 && jsplit % (2 * L) == 0) L *= 2;
    return L;
}

struct Tiles {
    int ipl = 0;     // i per lane
    int waves = 0;   // wavefronts per block
    int jsplit = 0;  // j ranges per i block
    int jtile = 0;   // j per FP32 partial
};


// Host-side description of a batched ensemble (md_batch_init).  The work lists
// are built on the host, kept here (they are the source of asynchronous uploads)
// and copied into the workspace.
struct Batch {
    int nb = 0;
    int64_t nmax = 0;
    int smax = 1;                   // largest j_split accepted (pieces of the largest realization)
    std::vector<int64_t> off;       // nb + 1 CSR offsets
    std::vector<double> eps, pref;  // per realization
    std::vector<int> items;         // pair items, 8 ints each: b, i0, i1, slot, j0, j1, 0, 0
    std::vector<int> rows;          // row items, 4 ints each: b, i0, i1, S_b
    std::vector<int> eitems;        // energy items, 8 ints each
    std::vector<int> eoff, roff;    // per-realization ranges of energy / row items
    int n_items = 0, n_rows = 0, n_eitems = 0, max_items = 0;
    void *d_items = nullptr, *d_rows = nullptr, *d_eitems = nullptr;
    // symmetric form: tile pairs within each realization, 8 ints each
    // (b, i0, i1, slot_i, j0, j1, slot_j, 0), the n_soff tile pairs a < b first,
    // then the n_sdiag diagonal tiles; srows: the row items with S_b = T_b tiles
    bool sym = false;  // the ensemble can take the symmetric form
    int tmax = 0;      // most tiles of one realization
    std::vector<int> sitems, srows;
    int n_soff = 0, n_sdiag = 0;
    void *d_sitems = nullptr, *d_srows = nullptr;
    double *d_eps = nullptr, *d_pref = nullptr, *d_ered = nullptr, *d_kred = nullptr;
    int *d_eoff = nullptr, *d_roff = nullptr;
    int64_t *d_off = nullptr;
};

}  // namespace md

namespace md {
// Events of md_timing_begin: a start and an end event per timed launch.
struct Timing {
    std::vector<hipEvent_t> ev;
    int used = 0;
    const char *kernel = "";
    ~Timing();
};
}  // namespace md

struct md_ctx {
    int model = 0, prec = 0, dev = 0;
    int64_t n = 0, npad = 0;
    double eps = 0.0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    // workspace carve-up
    void *ops = nullptr;      // pair operands: 2D [2][npad] FP32 copy; Ring [2][npad] cos,sin (FP32 or FP64)
    void *wops = nullptr;     // the Hessian-vector product's vector as operands: FP32 [d][npad] (mixed
                              // forms), FP64 [2][npad] with pads (2D FP64, symmetric form)
    double *part = nullptr;   // pair partials [jsplit][d][npad]; symmetric form: [npad / kSymTile][d][npad]
    double *red = nullptr;    // reduction partials [kRedSlots]
    double *scal = nullptr;   // small device scalars (HMF magnetization, ...)
    long long *macc = nullptr;  // HMF magnetization sums, fixed point: [3][kMSlots][kMLimbs]
    float *th32 = nullptr;    // HMF FP32 state
    float *p32 = nullptr;
    void *fops[2] = {nullptr, nullptr};  // fused stage operands, alternating (n <= kFusedMaxN): [2][npad] of T
    int launch = 0;                      // md_launch: auto / staged / fused / symmetric
    bool forced = false;                 // md_force has run (md_step needs f = force(q))
    bool checkable = false;              // an energy or magnetization has set the finiteness flag
    md::Tiles tiles;
    md::Batch *batch = nullptr;  // non-null for a batched ensemble (owned)
    md::Timing *timing = nullptr;  // non-null while md_timing_begin is on (owned)
    std::string err;
    ~md_ctx()
    {
        delete batch;
        delete timing;
    }
};

namespace md {

int64_t pad_n(int64_t n);  // n rounded up to a multiple of kSymTile
int sym_tile_n(int model, int prec, int64_t n);  // particles per tile of the symmetric form (256, 512, 1024)
int dims(int model);
// MD_LAUNCH_STAGED, MD_LAUNCH_FUSED or MD_LAUNCH_SYMMETRIC: the form the pair
// stages of this context take now (launch mode, tiles and n).
int launch_form(const md_ctx *c);
int max_j_split(int64_t n);
Tiles default_tiles(int model, int prec, int64_t n);
int hmf_grid(int64_t n);  // blocks of the HMF passes (fixed per n: reproducible sums)
// f = prefactor * (sum of the pair terms): -2/N (2D); -1/(2 sqrt2 N) for the Ring
// terms of eq. 9 (FP64); -1/(2N) for the half-angle Ring terms (FP32 forms).
inline double force_prefactor(int model, int prec, int64_t n)
{
    if (model == MD_GRAV2D) return -2.0 / (double)n;
    return prec == MD_FP64 ? -1.0 / (2.0 * 1.4142135623730951 * (double)n) : -1.0 / (2.0 * (double)n);
}

// Timing of the dominant kernel: timed_begin records the start event of one launch
// and returns its slot (-1 when timing is off, its events are used up, or the
// stream is being captured); timed_end(c, slot) records the end event.
int timed_begin(md_ctx *c, const char *kernel);
void timed_end(md_ctx *c, int slot);

// Launchers return hipSuccess or the launch error.  All enqueue on c->stream.
// pair.hip
// The pair partials of the context's launch form (staged or symmetric).
hipError_t launch_pair(md_ctx *c, const double *q);
// snap (nullable): with UPD_DRIFT, the drifted positions are also written there.
hipError_t launch_update(md_ctx *c, int flags, double kick1, double kick2, double drift,
                         double *q, double *p, double *f, double *snap = nullptr);
// Fused small-N stages: the update writing the fused operand form into ops, and
// one pair + update launch reading operands `in`, writing the new ones to `out`.
hipError_t launch_update_fused(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q,
                               double *p, double *f, void *ops, double *snap);
hipError_t launch_fused(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                        double *f, const void *in, void *out, double *snap);
// hmf.hip
// The passes of one call are numbered k = 0, 1, ...: pass k takes M from the limb
// sums pass k - 1 added, adds its own to buffer k mod 3 and zeroes buffer
// (k + 1) mod 3.  launch_hmf_begin zeroes buffer 0 before the first pass of a call
// whose passes read M.
// snap (nullable, FP64 state only): with HMF_DRIFT, the drifted angles are also written there.
hipError_t launch_hmf_begin(md_ctx *c);
hipError_t launch_hmf_pass(md_ctx *c, int k, int flags, double kick1, double kick2, double drift,
                           double *th, double *p, const double *f_in, double *f_out,
                           bool f32state, double *snap = nullptr);
hipError_t launch_hmf_hvp_sums(md_ctx *c, const double *th, const double *w);
hipError_t launch_hmf_adj_update(md_ctx *c, const double *th, int flags, double h, double h2, double a,
                                 double *lq, double *lp, double *out);
// M from the limb sums of a call's pass 0, to out2[0..1] and the context scalars.
hipError_t launch_hmf_magnetization(md_ctx *c, double *out2);
const double *hmf_partials(const md_ctx *c);  // block partials of the latest reducing pass
hipError_t launch_hmf_convert(md_ctx *c, double *th, double *p, bool to_f32);
// batch.hip
hipError_t batch_pair(md_ctx *c, const double *q);
hipError_t batch_update(md_ctx *c, int flags, double kick1, double kick2, double drift, double *q, double *p,
                        double *f);
hipError_t batch_energy(md_ctx *c, const double *q, const double *p, double *out);
// adjoint.hip
enum : int {
    ADJ_OUT = 1 << 0,    // out = H w (combine the partials)
    ADJ_KICK = 1 << 1,   // lq -= h * (H w)
    ADJ_DRIFT = 1 << 2,  // lp += a * lq
    ADJ_PREPQ = 1 << 3,  // pair operands from the positions pos
    ADJ_PREPW = 1 << 4,  // FP32 vector operand from lp (mixed forms)
    ADJ_KICK2 = 1 << 5,  // then lq -= h2 * (H w): a second kick at the same positions
};
hipError_t launch_hvp_pair(md_ctx *c, const double *pos, const double *w);
hipError_t launch_adj_update(md_ctx *c, int flags, double h, double h2, double a, double *lq, double *lp,
                             double *out, const double *pos);
// energy.hip
hipError_t launch_energy(md_ctx *c, const double *q, const double *p, double *out3);
// The finiteness flag (an unsigned in the context scalars): launch_finite_flag sets
// it to 1 if any of vals[0 .. count) is NaN or infinite, else to 0.
constexpr int kScalFlag = 16;  // index in c->scal
inline unsigned *finite_flag(md_ctx *c) { return reinterpret_cast<unsigned *>(c->scal + kScalFlag); }
hipError_t launch_finite_flag(md_ctx *c, const double *vals, int count);
hipError_t launch_magnetization(md_ctx *c, const double *q, double *out2);

}  // namespace md
