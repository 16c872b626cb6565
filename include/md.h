/*
 * md.h -- C ABI of libmd, the MI355X (gfx950) force engine for long-range
 * molecular dynamics (T. M. Rocha Filho, "Molecular dynamics for long-range
 * interacting systems on Graphic Processing Units").
 *
 * What the library computes
 *   The force evaluation inside the fourth-order Yoshida symplectic integrator
 *   (Sec. 3, eq. 4) for the three models of Sec. 2, unit masses, 1/N coupling:
 *     MD_RING    eq. 1: V = -(1/N) sum_{i<j} 1/(sqrt2 sqrt(1 - cos(ti - tj) + eps))
 *                force: the all-pairs sum of eqs. 8-9 (Sec. 3.2), taken as
 *                -dV/dtheta_i (the sign printed in eqs. 8-9 is +dV/dtheta_i).
 *     MD_HMF     eq. 2: V = (1/N) sum_{i<j} [1 - cos(ti - tj)], evaluated in O(N)
 *                through the magnetization (Sec. 3.1, eqs. 5-7).
 *     MD_GRAV2D  eq. 3: V = (1/N) sum_{i<j} log(|r_i - r_j|^2 + eps); force
 *                -(2/N) sum_j (r_i - r_j)/(|r_i - r_j|^2 + eps), the all-pairs
 *                sum of Sec. 3.2 (natural logarithm).
 *
 * Data layout (every array argument)
 *   Device pointers to contiguous FP64 structure-of-arrays [d][n]: d = 1 for
 *   MD_RING and MD_HMF (angle theta, momentum p_theta), d = 2 for MD_GRAV2D
 *   (x row of n values, then y row; px then py).  f has the shape of q.
 *   Pointers must be 8-byte aligned (torch allocations are 256-byte aligned).
 *
 * Ownership
 *   The caller owns q, p, f, the energy output and the workspace (sized by
 *   md_workspace_bytes).  The library owns only the host-side context; it never
 *   allocates device memory.  The workspace must stay alive and untouched by the
 *   caller for the life of the context.
 *
 * Streams and synchronisation
 *   Every call only enqueues kernels on the HIP stream given to md_init (NULL =
 *   the legacy default stream) and returns without waiting; results are ready
 *   once that stream has reached them.  No call allocates, and no call but
 *   md_check and md_timing_end synchronises the host, so the others may be
 *   captured into a HIP graph.
 *
 * Errors
 *   Every function returns an md_status; nothing is thrown across the ABI.
 *   Arguments are validated before anything is enqueued, so a call that returns
 *   MD_EINVAL, MD_ESTATE or MD_EUNSUPPORTED has changed nothing.  A launch failure
 *   returns MD_EDEVICE; md_last_error gives the detail.  A context is not
 *   thread-safe; distinct contexts are independent.
 *
 * Determinism
 *   Same device, same inputs, same tile configuration: bitwise-identical
 *   outputs (fixed reduction trees, no floating-point atomics).
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_ctx md_ctx; /* opaque, host-side */

/* Models of Sec. 2 (eqs. 1-3). */
enum md_model { MD_HMF = 0, MD_RING = 1, MD_GRAV2D = 2 };

/*
 * Arithmetic of the force evaluation.  State (q, p, f), energies and the HMF
 * magnetization are FP64 in every mode except MD_MIXED_F32STATE.
 *   MD_FP64            all FP64.
 *   MD_MIXED           FP32 copies of the positions (Sec. 3.2, 2D scheme), FP32
 *                      pair arithmetic, FP32 partial sums over a j-tile folded
 *                      into an FP64 per-particle accumulator once per tile.
 *   MD_MIXED_KAHAN     FP32 pair arithmetic, Kahan-compensated FP32 accumulation
 *                      of every pair term (no FP64 in the pair loop).
 *   MD_MIXED_PAIRF64   FP32 pair arithmetic, each pair term added into an FP64
 *                      accumulator (the literal scheme of Sec. 3.2 for 2D).
 *   MD_MIXED_F32STATE  HMF only: FP32 angles (wrapped to [-pi, pi)), momenta,
 *                      sines/cosines and kicks inside md_step; FP64 reduction of
 *                      the magnetization (eq. 7).  q, p, f stay FP64 at the ABI.
 * MD_RING and MD_GRAV2D accept the first four; MD_HMF accepts MD_FP64 and
 * MD_MIXED_F32STATE.
 */
enum md_prec {
    MD_FP64 = 0,
    MD_MIXED = 1,
    MD_MIXED_KAHAN = 2,
    MD_MIXED_PAIRF64 = 3,
    MD_MIXED_F32STATE = 4
};

enum md_status {
    MD_OK = 0,
    MD_EINVAL = -1,       /* bad argument (null/misaligned pointer, n < 1, eps <= 0, ...) */
    MD_EDEVICE = -2,      /* a HIP call or kernel launch failed */
    MD_ENOMEM = -3,       /* workspace smaller than md_workspace_bytes, or host alloc failed */
    MD_ESTATE = -4,       /* call out of order (md_step before any md_force, md_check with nothing to check) */
    MD_ENONFINITE = -5,   /* md_check: the last energies or magnetization were not finite */
    MD_EUNSUPPORTED = -6  /* model/precision combination or tile configuration not built */
};

/*
 * Workspace bytes a context for (model, prec, n) needs; 0 for an invalid
 * combination.  The figure covers every tile configuration md_set_tiles
 * accepts for this n, and every launch form the context can take: for
 * MD_GRAV2D and MD_RING with 2048 <= n <= 1048576 it
 * includes the symmetric form's partial slots, 8 d n'^2 / 1024 bytes with n' = n
 * rounded up to a multiple of 1024 (1.07 GB for 2D at n = 262144).
 */
size_t md_workspace_bytes(int model, int prec, int64_t n);

/*
 * The softening eps (eqs. 1 and 3) each pair model and precision accepts
 * (MD_EINVAL outside; MD_HMF ignores eps): within them no pair term overflows,
 * loses its normal range or takes the square root of a negative number, for any
 * positions.  2D in FP64 adds up to four pair terms with one reciprocal of the
 * product of their |r_i - r_j|^2 + eps, which must stay a normal FP64 number
 * (particles closer than about 1e38 to each other); the FP32 forms round eps to
 * FP32 (the Ring's half-angle form raises 2 eps to the -3/2); the Ring in FP64
 * (eq. 9) forms 1 + eps - cos(ti - tj), which has to stay positive for two
 * particles at the same angle.  No upper bound for the Ring in FP64.
 */
#define MD_EPS_MIN_2D_FP64 1e-75
#define MD_EPS_MAX_2D_FP64 1e75
#define MD_EPS_MIN_2D_FP32 1e-30
#define MD_EPS_MIN_RING_FP64 1e-12
#define MD_EPS_MIN_RING_FP32 1e-25
#define MD_EPS_MAX_FP32 1e30

/*
 * Create a context for n particles of `model` (eqs. 1-3) with softening eps
 * (eqs. 1 and 3, in the range above; ignored for MD_HMF), computing in
 * `prec`.  hip_stream: a hipStream_t, or NULL for the default stream.
 * workspace: device memory of at least md_workspace_bytes(model, prec, n)
 * bytes, 256-byte aligned.  On success *out holds the new context.
 * The context records the current HIP device; md_init enqueues nothing.
 */
int md_init(md_ctx **out, int model, int prec, int64_t n, double eps,
            void *hip_stream, void *workspace, size_t workspace_bytes);

/*
 * Batched ensembles: nb independent realizations of one pair model (MD_RING or
 * MD_GRAV2D; MD_HMF is MD_EUNSUPPORTED) advanced together, e.g. for ensemble
 * averages over initial conditions of quasi-stationary states (Sec. 1).  Each
 * realization b is the system of eqs. 1 or 3 with its own N_b = offsets[b+1] -
 * offsets[b] >= 1 particles, its own 1/N_b coupling and its own eps[b] (in
 * the range md_init takes); realizations do not interact.
 *   offsets: host int64 [nb + 1], offsets[0] = 0, strictly increasing,
 *            offsets[nb] <= 2^24 (total particles).
 *   eps:     host FP64 [nb].
 * Arrays passed to md_force / md_step / md_energy are the realizations
 * concatenated in order: device FP64 [d][offsets[nb]].  md_energy then writes
 * 3*nb doubles, {K, V, E} of realization b at out[3b .. 3b+2].  md_set_tiles
 * applies to every realization; j_split is the number of j chunks of the largest
 * realization (smaller ones use the same chunk length, so fewer chunks), up to
 * min(32, N_max/64).  md_batch_init copies its work lists into the workspace with
 * asynchronous copies on hip_stream (the host arrays may be freed on return);
 * md_set_tiles on a batch context re-uploads the tile-dependent lists the same way.
 * The workspace figure includes the symmetric launch form's tile-pair lists and
 * slots when the ensemble can take it (md_set_launch).
 * Errors as md_init (MD_EINVAL for a bad offsets/eps array).
 */
size_t md_batch_workspace_bytes(int model, int prec, int nb, const int64_t *offsets, const double *eps);
int md_batch_init(md_ctx **out, int model, int prec, int nb, const int64_t *offsets, const double *eps,
                  void *hip_stream, void *workspace, size_t workspace_bytes);

/* Number of realizations of a context: nb for a batch, 1 otherwise, 0 for NULL. */
int md_batch_size(const md_ctx *c);

/* Change the stream later calls enqueue on. */
int md_set_stream(md_ctx *c, void *hip_stream);

/*
 * Tile configuration of the O(N^2) pair kernels (Sec. 3.2: i-tiles over blocks,
 * j-tiles streamed through the whole j range).  Results are the same sums in a
 * different order, so they agree to rounding across configurations.
 *   i_per_lane   particles i held in registers by each lane: 1, 2 or 4
 *   waves        wavefronts (64 lanes) per block: 1, 2 or 4
 *   j_split      number of j ranges computed by separate blocks and combined
 *                in a fixed order: 1 .. md_max_j_split(n)
 *   j_tile       j per FP32 partial sum before the FP64 fold (MD_MIXED):
 *                a multiple of 16 in [16, 4096]
 * 0 in any field keeps the built-in choice for this n.  MD_HMF ignores it.
 */
int md_set_tiles(md_ctx *c, int i_per_lane, int waves, int j_split, int j_tile);

/* Current tile configuration (after defaults were resolved): out[4] host ints. */
int md_get_tiles(const md_ctx *c, int *out4);

/* Largest j_split md_set_tiles accepts for n particles (>= 1). */
int md_max_j_split(int64_t n);

/*
 * Launch form of md_step for single Ring and 2D systems (eq. 4's stages):
 *   MD_LAUNCH_STAGED  two launches per force evaluation: the pair kernel over
 *                     (i block, j range) tiles, then an elementwise kernel that
 *                     adds the j-range partials and kicks, drifts and refreshes
 *                     the pair operands;
 *   MD_LAUNCH_FUSED   one launch per force evaluation (small N, where latency
 *                     dominates): a block owns one i tile and all its j ranges,
 *                     the partials are added in LDS and the same block runs the
 *                     stage on its own particles.
 *                     The j ranges, folds and order of additions are the staged
 *                     ones, so both forms give bit-identical results for the same
 *                     tiles.  Needs n <= 65536 and tiles a block can hold:
 *                     the j ranges are j_split / L wavefronts of L lane groups
 *                     (L the largest power of two <= 8 dividing j_split), at
 *                     most 16 wavefronts, and i_per_lane * d * 512 bytes of
 *                     partials per wavefront within 48 KiB / wavefronts
 *                     (MD_EUNSUPPORTED otherwise; md_set_tiles then refuses
 *                     tiles outside that range);
 *   MD_LAUNCH_SYMMETRIC  2D gravity or Ring, every precision form they accept,
 *                     2048 <= n <= 1048576: each pair is evaluated once and
 *                     added to both particles with opposite signs (the terms of
 *                     the gradient of eq. 3 and of eq. 9 are odd in the pair's
 *                     difference), which halves the pair evaluations of the
 *                     all-pairs sum.  The particles are cut into tiles of 1024;
 *                     one block takes a tile pair (a, b), a < b, and writes its
 *                     i-side and j-side sums to separate slots (FP32 for
 *                     MD_MIXED, FP64 otherwise), the blocks
 *                     of the diagonal tiles take every pair of their tile; the
 *                     elementwise kernel adds the slots in a fixed order.  The
 *                     accumulation of the precision form applies on both sides
 *                     (MD_MIXED: FP32 runs of at most 256 terms added in FP64;
 *                     MD_MIXED_KAHAN: compensated FP32 sums over the tile, the
 *                     compensation moving with the j-side sums; MD_MIXED_PAIRF64:
 *                     every FP32 term added in FP64).  No
 *                     atomics: bit-reproducible run to run, but the sums are
 *                     grouped differently from the staged form (results agree
 *                     to the precision's rounding, not bit for bit).  The
 *                     particles past n in the last tile contribute nothing: the
 *                     Ring form gives them zero operands (exact zeros), the 2D
 *                     FP32 form positions at 1e30 (exact zeros), the 2D FP64
 *                     form positions at 1e150 (terms of about 5e-151); 2D
 *                     positions must stay far below both.  Every operand refresh
 *                     (the first stage of md_force and md_step) writes the
 *                     pads.  Tiles
 *                     (md_set_tiles) do not apply to it.  Ensembles
 *                     (md_batch_init) take tile pairs within each realization:
 *                     Ring with MD_MIXED, MD_MIXED_KAHAN (the compensated sums
 *                     kept on both sides) or MD_FP64, 2D with MD_MIXED or
 *                     MD_MIXED_KAHAN, every N_b <= 1048576.  MD_EUNSUPPORTED for
 *                     other models, precisions or n;
 *   MD_LAUNCH_AUTO    (default) fused when it applies and n <= 4096 (Ring)
 *                     or 6144 (2D gravity) (the built-in tiles there are the
 *                     fused form's), symmetric
 *                     when it applies and n reaches the model's threshold
 *                     (MD_SYMMETRIC_AUTO_N for 2D gravity with MD_MIXED
 *                     or MD_FP64, MD_SYMMETRIC_AUTO_N_COMP with the
 *                     compensated forms; for the Ring MD_SYMMETRIC_AUTO_N_RING
 *                     with the FP32 forms and MD_SYMMETRIC_AUTO_N_RING64 with
 *                     MD_FP64: measured crossovers on MI355X), else staged;
 *                     for ensembles, symmetric when it applies and their tile
 *                     pairs a < b outnumber their diagonal tiles.
 * md_get_launch returns the form md_step will take (STAGED, FUSED or
 * SYMMETRIC), or a negative status.  HMF contexts are always STAGED, ensembles
 * STAGED or SYMMETRIC.
 * md_get_sym_tile returns the particles per tile of the symmetric form when
 * md_get_launch is SYMMETRIC (single systems: 256 up to 65536 particles, 512
 * for the Ring up to 131072, 1024 above -- more, shorter tile pairs where they
 * are few; ensembles: 512 within each realization), else 0; a negative status
 * for a null context.  The force then evaluates T (T - 1) / 2 tile pairs of T^2 pairs
 * each and T diagonal tiles of T^2 ordered pairs, T = the padded n over the tile.
 */
enum md_launch { MD_LAUNCH_AUTO = 0, MD_LAUNCH_STAGED = 1, MD_LAUNCH_FUSED = 2, MD_LAUNCH_SYMMETRIC = 3 };
#define MD_SYMMETRIC_AUTO_N 13312
#define MD_SYMMETRIC_AUTO_N_COMP 15360
#define MD_SYMMETRIC_AUTO_N_RING 13312
#define MD_SYMMETRIC_AUTO_N_RING64 10240
int md_set_launch(md_ctx *c, int mode);
int md_get_launch(const md_ctx *c);
int md_get_sym_tile(const md_ctx *c);

/*
 * f = -dV/dq at positions q (eqs. 6-9 and the 2D gradient of eq. 3).
 * q: device [d][n] FP64, read only.  f: device [d][n] FP64, written.
 * For MD_HMF this also caches the magnetization of q in the workspace.
 */
int md_force(md_ctx *c, const double *q, double *f);

/*
 * md_force for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It takes no context and no
 * workspace, and calls no allocating routine (device or host): its workspace is
 * the library's own static device array of MD_NOALLOC_SCRATCH_BYTES, one per
 * GPU, held from the library's load to the end of the process.
 *   model, prec, n, eps: as md_init (same validation and statuses).
 *   hip_stream: the stream to enqueue on (NULL = the legacy default stream).
 *   q, f: device [d][n] FP64 on the current device, as md_force.
 * Works on the current device.  Computes what md_force computes in the staged
 * form (MD_LAUNCH_STAGED) with the built-in tiles, except that the j split is
 * halved until the pair partials fit the array: where it is not halved the
 * result is bit-identical to md_force on a context with the same tiles and
 * launch form.  MD_ENOMEM if n needs more than the array even with one j range
 * (24 bytes a particle for 2D with FP32 operands and for Ring FP64, so above
 * about 2.7 million particles; 16 for 2D FP64 and Ring with FP32 operands, above
 * about 4.1 million; HMF never).  MD_EDEVICE for a failed launch (no detail: there is no context).
 * Every call on a GPU shares that GPU's array, which keeps the previous call's
 * contents: calls that overlap on one GPU (concurrent streams, or threads) race,
 * so the caller must order them.
 */
#define MD_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int md_force_noalloc(int model, int prec, int64_t n, double eps, void *hip_stream, const double *q, double *f);

/*
 * nsteps Yoshida steps of size dt (eq. 4), in place.  On entry f must equal
 * force(q) (from md_force or the previous md_step); on exit q, p hold the state
 * at t + nsteps*dt and f = force(q).  Three force evaluations per step; the
 * force at the end of a step is reused at the start of the next.  dt may be
 * negative (reverse integration).  nsteps = 0 is a no-op.  MD_ESTATE if the
 * context has never run md_force (the library cannot check f itself; this
 * catches the missing first evaluation the step list of Sec. 3 starts from).
 */
int md_step(md_ctx *c, double *q, double *p, double *f, double dt, int64_t nsteps);

/*
 * Energies of the state (q, p): out_dev3[0] = K = (1/2) sum p^2,
 * out_dev3[1] = V of eqs. 1-3 (HMF through eq. 5), out_dev3[2] = K + V.
 * Always FP64 arithmetic and FP64 accumulation, whatever `prec` is.
 * out_dev3: device pointer to 3 doubles.  Also records on the device whether the
 * three values are finite, for md_check.
 */
int md_energy(md_ctx *c, const double *q, const double *p, double *out_dev3);

/*
 * Whether the energies (md_energy) or the magnetization (md_magnetization) most
 * recently enqueued on this context were finite.  Waits on the host for the
 * context's stream, so it cannot be captured into a graph.  Returns MD_OK if every
 * value was finite, MD_ENONFINITE if one was NaN or infinite (the state has left
 * FP64's range, e.g. after too large a step dt; the relative energy error of
 * Sec. 4 is then meaningless).  MD_ESTATE if neither call has run on this
 * context, or if the stream is being captured; MD_EDEVICE if the read fails.
 */
int md_check(md_ctx *c);

/*
 * HMF magnetization of eq. 7 at positions q: out_dev2[0] = Mx, out_dev2[1] = My.
 * The sum is reproducible bit for bit and the same one md_force and md_step use:
 * for n <= 2097152 the exact sum of the FP64 block partials (in 64-bit fixed
 * point) rounded once to FP64, above that the block partials added in FP64 in a
 * fixed order.  MD_HMF contexts only.  Records finiteness for md_check as
 * md_energy does, judged on the FP64 block partials (a NaN cannot pass through
 * the fixed-point sum, so the output alone would not show it).
 */
int md_magnetization(md_ctx *c, const double *q, double *out_dev2);

/*
 * Derivatives (single-system contexts; batched ones MD_EUNSUPPORTED).  They
 * differentiate the same discrete map md_step computes (eq. 4 with the forces of
 * eqs. 1-3), in the context's precision.  HMF md_step_vjp needs an MD_FP64
 * context (MD_EUNSUPPORTED otherwise); HMF md_hvp runs in FP64 for either.
 *
 * md_hvp: out = H(q) w, H the Hessian of the potential V (the force is -grad V, so
 * its Jacobian is -H).  q, w, out: device [d][n] FP64.  HMF uses the mean-field
 * form of eqs. 6 and 7: (H w)_i = w_i (cos q_i Mx + sin q_i My) - cos q_i Cw
 * - sin q_i Sw with Cw, Sw the averages of cos q_j w_j and sin q_j w_j, O(N).
 * 2D MD_FP64 contexts whose force takes the symmetric launch form (md_get_launch)
 * take it for the product too: each pair evaluated once for both particles,
 * the per-tile sums added in a fixed order (reproducible bit for bit).
 *
 * md_step_vjp: reverse-mode derivative of nsteps Yoshida steps started from the
 * state (q0, p0) (e.g. a checkpoint kept during the forward run).  On entry
 * (lam_q, lam_p) hold dJ/dq, dJ/dp of some scalar J at the state nsteps later;
 * on exit they hold dJ/dq0, dJ/dp0.  The steps are recomputed forward from
 * (q0, p0) (q0, p0 are not modified) and every position at which a kick evaluates
 * the force is kept in `stage`; kicks and drifts are then undone in reverse:
 * a drift q += a p by lam_p += a lam_q, a kick p += h F(q) by lam_q -= h H(q) lam_p.
 * stage: caller device scratch of at least md_vjp_stage_bytes(c, nsteps) bytes
 * (3 nsteps + 3 slots, each [d][n] FP64 rounded up to an even count of doubles);
 * 8-byte aligned at least.  With stage, q0, p0 16-byte aligned the recomputed
 * trajectory is bit-identical to md_step's.  nsteps = 0 is a no-op.
 */
int md_hvp(md_ctx *c, const double *q, const double *w, double *out);
size_t md_vjp_stage_bytes(const md_ctx *c, int64_t nsteps);
int md_step_vjp(md_ctx *c, const double *q0, const double *p0, double dt, int64_t nsteps,
                double *lam_q, double *lam_p, double *stage, size_t stage_bytes);

/*
 * The reverse sweep without recomputation, for callers that can hold every kick
 * position of a run (3 nsteps slots of [d][n] FP64, each rounded up to an even
 * count of doubles: md_record_stage_bytes; e.g. 1.6 GB for the 2D system at
 * n = 32768 over 1000 steps).
 *
 * md_step_record: md_step (same arguments, same results bit for bit, the same
 * MD_ESTATE before any md_force) that also
 * writes the positions after each of its 3 nsteps drifts into `stage` (caller
 * device memory of at least md_record_stage_bytes(c, nsteps) bytes).  HMF needs
 * an MD_FP64 context.
 *
 * md_step_vjp_recorded: the reverse sweep of md_step_vjp over a run recorded by
 * md_step_record from positions q0 with the same dt and nsteps on this context:
 * (lam_q, lam_p) go from the adjoints at the end of the run to those at its
 * start.  stage is only read.
 */
size_t md_record_stage_bytes(const md_ctx *c, int64_t nsteps);
int md_step_record(md_ctx *c, double *q, double *p, double *f, double dt, int64_t nsteps,
                   double *stage, size_t stage_bytes);
int md_step_vjp_recorded(md_ctx *c, const double *q0, double dt, int64_t nsteps, double *lam_q,
                         double *lam_p, const double *stage, size_t stage_bytes);

/* Timing of the dominant kernel, for measurement (it is no part of the method).
 * md_timing_begin: from now on the first max_launches launches of the context's
 * dominant kernel (1 <= max_launches <= 65536) are each bracketed by two HIP
 * events recorded on the context's stream; later launches run untimed.  The
 * dominant kernel is the one that evaluates the pairs: the tile-pair kernel of the
 * symmetric form (not its diagonal tiles), the pair kernel of the staged form, the
 * fused kernel, the HMF stage pass (not the one-block sum after it); for ensembles the tile-pair
 * or the pair kernel; in md_hvp and the reverse sweeps, the Ring and 2D
 * Hessian-vector product's pair kernel (the timed launches of a call sequence are
 * those of every such kernel it runs, and the name is the last one's).  Launches enqueued while the stream is being captured into
 * a graph are not timed.  It creates 2 max_launches HIP events (host-side
 * objects: no workspace or device memory is taken); calling it again starts over.
 * md_timing_end: waits for the last timed launch, writes the summed duration of
 * the timed launches (ms) to *ms_total and their number to *launches, copies the
 * timed kernel's name (NUL-terminated, at most name_bytes bytes) to name unless
 * name is NULL, then destroys the events and turns timing off.
 * Errors: MD_EINVAL for a null context or output or max_launches out of range;
 * MD_ESTATE from md_timing_end when timing is not on; MD_EDEVICE when an event
 * call fails (detail in md_last_error; timing is off afterwards). */
int md_timing_begin(md_ctx *c, int max_launches);
int md_timing_end(md_ctx *c, double *ms_total, int *launches, char *name, size_t name_bytes);

/* Destroy a context (does not touch the workspace).  NULL is accepted. */
int md_destroy(md_ctx *c);

/* Static text for a status code. */
const char *md_strerror(int status);

/* Detail of the last failure on this context ("" if none); valid until the next call. */
const char *md_last_error(const md_ctx *c);

/* Library version string. */
const char *md_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MD_H */
