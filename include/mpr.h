/*
 * mpr.h -- C ABI of the MI355X (gfx950) library for conditional simulation
 * of gappy gridded data with the modified planar rotator (MPR) Gibbs random
 * field by hybrid Monte Carlo.
 *
 * Paper: M. Zukovic and D. T. Hristopulos, "Gibbs Markov random fields with
 * continuous values based on the modified planar rotator model"
 * (arXiv 1710.03038).  Equation numbers are the paper's: (2) data -> angle
 * map, (3) MPR energy, (4) sample specific energy, (5) equilibrium specific
 * energy, (6) over-relaxation; Algorithm 1 is the hybrid UPDATE,
 * Algorithm 2 the simulation driver.
 *
 * Conventions shared by every entry point
 *  - Every call returns an mpr_status; nothing aborts, exits or throws
 *    across the ABI.  On failure mpr_last_error() describes the problem.
 *  - Device pointers are HIP device addresses owned by the caller, who
 *    keeps them alive until mpr_destroy() or until the stream has drained.
 *    The library never allocates device memory: all of its device state
 *    lives in the caller's workspace (see mpr_init_field).
 *  - All device work is ordered on the stream given to mpr_init_field.
 *    Calls that return host values synchronise that stream.
 *  - Validation happens before any launch; a call that fails validation
 *    leaves the context unchanged.
 *  - One context per stream; concurrent calls on one context are not
 *    allowed.
 *  - Angles: sample sites hold phi in [0, 2*pi] (Eq. 2, closed interval),
 *    gap sites live in [0, 2*pi).  Grids are ny rows of nx sites, row
 *    major, site (x, y) at index y*nx + x; boundaries are open (Sec. 2.2).
 */
#ifndef MPR_H
#define MPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPR_OK = 0,
  MPR_E_ARG = 1,        /* an argument value is invalid */
  MPR_E_SHAPE = 2,      /* a grid shape is invalid */
  MPR_E_DEGENERATE = 3, /* a grid has one distinct sample value: Eq. (2) undefined */
  MPR_E_NOPAIRS = 4,    /* a grid has no sample-sample neighbour pair: Eq. (4) undefined */
  MPR_E_RANGE = 5,      /* e_s outside the e(T) table: T clamped to its end */
  MPR_E_WORKSPACE = 6,  /* workspace missing, too small or misaligned */
  MPR_E_HIP = 7,        /* the HIP runtime reported an error */
  MPR_E_STATE = 8       /* the context is not in a state that allows the call */
} mpr_status;

typedef enum { MPR_FP32 = 0, MPR_FP64 = 1 } mpr_dtype;

/* Pair interaction H_ij of H = -sum H_ij: the MPR energy of Eq. (3),
 * cos(q (phi_i - phi_j)), or the Gaussian model on the same angles
 * compared in Sec. 4.4, 1 - (phi_i - phi_j)^2 / (2 pi^2) (q unused).  The
 * specific energies, the sample specific energy, over-relaxation (about the
 * neighbours' mean for GMRF) and the Metropolis energy change follow the
 * chosen interaction; the e(T) table must be that model's. */
typedef enum { MPR_MODEL_MPR = 0, MPR_MODEL_GMRF = 1 } mpr_model;

/* Boundary of the sweeps.  MPR_BC_OPEN: open boundaries, edge sites have
 * fewer neighbours (Sec. 2.1).  MPR_BC_REPLICATE: the auxiliary nodes of
 * Sec. 2.5, a ring around the grid whose nodes copy their nearest grid
 * site; the augmented grid is swept with open boundaries and the ring is
 * refreshed at the start of every half-sweep, so each off-grid neighbour
 * of an edge site holds that site's own value from before the half-sweep
 * (two for a corner).  Only the updates change: the specific energies and
 * the equilibration trace stay on the grid's own pairs.  The replicate
 * update depends on the site's previous value and so does not satisfy
 * detailed balance for Eq. (3); the e(T) tables are those of the open
 * boundary. */
typedef enum { MPR_BC_OPEN = 0, MPR_BC_REPLICATE = 1 } mpr_boundary;

/* mpr_sweep flags */
#define MPR_ADAPT   1u /* apply the a-rule of Algorithm 2, step 4.2 */
#define MPR_TRACE_E 2u /* record the specific energy e of Eq. (5) after every sweep */
#define MPR_NO_OR   4u /* leave out Algorithm 1, step 1 (over-relaxation): restricted Metropolis
                          alone, or standard Metropolis without MPR_ADAPT (a = 1, Sec. 2.4) */

/* mpr_specific_energy selectors */
#define MPR_SAMPLE_PAIRS 0 /* Eq. (4), one value per grid */
#define MPR_STATE        1 /* Eq. (5) of the current state, one value per chain */

typedef struct mpr_ctx mpr_ctx; /* opaque; host-side metadata only */

/* One gappy grid (Sec. 2: the grid G, the samples G_s and the gaps G_p). */
typedef struct {
  int32_t nx, ny;        /* nx >= 1, ny >= 1, nx*ny >= 2 */
  int32_t chains;        /* >= 1 independent Markov chains of this grid */
  int32_t reserved;      /* must be 0 */
  const double *z;       /* device, ny*nx values; read only at sample sites (gap values are ignored, NaN allowed) */
  const uint8_t *known;  /* device, ny*nx; nonzero = sample site (frozen), 0 = gap.
                            A grid without samples is an unconditional simulation (Sec. 2.4). */
} mpr_grid;

typedef struct {
  double q;               /* modification factor of Eq. (3): 0 < q <= 0.5, or exactly 1 (planar rotator, test mode) */
  double a_targ;          /* target acceptance A_targ of the a-rule (paper: 0.3) */
  double k_a;             /* rate k_a of the a-rule (paper: 3) */
  int32_t adapt_every;    /* a-rule period in sweeps, using the window's mean acceptance (paper: 1) */
  int32_t a_sample_keep;  /* 0: a = 1 while sampling, as in Algorithm 2 step 5.2; 1: keep the adapted a */
  int32_t dtype;          /* mpr_dtype of the sweeps' arithmetic and the stored angles */
  int32_t sweeps_per_pass;/* sweeps fused per HBM pass, 1..16; 0 = library choice */
  int32_t tile_x, tile_y; /* interior tile of one workgroup (even, 8..188); 0 = library choice */
  uint64_t seed;          /* Philox4x32-10 key: (seed mod 2^32, seed >> 32).  Same-colour sites
                             (x, y) and (x, y + 2) with y mod 4 in {0, 1} share one call per sweep:
                             counter (y*nx + x, sweep, chain, grid), words (w0, w1) -> (u, r) of the
                             first site, (w2, w3) of the second; the hot start uses counter
                             (y*nx + x, 0xFFFFFFFF, chain, grid) and w0 */
  int32_t model;          /* pair interaction: MPR_MODEL_MPR (Eq. 3) or MPR_MODEL_GMRF (Sec. 4.4) */
  int32_t boundary;       /* mpr_boundary: MPR_BC_OPEN (default) or MPR_BC_REPLICATE */
} mpr_params;

typedef struct {
  int32_t records;        /* realisations recorded per chain */
  int32_t reserved;
  double *a_eq;           /* host [total chains] or NULL: a at the end of equilibration */
  double *acc_eq;         /* host [total chains] or NULL: mean acceptance over the equilibration sweeps */
  double *acc_samp;       /* host [total chains] or NULL: mean acceptance over the sampling sweeps */
} mpr_fill_report;

/* Fill *p with the paper's defaults (Sec. 2.5): q = 0.5, A_targ = 0.3,
 * k_a = 3, adapt_every = 1, a_sample_keep = 0, FP32, library-chosen tiles,
 * seed 0, the MPR interaction, open boundaries. */
void mpr_default_params(mpr_params *p);

/*
 * Set up grids for simulation: Eq. (2) maps each grid's samples onto
 * [0, 2*pi] with that grid's z_min, z_max; gaps are hot-started with
 * phi = 2*pi*U (Algorithm 2, steps 1.8 and 2.1); the a of every chain is 1
 * (step 1.10) and the sweep counter is 0.
 *
 * grids[n_grids]: host array of grid descriptors (device data pointers).
 *   Total chains must not exceed 2^31 - 1.
 * workspace: device memory, 256-byte aligned, of at least *ws_bytes bytes.
 *   With workspace == NULL the call only writes the required size to
 *   *ws_bytes and returns MPR_OK without creating a context.
 * hip_stream: hipStream_t the context orders its work on (NULL = default).
 * On success *ctx receives a new context.
 * Errors: MPR_E_ARG (bad params, non-finite z at a sample site),
 *   MPR_E_SHAPE, MPR_E_DEGENERATE (all samples of a grid equal; a grid with
 *   no sample is allowed), MPR_E_WORKSPACE, MPR_E_HIP.
 * Synchronises the stream (the per-grid z_min / z_max are validated).
 */
mpr_status mpr_init_field(mpr_ctx **ctx, const mpr_grid *grids, int32_t n_grids, const mpr_params *p,
                          void *workspace, size_t *ws_bytes, void *hip_stream);

/*
 * Run n_sweeps hybrid sweeps (Algorithm 1: over-relaxation then restricted
 * Metropolis at every gap site, in checkerboard order) of every chain.
 * T: host [n_grids], reduced temperatures; +INF (beta = 0) and 0 allowed.
 * flags: MPR_ADAPT applies the a-rule after every adapt_every sweeps
 *   (Algorithm 2, step 4.2) with the global sweep index as its counter;
 *   MPR_TRACE_E evaluates e of Eq. (5) after every sweep;
 *   MPR_NO_OR leaves out over-relaxation.
 * trace: device [n_sweeps][total chains][2] doubles or NULL; receives the
 *   acceptance ratio A and (with MPR_TRACE_E, else NaN) e of each sweep.
 * With MPR_ADAPT, adapt_every = 1 and an FP32 context whose launch shape
 * allows it (below), a-rule sweeps from global sweep 8 on may run two per
 * pass: the second with the a that each chain's last outcome predicts, the
 * pass rerun for the chains whose first-sweep outcome differs.  Results are
 * bitwise those of one sweep per pass.  MPR_SPECULATE=0 in the environment
 * when the context is created turns this off.
 * Asynchronous.  Errors: MPR_E_ARG, MPR_E_STATE, MPR_E_HIP.
 */
mpr_status mpr_sweep(mpr_ctx *ctx, int32_t n_sweeps, const double *T, uint32_t flags, double *trace);

/*
 * Algorithm 2, step 4 with automatic detection of equilibrium: sweeps of
 * every chain (step 4.1; over-relaxation unless MPR_NO_OR), the a-rule
 * (4.2) with MPR_ADAPT, the specific energy e of Eq. (5) after every sweep
 * (4.3), and after sweep i + 1 (i counting this call's sweeps from 0), when
 * i >= n_fit and i is a multiple of n_f, the slope of each chain's last
 * n_fit energies by the Savitzky-Golay filter of degree 1, i.e. of their
 * least-squares line (4.4).  A chain is equilibrated at the first check
 * whose slope is >= 0; the chains of the context sweep in lock-step until
 * all are, or for i_max + 1 sweeps.  The a-rule's counter is the global
 * sweep index, as in mpr_sweep.  Follow with mpr_fill(n_eq = 0) to sample.
 * T: host [n_grids].  flags: MPR_ADAPT, MPR_NO_OR.  n_f >= 1, n_fit >= 2,
 * i_max >= 0.
 * trace: device [i_max + 1][total chains][2] doubles (required): A and e
 *   of each sweep run.
 * n_done: host, nullable: sweeps run.  eq_at: host [total chains],
 *   nullable: sweeps after which each chain's slope was first >= 0, or -1.
 * Synchronises the stream every n_f sweeps once i >= n_fit (host-driven
 * checks).  Errors: MPR_E_ARG, MPR_E_STATE, MPR_E_HIP.
 */
mpr_status mpr_equilibrate(mpr_ctx *ctx, const double *T, int32_t n_f, int32_t n_fit, int32_t i_max, uint32_t flags,
                           double *trace, int32_t *n_done, int32_t *eq_at);

/*
 * Specific energies of the current state.
 * what == MPR_SAMPLE_PAIRS: e_out[n_grids] receives Eq. (4), the mean of
 *   -cos(q dphi) over unordered sample-sample nearest-neighbour pairs, and
 *   npairs_out[n_grids] (nullable) their count N_SP; a grid with N_SP = 0
 *   gets NaN and the call returns MPR_E_NOPAIRS.
 * what == MPR_STATE: e_out[total chains] receives Eq. (5), H / N_GP over all
 *   pairs of each chain's current state; npairs_out[total chains] gets N_GP.
 * Per-pair terms are summed as 2 sin^2(q dphi / 2) in the context's dtype
 * within a workgroup and in FP64 across workgroups.
 * Host outputs; synchronises the stream.
 */
mpr_status mpr_specific_energy(mpr_ctx *ctx, int32_t what, double *e_out, int64_t *npairs_out);

/*
 * Specific energy matching (Sec. 2.3): solve e(T) = e_s for each e_s[i] on
 * a tabulated equilibrium curve (tab_T[k], tab_e[k]), k < n_tab.  The curve
 * is the monotone piecewise-cubic Hermite (PCHIP, Fritsch-Carlson) fit of
 * log(1 + e) against log T; the root is bracketed between table nodes and
 * refined by bisection to the last bit.  Pure host FP64; no context needed.
 * tab_T strictly increasing and > 0; tab_e non-decreasing, in (-1, 0);
 * n_tab >= 2.  An e_s outside [tab_e[0], tab_e[n_tab-1]] is clamped to the
 * nearer end: T_out = that end's T and item_status[i] (nullable) =
 * MPR_E_RANGE, and the call returns MPR_E_RANGE.  NaN e_s gives NaN and
 * MPR_E_ARG for that item.
 */
mpr_status mpr_match_T(const double *e_s, int32_t n, const double *tab_T, const double *tab_e, int32_t n_tab,
                       double *T_out, mpr_status *item_status);

/*
 * Algorithm 2, steps 4-6, with fixed sweep counts: n_eq equilibration
 * sweeps with the a-rule, then n_samp sampling sweeps (a = 1 unless
 * a_sample_keep) of which every stride-th is recorded as a realisation;
 * the conditional mean and standard deviation over all recorded states of
 * all chains of a grid are mapped back with the inverse of Eq. (2).
 * Continues from the context's current state and sweep counter.
 * T: host [n_grids].  zhat, zstd: device [sum nx*ny] doubles, grids back to
 * back in order (zstd nullable); sample sites get z and 0.
 * rep: host, nullable.  Requires n_samp / stride >= 1 and every grid to have
 * samples (else MPR_E_DEGENERATE).  Synchronises the stream.
 */
mpr_status mpr_fill(mpr_ctx *ctx, const double *T, int32_t n_eq, int32_t n_samp, int32_t stride, double *zhat,
                    double *zstd, mpr_fill_report *rep);

/*
 * Validation measures of Sec. 3.3 for grid `grid` over its prediction sites
 * (known == 0 in the context's mask), with eps = Z - Z_hat:
 * out (host [8]) = AAE (mean |eps|), ARE (mean eps/Z), AARE (mean
 * |eps|/Z), RASE (sqrt of mean eps^2), R (linear correlation coefficient
 * of Z and Z_hat), P (number of prediction sites), mean Z, mean Z_hat.
 * z_true: device [ny*nx], the complete field (the values the gaps hide);
 * a gap site whose z_true is NaN is left out, which scores a subset of the
 * gaps (an edge band, or held-out samples in a cross-validation).
 * zhat: device [ny*nx], e.g. this grid's part of mpr_fill's output.
 * FP64, deterministic order.  Synchronises the stream.  Errors: MPR_E_ARG,
 * MPR_E_DEGENERATE (no prediction site left; out[5] = 0), MPR_E_HIP.
 */
mpr_status mpr_validation_measures(mpr_ctx *ctx, int32_t grid, const double *z_true, const double *zhat,
                                   double *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): the validation measures of
 * mpr_validation_measures without a context, on the library's own static
 * device scratch (one fixed array per device, kept until the process
 * ends); no hipMalloc, no allocating library call, no synchronisation.
 * z_true, zhat: device [n_sites] doubles; known: device [n_sites] bytes
 * (1 = sample, left out); shift: subtracted from Z and Z_hat before the
 * second moments of R (pass the grid's z_min to reproduce
 * mpr_validation_measures bit for bit); out: DEVICE [8] doubles, the same
 * eight values, written asynchronously on hip_stream (out[5] = 0 when no
 * gap site has a finite z_true).  n_sites at most 107 372 544 (26214 chunks
 * of 4096 sites), else MPR_E_ARG.  Every call on a device shares that
 * device's scratch: calls that overlap on one device race.  Errors:
 * MPR_E_ARG, MPR_E_HIP.
 */
mpr_status mpr_validation_measures_static(const double *z_true, const double *zhat, const uint8_t *known,
                                          int64_t n_sites, double shift, double *out, void *hip_stream);

/*
 * Give every grid of the context its own modification factor q of Eq. (3)
 * (q: host [n_grids], each in (0, 0.5]), in place of mpr_params.q.  The
 * sample and state specific energies and the sweeps of each grid then use
 * its q; a batch can hold fits of several q, as the q selection of Sec. 6
 * needs.  Kept by mpr_reinit.  Errors: MPR_E_ARG, MPR_E_STATE (GMRF
 * interaction, or a context created with q = 1), MPR_E_HIP.  Synchronises
 * the stream.
 */
mpr_status mpr_set_grid_q(mpr_ctx *ctx, const double *q);

/*
 * Choose q in (0, 1/2] by K-fold cross-validation, the extension proposed
 * in Sec. 6.  The sample sites are split into n_folds folds by `fold`; for
 * candidate i and fold k, the fold's samples are hidden and the method runs
 * on the rest: Eq. (2) on the training samples, e_s (Eq. 4) at q[i], T-hat
 * by specific energy matching on candidate i's own table (as mpr_match_T; a
 * clamped T-hat is used as it is), then mpr_fill(n_eq, n_samp, stride).
 * All n_q * n_folds fits run as one batch (fit (i, k) is grid
 * i * n_folds + k of the batch, which keys its random stream).  The score
 * of a candidate is the AAE over all held-out samples (each is held out
 * once); the least score wins, and among equal scores the larger q.
 *
 * grid: the data (device z and known, as for mpr_init_field); chains =
 *   chains per fit.  p: the fits' parameters (p->q is ignored; the MPR
 *   interaction is required).
 * fold: device [ny*nx] uint8: the fold of each sample site; a sample whose
 *   id is >= n_folds is never held out; ignored at gaps.  2 <= n_folds <= 254.
 * q: host [n_q], the candidates.  tab_T, tab_e: host [n_q] pointers to each
 *   candidate's e(T) table (host arrays of n_tab[i] >= 2 values, as for
 *   mpr_match_T).
 * workspace, ws_bytes: device memory for the batch and its fold masks,
 *   256-byte aligned; with workspace == NULL only *ws_bytes is set.
 * score: host [n_q * 3] or NULL: pooled AAE, pooled RASE over the held-out
 *   samples, and the mean T-hat over the folds.  best: host, the chosen
 *   candidate's index.
 * Errors: MPR_E_ARG, MPR_E_SHAPE, MPR_E_WORKSPACE, MPR_E_DEGENERATE (a fold
 * with no held-out sample, or training samples of one value),
 * MPR_E_NOPAIRS, MPR_E_HIP; the message is mpr_last_error(NULL).
 * Synchronises the stream.
 */
mpr_status mpr_cv_select_q(const mpr_grid *grid, const mpr_params *p, const uint8_t *fold, int32_t n_folds,
                           const double *q, int32_t n_q, const double *const *tab_T, const double *const *tab_e,
                           const int32_t *n_tab, int32_t n_eq, int32_t n_samp, int32_t stride, void *workspace,
                           size_t *ws_bytes, void *hip_stream, double *score, int32_t *best);

/*
 * Set the context up again from the caller's z and known buffers given to
 * mpr_init_field (same shapes; the values and the gap pattern may have
 * changed): Eq. (2) bounds, the hot start of Algorithm 2, steps 1.8 and
 * 2.1, a = 1 (step 1.10), sweep counter 0 -- the state of a fresh context,
 * without its host set-up.  Keeps the tuned launch shape and the fill
 * graph.  Synchronises the stream.  Errors: MPR_E_ARG (non-finite z at a
 * sample site), MPR_E_DEGENERATE (z_max == z_min); the context is then
 * unusable until a successful mpr_reinit.
 */
mpr_status mpr_reinit(mpr_ctx *ctx);

/*
 * Fill graph (enable != 0; off by default): mpr_fill records its device
 * work from the equilibration sweeps to the last sampling pass into a
 * hipGraph and replays it when called again from the same sweep counter,
 * pass parity, launch shape and sweep counts -- e.g. after mpr_reinit --
 * recording afresh otherwise.  Results are bitwise those of the plain
 * path.  The temperatures, the a-rule state and the accumulators live in
 * device memory, so a replay reads the current ones.  enable == 0 drops the
 * graph.
 */
mpr_status mpr_set_graph(mpr_ctx *ctx, int32_t enable);

/*
 * Copy the angles of one chain out (mpr_get_phi) or in (mpr_set_phi), as
 * ny*nx device doubles in natural row-major order.  mpr_set_phi writes gap
 * sites only (sample sites keep their Eq. (2) values); gap values must lie
 * in [0, 2*pi).  In FP32 contexts values are rounded to float and kept
 * below 2*pi.  Asynchronous.  Errors: MPR_E_ARG.
 */
mpr_status mpr_get_phi(mpr_ctx *ctx, int32_t grid, int32_t chain, double *phi);
mpr_status mpr_set_phi(mpr_ctx *ctx, int32_t grid, int32_t chain, const double *phi);

/*
 * The rest of a chain's state: the global sweep counter (which keys the
 * random stream and the a-rule) and the a of every chain (host [total
 * chains]).  With the angles this is a complete checkpoint: a run resumed
 * from it continues bit for bit.  Synchronise the stream.
 */
mpr_status mpr_get_chain_state(mpr_ctx *ctx, int64_t *sweep_index, double *a);
mpr_status mpr_set_chain_state(mpr_ctx *ctx, int64_t sweep_index, const double *a);

/*
 * Autotuner: choose the sweeps fused per pass (up to the context's
 * sweeps_per_pass) and the sweep workgroup size (256, 512 or 1024 threads;
 * also 64 and 128 when no tile holds more than 1024 sites, i.e. for batches
 * of small grids) by timing trial passes of
 * at least trial_sweeps sweeps on the context's own grids at the host
 * temperatures T[n_grids].  The angles, the sweep counter and every chain's
 * a are restored exactly afterwards, so the call has no effect on results;
 * neither choice changes results either (tiling and fusion are bitwise
 * invariant).  The workgroup size of single-sweep passes (the a-rule runs
 * one sweep per pass) is chosen apart, as the fastest at one sweep per
 * pass.  Choices are cached per batch shape for the process, so a later
 * context of the same shape reuses them without timing.  nsw_out,
 * threads_out (nullable) receive the choice for multi-sweep passes,
 * threads1_out (nullable) the workgroup size of single-sweep passes, and
 * persist1_out (nullable) 1 if those passes run on persistent workgroups
 * (each looping over many items and loading the next item while it sweeps
 * the current one), 0 if on one workgroup per item; both kernels are timed.
 * The two-sweep a-rule passes of mpr_sweep are kept (FP32) where their
 * timed two-sweep pass, with 8 us for the check and redo launches, beats a
 * one-sweep pass, at their own fastest workgroup size.
 * Uses the fill accumulators as scratch: do not call during a fill.
 * Synchronises the stream.
 */
mpr_status mpr_autotune(mpr_ctx *ctx, const double *T, int32_t trial_sweeps, int32_t *nsw_out, int32_t *threads_out,
                        int32_t *threads1_out, int32_t *persist1_out);

/*
 * Set the launch shape by hand, as mpr_autotune would: sweeps fused per
 * multi-sweep pass (1 .. the context's sweeps_per_pass), the workgroup size
 * of those passes and of single-sweep passes (64, 128, 256, 512 or 1024),
 * and whether single-sweep passes that record nothing run on persistent
 * workgroups (persist1 != 0; used where a thread's registers hold an
 * item's staged sites and plan entries, else one workgroup per item).  For
 * callers that know their shape (repeated runs, profiling, where timing
 * the candidates would sway the choice).  nsw >= 2 also runs a-rule sweeps
 * two per pass where mpr_sweep allows it, at the multi-sweep workgroup size.
 * The shape does not change results.  MPR_E_ARG if a value is out of range or the pass's LDS exceeds
 * the device's; the context is then unchanged.  No device work.
 */
mpr_status mpr_set_launch_shape(mpr_ctx *ctx, int32_t nsw, int32_t threads, int32_t threads1, int32_t persist1);

/*
 * Tile autotuner: choose the tile shape (mpr_params.tile_x, tile_y) and the
 * most sweeps per pass (sweeps_per_pass) for mpr_init_field of these grids
 * and params, before any context exists.  Each candidate tile (FP32: 64x64,
 * 32x32, 64x32, 128x32, 128x64, 96x96; FP64: 32x32, 16x16, 32x16, 64x32,
 * 64x64), at the largest sweeps_per_pass up to p->sweeps_per_pass (or the
 * default, 8 in FP32 and 1 in FP64) whose LDS the device holds, is set up
 * as a context in the workspace and its launch shape tuned as by
 * mpr_autotune at the host temperatures T[n_grids]; the tile whose fill
 * would take the least time wins, a fill costed as n_eq sweeps at one sweep
 * per pass (the a-rule's pace when adapt_every == 1, else the tuned pace)
 * plus n_samp sweeps at the tuned pace.  Another tile replaces the library
 * default (the first candidate) only when its fill costs at least 5 % less:
 * closer candidates differ by timing noise.
 * Tiling and fusion do not change results (every tile keeps the
 * checkerboard order of Sec. 5.2), so the choice affects speed only.  p's own tile is
 * ignored.  Choices, and each candidate's launch shape, are cached per
 * batch shape for the process; mpr_autotune on a context initialised with
 * the chosen tile and sweeps_per_pass then reuses the cached shape.
 *
 * workspace: device memory, 256-byte aligned, of at least *ws_bytes bytes
 *   (the largest candidate's mpr_init_field need); with workspace == NULL
 *   the call only writes that size to *ws_bytes.  Its contents are scratch.
 * tile_x, tile_y, sweeps_per_pass (nullable) receive the choice.
 * Errors: those of mpr_init_field for the grids and params; MPR_E_ARG for
 *   n_eq < 0, n_samp < 0, n_eq + n_samp < 1, trial_sweeps < 1 or no
 *   candidate that fits the LDS at a requested sweeps_per_pass.
 * Synchronises the stream.
 */
mpr_status mpr_autotune_tile(const mpr_grid *grids, int32_t n_grids, const mpr_params *p, const double *T,
                             int32_t n_eq, int32_t n_samp, int32_t trial_sweeps, void *workspace, size_t *ws_bytes,
                             void *hip_stream, int32_t *tile_x, int32_t *tile_y, int32_t *sweeps_per_pass);

/*
 * Kernel timing, for measurement.  With enable != 0 every later run of
 * back-to-back sweep-kernel launches (one mpr_sweep call, or one phase of
 * mpr_fill) is bracketed by two HIP events on the context's stream, with no
 * other kernel inside the bracket; mpr_get_timing synchronises the stream
 * and returns the summed milliseconds between those event pairs, the number
 * of sweep launches and the site-sweeps they processed (lattice sites times
 * sweeps, summed over chains), then resets the sums.  The bracket includes
 * the short queue gaps between launches; with the fill graph on, it spans
 * the whole graph, whose few clearing and copy kernels are then inside it.
 * enable == 0 stops recording.
 */
mpr_status mpr_set_timing(mpr_ctx *ctx, int32_t enable);
mpr_status mpr_get_timing(mpr_ctx *ctx, double *sweep_ms, int64_t *launches, int64_t *site_sweeps);

/* Release a context (NULL-safe).  Does not free the workspace. */
void mpr_destroy(mpr_ctx *ctx);

/* Last error message of ctx, or of the calling thread when ctx == NULL.
 * Never NULL; valid until the next call on the same context or thread. */
const char *mpr_last_error(const mpr_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MPR_H */
