// Internal declarations shared by the kernels and the host side of libmpr.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpr {

constexpr int kThreads = 256;       // threads per workgroup of every kernel (4 wave64)
constexpr int kMaxPass = 16;        // sweeps fused into one pass, at most
constexpr int kChunk = 4096;        // sites per workgroup in the streaming kernels

// One grid of a batch, as the device sees it.  Angles of chain c of grid g
// live at state[state_off + c*ny*nx + y*nx + x]; z and the fill outputs at
// site_off + y*nx + x.  A sample (frozen) site is stored with its sign bit
// set: the angle is |v|, and gap angles are >= +0.
struct GridDesc {
  int32_t nx, ny, chains, reserved0;
  int32_t tiles_x, tiles_y;        // sweep tiles of one chain
  int32_t chain_base;              // global index of chain 0
  int32_t grid_id;                 // index of the grid in the batch
  int64_t item_begin;              // first sweep work item (grid, chain, tile)
  int64_t plan_begin;              // first tile of this grid in the gap-site plan
  int64_t plan_ebase;              // first plan entry of this grid
  int64_t plan_cap;                // plan entries reserved per tile of this grid
  int64_t cb_begin;                // first chain-chunk block (init, per-chain energy)
  int64_t sb_begin;                // first site-chunk block (min/max, sample energy, finalize)
  int64_t state_off, site_off;
  int64_t n_gap;                   // gap sites per chain
  int64_t n_pairs;                 // N_GP of Eq. (5)
  double zmin, zmax;               // Eq. (2) over the samples; NaN without samples
  double q, inv_q;                 // modification factor of Eq. (3) for this grid, and 1/q
};

// The end of a pass whose per-chain acceptance and energy sums are complete
// but not yet applied: turned into acceptance ratios and trace rows, and run
// through the a-rule, by the next pass's sweep kernel (or k_pass_end).
struct PassEnd {
  int32_t valid;                   // 0: nothing pending
  int32_t nsw, adapt, has_energy;
  uint32_t sweep0;                 // global index of that pass's first sweep
  int64_t trace_row0;
  double *trace;                   // [rows][chains][2] or nullptr
  const uint32_t *counts;          // that pass's accepted counts [chains][kMaxPass]
  const double *energy;            // that pass's energy sums, or nullptr
  const double *a_in, *win_in;     // a and a-rule window before that pass
};

// Pair interaction of the sweep kernel, a template parameter: the MPR
// energy of Eq. (3) with q < 1 or q = 1, or the Gaussian (GMRF) variant
// H_ij = 1 - dphi^2 / (2 pi^2) of Sec. 4.4.
enum SweepModel : int { kMprQ = 0, kMprQ1 = 1, kGmrf = 2 };

template <typename P>
struct SweepArgs {
  const GridDesc *grids;
  int32_t n_grids, total_chains;
  int32_t tile_x, tile_y;
  int32_t nsw;                     // sweeps in this pass
  int32_t lds_w, lds_h;            // LDS extent in sites (lds_w even)
  int32_t q_is_one;
  int32_t gmrf;                    // 1: GMRF pair interaction (mpr_params.model)
  int32_t or_step;                 // 1: Algorithm 1, step 1 (over-relaxation); 0: Metropolis only
  int32_t rep;                     // 1: replicate auxiliary nodes around the grid (mpr_params.boundary)
  uint32_t key0, key1;
  uint32_t sweep0;                 // global index of the pass's first sweep
  uint32_t record_mask, first_mask;
  int32_t adapt, adapt_every;      // a-rule (Algorithm 2, step 4.2)
  double a_targ, k_a;
  // Speculative two-sweep a-rule pass (adapt_every == 1): sweep 1 runs with
  // the a that the last known outcome predicts; tile 0 of each chain stores
  // that prediction (1: acceptance below a_targ) in pred[chain] and item 0
  // clears pred[chains], the count of the redo list that follows.  The redo
  // launch reruns the chains listed in redo[1 .. redo[0]] with the other
  // outcome (redo = pred + chains).
  int32_t spec;
  uint32_t *pred;
  const uint32_t *redo;
  const P *src;
  P *dst;
  const double *beta;              // per chain
  PassEnd pe;                      // previous pass, if its end is pending
  double *a_now, *win_now;         // a and window this pass runs with (written by tile 0 if pe.valid)
  double *accsum;                  // per chain, sum of acceptance ratios (written by tile 0)
  uint32_t *counts;                // this pass: [chains][kMaxPass] accepted updates
  double *energy;                  // this pass: [chains][kMaxPass] or nullptr (written by k_energy_reduce)
  double *energy_part;             // this pass: [kMaxPass][n_items] energy of each item's interior pairs
  uint32_t *counts_clear;          // buffer of the pass after next, cleared by tile 0
  P *acc_ref, *acc_s1, *acc_s2;    // fill accumulators (state layout)
  // Gap-site plan (k_plan): per tile, the pairs of same-colour sites
  // (y, y + 2) in a column, y mod 4 in {0, 1}, that hold a gap site within
  // ring distance plan_dmax of the interior, colour 0 then colour 1, each
  // sorted by ring (a pair's ring: the least Manhattan distance from the
  // interior rectangle of its gap sites within plan_dmax); entry =
  // ((y - y0 + kPlanOffset) << 8) | (x - x0 + kPlanOffset) of the pair's
  // first site.  plan_cum[tile][c][r] = number of colour-c pairs with
  // ring < r, r = 0 .. plan_dmax + 1.
  const uint16_t *plan;
  const uint32_t *plan_cum;
  int32_t plan_dmax;
  int64_t n_items;                 // workgroups of the launch: (grid, chain, tile) items
  // Grid of item k * kItemStride, k = 0 .. (n_items - 1) / kItemStride,
  // then n_grids - 1: the grid of an item lies between two entries.
  const int32_t *item_grid;
};

// Items per entry of SweepArgs::item_grid.
constexpr int kItemStride = 256;

// Entries of the gap-site plan are packed into 16 bits with an offset of 34
// around the tile origin (a pair's first site lies up to plan_dmax + 2
// rows above the tile); with plan_dmax <= 32 this bounds the tile to 188
// sites (188 - 1 + 32 + 34 <= 255).
constexpr int kPlanOffset = 34;
constexpr int kMaxTile = 188;

// Launchers (kernels.hip).  All return the hipError_t of the launch.
template <typename P>
hipError_t launch_sweep(const SweepArgs<P> &a, int threads, int64_t n_items, size_t lds_bytes, hipStream_t s);
// The redo launch of a speculative pass (FP32): same arguments, redo set;
// `blocks` workgroups share the listed chains' items.
hipError_t launch_sweep_redo(const SweepArgs<float> &a, int threads, int blocks, size_t lds_bytes, hipStream_t s);
// After a speculative pass: per chain, compare sweep 0's a-rule outcome with
// the prediction; where they differ clear the chain's counts of the pass and
// list the chain in redo[1 ..], counted in redo[0].
hipError_t launch_spec_check(const GridDesc *g, int n_grids, int total_chains, uint32_t *counts, const double *win_in,
                             int adapt_every, double a_targ, const uint32_t *pred, uint32_t *redo, hipStream_t s);
template <typename P>
hipError_t launch_pass_end(const SweepArgs<P> &a, hipStream_t s);
// Per chain and sweep of a pass with the energy traced: the sum of the
// chain's per-item partials in a fixed order -> energy[chain][s].
hipError_t launch_energy_reduce(const GridDesc *g, int n_grids, int total_chains, int64_t n_items, int nsw,
                                const double *part, double *energy, hipStream_t s);
// Persistent single-sweep kernel (k_sweep1): registers a thread holds for
// the next item, which bound the tiles it can run.
// LDS sites a thread stages (lds_w * lds_h <= threads * p1_sites) and plan
// pairs it holds per colour (pairs within the pass's reach <= threads *
// p1_plan), by workgroup size.
constexpr int p1_sites(int threads) { return threads >= 1024 ? 6 : (threads >= 512 ? 11 : 12); }
constexpr int p1_plan(int threads) { return threads >= 1024 ? 2 : (threads >= 512 ? 3 : 6); }
template <typename P>
hipError_t launch_sweep1(const SweepArgs<P> &a, int threads, int64_t blocks, size_t lds_bytes, hipStream_t s);
// Workgroups of k_sweep1 that are resident at once on the device (a multiple
// of 8, one share per XCD), or 0 if the occupancy cannot be queried.
template <typename P>
int64_t sweep1_resident(int threads, int model, bool rep, size_t lds_bytes);
// Largest workgroup the sweep kernel instance for `threads` can run with
// (0 if it cannot be queried).
template <typename P>
int sweep_max_threads(int threads);
template <typename P>
hipError_t launch_plan(const GridDesc *g, int n_grids, int64_t n_tiles, const P *state, int tile_x, int tile_y,
                       int dmax, uint16_t *plan, uint32_t *plan_cum, hipStream_t s);
hipError_t launch_minmax(const GridDesc *g, int n_grids, int64_t n_blocks, const double *const *z,
                         const uint8_t *const *known, double *part, hipStream_t s);
hipError_t launch_minmax_final(const GridDesc *g, int n_grids, const double *part, double *out, hipStream_t s);
template <typename P>
hipError_t launch_init(const GridDesc *g, int n_grids, int64_t n_blocks, const double *const *z,
                       const uint8_t *const *known, P *s0, P *s1, P q_unused, uint32_t k0, uint32_t k1,
                       hipStream_t s);
template <typename P>
hipError_t launch_energy(const GridDesc *g, int n_grids, int64_t n_blocks, int what, const P *state, int gmrf,
                         double *part, hipStream_t s);
hipError_t launch_energy_final(const GridDesc *g, int n_grids, int what, int n_units, const double *part,
                               double *out, hipStream_t s);
template <typename P>
hipError_t launch_finalize(const GridDesc *g, int n_grids, int64_t n_blocks, const double *const *z,
                           const P *state, const P *ref, const P *s1, const P *s2, int32_t records,
                           double *zhat, double *zstd, hipStream_t s);
template <typename P>
hipError_t launch_get_phi(const P *state, int64_t n, double *out, hipStream_t s);
template <typename P>
hipError_t launch_set_phi(P *s0, P *s1, int64_t n, const double *in, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);
hipError_t launch_copy_f64(double *dst, const double *src, int64_t n, hipStream_t s);
hipError_t launch_cv_prepare(const double *z, const uint8_t *known, const uint8_t *fold, int n_folds, int64_t n,
                             uint8_t *masks, double *zt, hipStream_t s);
// Validation measures of one grid (kMeasureSums partial sums per chunk of
// kChunk sites in part; eight results in out).
constexpr int kMeasureSums = 10;
hipError_t launch_measures(const double *z, const double *zh, const uint8_t *known, int64_t n, double shift,
                           double *part, double *out, hipStream_t s);

}  // namespace mpr
