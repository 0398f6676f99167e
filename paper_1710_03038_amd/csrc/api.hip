// Host side of libmpr: the C ABI declared in include/mpr.h.
//
// The library owns no device memory.  mpr_init_field carves every device
// array it needs out of the caller's workspace; the context holds only
// host metadata and views into that workspace.  All work is ordered on the
// caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "mpr.h"

using namespace mpr;

namespace {

thread_local std::string g_thread_err;

struct Views {
  GridDesc *gd = nullptr;
  const double **zp = nullptr;
  const uint8_t **kp = nullptr;
  void *st[2] = {nullptr, nullptr};
  void *acc_ref = nullptr, *acc_s1 = nullptr, *acc_s2 = nullptr;
  double *a = nullptr, *beta = nullptr, *window = nullptr, *accsum = nullptr;
  uint32_t *counts = nullptr;
  double *energy = nullptr;
  double *energy_part = nullptr;  // per-item energies of a traced pass [kMaxPass][n_items]
  double *part = nullptr, *out = nullptr;
  double *rep = nullptr;  // fill report scratch: a and acceptance after equilibration [2][C]
  uint16_t *plan = nullptr;
  uint32_t *plan_cum = nullptr;
  int32_t *item_grid = nullptr;  // coarse item -> grid index (SweepArgs::item_grid)
  uint32_t *spec = nullptr;      // speculative a-rule passes: predictions [chains], then the redo list (count, chains)
};

struct Plan {
  std::vector<GridDesc> gd;
  std::vector<int32_t> item_grid;  // host copy of the coarse item -> grid index
  int total_chains = 0;
  int64_t n_items = 0, n_cblocks = 0, n_sblocks = 0, state_elems = 0, sites = 0;
  int64_t n_tiles = 0, plan_entries = 0;
  int tile_x = 0, tile_y = 0, nsw_max = 1, dmax = 2;
  size_t elem = 0;
  size_t bytes = 0;
  Views v;  // offsets from the workspace base until bound
};

}  // namespace

struct mpr_ctx {
  hipStream_t stream = nullptr;
  mpr_params p{};
  int n_grids = 0;
  Plan plan;
  Views v;
  int cur = 0;                 // index of the state buffer holding the current angles
  int64_t sweep_index = 0;     // global sweep counter (keys the random stream)
  int64_t pass_no = 0;         // passes run so far: selects the counter and a buffers
  PassEnd pending{};           // the last pass, until its end has been applied
  int nsw_max = 1;             // the most sweeps per pass the plan supports
  int nsw_run = 1;             // sweeps per pass used (autotuned, <= nsw_max)
  int threads = 256;           // workgroup size of the sweep kernel
  int threads1 = 256;          // ... for single-sweep passes (the a-rule's); tuned apart
  bool persist1 = false;       // single-sweep passes on persistent workgroups (k_sweep1) where they fit
  // a-rule sweeps (adapt_every == 1) two per pass, the second with a
  // predicted a and a per-chain redo where the prediction fails (FP32)
  bool spec2 = false;
  int threads2 = 256;          // workgroup size of the speculative two-sweep passes
  bool spec_ok = false;        // FP32, a plan of two or more sweeps per pass, and MPR_SPECULATE not 0
  std::map<std::pair<int, size_t>, int64_t> resident1;  // (threads, LDS bytes) -> k_sweep1 workgroups
  size_t lds_limit = 65536;
  std::vector<double> beta_h;  // staging for per-chain inverse temperatures
  std::string err;
  // kernel timing (mpr_set_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop) of pending launches
  size_t ev_used = 0;
  double t_ms = 0.0;
  int64_t t_launches = 0, t_site_sweeps = 0;
  int64_t sites_all_chains = 0;
  std::vector<const uint8_t *> known_h;  // the caller's known buffers, per grid
  // hipGraph of the fill's sweep sequence (mpr_set_graph): valid for the
  // host state and arguments in key, after which the host state is post.
  bool graph_on = false;
  bool capturing = false;
  struct GraphState {
    int64_t sweep_index, pass_no;
    int cur, nsw_run, threads, threads1, threads2;
    int32_t n_eq, n_samp, stride;
    bool keep_a, persist1, spec2;
    bool operator==(const GraphState &o) const {
      return sweep_index == o.sweep_index && pass_no == o.pass_no && cur == o.cur && nsw_run == o.nsw_run &&
             threads == o.threads && threads1 == o.threads1 && threads2 == o.threads2 && n_eq == o.n_eq &&
             n_samp == o.n_samp &&
             stride == o.stride && keep_a == o.keep_a && persist1 == o.persist1 && spec2 == o.spec2;
    }
  };
  GraphState g_key{}, g_post{};
  int64_t g_launches = 0, g_site_sweeps = 0;  // sweep launches inside the graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  ~mpr_ctx() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

namespace {

mpr_status fail(mpr_ctx *c, mpr_status st, const std::string &msg) {
  if (c) c->err = msg;
  else g_thread_err = msg;
  return st;
}

mpr_status hip_fail(mpr_ctx *c, hipError_t e, const char *where) {
  return fail(c, MPR_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, call)                                  \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);  \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

mpr_status check_params(const mpr_params *p) {
  if (!p) return fail(nullptr, MPR_E_ARG, "params is NULL");
  if (!(p->q > 0.0 && p->q <= 0.5) && p->q != 1.0)
    return fail(nullptr, MPR_E_ARG, "q must lie in (0, 0.5] or equal 1");
  if (!(p->a_targ >= 0.0 && p->a_targ <= 1.0)) return fail(nullptr, MPR_E_ARG, "a_targ must lie in [0, 1]");
  if (!(p->k_a > 0.0) || !std::isfinite(p->k_a)) return fail(nullptr, MPR_E_ARG, "k_a must be positive");
  if (p->adapt_every < 1) return fail(nullptr, MPR_E_ARG, "adapt_every must be >= 1");
  if (p->a_sample_keep != 0 && p->a_sample_keep != 1) return fail(nullptr, MPR_E_ARG, "a_sample_keep must be 0 or 1");
  if (p->dtype != MPR_FP32 && p->dtype != MPR_FP64) return fail(nullptr, MPR_E_ARG, "dtype must be MPR_FP32 or MPR_FP64");
  if (p->sweeps_per_pass < 0 || p->sweeps_per_pass > kMaxPass)
    return fail(nullptr, MPR_E_ARG, "sweeps_per_pass must lie in [0, 16]");
  for (int t : {p->tile_x, p->tile_y})
    if (t != 0 && (t < 8 || t > kMaxTile || (t & 1)))
      return fail(nullptr, MPR_E_ARG, "tile sizes must be 0 or even in [8, 188]");
  if (p->model != MPR_MODEL_MPR && p->model != MPR_MODEL_GMRF)
    return fail(nullptr, MPR_E_ARG, "model must be MPR_MODEL_MPR or MPR_MODEL_GMRF");
  if (p->boundary != MPR_BC_OPEN && p->boundary != MPR_BC_REPLICATE)
    return fail(nullptr, MPR_E_ARG, "boundary must be MPR_BC_OPEN or MPR_BC_REPLICATE");
  return MPR_OK;
}

// Lay out the grids and the workspace.  Offsets are relative to the base.
mpr_status make_plan(const mpr_grid *grids, int n, const mpr_params *p, bool need_ptrs, Plan &pl) {
  if (!grids || n < 1) return fail(nullptr, MPR_E_ARG, "need at least one grid");
  pl = Plan();
  pl.elem = p->dtype == MPR_FP64 ? 8 : 4;
  pl.tile_x = p->tile_x ? p->tile_x : (p->dtype == MPR_FP64 ? 32 : 64);
  pl.tile_y = p->tile_y ? p->tile_y : (p->dtype == MPR_FP64 ? 32 : 64);
  // Default: 8 sweeps per pass in FP32 (64 x 64 tiles fit in LDS with the
  // 17-site halo), 1 in FP64 (the plain reference arm).
  pl.nsw_max = p->sweeps_per_pass ? p->sweeps_per_pass : (p->dtype == MPR_FP64 ? 1 : 8);
  pl.dmax = 2 * pl.nsw_max;
  int64_t chains = 0;
  for (int g = 0; g < n; ++g) {
    const mpr_grid &G = grids[g];
    if (G.nx < 1 || G.ny < 1 || (int64_t)G.nx * G.ny < 2 || G.nx > 65536 || G.ny > 65536)
      return fail(nullptr, MPR_E_SHAPE, "grid " + std::to_string(g) + ": need 1 <= nx, ny <= 65536 and nx*ny >= 2");
    if (G.chains < 1) return fail(nullptr, MPR_E_SHAPE, "grid " + std::to_string(g) + ": chains must be >= 1");
    if (G.reserved != 0) return fail(nullptr, MPR_E_ARG, "grid " + std::to_string(g) + ": reserved must be 0");
    if (need_ptrs && (!G.z || !G.known))
      return fail(nullptr, MPR_E_ARG, "grid " + std::to_string(g) + ": z and known must be device pointers");
    GridDesc d{};
    d.nx = G.nx;
    d.ny = G.ny;
    d.chains = G.chains;
    d.tiles_x = (G.nx + pl.tile_x - 1) / pl.tile_x;
    d.tiles_y = (G.ny + pl.tile_y - 1) / pl.tile_y;
    d.chain_base = (int32_t)chains;
    d.grid_id = g;
    const int64_t sites = (int64_t)G.nx * G.ny;
    const int64_t per_chain_blocks = (sites + kChunk - 1) / kChunk;
    d.item_begin = pl.n_items;
    d.plan_begin = pl.n_tiles;
    d.plan_ebase = pl.plan_entries;
    d.plan_cap = (int64_t)std::min(pl.tile_x + 2 * pl.dmax, G.nx) * std::min(pl.tile_y + 2 * pl.dmax, G.ny);
    d.cb_begin = pl.n_cblocks;
    d.sb_begin = pl.n_sblocks;
    d.state_off = pl.state_elems;
    d.site_off = pl.sites;
    d.n_pairs = (int64_t)G.ny * (G.nx - 1) + (int64_t)G.nx * (G.ny - 1);
    d.zmin = d.zmax = NAN;
    d.q = p->q;
    d.inv_q = 1.0 / p->q;
    pl.n_items += (int64_t)G.chains * d.tiles_x * d.tiles_y;
    pl.n_tiles += (int64_t)d.tiles_x * d.tiles_y;
    pl.plan_entries += (int64_t)d.tiles_x * d.tiles_y * d.plan_cap;
    pl.n_cblocks += (int64_t)G.chains * per_chain_blocks;
    pl.n_sblocks += per_chain_blocks;
    pl.state_elems += (int64_t)G.chains * sites;
    pl.sites += sites;
    chains += G.chains;
    if (chains > 0x7fffffff) return fail(nullptr, MPR_E_SHAPE, "more than 2^31 - 1 chains in total");
    pl.gd.push_back(d);
  }
  if (pl.n_items > 0x7fffffff || pl.n_cblocks > 0x7fffffff)
    return fail(nullptr, MPR_E_SHAPE, "batch too large for one launch");
  pl.total_chains = (int)chains;
  {
    const int64_t K = (pl.n_items - 1) / kItemStride + 1;
    pl.item_grid.resize(K + 1);
    int g = 0;
    for (int64_t k = 0; k < K; ++k) {
      const int64_t item = k * kItemStride;
      while (g + 1 < n && pl.gd[g + 1].item_begin <= item) ++g;
      pl.item_grid[k] = g;
    }
    pl.item_grid[K] = n - 1;
  }

  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  Views &v = pl.v;
  const size_t C = (size_t)pl.total_chains;
  v.gd = (GridDesc *)take(sizeof(GridDesc) * n);
  v.zp = (const double **)take(sizeof(void *) * n);
  v.kp = (const uint8_t **)take(sizeof(void *) * n);
  v.st[0] = (void *)take(pl.elem * pl.state_elems);
  v.st[1] = (void *)take(pl.elem * pl.state_elems);
  v.acc_ref = (void *)take(pl.elem * pl.state_elems);
  v.acc_s1 = (void *)take(pl.elem * pl.state_elems);
  v.acc_s2 = (void *)take(pl.elem * pl.state_elems);
  v.a = (double *)take(8 * 2 * C);                 // by pass parity
  v.beta = (double *)take(8 * C);
  v.window = (double *)take(8 * 2 * C);            // by pass parity
  v.accsum = (double *)take(8 * C);
  v.counts = (uint32_t *)take(4 * 3 * C * kMaxPass);  // by pass number mod 3
  v.energy = (double *)take(8 * 3 * C * kMaxPass);
  v.energy_part = (double *)take(8 * (size_t)pl.n_items * kMaxPass);
  v.part = (double *)take(8 * (size_t)std::max<int64_t>(pl.n_sblocks * kMeasureSums, pl.n_cblocks * 2));
  v.out = (double *)take(8 * std::max<size_t>({(size_t)n * 4, C * 2, (size_t)8}));
  v.rep = (double *)take(8 * 2 * C);
  v.plan = (uint16_t *)take(2 * (size_t)pl.plan_entries);
  v.plan_cum = (uint32_t *)take(4 * (size_t)pl.n_tiles * 2 * (pl.dmax + 2));
  v.item_grid = (int32_t *)take(4 * pl.item_grid.size());
  v.spec = (uint32_t *)take(4 * (2 * C + 1));
  pl.bytes = off;
  return MPR_OK;
}

template <typename T> T *rebase(T *off, char *base) { return (T *)(base + (size_t)off); }

void bind(Views &v, const Views &o, void *ws) {
  char *b = (char *)ws;
  v.gd = rebase(o.gd, b);
  v.zp = rebase(o.zp, b);
  v.kp = rebase(o.kp, b);
  for (int i = 0; i < 2; ++i) v.st[i] = rebase((char *)o.st[i], b);
  v.acc_ref = rebase((char *)o.acc_ref, b);
  v.acc_s1 = rebase((char *)o.acc_s1, b);
  v.acc_s2 = rebase((char *)o.acc_s2, b);
  v.a = rebase(o.a, b);
  v.beta = rebase(o.beta, b);
  v.window = rebase(o.window, b);
  v.accsum = rebase(o.accsum, b);
  v.counts = rebase(o.counts, b);
  v.energy = rebase(o.energy, b);
  v.energy_part = rebase(o.energy_part, b);
  v.part = rebase(o.part, b);
  v.out = rebase(o.out, b);
  v.rep = rebase(o.rep, b);
  v.plan = rebase(o.plan, b);
  v.plan_cum = rebase(o.plan_cum, b);
  v.item_grid = rebase(o.item_grid, b);
  v.spec = rebase(o.spec, b);
}

// LDS extent of a pass with nsw sweeps: the tile with a halo of H = 2*nsw
// sites (one more with the energy traced; columns rounded to an even
// count), or the whole grid plus a zero ring when that is smaller.
void lds_extent(const Plan &pl, int nsw, bool energy, int &w, int &h, size_t &bytes) {
  const int H = 2 * nsw + (energy ? 1 : 0), Hx = (H + 1) & ~1;
  w = 0;
  h = 0;
  for (const GridDesc &d : pl.gd) {
    w = std::max(w, std::min(pl.tile_x + 2 * Hx, d.nx + 3));
    h = std::max(h, std::min(pl.tile_y + 2 * H, d.ny + 2));
  }
  w = (w + 1) & ~1;
  // angle + (cos, sin) of both colours, and the staged plan pairs: their
  // first sites lie in rows [oy - 2, oy + h), two rows in every four, so at
  // most w (h + 4) / 2 pairs of 2 bytes
  bytes = (size_t)w * h * 3 * pl.elem + (size_t)w * (h + 4);
}

void lds_extent(const mpr_ctx *c, int nsw, bool energy, int &w, int &h, size_t &bytes) {
  lds_extent(c->plan, nsw, energy, w, h, bytes);
}

double *a_buf(mpr_ctx *c, int64_t pass) { return c->v.a + (pass & 1) * c->plan.total_chains; }
double *win_buf(mpr_ctx *c, int64_t pass) { return c->v.window + (pass & 1) * c->plan.total_chains; }
uint32_t *counts_buf(mpr_ctx *c, int64_t pass) {
  return c->v.counts + (pass % 3) * (int64_t)c->plan.total_chains * kMaxPass;
}
double *energy_buf(mpr_ctx *c, int64_t pass) {
  return c->v.energy + (pass % 3) * (int64_t)c->plan.total_chains * kMaxPass;
}

mpr_status set_beta(mpr_ctx *c, const double *T) {
  if (!T) return fail(c, MPR_E_ARG, "T is NULL");
  c->beta_h.assign(c->plan.total_chains, 0.0);
  for (int g = 0; g < c->n_grids; ++g) {
    const double t = T[g];
    if (std::isnan(t) || t < 0.0) return fail(c, MPR_E_ARG, "T must be >= 0 (or +inf) for every grid");
    const double beta = std::isinf(t) ? 0.0 : (t == 0.0 ? INFINITY : 1.0 / t);
    const GridDesc &d = c->plan.gd[g];
    for (int k = 0; k < d.chains; ++k) c->beta_h[d.chain_base + k] = beta;
  }
  HIP_TRY(c, hipMemcpyAsync(c->v.beta, c->beta_h.data(), 8 * c->beta_h.size(), hipMemcpyHostToDevice, c->stream));
  return MPR_OK;
}

// Sum the elapsed time of all recorded event pairs (synchronises).
mpr_status drain_timing(mpr_ctx *c) {
  if (c->ev_used == 0) return MPR_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < c->ev_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
    c->t_ms += ms;
  }
  c->ev_used = 0;
  return MPR_OK;
}

// Workgroups for a single-sweep pass on persistent workgroups (k_sweep1):
// as many as are resident at once, or fewer for a small batch (a multiple
// of 8, one share per XCD); 0 to use the one-workgroup-per-item kernel:
// when switched off, or when an item's staged sites or plan entries exceed
// what a thread holds in registers.
int64_t resident_blocks1(mpr_ctx *c, int thr, size_t lds) {
  const auto key = std::make_pair(thr, lds);
  auto it = c->resident1.find(key);
  if (it == c->resident1.end()) {
    const int model = c->p.model == MPR_MODEL_GMRF ? kGmrf : (c->p.q == 1.0 ? kMprQ1 : kMprQ);
    const bool rep = c->p.boundary == MPR_BC_REPLICATE;
    const int64_t n = c->p.dtype == MPR_FP64 ? sweep1_resident<double>(thr, model, rep, lds)
                                             : sweep1_resident<float>(thr, model, rep, lds);
    it = c->resident1.emplace(key, n).first;
  }
  return it->second;
}

// Workgroups of k_sweep1 for a one-sweep pass of `thr` threads over this
// LDS extent, or 0 where a thread's registers cannot hold an item (or no
// persistent kernel exists for that size).
int64_t persistent_fit(mpr_ctx *c, int thr, int lds_w, int lds_h, bool energy, size_t lds) {
  if ((int64_t)lds_w * lds_h > (int64_t)thr * p1_sites(thr)) return 0;
  const int D0 = energy ? 2 : 1;  // reach of the colour-0 half-sweep, in rings
  // plan pairs of colour 0 within that reach, at most: their first sites
  // lie in rows [y0 - D0 - 2, iy1 + D0), two rows in every four, with one
  // site of the colour in every 2 columns of [x0 - D0, ix1 + D0)
  const int64_t reach = (int64_t)((c->plan.tile_y + 2 * D0) / 2 + 2) * ((c->plan.tile_x + 2 * D0) / 2 + 1);
  if (reach > (int64_t)thr * p1_plan(thr)) return 0;
  const int64_t res = resident_blocks1(c, thr, lds);
  if (res < 8) return 0;  // also: no persistent kernel for this workgroup size
  return std::min<int64_t>(res, (c->plan.n_items + 7) / 8 * 8);
}

template <typename P> int64_t persistent_blocks(mpr_ctx *c, const SweepArgs<P> &A, size_t lds) {
  if (!c->persist1) return 0;
  return persistent_fit(c, c->threads1, A.lds_w, A.lds_h, A.energy != nullptr, lds);
}

template <typename P>
mpr_status run_pass(mpr_ctx *c, int nsw, bool adapt, bool trace_e, double *trace, int64_t trace_row0,
                    uint32_t record_mask, uint32_t first_mask, bool or_step, bool spec = false) {
  SweepArgs<P> A{};
  int w, h;
  size_t lds;
  lds_extent(c, nsw, trace_e, w, h, lds);
  if (lds > c->lds_limit)
    return fail(c, MPR_E_ARG, "tile and sweeps_per_pass need " + std::to_string(lds) + " bytes of LDS, limit " +
                                  std::to_string(c->lds_limit));
  A.grids = c->v.gd;
  A.n_grids = c->n_grids;
  A.total_chains = c->plan.total_chains;
  A.tile_x = c->plan.tile_x;
  A.tile_y = c->plan.tile_y;
  A.nsw = nsw;
  A.lds_w = w;
  A.lds_h = h;
  A.q_is_one = c->p.q == 1.0;
  A.gmrf = c->p.model == MPR_MODEL_GMRF ? 1 : 0;
  A.rep = c->p.boundary == MPR_BC_REPLICATE ? 1 : 0;
  A.or_step = or_step ? 1 : 0;
  A.key0 = (uint32_t)(c->p.seed & 0xffffffffu);
  A.key1 = (uint32_t)(c->p.seed >> 32);
  A.sweep0 = (uint32_t)c->sweep_index;
  A.record_mask = record_mask;
  A.first_mask = first_mask;
  A.adapt = adapt;
  A.adapt_every = c->p.adapt_every;
  A.a_targ = c->p.a_targ;
  A.k_a = c->p.k_a;
  A.spec = spec ? 1 : 0;
  A.pred = spec ? c->v.spec : nullptr;
  A.redo = nullptr;
  A.src = (const P *)c->v.st[c->cur];
  A.dst = (P *)c->v.st[c->cur ^ 1];
  A.beta = c->v.beta;
  const int64_t pn = c->pass_no;
  A.pe = c->pending;
  A.a_now = a_buf(c, pn);
  A.win_now = win_buf(c, pn);
  A.accsum = c->v.accsum;
  A.counts = counts_buf(c, pn);
  A.energy = trace_e ? energy_buf(c, pn) : nullptr;
  A.energy_part = trace_e ? c->v.energy_part : nullptr;
  A.counts_clear = counts_buf(c, pn + 1);
  A.acc_ref = (P *)c->v.acc_ref;
  A.acc_s1 = (P *)c->v.acc_s1;
  A.acc_s2 = (P *)c->v.acc_s2;
  A.plan = c->v.plan;
  A.plan_cum = c->v.plan_cum;
  A.plan_dmax = c->plan.dmax;
  A.n_items = c->plan.n_items;
  A.item_grid = c->v.item_grid;
  const int64_t blocks1 = nsw == 1 && record_mask == 0 ? persistent_blocks<P>(c, A, lds) : 0;
  if (blocks1 > 0) HIP_TRY(c, launch_sweep1<P>(A, c->threads1, blocks1, lds, c->stream));
  else HIP_TRY(c, launch_sweep<P>(A, spec ? c->threads2 : (nsw == 1 ? c->threads1 : c->threads), c->plan.n_items,
                                  lds, c->stream));
  if (spec) {
    // Check sweep 0's outcome per chain, and rerun the chains it did not
    // predict (the others' workgroups of the redo launch exit at once).
    if constexpr (sizeof(P) == 4) {
      const int C = c->plan.total_chains;
      HIP_TRY(c, launch_spec_check(c->v.gd, c->n_grids, C, A.counts, A.win_now, c->p.adapt_every, c->p.a_targ,
                                   c->v.spec, c->v.spec + C, c->stream));
      A.redo = c->v.spec + C;
      // a few workgroups per CU share the listed chains' items
      const int blocks = (int)std::min<int64_t>(c->plan.n_items, 1024);
      HIP_TRY(c, launch_sweep_redo(A, c->threads2, blocks, lds, c->stream));
    } else {
      return fail(c, MPR_E_STATE, "speculative passes run in FP32 only");
    }
  }
  if (trace_e)
    HIP_TRY(c, launch_energy_reduce(c->v.gd, c->n_grids, c->plan.total_chains, c->plan.n_items, nsw,
                                    c->v.energy_part, A.energy, c->stream));
  if (c->capturing) {
    c->g_launches += 1;
    c->g_site_sweeps += (int64_t)nsw * c->sites_all_chains;
  } else if (c->timing) {
    c->t_launches += 1;
    c->t_site_sweeps += (int64_t)nsw * c->sites_all_chains;
  }
  PassEnd &E = c->pending;
  E.valid = 1;
  E.nsw = nsw;
  E.adapt = adapt;
  E.has_energy = trace_e;
  E.sweep0 = (uint32_t)c->sweep_index;
  E.trace_row0 = trace_row0;
  E.trace = trace;
  E.counts = A.counts;
  E.energy = A.energy;
  E.a_in = A.a_now;
  E.win_in = A.win_now;
  c->cur ^= 1;
  c->sweep_index += nsw;
  c->pass_no += 1;
  return MPR_OK;
}

// Apply the end of the last pass (a-rule, trace, acceptance sums) so that
// a, the window and the sums are current in the buffers of pass pass_no.
template <typename P> mpr_status close_pending(mpr_ctx *c) {
  if (!c->pending.valid) return MPR_OK;
  SweepArgs<P> A{};
  A.grids = c->v.gd;
  A.n_grids = c->n_grids;
  A.total_chains = c->plan.total_chains;
  A.adapt_every = c->p.adapt_every;
  A.a_targ = c->p.a_targ;
  A.k_a = c->p.k_a;
  A.pe = c->pending;
  A.a_now = a_buf(c, c->pass_no);
  A.win_now = win_buf(c, c->pass_no);
  A.accsum = c->v.accsum;
  HIP_TRY(c, launch_pass_end<P>(A, c->stream));
  c->pending.valid = 0;
  return MPR_OK;
}

mpr_status close_pending(mpr_ctx *c) {
  return c->p.dtype == MPR_FP64 ? close_pending<double>(c) : close_pending<float>(c);
}

// Cost of a speculative pass beyond its two sweeps: the per-chain check and
// a redo launch whose workgroups exit at once, about 4 us each (ms).
constexpr double kSpecOverheadMs = 0.008;
// The a-rule's outcome flips back and forth over the first sweeps after a
// hot start while the proposal width settles (on the 8192^2 workload the
// chains' mean acceptance runs 0.47, 0.31, 0.24, 0.31, 0.28, ... about the
// target 0.3), so most early predictions would fail: speculation starts at
// this sweep index.
constexpr int64_t kSpecFromSweep = 8;

// n sweeps in passes of at most nsw_max; with the a-rule no pass crosses the
// end of an adapt_every window, so a is constant within every pass, except
// in speculative two-sweep passes (adapt_every == 1, spec2), whose second
// sweep runs with a predicted a and is redone per chain where the
// prediction fails (run_pass).  rec_stride > 0 records every rec_stride-th
// sweep of this run.
mpr_status run_sweeps(mpr_ctx *c, int64_t n, bool adapt, bool trace_e, double *trace, int rec_stride,
                      bool or_step = true) {
  if (c->sweep_index + n >= 0xFFFFFFFFLL) return fail(c, MPR_E_STATE, "sweep counter would reach 2^32 - 1");
  // Timing brackets the whole run of back-to-back sweep launches with one
  // event pair: per-launch events would stall the queue between launches.
  const bool timed = c->timing && !c->capturing && n > 0;
  if (timed) {
    if (c->ev_used + 2 > c->ev.size()) {
      if (c->ev.size() < 64) {
        for (int i = 0; i < 2; ++i) {
          hipEvent_t e;
          HIP_TRY(c, hipEventCreate(&e));
          c->ev.push_back(e);
        }
      } else {
        const mpr_status st = drain_timing(c);
        if (st != MPR_OK) return st;
      }
    }
    HIP_TRY(c, hipEventRecord(c->ev[c->ev_used], c->stream));
  }
  int64_t done = 0;
  while (done < n) {
    int64_t len = std::min<int64_t>(c->nsw_run, n - done);
    bool spec = false;
    if (adapt) {
      const int64_t ae = c->p.adapt_every;
      len = std::min<int64_t>(len, ae - (c->sweep_index % ae));
      // a-rule sweeps two per pass, the second speculative (see run_pass)
      if (ae == 1 && c->spec2 && !trace_e && rec_stride == 0 && n - done >= 2 && c->nsw_max >= 2 &&
          c->p.dtype == MPR_FP32 && c->sweep_index >= kSpecFromSweep) {
        len = 2;
        spec = true;
      }
    }
    uint32_t rec = 0, first = 0;
    if (rec_stride > 0)
      for (int s = 0; s < len; ++s) {
        const int64_t j = done + s;
        if ((j + 1) % rec_stride == 0) {
          rec |= 1u << s;
          if (j + 1 == rec_stride) first |= 1u << s;
        }
      }
    const mpr_status st =
        c->p.dtype == MPR_FP64 ? run_pass<double>(c, (int)len, adapt, trace_e, trace, done, rec, first, or_step)
                               : run_pass<float>(c, (int)len, adapt, trace_e, trace, done, rec, first, or_step, spec);
    if (st != MPR_OK) return st;
    done += len;
  }
  if (timed) {
    HIP_TRY(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
    c->ev_used += 2;
  }
  return close_pending(c);
}

mpr_status reduce_energy(mpr_ctx *c, int what, std::vector<double> &out) {
  const int units = what ? c->plan.total_chains : c->n_grids;
  const int64_t blocks = what ? c->plan.n_cblocks : c->plan.n_sblocks;
  if (c->p.dtype == MPR_FP64) {
    HIP_TRY(c, launch_energy<double>(c->v.gd, c->n_grids, blocks, what, (const double *)c->v.st[c->cur],
                                     c->p.model, c->v.part, c->stream));
  } else {
    HIP_TRY(c, launch_energy<float>(c->v.gd, c->n_grids, blocks, what, (const float *)c->v.st[c->cur],
                                    c->p.model, c->v.part, c->stream));
  }
  HIP_TRY(c, launch_energy_final(c->v.gd, c->n_grids, what, units, c->v.part, c->v.out, c->stream));
  out.resize((size_t)units * 2);
  HIP_TRY(c, hipMemcpyAsync(out.data(), c->v.out, 16 * (size_t)units, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MPR_OK;
}

// Device part of set-up (mpr_init_field, mpr_reinit): Eq. (2) bounds and
// gap counts of every grid from the caller's z and known, the hot start,
// the gap-site plan, a = 1 and cleared counters; resets the host-side
// sweep state.  Synchronises the stream.
mpr_status device_init(mpr_ctx *c) {
  const int n_grids = c->n_grids;
  std::vector<double> mm((size_t)n_grids * 4);
  for (GridDesc &d : c->plan.gd) d.zmin = d.zmax = NAN;
  HIP_TRY(c, hipMemcpyAsync(c->v.gd, c->plan.gd.data(), sizeof(GridDesc) * n_grids, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, launch_minmax(c->v.gd, n_grids, c->plan.n_sblocks, c->v.zp, c->v.kp, c->v.part, c->stream));
  HIP_TRY(c, launch_minmax_final(c->v.gd, n_grids, c->v.part, c->v.out, c->stream));
  HIP_TRY(c, hipMemcpyAsync(mm.data(), c->v.out, 8 * mm.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int g = 0; g < n_grids; ++g) {
    const double mn = mm[g * 4], mx = mm[g * 4 + 1], cnt = mm[g * 4 + 2], bad = mm[g * 4 + 3];
    if (bad > 0) return fail(c, MPR_E_ARG, "grid " + std::to_string(g) + ": non-finite z at a sample site");
    GridDesc &d = c->plan.gd[g];
    d.n_gap = (int64_t)d.nx * d.ny - (int64_t)cnt;
    if (cnt > 0) {
      if (!(mx > mn)) return fail(c, MPR_E_DEGENERATE, "grid " + std::to_string(g) + ": z_max == z_min");
      d.zmin = mn;
      d.zmax = mx;
    }
  }
  HIP_TRY(c, hipMemcpyAsync(c->v.gd, c->plan.gd.data(), sizeof(GridDesc) * n_grids, hipMemcpyHostToDevice,
                            c->stream));
  const uint32_t key0 = (uint32_t)(c->p.seed & 0xffffffffu), key1 = (uint32_t)(c->p.seed >> 32);
  if (c->p.dtype == MPR_FP64) {
    HIP_TRY(c, launch_init<double>(c->v.gd, n_grids, c->plan.n_cblocks, c->v.zp, c->v.kp, (double *)c->v.st[0],
                                   (double *)c->v.st[1], 0.0, key0, key1, c->stream));
    HIP_TRY(c, launch_plan<double>(c->v.gd, n_grids, c->plan.n_tiles, (const double *)c->v.st[0], c->plan.tile_x,
                                   c->plan.tile_y, c->plan.dmax, c->v.plan, c->v.plan_cum, c->stream));
  } else {
    HIP_TRY(c, launch_init<float>(c->v.gd, n_grids, c->plan.n_cblocks, c->v.zp, c->v.kp, (float *)c->v.st[0],
                                  (float *)c->v.st[1], 0.0f, key0, key1, c->stream));
    HIP_TRY(c, launch_plan<float>(c->v.gd, n_grids, c->plan.n_tiles, (const float *)c->v.st[0], c->plan.tile_x,
                                  c->plan.tile_y, c->plan.dmax, c->v.plan, c->v.plan_cum, c->stream));
  }
  const int64_t C = c->plan.total_chains;
  HIP_TRY(c, launch_fill_f64(c->v.a, 2 * C, 1.0, c->stream));
  HIP_TRY(c, launch_fill_f64(c->v.beta, C, 0.0, c->stream));
  HIP_TRY(c, launch_fill_f64(c->v.window, 2 * C, 0.0, c->stream));
  HIP_TRY(c, launch_fill_f64(c->v.accsum, C, 0.0, c->stream));
  HIP_TRY(c, launch_zero_u32(c->v.counts, 3 * C * kMaxPass, c->stream));
  HIP_TRY(c, launch_fill_f64(c->v.energy, 3 * C * kMaxPass, 0.0, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->cur = 0;
  c->sweep_index = 0;
  c->pass_no = 0;
  c->pending = PassEnd{};
  return MPR_OK;
}

// ---------------------------------------------------------------- PCHIP
// Monotone piecewise-cubic Hermite interpolation (Fritsch & Carlson 1980),
// interior slopes by the weighted harmonic mean of Fritsch & Butland (1984),
// end slopes by the shape-preserving one-sided three-point formula
// (Moler, Numerical Computing with MATLAB, Sec. 3.6).
struct Pchip {
  std::vector<double> x, y, d;
  void build(const std::vector<double> &xs, const std::vector<double> &ys) {
    x = xs;
    y = ys;
    const size_t n = x.size();
    d.assign(n, 0.0);
    std::vector<double> h(n - 1), m(n - 1);
    for (size_t k = 0; k + 1 < n; ++k) {
      h[k] = x[k + 1] - x[k];
      m[k] = (y[k + 1] - y[k]) / h[k];
    }
    if (n == 2) {
      d[0] = d[1] = m[0];
      return;
    }
    auto sgn = [](double v) { return (v > 0) - (v < 0); };
    for (size_t k = 1; k + 1 < n; ++k) {
      if (sgn(m[k - 1]) != sgn(m[k]) || m[k - 1] == 0.0 || m[k] == 0.0) {
        d[k] = 0.0;
      } else {
        const double w1 = 2.0 * h[k] + h[k - 1], w2 = h[k] + 2.0 * h[k - 1];
        d[k] = (w1 + w2) / (w1 / m[k - 1] + w2 / m[k]);
      }
    }
    auto edge = [&](double h0, double h1, double m0, double m1) {
      double e = ((2.0 * h0 + h1) * m0 - h0 * m1) / (h0 + h1);
      if (sgn(e) != sgn(m0)) e = 0.0;
      else if (sgn(m0) != sgn(m1) && std::fabs(e) > 3.0 * std::fabs(m0)) e = 3.0 * m0;
      return e;
    };
    d[0] = edge(h[0], h[1], m[0], m[1]);
    d[n - 1] = edge(h[n - 2], h[n - 3], m[n - 2], m[n - 3]);
  }
  double eval(size_t k, double xv) const {
    const double hk = x[k + 1] - x[k], t = xv - x[k];
    const double mk = (y[k + 1] - y[k]) / hk;
    const double c2 = (3.0 * mk - 2.0 * d[k] - d[k + 1]) / hk;
    const double c3 = (d[k] + d[k + 1] - 2.0 * mk) / (hk * hk);
    return y[k] + t * (d[k] + t * (c2 + t * c3));
  }
};

}  // namespace

// ------------------------------------------------------- static scratch
// Device memory of mpr_validation_measures_static, which allocates nothing:
// the per-chunk partial sums of the measures kernels.  Each device holds its
// own copy for the life of the process.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address, per device, is
// taken once with hipGetSymbolAddress and used everywhere instead.
constexpr int64_t kStaticBlocks = 26214;                        // chunks of kChunk sites
constexpr int64_t kStaticMaxSites = kStaticBlocks * kChunk;      // 107 372 544 sites; 2 MiB of scratch
static __device__ __align__(256) double scratch[kStaticBlocks * kMeasureSums];

namespace {
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_dev;  // device -> address of that device's `scratch`

// The current device's address of `scratch`, looked up on its first use there.
mpr_status static_scratch(double **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_dev.find(dev);
  if (it == g_scratch_dev.end()) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    it = g_scratch_dev.emplace(dev, static_cast<double *>(p)).first;
  }
  *ptr = it->second;
  return MPR_OK;
}
}  // namespace

// =================================================================== ABI
extern "C" {

void mpr_default_params(mpr_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->q = 0.5;
  p->a_targ = 0.3;
  p->k_a = 3.0;
  p->adapt_every = 1;
  p->a_sample_keep = 0;
  p->dtype = MPR_FP32;
  p->sweeps_per_pass = 0;
  p->tile_x = 0;
  p->tile_y = 0;
  p->seed = 0;
  p->model = MPR_MODEL_MPR;
  p->boundary = MPR_BC_OPEN;
}

const char *mpr_last_error(const mpr_ctx *ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

void mpr_destroy(mpr_ctx *ctx) { delete ctx; }

mpr_status mpr_init_field(mpr_ctx **ctx, const mpr_grid *grids, int32_t n_grids, const mpr_params *p,
                          void *workspace, size_t *ws_bytes, void *hip_stream) {
  g_thread_err.clear();
  if (!ws_bytes) return fail(nullptr, MPR_E_ARG, "ws_bytes is NULL");
  mpr_status st = check_params(p);
  if (st != MPR_OK) return st;
  Plan plan;
  st = make_plan(grids, n_grids, p, workspace != nullptr, plan);
  if (st != MPR_OK) return st;
  if (!workspace) {
    *ws_bytes = plan.bytes;
    return MPR_OK;
  }
  if (!ctx) return fail(nullptr, MPR_E_ARG, "ctx is NULL");
  if (*ws_bytes < plan.bytes)
    return fail(nullptr, MPR_E_WORKSPACE,
                "workspace of " + std::to_string(*ws_bytes) + " bytes, need " + std::to_string(plan.bytes));
  if (((uintptr_t)workspace) & 255) return fail(nullptr, MPR_E_WORKSPACE, "workspace must be 256-byte aligned");

  mpr_ctx *c = new mpr_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->p = *p;
  c->n_grids = n_grids;
  c->plan = plan;
  bind(c->v, plan.v, workspace);
  c->nsw_max = plan.nsw_max;
  c->nsw_run = plan.nsw_max;
  c->threads = p->dtype == MPR_FP64 ? 256 : 1024;
  if (const char *env = std::getenv("MPR_SWEEP_THREADS")) {
    const int t = std::atoi(env);
    if (t == 64 || t == 128 || t == 256 || t == 512 || t == 1024) c->threads = t;
  }
  c->threads1 = c->threads;
  c->threads2 = c->threads;
  // One workgroup per item by default; mpr_autotune times the persistent
  // single-sweep kernel against it (equal or slower on the workloads
  // measured so far), mpr_set_launch_shape selects it.
  c->persist1 = false;
  {
    const char *env = std::getenv("MPR_SPECULATE");
    c->spec_ok = p->dtype == MPR_FP32 && plan.nsw_max >= 2 && !(env && std::atoi(env) == 0);
  }
  // Speculative a-rule passes by default where the plan allows two sweeps
  // per pass; mpr_autotune keeps them only where they are faster.
  c->spec2 = c->spec_ok;
  c->sites_all_chains = plan.state_elems;
  auto bail = [&](mpr_status s) {
    g_thread_err = c->err;
    delete c;
    return s;
  };
  int dev = 0, lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return bail(hip_fail(c, e, "device query"));
  c->lds_limit = (size_t)lds;
  {
    int w, h;
    size_t need;
    lds_extent(c, c->nsw_max, true, w, h, need);
    if (need > c->lds_limit)
      return bail(fail(c, MPR_E_ARG, "tile and sweeps_per_pass need " + std::to_string(need) +
                                         " bytes of LDS per workgroup, the device allows " + std::to_string(lds)));
  }

  std::vector<const double *> zp(n_grids);
  std::vector<const uint8_t *> kp(n_grids);
  for (int g = 0; g < n_grids; ++g) {
    zp[g] = grids[g].z;
    kp[g] = grids[g].known;
  }
  c->known_h = kp;
#define TRY(call)                                      \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return bail(hip_fail(c, e_, #call)); \
  } while (0)
  TRY(hipMemcpyAsync(c->v.zp, zp.data(), sizeof(void *) * n_grids, hipMemcpyHostToDevice, c->stream));
  TRY(hipMemcpyAsync(c->v.kp, kp.data(), sizeof(void *) * n_grids, hipMemcpyHostToDevice, c->stream));
  TRY(hipMemcpyAsync(c->v.item_grid, c->plan.item_grid.data(), 4 * c->plan.item_grid.size(), hipMemcpyHostToDevice,
                     c->stream));
  const mpr_status ist = device_init(c);
  if (ist != MPR_OK) return bail(ist);
#undef TRY
  *ctx = c;
  return MPR_OK;
}

mpr_status mpr_sweep(mpr_ctx *ctx, int32_t n_sweeps, const double *T, uint32_t flags, double *trace) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (n_sweeps < 0) return fail(ctx, MPR_E_ARG, "n_sweeps must be >= 0");
  if (flags & ~(MPR_ADAPT | MPR_TRACE_E | MPR_NO_OR)) return fail(ctx, MPR_E_ARG, "unknown flag");
  mpr_status st = set_beta(ctx, T);
  if (st != MPR_OK) return st;
  return run_sweeps(ctx, n_sweeps, (flags & MPR_ADAPT) != 0, (flags & MPR_TRACE_E) != 0, trace, 0,
                    (flags & MPR_NO_OR) == 0);
}

// Slope of the least-squares line through (k, y[k * stride]), k = 0..n-1,
// from the differences of mirrored values: sum_{k < n/2} x_k (y_k -
// y_{n-1-k}) / sum x_k^2 with x centred, exactly 0 for a flat window.
static double ls_slope(const double *y, int n, int64_t stride) {
  const double c = 0.5 * (n - 1);
  double num = 0.0, den = 0.0;
  for (int k = 0; k < n / 2; ++k) num += (k - c) * (y[k * stride] - y[(n - 1 - k) * stride]);
  for (int k = 0; k < n; ++k) den += (k - c) * (k - c);
  return num / den;
}

mpr_status mpr_equilibrate(mpr_ctx *ctx, const double *T, int32_t n_f, int32_t n_fit, int32_t i_max, uint32_t flags,
                           double *trace, int32_t *n_done, int32_t *eq_at) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (flags & ~(MPR_ADAPT | MPR_NO_OR)) return fail(ctx, MPR_E_ARG, "unknown flag");
  if (n_f < 1 || n_fit < 2 || i_max < 0) return fail(ctx, MPR_E_ARG, "need n_f >= 1, n_fit >= 2, i_max >= 0");
  if (!trace) return fail(ctx, MPR_E_ARG, "trace is NULL");
  if (ctx->sweep_index + (int64_t)i_max + 1 >= 0xFFFFFFFFLL)
    return fail(ctx, MPR_E_STATE, "sweep counter would reach 2^32 - 1");
  mpr_status st = set_beta(ctx, T);
  if (st != MPR_OK) return st;
  st = close_pending(ctx);
  if (st != MPR_OK) return st;
  const int64_t C = ctx->plan.total_chains;
  const bool adapt = (flags & MPR_ADAPT) != 0, or_step = (flags & MPR_NO_OR) == 0;
  if (adapt) HIP_TRY(ctx, launch_fill_f64(win_buf(ctx, ctx->pass_no), C, 0.0, ctx->stream));
  std::vector<int32_t> at((size_t)C, -1);
  std::vector<double> rows((size_t)n_fit * C * 2);
  int64_t left = C;
  int32_t i = 0;  // sweeps run by this call
  while (i <= i_max && left > 0) {
    // the next check follows sweep chk: chk >= n_fit and a multiple of n_f
    int32_t chk = std::max(i, n_fit);
    chk = (chk + n_f - 1) / n_f * n_f;
    const int32_t last = std::min(chk, i_max);
    st = run_sweeps(ctx, last - i + 1, adapt, true, trace + (size_t)i * C * 2, 0, or_step);
    if (st != MPR_OK) return st;
    i = last + 1;
    if (last != chk) break;  // i_max reached before the check
    HIP_TRY(ctx, hipMemcpyAsync(rows.data(), trace + (size_t)(chk + 1 - n_fit) * C * 2, rows.size() * sizeof(double),
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t c = 0; c < C; ++c)
      if (at[c] < 0 && ls_slope(rows.data() + c * 2 + 1, n_fit, C * 2) >= 0.0) {
        at[c] = chk + 1;
        --left;
      }
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (n_done) *n_done = i;
  if (eq_at) std::copy(at.begin(), at.end(), eq_at);
  return MPR_OK;
}

mpr_status mpr_specific_energy(mpr_ctx *ctx, int32_t what, double *e_out, int64_t *npairs_out) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (what != MPR_SAMPLE_PAIRS && what != MPR_STATE) return fail(ctx, MPR_E_ARG, "unknown selector");
  if (!e_out) return fail(ctx, MPR_E_ARG, "e_out is NULL");
  std::vector<double> out;
  mpr_status st = reduce_energy(ctx, what, out);
  if (st != MPR_OK) return st;
  mpr_status ret = MPR_OK;
  if (what == MPR_SAMPLE_PAIRS) {
    for (int g = 0; g < ctx->n_grids; ++g) {
      const double s = out[g * 2], n = out[g * 2 + 1];
      if (npairs_out) npairs_out[g] = (int64_t)n;
      if (n > 0) {
        e_out[g] = s / n - 1.0;
      } else {
        e_out[g] = NAN;
        ret = fail(ctx, MPR_E_NOPAIRS, "grid " + std::to_string(g) + " has no sample-sample neighbour pair");
      }
    }
  } else {
    for (const GridDesc &d : ctx->plan.gd)
      for (int k = 0; k < d.chains; ++k) {
        const int u = d.chain_base + k;
        e_out[u] = out[u * 2] / (double)d.n_pairs - 1.0;
        if (npairs_out) npairs_out[u] = d.n_pairs;
      }
  }
  return ret;
}

mpr_status mpr_match_T(const double *e_s, int32_t n, const double *tab_T, const double *tab_e, int32_t n_tab,
                       double *T_out, mpr_status *item_status) {
  g_thread_err.clear();
  if (n < 0 || (n > 0 && (!e_s || !T_out))) return fail(nullptr, MPR_E_ARG, "bad e_s / T_out");
  if (n_tab < 2 || !tab_T || !tab_e) return fail(nullptr, MPR_E_ARG, "need a table of at least 2 points");
  for (int k = 0; k < n_tab; ++k) {
    if (!(tab_T[k] > 0.0) || !std::isfinite(tab_T[k]) || (k && !(tab_T[k] > tab_T[k - 1])))
      return fail(nullptr, MPR_E_ARG, "tab_T must be finite, positive and strictly increasing");
    if (!(tab_e[k] > -1.0) || !std::isfinite(tab_e[k]) || (k && !(tab_e[k] >= tab_e[k - 1])))
      return fail(nullptr, MPR_E_ARG, "tab_e must be finite, > -1 and non-decreasing");
  }
  std::vector<double> lx(n_tab), ly(n_tab);
  for (int k = 0; k < n_tab; ++k) {
    lx[k] = std::log(tab_T[k]);
    ly[k] = std::log1p(tab_e[k]);
  }
  Pchip pc;
  pc.build(lx, ly);
  mpr_status ret = MPR_OK;
  for (int i = 0; i < n; ++i) {
    const double e = e_s[i];
    mpr_status s = MPR_OK;
    double T;
    if (std::isnan(e)) {
      T = NAN;
      s = MPR_E_ARG;
    } else if (e <= tab_e[0]) {
      T = tab_T[0];
      if (e < tab_e[0]) s = MPR_E_RANGE;
    } else if (e >= tab_e[n_tab - 1]) {
      T = tab_T[n_tab - 1];
      if (e > tab_e[n_tab - 1]) s = MPR_E_RANGE;
    } else {
      // last node with tab_e <= e; the root lies in [x_j, x_{j+1})
      const int j = (int)(std::upper_bound(tab_e, tab_e + n_tab, e) - tab_e) - 1;
      if (tab_e[j] == e) {
        T = tab_T[j];
      } else {
        const double target = std::log1p(e);
        double lo = lx[j], hi = lx[j + 1];
        for (int it = 0; it < 400; ++it) {
          const double mid = 0.5 * (lo + hi);
          if (!(mid > lo && mid < hi)) break;
          if (pc.eval(j, mid) < target) lo = mid;
          else hi = mid;
        }
        const double flo = std::fabs(pc.eval(j, lo) - target), fhi = std::fabs(pc.eval(j, hi) - target);
        T = std::exp(flo <= fhi ? lo : hi);
      }
    }
    if (item_status) item_status[i] = s;
    if (s == MPR_E_ARG) ret = fail(nullptr, MPR_E_ARG, "NaN e_s");
    else if (s == MPR_E_RANGE && ret == MPR_OK) ret = fail(nullptr, MPR_E_RANGE, "e_s outside the table; T clamped");
    T_out[i] = T;
  }
  return ret;
}

// The device work of a fill up to its last sampling pass (Algorithm 2,
// steps 4-5): no host synchronisation, so a stream capture can record it.
// The a and acceptance sums after equilibration go to the report scratch.
static mpr_status fill_sweeps(mpr_ctx *ctx, int32_t n_eq, int32_t n_samp, int32_t stride) {
  const int64_t C = ctx->plan.total_chains;
  HIP_TRY(ctx, launch_fill_f64(ctx->v.accsum, C, 0.0, ctx->stream));
  HIP_TRY(ctx, launch_fill_f64(win_buf(ctx, ctx->pass_no), C, 0.0, ctx->stream));
  mpr_status st = run_sweeps(ctx, n_eq, true, false, nullptr, 0);
  if (st != MPR_OK) return st;
  HIP_TRY(ctx, launch_copy_f64(ctx->v.rep, a_buf(ctx, ctx->pass_no), C, ctx->stream));
  HIP_TRY(ctx, launch_copy_f64(ctx->v.rep + C, ctx->v.accsum, C, ctx->stream));
  if (!ctx->p.a_sample_keep) HIP_TRY(ctx, launch_fill_f64(a_buf(ctx, ctx->pass_no), C, 1.0, ctx->stream));
  HIP_TRY(ctx, launch_fill_f64(ctx->v.accsum, C, 0.0, ctx->stream));
  return run_sweeps(ctx, n_samp, false, false, nullptr, stride);
}

// fill_sweeps through the context's graph: replayed when the host state and
// arguments match those it was captured for, captured afresh otherwise.
// Clears use fill kernels, never memset nodes.
static mpr_status fill_sweeps_graph(mpr_ctx *ctx, int32_t n_eq, int32_t n_samp, int32_t stride) {
  const mpr_ctx::GraphState key{ctx->sweep_index, ctx->pass_no, ctx->cur, ctx->nsw_run, ctx->threads,
                                ctx->threads1,    ctx->threads2, n_eq,         n_samp,    stride,       ctx->p.a_sample_keep != 0,
                                ctx->persist1,    ctx->spec2};
  if (!ctx->graph_exec || !(key == ctx->g_key)) {
    ctx->drop_graph();
    {  // the occupancy query of persistent single-sweep passes, outside the capture
      int w, h;
      size_t lds;
      lds_extent(ctx, 1, false, w, h, lds);
      (void)resident_blocks1(ctx, ctx->threads1, lds);
    }
    if (!ctx->cap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const hipStream_t user = ctx->stream;
    const int64_t sweep0 = ctx->sweep_index, pass0 = ctx->pass_no;
    const int cur0 = ctx->cur;
    ctx->stream = ctx->cap_stream;
    ctx->capturing = true;
    ctx->g_launches = ctx->g_site_sweeps = 0;
    hipGraph_t g = nullptr;
    mpr_status st = MPR_OK;
    hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      st = fill_sweeps(ctx, n_eq, n_samp, stride);
      e = hipStreamEndCapture(ctx->stream, &g);
    }
    ctx->capturing = false;
    ctx->stream = user;
    const mpr_ctx::GraphState post{ctx->sweep_index, ctx->pass_no, ctx->cur, ctx->nsw_run, ctx->threads,
                                   ctx->threads1,    ctx->threads2, n_eq,         n_samp,    stride,       key.keep_a,
                                   ctx->persist1,    ctx->spec2};
    // nothing has run yet: the host state goes back until the graph launches
    ctx->sweep_index = sweep0;
    ctx->pass_no = pass0;
    ctx->cur = cur0;
    ctx->pending = PassEnd{};
    if (st == MPR_OK && e != hipSuccess) st = hip_fail(ctx, e, "graph capture");
    if (st == MPR_OK) {
      e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) st = hip_fail(ctx, e, "hipGraphInstantiate");
    }
    if (st != MPR_OK) {
      if (g) (void)hipGraphDestroy(g);
      ctx->graph_exec = nullptr;
      return st;
    }
    ctx->graph = g;
    ctx->g_key = key;
    ctx->g_post = post;
  }
  const bool timed = ctx->timing;
  if (timed) {
    if (ctx->ev_used + 2 > ctx->ev.size()) {
      if (ctx->ev.size() < 64) {
        for (int i = 0; i < 2; ++i) {
          hipEvent_t ev;
          HIP_TRY(ctx, hipEventCreate(&ev));
          ctx->ev.push_back(ev);
        }
      } else {
        const mpr_status st = drain_timing(ctx);
        if (st != MPR_OK) return st;
      }
    }
    HIP_TRY(ctx, hipEventRecord(ctx->ev[ctx->ev_used], ctx->stream));
  }
  HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
  if (timed) {
    HIP_TRY(ctx, hipEventRecord(ctx->ev[ctx->ev_used + 1], ctx->stream));
    ctx->ev_used += 2;
    ctx->t_launches += ctx->g_launches;
    ctx->t_site_sweeps += ctx->g_site_sweeps;
  }
  ctx->sweep_index = ctx->g_post.sweep_index;
  ctx->pass_no = ctx->g_post.pass_no;
  ctx->cur = ctx->g_post.cur;
  ctx->pending = PassEnd{};
  return MPR_OK;
}

mpr_status mpr_fill(mpr_ctx *ctx, const double *T, int32_t n_eq, int32_t n_samp, int32_t stride, double *zhat,
                    double *zstd, mpr_fill_report *rep) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (n_eq < 0 || n_samp < 1 || stride < 1 || n_samp / stride < 1)
    return fail(ctx, MPR_E_ARG, "need n_eq >= 0, n_samp >= 1, 1 <= stride <= n_samp");
  if (!zhat) return fail(ctx, MPR_E_ARG, "zhat is NULL");
  for (int g = 0; g < ctx->n_grids; ++g)
    if (std::isnan(ctx->plan.gd[g].zmin))
      return fail(ctx, MPR_E_DEGENERATE, "grid " + std::to_string(g) + " has no samples to fill from");
  if (ctx->sweep_index + (int64_t)n_eq + n_samp >= 0xFFFFFFFFLL)
    return fail(ctx, MPR_E_STATE, "sweep counter would reach 2^32 - 1");
  mpr_status st = set_beta(ctx, T);
  if (st != MPR_OK) return st;
  st = close_pending(ctx);
  if (st != MPR_OK) return st;
  st = ctx->graph_on ? fill_sweeps_graph(ctx, n_eq, n_samp, stride) : fill_sweeps(ctx, n_eq, n_samp, stride);
  if (st != MPR_OK) return st;
  const int32_t records = n_samp / stride;
  if (ctx->p.dtype == MPR_FP64) {
    HIP_TRY(ctx, launch_finalize<double>(ctx->v.gd, ctx->n_grids, ctx->plan.n_sblocks, ctx->v.zp,
                                         (const double *)ctx->v.st[ctx->cur], (const double *)ctx->v.acc_ref,
                                         (const double *)ctx->v.acc_s1, (const double *)ctx->v.acc_s2, records, zhat,
                                         zstd, ctx->stream));
  } else {
    HIP_TRY(ctx, launch_finalize<float>(ctx->v.gd, ctx->n_grids, ctx->plan.n_sblocks, ctx->v.zp,
                                        (const float *)ctx->v.st[ctx->cur], (const float *)ctx->v.acc_ref,
                                        (const float *)ctx->v.acc_s1, (const float *)ctx->v.acc_s2, records, zhat,
                                        zstd, ctx->stream));
  }
  if (rep) {
    rep->records = records;
    if (rep->a_eq || rep->acc_eq || rep->acc_samp) {
      const int64_t C = ctx->plan.total_chains;
      std::vector<double> hv((size_t)C * 3);
      HIP_TRY(ctx, hipMemcpyAsync(hv.data(), ctx->v.rep, 16 * C, hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(ctx, hipMemcpyAsync(hv.data() + 2 * C, ctx->v.accsum, 8 * C, hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      for (int64_t k = 0; k < C; ++k) {
        if (rep->a_eq) rep->a_eq[k] = hv[k];
        if (rep->acc_eq) rep->acc_eq[k] = n_eq ? hv[C + k] / n_eq : NAN;
        if (rep->acc_samp) rep->acc_samp[k] = hv[2 * C + k] / n_samp;
      }
    }
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MPR_OK;
}

mpr_status mpr_validation_measures(mpr_ctx *ctx, int32_t grid, const double *z_true, const double *zhat,
                                   double *out) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (grid < 0 || grid >= ctx->n_grids) return fail(ctx, MPR_E_ARG, "grid index out of range");
  if (!z_true || !zhat || !out) return fail(ctx, MPR_E_ARG, "z_true, zhat and out are required");
  const GridDesc &d = ctx->plan.gd[grid];
  if (d.n_gap == 0) return fail(ctx, MPR_E_DEGENERATE, "grid " + std::to_string(grid) + " has no prediction sites");
  const double shift = std::isnan(d.zmin) ? 0.0 : d.zmin;
  HIP_TRY(ctx, launch_measures(z_true, zhat, ctx->known_h[grid], (int64_t)d.nx * d.ny, shift, ctx->v.part,
                               ctx->v.out, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(out, ctx->v.out, 8 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (out[5] == 0.0)
    return fail(ctx, MPR_E_DEGENERATE, "grid " + std::to_string(grid) + ": no prediction site with a finite z_true");
  return MPR_OK;
}

mpr_status mpr_validation_measures_static(const double *z_true, const double *zhat, const uint8_t *known,
                                          int64_t n_sites, double shift, double *out, void *hip_stream) {
  g_thread_err.clear();
  if (!z_true || !zhat || !known || !out) return fail(nullptr, MPR_E_ARG, "z_true, zhat, known and out are required");
  if (n_sites < 1) return fail(nullptr, MPR_E_ARG, "n_sites must be >= 1");
  if (n_sites > kStaticMaxSites)
    return fail(nullptr, MPR_E_ARG, "n_sites = " + std::to_string(n_sites) + " exceeds the static scratch, which holds " +
                                        std::to_string(kStaticMaxSites) + " sites");
  if (!std::isfinite(shift)) return fail(nullptr, MPR_E_ARG, "shift must be finite");
  double *scr = nullptr;
  const mpr_status st = static_scratch(&scr);
  if (st != MPR_OK) return st;
  const hipError_t e = launch_measures(z_true, zhat, known, n_sites, shift, scr, out, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "launch_measures");
  return MPR_OK;
}

mpr_status mpr_set_grid_q(mpr_ctx *ctx, const double *q) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (!q) return fail(ctx, MPR_E_ARG, "q is NULL");
  if (ctx->p.model != MPR_MODEL_MPR) return fail(ctx, MPR_E_STATE, "q has no role in the GMRF interaction");
  if (ctx->p.q == 1.0) return fail(ctx, MPR_E_STATE, "the context was created with q = 1 (test mode)");
  for (int g = 0; g < ctx->n_grids; ++g)
    if (!(q[g] > 0.0 && q[g] <= 0.5)) return fail(ctx, MPR_E_ARG, "grid " + std::to_string(g) + ": q must be in (0, 0.5]");
  const mpr_status st = close_pending(ctx);
  if (st != MPR_OK) return st;
  for (int g = 0; g < ctx->n_grids; ++g) {
    ctx->plan.gd[g].q = q[g];
    ctx->plan.gd[g].inv_q = 1.0 / q[g];
  }
  HIP_TRY(ctx, hipMemcpyAsync(ctx->v.gd, ctx->plan.gd.data(), sizeof(GridDesc) * ctx->n_grids,
                              hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MPR_OK;
}

mpr_status mpr_cv_select_q(const mpr_grid *grid, const mpr_params *p, const uint8_t *fold, int32_t n_folds,
                           const double *q, int32_t n_q, const double *const *tab_T, const double *const *tab_e,
                           const int32_t *n_tab, int32_t n_eq, int32_t n_samp, int32_t stride, void *workspace,
                           size_t *ws_bytes, void *hip_stream, double *score, int32_t *best) {
  g_thread_err.clear();
  if (!grid || !p || !ws_bytes) return fail(nullptr, MPR_E_ARG, "grid, p and ws_bytes are required");
  if (n_folds < 2 || n_folds > 254) return fail(nullptr, MPR_E_ARG, "n_folds must be in [2, 254]");
  if (n_q < 1 || !q) return fail(nullptr, MPR_E_ARG, "need at least one candidate q");
  for (int i = 0; i < n_q; ++i)
    if (!(q[i] > 0.0 && q[i] <= 0.5)) return fail(nullptr, MPR_E_ARG, "candidate q must be in (0, 0.5]");
  if (p->model != MPR_MODEL_MPR) return fail(nullptr, MPR_E_ARG, "q selection needs the MPR interaction");
  if (n_eq < 0 || n_samp < 1 || stride < 1 || n_samp / stride < 1)
    return fail(nullptr, MPR_E_ARG, "need n_eq >= 0 and n_samp / stride >= 1");
  const int nb = n_q * n_folds;
  if ((int64_t)nb * grid->chains > 0x7fffffff) return fail(nullptr, MPR_E_SHAPE, "too many fits");
  mpr_params pq = *p;
  pq.q = q[0];
  // One batch of n_q * n_folds copies of the grid: fit (i, k) = grid i * n_folds + k.
  std::vector<mpr_grid> batch((size_t)nb, *grid);
  size_t ctx_bytes = 0;
  mpr_status st = mpr_init_field(nullptr, batch.data(), nb, &pq, nullptr, &ctx_bytes, nullptr);
  if (st != MPR_OK) return st;
  const int64_t n = (int64_t)grid->nx * grid->ny;
  const size_t off_mask = align_up(ctx_bytes, 256);
  const size_t off_zt = align_up(off_mask + (size_t)n_folds * n, 256);
  const size_t off_zh = align_up(off_zt + sizeof(double) * n_folds * n, 256);
  const size_t total = align_up(off_zh + sizeof(double) * nb * n, 256);
  if (!workspace) {
    *ws_bytes = total;
    return MPR_OK;
  }
  if (*ws_bytes < total)
    return fail(nullptr, MPR_E_WORKSPACE, "workspace of " + std::to_string(*ws_bytes) + " bytes, need " +
                                              std::to_string(total));
  if (((uintptr_t)workspace) & 255) return fail(nullptr, MPR_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (!fold || !grid->z || !grid->known) return fail(nullptr, MPR_E_ARG, "z, known and fold must be device pointers");
  if (!tab_T || !tab_e || !n_tab) return fail(nullptr, MPR_E_ARG, "tables are required");
  for (int i = 0; i < n_q; ++i)
    if (!tab_T[i] || !tab_e[i] || n_tab[i] < 2) return fail(nullptr, MPR_E_ARG, "candidate table missing or short");
  if (!best) return fail(nullptr, MPR_E_ARG, "best is NULL");
  unsigned char *base = (unsigned char *)workspace;
  uint8_t *masks = base + off_mask;
  double *zt = (double *)(base + off_zt), *zh = (double *)(base + off_zh);
  const hipStream_t s = (hipStream_t)hip_stream;
  hipError_t he = launch_cv_prepare(grid->z, grid->known, fold, n_folds, n, masks, zt, s);
  if (he != hipSuccess) return hip_fail(nullptr, he, "cross-validation fold masks");
  for (int g = 0; g < nb; ++g) batch[g].known = masks + (int64_t)(g % n_folds) * n;

  mpr_ctx *c = nullptr;
  st = mpr_init_field(&c, batch.data(), nb, &pq, workspace, &ctx_bytes, hip_stream);
  if (st != MPR_OK) return st;
  auto done = [&](mpr_status r) {
    if (r != MPR_OK) g_thread_err = c->err;
    mpr_destroy(c);
    return r;
  };
  std::vector<double> qg((size_t)nb), e((size_t)nb), T((size_t)nb);
  for (int g = 0; g < nb; ++g) qg[g] = q[g / n_folds];
  if ((st = mpr_set_grid_q(c, qg.data())) != MPR_OK) return done(st);
  if ((st = mpr_specific_energy(c, MPR_SAMPLE_PAIRS, e.data(), nullptr)) != MPR_OK) return done(st);
  for (int g = 0; g < nb; ++g) {
    const int i = g / n_folds;
    mpr_status item = MPR_OK;
    st = mpr_match_T(&e[g], 1, tab_T[i], tab_e[i], n_tab[i], &T[g], &item);
    if (st != MPR_OK && st != MPR_E_RANGE) {  // a clamped T-hat is used as it is, as in a fill
      c->err = "fit " + std::to_string(g) + ": " + g_thread_err;
      return done(st);
    }
  }
  if ((st = mpr_fill(c, T.data(), n_eq, n_samp, stride, zh, nullptr, nullptr)) != MPR_OK) return done(st);
  std::vector<double> aae((size_t)n_q, 0.0), sq((size_t)n_q, 0.0), cnt((size_t)n_q, 0.0), tm((size_t)n_q, 0.0);
  for (int g = 0; g < nb; ++g) {
    const int i = g / n_folds, k = g % n_folds;
    double m[8];
    if ((st = mpr_validation_measures(c, g, zt + (int64_t)k * n, zh + (int64_t)g * n, m)) != MPR_OK) return done(st);
    aae[i] += m[0] * m[5];         // sum |eps| of the fold
    sq[i] += m[3] * m[3] * m[5];   // sum eps^2
    cnt[i] += m[5];
    tm[i] += T[g] / n_folds;
  }
  int b = 0;
  for (int i = 0; i < n_q; ++i) {
    aae[i] /= cnt[i];
    sq[i] = std::sqrt(sq[i] / cnt[i]);
    if (score) {
      score[i * 3] = aae[i];
      score[i * 3 + 1] = sq[i];
      score[i * 3 + 2] = tm[i];
    }
    // least pooled AAE; among equal ones the larger q
    if (aae[i] < aae[b] || (aae[i] == aae[b] && q[i] > q[b])) b = i;
  }
  *best = b;
  return done(MPR_OK);
}

mpr_status mpr_reinit(mpr_ctx *ctx) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  const mpr_status st = close_pending(ctx);
  if (st != MPR_OK) return st;
  return device_init(ctx);
}

mpr_status mpr_set_graph(mpr_ctx *ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  ctx->graph_on = enable != 0;
  if (!ctx->graph_on) ctx->drop_graph();
  return MPR_OK;
}

static mpr_status chain_view(mpr_ctx *ctx, int32_t grid, int32_t chain, int64_t &off, int64_t &n) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (grid < 0 || grid >= ctx->n_grids) return fail(ctx, MPR_E_ARG, "grid index out of range");
  const GridDesc &d = ctx->plan.gd[grid];
  if (chain < 0 || chain >= d.chains) return fail(ctx, MPR_E_ARG, "chain index out of range");
  n = (int64_t)d.nx * d.ny;
  off = d.state_off + (int64_t)chain * n;
  return MPR_OK;
}

mpr_status mpr_get_phi(mpr_ctx *ctx, int32_t grid, int32_t chain, double *phi) {
  int64_t off, n;
  mpr_status st = chain_view(ctx, grid, chain, off, n);
  if (st != MPR_OK) return st;
  if (!phi) return fail(ctx, MPR_E_ARG, "phi is NULL");
  if (ctx->p.dtype == MPR_FP64) {
    HIP_TRY(ctx, launch_get_phi<double>((const double *)ctx->v.st[ctx->cur] + off, n, phi, ctx->stream));
  } else {
    HIP_TRY(ctx, launch_get_phi<float>((const float *)ctx->v.st[ctx->cur] + off, n, phi, ctx->stream));
  }
  return MPR_OK;
}

mpr_status mpr_set_phi(mpr_ctx *ctx, int32_t grid, int32_t chain, const double *phi) {
  int64_t off, n;
  mpr_status st = chain_view(ctx, grid, chain, off, n);
  if (st != MPR_OK) return st;
  if (!phi) return fail(ctx, MPR_E_ARG, "phi is NULL");
  if (ctx->p.dtype == MPR_FP64) {
    HIP_TRY(ctx, launch_set_phi<double>((double *)ctx->v.st[ctx->cur] + off, (double *)ctx->v.st[ctx->cur ^ 1] + off,
                                        n, phi, ctx->stream));
  } else {
    HIP_TRY(ctx, launch_set_phi<float>((float *)ctx->v.st[ctx->cur] + off, (float *)ctx->v.st[ctx->cur ^ 1] + off, n,
                                       phi, ctx->stream));
  }
  return MPR_OK;
}

// FNV-1a over the grid shapes and gap counts of a batch.
static uint64_t shape_hash(const std::vector<GridDesc> &gd) {
  uint64_t h = 1469598103934665603ull;
  for (const GridDesc &d : gd)
    for (int64_t v : {(int64_t)d.nx, (int64_t)d.ny, (int64_t)d.chains, d.n_gap}) {
      h ^= (uint64_t)v;
      h *= 1099511628211ull;
    }
  return h;
}

// Key of a batch shape for the autotuners' process-wide caches: what
// selects the kernel (precision, interaction, boundary) and the grids.
static std::string batch_key(const mpr_params &p, const std::vector<GridDesc> &gd) {
  return std::to_string(p.dtype) + ":" + std::to_string(p.model) + ":" + std::to_string(p.boundary) + ":" +
         std::to_string(p.q == 1.0) + ":" + std::to_string(gd.size()) + ":" + std::to_string(shape_hash(gd));
}

static std::string tune_key(const mpr_ctx *c) {
  return batch_key(c->p, c->plan.gd) + ":" + std::to_string(c->plan.tile_x) + "x" + std::to_string(c->plan.tile_y) +
         ":" + std::to_string(c->nsw_max);
}

static std::mutex g_tune_mu;
struct TuneChoice {
  int nsw, threads, threads1;  // sweeps per pass and workgroup size; workgroup size of single-sweep passes
  double ms, ms1;              // their time per sweep; per sweep at one sweep per pass
  bool persist1;               // single-sweep passes on persistent workgroups
  bool spec2;                  // a-rule sweeps in speculative two-sweep passes
  int threads2;                // their workgroup size
  double ms_arule;             // time per a-rule sweep (adapt_every == 1) with that choice
};
static std::map<std::string, TuneChoice> g_tune_cache;

// Time trial passes over (workgroup size x sweeps per pass) on the
// context's grids and restore the chains afterwards.
static mpr_status time_launch_shapes(mpr_ctx *ctx, const double *T, int32_t trial_sweeps, TuneChoice &out) {
  mpr_status st = set_beta(ctx, T);
  if (st != MPR_OK) return st;
  const int64_t C = ctx->plan.total_chains;
  // Save the state, the sweep counter, the pass number and a; the fill
  // accumulator `ref` serves as the copy of the angles.
  const size_t bytes = ctx->plan.elem * (size_t)ctx->plan.state_elems;
  std::vector<double> a_save(C);
  HIP_TRY(ctx, hipMemcpyAsync(ctx->v.acc_ref, ctx->v.st[ctx->cur], bytes, hipMemcpyDeviceToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(a_save.data(), a_buf(ctx, ctx->pass_no), 8 * C, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const int cur0 = ctx->cur;
  const int64_t sweep0 = ctx->sweep_index, pass0 = ctx->pass_no;
  const bool timing0 = ctx->timing;
  const int nsw0 = ctx->nsw_run, thr0 = ctx->threads, thr10 = ctx->threads1;
  const bool persist0 = ctx->persist1;
  ctx->timing = false;

  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  double best = 1e300, best1 = 1e300;
  std::map<int, double> two;  // per sweep in two-sweep passes, by workgroup size
  int best_nsw = ctx->nsw_run, best_thr = ctx->threads, best_thr1 = ctx->threads1;
  bool best_p1 = false;
  const int nsws[] = {1, 2, 3, 4, 6, 8, 12, 16};
  // Workgroups of 64 and 128 threads are tried only where every tile is
  // small (grids below 32 x 32 sites): there many more of them share a CU.
  int64_t max_tile_sites = 0;
  for (const GridDesc &d : ctx->plan.gd)
    max_tile_sites = std::max<int64_t>(max_tile_sites, (int64_t)std::min(d.nx, ctx->plan.tile_x) *
                                                           std::min(d.ny, ctx->plan.tile_y));
  for (int thr : {64, 128, 256, 512, 1024}) {
    if (thr < 256 && max_tile_sites > 1024) continue;
    const bool ok = (ctx->p.dtype == MPR_FP64 ? sweep_max_threads<double>(thr) : sweep_max_threads<float>(thr)) >= thr;
    if (!ok) continue;
    for (int nsw : nsws) {
      if (nsw > ctx->nsw_max) break;
      int w, h;
      size_t lds;
      lds_extent(ctx, nsw, false, w, h, lds);
      if (lds > ctx->lds_limit) break;
      ctx->threads = thr;
      ctx->threads1 = thr;
      ctx->nsw_run = nsw;
      // Single-sweep passes (the a-rule's) are timed on both kernels: one
      // workgroup per item, and persistent workgroups where they run.
      const bool p1_runs = nsw == 1 && persistent_fit(ctx, thr, w, h, false, lds) > 0;
      for (int pv = 0; pv < (p1_runs ? 2 : 1) && st == MPR_OK; ++pv) {
        ctx->persist1 = pv == 1;
        int64_t n = ((trial_sweeps + nsw - 1) / nsw) * nsw;
        st = run_sweeps(ctx, nsw, false, false, nullptr, 0);  // warm-up pass
        // Timed runs of at least ~2 ms each (a short run is lengthened after
        // the first), the fastest kept: close candidates are otherwise
        // decided by one-off delays.
        float ms = 1e30f;
        bool lengthened = false;
        for (int rep = 0; rep < 3 && st == MPR_OK; ++rep) {
          if (rep == 1 && ms < 2.0f) {
            const int64_t want = (int64_t)std::ceil(n * 2.0 / std::max(ms, 0.01f));
            n = ((std::min<int64_t>(want, 64 * n) + nsw - 1) / nsw) * nsw;
            ms = 1e30f;  // compare runs of the new length only
            lengthened = true;
          }
          if (rep == 2 && !lengthened) break;  // two long runs suffice
          HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
          st = run_sweeps(ctx, n, false, false, nullptr, 0);
          HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
          if (st != MPR_OK) break;
          HIP_TRY(ctx, hipEventSynchronize(e1));
          float m = 0.f;
          HIP_TRY(ctx, hipEventElapsedTime(&m, e0, e1));
          ms = std::min(ms, m);
        }
        if (st != MPR_OK) break;
        const double per_sweep = ms / (double)n;
        if (pv == 0 && nsw == 2) two[thr] = per_sweep;
        if (pv == 0 && per_sweep < best) {  // multi-sweep passes, and passes that record
          best = per_sweep;
          best_nsw = nsw;
          best_thr = thr;
        }
        if (nsw == 1 && per_sweep < best1) {  // the a-rule runs one sweep per pass
          best1 = per_sweep;
          best_thr1 = thr;
          best_p1 = pv == 1;
        }
      }
      if (st != MPR_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // Restore everything the trial passes changed.
  ctx->cur = cur0;
  HIP_TRY(ctx, hipMemcpyAsync(ctx->v.st[ctx->cur], ctx->v.acc_ref, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  ctx->sweep_index = sweep0;
  ctx->pass_no = pass0;
  ctx->pending.valid = 0;
  HIP_TRY(ctx, hipMemcpyAsync(a_buf(ctx, ctx->pass_no), a_save.data(), 8 * C, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, launch_zero_u32(ctx->v.counts, 3 * C * kMaxPass, ctx->stream));
  HIP_TRY(ctx, launch_fill_f64(ctx->v.energy, 3 * C * kMaxPass, 0.0, ctx->stream));
  HIP_TRY(ctx, launch_fill_f64(ctx->v.accsum, C, 0.0, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->timing = timing0;
  ctx->nsw_run = nsw0;
  ctx->threads = thr0;
  ctx->threads1 = thr10;
  ctx->persist1 = persist0;
  if (st != MPR_OK) return st;
  // Speculative a-rule passes: two sweeps at their own best workgroup size,
  // kept where that beats one sweep per pass, check and redo launch included.
  int thr2 = best_thr;
  double ms_spec = 1e300;
  for (const auto &kv : two)
    if (kv.second + kSpecOverheadMs / 2 < ms_spec) {
      ms_spec = kv.second + kSpecOverheadMs / 2;
      thr2 = kv.first;
    }
  const bool spec2 = ctx->spec_ok && ms_spec < best1;
  out = {best_nsw, best_thr, best_thr1, best, best1, best_p1, spec2, thr2, spec2 ? ms_spec : best1};
  return MPR_OK;
}

// The context's launch shape, from the cache or timed.
static mpr_status tuned_shape(mpr_ctx *ctx, const double *T, int32_t trial_sweeps, TuneChoice &ch) {
  const std::string key = tune_key(ctx);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      ch = it->second;
      return MPR_OK;
    }
  }
  const mpr_status st = time_launch_shapes(ctx, T, trial_sweeps, ch);
  if (st != MPR_OK) return st;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = ch;
  return MPR_OK;
}

mpr_status mpr_autotune(mpr_ctx *ctx, const double *T, int32_t trial_sweeps, int32_t *nsw_out, int32_t *threads_out,
                        int32_t *threads1_out, int32_t *persist1_out) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (trial_sweeps < 1) return fail(ctx, MPR_E_ARG, "trial_sweeps must be >= 1");
  TuneChoice ch{};
  const mpr_status st = tuned_shape(ctx, T, trial_sweeps, ch);
  if (st != MPR_OK) return st;
  ctx->nsw_run = ch.nsw;
  ctx->threads = ch.threads;
  ctx->threads1 = ch.threads1;
  ctx->persist1 = ch.persist1;
  ctx->spec2 = ch.spec2 && ctx->spec_ok;
  ctx->threads2 = ch.threads2;
  if (nsw_out) *nsw_out = ch.nsw;
  if (threads_out) *threads_out = ch.threads;
  if (threads1_out) *threads1_out = ch.threads1;
  if (persist1_out) *persist1_out = ch.persist1 ? 1 : 0;
  return MPR_OK;
}

mpr_status mpr_set_launch_shape(mpr_ctx *ctx, int32_t nsw, int32_t threads, int32_t threads1, int32_t persist1) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (nsw < 1 || nsw > ctx->nsw_max)
    return fail(ctx, MPR_E_ARG, "nsw must be in 1.." + std::to_string(ctx->nsw_max));
  for (int t : {threads, threads1}) {
    if (t != 64 && t != 128 && t != 256 && t != 512 && t != 1024)
      return fail(ctx, MPR_E_ARG, "workgroup sizes must be 64, 128, 256, 512 or 1024");
    const int mx = ctx->p.dtype == MPR_FP64 ? sweep_max_threads<double>(t) : sweep_max_threads<float>(t);
    if (mx < t) return fail(ctx, MPR_E_ARG, "the sweep kernel cannot run " + std::to_string(t) + " threads");
  }
  int w, h;
  size_t lds;
  lds_extent(ctx, nsw, true, w, h, lds);
  if (lds > ctx->lds_limit) return fail(ctx, MPR_E_ARG, "the pass needs more LDS than the device has");
  ctx->nsw_run = nsw;
  ctx->threads = threads;
  ctx->threads1 = threads1;
  ctx->persist1 = persist1 != 0;
  ctx->spec2 = ctx->spec_ok && nsw >= 2;  // a shape of multi-sweep passes also speculates
  ctx->threads2 = threads;
  return MPR_OK;
}

// Tile candidates of mpr_autotune_tile, the library default first so that
// a tie keeps it.  Tiles are even and row-major wide where they are not
// square: a workgroup stages whole tile rows.
static const int kTileCand32[][2] = {{64, 64}, {64, 56}, {64, 48}, {32, 32}, {64, 32}, {128, 32}, {128, 64}, {96, 96}};
static const int kTileCand64[][2] = {{32, 32}, {16, 16}, {32, 16}, {64, 32}, {64, 64}};

static constexpr double kTileMargin = 0.95;  // a tile must cost 5 % less than the default to replace it

struct TileChoice {
  int tile_x, tile_y, nsw;
};
static std::map<std::string, TileChoice> g_tile_cache;

mpr_status mpr_autotune_tile(const mpr_grid *grids, int32_t n_grids, const mpr_params *p, const double *T,
                             int32_t n_eq, int32_t n_samp, int32_t trial_sweeps, void *workspace, size_t *ws_bytes,
                             void *hip_stream, int32_t *tile_x, int32_t *tile_y, int32_t *sweeps_per_pass) {
  g_thread_err.clear();
  if (!ws_bytes) return fail(nullptr, MPR_E_ARG, "ws_bytes is NULL");
  mpr_status st = check_params(p);
  if (st != MPR_OK) return st;
  if (n_eq < 0 || n_samp < 0 || (int64_t)n_eq + n_samp < 1)
    return fail(nullptr, MPR_E_ARG, "need n_eq >= 0, n_samp >= 0 and n_eq + n_samp >= 1");
  if (trial_sweeps < 1) return fail(nullptr, MPR_E_ARG, "trial_sweeps must be >= 1");
  Plan pl0;  // validates the grids before the device is touched
  st = make_plan(grids, n_grids, p, workspace != nullptr, pl0);
  if (st != MPR_OK) return st;
  int dev = 0, lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "device query");
  // Each candidate with the most sweeps per pass its LDS holds, up to the
  // requested (or default) maximum.
  struct Cand {
    mpr_params p;
    size_t bytes;
  };
  std::vector<Cand> cands;
  const bool f64 = p->dtype == MPR_FP64;
  const int n_cand = f64 ? (int)(sizeof(kTileCand64) / sizeof(kTileCand64[0]))
                         : (int)(sizeof(kTileCand32) / sizeof(kTileCand32[0]));
  const int nsw_req = p->sweeps_per_pass ? p->sweeps_per_pass : (f64 ? 1 : 8);
  size_t need = 0;
  for (int i = 0; i < n_cand; ++i) {
    mpr_params pp = *p;
    pp.tile_x = f64 ? kTileCand64[i][0] : kTileCand32[i][0];
    pp.tile_y = f64 ? kTileCand64[i][1] : kTileCand32[i][1];
    for (int nsw = nsw_req; nsw >= 1; --nsw) {
      pp.sweeps_per_pass = nsw;
      Plan pl;
      st = make_plan(grids, n_grids, &pp, workspace != nullptr, pl);
      if (st != MPR_OK) return st;
      int w, h;
      size_t b;
      lds_extent(pl, nsw, true, w, h, b);
      if (b <= (size_t)lds) {
        cands.push_back({pp, pl.bytes});
        need = std::max(need, pl.bytes);
        break;
      }
      if (p->sweeps_per_pass) break;  // a requested depth is not lowered
    }
  }
  if (cands.empty()) return fail(nullptr, MPR_E_ARG, "no candidate tile fits the device's LDS at this sweeps_per_pass");
  if (!workspace) {
    *ws_bytes = need;
    return MPR_OK;
  }
  if (*ws_bytes < need)
    return fail(nullptr, MPR_E_WORKSPACE,
                "workspace of " + std::to_string(*ws_bytes) + " bytes, need " + std::to_string(need));
  if (((uintptr_t)workspace) & 255) return fail(nullptr, MPR_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (!T) return fail(nullptr, MPR_E_ARG, "T is NULL");

  // Each candidate is set up as a context in the workspace.  The cache key
  // holds the grids' gap counts, known once the first context exists.
  auto init_cand = [&](const Cand &cd, mpr_ctx *&c) {
    size_t have = *ws_bytes;
    return mpr_init_field(&c, grids, n_grids, &cd.p, workspace, &have, hip_stream);
  };
  mpr_ctx *c0 = nullptr;
  st = init_cand(cands[0], c0);
  if (st != MPR_OK) return st;
  const std::string key = batch_key(*p, c0->plan.gd) + ":" + std::to_string(p->sweeps_per_pass) + ":" +
                          std::to_string(n_eq) + ":" + std::to_string(n_samp);
  TileChoice best{cands[0].p.tile_x, cands[0].p.tile_y, cands[0].p.sweeps_per_pass};
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tile_cache.find(key);
    if (it != g_tile_cache.end()) {
      best = it->second;
      cached = true;
    }
  }
  if (cached) {
    mpr_destroy(c0);
  } else {
    // Fill time model: n_eq sweeps at one sweep per pass (the a-rule's
    // pace when it adapts after every sweep) and n_samp at the tuned pace,
    // each candidate's launch shape tuned (or taken from the cache).  With
    // a longer a-rule period the equilibration passes are costed at the
    // tuned pace too.
    double best_cost = 1e300, default_cost = 1e300;
    for (size_t i = 0; i < cands.size(); ++i) {
      mpr_ctx *c = c0;
      c0 = nullptr;
      if (i > 0) {
        st = init_cand(cands[i], c);
        if (st != MPR_OK) return st;
      }
      TuneChoice ch{};
      st = tuned_shape(c, T, trial_sweeps, ch);
      if (st != MPR_OK) {
        g_thread_err = c->err;
        mpr_destroy(c);
        return st;
      }
      mpr_destroy(c);
      const double cost = n_eq * (p->adapt_every == 1 ? ch.ms_arule : ch.ms) + n_samp * ch.ms;
      if (i == 0) default_cost = cost;
      if (cost < best_cost) {
        best_cost = cost;
        best = {cands[i].p.tile_x, cands[i].p.tile_y, cands[i].p.sweeps_per_pass};
      }
    }
    // Another tile replaces the default only when it is clearly faster:
    // candidates within a few per cent of each other differ by timing noise.
    if (best_cost > kTileMargin * default_cost)
      best = {cands[0].p.tile_x, cands[0].p.tile_y, cands[0].p.sweeps_per_pass};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tile_cache[key] = best;
  }
  e = hipStreamSynchronize((hipStream_t)hip_stream);  // the last context's set-up work
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipStreamSynchronize");
  if (tile_x) *tile_x = best.tile_x;
  if (tile_y) *tile_y = best.tile_y;
  if (sweeps_per_pass) *sweeps_per_pass = best.nsw;
  return MPR_OK;
}

mpr_status mpr_set_timing(mpr_ctx *ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  ctx->timing = enable != 0;
  return MPR_OK;
}

mpr_status mpr_get_timing(mpr_ctx *ctx, double *sweep_ms, int64_t *launches, int64_t *site_sweeps) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  const mpr_status st = drain_timing(ctx);
  if (st != MPR_OK) return st;
  if (sweep_ms) *sweep_ms = ctx->t_ms;
  if (launches) *launches = ctx->t_launches;
  if (site_sweeps) *site_sweeps = ctx->t_site_sweeps;
  ctx->t_ms = 0.0;
  ctx->t_launches = 0;
  ctx->t_site_sweeps = 0;
  return MPR_OK;
}

mpr_status mpr_get_chain_state(mpr_ctx *ctx, int64_t *sweep_index, double *a) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (sweep_index) *sweep_index = ctx->sweep_index;
  if (a) {
    HIP_TRY(ctx, hipMemcpyAsync(a, a_buf(ctx, ctx->pass_no), 8 * (size_t)ctx->plan.total_chains,
                                hipMemcpyDeviceToHost, ctx->stream));
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MPR_OK;
}

mpr_status mpr_set_chain_state(mpr_ctx *ctx, int64_t sweep_index, const double *a) {
  if (!ctx) return fail(nullptr, MPR_E_STATE, "ctx is NULL");
  if (sweep_index < 0 || sweep_index >= 0xFFFFFFFFLL) return fail(ctx, MPR_E_ARG, "sweep_index out of range");
  if (a) {
    for (int k = 0; k < ctx->plan.total_chains; ++k)
      if (!(a[k] >= 1.0) || !std::isfinite(a[k])) return fail(ctx, MPR_E_ARG, "every a must be finite and >= 1");
    HIP_TRY(ctx, hipMemcpyAsync(a_buf(ctx, ctx->pass_no), a, 8 * (size_t)ctx->plan.total_chains,
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  ctx->sweep_index = sweep_index;
  return MPR_OK;
}

}  // extern "C"
