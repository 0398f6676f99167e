// gfx950 kernels of the MPR hybrid Monte Carlo path.
//
// Method: Zukovic & Hristopulos, arXiv 1710.03038.  Eq. (2) maps data to
// angles, Eq. (3) is the MPR energy -sum cos(q (phi_i - phi_j)) over
// nearest-neighbour pairs with open boundaries, Eqs. (4)-(5) the sample and
// equilibrium specific energies, Eq. (6) the over-relaxation; Algorithm 1
// is the hybrid update (over-relaxation, then restricted Metropolis) and
// Algorithm 2 the driver.  The sweep runs the sites of one checkerboard
// colour at a time (Sec. 5.2).
//
// Layout: angles are stored per (grid, chain) in natural row-major order;
// the sign bit marks a frozen sample site (|v| is its angle).  A sweep
// workgroup stages its tile plus a halo of 2*nsw (+1) sites in LDS, split by
// colour so that the sites of one colour and the neighbours they read are
// contiguous, runs nsw sweeps there, and writes the tile interior to the
// other buffer of a ping-pong pair.  Sites of the halo are updated
// redundantly by neighbouring tiles with identical arithmetic and random
// numbers, so results do not depend on the tiling.  One Philox4x32-10 call
// per sweep serves a pair of same-colour sites (y, y + 2) of a column,
// y mod 4 in {0, 1}: counter (first site, sweep, chain, grid).
#include "internal.h"

#include <algorithm>
#include <cmath>

#include "fastmath.h"

namespace mpr {

// A launch counts its work-items in 32 bits per dimension.  Launches that
// would pass 2^32 - 1 get rows of 65536 workgroups; each kernel takes its
// linear workgroup index and skips those past its count.
static dim3 block_grid(int64_t n_blocks, int threads) {
  if (n_blocks * threads <= 0xFFFFFFFFLL) return dim3((unsigned)n_blocks);
  return dim3(65536u, (unsigned)((n_blocks + 65535) / 65536));
}
__device__ __forceinline__ int64_t block_index() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }
// Work item of this workgroup when items are dealt to the 8 XCDs in
// contiguous ranges: workgroup b runs on XCD b % 8, which takes items
// (b % 8) * per + b / 8 with per = ceil(n_items / 8), so the workgroups an
// XCD runs at one time sweep neighbouring tiles and share their halo rows
// and columns in its L2.  The launch has at least 8 * per workgroups;
// those past the last item get n_items.
__device__ __forceinline__ int64_t xcd_item(int64_t n_items) {
  const int64_t b = block_index(), per = (n_items + 7) >> 3, lb = b >> 3;
  return lb < per ? (b & 7) * per + lb : n_items;
}


// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon et al., SC'11): rounds multiply words 0 and 2 by
// 0xD2511F53 and 0xCD9E8D57 (32x32 -> 64 bit), swap and xor in the key; the
// key advances by 0x9E3779B9 / 0xBB67AE85 between rounds.
// The 32x32 -> 64-bit products use one v_mad_u64_u32 each (both halves at
// once); the compiler would otherwise split them into mul_lo + mul_hi.
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t b) {
  uint64_t r, carry;
  asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "v"(a), "v"(b));
  return r;
}

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = mul_wide(0xD2511F53u, c0), p1 = mul_wide(0xCD9E8D57u, c2);
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// ------------------------------------------------------------ precision
// FP32 uses the bounded-argument routines of fastmath.h; FP64 (the plain
// reference arm) uses the device library's correctly rounded functions.
template <typename P> struct Prec;
template <> struct Prec<float> {
  using V2 = float2;
  static constexpr float two_pi = 6.28318530717958647692f;  // rounds up: 6.2831855f
  static constexpr float below_two_pi = 6.2831850f;         // largest float < two_pi
  static constexpr float tiny_h2 = 1e-12f;
  static constexpr float inv_2pi2 = 0.0506605918211688857f;  // 1 / (2 pi^2)
  __device__ static float sin_(float x) { return fm::sin(x); }
  __device__ static float sin_dh_(float x) { return fm::sin_hw(x); }
  __device__ static void sincos_(float x, float *s, float *c) { fm::sincos(x, s, c); }
  __device__ static void sincos_0pi_(float x, float *s, float *c) { fm::sincos_0pi(x, s, c); }
  __device__ static float atan2_(float y, float x) { return fm::atan2(y, x); }
  __device__ static float exp_(float x) { return fm::exp(x); }
  __device__ static float sqrt_(float x) { return fm::sqrt(x); }
  __device__ static float floor_(float x) { return floorf(x); }
};
template <> struct Prec<double> {
  using V2 = double2;
  static constexpr double two_pi = 6.28318530717958647692;
  static constexpr double below_two_pi = 6.2831853071795853;  // nextafter(2*pi, 0)
  static constexpr double tiny_h2 = 1e-24;
  static constexpr double inv_2pi2 = 0.0506605918211688857;
  __device__ static double sin_(double x) { return ::sin(x); }
  __device__ static double sin_dh_(double x) { return ::sin(x); }
  __device__ static void sincos_(double x, double *s, double *c) { ::sincos(x, s, c); }
  __device__ static void sincos_0pi_(double x, double *s, double *c) { ::sincos(x, s, c); }
  __device__ static double atan2_(double y, double x) { return ::atan2(y, x); }
  __device__ static double exp_(double x) { return ::exp(x); }
  __device__ static double sqrt_(double x) { return ::sqrt(x); }
  __device__ static double floor_(double x) { return ::floor(x); }
};

// A 32-bit word to [0, 1 - 2^-24]: (w >> 8) * 2^-24, exact in either precision.
template <typename P> __device__ __forceinline__ P unit(uint32_t w) {
  return (P)(w >> 8) * (P)5.9604644775390625e-08;
}

// Proposal wrap for |shift| <= pi (Algorithm 1, step 3): into [0, 2*pi),
// with a rounding result of exactly 2*pi folded to 0.
template <typename P> __device__ __forceinline__ P wrap_step(P x) {
  const P tp = Prec<P>::two_pi;
  x = (x < P(0)) ? x + tp : ((x >= tp) ? x - tp : x);
  return (x >= tp) ? P(0) : x;
}
// General wrap (q = 1 over-relaxation): x - 2*pi*floor(x / 2*pi), folded.
template <typename P> __device__ __forceinline__ P wrap_any(P x) {
  const P tp = Prec<P>::two_pi;
  P y = x - tp * Prec<P>::floor_(x / tp);
  y = (y < P(0)) ? y + tp : y;
  return (y >= tp) ? P(0) : y;
}

// --------------------------------------------------------- block reductions
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Sum over the workgroup of NT threads; the result is valid in thread 0.
// Fixed order, so the result does not depend on scheduling.
template <int NT, typename T> __device__ __forceinline__ T block_sum(T v, T *scratch) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) scratch[w] = v;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) r += scratch[i];
  return r;
}

__device__ __forceinline__ int find_by(const GridDesc *g, int n, int64_t key, int64_t GridDesc::*field, int lo = 0,
                                       int hi = -1) {
  if (hi < 0) hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g[mid].*field <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Row r and column offset of flat index f over rows of npr entries, without
// an integer division (f < 2^22, so the float estimate is off by at most one).
__device__ __forceinline__ void split_index(int f, int npr, float inv, int &r, int &c) {
  r = (int)((float)f * inv);
  c = f - r * npr;
  if (c >= npr) {
    ++r;
    c -= npr;
  } else if (c < 0) {
    --r;
    c += npr;
  }
}

// End of a pending pass for one chain: turn the accepted counts into
// acceptance ratios and trace rows, and apply the a-rule of Algorithm 2,
// step 4.2: after sweep i, if the mean acceptance of the adapt_every-window
// ending there is below A_targ, then a = 1 + (i + 1)/k_a.  Every caller
// computes the same a from the same read-only inputs; only the caller with
// write = true stores a, the window, the trace and the acceptance sums.
template <typename P>
__device__ double apply_pass_end(const SweepArgs<P> &A, const GridDesc &G, int ch, bool write, int *below = nullptr) {
  const PassEnd &E = A.pe;
  double a = E.a_in[ch], win = E.win_in[ch];
  double accs = 0.0;
  for (int s = 0; s < E.nsw; ++s) {
    const int64_t k = (int64_t)ch * kMaxPass + s;
    const double acc = G.n_gap > 0 ? (double)E.counts[k] / (double)G.n_gap : 1.0;
    accs += acc;
    if (write && E.trace) {
      double *tr = E.trace + ((E.trace_row0 + s) * A.total_chains + ch) * 2;
      tr[0] = acc;
      tr[1] = E.has_energy ? E.energy[k] / (double)G.n_pairs - 1.0 : __builtin_nan("");
    }
    if (E.adapt) {
      win += acc;
      const uint32_t i = E.sweep0 + (uint32_t)s;
      if ((i + 1) % (uint32_t)A.adapt_every == 0) {
        const bool low = win / (double)A.adapt_every < A.a_targ;
        if (low) a = 1.0 + (double)(i + 1) / A.k_a;
        if (below) *below = low ? 1 : 0;
        win = 0.0;
      }
    }
  }
  if (write) {
    A.a_now[ch] = a;
    A.win_now[ch] = win;
    A.accsum[ch] += accs;
  }
  return a;
}

// ---------------------------------------------------------------- sweep
// What one colour phase of the sweep kernel needs to update a site.
template <typename P> struct UpdateCtx {
  using V2 = typename Prec<P>::V2;
  P *pc;               // this colour's angle plane
  V2 *cc;              // this colour's (cos, sin) plane
  const V2 *cn;        // the other colour's (cos, sin) plane
  const P *pn;         // the other colour's angle plane
  int Ly, Lx, P2;
  uint32_t sbase;      // Philox site index of LDS site (0, 0), mod 2^32
  int gnx;             // grid width: LDS site (ly, lx) has index sbase + ly * gnx + lx
  uint32_t sweep, cid, gid, k0, k1;
  P q, inv_q, alpha, beta;
  bool or_step;        // over-relaxation on
  // LDS column of grid x = 0 and x = nx - 1, row of y = 0 and y = ny - 1
  // (outside the LDS range when the tile is away from that edge).
  int ex0, ex1, ey0, ey1;
  // Store the updated sites' (cos, sin): false in the pass's last
  // half-sweep, after which nothing reads them.
  bool store_cs;
  // The interior in LDS columns ix0 .. ix1 and rows iy0 .. iy1, and the
  // reach D of this half-sweep: a site takes part if its distance from the
  // interior is at most D.
  int ix0, ix1, iy0, iy1, D;
};

// Replicate auxiliary nodes (Sec. 2.5): the number of a site's neighbours
// that lie off the grid, each an auxiliary node that holds the site's own
// value from before the half-sweep.
template <typename P>
__device__ __forceinline__ int aux_count(const UpdateCtx<P> &U, int ly, int lx) {
  return (lx == U.ex0 ? 1 : 0) + (lx == U.ex1 ? 1 : 0) + (ly == U.ey0 ? 1 : 0) + (ly == U.ey1 ? 1 : 0);
}

// Algorithm 1 for one plan entry: a pair of sites of this colour in one
// column, the first at LDS (ly, lx) and the second at (ly + 2, lx), whose
// random words come from one Philox call keyed by (first site, sweep,
// chain, grid): (w0, w1) are the first site's (u, r), (w2, w3) the
// second's.  A site takes part if it lies in the grid, within the
// half-sweep's reach and is a gap site; one that does not reads a harmless
// slot and writes nothing.  The two updates are interleaved step by step.
// Returns the accepted updates of interior sites.
//
// MPR pair interaction (Eq. 3): h = sum_j (cos q phi_j, sin q phi_j).
// GMRF (Sec. 4.4): a site's energy is a parabola in its angle about the
// mean m = S/n of its n in-grid neighbours (NaN in the angle plane marks
// none), so over-relaxation reflects about m, kept inside [0, 2 pi), and
// dH = ((p2 - p1) (n (p2 + p1) - 2 S)) / (2 pi^2).  With REP, g auxiliary
// neighbours (Sec. 2.5) add g copies of the site's own value.
template <typename P, int MODEL, bool REP>
__device__ __forceinline__ uint32_t update_pair(const UpdateCtx<P> &U, uint32_t e) {
  constexpr bool QONE = MODEL == kMprQ1, GMRF = MODEL == kGmrf;
  using V2 = typename Prec<P>::V2;
  const P q = U.q;
  const int ly = (int)(e >> 8) + U.Ly, lx = (int)(e & 255u) + U.Lx;
  const int par = lx & 1;  // the parity of both sites' x
  const int rx = max(max(U.ix0 - lx, lx - U.ix1), 0);
  uint32_t w[4];
  philox4x32_10(U.sbase + (uint32_t)(ly * U.gnx + lx), U.sweep, U.cid, U.gid, U.k0, U.k1, w);
  int o[2];
  bool act[2], inner[2];
  P phi[2], hx[2], hy[2], u[2], rr[2];
  // A site's reads (gather) and its update and writes (finish).  FP32
  // interleaves the two sites' steps; FP64 finishes the first site before
  // the second one's reads, which halves the live FP64 temporaries.
  // Neighbouring lanes hold neighbouring pairs of a row: their reads are
  // consecutive in both colour planes.
  auto gather = [&](const int k) __attribute__((always_inline)) {
    const int y = ly + 2 * k;
    const int ring = rx + max(max(U.iy0 - y, y - U.iy1), 0);
    const bool geo = ring <= U.D && y <= U.ey1;
    inner[k] = ring == 0;
    // (LDS row 1, pair 1: every neighbour of it lies in the LDS)
    o[k] = geo ? y * U.P2 + (lx >> 1) : U.P2 + 1;
    phi[k] = U.pc[o[k]];
    act[k] = geo && !signbit(phi[k]);
    if constexpr (GMRF) {
      const P nb[4] = {U.pn[o[k] - 1 + par], U.pn[o[k] + par], U.pn[o[k] - U.P2], U.pn[o[k] + U.P2]};
      P sum = P(0), n = P(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const bool in = !__builtin_isnan(nb[m]);
        sum += in ? fabs(nb[m]) : P(0);
        n += in ? P(1) : P(0);
      }
      if constexpr (REP) {
        const P g = (P)aux_count(U, y, lx);
        sum = fma(g, phi[k], sum);
        n += g;
      }
      hx[k] = sum;  // S and n of the GMRF update
      hy[k] = n;
    } else {
      const V2 nl = U.cn[o[k] - 1 + par], nr = U.cn[o[k] + par];
      const V2 nu = U.cn[o[k] - U.P2], nd = U.cn[o[k] + U.P2];
      hx[k] = nl.x + nr.x + nu.x + nd.x;
      hy[k] = nl.y + nr.y + nu.y + nd.y;
      if constexpr (REP) {
        // off-grid neighbours read (0, 0); each auxiliary one adds the site's own (cos, sin)
        const P g = (P)aux_count(U, y, lx);
        const V2 own = U.cc[o[k]];
        hx[k] = fma(g, own.x, hx[k]);
        hy[k] = fma(g, own.y, hy[k]);
      }
    }
    u[k] = unit<P>(w[2 * k]);
    rr[k] = unit<P>(w[2 * k + 1]);
  };
  uint32_t acc = 0;
  auto finish = [&](const int k) __attribute__((always_inline)) {
    P p1 = phi[k], p2, dH;
    if constexpr (GMRF) {
      const P sum = hx[k], n = hy[k];
      if (U.or_step && n > P(0)) {
        const P star = P(2) * sum / n - phi[k];
        if (star >= P(0) && star < Prec<P>::two_pi) p1 = star;
      }
      p2 = wrap_step(p1 + U.alpha * (u[k] - P(0.5)));
      dH = (p2 - p1) * (n * (p2 + p1) - P(2) * sum) * Prec<P>::inv_2pi2;
    } else {
      // Algorithm 1, step 1: over-relaxation, Eq. (6) with the field of q*phi.
      const P h2 = hx[k] * hx[k] + hy[k] * hy[k];
      const bool live = h2 > Prec<P>::tiny_h2;
      const P psi = live ? Prec<P>::atan2_(hy[k], hx[k]) : P(0);
      if (live && U.or_step) {
        const P star = (P(2) * psi - q * phi[k]) * U.inv_q;
        // (+ 0 turns a reflection to -0 into +0: a set sign bit marks a sample site)
        if (QONE) p1 = wrap_any(star);
        else if (star >= P(0) && star < Prec<P>::two_pi) p1 = star + P(0);
      }
      // Steps 2-3: restricted Metropolis proposal.
      p2 = wrap_step(p1 + U.alpha * (u[k] - P(0.5)));
      // Step 4: dH = -sum_j [cos q(p2 - phi_j) - cos q(p1 - phi_j)]
      //            = 2 |h| sin(q (p2 + p1)/2 - psi) sin(q (p2 - p1)/2).
      dH = P(2) * Prec<P>::sqrt_(h2) * Prec<P>::sin_dh_(q * (p2 + p1) * P(0.5) - psi) *
           Prec<P>::sin_dh_(q * (p2 - p1) * P(0.5));
      dH = live ? dH : P(0);
    }
    // Steps 5-6: accept iff dH <= 0 or r < exp(-dH / T).
    const bool ok = (dH <= P(0)) || (rr[k] < Prec<P>::exp_(-U.beta * dH));
    const P nv = ok ? p2 : p1;
    if (act[k]) {
      U.pc[o[k]] = nv;
      if (!GMRF && U.store_cs) {
        P s_, c_;
        if (QONE) Prec<P>::sincos_(q * nv, &s_, &c_);
        else Prec<P>::sincos_0pi_(q * nv, &s_, &c_);
        U.cc[o[k]] = V2{c_, s_};
      }
    }
    acc += (act[k] && ok && inner[k]) ? 1u : 0u;
  };
  if constexpr (sizeof(P) == 4) {
    gather(0);
    gather(1);
    finish(0);
    finish(1);
  } else {
    gather(0);
    finish(0);
    gather(1);
    finish(1);
  }
  return acc;
}

// One workgroup = one (grid, chain, tile) item.  Distances from the
// interior are Manhattan distances (dx + dy outside the tile), the reach of
// nearest-neighbour dependencies.  Half-sweep hs of the pass updates the
// colour-(hs & 1) gap sites within distance D = 2*nsw - 1 - hs: each reads
// neighbours within D + 1, exact after half-sweep hs - 1 (the staged halo of
// 2*nsw sites covers hs = 0), so the interior is exact after the last
// half-sweep.  When the energy of interior pairs is traced, every D and the
// halo are one larger, so that the interior plus one ring is exact after
// each sweep.  The gap sites come from the tile's plan as pairs (one Philox
// call each): thread i updates pairs i, i + NT, ... of a half-sweep.
// With RREG (an FP32 pass that records two or more sweeps), the fill sums of
// a thread's first interior sites stay in registers for the whole pass:
// loaded before the first record and stored after the last, instead of a
// read-modify-write in HBM per record.  The sums are the same, term by term.
// With REDO (the redo of a speculative pass's mispredicted chains), the
// previous pass's end is not applied a second time.
template <typename P, int NT, int MODEL, bool REP, bool RREG, bool REDO>
__device__ __forceinline__ void sweep_item(const SweepArgs<P> &A, const int64_t item) {
  constexpr bool QONE = MODEL == kMprQ1;
  using V2 = typename Prec<P>::V2;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_d[NT / 64];
  __shared__ uint32_t acc_lds[kMaxPass];
  __shared__ double a_lds, a1_lds;

  if (item >= A.n_items) return;  // past the last item
  // The coarse index narrows the search to the grids between two entries
  // (usually one or two in a batch of large grids).
  int gi = 0;
  if (A.n_grids > 1) {
    const int64_t ik = item / kItemStride;
    gi = find_by(A.grids, A.n_grids, item, &GridDesc::item_begin, A.item_grid[ik], A.item_grid[ik + 1]);
  }
  const GridDesc G = A.grids[gi];  // by value: kept in registers across LDS stores
  const int64_t local = item - G.item_begin;
  const int tiles = G.tiles_x * G.tiles_y;
  const int chain = (int)(local / tiles);
  const int t = (int)(local - (int64_t)chain * tiles);
  const int nx = G.nx, ny = G.ny;
  const int x0 = (t % G.tiles_x) * A.tile_x, y0 = (t / G.tiles_x) * A.tile_y;
  const int ix1 = min(x0 + A.tile_x, nx), iy1 = min(y0 + A.tile_y, ny);
  // Halo: 2 * nsw sites, one more when the energy is traced (the reach of
  // the pass's first half-sweep plus one).  LDS columns start at an even
  // grid x (LDS x has the parity of grid x, so both colour planes pair
  // sites lx / 2); a grid edge within the halo leaves zeros outside.
  const int H = 2 * A.nsw + (A.energy ? 1 : 0), Hx = (H + 1) & ~1;
  const int ox = max(x0 - Hx, -2);
  const int oy = max(y0 - H, -1);
  const int lxs = max(x0 - H, 0), lxe = min(ix1 + H, nx);
  const int lys = max(y0 - H, 0), lye = min(iy1 + H, ny);
  const int W = A.lds_w, P2 = W >> 1, plane = A.lds_h * P2;

  V2 *cs = reinterpret_cast<V2 *>(smem);                         // (cos q phi, sin q phi)
  P *ph = reinterpret_cast<P *>(smem + 2 * plane * sizeof(V2));  // encoded angle
  const P q = (P)G.q, inv_q = (P)G.inv_q;
  const int64_t cbase = G.state_off + (int64_t)chain * nx * ny;
  const P *src = A.src + cbase;

  // The tile's plan counts, loaded before the kernel's first store to
  // global memory (so that they come through the scalar cache, uniform and
  // without a wait on the vector loads below).
  const int64_t pitem = G.plan_begin + t;
  const uint32_t *cum = A.plan_cum + pitem * 2 * (A.plan_dmax + 2);
  const int cstride = A.plan_dmax + 2;
  const uint32_t n0_all = cum[A.plan_dmax + 1];
  const uint32_t na = cum[2 * A.nsw + 1], nb = cum[cstride + 2 * A.nsw];
  // Stage the tile, its halo (with a frozen zero row or column where a grid
  // edge lies within it), and this pass's part of the tile's plan:
  // colour-0 pairs within distance 2*nsw, then colour-1 pairs within
  // distance 2*nsw - 1.  Each thread issues the loads of up to kStage site
  // slots and kPlanStage plan pairs before it waits for any, so the staging
  // costs one memory latency per batch (one batch for the library's
  // default shapes).
  if (threadIdx.x < kMaxPass) acc_lds[threadIdx.x] = 0u;
  const int gchain = G.chain_base + chain;
  // Close the previous pass (every tile derives the same a; tile 0 records,
  // except in a redo, where the first launch has recorded it): one thread,
  // while the staging loads are in flight.  A speculative pass predicts the
  // a-rule outcome of its sweep 0 to be that of the last known sweep
  // (acceptance below a_targ when none is known); its redo takes the other.
  if (threadIdx.x == 0) {
    int below = 1;
    const double a0 = A.pe.valid ? apply_pass_end(A, G, gchain, t == 0 && !REDO, &below) : A.a_now[gchain];
    a_lds = a0;
    if (A.spec) {
      const int pb = REDO ? 1 - below : below;
      a1_lds = pb ? 1.0 + (double)(A.sweep0 + 1) / A.k_a : a0;
      if (!REDO && t == 0) A.pred[gchain] = (uint32_t)pb;
      // (the redo list's count follows the predictions; k_spec_check counts
      // from zero after this launch)
      if (!REDO && item == 0) A.pred[A.total_chains] = 0u;
    }
  }
  if (!REDO && t == 0 && threadIdx.x < kMaxPass) A.counts_clear[(int64_t)gchain * kMaxPass + threadIdx.x] = 0u;
  uint16_t *list = reinterpret_cast<uint16_t *>(ph + 2 * plane);  // past both planes
  // LDS site (ly, lx) is grid site (oy + ly, ox + lx); its colour is
  // (lx + ly + par0) & 1.
  const int par0 = (ox + oy) & 1;
  {
    // Sites are staged two at a time: LDS sites (ly, 2j) and (ly, 2j + 1),
    // one of each colour, both at index ly * P2 + j of their colour's
    // planes.  The colour-1 site's (cos, sin) is always needed, so every
    // lane computes one; the colour-0 site's only for a sample, an off-grid
    // site or at the replicate boundary (see below), which most waves skip
    // as a whole.  One batch covers a 64 x 64 tile's sites and one-sweep
    // plan at 512 threads or more.
    constexpr int kStage = 8, kPlanStage = NT >= 512 ? 5 : 8;
    using Pair = typename Prec<P>::V2;  // two consecutive angles
    const int n_slots = P2 * A.lds_h;
    const float invp = 1.0f / (float)P2;
    const uint16_t *pl = A.plan + G.plan_ebase + (int64_t)t * G.plan_cap;
    const uint32_t n_all = na + nb;
    // Thread i stages slots i, i + NT, ... in row-major order: its (ly, j)
    // moves by (NT / P2, NT % P2) per slot, with a carry.  The in-grid part
    // of the LDS rectangle is [ax, ax + aw) x [ay, ay + ah); the chain's
    // angle of LDS site (ly, lx) is src[ib + ly * nx + lx], an index below
    // 2^32 for every in-grid site.  When nx and the chain's first index are
    // even, both angles of a slot come in one 2-element load (ox is even).
    const int dly = NT / P2, dlj = NT - (NT / P2) * P2;
    int sly, sj;
    split_index((int)threadIdx.x, P2, invp, sly, sj);
    const int ax = lxs - ox, aw = lxe - lxs, ay = lys - oy, ah = lye - lys;
    const uint32_t ib = (uint32_t)((int64_t)oy * nx + ox);
    const bool wide = ((nx | (int)(cbase & 1)) & 1) == 0;
    for (int base = 0, pb = 0; base < n_slots || pb < (int)n_all; base += NT * kStage, pb += NT * kPlanStage) {
      // Slots wholly past the end (a workgroup-uniform test) issue nothing.
      // The angles load first: their addresses do not wait for the counts.
      P va[kStage], vb[kStage];
      int jj[kStage], ca[kStage];
      bool ina[kStage], inb[kStage];
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        jj[k] = -1;  // every slot, also those past the loop's break below
        ca[k] = 0;
        ina[k] = inb[k] = false;
        va[k] = vb[k] = P(0);
      }
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        if (base + k * NT >= n_slots) break;
        if (sly < A.lds_h) {
          const int slx = 2 * sj;
          jj[k] = sly * P2 + sj;
          ca[k] = (sly + par0) & 1;  // colour of the slot's first site
          const bool iny = (uint32_t)(sly - ay) < (uint32_t)ah;
          ina[k] = iny && (uint32_t)(slx - ax) < (uint32_t)aw;
          inb[k] = iny && (uint32_t)(slx + 1 - ax) < (uint32_t)aw;
          const uint32_t i0 = ib + (uint32_t)(sly * nx + slx);
          if (wide && ina[k] && inb[k]) {
            const Pair two = *reinterpret_cast<const Pair *>(src + i0);
            va[k] = two.x;
            vb[k] = two.y;
          } else {
            if (ina[k]) va[k] = src[i0];
            if (inb[k]) vb[k] = src[i0 + 1];
          }
        }
        sj += dlj;
        sly += dly;
        if (sj >= P2) {
          sj -= P2;
          ++sly;
        }
      }
      uint16_t e[kPlanStage] = {};
#pragma unroll
      for (int k = 0; k < kPlanStage; ++k) {
        if (pb + k * NT >= (int)n_all) break;
        const uint32_t f = (uint32_t)(pb + k * NT) + threadIdx.x;
        e[k] = pl[f < na ? f : (f < n_all ? n0_all + (f - na) : 0u)];
      }
#pragma unroll
      for (int k = 0; k < kStage; ++k) {
        if (jj[k] < 0) continue;
        // the slot's colour-0 and colour-1 sites
        const bool in0 = ca[k] ? inb[k] : ina[k], in1 = ca[k] ? ina[k] : inb[k];
        const P v0 = ca[k] ? vb[k] : va[k], v1 = ca[k] ? va[k] : vb[k];
        const int j = jj[k];
        if constexpr (MODEL == kGmrf) {
          // angles only; NaN marks a site outside the grid or the halo
          ph[j] = in0 ? v0 : P(__builtin_nan(""));
          ph[plane + j] = in1 ? v1 : P(__builtin_nan(""));
        } else {
          const P a0 = in0 ? v0 : -P(0), a1 = in1 ? v1 : -P(0);
          {
            P s_, c_;
            if (QONE) Prec<P>::sincos_(q * fabs(a1), &s_, &c_);
            else Prec<P>::sincos_0pi_(q * fabs(a1), &s_, &c_);
            cs[plane + j] = in1 ? V2{c_, s_} : V2{P(0), P(0)};
          }
          // (cos, sin) of colour-0 gap sites is never read before the
          // pass's first half-sweep recomputes it (every colour-0 gap site
          // a colour-1 update reads lies in that half-sweep's reach), except
          // for a site's own value at the replicate boundary.
          if (!in0 || REP || signbit(a0)) {
            P s_ = P(0), c_ = P(0);
            if (in0) {
              if (QONE) Prec<P>::sincos_(q * fabs(a0), &s_, &c_);
              else Prec<P>::sincos_0pi_(q * fabs(a0), &s_, &c_);
            }
            cs[j] = V2{c_, s_};
          }
          ph[j] = a0;
          ph[plane + j] = a1;
        }
      }
#pragma unroll
      for (int k = 0; k < kPlanStage; ++k) {
        const uint32_t f = (uint32_t)(pb + k * NT) + threadIdx.x;
        if (f < n_all) list[f] = e[k];
      }
    }
  }
  __syncthreads();
  const double a_d = a_lds;
  const P beta = (P)A.beta[gchain], alpha = (P)(6.28318530717958647692 / a_d);
  const P alpha1 = A.spec ? (P)(6.28318530717958647692 / a1_lds) : alpha;  // sweep 1's
  const uint32_t k0 = A.key0, k1 = A.key1, cid = (uint32_t)chain, gid = (uint32_t)G.grid_id;
  const int iw = ix1 - x0, ih = iy1 - y0;
  const float inv_iw = 1.0f / (float)iw;
  // Plan entries are decoded relative to these LDS offsets; LDS site
  // (ly, lx) is grid site (oy + ly, ox + lx), Philox site index
  // sbase + ly * nx + lx (mod 2^32).
  const int Ly = y0 - oy - kPlanOffset, Lx = x0 - ox - kPlanOffset;
  const uint32_t sbase = (uint32_t)((int64_t)oy * nx + ox);
  // Register-held fill sums (RREG): sites f = threadIdx.x + j * NT, j < kRegSites.
  constexpr int kRegSites = RREG ? (NT >= 512 ? 4096 / NT : 8) : 1;
  P r_ref[kRegSites], r_s1[kRegSites], r_s2[kRegSites];
  auto reg_site = [&](int j, int64_t &k, P &v) __attribute__((always_inline)) {
    const int f = (int)threadIdx.x + j * NT;
    if (f >= iw * ih) return false;
    int r, cx;
    split_index(f, iw, inv_iw, r, cx);
    const int gx = x0 + cx, gy = y0 + r;
    k = cbase + (int64_t)gy * nx + gx;
    v = ph[((gx + gy) & 1) * plane + (gy - oy) * P2 + ((gx - ox) >> 1)];
    return !signbit(v);  // sample sites carry no sums
  };
  if constexpr (RREG) {
    // The pass's first record continues the fill's sums unless it starts them.
    const uint32_t low = A.record_mask & (0u - A.record_mask);
    if (!(A.first_mask & low)) {
#pragma unroll
      for (int j = 0; j < kRegSites; ++j) {
        int64_t k;
        P v;
        if (reg_site(j, k, v)) {
          r_ref[j] = A.acc_ref[k];
          r_s1[j] = A.acc_s1[k];
          r_s2[j] = A.acc_s2[k];
        }
      }
    }
  }

  for (int s = 0; s < A.nsw; ++s) {
    const uint32_t sweep = A.sweep0 + (uint32_t)s;
    uint32_t acc = 0;
    // One colour phase (half-sweep): thread i updates the plan pairs
    // i, i + NT, ... within this half-sweep's reach.
    for (int c = 0; c < 2; ++c) {
      const int D = 2 * A.nsw - (2 * s + c) - (A.energy ? 0 : 1);
      const uint32_t n = cum[c * cstride + D + 1];  // pairs within ring D
      const uint16_t *lc = list + (c ? na : 0);
      const UpdateCtx<P> U{ph + c * plane,  cs + c * plane,  cs + (c ^ 1) * plane, ph + (c ^ 1) * plane,
                           Ly,    Lx,  P2,  sbase, nx,
                           sweep, cid, gid, k0,    k1,
                           q,     inv_q, s == 1 ? alpha1 : alpha, beta, A.or_step != 0,
                           -ox,   nx - 1 - ox, -oy, ny - 1 - oy,
                           !(c == 1 && s == A.nsw - 1),
                           x0 - ox, ix1 - 1 - ox, y0 - oy, iy1 - 1 - oy, D};
      for (uint32_t f = threadIdx.x; f < n; f += NT) acc += update_pair<P, MODEL, REP>(U, lc[f]);
      __syncthreads();
    }

    {
      const uint32_t wsum = wave_sum(acc);
      if ((threadIdx.x & 63) == 0 && wsum) atomicAdd(&acc_lds[s], wsum);
    }
    const bool rec = (A.record_mask >> s) & 1u;
    if (A.energy) {
      // Eq. (5): pairs (x, y)-(x+1, y) and (x, y)-(x, y+1) owned by interior sites.
      P e = P(0);
      for (int f = threadIdx.x; f < iw * ih; f += NT) {
        int r, cx;
        split_index(f, iw, inv_iw, r, cx);
        const int gx = x0 + cx, gy = y0 + r;
        const int lx = gx - ox, ly = gy - oy;
        const int col = (gx + gy) & 1;
        const P v = fabs(ph[col * plane + ly * P2 + (lx >> 1)]);
        // 1 - H_ij: 2 sin^2(q d / 2) (MPR), d^2 / (2 pi^2) (GMRF)
        auto pair = [&](P d) {
          if constexpr (MODEL == kGmrf) return d * d * Prec<P>::inv_2pi2;
          const P sn = Prec<P>::sin_(q * d * P(0.5));
          return P(2) * sn * sn;
        };
        if (gx + 1 < nx) e += pair(v - fabs(ph[(col ^ 1) * plane + ly * P2 + ((lx + 1) >> 1)]));
        if (gy + 1 < ny) e += pair(v - fabs(ph[(col ^ 1) * plane + (ly + 1) * P2 + (lx >> 1)]));
      }
      // One partial per item; k_energy_reduce sums a chain's partials in a
      // fixed order, so the trace does not depend on workgroup timing.
      const double et = block_sum<NT>((double)e, red_d);
      if (threadIdx.x == 0) A.energy_part[(int64_t)s * A.n_items + item] = et;
    }
    if (rec) {
      // Algorithm 2, step 5.3: one realisation; shifted sums about the first.
      const bool first = (A.first_mask >> s) & 1u;
      if constexpr (RREG) {
#pragma unroll
        for (int j = 0; j < kRegSites; ++j) {
          int64_t k;
          P v;
          if (!reg_site(j, k, v)) continue;
          if (first) {
            r_ref[j] = v;
            r_s1[j] = P(0);
            r_s2[j] = P(0);
          } else {
            const P d = v - r_ref[j];
            r_s1[j] += d;
            r_s2[j] += d * d;
          }
        }
      }
      for (int f = threadIdx.x + (RREG ? kRegSites * NT : 0); f < iw * ih; f += NT) {
        int r, cx;
        split_index(f, iw, inv_iw, r, cx);
        const int gx = x0 + cx, gy = y0 + r;
        const int lx = gx - ox, ly = gy - oy;
        const P v = ph[((gx + gy) & 1) * plane + ly * P2 + (lx >> 1)];
        if (signbit(v)) continue;
        const int64_t k = cbase + (int64_t)gy * nx + gx;
        if (first) {
          A.acc_ref[k] = v;
          A.acc_s1[k] = P(0);
          A.acc_s2[k] = P(0);
        } else {
          const P d = v - A.acc_ref[k];
          A.acc_s1[k] += d;
          A.acc_s2[k] += d * d;
        }
      }
    }
    if (A.energy || rec) __syncthreads();  // the next sweep overwrites what was read
  }
  __syncthreads();
  if (threadIdx.x < A.nsw && acc_lds[threadIdx.x])
    atomicAdd(&A.counts[(int64_t)gchain * kMaxPass + threadIdx.x], acc_lds[threadIdx.x]);

  if constexpr (RREG) {
    const bool started = (A.first_mask & A.record_mask) != 0;
#pragma unroll
    for (int j = 0; j < kRegSites; ++j) {
      int64_t k;
      P v;
      if (!reg_site(j, k, v)) continue;
      if (started) A.acc_ref[k] = r_ref[j];
      A.acc_s1[k] = r_s1[j];
      A.acc_s2[k] = r_s2[j];
    }
  }

  // Write the interior's gap sites to the other buffer (sample sites hold
  // the same value in both buffers from set-up on).  Thread i writes
  // interior sites i, i + NT, ... in row-major order, its (row, column)
  // moved by (NT / iw, NT % iw) per site.
  // Batches of kOut sites: every LDS read of a batch is issued before its
  // first store.
  {
    constexpr int kOut = 8;
    P *dst = A.dst + cbase;
    const int dr = NT / iw, dc = NT - (NT / iw) * iw;
    int r, cx;
    split_index((int)threadIdx.x, iw, inv_iw, r, cx);
    for (int f0 = 0; f0 < iw * ih; f0 += kOut * NT) {
      P v[kOut];
      uint32_t at[kOut];
#pragma unroll
      for (int k = 0; k < kOut; ++k) {
        v[k] = -P(0);
        if (f0 + k * NT + (int)threadIdx.x < iw * ih) {
          const int lx = x0 - ox + cx, ly = y0 - oy + r;
          v[k] = ph[((lx + ly + par0) & 1) * plane + ly * P2 + (lx >> 1)];
        }
        at[k] = (uint32_t)(y0 + r) * (uint32_t)nx + (uint32_t)(x0 + cx);
        cx += dc;
        r += dr;
        if (cx >= iw) {
          cx -= iw;
          ++r;
        }
      }
#pragma unroll
      for (int k = 0; k < kOut; ++k)
        if (!signbit(v[k])) dst[at[k]] = v[k];
    }
  }
}

template <typename P, int NT, int MODEL, bool REP, bool RREG>
__global__ void __launch_bounds__(NT) k_sweep(const SweepArgs<P> A) {
  sweep_item<P, NT, MODEL, REP, RREG, false>(A, xcd_item(A.n_items));
}

// The redo of a speculative pass: the workgroups share the items of the
// chains listed by k_spec_check (none, mostly, and then they exit at once).
template <typename P, int NT, int MODEL, bool REP>
__global__ void __launch_bounds__(NT) k_sweep_redo(const SweepArgs<P> A) {
  const uint32_t n_list = A.redo[0];
  for (uint32_t k = 0; k < n_list; ++k) {
    const int ch = (int)A.redo[1 + k];
    int lo = 0, hi = A.n_grids - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.grids[mid].chain_base <= ch) lo = mid;
      else hi = mid - 1;
    }
    const GridDesc &G = A.grids[lo];
    const int64_t tiles = (int64_t)G.tiles_x * G.tiles_y;
    const int64_t i0 = G.item_begin + (int64_t)(ch - G.chain_base) * tiles;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
      sweep_item<P, NT, MODEL, REP, false, true>(A, i0 + t);
      __syncthreads();  // the next item restages the LDS
    }
  }
}

// ------------------------------------------------- persistent single sweep
// One sweep per pass (the a-rule's passes) with persistent workgroups:
// each workgroup runs a fixed share of the (grid, chain, tile) items and,
// while it sweeps one item out of LDS, has the next item's angles and
// gap-site plan entries already loading into registers, so the memory
// latency of staging overlaps the arithmetic of the previous item.  The
// plan entries stay in registers (thread i updates entries i, i + NT, ...
// of each colour), so the pass stages no list in LDS.  Same arithmetic per
// site and the same random words as k_sweep: results are bit-identical.
//
// Items are cut into 8 contiguous ranges, one per XCD (a workgroup runs on
// XCD blockIdx.x % 8): tiles that share halo rows go through the same L2.
// A grid descriptor in scalar registers: loaded and read from the first
// lane (every lane loads the same one).
__device__ __forceinline__ GridDesc uniform_desc(const GridDesc *p) {
  static_assert(sizeof(GridDesc) % 4 == 0, "GridDesc is a whole number of words");
  GridDesc d = *p;
  uint32_t w[sizeof(GridDesc) / 4];
  __builtin_memcpy(w, &d, sizeof(d));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(GridDesc) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  __builtin_memcpy(&d, w, sizeof(d));
  return d;
}

// Where item `item` lies: its grid (from the coarse index), chain and tile.
__device__ __forceinline__ int item_grid_of(const int32_t *item_grid, const GridDesc *grids, int n_grids,
                                            int64_t item) {
  const int64_t ik = item / kItemStride;
  return find_by(grids, n_grids, item, &GridDesc::item_begin, item_grid[ik], item_grid[ik + 1]);
}

// Where item `it` of grid gi lies, and the addresses its loads use.
template <typename P> struct ItemGeo {
  int chain, t, nx, x0, y0, ox, oy;
  int ax, aw, ay, ah;       // in-grid part of the LDS rectangle
  uint32_t ib;              // chain index of LDS site (0, 0), mod 2^32
  const P *src;             // the chain's angles
  const uint32_t *cum;      // the tile's plan counts
  const uint16_t *pl;       // the tile's plan entries
};

template <typename P>
__device__ __forceinline__ ItemGeo<P> item_geo(const SweepArgs<P> &A, const GridDesc &G, int64_t it, int H) {
  ItemGeo<P> g;
  const int64_t local = it - G.item_begin;
  const int tiles = G.tiles_x * G.tiles_y;
  g.chain = (int)(local / tiles);
  g.t = (int)(local - (int64_t)g.chain * tiles);
  g.nx = G.nx;
  const int ny = G.ny;
  g.x0 = (g.t % G.tiles_x) * A.tile_x;
  g.y0 = (g.t / G.tiles_x) * A.tile_y;
  const int ix1 = min(g.x0 + A.tile_x, g.nx), iy1 = min(g.y0 + A.tile_y, ny);
  g.ox = max(g.x0 - ((H + 1) & ~1), -2);
  g.oy = max(g.y0 - H, -1);
  g.ax = max(g.x0 - H, 0) - g.ox;
  g.aw = min(ix1 + H, g.nx) - max(g.x0 - H, 0);
  g.ay = max(g.y0 - H, 0) - g.oy;
  g.ah = min(iy1 + H, ny) - max(g.y0 - H, 0);
  g.ib = (uint32_t)((int64_t)g.oy * g.nx + g.ox);
  g.src = A.src + G.state_off + (int64_t)g.chain * g.nx * ny;
  g.cum = A.plan_cum + (G.plan_begin + g.t) * 2 * (A.plan_dmax + 2);
  g.pl = A.plan + G.plan_ebase + (int64_t)g.t * G.plan_cap;
  return g;
}

template <typename P, int NT, int MODEL, bool REP>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT >= 512 ? 4 : 2)))
    k_sweep1(const SweepArgs<P> A) {
  constexpr bool QONE = MODEL == kMprQ1;
  constexpr int kS = p1_sites(NT), kE = p1_plan(NT);
  using V2 = typename Prec<P>::V2;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red_d[NT / 64];
  __shared__ double a_lds;
  __shared__ uint32_t acc_lds;

  const int W = A.lds_w, P2 = W >> 1, plane = A.lds_h * P2, n_lds = W * A.lds_h;
  V2 *cs = reinterpret_cast<V2 *>(smem);
  P *ph = reinterpret_cast<P *>(smem + 2 * plane * sizeof(V2));
  const int H = A.energy ? 3 : 2;  // the halo of a one-sweep pass (as k_sweep)
  const int cstride = A.plan_dmax + 2;
  // Reach of the two half-sweeps (rings), one more with the energy traced.
  const int D0 = A.energy ? 2 : 1, D1 = D0 - 1;
  // The LDS site of a thread's k-th staging slot, the same for every item.
  const float invw = 1.0f / (float)W;
  const int dly = NT / W, dlx = NT - (NT / W) * W;
  int sly0, slx0;
  split_index((int)threadIdx.x, W, invw, sly0, slx0);

  // This workgroup's items: xcd range [r0, r1), items r0 + lb + k * g8.
  const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3, g8 = gridDim.x >> 3;
  const int64_t per = (A.n_items + 7) / 8;
  const int64_t r0 = (int64_t)xcd * per, r1 = min(r0 + per, A.n_items);
  int64_t item = r0 + lb;
  if (item >= r1) return;

  // The loads are ordered so that a wait for one of them never waits for a
  // later item's angles or entries (the counter of outstanding loads
  // retires in issue order): the next item's plan counts are loaded one
  // item ahead, its grid descriptor reused while the grid stays the same.
  //   vn, inmask: angles of the next item (and which slots lie in the grid)
  //   en[c][j]: plan entry threadIdx.x + j * NT of colour c of the next item
  //   cum_n / cum_nn: plan counts of the next item / the one after
  P vn[kS];
  uint32_t inmask = 0;
  uint32_t en[2][kE];
  struct Counts { uint32_t n[2], c1; };
  // The same counts in scalar registers (read from the first lane): used
  // there, they keep the sweep's loops free of waits for vector loads.
  auto scalar = [](const Counts &k) __attribute__((always_inline)) {
    Counts u;
    u.n[0] = __builtin_amdgcn_readfirstlane(k.n[0]);
    u.n[1] = __builtin_amdgcn_readfirstlane(k.n[1]);
    u.c1 = __builtin_amdgcn_readfirstlane(k.c1);
    return u;
  };
  auto load_counts = [&](const uint32_t *cum) __attribute__((always_inline)) {
    Counts k;
    k.n[0] = cum[D0 + 1];
    k.n[1] = cum[cstride + D1 + 1];
    k.c1 = cum[A.plan_dmax + 1];
    return k;
  };
  auto load_sites = [&](const ItemGeo<P> &g) __attribute__((always_inline)) {
    int sly = sly0, slx = slx0;
    inmask = 0;
#pragma unroll
    for (int k = 0; k < kS; ++k) {
      vn[k] = P(0);
      if (k * NT < n_lds && sly < A.lds_h && (uint32_t)(slx - g.ax) < (uint32_t)g.aw &&
          (uint32_t)(sly - g.ay) < (uint32_t)g.ah) {
        vn[k] = g.src[g.ib + (uint32_t)(sly * g.nx + slx)];
        inmask |= 1u << k;
      }
      slx += dlx;
      sly += dly;
      if (slx >= W) {
        slx -= W;
        ++sly;
      }
    }
  };
  // (One register per entry: nothing uses a loaded entry before the next
  // item, so no wait follows these loads.)
  auto load_plan = [&](const ItemGeo<P> &g, int c, uint32_t n, uint32_t base) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < kE; ++j) {
      const uint32_t f = threadIdx.x + (uint32_t)(j * NT);
      if (f < n) en[c][j] = g.pl[base + f];
    }
  };
  // Grid of an item: the cached one while the item lies in it.
  auto in_grid = [&](const GridDesc &G, int64_t it) __attribute__((always_inline)) {
    return it >= G.item_begin && it < G.item_begin + (int64_t)G.chains * G.tiles_x * G.tiles_y;
  };

  GridDesc G = uniform_desc(A.grids + item_grid_of(A.item_grid, A.grids, A.n_grids, item));  // grid of `item`
  // Plan counts of the current and of the next item, in two sets whose
  // roles alternate between iterations (the loop body is written twice):
  // the set that held the current item's counts receives those of the item
  // after next once its last reader is done, so no counts move between
  // registers (a move would wait for the load, and with it for every load
  // issued earlier).
  Counts kA, kB{};
  {
    const ItemGeo<P> g = item_geo(A, G, item, H);
    kA = load_counts(g.cum);
    load_sites(g);
    load_plan(g, 0, kA.n[0], 0u);
    load_plan(g, 1, kA.n[1], kA.c1);
  }
  GridDesc Gn = G;  // grid of the next item
  int64_t next = item + g8;
  if (next < r1) {
    if (!in_grid(Gn, next)) Gn = uniform_desc(A.grids + item_grid_of(A.item_grid, A.grids, A.n_grids, next));
    kB = load_counts(item_geo(A, Gn, next, H).cum);
  }
  int a_chain = -1, b_chain = -1;
  P beta = P(0);
  if (threadIdx.x == 0) acc_lds = 0u;

  // One item; returns false after the workgroup's last item.
  auto step = [&](Counts &kc_v, Counts &kn_v) __attribute__((always_inline)) {
    // (this item's counts were loaded two items ago, the next item's during
    // the previous write-out: waiting for them here waits for no angle)
    const Counts kc = scalar(kc_v), kn = scalar(kn_v);
    const ItemGeo<P> g = item_geo(A, G, item, H);
    const int nx = g.nx, ny = G.ny;
    const int x0 = g.x0, y0 = g.y0, ox = g.ox, oy = g.oy, chain = g.chain, t = g.t;
    const int ix1 = min(x0 + A.tile_x, nx), iy1 = min(y0 + A.tile_y, ny);
    const int par0 = (ox + oy) & 1;
    const P q = (P)G.q, inv_q = (P)G.inv_q;
    const int64_t cbase = G.state_off + (int64_t)chain * nx * ny;
    const int gchain = G.chain_base + chain;

    // Stage this item from the registers (as k_sweep does).
    {
      int sly = sly0, slx = slx0;
#pragma unroll
      for (int k = 0; k < kS; ++k) {
        if (k * NT < n_lds && sly < A.lds_h) {
          const int o = ((slx + sly + par0) & 1) * plane + sly * P2 + (slx >> 1);
          const bool in = (inmask >> k) & 1u;
          if constexpr (MODEL == kGmrf) {
            ph[o] = in ? vn[k] : P(__builtin_nan(""));
          } else {
            const P val = in ? vn[k] : -P(0);
            if (!in || REP || o >= plane || signbit(val)) {
              P s_ = P(0), c_ = P(0);
              if (in) {
                if (QONE) Prec<P>::sincos_(q * fabs(val), &s_, &c_);
                else Prec<P>::sincos_0pi_(q * fabs(val), &s_, &c_);
              }
              cs[o] = V2{c_, s_};
            }
            ph[o] = val;
          }
        }
        slx += dlx;
        sly += dly;
        if (slx >= W) {
          slx -= W;
          ++sly;
        }
      }
    }
    // The previous pass's end for this chain: once per chain, and by tile 0.
    if (threadIdx.x == 0) {
      if (gchain != a_chain || t == 0) {
        a_lds = A.pe.valid ? apply_pass_end(A, G, gchain, t == 0) : A.a_now[gchain];
        a_chain = gchain;
      }
    }
    if (t == 0 && threadIdx.x < kMaxPass) A.counts_clear[(int64_t)gchain * kMaxPass + threadIdx.x] = 0u;
    if (gchain != b_chain) {  // one inverse temperature per chain, in scalar registers
      const double b = A.beta[gchain];
      uint32_t w[2];
      __builtin_memcpy(w, &b, 8);
      w[0] = __builtin_amdgcn_readfirstlane(w[0]);
      w[1] = __builtin_amdgcn_readfirstlane(w[1]);
      double bu;
      __builtin_memcpy(&bu, w, 8);
      beta = (P)bu;
      b_chain = gchain;
    }
    __syncthreads();

    // The next item: its angles load during this item's first half-sweep,
    // its colour-0 entries during the second, its colour-1 entries and the
    // counts of the item after it during the write-out.
    const bool more = next < r1;
    const int64_t next2 = next + g8;
    ItemGeo<P> gn{};
    if (more) {
      gn = item_geo(A, Gn, next, H);
      load_sites(gn);
    }

    const P alpha = (P)(6.28318530717958647692 / a_lds);
    const uint32_t sbase = g.ib;
    const int Ly = y0 - oy - kPlanOffset, Lx = x0 - ox - kPlanOffset;
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const UpdateCtx<P> U{ph + c * plane, cs + c * plane, cs + (c ^ 1) * plane, ph + (c ^ 1) * plane,
                           Ly, Lx, P2, sbase, nx,
                           A.sweep0, (uint32_t)chain, (uint32_t)G.grid_id, A.key0, A.key1,
                           q, inv_q, alpha, beta, A.or_step != 0,
                           -ox, nx - 1 - ox, -oy, ny - 1 - oy,
                           c == 0,
                           x0 - ox, ix1 - 1 - ox, y0 - oy, iy1 - 1 - oy, c == 0 ? D0 : D1};
      const uint32_t n = kc.n[c];
#pragma unroll
      for (int j = 0; j < kE; ++j) {
        if ((uint32_t)(j * NT) >= n) break;
        if (threadIdx.x + (uint32_t)(j * NT) < n) acc += update_pair<P, MODEL, REP>(U, en[c][j]);
      }
      __syncthreads();
      if (more) load_plan(gn, c, kn.n[c], c ? kn.c1 : 0u);
    }
    // The counts of the item after next, into the set this item's counts
    // held (read for the last time above).
    GridDesc Gx = Gn;
    if (more && next2 < r1) {
      if (!in_grid(Gx, next2)) Gx = uniform_desc(A.grids + item_grid_of(A.item_grid, A.grids, A.n_grids, next2));
      kc_v = load_counts(item_geo(A, Gx, next2, H).cum);
    }
    {
      const uint32_t wsum = wave_sum(acc);
      if ((threadIdx.x & 63) == 0 && wsum) atomicAdd(&acc_lds, wsum);
    }
    const int iw = ix1 - x0, ih = iy1 - y0;
    const float inv_iw = 1.0f / (float)iw;
    if (A.energy) {
      // Eq. (5): pairs owned by interior sites (as k_sweep), one partial per item.
      P e = P(0);
      for (int f = threadIdx.x; f < iw * ih; f += NT) {
        int r, cx;
        split_index(f, iw, inv_iw, r, cx);
        const int gx = x0 + cx, gy = y0 + r;
        const int lx = gx - ox, ly = gy - oy;
        const int col = (gx + gy) & 1;
        const P v = fabs(ph[col * plane + ly * P2 + (lx >> 1)]);
        auto pair = [&](P d) {
          if constexpr (MODEL == kGmrf) return d * d * Prec<P>::inv_2pi2;
          const P sn = Prec<P>::sin_(q * d * P(0.5));
          return P(2) * sn * sn;
        };
        if (gx + 1 < nx) e += pair(v - fabs(ph[(col ^ 1) * plane + ly * P2 + ((lx + 1) >> 1)]));
        if (gy + 1 < ny) e += pair(v - fabs(ph[(col ^ 1) * plane + (ly + 1) * P2 + (lx >> 1)]));
      }
      const double et = block_sum<NT>((double)e, red_d);
      if (threadIdx.x == 0) A.energy_part[item] = et;
    }
    // Write the interior's gap sites (as k_sweep), in a fixed number of
    // slots (the interior is part of the staged rectangle).
    {
      P *dst = A.dst + cbase;
      const int dr = NT / iw, dc = NT - (NT / iw) * iw;
      int r, cx;
      split_index((int)threadIdx.x, iw, inv_iw, r, cx);
#pragma unroll
      for (int k = 0; k < kS; ++k) {
        if (k * NT + (int)threadIdx.x < iw * ih) {
          const int lx = x0 - ox + cx, ly = y0 - oy + r;
          const P v = ph[((lx + ly + par0) & 1) * plane + ly * P2 + (lx >> 1)];
          if (!signbit(v)) dst[(uint32_t)(y0 + r) * (uint32_t)nx + (uint32_t)(x0 + cx)] = v;
        }
        cx += dc;
        r += dr;
        if (cx >= iw) {
          cx -= iw;
          ++r;
        }
      }
    }
    __syncthreads();  // LDS is restaged next; acc_lds is complete
    // Accepted counts: one device atomic per run of items of one chain.
    const int next_chain = more ? Gn.chain_base + gn.chain : -1;
    if (threadIdx.x == 0 && (!more || next_chain != gchain)) {
      if (acc_lds) atomicAdd(&A.counts[(int64_t)gchain * kMaxPass], acc_lds);
      acc_lds = 0u;
    }
    if (!more) return false;
    item = next;
    next = next2;
    G = Gn;
    Gn = Gx;
    return true;
  };
  while (step(kA, kB) && step(kB, kA)) {
  }
}

// ------------------------------------------------------------------- plan
// One workgroup per (grid, tile): list the pairs of same-colour sites
// (y, y + 2) of a column, y mod 4 in {0, 1}, that hold a gap site within
// Manhattan distance dmax of the tile's interior, colour 0 first, each
// colour sorted by the pair's distance (the least over its gap sites within
// dmax) and, within one distance, in the row-major order of the pair's
// first such site (a counting sort that keeps the scan order), so that
// neighbouring lanes of the sweep update neighbouring sites.  The plan is
// the same on every run.
template <typename P>
__global__ void __launch_bounds__(kThreads)
    k_plan(const GridDesc *grids, int n_grids, int64_t n_tiles, const P *state, int tile_x, int tile_y, int dmax,
           uint16_t *plan, uint32_t *plan_cum) {
  constexpr int kBuckets = 2 * (2 * kMaxPass + 2);  // (colour, ring) pairs, ring <= 2 * kMaxPass + 1
  constexpr int kWaves = kThreads / 64;
  __shared__ uint32_t cnt[kBuckets];
  __shared__ uint32_t cur[kBuckets];
  __shared__ uint32_t wcnt[kWaves][kBuckets];
  const int64_t item = block_index();
  if (item >= n_tiles) return;
  const int gi = find_by(grids, n_grids, item, &GridDesc::plan_begin);
  const GridDesc G = grids[gi];
  const int t = (int)(item - G.plan_begin);
  const int nx = G.nx, ny = G.ny;
  const int x0 = (t % G.tiles_x) * tile_x, y0 = (t / G.tiles_x) * tile_y;
  const int ix1 = min(x0 + tile_x, nx), iy1 = min(y0 + tile_y, ny);
  const int rx0 = max(x0 - dmax, 0), rx1 = min(ix1 + dmax, nx);
  const int ry0 = max(y0 - dmax, 0), ry1 = min(iy1 + dmax, ny);
  const int rw = rx1 - rx0, n = rw * (ry1 - ry0);
  const float inv = 1.0f / (float)rw;
  const int nb = 2 * (dmax + 2);
  const P *st = state + G.state_off;  // chain 0: the sample sites are those of every chain
  // A site of the scanned rectangle that the plan covers: a gap site
  // within distance dmax (its distance in ring).
  auto covered = [&](int gx, int gy, int &ring) {
    if (gx < rx0 || gx >= rx1 || gy < ry0 || gy >= ry1) return false;
    if (signbit(st[(int64_t)gy * nx + gx])) return false;
    ring = max(max(x0 - gx, gx - (ix1 - 1)), 0) + max(max(y0 - gy, gy - (iy1 - 1)), 0);
    return ring <= dmax;
  };
  // Bucket of scanned site f: colour * (dmax + 2) + the pair's ring if f is
  // the first covered site of its pair, else -1.
  auto bucket = [&](int f, uint16_t &entry) {
    int r, cx;
    split_index(f, rw, inv, r, cx);
    const int gx = rx0 + cx, gy = ry0 + r;
    int ring, other;
    if (!covered(gx, gy, ring)) return -1;
    const int b = gy & ~2;  // the row of the pair's first site
    if (gy != b) {
      if (covered(gx, b, other)) return -1;  // listed from the first site
    } else if (covered(gx, b + 2, other)) {
      ring = min(ring, other);
    }
    entry = (uint16_t)(((b - y0 + kPlanOffset) << 8) | (gx - x0 + kPlanOffset));
    return ((gx + gy) & 1) * (dmax + 2) + ring;
  };
  for (int i = threadIdx.x; i < kBuckets; i += kThreads) {
    cnt[i] = 0u;
    for (int w = 0; w < kWaves; ++w) wcnt[w][i] = 0u;
  }
  __syncthreads();
  for (int f = threadIdx.x; f < n; f += kThreads) {
    uint16_t e;
    const int b = bucket(f, e);
    if (b >= 0) atomicAdd(&cnt[b], 1u);
  }
  __syncthreads();
  uint32_t *cum = plan_cum + item * 2 * (dmax + 2);
  if (threadIdx.x == 0) {
    uint32_t base = 0;
    for (int c = 0; c < 2; ++c) {
      uint32_t acc = 0;
      for (int r = 0; r <= dmax + 1; ++r) {
        cum[c * (dmax + 2) + r] = acc;
        cur[c * (dmax + 2) + r] = base + acc;
        if (r <= dmax) acc += cnt[c * (dmax + 2) + r];
      }
      base += acc;
    }
  }
  __syncthreads();
  // Placement in scan order: per chunk of kThreads sites, a site's slot is
  // its bucket's running start, plus the bucket's sites in earlier waves of
  // the chunk, plus those in earlier lanes of its own wave (by ballot).
  uint16_t *out = plan + G.plan_ebase + (int64_t)t * G.plan_cap;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int base = 0; base < n; base += kThreads) {
    const int f = base + (int)threadIdx.x;
    uint16_t e = 0;
    const int b = f < n ? bucket(f, e) : -1;
    int rank = 0;
    uint64_t todo = __ballot(b >= 0);
    while (todo) {
      const int lead = __ffsll((unsigned long long)todo) - 1;
      const int bl = __shfl(b, lead, 64);
      const uint64_t m = __ballot(b == bl);
      if (b == bl) rank = __popcll(m & below);
      if (lane == 0) wcnt[wv][bl] = (uint32_t)__popcll(m);
      todo &= ~m;
    }
    __syncthreads();
    if (b >= 0) {
      uint32_t pos = cur[b] + (uint32_t)rank;
      for (int w = 0; w < wv; ++w) pos += wcnt[w][b];
      out[pos] = e;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kThreads) {
      uint32_t add = 0;
      for (int w = 0; w < kWaves; ++w) {
        add += wcnt[w][i];
        wcnt[w][i] = 0u;
      }
      cur[i] += add;
    }
    __syncthreads();
  }
}

template <typename P>
hipError_t launch_plan(const GridDesc *g, int n_grids, int64_t n_tiles, const P *state, int tile_x, int tile_y,
                       int dmax, uint16_t *plan, uint32_t *plan_cum, hipStream_t s) {
  hipLaunchKernelGGL(k_plan<P>, block_grid(n_tiles, kThreads), dim3(kThreads), 0, s, g, n_grids, n_tiles, state, tile_x,
                     tile_y, dmax, plan, plan_cum);
  return hipGetLastError();
}
template hipError_t launch_plan<float>(const GridDesc *, int, int64_t, const float *, int, int, int, uint16_t *,
                                       uint32_t *, hipStream_t);
template hipError_t launch_plan<double>(const GridDesc *, int, int64_t, const double *, int, int, int, uint16_t *,
                                        uint32_t *, hipStream_t);

// One thread per chain: close the last pass of a run.
template <typename P>
__global__ void k_pass_end(const SweepArgs<P> A) {
  const int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= A.total_chains) return;
  int lo = 0, hi = A.n_grids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.grids[mid].chain_base <= ch) lo = mid;
    else hi = mid - 1;
  }
  apply_pass_end(A, A.grids[lo], ch, true);
}

// One workgroup per chain: for each sweep s of the pass, the energies of
// the chain's items (tiles) summed by thread-strided partial sums and a
// fixed-order workgroup sum.
__global__ void __launch_bounds__(kThreads)
    k_energy_reduce(const GridDesc *grids, int n_grids, int total_chains, int64_t n_items, int nsw,
                    const double *part, double *energy) {
  __shared__ double red[kThreads / 64];
  const int64_t ch = block_index();
  if (ch >= total_chains) return;
  int lo = 0, hi = n_grids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (grids[mid].chain_base <= ch) lo = mid;
    else hi = mid - 1;
  }
  const GridDesc &G = grids[lo];
  const int tiles = G.tiles_x * G.tiles_y;
  const int64_t i0 = G.item_begin + (ch - G.chain_base) * (int64_t)tiles;
  for (int s = 0; s < nsw; ++s) {
    double acc = 0.0;
    for (int t = threadIdx.x; t < tiles; t += kThreads) acc += part[(int64_t)s * n_items + i0 + t];
    const double tot = block_sum<kThreads>(acc, red);
    if (threadIdx.x == 0) energy[ch * kMaxPass + s] = tot;
  }
}

hipError_t launch_energy_reduce(const GridDesc *g, int n_grids, int total_chains, int64_t n_items, int nsw,
                                const double *part, double *energy, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_reduce, block_grid(total_chains, kThreads), dim3(kThreads), 0, s, g, n_grids,
                     total_chains, n_items, nsw, part, energy);
  return hipGetLastError();
}

template <typename P, int MODEL, bool REP, bool RREG>
static void launch_sweep_q(const SweepArgs<P> &a, int threads, int64_t n_items, size_t lds, hipStream_t s) {
  const dim3 grid = block_grid((n_items + 7) / 8 * 8, threads);  // xcd_item's workgroups
  switch (threads) {
    case 64: hipLaunchKernelGGL((k_sweep<P, 64, MODEL, REP, RREG>), grid, dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((k_sweep<P, 128, MODEL, REP, RREG>), grid, dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((k_sweep<P, 256, MODEL, REP, RREG>), grid, dim3(256), lds, s, a); break;
    case 512: hipLaunchKernelGGL((k_sweep<P, 512, MODEL, REP, RREG>), grid, dim3(512), lds, s, a); break;
    default: hipLaunchKernelGGL((k_sweep<P, 1024, MODEL, REP, RREG>), grid, dim3(1024), lds, s, a); break;
  }
}

template <typename P, bool REP, bool RREG = false>
static void launch_sweep_m(const SweepArgs<P> &a, int threads, int64_t n_items, size_t lds, hipStream_t s) {
  if (a.gmrf) launch_sweep_q<P, kGmrf, REP, RREG>(a, threads, n_items, lds, s);
  else if (a.q_is_one) launch_sweep_q<P, kMprQ1, REP, RREG>(a, threads, n_items, lds, s);
  else launch_sweep_q<P, kMprQ, REP, RREG>(a, threads, n_items, lds, s);
}

template <int MODEL, bool REP>
static void launch_redo_q(const SweepArgs<float> &a, int threads, int blocks, size_t lds, hipStream_t s) {
  switch (threads) {
    case 64: hipLaunchKernelGGL((k_sweep_redo<float, 64, MODEL, REP>), dim3(blocks), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((k_sweep_redo<float, 128, MODEL, REP>), dim3(blocks), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((k_sweep_redo<float, 256, MODEL, REP>), dim3(blocks), dim3(256), lds, s, a); break;
    case 512: hipLaunchKernelGGL((k_sweep_redo<float, 512, MODEL, REP>), dim3(blocks), dim3(512), lds, s, a); break;
    default: hipLaunchKernelGGL((k_sweep_redo<float, 1024, MODEL, REP>), dim3(blocks), dim3(1024), lds, s, a); break;
  }
}
template <bool REP>
static void launch_redo_m(const SweepArgs<float> &a, int threads, int blocks, size_t lds, hipStream_t s) {
  if (a.gmrf) launch_redo_q<kGmrf, REP>(a, threads, blocks, lds, s);
  else if (a.q_is_one) launch_redo_q<kMprQ1, REP>(a, threads, blocks, lds, s);
  else launch_redo_q<kMprQ, REP>(a, threads, blocks, lds, s);
}

template <typename P>
hipError_t launch_sweep(const SweepArgs<P> &a, int threads, int64_t n_items, size_t lds, hipStream_t s) {
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
    return hipErrorInvalidValue;
  // FP32 passes recording two or more sweeps keep their fill sums in registers.
  bool rreg = false;
  if constexpr (sizeof(P) == 4) rreg = !a.rep && __builtin_popcount(a.record_mask) >= 2;
  if (a.rep) launch_sweep_m<P, true>(a, threads, n_items, lds, s);
  else if (rreg) {
    if constexpr (sizeof(P) == 4) launch_sweep_m<P, false, true>(a, threads, n_items, lds, s);
  } else {
    launch_sweep_m<P, false>(a, threads, n_items, lds, s);
  }
  return hipGetLastError();
}

hipError_t launch_sweep_redo(const SweepArgs<float> &a, int threads, int blocks, size_t lds, hipStream_t s) {
  if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
    return hipErrorInvalidValue;
  if (!a.spec || !a.redo || a.record_mask || blocks < 1) return hipErrorInvalidValue;
  if (a.rep) launch_redo_m<true>(a, threads, blocks, lds, s);
  else launch_redo_m<false>(a, threads, blocks, lds, s);
  return hipGetLastError();
}

// One thread per chain, after a speculative pass: sweep 0's a-rule outcome
// (Algorithm 2, step 4.2, with the window the pass started with) against
// the prediction the pass ran sweep 1 with.
__global__ void __launch_bounds__(kThreads)
    k_spec_check(const GridDesc *grids, int n_grids, int total_chains, uint32_t *counts, const double *win_in,
                 int adapt_every, double a_targ, const uint32_t *pred, uint32_t *redo) {
  // redo[0]: number of listed chains (cleared by the pass), redo[1 ..]: the chains
  const int64_t ch = block_index() * kThreads + threadIdx.x;
  if (ch >= total_chains) return;
  int lo = 0, hi = n_grids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (grids[mid].chain_base <= ch) lo = mid;
    else hi = mid - 1;
  }
  const GridDesc &G = grids[lo];
  uint32_t *k = counts + ch * kMaxPass;
  const double acc = G.n_gap > 0 ? (double)k[0] / (double)G.n_gap : 1.0;
  const double win = win_in[ch] + acc;
  const int low = win / (double)adapt_every < a_targ ? 1 : 0;
  if (low != (int)pred[ch]) {
    k[0] = 0u;
    k[1] = 0u;
    redo[1 + atomicAdd(&redo[0], 1u)] = (uint32_t)ch;
  }
}

hipError_t launch_spec_check(const GridDesc *g, int n_grids, int total_chains, uint32_t *counts, const double *win_in,
                             int adapt_every, double a_targ, const uint32_t *pred, uint32_t *redo, hipStream_t s) {
  hipLaunchKernelGGL(k_spec_check, block_grid((total_chains + kThreads - 1) / kThreads, kThreads), dim3(kThreads), 0,
                     s, g, n_grids, total_chains, counts, win_in, adapt_every, a_targ, pred, redo);
  return hipGetLastError();
}

// Persistent single-sweep workgroups of 256 and 1024 threads (the kernel's
// register budget holds a 64 x 64 tile's staging at 1024 threads without
// spilling; at 512 it does not).  Other sizes use one workgroup per item.
template <typename P, int MODEL, bool REP>
static const void *sweep1_fn(int threads) {
  switch (threads) {
    case 256: return reinterpret_cast<const void *>(&k_sweep1<P, 256, MODEL, REP>);
    case 1024: return reinterpret_cast<const void *>(&k_sweep1<P, 1024, MODEL, REP>);
    default: return nullptr;
  }
}
template <typename P> static const void *sweep1_fn(int threads, int model, bool rep) {
  if (rep) {
    if (model == kGmrf) return sweep1_fn<P, kGmrf, true>(threads);
    if (model == kMprQ1) return sweep1_fn<P, kMprQ1, true>(threads);
    return sweep1_fn<P, kMprQ, true>(threads);
  }
  if (model == kGmrf) return sweep1_fn<P, kGmrf, false>(threads);
  if (model == kMprQ1) return sweep1_fn<P, kMprQ1, false>(threads);
  return sweep1_fn<P, kMprQ, false>(threads);
}

template <typename P>
hipError_t launch_sweep1(const SweepArgs<P> &a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
  const int model = a.gmrf ? kGmrf : (a.q_is_one ? kMprQ1 : kMprQ);
  const void *fn = sweep1_fn<P>(threads, model, a.rep != 0);
  if (!fn || blocks < 8 || blocks % 8 != 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  void *args[] = {const_cast<SweepArgs<P> *>(&a)};
  return hipLaunchKernel(fn, dim3((unsigned)blocks), dim3((unsigned)threads), args, lds, s);
}
template hipError_t launch_sweep1<float>(const SweepArgs<float> &, int, int64_t, size_t, hipStream_t);
template hipError_t launch_sweep1<double>(const SweepArgs<double> &, int, int64_t, size_t, hipStream_t);

// Workgroups per CU: the least of what the CU's LDS, its thread slots and
// the kernel's registers allow (the occupancy query's own figure, or the
// LDS bound where the query assumes less LDS per CU than gfx950 has).
template <typename P> int64_t sweep1_resident(int threads, int model, bool rep, size_t lds) {
  const void *fn = sweep1_fn<P>(threads, model, rep);
  if (!fn) return 0;
  int per_cu = 0, dev = 0, cus = 0, lds_cu = 0, lds_blk = 0, thr_cu = 0, regs = 0;
  hipFuncAttributes at{};
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_blk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      hipDeviceGetAttribute(&thr_cu, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&regs, hipDeviceAttributeMaxRegistersPerMultiprocessor, dev) != hipSuccess ||
      hipFuncGetAttributes(&at, fn) != hipSuccess)
    return 0;
  const size_t lds_all = lds + at.sharedSizeBytes;
  int64_t n = std::max<int64_t>(lds_cu, lds_blk) / std::max<size_t>(lds_all, 1);
  n = std::min<int64_t>(n, thr_cu / threads);
  if (at.numRegs > 0 && regs > 0) n = std::min<int64_t>(n, regs / ((int64_t)at.numRegs * threads));
  n = std::max<int64_t>(n, per_cu);
  n = std::max<int64_t>(n, 1) * cus;
  return n / 8 * 8;
}
template int64_t sweep1_resident<float>(int, int, bool, size_t);
template int64_t sweep1_resident<double>(int, int, bool, size_t);

template <typename P> int sweep_max_threads(int threads) {
  hipFuncAttributes at{};
  hipError_t e = hipErrorInvalidValue;
  switch (threads) {
    case 64: e = hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_sweep<P, 64, kMprQ, false, false>)); break;
    case 128: e = hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_sweep<P, 128, kMprQ, false, false>)); break;
    case 256: e = hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_sweep<P, 256, kMprQ, false, false>)); break;
    case 512: e = hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_sweep<P, 512, kMprQ, false, false>)); break;
    case 1024: e = hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_sweep<P, 1024, kMprQ, false, false>)); break;
    default: break;
  }
  return e == hipSuccess ? at.maxThreadsPerBlock : 0;
}
template int sweep_max_threads<float>(int);
template int sweep_max_threads<double>(int);

template <typename P> hipError_t launch_pass_end(const SweepArgs<P> &a, hipStream_t s) {
  hipLaunchKernelGGL(k_pass_end<P>, dim3((a.total_chains + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_pass_end<float>(const SweepArgs<float> &, hipStream_t);
template hipError_t launch_pass_end<double>(const SweepArgs<double> &, hipStream_t);
template hipError_t launch_sweep<float>(const SweepArgs<float> &, int, int64_t, size_t, hipStream_t);
template hipError_t launch_sweep<double>(const SweepArgs<double> &, int, int64_t, size_t, hipStream_t);

// ------------------------------------------------------ min / max of samples
// Eq. (2) needs z_min, z_max over the samples of each grid.  Stage 1: one
// workgroup per chunk of kChunk sites -> (min, max, #samples, #non-finite).
__global__ void __launch_bounds__(kThreads)
    k_minmax(const GridDesc *grids, int n_grids, int64_t n_blocks, const double *const *zp, const uint8_t *const *kp,
             double *part) {
  __shared__ double smin[kThreads], smax[kThreads], scnt[kThreads], sbad[kThreads];
  const int64_t b = block_index();
  if (b >= n_blocks) return;
  const int gi = find_by(grids, n_grids, b, &GridDesc::sb_begin);
  const GridDesc &G = grids[gi];
  const int64_t n = (int64_t)G.nx * G.ny;
  const int64_t base = (b - G.sb_begin) * kChunk;
  const double *z = zp[gi];
  const uint8_t *kn = kp[gi];
  double mn = INFINITY, mx = -INFINITY, cnt = 0, bad = 0;
  for (int64_t i = base + threadIdx.x; i < min(base + kChunk, n); i += kThreads) {
    if (kn[i]) {
      const double v = z[i];
      cnt += 1;
      if (!isfinite(v)) bad += 1;
      else {
        mn = fmin(mn, v);
        mx = fmax(mx, v);
      }
    }
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  scnt[threadIdx.x] = cnt;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      scnt[threadIdx.x] += scnt[threadIdx.x + o];
      sbad[threadIdx.x] += sbad[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[b * 4 + 0] = smin[0];
    part[b * 4 + 1] = smax[0];
    part[b * 4 + 2] = scnt[0];
    part[b * 4 + 3] = sbad[0];
  }
}

// Stage 2: one workgroup per grid, partials in fixed order -> out[g*4 + ...].
__global__ void __launch_bounds__(kThreads)
    k_minmax_final(const GridDesc *grids, int n_grids, const double *part, double *out) {
  __shared__ double smin[kThreads], smax[kThreads], scnt[kThreads], sbad[kThreads];
  const int64_t gi = block_index();
  if (gi >= n_grids) return;
  const GridDesc &G = grids[gi];
  const int64_t nb = (gi + 1 < n_grids ? grids[gi + 1].sb_begin : G.sb_begin + ((int64_t)G.nx * G.ny + kChunk - 1) / kChunk) - G.sb_begin;
  double mn = INFINITY, mx = -INFINITY, cnt = 0, bad = 0;
  for (int64_t i = threadIdx.x; i < nb; i += kThreads) {
    const double *p = part + (G.sb_begin + i) * 4;
    mn = fmin(mn, p[0]);
    mx = fmax(mx, p[1]);
    cnt += p[2];
    bad += p[3];
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  scnt[threadIdx.x] = cnt;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      scnt[threadIdx.x] += scnt[threadIdx.x + o];
      sbad[threadIdx.x] += sbad[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[gi * 4 + 0] = smin[0];
    out[gi * 4 + 1] = smax[0];
    out[gi * 4 + 2] = scnt[0];
    out[gi * 4 + 3] = sbad[0];
  }
}

hipError_t launch_minmax(const GridDesc *g, int n_grids, int64_t n_blocks, const double *const *z,
                         const uint8_t *const *known, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax, block_grid(n_blocks, kThreads), dim3(kThreads), 0, s, g, n_grids, n_blocks, z, known,
                     part);
  return hipGetLastError();
}
hipError_t launch_minmax_final(const GridDesc *g, int n_grids, const double *part, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_minmax_final, block_grid(n_grids, kThreads), dim3(kThreads), 0, s, g, n_grids, part, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ init
// Eq. (2) at the samples, hot start 2*pi*U at the gaps (Algorithm 2, steps
// 1.8 and 2.1), written to both state buffers.  One workgroup per chunk of
// one chain.  The hot start draws the u word of sweep 0xFFFFFFFF.
template <typename P>
__global__ void __launch_bounds__(kThreads)
    k_init(const GridDesc *grids, int n_grids, int64_t n_blocks, const double *const *zp, const uint8_t *const *kp,
           P *s0, P *s1, uint32_t k0, uint32_t k1) {
  const int64_t b = block_index();
  if (b >= n_blocks) return;
  const int gi = find_by(grids, n_grids, b, &GridDesc::cb_begin);
  const GridDesc &G = grids[gi];
  const int64_t n = (int64_t)G.nx * G.ny;
  const int64_t per_chain = (n + kChunk - 1) / kChunk;
  const int64_t lb = b - G.cb_begin;
  const int chain = (int)(lb / per_chain);
  const int64_t base = (lb - (int64_t)chain * per_chain) * kChunk;
  const double *z = zp[gi];
  const uint8_t *kn = kp[gi];
  const double zmin = G.zmin, span = G.zmax - G.zmin;
  for (int64_t i = base + threadIdx.x; i < min(base + kChunk, n); i += kThreads) {
    P v;
    if (kn[i]) {
      v = -(P)((z[i] - zmin) / span * 6.28318530717958647692);
    } else {
      // the site's counter with word 0xFFFFFFFF (the sweep word never reaches it); word w0
      uint32_t w[4];
      philox4x32_10((uint32_t)i, 0xFFFFFFFFu, (uint32_t)chain, (uint32_t)G.grid_id, k0, k1, w);
      // Float angles are rounded to the nearest float; keep gaps below 2*pi.
      v = (P)(6.28318530717958647692 * unit<double>(w[0]));
      if (v >= Prec<P>::two_pi) v = Prec<P>::below_two_pi;
    }
    const int64_t k = G.state_off + (int64_t)chain * n + i;
    s0[k] = v;
    s1[k] = v;
  }
}

template <typename P>
hipError_t launch_init(const GridDesc *g, int n_grids, int64_t n_blocks, const double *const *z,
                       const uint8_t *const *known, P *s0, P *s1, P, uint32_t k0, uint32_t k1, hipStream_t s) {
  hipLaunchKernelGGL(k_init<P>, block_grid(n_blocks, kThreads), dim3(kThreads), 0, s, g, n_grids, n_blocks, z, known, s0,
                     s1, k0, k1);
  return hipGetLastError();
}
template hipError_t launch_init<float>(const GridDesc *, int, int64_t, const double *const *, const uint8_t *const *,
                                       float *, float *, float, uint32_t, uint32_t, hipStream_t);
template hipError_t launch_init<double>(const GridDesc *, int, int64_t, const double *const *,
                                        const uint8_t *const *, double *, double *, double, uint32_t, uint32_t,
                                        hipStream_t);

// --------------------------------------------------------------- energies
// what = 0: Eq. (4) per grid over sample-sample pairs of chain 0;
// what = 1: Eq. (5) per chain over all pairs.  Each site owns its right and
// lower pair; terms 2 sin^2(q dphi / 2) are summed per thread in P and per
// workgroup in FP64 -> part[b*2] = sum, part[b*2+1] = #pairs.
// 1 - H_ij of one pair with angle difference d: 2 sin^2(q d / 2) for MPR,
// d^2 / (2 pi^2) for the GMRF variant.
template <typename P> __device__ __forceinline__ P pair_eps(P d, P q, int gmrf) {
  if (gmrf) return d * d * Prec<P>::inv_2pi2;
  const P sn = Prec<P>::sin_(q * d * P(0.5));
  return P(2) * sn * sn;
}

template <typename P>
__global__ void __launch_bounds__(kThreads)
    k_energy(const GridDesc *grids, int n_grids, int64_t n_blocks, int what, const P *state, int gmrf, double *part) {
  __shared__ double red[kThreads / 64];
  const int64_t b = block_index();
  if (b >= n_blocks) return;
  const int gi = find_by(grids, n_grids, b, what ? &GridDesc::cb_begin : &GridDesc::sb_begin);
  const GridDesc &G = grids[gi];
  const P q = (P)G.q;
  const int nx = G.nx;
  const int64_t n = (int64_t)nx * G.ny;
  const int64_t per_chain = (n + kChunk - 1) / kChunk;
  const int64_t lb = b - (what ? G.cb_begin : G.sb_begin);
  const int chain = what ? (int)(lb / per_chain) : 0;
  const int64_t base = (lb - (int64_t)chain * per_chain) * kChunk;
  const P *st = state + G.state_off + (int64_t)chain * n;
  P e = P(0);
  double cnt = 0.0;
  for (int64_t i = base + threadIdx.x; i < min(base + kChunk, n); i += kThreads) {
    const int y = (int)(i / nx), x = (int)(i - (int64_t)y * nx);
    const P v = st[i];
    if (what == 0 && !signbit(v)) continue;
    if (x + 1 < nx) {
      const P w = st[i + 1];
      if (what == 1 || signbit(w)) {
        e += pair_eps(fabs(v) - fabs(w), q, gmrf);
        cnt += 1.0;
      }
    }
    if (y + 1 < G.ny) {
      const P w = st[i + nx];
      if (what == 1 || signbit(w)) {
        e += pair_eps(fabs(v) - fabs(w), q, gmrf);
        cnt += 1.0;
      }
    }
  }
  const double se = block_sum<kThreads>((double)e, red);
  const double sc = block_sum<kThreads>(cnt, red);
  if (threadIdx.x == 0) {
    part[b * 2] = se;
    part[b * 2 + 1] = sc;
  }
}

// One workgroup per unit (grid or chain): fixed-order sum of its partials.
__global__ void __launch_bounds__(kThreads)
    k_energy_final(const GridDesc *grids, int n_grids, int what, int n_units, const double *part, double *out) {
  __shared__ double red[kThreads / 64];
  const int unit = (int)block_index();
  if (unit >= n_units) return;
  int gi = 0, chain = 0;
  if (what) {
    int lo = 0, hi = n_grids - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (grids[mid].chain_base <= unit) lo = mid;
      else hi = mid - 1;
    }
    gi = lo;
    chain = unit - grids[gi].chain_base;
  } else {
    gi = unit;
  }
  const GridDesc &G = grids[gi];
  const int64_t per_chain = ((int64_t)G.nx * G.ny + kChunk - 1) / kChunk;
  const int64_t b0 = (what ? G.cb_begin + chain * per_chain : G.sb_begin);
  double e = 0.0, c = 0.0;
  for (int64_t i = threadIdx.x; i < per_chain; i += kThreads) {
    e += part[(b0 + i) * 2];
    c += part[(b0 + i) * 2 + 1];
  }
  const double se = block_sum<kThreads>(e, red);
  const double sc = block_sum<kThreads>(c, red);
  if (threadIdx.x == 0) {
    out[unit * 2] = se;
    out[unit * 2 + 1] = sc;
  }
}

template <typename P>
hipError_t launch_energy(const GridDesc *g, int n_grids, int64_t n_blocks, int what, const P *state, int gmrf,
                         double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_energy<P>, block_grid(n_blocks, kThreads), dim3(kThreads), 0, s, g, n_grids, n_blocks, what, state,
                     gmrf, part);
  return hipGetLastError();
}
template hipError_t launch_energy<float>(const GridDesc *, int, int64_t, int, const float *, int, double *,
                                         hipStream_t);
template hipError_t launch_energy<double>(const GridDesc *, int, int64_t, int, const double *, int, double *,
                                          hipStream_t);
hipError_t launch_energy_final(const GridDesc *g, int n_grids, int what, int n_units, const double *part,
                               double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_final, block_grid(n_units, kThreads), dim3(kThreads), 0, s, g, n_grids, what, n_units, part,
                     out);
  return hipGetLastError();
}

// ---------------------------------------------------- validation measures
// Sums over the gap sites of one chunk of a grid (Sec. 3.3): count, |eps|,
// eps / Z, |eps| / Z, eps^2 with eps = Z - Z_hat, and the first and second
// moments of Z - shift and Z_hat - shift for the correlation coefficient.
__global__ void __launch_bounds__(kThreads)
    k_measures(const double *z, const double *zh, const uint8_t *known, int64_t n, double shift, double *part) {
  __shared__ double red[kThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double s[kMeasureSums] = {};
  for (int64_t i = base + threadIdx.x; i < min(base + (int64_t)kChunk, n); i += kThreads) {
    if (known[i] || __builtin_isnan(z[i])) continue;  // a NaN in z_true leaves the site out
    const double zt = z[i], zp = zh[i], e = zt - zp, a = zt - shift, b = zp - shift;
    s[0] += 1.0;
    s[1] += fabs(e);
    s[2] += e / zt;
    s[3] += fabs(e) / zt;
    s[4] += e * e;
    s[5] += a;
    s[6] += b;
    s[7] += a * a;
    s[8] += b * b;
    s[9] += a * b;
  }
  for (int k = 0; k < kMeasureSums; ++k) {
    const double v = block_sum<kThreads>(s[k], red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * kMeasureSums + k] = v;
  }
}

// One workgroup: the chunk sums in a fixed order, then AAE, ARE, AARE, RASE,
// R, P and the means of Z and Z_hat into out[0..7].
__global__ void __launch_bounds__(kThreads) k_measures_final(const double *part, int64_t n_blocks, double shift,
                                                             double *out) {
  __shared__ double red[kThreads / 64];
  __shared__ double tot[kMeasureSums];
  for (int k = 0; k < kMeasureSums; ++k) {
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < n_blocks; j += kThreads) acc += part[j * kMeasureSums + k];
    const double v = block_sum<kThreads>(acc, red);
    if (threadIdx.x == 0) tot[k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double P = tot[0];
    const double ma = tot[5] / P, mb = tot[6] / P;
    const double saa = tot[7] - P * ma * ma, sbb = tot[8] - P * mb * mb, sab = tot[9] - P * ma * mb;
    out[0] = tot[1] / P;
    out[1] = tot[2] / P;
    out[2] = tot[3] / P;
    out[3] = sqrt(tot[4] / P);
    out[4] = sab / sqrt(saa * sbb);
    out[5] = P;
    out[6] = ma + shift;
    out[7] = mb + shift;
  }
}

hipError_t launch_measures(const double *z, const double *zh, const uint8_t *known, int64_t n, double shift,
                           double *part, double *out, hipStream_t s) {
  const int64_t blocks = (n + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_measures, dim3((unsigned)blocks), dim3(kThreads), 0, s, z, zh, known, n, shift, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_measures_final, dim3(1), dim3(kThreads), 0, s, part, blocks, shift, out);
  return hipGetLastError();
}

// -------------------------------------------------------------- finalize
// Per site of each grid: pool the chains' recorded states (mean and
// variance about each chain's first record), then map back with the
// inverse of Eq. (2).  Samples: z and 0.  One pass over the chains: each
// chain's mean m_c and variance v_c go into sums of (m_c - K) and
// v_c + (m_c - K)^2, K the first chain's mean, so that the pooled variance
// (1/C) sum_c (v_c + (m_c - K)^2) - (mean - K)^2 subtracts no large terms.
template <typename P>
__global__ void __launch_bounds__(kThreads)
    k_finalize(const GridDesc *grids, int n_grids, const double *const *zp, const P *state, const P *ref, const P *s1,
               const P *s2, int32_t records, int64_t n_blocks, double *zhat, double *zstd) {
  const int64_t b = block_index();
  if (b >= n_blocks) return;
  const int gi = find_by(grids, n_grids, b, &GridDesc::sb_begin);
  const GridDesc &G = grids[gi];
  const int64_t n = (int64_t)G.nx * G.ny;
  const int64_t base = (b - G.sb_begin) * kChunk;
  const double *z = zp[gi];
  const double inv_m = 1.0 / (double)records, C = (double)G.chains;
  for (int64_t i = base + threadIdx.x; i < min(base + kChunk, n); i += kThreads) {
    const int64_t o = G.site_off + i;
    if (signbit(state[G.state_off + i])) {
      zhat[o] = z[i];
      if (zstd) zstd[o] = 0.0;
      continue;
    }
    double K = 0.0, sd = 0.0, sq = 0.0;
    for (int c = 0; c < G.chains; ++c) {
      const int64_t k = G.state_off + (int64_t)c * n + i;
      const double m1 = (double)s1[k] * inv_m;
      const double mc = (double)ref[k] + m1;
      const double vc = fmax((double)s2[k] * inv_m - m1 * m1, 0.0);
      if (c == 0) K = mc;
      const double d = mc - K;
      sd += d;
      sq += vc + d * d;
    }
    const double dm = sd / C;
    const double mean = K + dm;
    const double var = fmax(sq / C - dm * dm, 0.0);
    const double span = G.zmax - G.zmin;
    zhat[o] = G.zmin + span * (mean / 6.28318530717958647692);
    if (zstd) zstd[o] = span / 6.28318530717958647692 * sqrt(var);
  }
}

template <typename P>
hipError_t launch_finalize(const GridDesc *g, int n_grids, int64_t n_blocks, const double *const *z, const P *state,
                           const P *ref, const P *s1, const P *s2, int32_t records, double *zhat, double *zstd,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalize<P>, block_grid(n_blocks, kThreads), dim3(kThreads), 0, s, g, n_grids, z, state, ref, s1,
                     s2, records, n_blocks, zhat, zstd);
  return hipGetLastError();
}
template hipError_t launch_finalize<float>(const GridDesc *, int, int64_t, const double *const *, const float *,
                                           const float *, const float *, const float *, int32_t, double *, double *,
                                           hipStream_t);
template hipError_t launch_finalize<double>(const GridDesc *, int, int64_t, const double *const *, const double *,
                                            const double *, const double *, const double *, int32_t, double *,
                                            double *, hipStream_t);

// ------------------------------------------------------------ state copies
template <typename P> __global__ void k_get_phi(const P *st, int64_t n, double *out) {
  const int64_t i = block_index() * blockDim.x + threadIdx.x;
  if (i < n) out[i] = fabs((double)st[i]);
}
template <typename P> __global__ void k_set_phi(P *s0, P *s1, int64_t n, const double *in) {
  const int64_t i = block_index() * blockDim.x + threadIdx.x;
  if (i >= n || signbit(s0[i])) return;  // sample sites keep their angle
  P v = (P)in[i];
  v = (v > P(0)) ? v : P(0);  // also turns -0 into +0
  if (v >= Prec<P>::two_pi) v = Prec<P>::below_two_pi;
  s0[i] = v;
  s1[i] = v;
}
template <typename P> hipError_t launch_get_phi(const P *st, int64_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_get_phi<P>, block_grid((n + kThreads - 1) / kThreads, kThreads), dim3(kThreads), 0, s, st, n, out);
  return hipGetLastError();
}
template <typename P> hipError_t launch_set_phi(P *s0, P *s1, int64_t n, const double *in, hipStream_t s) {
  hipLaunchKernelGGL(k_set_phi<P>, block_grid((n + kThreads - 1) / kThreads, kThreads), dim3(kThreads), 0, s, s0, s1, n,
                     in);
  return hipGetLastError();
}
template hipError_t launch_get_phi<float>(const float *, int64_t, double *, hipStream_t);
template hipError_t launch_get_phi<double>(const double *, int64_t, double *, hipStream_t);
template hipError_t launch_set_phi<float>(float *, float *, int64_t, const double *, hipStream_t);
template hipError_t launch_set_phi<double>(double *, double *, int64_t, const double *, hipStream_t);

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  const int64_t i = block_index() * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_zero_u32(uint32_t *p, int64_t n) {
  const int64_t i = block_index() * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, block_grid((n + kThreads - 1) / kThreads, kThreads), dim3(kThreads), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, block_grid((n + kThreads - 1) / kThreads, kThreads), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}
__global__ void k_copy_f64(double *dst, const double *src, int64_t n) {
  const int64_t i = block_index() * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
hipError_t launch_copy_f64(double *dst, const double *src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f64, block_grid((n + kThreads - 1) / kThreads, kThreads), dim3(kThreads), 0, s, dst, src, n);
  return hipGetLastError();
}

// --------------------------------------------------- cross-validation folds
// Per site and fold k: the training mask (a sample whose fold id is not k)
// and the scoring field (z at the samples of fold k, NaN elsewhere, so that
// the validation measures see only the held-out samples).
__global__ void k_cv_prepare(const double *z, const uint8_t *known, const uint8_t *fold, int n_folds, int64_t n,
                             uint8_t *masks, double *zt) {
  const int64_t i = block_index() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool smp = known[i] != 0;
  const int f = fold[i];
  const double v = z[i];
  for (int k = 0; k < n_folds; ++k) {
    const bool held = smp && f == k;
    masks[(int64_t)k * n + i] = (smp && !held) ? 1 : 0;
    zt[(int64_t)k * n + i] = held ? v : __builtin_nan("");
  }
}
hipError_t launch_cv_prepare(const double *z, const uint8_t *known, const uint8_t *fold, int n_folds, int64_t n,
                             uint8_t *masks, double *zt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cv_prepare, block_grid((n + kThreads - 1) / kThreads, kThreads), dim3(kThreads), 0, s, z, known,
                     fold, n_folds, n, masks, zt);
  return hipGetLastError();
}

}  // namespace mpr
