"""Plain FP64 CPU oracle of the MPR hybrid Monte Carlo gap-filling method.

TEST INFRASTRUCTURE.  This module is the checker for the GPU library: only
tests, the smoke check and the benchmark's CPU-baseline leg may import it.
It shares no code with the HIP library and is slow on purpose: every step is
written out in the order the paper gives it, vectorised over whole
half-lattices and over independent chains with NumPy, in float64.

Paper: Zukovic & Hristopulos, "Gibbs Markov random fields with continuous
values based on the modified planar rotator model" (arXiv 1710.03038).
Equation numbers follow the paper: (2) data -> angle map, (3) MPR energy,
(4) sample specific energy, (5) equilibrium specific energy, (6) over-
relaxation; Algorithm 1 is the hybrid UPDATE, Algorithm 2 the simulation
driver.

Readings of points the paper leaves open (each also used by the library):

* Over-relaxation (Eq. 6) is printed with the q = 1 molecular field.  For
  q = 1/2 that map does not conserve the energy, although the text says it
  does.  We reflect q*phi about Psi = atan2(sum sin q*phi_j, sum cos q*phi_j):
  phi* = (2 Psi - q phi)/q, which conserves Eq. (3) exactly.  Because the
  energy is not 2*pi-periodic for q < 1, phi* is used only when it lies in
  [0, 2*pi); otherwise the site keeps phi.  For q = 1 the result is wrapped
  mod 2*pi.  With |h| = 0 the move is the identity.
* Restricted Metropolis proposals are wrapped into [0, 2*pi) and the energy
  change is evaluated at the wrapped angle (Algorithm 1, step 3).
* A proposal is accepted iff dH <= 0 or r < exp(-dH/T); r, u are
  (w >> 8) * 2^-24 for Philox words w (Algorithm 1, steps 2, 5, 6).
* The sweep is a checkerboard: all gap sites with (x + y) even, then all
  with (x + y) odd (Sec. 5.2).  Open boundaries: in-grid neighbours only.
* Eq. (4) averages over unordered sample-sample neighbour pairs, the same
  normalisation as Eq. (5).
* The a-rule (Algorithm 2, step 4.2) is applied after every
  ``adapt_every``-th equilibration sweep using the mean acceptance over that
  window (1 = every sweep, as printed); a is reset to 1 for sampling
  (Algorithm 2, step 5.2) unless ``a_sample_keep``.
* The fill records every ``stride``-th sampling sweep; the prediction is the
  arithmetic mean in angle space mapped back by the inverse of Eq. (2).
* The Savitzky-Golay filter of Algorithm 2, step 4.4 has degree 1: the
  slope is that of the least-squares line through the last n_fit specific
  energies (one per sweep), checked after sweep i + 1 when i >= n_fit and
  i is a multiple of n_f.  Chains of a batch sweep in lock-step until every
  chain has passed a check.

Replicate auxiliary nodes (Sec. 2.5), an option (``boundary=REPLICATE``):
the grid is padded with a ring of auxiliary nodes holding copies of their
nearest grid sites and the padded grid is swept with open boundaries, the
ring frozen.  The ring is refreshed from the state at the start of every
half-sweep, so an edge site's auxiliary neighbour holds that site's own
value from before the half-sweep (a corner site has two such neighbours).
Energies (Eqs. 4, 5, the e(T) table and the equilibration trace) stay on
the grid's own 2 L (L - 1) pairs: an auxiliary pair would only add the
constant -1.  The update then depends on the site's previous value, so it
no longer satisfies detailed balance for Eq. (3); the open boundary is the
default.

Cross-validation of q (Sec. 6 proposes choosing q in [0, 1/2] this way;
the procedure is this project's reading): the samples are split into K
folds; for each candidate q and fold, the method runs with that fold's
samples hidden, each candidate with its own e(T) table, and the candidate
with the least pooled absolute error on the held-out samples wins (ties:
the larger q).  q = 0 is left out: it makes every state equally likely.
The equilibration of each fit is a fixed sweep count with the a-rule.

The GMRF variant (Sec. 4.4) replaces the pair interaction by
H_ij = 1 - dphi^2 / (2 pi^2) on the same non-periodic angles; its
over-relaxation reflects phi about the mean of its neighbours, kept only
inside [0, 2 pi), and everything else is unchanged.

Random stream (a definition of this project): key = (seed mod 2^32,
seed >> 32).  The sites of one colour in a column come in pairs
(y, y + 2) with y mod 4 in {0, 1}; one call with counter (pair, sweep,
chain, grid), pair = (y with bit 1 cleared) * nx + x, serves both sites of
a pair in one sweep: words (w0 -> u, w1 -> r) to the pair's first site,
(w2 -> u, w3 -> r) to its second.  The hot start uses counter (site, 0xFFFFFFFF,
chain, grid) with site = y * nx + x (the sweep word never reaches
0xFFFFFFFF) and the u word w0.
"""
import math

import numpy as np

from .philox import philox4x32, unit_float

TWO_PI = 2.0 * math.pi
HOT_START_SWEEP = 0xFFFFFFFF

# Pair interactions (Sec. 4.4): the MPR energy of Eq. (3), H_ij = cos(q dphi),
# or the Gaussian (GMRF) one, H_ij = 1 - dphi^2 / (2 pi^2); H = -sum H_ij.
MPR, GMRF = "mpr", "gmrf"
# Boundary of the sweep (Sec. 2.1 open; Sec. 2.5 replicate auxiliary nodes).
OPEN, REPLICATE = "open", "replicate"
TWO_PI_SQ = 2.0 * math.pi * math.pi


class OracleError(ValueError):
    """Raised for inputs the method cannot process (no samples, no pairs)."""


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def split_seed(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def site_uniforms(seed, ny, nx, sweep, chains, grid, origin=(0, 0), gnx=None):
    """Uniforms (u, r) of every site for one sweep; arrays (C, ny, nx).

    ``origin`` and ``gnx`` place the array as a window at (y0, x0) of a
    larger grid of width ``gnx``: the stream is keyed by the sites'
    coordinates in that grid.
    """
    k0, k1 = split_seed(seed)
    chains = np.asarray(chains, dtype=np.uint64).reshape(-1, 1, 1)
    # int64 so that a window may start left of or above the grid (the ring of
    # auxiliary nodes); the counter word is the site index mod 2^32
    y = np.arange(origin[0], origin[0] + ny, dtype=np.int64).reshape(1, ny, 1)
    x = np.arange(origin[1], origin[1] + nx, dtype=np.int64).reshape(1, 1, nx)
    gnx = nx if gnx is None else gnx
    sweep = int(sweep)
    if sweep == HOT_START_SWEEP:
        site = ((y * gnx + x) % (1 << 32)).astype(np.uint64)
        w0, w1, _, _ = philox4x32(site, HOT_START_SWEEP, chains, grid, k0, k1)
        return unit_float(w0), unit_float(w1)
    # y & ~2: the pair's first site (two's complement, also above the grid)
    pair = (((y & ~2) * gnx + x) % (1 << 32)).astype(np.uint64)
    second = np.broadcast_to(((y >> 1) & 1).astype(bool), pair.shape)
    w0, w1, w2, w3 = philox4x32(pair, sweep, chains, grid, k0, k1)
    return unit_float(np.where(second, w2, w0)), unit_float(np.where(second, w3, w1))


# --------------------------------------------------------------------------
# Data transform, Eq. (2), and its inverse (Algorithm 2, step 5.3)
# --------------------------------------------------------------------------
def transform(z, known, bounds=None):
    """Map sample values linearly onto [0, 2*pi]; gaps are set to 0.

    Returns (phi, z_min, z_max) with z_min, z_max taken over the samples,
    or given as ``bounds`` (for a window of a larger grid).
    """
    z = np.asarray(z, dtype=np.float64)
    known = np.asarray(known, dtype=bool)
    zs = z[known]
    if bounds is not None:
        zmin, zmax = bounds
        phi = np.zeros(z.shape, dtype=np.float64)
        phi[known] = (zs - zmin) / (zmax - zmin) * TWO_PI
        return phi, float(zmin), float(zmax)
    if not known.any():
        raise OracleError("no sample sites")
    if not np.all(np.isfinite(zs)):
        raise OracleError("non-finite sample value")
    zmin, zmax = zs.min(), zs.max()
    if zmax == zmin:
        raise OracleError("z_max == z_min")
    phi = np.zeros(z.shape, dtype=np.float64)
    phi[known] = (zs - zmin) / (zmax - zmin) * TWO_PI
    return phi, float(zmin), float(zmax)


def inverse_transform(phi, zmin, zmax):
    return zmin + (zmax - zmin) * (np.asarray(phi, dtype=np.float64) / TWO_PI)


def hot_start(phi_s, known, seed, chains, grid, origin=(0, 0), gnx=None):
    """Paramagnetic start: every gap gets 2*pi*U (Algorithm 2, step 1.8).
    origin, gnx: a window of a larger grid (see site_uniforms)."""
    ny, nx = phi_s.shape
    chains = np.atleast_1d(np.asarray(chains))
    u, _ = site_uniforms(seed, ny, nx, HOT_START_SWEEP, chains, grid, origin, gnx)
    phi = np.where(known[None], phi_s[None], TWO_PI * u)
    return phi


# --------------------------------------------------------------------------
# Energies, Eqs. (3)-(5)
# --------------------------------------------------------------------------
def _pairs(a):
    """The two members of every horizontal and vertical nearest-neighbour pair."""
    return ((a[..., :, :-1], a[..., :, 1:]), (a[..., :-1, :], a[..., 1:, :]))


def _pair_eps(a, b, q, model):
    """1 - H_ij of a pair: 2 sin^2(q (a - b) / 2) = 1 - cos(q (a - b)) for
    MPR (the half-angle form keeps its relative precision for small
    differences), (a - b)^2 / (2 pi^2) for GMRF."""
    if model == GMRF:
        d = a - b
        return d * d / TWO_PI_SQ
    return 2.0 * np.sin(0.5 * q * (a - b)) ** 2


def energy(phi, q, model=MPR):
    """Eq. (3) with J = 1: H = -sum over pairs H_ij, with H_ij =
    cos(q (phi_i - phi_j)) (MPR) or 1 - (phi_i - phi_j)^2 / (2 pi^2) (GMRF)."""
    tot = 0.0
    for a, b in _pairs(np.asarray(phi, dtype=np.float64)):
        if model == GMRF:
            tot = tot + ((a - b) ** 2 / TWO_PI_SQ - 1.0).sum(axis=(-2, -1))
        else:
            tot = tot - np.cos(q * (a - b)).sum(axis=(-2, -1))
    return tot


def n_pairs(ny, nx):
    """N_GP: nearest-neighbour pairs of an ny x nx grid, open boundaries."""
    return ny * (nx - 1) + nx * (ny - 1)


def state_specific_energy(phi, q, model=MPR):
    """Eq. (5) for one state: e = H / N_GP.  Returns (e, eps) with eps = 1 + e.

    eps is summed as the pairs' 1 - H_ij (see _pair_eps), which keeps its
    relative precision when the field is nearly uniform.
    """
    phi = np.asarray(phi, dtype=np.float64)
    ny, nx = phi.shape[-2:]
    s = 0.0
    for a, b in _pairs(phi):
        s = s + _pair_eps(a, b, q, model).sum(axis=(-2, -1))
    eps = s / n_pairs(ny, nx)
    return eps - 1.0, eps


def sample_specific_energy(phi, known, q, model=MPR):
    """Eq. (4): mean of -H_ij over unordered sample-sample pairs (for GMRF
    the sample specific energy of Sec. 4.4, the mean of dphi^2 / (2 pi^2) - 1).

    Returns (e_s, eps_s, N_SP).  Raises OracleError when N_SP = 0.
    """
    phi = np.asarray(phi, dtype=np.float64)
    known = np.asarray(known, dtype=bool)
    s = 0.0
    n = 0
    for (a, b), (ka, kb) in zip(_pairs(phi), _pairs(known)):
        both = ka & kb
        s += _pair_eps(a[both], b[both], q, model).sum()
        n += int(both.sum())
    if n == 0:
        raise OracleError("no sample-sample pairs")
    eps = s / n
    return eps - 1.0, eps, n


# --------------------------------------------------------------------------
# Algorithm 1 (hybrid UPDATE), checkerboard order
# --------------------------------------------------------------------------
def wrap(x):
    """Angle into [0, 2*pi): x - 2*pi*floor(x / 2*pi), with the rounding
    cases folded back (a result of exactly 2*pi becomes 0)."""
    y = x - TWO_PI * np.floor(x / TWO_PI)
    y = np.where(y < 0.0, y + TWO_PI, y)
    return np.where(y >= TWO_PI, 0.0, y)


def _neighbours(phi, boundary=OPEN):
    """Angles of the four neighbours of every site, NaN where off the grid;
    with REPLICATE the off-grid neighbours are auxiliary nodes that copy
    their nearest grid site."""
    ny, nx = phi.shape[-2:]
    if boundary == REPLICATE:
        pad = np.pad(phi, [(0, 0)] * (phi.ndim - 2) + [(1, 1), (1, 1)], mode="edge")
    else:
        pad = np.full(phi.shape[:-2] + (ny + 2, nx + 2), np.nan)
        pad[..., 1:-1, 1:-1] = phi
    return [pad[..., 1:-1, :-2], pad[..., 1:-1, 2:], pad[..., :-2, 1:-1], pad[..., 2:, 1:-1]]


def over_relax(phi, nbrs, q, model=MPR):
    """Energy-conserving reflection of each spin about its local field, Eq. (6)
    in the q-aware reading.  ``nbrs`` are the neighbour angles (NaN = none).
    For GMRF the site's energy is a parabola in phi about the neighbours'
    mean m, and the reflection is 2 m - phi, kept only inside [0, 2 pi)."""
    if model == GMRF:
        cnt = sum((~np.isnan(n)).astype(np.float64) for n in nbrs)
        tot = sum(np.nan_to_num(n) for n in nbrs)
        with np.errstate(invalid="ignore", divide="ignore"):
            star = 2.0 * tot / cnt - phi
        ok = (cnt > 0) & (star >= 0.0) & (star < TWO_PI)
        return np.where(ok, star, phi)
    hx = sum(np.where(np.isnan(n), 0.0, np.cos(q * np.nan_to_num(n))) for n in nbrs)
    hy = sum(np.where(np.isnan(n), 0.0, np.sin(q * np.nan_to_num(n))) for n in nbrs)
    psi = np.arctan2(hy, hx)
    star = (2.0 * psi - q * phi) / q
    if q == 1.0:
        out = wrap(star)
    else:
        out = np.where((star >= 0.0) & (star < TWO_PI), star, phi)
    return np.where(hx * hx + hy * hy <= 1e-24, phi, out)


def site_energy(phi, nbrs, q, model=MPR):
    """Energy of the bonds of one site: -sum_j H_ij."""
    if model == GMRF:
        return sum(np.where(np.isnan(n), 0.0, (phi - np.nan_to_num(n)) ** 2 / TWO_PI_SQ - 1.0) for n in nbrs)
    return -sum(np.where(np.isnan(n), 0.0, np.cos(q * (phi - np.nan_to_num(n)))) for n in nbrs)


def hybrid_sweep(phi, known, beta, alpha, q, seed, sweep, chains, grid, margins=None, origin=(0, 0), gnx=None,
                 or_step=True, model=MPR, boundary=OPEN):
    """One sweep of Algorithm 1 over all gap sites, colour 0 then colour 1.

    phi: (C, ny, nx) float64 current states (not modified).
    known: (ny, nx) bool, True at frozen sample sites.
    beta: (C,) inverse temperatures 1/T (0 and inf allowed).
    alpha: (C,) proposal widths 2*pi/a.
    margins: optional dict, filled with per-site distances of this sweep's
      discrete decisions from their thresholds (for judging rounding flips
      of another implementation): "accept" = |r - min(1, exp(-dH/T))|,
      "or_edge" = distance of the reflected angle from 0 and 2*pi, "wrap" =
      distance of the unwrapped proposal from 0 and 2*pi.  inf at sites not
      updated.
    origin, gnx: run on a window of a larger grid (see site_uniforms);
      the window's edges are then open boundaries, which is exact only for
      sites far enough from them.
    or_step: False skips step 1 (no over-relaxation): the restricted
      Metropolis update alone, or standard Metropolis with a = 1 (Sec. 2.4).
    model: MPR or GMRF pair interactions (Sec. 4.4).
    boundary: OPEN, or REPLICATE auxiliary nodes (Sec. 2.5), refreshed at
      the start of each half-sweep.
    Returns (new phi, accepted count per chain).
    """
    phi = np.array(phi, dtype=np.float64, copy=True)
    C, ny, nx = phi.shape
    beta = np.broadcast_to(np.asarray(beta, dtype=np.float64), (C,)).reshape(C, 1, 1)
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (C,)).reshape(C, 1, 1)
    u, r = site_uniforms(seed, ny, nx, sweep, chains, grid, origin, gnx)
    yy, xx = np.mgrid[origin[0]:origin[0] + ny, origin[1]:origin[1] + nx]
    accepted = np.zeros(C, dtype=np.int64)
    if margins is not None:
        for k in ("accept", "or_edge", "wrap"):
            margins[k] = np.full(phi.shape, np.inf)
    for colour in (0, 1):
        update = (((xx + yy) % 2) == colour) & ~known
        nbrs = _neighbours(phi, boundary)
        phi1 = over_relax(phi, nbrs, q, model) if or_step else phi  # step 1
        phi2 = wrap(phi1 + alpha * (u - 0.5))                # steps 2-3
        dH = site_energy(phi2, nbrs, q, model) - site_energy(phi1, nbrs, q, model)   # step 4
        with np.errstate(invalid="ignore", over="ignore"):
            boltz = np.exp(-beta * dH)                       # step 5
        accept = (dH <= 0.0) | (r < boltz)                   # step 6
        if margins is not None:
            sel = np.broadcast_to(update[None], phi.shape)
            ap = np.where(dH <= 0.0, 1.0, np.nan_to_num(boltz))
            if model == GMRF:
                cnt = sum((~np.isnan(n)).astype(np.float64) for n in nbrs)
                with np.errstate(invalid="ignore", divide="ignore"):
                    star = 2.0 * sum(np.nan_to_num(n) for n in nbrs) / cnt - phi
            else:
                hx = sum(np.where(np.isnan(n), 0.0, np.cos(q * np.nan_to_num(n))) for n in nbrs)
                hy = sum(np.where(np.isnan(n), 0.0, np.sin(q * np.nan_to_num(n))) for n in nbrs)
                star = (2.0 * np.arctan2(hy, hx) - q * phi) / q
            raw = phi1 + alpha * (u - 0.5)
            margins["accept"] = np.where(sel, np.abs(r - ap), margins["accept"])
            if or_step:
                margins["or_edge"] = np.where(sel, np.minimum(np.abs(star), np.abs(star - TWO_PI)),
                                              margins["or_edge"])
            margins["wrap"] = np.where(sel, np.minimum(np.abs(raw), np.abs(raw - TWO_PI)), margins["wrap"])
        new = np.where(accept, phi2, phi1)
        phi = np.where(update[None], new, phi)
        accepted += (update[None] & accept).sum(axis=(1, 2))
    return phi, accepted


def hybrid_sweep_literal(phi, known, beta, alpha, q, seed, sweep, chain, grid, or_step=True, model=MPR,
                         boundary=OPEN):
    """Algorithm 1 for one chain as a plain per-site loop (small grids only).

    Same checkerboard order and random stream as ``hybrid_sweep``; written
    with scalar ``math`` calls so the two can be checked against each other.
    With REPLICATE, each missing neighbour of a site contributes the site's
    own value at the start of its update (its value before the half-sweep).
    """
    phi = [list(map(float, row)) for row in np.asarray(phi, dtype=np.float64)]
    ny, nx = len(phi), len(phi[0])
    k0, k1 = split_seed(seed)
    accepted = 0
    for colour in (0, 1):
        for y in range(ny):
            for x in range(nx):
                if (x + y) % 2 != colour or known[y][x]:
                    continue
                w = philox4x32((y & ~2) * nx + x, sweep, chain, grid, k0, k1)
                wu, wr = (w[2], w[3]) if (y >> 1) & 1 else (w[0], w[1])
                u = float(unit_float(wu))
                r = float(unit_float(wr))
                cur = phi[y][x]
                nb = []
                for yy, xx in ((y, x - 1), (y, x + 1), (y - 1, x), (y + 1, x)):
                    if 0 <= yy < ny and 0 <= xx < nx:
                        nb.append(phi[yy][xx])
                    elif boundary == REPLICATE:
                        nb.append(cur)
                if model == GMRF:
                    p1 = cur
                    if or_step and nb:
                        star = 2.0 * sum(nb) / len(nb) - cur
                        p1 = star if 0.0 <= star < TWO_PI else cur
                    p2 = float(wrap(np.float64(p1 + alpha * (u - 0.5))))
                    dH = sum((p2 - v) ** 2 - (p1 - v) ** 2 for v in nb) / TWO_PI_SQ
                else:
                    hx = sum(math.cos(q * v) for v in nb)
                    hy = sum(math.sin(q * v) for v in nb)
                    if not or_step or hx * hx + hy * hy <= 1e-24:
                        p1 = cur
                    else:
                        star = (2.0 * math.atan2(hy, hx) - q * cur) / q
                        if q == 1.0:
                            p1 = float(wrap(np.float64(star)))
                        else:
                            p1 = star if 0.0 <= star < TWO_PI else cur
                    p2 = float(wrap(np.float64(p1 + alpha * (u - 0.5))))
                    dH = -sum(math.cos(q * (p2 - v)) - math.cos(q * (p1 - v)) for v in nb)
                if dH <= 0.0:
                    ok = True
                elif beta == math.inf:
                    ok = False
                else:
                    ok = r < math.exp(-beta * dH)
                phi[y][x] = p2 if ok else p1
                accepted += int(ok)
    return np.array(phi), accepted


# --------------------------------------------------------------------------
# Algorithm 2: the a-rule and the fill driver (fixed sweep counts)
# --------------------------------------------------------------------------
def adapt_a(a, acceptance, i, a_targ=0.3, k_a=3.0):
    """Algorithm 2, step 4.2: after sweep i (0-based) with acceptance A,
    a(i+1) = 1 + (i+1)/k_a if A < A_targ, else a(i+1) = a(i)."""
    return np.where(np.asarray(acceptance) < a_targ, 1.0 + (i + 1) / k_a, a)


def run_sweeps(phi, known, T, a, q, seed, first_sweep, n_sweeps, chains, grid,
               adapt=False, adapt_every=1, a_targ=0.3, k_a=3.0, trace_energy=False, or_step=True, window=None,
               model=MPR, boundary=OPEN):
    """Advance C chains of one grid by ``n_sweeps`` hybrid sweeps.

    Returns (phi, a, acceptance per sweep (n, C), specific energy per sweep
    (n, C) or None).  With ``adapt`` the a-rule is applied every
    ``adapt_every`` sweeps using the mean acceptance of that window; the
    rule's counter i is the global sweep index.  ``window`` (C,), if given,
    carries the running window sum across calls and is updated in place.
    ``or_step`` = False leaves out over-relaxation; ``boundary`` as in
    ``hybrid_sweep``.
    """
    C = phi.shape[0]
    T = np.broadcast_to(np.asarray(T, dtype=np.float64), (C,))
    with np.errstate(divide="ignore"):
        beta = np.where(np.isinf(T), 0.0, 1.0 / T)
    a = np.array(np.broadcast_to(np.asarray(a, dtype=np.float64), (C,)), copy=True)
    n_gap = int((~np.asarray(known, dtype=bool)).sum())
    acc_trace = np.zeros((n_sweeps, C))
    e_trace = np.zeros((n_sweeps, C)) if trace_energy else None
    if window is None:
        window = np.zeros(C)
    for s in range(n_sweeps):
        i = first_sweep + s
        phi, acc = hybrid_sweep(phi, known, beta, TWO_PI / a, q, seed, i, chains, grid, or_step=or_step, model=model,
                                boundary=boundary)
        A = acc / n_gap if n_gap > 0 else np.ones(C)
        acc_trace[s] = A
        if trace_energy:
            e_trace[s] = state_specific_energy(phi, q, model)[0]
        if adapt:
            window += A
            if (i + 1) % adapt_every == 0:
                a = adapt_a(a, window / adapt_every, i, a_targ, k_a)
                window[:] = 0.0
    return phi, a, acc_trace, e_trace


def fill(z, known, T, n_eq, n_samp, stride, q=0.5, seed=0, chains=1, grid=0,
         a_targ=0.3, k_a=3.0, adapt_every=1, a_sample_keep=False, model=MPR, boundary=OPEN):
    """Algorithm 2 with fixed sweep counts (no Savitzky-Golay stop).

    Hot start, ``n_eq`` equilibration sweeps with the a-rule, then
    ``n_samp`` sampling sweeps of which every ``stride``-th is recorded, for
    each of ``chains`` independent chains.  Returns a dict with z_hat (the
    conditional mean mapped back, samples copied through), z_std, the
    recorded count and the per-sweep acceptance trace.
    """
    known = np.asarray(known, dtype=bool)
    phi_s, zmin, zmax = transform(z, known)
    chain_ids = np.arange(chains)
    phi = hot_start(phi_s, known, seed, chain_ids, grid)
    a = np.ones(chains)
    phi, a, acc_eq, _ = run_sweeps(phi, known, T, a, q, seed, 0, n_eq, chain_ids, grid,
                                   adapt=True, adapt_every=adapt_every, a_targ=a_targ, k_a=k_a, model=model,
                                   boundary=boundary)
    a_eq = a.copy()
    if not a_sample_keep:
        a = np.ones(chains)
    s1 = np.zeros(known.shape)
    s2 = np.zeros(known.shape)
    m = 0
    acc_samp = []
    for j in range(n_samp):
        phi, a, acc, _ = run_sweeps(phi, known, T, a, q, seed, n_eq + j, 1, chain_ids, grid, model=model,
                                    boundary=boundary)
        acc_samp.append(acc[0])
        if (j + 1) % stride == 0:
            s1 += phi.sum(axis=0)
            s2 += (phi * phi).sum(axis=0)
            m += chains
    if m == 0:
        raise OracleError("no recorded realisation")
    mean = s1 / m
    var = np.maximum(s2 / m - mean * mean, 0.0)
    z_hat = np.where(known, np.asarray(z, dtype=np.float64), inverse_transform(mean, zmin, zmax))
    z_std = np.where(known, 0.0, (zmax - zmin) / TWO_PI * np.sqrt(var))
    return dict(z_hat=z_hat, z_std=z_std, records=m, zmin=zmin, zmax=zmax, a_eq=a_eq,
                acc_eq=acc_eq, acc_samp=np.array(acc_samp), phi=phi)


# --------------------------------------------------------------------------
# Algorithm 2, step 4: automatic detection of equilibrium
# --------------------------------------------------------------------------
def ols_slope(y):
    """Slope of the least-squares line through (k, y[k]), k = 0..n-1, over
    the last axis.  This is the derivative estimate of the Savitzky-Golay
    filter of degree 1 on that window (the same at every point of it).

    With x centred, sum x_k y_k pairs mirrored points:
    sum_{k < n/2} x_k (y_k - y_{n-1-k}); a constant or mirror-symmetric
    window then gives exactly 0, so a flat energy never reads as falling.
    """
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[-1]
    h = n // 2
    x = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    num = (x[:h] * (y[..., :h] - y[..., ::-1][..., :h])).sum(axis=-1)
    return num / (x * x).sum()


def sg_stop_index(e_after, n_f, n_fit, i_max):
    """The loop of Algorithm 2, step 4, for one chain, on a given energy
    series: e_after[j] is the specific energy after sweep j + 1.  The
    slope k starts at -1; after sweep i + 1, when i >= n_fit and i is a
    multiple of n_f, k becomes the degree-1 Savitzky-Golay slope of the
    last n_fit energies (step 4.4); the loop runs while k < 0 and
    i <= i_max.  Returns the number of sweeps it runs, or None when the
    series is too short to tell."""
    i, k = 0, -1.0
    while k < 0 and i <= i_max:
        if i >= len(e_after):
            return None
        if i >= n_fit and i % n_f == 0:
            k = float(ols_slope(e_after[i + 1 - n_fit:i + 1]))
        i += 1
    return i


def equilibrate(phi, known, T, a, q, seed, first_sweep, chains, grid, n_f=5, n_fit=20, i_max=1000,
                adapt=True, or_step=True, adapt_every=1, a_targ=0.3, k_a=3.0, model=MPR, boundary=OPEN):
    """Algorithm 2, step 4, for C chains of one grid swept in lock-step:
    hybrid sweeps (4.1), the a-rule (4.2, with ``adapt``), the specific
    energy after every sweep (4.3) and the Savitzky-Golay slope check of
    ``sg_stop_index`` per chain (4.4).  The batch runs until every chain's
    slope has been >= 0 at a check, or i_max + 1 sweeps.  i counts the
    sweeps of this call; the a-rule's counter is first_sweep + i.

    Returns (phi, a, sweeps run, eq_at (C,): the sweep count after which
    each chain's slope was first >= 0, or -1; energy trace (n, C);
    acceptance trace (n, C)).
    """
    C = phi.shape[0]
    eq_at = np.full(C, -1)
    window = np.zeros(C)
    e_hist, acc_hist = [], []
    i = 0
    while i <= i_max and np.any(eq_at < 0):
        phi, a, acc, e = run_sweeps(phi, known, T, a, q, seed, first_sweep + i, 1, chains, grid, adapt=adapt,
                                    adapt_every=adapt_every, a_targ=a_targ, k_a=k_a, trace_energy=True,
                                    or_step=or_step, window=window, model=model, boundary=boundary)
        e_hist.append(e[0])
        acc_hist.append(acc[0])
        if i >= n_fit and i % n_f == 0:
            k = ols_slope(np.array(e_hist[i + 1 - n_fit:i + 1]).T)
            eq_at = np.where((eq_at < 0) & (k >= 0), i + 1, eq_at)
        i += 1
    return phi, a, i, eq_at, np.array(e_hist), np.array(acc_hist)


# --------------------------------------------------------------------------
# Specific energy matching (Sec. 2.3)
# --------------------------------------------------------------------------
RANGE_CLAMPED = 1


def match_T(e_s, tab_T, tab_e):
    """Solve e(T) = e_s on a tabulated equilibrium curve (Sec. 2.3).

    The curve is interpolated monotonically (PCHIP) in (log T, log(1 + e)),
    and the root is found by Brent's method to 1e-14 relative.  Values
    outside the table are clamped to its ends and flagged RANGE_CLAMPED.
    Returns (T_hat array, status array).
    """
    from scipy.interpolate import PchipInterpolator
    from scipy.optimize import brentq

    tab_T = np.asarray(tab_T, dtype=np.float64)
    tab_e = np.asarray(tab_e, dtype=np.float64)
    lt = np.log(tab_T)
    le = np.log1p(tab_e)
    curve = PchipInterpolator(lt, le)
    e_s = np.atleast_1d(np.asarray(e_s, dtype=np.float64))
    T_out = np.empty_like(e_s)
    status = np.zeros(e_s.shape, dtype=np.int32)
    for k, e in enumerate(e_s):
        if e <= tab_e[0]:
            T_out[k] = tab_T[0]
            status[k] = RANGE_CLAMPED if e < tab_e[0] else 0
            continue
        if e >= tab_e[-1]:
            T_out[k] = tab_T[-1]
            status[k] = RANGE_CLAMPED if e > tab_e[-1] else 0
            continue
        target = math.log1p(e)
        j = int(np.searchsorted(tab_e, e, side="right")) - 1
        if tab_e[j] == e:
            T_out[k] = tab_T[j]
            continue
        root = brentq(lambda x: float(curve(x)) - target, lt[j], lt[j + 1],
                      xtol=1e-15, rtol=1e-15, maxiter=200)
        T_out[k] = math.exp(root)
    return T_out, status


def validation_measures(z_true, z_hat, gaps):
    """The validation measures of Sec. 3.3 over the prediction sites (gaps),
    with the estimation error eps = Z - Z_hat: AAE = mean |eps|,
    ARE = mean eps / Z, AARE = mean |eps| / Z, RASE = sqrt(mean eps^2), and
    R, the linear (Pearson) correlation coefficient of Z and Z_hat.  P is
    the number of prediction sites."""
    gaps = np.asarray(gaps, dtype=bool)
    z = np.asarray(z_true, dtype=np.float64)[gaps]
    zh = np.asarray(z_hat, dtype=np.float64)[gaps]
    eps = z - zh
    dz, dh = z - z.mean(), zh - zh.mean()
    return dict(AAE=float(np.abs(eps).mean()), ARE=float((eps / z).mean()), AARE=float((np.abs(eps) / z).mean()),
                RASE=float(math.sqrt((eps * eps).mean())),
                R=float((dz * dh).sum() / math.sqrt((dz * dz).sum() * (dh * dh).sum())), P=int(z.size))


def mae(z_true, z_hat, gaps):
    """Average absolute error over the prediction sites (Sec. 3, AAE)."""
    gaps = np.asarray(gaps, dtype=bool)
    return float(np.abs(np.asarray(z_true)[gaps] - np.asarray(z_hat)[gaps]).mean())


# --------------------------------------------------------------------------
# Selection of q by cross-validation (Sec. 6)
# --------------------------------------------------------------------------
def cv_masks(known, fold, k):
    """Masks of fold k: the training samples (every sample whose fold id is
    not k) and the held-out ones (fold id k), which become gaps and are
    scored."""
    known = np.asarray(known, dtype=bool)
    held = known & (np.asarray(fold) == k)
    return known & ~held, held


def cv_pool(parts):
    """Pool held-out errors over the folds.  parts: per fold (sum |eps|,
    sum eps^2, count).  Returns (AAE, RASE) over all held-out samples: each
    sample is held out once, so this is the K-fold estimate of the
    prediction error."""
    s_abs = sum(p[0] for p in parts)
    s_sq = sum(p[1] for p in parts)
    n = sum(p[2] for p in parts)
    if n == 0:
        raise OracleError("no held-out samples")
    return s_abs / n, math.sqrt(s_sq / n)


def cv_best(qs, scores):
    """Index of the candidate with the least score; among equal scores the
    largest q (nearest the paper's q = 1/2)."""
    qs = np.asarray(qs, dtype=np.float64)
    scores = np.asarray(scores, dtype=np.float64)
    low = scores == scores.min()
    return int(np.flatnonzero(low)[np.argmax(qs[low])])


def cv_select_q(z, known, fold, n_folds, qs, tables, n_eq, n_samp, stride, seed=0, chains=1, a_targ=0.3, k_a=3.0,
                boundary=OPEN):
    """Choose q in (0, 1/2] by K-fold cross-validation (the extension
    proposed in Sec. 6).  For candidate i and fold k the fold's samples are
    hidden and the method runs on the rest: Eq. (2) on the training
    samples, e_s (Eq. 4) at q_i, T-hat by SEM on candidate i's own e(T)
    table, then ``fill`` (hot start, n_eq sweeps with the a-rule, n_samp
    sampling sweeps, every stride-th recorded) on grid id i * n_folds + k.
    The score of a candidate is the pooled AAE (and RASE) over the
    held-out samples.

    fold: integer fold id in [0, n_folds) at every sample site (ignored at
    gaps).  tables: per candidate (tab_T, tab_e).
    Returns dict(aae (n_q,), rase (n_q,), T (n_q, n_folds), best index).
    """
    z = np.asarray(z, dtype=np.float64)
    known = np.asarray(known, dtype=bool)
    aae, rase, Ts = [], [], []
    for i, q in enumerate(qs):
        tab_T, tab_e = tables[i]
        parts, Tq = [], []
        for k in range(n_folds):
            train, held = cv_masks(known, fold, k)
            phi_s, _, _ = transform(z, train)
            e_s, _, _ = sample_specific_energy(phi_s, train, q)
            T, _ = match_T(e_s, tab_T, tab_e)
            out = fill(z, train, T[0], n_eq, n_samp, stride, q=q, seed=seed, chains=chains, grid=i * n_folds + k,
                       a_targ=a_targ, k_a=k_a, boundary=boundary)
            eps = z[held] - out["z_hat"][held]
            parts.append((float(np.abs(eps).sum()), float((eps * eps).sum()), int(held.sum())))
            Tq.append(float(T[0]))
        a, r = cv_pool(parts)
        aae.append(a)
        rase.append(r)
        Ts.append(Tq)
    return dict(aae=np.array(aae), rase=np.array(rase), T=np.array(Ts), best=cv_best(qs, aae))
