"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each checks a published
vector, a closed form, an invariant, an exact law computed by quadrature or
a hand-derived value.
"""
import math
import os

import numpy as np
import pytest
from scipy.stats import chi2

from oracle import exact, mpr
from oracle.philox import philox4x32, unit_float

TWO_PI = 2.0 * math.pi


def chi2_pvalue(counts, probs):
    """Pearson chi-square p-value of binned counts against bin
    probabilities.  Adjacent bins are pooled, in order, until every cell
    expects at least 5 counts (a remainder joins the last cell), the
    condition for the chi-square approximation."""
    counts = np.asarray(counts, dtype=np.float64)
    exp = np.asarray(probs) * counts.sum()
    c, e = [], []
    cc = ee = 0.0
    for ci, ei in zip(counts, exp):
        cc += ci
        ee += ei
        if ee >= 5.0:
            c.append(cc)
            e.append(ee)
            cc = ee = 0.0
    if ee > 0.0 or cc > 0.0:
        if e:
            c[-1] += cc
            e[-1] += ee
        else:
            c, e = [cc], [ee]
    c, e = np.array(c), np.array(e)
    stat = ((c - e) ** 2 / e).sum()
    return chi2.sf(stat, max(len(c) - 1, 1))


def run_chains(known, phi0, T, a, q, seed, n_sweeps, grid=0):
    C = phi0.shape[0]
    phi, _, _, _ = mpr.run_sweeps(phi0, known, T, a, q, seed, 0, n_sweeps, np.arange(C), grid)
    return phi


# ---------------------------------------------------------------- Philox
def test_philox_known_answers(golden_dir):
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(t, 16) for t in row]
        out = philox4x32(*v[:6])
        assert [int(w) for w in out] == v[6:]


def test_unit_float_range():
    assert unit_float(0) == 0.0
    assert unit_float(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert unit_float(0x80000000) == 0.5


# ---------------------------------------------------------------- Eq. (2)
def test_transform_endpoints_and_inverse():
    rng = np.random.default_rng(0)
    z = rng.normal(50, 10, size=(9, 11))
    known = rng.random((9, 11)) < 0.5
    phi, zmin, zmax = mpr.transform(z, known)
    assert zmin == z[known].min() and zmax == z[known].max()
    assert phi[known].min() == 0.0
    assert phi[known].max() == TWO_PI            # closed interval, exactly 2*pi
    lin = TWO_PI * (z[known] - zmin) / (zmax - zmin)
    np.testing.assert_allclose(phi[known], lin, rtol=1e-15, atol=1e-15)
    back = mpr.inverse_transform(phi, zmin, zmax)
    np.testing.assert_allclose(back[known], z[known], rtol=1e-14)


def test_transform_degenerate():
    z = np.full((3, 3), 4.0)
    with pytest.raises(mpr.OracleError):
        mpr.transform(z, np.ones((3, 3), bool))
    with pytest.raises(mpr.OracleError):
        mpr.transform(z, np.zeros((3, 3), bool))


# ---------------------------------------------------------------- Eqs. (3)-(5)
def test_uniform_field_is_ground_state():
    # H = -N_GP for a uniform field: e = -1, eps = 0 (Eq. 3, Eq. 5)
    for ny, nx in ((1, 2), (4, 4), (5, 3)):
        phi = np.full((ny, nx), 2.3)
        e, eps = mpr.state_specific_energy(phi, 0.5)
        assert e == -1.0 and eps == 0.0
        assert mpr.energy(phi, 0.5) == -mpr.n_pairs(ny, nx)
    assert mpr.n_pairs(7, 7) == 2 * 7 * 6          # N_GP = 2L(L-1), Eq. (5)


def test_hand_energies():
    q = 0.5
    # 2 x 3, columns (0, 0, 2*pi): horizontal pairs cos 0 = 1 and cos(pi) = -1 per
    # row, three vertical pairs of equal values: sum cos = 3 over 7 pairs.
    phi = np.array([[0, 0, TWO_PI], [0, 0, TWO_PI]], dtype=float)
    assert mpr.state_specific_energy(phi, q)[0] == pytest.approx(-3.0 / 7.0, abs=1e-15)
    # checkerboard of 0 and pi: every pair has q*dphi = pi/2, cos = 0
    phi = np.array([[0, math.pi], [math.pi, 0]])
    assert mpr.state_specific_energy(phi, q)[0] == pytest.approx(0.0, abs=1e-15)
    # chain 0, 2pi/3, 4pi/3: two pairs with cos(pi/3) = 1/2
    phi = np.array([[0, TWO_PI / 3, 2 * TWO_PI / 3]])
    assert mpr.state_specific_energy(phi, q)[0] == pytest.approx(-0.5, abs=1e-15)
    # literal Eq. (3) sum agrees with the eps form on a random field
    rng = np.random.default_rng(3)
    phi = rng.uniform(0, TWO_PI, (6, 7))
    e, _ = mpr.state_specific_energy(phi, q)
    assert e == pytest.approx(mpr.energy(phi, q) / mpr.n_pairs(6, 7), abs=1e-14)


def test_sample_specific_energy_counts_unordered_pairs():
    q = 0.5
    # 3 x 3, known = top row and the left column; sample pairs:
    # (0,0)-(0,1), (0,1)-(0,2), (0,0)-(1,0), (1,0)-(2,0)  -> N_SP = 4
    known = np.array([[1, 1, 1], [1, 0, 0], [1, 0, 0]], bool)
    phi = np.array([[0.0, math.pi, 0.0], [TWO_PI, 9, 9], [TWO_PI, 9, 9]])
    e_s, eps, n = mpr.sample_specific_energy(phi, known, q)
    # cos(pi/2) = 0, cos(-pi/2) = 0, cos(-pi) = -1, cos(0) = 1  -> sum 0
    assert n == 4
    assert e_s == pytest.approx(0.0, abs=1e-15)
    with pytest.raises(mpr.OracleError):
        mpr.sample_specific_energy(phi, np.eye(3, dtype=bool), q)


# ---------------------------------------------------------------- Eq. (6)
def test_over_relaxation_conserves_energy_and_is_an_involution():
    rng = np.random.default_rng(5)
    q = 0.5
    phi = rng.uniform(0, TWO_PI, (200, 6, 7))
    nbrs = mpr._neighbours(phi)
    e0 = mpr.site_energy(phi, nbrs, q)
    p1 = mpr.over_relax(phi, nbrs, q)
    e1 = mpr.site_energy(p1, nbrs, q)
    assert np.abs(e1 - e0).max() < 1e-12
    assert np.all((p1 >= 0) & (p1 < TWO_PI))
    moved = np.abs(p1 - phi) > 1e-9
    assert moved.mean() > 0.2                       # the reflection does act
    p2 = mpr.over_relax(p1, nbrs, q)
    assert np.abs(p2 - phi).max() < 1e-12           # R(R(phi)) = phi


def test_printed_over_relaxation_breaks_energy_for_q_half():
    # Reading of Eq. (6): the printed q = 1 field does not conserve Eq. (3)
    # for q = 1/2 (one neighbour at 0, phi = 1 goes to 2*pi - 1).
    q = 0.5
    nb, phi = 0.0, 1.0
    printed = (2 * math.atan2(math.sin(nb), math.cos(nb)) - phi) % TWO_PI
    assert -math.cos(q * (printed - nb)) == pytest.approx(0.8775825618903728)
    assert -math.cos(q * (phi - nb)) == pytest.approx(-0.8775825618903728)


def test_uniform_field_fixed_point():
    phi = np.full((1, 5, 5), 1.7)
    nbrs = mpr._neighbours(phi)
    np.testing.assert_allclose(mpr.over_relax(phi, nbrs, 0.5), phi, atol=1e-14)
    known = np.zeros((5, 5), bool)
    out = run_chains(known, phi, 0.0, 1.0, 0.5, 9, 3)      # T = 0: nothing moves uphill
    np.testing.assert_allclose(out, phi, atol=1e-14)


# ---------------------------------------------------------------- Algorithm 1
@pytest.mark.parametrize("shape", [(2, 2), (3, 3), (4, 5), (9, 7), (1, 6)])
def test_vectorised_sweep_matches_literal_loop(shape):
    ny, nx = shape
    rng = np.random.default_rng(ny * 31 + nx)
    z = rng.normal(size=shape)
    known = rng.random(shape) < 0.35
    known.flat[0] = True
    known.flat[-1] = True
    phi_s, _, _ = mpr.transform(z, known)
    phi = mpr.hot_start(phi_s, known, 77, [5], 1)
    for T, a in ((0.2, 1.0), (0.01, 6.0), (math.inf, 1.0), (0.0, 2.0)):
        beta = 0.0 if T == math.inf else (math.inf if T == 0 else 1 / T)
        for q in (0.5, 1.0):
            v, acc = mpr.hybrid_sweep(phi, known, [beta], [TWO_PI / a], q, 77, 3, [5], 1)
            l, acc2 = mpr.hybrid_sweep_literal(phi[0], known, beta, TWO_PI / a, q, 77, 3, 5, 1)
            assert np.abs(v[0] - l).max() <= 1e-13
            assert acc[0] == acc2


def test_frozen_sites_never_change():
    rng = np.random.default_rng(8)
    z = rng.normal(size=(8, 8))
    known = rng.random((8, 8)) < 0.5
    phi_s, _, _ = mpr.transform(z, known)
    phi = mpr.hot_start(phi_s, known, 1, np.arange(4), 0)
    for T in (0.0, 0.05, 1.0, math.inf):
        out = run_chains(known, phi, T, 1.0, 0.5, 1, 20)
        assert np.array_equal(out[:, known], phi[:, known])
        assert np.all(out[:, ~known] >= 0) and np.all(out[:, ~known] < TWO_PI)


def test_infinite_temperature_one_sweep_gives_uniform_gaps():
    # beta = 0, a = 1: every proposal wrap(phi' + 2*pi*(u - 1/2)) is accepted
    # and uniform on [0, 2*pi) whatever phi' is.
    C, n = 64, 32
    known = np.zeros((n, n), bool)
    known[::4, ::4] = True
    phi0 = np.zeros((C, n, n))
    phi0[:, known] = 1.0
    phi, acc, _, _ = mpr.run_sweeps(phi0, known, math.inf, 1.0, 0.5, 11, 0, 1, np.arange(C), 0)
    assert np.all(acc == 1.0)
    gaps = phi[:, ~known]
    counts, _ = np.histogram(gaps, bins=16, range=(0, TWO_PI))
    assert chi2_pvalue(counts, np.full(16, 1 / 16)) > 1e-3
    # gap-gap pairs: E cos(q dphi) = (sin(pi q)/(pi q))^2 = 4/pi^2 for q = 1/2
    a, b = phi[:, 1:3, :-1], phi[:, 1:3, 1:]
    vals = np.cos(0.5 * (a - b)).ravel()
    assert abs(vals.mean() - exact.uniform_gap_gap_cos(0.5)) < 4 * vals.std() / math.sqrt(vals.size)
    # gap-sample pairs with the sample at 1.0: E = 2 sin(phi_j/2)/pi
    s = known.nonzero()
    left = phi[:, s[0][1:4], s[1][1:4] - 1]
    vals = np.cos(0.5 * (left - 1.0)).ravel()
    ref = exact.uniform_gap_sample_cos(0.5, 1.0)
    assert ref == pytest.approx(2 * math.sin(0.5) / math.pi)
    assert abs(vals.mean() - ref) < 4 * vals.std() / math.sqrt(vals.size)


def test_zero_temperature_energy_never_increases():
    rng = np.random.default_rng(12)
    n = 12
    known = rng.random((n, n)) < 0.3
    phi_s, _, _ = mpr.transform(rng.normal(size=(n, n)), known)
    phi = mpr.hot_start(phi_s, known, 4, np.arange(3), 0)
    prev = mpr.energy(phi, 0.5)
    for s in range(25):
        phi, acc = mpr.hybrid_sweep(phi, known, [math.inf] * 3, [TWO_PI / 2] * 3, 0.5, 4, s, np.arange(3), 0)
        cur = mpr.energy(phi, 0.5)
        assert np.all(cur <= prev + 1e-12)
        prev = cur


def test_single_gap_relaxes_to_field_direction():
    # One free site among frozen neighbours at T -> 0 ends at phi = Psi/q,
    # the minimiser of -|h| cos(q phi - Psi).
    q = 0.5
    known = np.ones((3, 3), bool)
    known[1, 1] = False
    phi0 = np.array([[0, 1.0, 0], [2.0, 5.0, 2.5], [0, 3.0, 0]])[None]
    phi, a, acc, _ = mpr.run_sweeps(phi0, known, 1e-9, 1.0, q, 2, 0, 300, [0], 0, adapt=True)
    psi = math.atan2(sum(math.sin(q * v) for v in (1.0, 2.0, 2.5, 3.0)),
                     sum(math.cos(q * v) for v in (1.0, 2.0, 2.5, 3.0)))
    assert abs(phi[0, 1, 1] - psi / q) < 2e-3
    assert a[0] > 50                        # the a-rule kept shrinking the step


# ------------------------------------------------ exact laws of tiny grids
@pytest.mark.parametrize("T,a", [(0.1, 1.0), (0.5, 1.0), (2.0, 1.0), (0.1, 4.0), (0.5, 3.0)])
def test_3x3_checkerboard_frozen_exact(T, a):
    # colour-0 sites frozen; each edge site is an independent 1D law.  a > 1
    # makes the proposal a short symmetric step, whose symmetry matters.
    q, C = 0.5, 4096
    known = np.zeros((3, 3), bool)
    for y, x in ((0, 0), (0, 2), (1, 1), (2, 0), (2, 2)):
        known[y, x] = True
    vals = np.zeros((3, 3))
    vals[0, 0], vals[0, 2], vals[1, 1], vals[2, 0], vals[2, 2] = 0.3, 2.0, 3.5, 4.5, 6.0
    phi0 = np.broadcast_to(vals, (C, 3, 3)).copy()
    phi = run_chains(known, phi0, T, a, q, 1000 + int(T * 10), 60)
    for (y, x), nb in (((0, 1), ((0, 0), (0, 2), (1, 1))), ((1, 0), ((0, 0), (2, 0), (1, 1))),
                       ((1, 2), ((0, 2), (2, 2), (1, 1))), ((2, 1), ((2, 0), (2, 2), (1, 1)))):
        probs = exact.single_site_bins([vals[k] for k in nb], 1.0 / T, q, nbins=8)
        counts, _ = np.histogram(phi[:, y, x], bins=8, range=(0, TWO_PI))
        assert chi2_pvalue(counts, probs) > 1e-3, ((y, x), counts, probs * C)


@pytest.mark.parametrize("T,a", [(0.1, 1.0), (0.5, 1.0), (2.0, 1.0), (0.3, 3.0)])
def test_3x3_corners_frozen_exact(T, a):
    q, C = 0.5, 4096
    corners = {(0, 0): 0.5, (0, 2): 2.0, (2, 0): 4.0, (2, 2): 5.5}
    known = np.zeros((3, 3), bool)
    phi0 = np.zeros((C, 3, 3))
    for (y, x), v in corners.items():
        known[y, x] = True
        phi0[:, y, x] = v
    phi0 = mpr.hot_start(phi0[0], known, 21, np.arange(C), 0)
    phi = run_chains(known, phi0, T, a, q, 2000 + int(T * 10), 150)
    pc, pe = exact.corners_frozen_bins(corners, 1.0 / T, q, nbins=8)
    counts, _ = np.histogram(phi[:, 1, 1], bins=8, range=(0, TWO_PI))
    assert chi2_pvalue(counts, pc) > 1e-3, (counts, pc * C)
    for (y, x), p in pe.items():
        counts, _ = np.histogram(phi[:, y, x], bins=8, range=(0, TWO_PI))
        assert chi2_pvalue(counts, p) > 1e-3, ((y, x), counts, p * C)


@pytest.mark.parametrize("T", (0.3, 2.0))
def test_3x3_free_exact(T):
    # unconditional 3 x 3: centre marginal and mean specific energy
    q, C = 0.5, 4096
    known = np.zeros((3, 3), bool)
    phi0 = mpr.hot_start(np.zeros((3, 3)), known, 31, np.arange(C), 0)
    phi = run_chains(known, phi0, T, 1.0, q, 3000 + int(T * 10), 200)
    pc, _ = exact.free3x3(1.0 / T, q)
    counts, _ = np.histogram(phi[:, 1, 1], bins=8, range=(0, TWO_PI))
    assert chi2_pvalue(counts, pc) > 1e-3, (counts, pc * C)
    e = mpr.state_specific_energy(phi, q)[0]
    e_exact = exact.free3x3_specific_energy(1.0 / T, q)
    assert abs(e.mean() - e_exact) < 4 * e.std() / math.sqrt(C)


def test_1d_chain_q1_matches_bessel_ratio():
    # Eq. (16): open q = 1 chain, e = -I_1(beta)/I_0(beta)
    T, C, n = 0.5, 1024, 8
    known = np.zeros((1, n), bool)
    phi0 = mpr.hot_start(np.zeros((1, n)), known, 41, np.arange(C), 0)
    phi = run_chains(known, phi0, T, 1.0, 1.0, 41, 150)
    e = mpr.state_specific_energy(phi, 1.0)[0]
    ref = exact.chain1d_energy_q1(1.0 / T)
    assert ref == pytest.approx(exact.chain1d_specific_energy(1.0 / T, 1.0, n), abs=1e-8)
    assert abs(e.mean() - ref) < 4 * e.std() / math.sqrt(C)


def test_1d_chain_q_half_matches_transfer_matrix():
    T, C, n = 0.2, 1024, 6
    known = np.zeros((1, n), bool)
    phi0 = mpr.hot_start(np.zeros((1, n)), known, 43, np.arange(C), 0)
    phi = run_chains(known, phi0, T, 1.0, 0.5, 43, 200)
    e = mpr.state_specific_energy(phi, 0.5)[0]
    ref = exact.chain1d_specific_energy(1.0 / T, 0.5, n)
    assert abs(e.mean() - ref) < 4 * e.std() / math.sqrt(C)


def test_low_temperature_equipartition():
    # Harmonic limit of Eq. (3): <H> + N_GP = (N - 1) T / 2 for an unconditional
    # L x L grid, so eps = (L + 1) T / (4 L).
    L, C, T = 8, 32, 1e-4
    known = np.zeros((L, L), bool)
    phi = np.full((C, L, L), 3.0)
    phi, a, _, _ = mpr.run_sweeps(phi, known, T, 40.0, 0.5, 51, 0, 60, np.arange(C), 0)
    eps = []
    for s in range(60, 260):
        phi, _, _, _ = mpr.run_sweeps(phi, known, T, 40.0, 0.5, 51, s, 1, np.arange(C), 0)
        eps.append(mpr.state_specific_energy(phi, 0.5)[1])
    eps = np.array(eps)
    ref = (L + 1) * T / (4 * L)
    assert eps.mean() == pytest.approx(ref, rel=0.03)


# ---------------------------------------------------------------- Algorithm 2
def test_a_rule_sequence():
    a = np.array([1.0, 1.0])
    a = mpr.adapt_a(a, np.array([0.5, 0.1]), 0)     # only chain 1 below A_targ = 0.3
    np.testing.assert_array_equal(a, [1.0, 1.0 + 1 / 3])
    a = mpr.adapt_a(a, np.array([0.2, 0.4]), 5)
    np.testing.assert_array_equal(a, [3.0, 1.0 + 1 / 3])


def test_fill_small_grid():
    import mprgen
    z = mprgen.gaussian_field(24, 24, 4.0, 7, 50.0, 10.0)
    known = mprgen.mask_random(24, 24, 0.33, 8).astype(bool)
    phi_s, _, _ = mpr.transform(z, known)
    e_s, _, _ = mpr.sample_specific_energy(phi_s, known, 0.5)
    T = 4.0 * (1.0 + e_s)                           # low-T harmonic estimate
    out = mpr.fill(z, known, T, 40, 40, 2, seed=9, chains=2)
    assert out["records"] == 40
    assert np.array_equal(out["z_hat"][known], z[known])
    assert np.all(out["z_std"][known] == 0)
    err = mpr.mae(z, out["z_hat"], ~known)
    assert err < 0.5 * np.abs(z[~known] - z[known].mean()).mean()


# ---------------------------------------------------------------- Sec. 2.3
def test_match_T_inverts_a_power_law_table():
    # eps = T/4 is a straight line in (log T, log eps); PCHIP reproduces it
    T = np.logspace(-6, 0, 25)
    e = T / 4.0 - 1.0
    for es in (-1 + 3e-6, -1 + 1e-4, -0.9, -0.75 - 1e-9):
        That, st = mpr.match_T(es, T, e)
        assert st[0] == 0
        assert That[0] == pytest.approx(4.0 * (1.0 + es), rel=1e-12)


def test_match_T_nodes_monotone_and_clamped():
    T = np.logspace(-5, 0.5, 23)
    eps = T / 4.0 / (1 + T) + 0.05 * T ** 2 / (1 + T ** 2)
    e = eps - 1.0
    That, st = mpr.match_T(e, T, e)
    np.testing.assert_allclose(That, T, rtol=1e-12)
    assert np.all(st == 0)
    grid = np.linspace(e[0], e[-1], 400)[1:-1]
    That, _ = mpr.match_T(grid, T, e)
    assert np.all(np.diff(That) > 0)
    That, st = mpr.match_T([e[0] - 0.01, e[-1] + 0.01], T, e)
    assert list(That) == [T[0], T[-1]] and list(st) == [1, 1]


def test_site_words_distinct_across_sites_and_sweeps():
    # Every (site, sweep) draws its own (u, r): a pair's two sites, two
    # sweeps of one site and two chains never share a word pair (48 random
    # bits, so a chance collision among these 9600 draws is negligible),
    # and the u of a pair's two sites and of one site in consecutive sweeps
    # are uncorrelated.
    ny, nx = 40, 40
    draws = []
    for sweep in (6, 7, 8):
        u, r = mpr.site_uniforms(11, ny, nx, sweep, [0, 1], 3)
        draws.append((u, r))
    keys = np.concatenate([(u * 2.0 ** 24).astype(np.int64).ravel() * 2 ** 24 + (r * 2.0 ** 24).astype(np.int64).ravel()
                           for u, r in draws])
    assert len(np.unique(keys)) == keys.size
    u0 = draws[0][0][0]
    first = u0[0::4, :].ravel()
    second = u0[2::4, :].ravel()
    assert abs(np.corrcoef(first, second)[0, 1]) < 0.1
    assert abs(np.corrcoef(draws[0][0].ravel(), draws[1][0].ravel())[0, 1]) < 0.1
    assert abs(u0.mean() - 0.5) < 0.03
