"""Pins of the oracle's GMRF variant (Sec. 4.4): pair interaction
H_ij = 1 - dphi^2 / (2 pi^2).  Hand-computed energies, the reflection's
energy conservation and involution, the exact single-site law (a truncated
normal, closed form in erf), T -> 0 monotonicity, the literal loop, and the
equipartition of the harmonic model at low temperature."""
import math

import numpy as np
import pytest

from oracle import exact, mpr
from tests.test_oracle_pins import chi2_pvalue

TWO_PI = 2.0 * math.pi
G = mpr.GMRF


def test_hand_energies():
    # two sites pi apart: H_12 = 1 - pi^2 / (2 pi^2) = 1/2, H = -1/2
    phi = np.array([[0.0, math.pi]])
    assert mpr.energy(phi, 0.5, G) == pytest.approx(-0.5, abs=1e-15)
    e, eps = mpr.state_specific_energy(phi, 0.5, G)
    assert e == pytest.approx(-0.5) and eps == pytest.approx(0.5)
    # 2 x 2 grid (0, 1 / 2, 2): the four bonds' dphi^2 = 1, 4, 1, 4 (rows, then columns: (0,1), (2,3), (0,2), (1,3))
    phi = np.array([[0.0, 1.0], [2.0, 3.0]])
    want = sum(d * d / (2 * math.pi ** 2) - 1 for d in (1.0, 1.0, 2.0, 2.0))
    assert mpr.energy(phi, 0.5, G) == pytest.approx(want, abs=1e-14)
    # the sample specific energy counts only sample-sample pairs
    known = np.array([[True, True], [False, True]])
    es, eps_s, n = mpr.sample_specific_energy(phi, known, 0.5, G)
    assert n == 2 and es == pytest.approx((1.0 + 4.0) / (2 * math.pi ** 2) / 2 - 1, abs=1e-15)


def test_reflection_conserves_energy_and_is_an_involution():
    rng = np.random.default_rng(4)
    for _ in range(50):
        nb = list(rng.uniform(0, TWO_PI, rng.integers(1, 5)))
        nbrs = [np.array([v]) for v in nb] + [np.array([np.nan])] * (4 - len(nb))
        phi = np.array([rng.uniform(0, TWO_PI)])
        star = mpr.over_relax(phi, nbrs, 0.5, G)
        if star[0] != phi[0]:
            assert mpr.site_energy(star, nbrs, 0.5, G)[0] == pytest.approx(
                mpr.site_energy(phi, nbrs, 0.5, G)[0], abs=1e-12)
            assert mpr.over_relax(star, nbrs, 0.5, G)[0] == pytest.approx(phi[0], abs=1e-12)
        else:
            assert not (0.0 <= 2 * np.mean(nb) - phi[0] < TWO_PI)


@pytest.mark.parametrize("shape", [(3, 3), (4, 5), (9, 7)])
def test_vectorised_sweep_matches_literal_loop(shape):
    ny, nx = shape
    rng = np.random.default_rng(ny * 13 + nx)
    known = rng.random(shape) < 0.35
    known.flat[0] = True
    phi_s, _, _ = mpr.transform(rng.normal(size=shape), known)
    phi = mpr.hot_start(phi_s, known, 5, [1], 0)
    for T, a in ((0.05, 1.0), (0.01, 5.0), (math.inf, 1.0), (0.0, 2.0)):
        beta = 0.0 if T == math.inf else (math.inf if T == 0 else 1 / T)
        for or_step in (True, False):
            v, acc = mpr.hybrid_sweep(phi, known, [beta], [TWO_PI / a], 0.5, 5, 2, [1], 0, or_step=or_step, model=G)
            l, acc2 = mpr.hybrid_sweep_literal(phi[0], known, beta, TWO_PI / a, 0.5, 5, 2, 1, 0, or_step=or_step,
                                               model=G)
            assert np.abs(v[0] - l).max() <= 1e-13 and acc[0] == acc2


@pytest.mark.parametrize("T,a", [(0.05, 1.0), (0.3, 1.0), (0.05, 4.0)])
def test_3x3_checkerboard_frozen_exact(T, a):
    q, C = 0.5, 4096
    known = np.zeros((3, 3), bool)
    for y, x in ((0, 0), (0, 2), (1, 1), (2, 0), (2, 2)):
        known[y, x] = True
    vals = np.zeros((3, 3))
    vals[0, 0], vals[0, 2], vals[1, 1], vals[2, 0], vals[2, 2] = 0.3, 2.0, 3.5, 4.5, 6.0
    phi0 = np.broadcast_to(vals, (C, 3, 3)).copy()
    phi, _, _, _ = mpr.run_sweeps(phi0, known, T, a, q, 4000 + int(T * 100), 0, 80, np.arange(C), 0, model=G)
    for (y, x), nb in (((0, 1), ((0, 0), (0, 2), (1, 1))), ((1, 0), ((0, 0), (2, 0), (1, 1))),
                       ((1, 2), ((0, 2), (2, 2), (1, 1))), ((2, 1), ((2, 0), (2, 2), (1, 1)))):
        probs = exact.gmrf_single_site_bins([vals[k] for k in nb], 1.0 / T, nbins=8)
        counts, _ = np.histogram(phi[:, y, x], bins=8, range=(0, TWO_PI))
        assert chi2_pvalue(counts, probs) > 1e-3, ((y, x), counts, probs * C)


def test_exact_law_reduces_to_uniform_and_to_a_point():
    assert np.allclose(exact.gmrf_single_site_bins([1.0, 2.0], 0.0), np.full(8, 1 / 8))
    p = exact.gmrf_single_site_bins([1.0, 1.2], 1e6, nbins=8)     # sd ~ 2e-3 about 1.1: bin 1 of [0, 2 pi)
    assert p[1] > 1 - 1e-12


def test_zero_temperature_energy_never_increases():
    rng = np.random.default_rng(21)
    n = 12
    known = rng.random((n, n)) < 0.3
    phi_s, _, _ = mpr.transform(rng.normal(size=(n, n)), known)
    phi = mpr.hot_start(phi_s, known, 4, np.arange(3), 0)
    prev = mpr.energy(phi, 0.5, G)
    for s in range(25):
        phi, _ = mpr.hybrid_sweep(phi, known, [math.inf] * 3, [TWO_PI / 2] * 3, 0.5, 4, s, np.arange(3), 0, model=G)
        cur = mpr.energy(phi, 0.5, G)
        assert np.all(cur <= prev + 1e-12)
        prev = cur


def test_low_temperature_equipartition():
    # The GMRF energy is exactly quadratic: at low T (angles far from 0 and
    # 2 pi) each of the N - 1 non-uniform modes of an unconditional grid
    # holds T/2, so 1 + e = (N - 1) T / (2 N_GP).
    L, C, T = 8, 64, 2e-4
    known = np.zeros((L, L), bool)
    phi = np.full((C, L, L), math.pi)
    phi, a, _, _ = mpr.run_sweeps(phi, known, T, 20.0, 0.5, 3, 0, 200, np.arange(C), 0, adapt=True, model=G)
    _, _, _, e = mpr.run_sweeps(phi, known, T, a, 0.5, 3, 200, 400, np.arange(C), 0, trace_energy=True, model=G)
    want = (L * L - 1) * T / (2 * mpr.n_pairs(L, L))
    got = 1.0 + e.mean()
    se = (1.0 + e).mean(axis=0).std(ddof=1) / math.sqrt(C)
    assert abs(got - want) < 4 * se + 1e-3 * want, (got, want, se)
