"""Pins of the oracle's equilibrium detection (Algorithm 2, step 4) and of
its sweep without over-relaxation (the restricted and standard Metropolis
updates the paper compares with the hybrid, Sec. 2.4).

The slope is pinned to exact lines and to an independent Savitzky-Golay
derivative filter, the stopping rule to hand-derived stop points, the
no-over-relaxation sweep to the exact single-site law and to the literal
per-site loop.
"""
import math

import numpy as np
import pytest
from scipy.signal import savgol_coeffs

from oracle import exact, mpr
from tests.test_oracle_pins import chi2_pvalue

TWO_PI = 2.0 * math.pi


@pytest.mark.parametrize("n", [2, 5, 20, 33])
def test_ols_slope_exact_on_lines(n):
    rng = np.random.default_rng(n)
    for _ in range(5):
        m, c = rng.normal(size=2) * 10
        y = m * np.arange(n) + c
        assert mpr.ols_slope(y) == pytest.approx(m, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("n", [5, 21, 41])
def test_ols_slope_is_the_degree_one_savitzky_golay_derivative(n):
    rng = np.random.default_rng(100 + n)
    y = rng.normal(size=n).cumsum()
    sg = savgol_coeffs(n, 1, deriv=1, use="dot") @ y
    assert mpr.ols_slope(y) == pytest.approx(sg, rel=1e-10, abs=1e-12)
    assert mpr.ols_slope(y) == pytest.approx(np.polyfit(np.arange(n), y, 1)[0], rel=1e-10, abs=1e-12)


def test_ols_slope_zero_on_constants_and_palindromes():
    assert mpr.ols_slope(np.full(20, -0.7)) == 0.0
    half = np.random.default_rng(3).normal(size=10)
    assert abs(mpr.ols_slope(np.concatenate([half, half[::-1]]))) < 1e-14
    # batched over leading axes
    y = np.stack([np.arange(6.0), -2 * np.arange(6.0)])
    np.testing.assert_allclose(mpr.ols_slope(y), [1.0, -2.0])


def test_sg_stop_hand_cases():
    n_f, n_fit = 5, 20
    sweeps = np.arange(1, 400)
    # Energy falls by 1 per sweep until it is flat at 40 from sweep 60 on.
    # The window of the check after sweep i + 1 holds sweeps i + 2 - n_fit ..
    # i + 1; it is wholly flat from i = 78, and the first check at or after
    # 78 is i = 80, so the loop ends after 81 sweeps.
    e = np.maximum(100.0 - sweeps, 40.0)
    assert mpr.sg_stop_index(e, n_f, n_fit, 1000) == 81
    # flat from the start: the first check, i = n_fit, stops it
    assert mpr.sg_stop_index(np.full(100, -0.9), n_f, n_fit, 1000) == n_fit + 1
    # rising energy has a positive slope at the first check
    assert mpr.sg_stop_index(0.01 * sweeps, n_f, n_fit, 1000) == n_fit + 1
    # checks only at multiples of n_f: with n_f = 7 the first is i = 21
    assert mpr.sg_stop_index(np.full(100, 1.0), 7, n_fit, 1000) == 22
    # never flat: the loop runs i_max + 1 sweeps
    assert mpr.sg_stop_index(-0.001 * sweeps, n_f, n_fit, 30) == 31
    assert mpr.sg_stop_index(-0.001 * sweeps, n_f, n_fit, 100) == 101
    # too short a series to decide
    assert mpr.sg_stop_index(-0.001 * sweeps[:50], n_f, n_fit, 1000) is None


def _small_case(seed=5, n=14, p_gap=0.6, chains=3):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:n, 0:n]
    z = np.sin(xx / 3.0) + np.cos(yy / 4.0) + 0.1 * rng.normal(size=(n, n))
    known = rng.random((n, n)) >= p_gap
    known.flat[0] = True
    phi_s, _, _ = mpr.transform(z, known)
    phi = mpr.hot_start(phi_s, known, seed, np.arange(chains), 0)
    return known, phi


def test_equilibrate_is_the_sweeps_plus_the_stopping_rule():
    known, phi0 = _small_case()
    C = phi0.shape[0]
    T, q, seed = 0.02, 0.5, 9
    phi, a, n, eq_at, e, acc = mpr.equilibrate(phi0, known, T, np.ones(C), q, seed, 0, np.arange(C), 0,
                                               n_f=5, n_fit=20, i_max=400)
    assert e.shape == (n, C) and acc.shape == (n, C)
    assert np.all(eq_at > 0) and n == eq_at.max()
    for c in range(C):
        assert mpr.sg_stop_index(e[:, c], 5, 20, 400) == eq_at[c]
    # the same sweeps without the checks
    phi2, a2, acc2, e2 = mpr.run_sweeps(phi0, known, T, np.ones(C), q, seed, 0, n, np.arange(C), 0,
                                        adapt=True, trace_energy=True)
    assert np.array_equal(phi, phi2) and np.array_equal(a, a2)
    assert np.array_equal(e, e2) and np.array_equal(acc, acc2)


def test_equilibrate_caps_at_i_max():
    known, phi0 = _small_case(chains=2)
    phi, a, n, eq_at, e, _ = mpr.equilibrate(phi0, known, 0.02, np.ones(2), 0.5, 1, 0, np.arange(2), 0,
                                             n_f=5, n_fit=20, i_max=12)
    assert n == 13 and np.all(eq_at == -1)


@pytest.mark.parametrize("shape", [(3, 3), (4, 5), (9, 7)])
def test_no_over_relaxation_vectorised_matches_literal(shape):
    ny, nx = shape
    rng = np.random.default_rng(ny * 17 + nx)
    known = rng.random(shape) < 0.35
    known.flat[0] = True
    phi_s, _, _ = mpr.transform(rng.normal(size=shape), known)
    phi = mpr.hot_start(phi_s, known, 3, [2], 0)
    for T, a in ((0.2, 1.0), (0.05, 5.0), (math.inf, 1.0)):
        beta = 0.0 if T == math.inf else 1 / T
        v, acc = mpr.hybrid_sweep(phi, known, [beta], [TWO_PI / a], 0.5, 3, 4, [2], 0, or_step=False)
        l, acc2 = mpr.hybrid_sweep_literal(phi[0], known, beta, TWO_PI / a, 0.5, 3, 4, 2, 0, or_step=False)
        assert np.abs(v[0] - l).max() <= 1e-13 and acc[0] == acc2
        h, _ = mpr.hybrid_sweep(phi, known, [beta], [TWO_PI / a], 0.5, 3, 4, [2], 0)
        if T != math.inf:
            assert not np.array_equal(h, v)       # the switch does change the update


@pytest.mark.parametrize("T,a", [(0.1, 1.0), (0.5, 1.0), (0.1, 4.0)])
def test_no_over_relaxation_keeps_the_exact_law(T, a):
    # Metropolis alone has the same stationary law: edge sites of a 3x3 grid
    # with the colour-0 sites frozen follow the exact single-site density.
    q, C = 0.5, 4096
    known = np.zeros((3, 3), bool)
    for y, x in ((0, 0), (0, 2), (1, 1), (2, 0), (2, 2)):
        known[y, x] = True
    vals = np.zeros((3, 3))
    vals[0, 0], vals[0, 2], vals[1, 1], vals[2, 0], vals[2, 2] = 0.3, 2.0, 3.5, 4.5, 6.0
    phi0 = np.broadcast_to(vals, (C, 3, 3)).copy()
    phi, _, _, _ = mpr.run_sweeps(phi0, known, T, a, q, 3000 + int(T * 10), 0, 150, np.arange(C), 0,
                                  or_step=False)
    for (y, x), nb in (((0, 1), ((0, 0), (0, 2), (1, 1))), ((1, 0), ((0, 0), (2, 0), (1, 1)))):
        probs = exact.single_site_bins([vals[k] for k in nb], 1.0 / T, q, nbins=8)
        counts, _ = np.histogram(phi[:, y, x], bins=8, range=(0, TWO_PI))
        assert chi2_pvalue(counts, probs) > 1e-3, ((y, x), counts, probs * C)


def test_hybrid_relaxes_faster_than_standard_metropolis():
    # The paper's comparison (Sec. 2.4): at low T, from the hot start, the
    # hybrid update reaches a lower energy in the same number of sweeps
    # than standard Metropolis (a = 1, no over-relaxation).
    known, phi0 = _small_case(seed=11, n=24, p_gap=0.9, chains=4)
    C, T = phi0.shape[0], 0.01
    _, _, _, e_h = mpr.run_sweeps(phi0, known, T, np.ones(C), 0.5, 4, 0, 60, np.arange(C), 0,
                                  adapt=True, trace_energy=True)
    _, _, _, e_s = mpr.run_sweeps(phi0, known, T, np.ones(C), 0.5, 4, 0, 60, np.arange(C), 0,
                                  or_step=False, trace_energy=True)
    assert np.all(e_h[-1] < e_s[-1])
