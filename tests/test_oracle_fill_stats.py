"""Pins of the oracle's prediction statistics (Algorithm 2, steps 5.3 and 6:
the conditional mean and std pooled over every recorded state of every
chain, mapped back by the inverse of Eq. (2)) and of the windowed a-rule
(Algorithm 2, step 4.2, applied every adapt_every sweeps to the window's
mean acceptance).  Each expected value comes from a closed form, an exact
law by quadrature, or a sequence derived by hand, not from the oracle."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import mpr

TWO_PI = 2.0 * math.pi


def _isolated_gaps(n=9):
    """n x n grid whose gap sites (odd y, odd x) have only sample sites as
    neighbours, so that every gap is a single free site."""
    known = np.ones((n, n), dtype=bool)
    known[1::2, 1::2] = False
    return known


def test_fill_statistics_at_infinite_temperature():
    # At T = inf with a = 1 every proposal is accepted and is uniform on the
    # circle (Algorithm 1, steps 2-6 with beta = 0), so every recorded gap
    # state is iid U[0, 2 pi): z_hat has mean z_min + span / 2 and spread
    # span / sqrt(12 m) over the gaps, m = records x chains, and the pooled
    # population variance has mean (m - 1) / m * span^2 / 12.
    rng = np.random.default_rng(3)
    ny, nx = 40, 48
    known = rng.random((ny, nx)) < 0.05
    z = rng.normal(50.0, 10.0, (ny, nx))
    chains, n_samp, stride = 3, 8, 2
    out = mpr.fill(z, known, np.inf, 1, n_samp, stride, seed=21, chains=chains)
    m = chains * (n_samp // stride)
    assert out["records"] == m
    zmin, zmax = z[known].min(), z[known].max()
    span = zmax - zmin
    gap = ~known
    zh, zs = out["z_hat"][gap], out["z_std"][gap]
    n = zh.size
    sd_site = span / math.sqrt(12.0 * m)           # std of one site's z_hat
    assert abs(zh.mean() - (zmin + span / 2)) <= 4 * sd_site / math.sqrt(n)
    # spread of z_hat over the sites: chi-square with n - 1 degrees of freedom
    assert zh.var(ddof=1) / sd_site ** 2 == pytest.approx(1.0, abs=4 * math.sqrt(2.0 / (n - 1)))
    # pooled population variance: the mean of s^2 over m iid uniforms is
    # (m - 1)/m sigma^2; its variance is sigma^4 (kurt - (m - 3)/(m - 1)) / m
    # with kurtosis 9/5 for the uniform law
    sig2 = span ** 2 / 12.0
    v = zs ** 2
    sd_v = sig2 * (m - 1) / m * math.sqrt((1.8 - (m - 3) / (m - 1)) / m) / math.sqrt(n)
    assert abs(v.mean() - (m - 1) / m * sig2) <= 4 * sd_v
    # the sample-variance reading (m - 1 in the denominator) is excluded
    assert abs(v.mean() - sig2) > 4 * sd_v
    # samples are copied through with std 0
    assert np.array_equal(out["z_hat"][known], z[known]) and np.all(out["z_std"][known] == 0)


@pytest.mark.parametrize("T", [0.3, 1.0])
def test_fill_matches_the_exact_single_site_law(T):
    # Isolated gap sites are independent single free sites: each one's
    # conditional mean and variance follow from the exact density by
    # quadrature.  Records within a chain are correlated, so the tolerance
    # treats each chain as one sample.
    known = _isolated_gaps(9)
    rng = np.random.default_rng(11)
    z = rng.uniform(10.0, 20.0, known.shape)
    z[0, 0], z[0, 2] = 10.0, 20.0                   # fix z_min, z_max
    chains = 400
    out = mpr.fill(z, known, T, 20, 40, 4, seed=5, chains=chains)
    phi_s, zmin, zmax = mpr.transform(z, known)
    span = zmax - zmin
    for y, x in zip(*np.nonzero(~known)):
        nb = [phi_s[y - 1, x], phi_s[y + 1, x], phi_s[y, x - 1], phi_s[y, x + 1]]
        mean, var = exact.single_site_moments(nb, 1.0 / T, 0.5)
        zm = zmin + span * mean / TWO_PI
        zsd = span * math.sqrt(var) / TWO_PI
        assert abs(out["z_hat"][y, x] - zm) <= 4 * zsd / math.sqrt(chains), (y, x)
        assert out["z_std"][y, x] == pytest.approx(zsd, rel=4 * math.sqrt(2.0 / chains)), (y, x)


def test_fill_pools_every_recorded_state_of_every_chain():
    # The same sweeps run by hand, every stride-th sampling state kept
    # explicitly; z_hat and z_std are the mean and population std of the
    # stacked back-transformed states.  Pins which sweeps are recorded, a = 1
    # while sampling and the pooling over chains.
    import mprgen
    z = mprgen.gaussian_field(20, 24, 4.0, 17, 50.0, 10.0)
    known = mprgen.mask_random(20, 24, 0.5, 18).astype(bool)
    T, n_eq, n_samp, stride, chains, seed = 0.02, 6, 9, 3, 4, 33
    out = mpr.fill(z, known, T, n_eq, n_samp, stride, seed=seed, chains=chains)
    phi_s, zmin, zmax = mpr.transform(z, known)
    ids = np.arange(chains)
    phi = mpr.hot_start(phi_s, known, seed, ids, 0)
    phi, a, _, _ = mpr.run_sweeps(phi, known, T, np.ones(chains), 0.5, seed, 0, n_eq, ids, 0, adapt=True)
    kept = []
    for j in range(n_samp):
        phi, _, _, _ = mpr.run_sweeps(phi, known, T, np.ones(chains), 0.5, seed, n_eq + j, 1, ids, 0)
        if j % stride == stride - 1:
            kept.append(mpr.inverse_transform(phi, zmin, zmax))
    stack = np.concatenate(kept, axis=0)          # (records x chains, ny, nx)
    assert stack.shape[0] == out["records"] == chains * (n_samp // stride)
    gap = ~known
    np.testing.assert_allclose(out["z_hat"][gap], stack.mean(axis=0)[gap], rtol=0, atol=1e-9)
    np.testing.assert_allclose(out["z_std"][gap], stack.std(axis=0)[gap], rtol=0, atol=1e-6)
    np.testing.assert_array_equal(out["a_eq"], a)


def _window_run(adapt_every, T_seq):
    """Sweeps of a grid of isolated gaps, each sweep a call of its own at
    temperature T_seq[i]; before every T = 0 sweep the gaps are put back at
    their unique energy minimum, so that sweep accepts nothing, while a
    T = inf sweep accepts everything.  Returns a after each sweep."""
    known = _isolated_gaps(7)
    theta = 1.0
    phi_min = np.full((1,) + known.shape, theta)
    phi = phi_min.copy()
    a = np.ones(1)
    window = np.zeros(1)
    seq = []
    for i, T in enumerate(T_seq):
        if T == 0.0:
            phi = phi_min.copy()
        phi, a, acc, _ = mpr.run_sweeps(phi, known, T, a, 0.5, 77, i, 1, [0], 0, adapt=True,
                                        adapt_every=adapt_every, window=window)
        assert acc[0, 0] == (1.0 if T == np.inf else 0.0)
        seq.append(float(a[0]))
    return seq


def test_windowed_a_rule_by_hand():
    inf = np.inf
    # acceptances 1, 1, 0 | 0, 0, 1 | 0, 0, 0; k_a = 3, A_targ = 0.3
    T_seq = [inf, inf, 0.0, 0.0, 0.0, inf, 0.0, 0.0, 0.0]
    # adapt_every = 3: the window means 2/3 and 1/3 leave a at 1; the third
    # window's mean 0 gives a = 1 + 9/3 after sweep i = 8.  (Its last value
    # would have changed a after sweep 2, its first after sweep 5.)
    assert _window_run(3, T_seq) == [1, 1, 1, 1, 1, 1, 1, 1, 4.0]
    # adapt_every = 1 (the paper): a = 1 + (i + 1)/3 after every sweep i with
    # acceptance 0, unchanged after one with acceptance 1
    expect = [1, 1, 2.0, 1 + 4 / 3, 1 + 5 / 3, 1 + 5 / 3, 1 + 7 / 3, 1 + 8 / 3, 4.0]
    np.testing.assert_allclose(_window_run(1, T_seq), expect, rtol=0, atol=1e-15)
    # adapt_every = 2: windows (1, 1), (0, 0), (0, 1), (0, 0) -> a changes
    # after sweep 3 (mean 0) and sweep 7 (mean 0), not after sweep 5 (1/2)
    expect2 = [1, 1, 1, 1 + 4 / 3, 1 + 4 / 3, 1 + 4 / 3, 1 + 4 / 3, 1 + 8 / 3, 1 + 8 / 3]
    np.testing.assert_allclose(_window_run(2, T_seq), expect2, rtol=0, atol=1e-15)
