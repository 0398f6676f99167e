"""The seeded input generators: covariance functions against closed forms,
sampled fields against their covariance, masks against their definition."""
import math

import numpy as np
import pytest

import mprgen


def test_matern_correlation_closed_forms():
    h = np.linspace(0.0, 20.0, 81)
    for kappa in (0.2, 0.5, 1.3):
        np.testing.assert_allclose(mprgen.matern_corr(h, kappa, 0.5), np.exp(-kappa * h), rtol=1e-12)
        np.testing.assert_allclose(mprgen.matern_corr(h, kappa, 1.5), (1 + kappa * h) * np.exp(-kappa * h),
                                   rtol=1e-12)
    c = mprgen.matern_corr(h, 0.5, 0.25)
    assert c[0] == 1.0 and np.all(np.diff(c) < 0)


@pytest.mark.parametrize("kappa,nu", [(0.5, 0.5), (0.2, 0.25)])
def test_matern_field_matches_its_covariance(kappa, nu):
    z = mprgen.matern_field(256, 256, kappa, nu, 11, mean=50.0, std=10.0)
    assert z.shape == (256, 256)
    y = (z - 50.0) / 10.0
    for lag in (1, 2, 4):
        emp = 0.5 * ((y[:, lag:] * y[:, :-lag]).mean() + (y[lag:, :] * y[:-lag, :]).mean())
        want = float(mprgen.matern_corr(np.array([lag]), kappa, nu)[0])
        assert abs(emp - want) < 0.06, (lag, emp, want)
    assert abs(y.var() - 1.0) < 0.15


def test_squared_exponential_field_matches_its_covariance():
    z = mprgen.gaussian_field(256, 256, 4.0, 5)
    for lag in (1, 4):
        emp = 0.5 * ((z[:, lag:] * z[:, :-lag]).mean() + (z[lag:, :] * z[:-lag, :]).mean())
        assert abs(emp - math.exp(-lag * lag / 32.0)) < 0.1, lag


def test_random_mask_removes_exactly_floor_pN():
    for p in (0.0, 0.33, 0.5, 0.9):
        known = mprgen.mask_random(37, 41, p, 3)
        assert known.dtype == np.uint8
        assert int((known == 0).sum()) == math.floor(p * 37 * 41)


def test_single_block_mask():
    for seed in range(5):
        known = mprgen.mask_block(64, 48, 20, seed)
        gy, gx = np.nonzero(known == 0)
        assert gy.size == 400
        assert gy.max() - gy.min() == 19 and gx.max() - gx.min() == 19
