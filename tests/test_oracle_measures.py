"""Pins of the oracle's validation measures (Sec. 3.3): a hand-computed
example, the perfect prediction, and the correlation coefficient as the
library routine computes it."""
import math

import numpy as np
import pytest

from oracle import mpr


def test_hand_example():
    # Z = (1, 2, 4, 5), Z_hat = (2, 2, 3, 6): eps = (-1, 0, 1, -1).
    # AAE = 3/4; ARE = (-1 + 0 + 1/4 - 1/5)/4; AARE = (1 + 0 + 1/4 + 1/5)/4;
    # RASE = sqrt(3/4); centred Z = (-2, -1, 1, 2), centred Z_hat =
    # (-5, -5, -1, 11)/4: R = 9 / sqrt(10 * 10.75).
    z = np.array([[1.0, 2.0], [4.0, 5.0]])
    zh = np.array([[2.0, 2.0], [3.0, 6.0]])
    m = mpr.validation_measures(z, zh, np.ones((2, 2), bool))
    assert m["P"] == 4
    assert m["AAE"] == pytest.approx(0.75, abs=1e-15)
    assert m["ARE"] == pytest.approx(-0.2375, abs=1e-15)
    assert m["AARE"] == pytest.approx(0.3625, abs=1e-15)
    assert m["RASE"] == pytest.approx(math.sqrt(0.75), abs=1e-15)
    assert m["R"] == pytest.approx(9.0 / math.sqrt(107.5), abs=1e-15)


def test_only_prediction_sites_count():
    rng = np.random.default_rng(1)
    z = rng.normal(50, 10, (30, 30))
    zh = z + rng.normal(0, 2, (30, 30))
    gaps = rng.random((30, 30)) < 0.4
    zh_other = np.where(gaps, zh, -1e6)              # values at samples are ignored
    a = mpr.validation_measures(z, zh, gaps)
    b = mpr.validation_measures(z, zh_other, gaps)
    assert a == b and a["P"] == int(gaps.sum())
    assert a["R"] == pytest.approx(np.corrcoef(z[gaps], zh[gaps])[0, 1], rel=1e-12)
    assert a["RASE"] >= a["AAE"]                     # quadratic mean >= mean


def test_perfect_prediction():
    rng = np.random.default_rng(2)
    z = rng.normal(50, 10, (20, 20))
    m = mpr.validation_measures(z, z, np.ones_like(z, bool))
    assert m["AAE"] == 0 and m["ARE"] == 0 and m["AARE"] == 0 and m["RASE"] == 0
    assert m["R"] == pytest.approx(1.0, abs=1e-15)
