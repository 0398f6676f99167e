"""Pins of the oracle's choice of q by cross-validation (Sec. 6) and of its
inputs: the fold generator, the fold masks, the pooled score and the tie
rule by hand; the e(T) tables of every candidate q against the closed forms
that fix them (low-temperature equipartition, the same slope for every q,
and the infinite-temperature limit 1 + e = 1 - (sin(pi q) / (pi q))^2);
and the harmonic limit of the whole procedure: on smooth data T-hat grows
as q^2 and the fitted conditional law, hence the prediction, does not
depend on q."""
import math

import numpy as np
import pytest

import mprgen
from oracle import exact
from oracle import mpr as om
from oracle.etable import load_table
from tests.test_oracle_pins import chi2_pvalue, run_chains

QS = [0.125, 0.25, 0.375, 0.5]


def test_folds_partition_the_samples():
    known = mprgen.mask_random(30, 31, 0.35, 4)
    for k in (2, 3, 5):
        fold = mprgen.cv_folds(known, k, 9)
        assert fold.dtype == np.uint8 and fold.shape == known.shape
        assert np.all(fold[known == 0] == 255)
        ids = fold[known == 1]
        assert ids.max() == k - 1
        counts = np.bincount(ids, minlength=k)
        assert counts.sum() == int(known.sum()) and counts.max() - counts.min() <= 1
        assert np.array_equal(fold, mprgen.cv_folds(known, k, 9))
    assert not np.array_equal(mprgen.cv_folds(known, 3, 1), mprgen.cv_folds(known, 3, 2))
    with pytest.raises(ValueError):
        mprgen.cv_folds(known, 1, 0)


def test_masks_by_hand():
    known = np.array([[1, 0, 1], [1, 1, 0]], dtype=np.uint8)
    fold = np.array([[0, 255, 1], [1, 0, 255]], dtype=np.uint8)
    train, held = om.cv_masks(known, fold, 1)
    assert train.tolist() == [[True, False, False], [False, True, False]]
    assert held.tolist() == [[False, False, True], [True, False, False]]
    # a sample whose fold id is out of range is never held out
    fold2 = np.array([[0, 255, 7], [1, 0, 255]], dtype=np.uint8)
    train, held = om.cv_masks(known, fold2, 1)
    assert train[0, 2] and not held[0, 2]


def test_pooled_score_by_hand():
    # fold 1: |eps| = 1, 2 -> sum 3, sum eps^2 5; fold 2: eps = -1
    aae, rase = om.cv_pool([(3.0, 5.0, 2), (1.0, 1.0, 1)])
    assert aae == pytest.approx(4.0 / 3.0, abs=1e-15) and rase == pytest.approx(math.sqrt(2.0), abs=1e-15)
    with pytest.raises(om.OracleError):
        om.cv_pool([(0.0, 0.0, 0)])


def test_tie_rule():
    assert om.cv_best([0.125, 0.25, 0.5], [3.0, 2.0, 2.5]) == 1
    assert om.cv_best([0.125, 0.25, 0.5], [2.0, 3.0, 2.0]) == 2
    assert om.cv_best([0.5, 0.25], [1.0, 1.0]) == 0


@pytest.mark.parametrize("q", QS)
def test_tables_of_every_q(q):
    T, e, err = load_table(q=q)
    L = 32
    assert np.all(np.diff(T) > 0) and np.all(np.diff(e) > 0)
    eps = 1.0 + e
    # harmonic limit of Eq. (3): 1 - cos(q d) ~ q^2 d^2 / 2 has one zero
    # mode, so eps = (N - 1) T / (2 N_GP) = (L + 1) T / (4 L) for any q
    low = T < 1e-3
    ratio = eps[low] / ((L + 1) * T[low] / (4 * L))
    assert np.all(np.abs(ratio - 1.0) < 0.01), ratio
    # T = infinity: independent uniform angles, E cos(q (u - v)) = (sin(pi q) / (pi q))^2
    e_inf = -(math.sin(math.pi * q) / (math.pi * q)) ** 2
    assert np.all(e < e_inf)
    assert np.all(err < 1e-2 * eps + 1e-12)  # statistical error of the table below 1 % of 1 + e


def test_harmonic_limit_q_does_not_matter_on_smooth_data():
    # Smooth data give small angle steps: e_s(q) ~ -1 + q^2 <dphi^2>_s / 2,
    # and the tables' eps ~ (L + 1) T / (4 L), so T-hat ~ q^2; the site law
    # exp(-sum (1 - cos q dphi) / T-hat) ~ exp(-sum q^2 dphi^2 / (2 T-hat))
    # is then the same for every q, and so is the cross-validated error.
    z = mprgen.gaussian_field(20, 20, 6.0, 5, 50.0, 10.0)
    known = mprgen.mask_random(20, 20, 0.3, 6)
    fold = mprgen.cv_folds(known, 3, 7)
    tables = [load_table(q=q)[:2] for q in QS]
    out = om.cv_select_q(z, known, fold, 3, QS, tables, n_eq=60, n_samp=120, stride=2, seed=5, chains=4)
    r = out["T"] / np.asarray(QS)[:, None] ** 2
    assert np.all(np.abs(r / r[-1] - 1.0) < 0.02), r
    # the scores then differ only by Monte Carlo noise (~1 % here)
    assert np.all(np.abs(out["aae"] / out["aae"][-1] - 1.0) < 0.05), out["aae"]


@pytest.mark.parametrize("q,T", [(0.25, 0.1), (0.125, 0.02), (0.375, 0.5)])
def test_sweep_exact_law_at_other_q(q, T):
    # 3 x 3, colour-0 sites frozen: each edge site samples exactly
    # exp(sum_j cos(q (phi - phi_j)) / T) on [0, 2 pi)
    C = 4096
    known = np.zeros((3, 3), bool)
    vals = np.zeros((3, 3))
    for (y, x), v in zip(((0, 0), (0, 2), (1, 1), (2, 0), (2, 2)), (0.3, 2.0, 3.5, 4.5, 6.0)):
        known[y, x] = True
        vals[y, x] = v
    phi = run_chains(known, np.broadcast_to(vals, (C, 3, 3)).copy(), T, 1.0, q, 3000 + int(q * 1000), 60)
    for (y, x), nb in (((0, 1), ((0, 0), (0, 2), (1, 1))), ((1, 0), ((0, 0), (2, 0), (1, 1))),
                       ((1, 2), ((0, 2), (2, 2), (1, 1))), ((2, 1), ((2, 0), (2, 2), (1, 1)))):
        probs = exact.single_site_bins([vals[k] for k in nb], 1.0 / T, q, nbins=8)
        counts, _ = np.histogram(phi[:, y, x], bins=8, range=(0, 2 * math.pi))
        assert chi2_pvalue(counts, probs) > 1e-3, ((y, x), counts, probs * C)
