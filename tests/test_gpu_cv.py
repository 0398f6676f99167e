"""Per-grid q (mpr_set_grid_q) and the choice of q by cross-validation
(mpr_cv_select_q) on the GPU against the oracle, through the C ABI.

Sweeps of a batch whose grids carry different q are teacher-forced against
the oracle at each grid's q (FP64 1e-5 rad; FP32 flips explained by a
decision within 1e-4 of its threshold); specific energies to 1e-12; the
whole cross-validation in FP64 against the oracle's (same fits, same random
streams): scores to 1e-9 relative and the same chosen q."""
import math

import numpy as np
import pytest

import mprgen
from oracle import mpr as om
from oracle.etable import load_table
from tests.gpu_util import (TWO_PI, as_fp32_state, beta_of, chain_margins, explainable, fp32_cap, make_field,
                            mismatches, oracle_init, random_grid)

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64), (45, 67), (1, 9), (3, 3), (130, 33)]
QS = [0.125, 0.25, 0.375, 0.5, 0.3]


def _grids(seed, chains=2):
    return [(*random_grid(ny, nx, 0.4, seed + 10 * k, smooth=True), chains) for k, (ny, nx) in enumerate(SHAPES)]


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_specific_energies_per_grid_q(dtype):
    grids = _grids(3)
    f = make_field(grids, dtype=dtype, seed=4)
    f.set_grid_q(QS)
    e, n = f.specific_energy(0)
    es_state, _ = f.specific_energy(1)
    tol = 1e-12 if dtype == "fp64" else 2e-6
    k = 0
    for g, (z, known, chains) in enumerate(grids):
        phi0 = oracle_init(z, known, 4, 0, g, dtype)
        try:
            _, eps, ns = om.sample_specific_energy(phi0, known.astype(bool), QS[g])
            assert n[g] == ns and abs((1 + e[g]) - eps) <= tol * eps + 1e-15, (g, e[g], eps)
        except om.OracleError:
            assert math.isnan(e[g])
        for c in range(chains):
            _, eps = om.state_specific_energy(oracle_init(z, known, 4, c, g, dtype), QS[g])
            assert abs((1 + es_state[k]) - eps) <= tol * eps, (g, c)
            k += 1
    f.close()


@pytest.mark.parametrize("dtype,nsw", [("fp64", 2), ("fp32", 1)])
def test_teacher_forced_sweep_per_grid_q(dtype, nsw):
    grids = _grids(21)
    seed, sweep_index = 77, 11
    f = make_field(grids, dtype=dtype, seed=seed, tile_x=32, tile_y=24, sweeps_per_pass=nsw)
    f.set_grid_q(QS)
    total_bad = total_gap = 0
    for T, a in [(0.3, 1.0), (0.02, 5.0), (1e-3, 40.0)]:
        states = []
        for g, (z, known, chains) in enumerate(grids):
            phi = np.stack([oracle_init(z, known, seed, c, g, "fp64") for c in range(chains)])
            phi, _, _, _ = om.run_sweeps(phi, known.astype(bool), 0.05, 2.0, QS[g], seed, 0, 2, np.arange(chains), g)
            if dtype == "fp32":
                phi = np.stack([as_fp32_state(p, known) for p in phi])
            states.append(phi)
            for c in range(chains):
                f.set_phi(phi[c], g, c)
        f.set_chain_state(sweep_index, np.full(f.total_chains, a))
        f.sweep(nsw, np.full(len(grids), T))
        for g, (z, known, chains) in enumerate(grids):
            phi, sweep_margins = states[g], []
            for s in range(nsw):
                margins = {}
                phi, _ = om.hybrid_sweep(phi, known.astype(bool), [beta_of(T)] * chains, [TWO_PI / a] * chains,
                                         QS[g], seed, sweep_index + s, np.arange(chains), g, margins=margins)
                sweep_margins.append(margins)
            for c in range(chains):
                got = f.get_phi(g, c).cpu().numpy()
                if dtype == "fp64":
                    assert np.abs(got - phi[c]).max() <= 1e-5, (T, a, g, c)
                else:
                    expl = explainable([chain_margins(m, c) for m in sweep_margins])
                    n_bad, _, unexpl = mismatches(got, phi[c], expl, known, 1e-3)
                    assert len(unexpl) == 0, (T, a, g, c, unexpl[:5])
                    total_bad += n_bad
                    total_gap += int((~known.astype(bool)).sum())
    assert total_bad <= fp32_cap(total_gap), (total_bad, total_gap)
    f.close()


def test_set_grid_q_validation():
    from paper_1710_03038_amd import mpr as M
    grids = _grids(5)[:2]
    f = make_field(grids, dtype="fp64", seed=1)
    for bad in ([0.0, 0.5], [0.25, 0.51]):
        with pytest.raises(M.MPRError) as ei:
            f.set_grid_q(bad)
        assert ei.value.status == M.MPR_E_ARG
    f.close()
    f = make_field(grids, dtype="fp64", seed=1, model="gmrf")
    with pytest.raises(M.MPRError) as ei:
        f.set_grid_q([0.25, 0.25])
    assert ei.value.status == M.MPR_E_STATE
    f.close()


def _cv_inputs(ny=24, nx=20, seed=3, n_folds=3):
    z = mprgen.matern_field(ny, nx, 0.5, 0.5, seed, mean=50.0, std=10.0)
    known = mprgen.mask_random(ny, nx, 0.4, seed + 1)
    fold = mprgen.cv_folds(known, n_folds, seed + 2)
    return z, known, fold


def test_cross_validation_matches_oracle_fp64():
    import torch

    from paper_1710_03038_amd import mpr as M
    z, known, fold = _cv_inputs()
    qs = [0.125, 0.25, 0.5]
    tables = [load_table(q=q)[:2] for q in qs]
    kw = dict(n_eq=20, n_samp=10, stride=2)
    dev = torch.device("cuda:0")
    got = M.cv_select_q(torch.from_numpy(z).to(dev), torch.from_numpy(known).to(dev), torch.from_numpy(fold).to(dev),
                        3, qs, tables, params=M.default_params(dtype="fp64", seed=11), chains=2, **kw)
    ref = om.cv_select_q(z, known, fold, 3, qs, tables, seed=11, chains=2, **kw)
    np.testing.assert_allclose(got["aae"], ref["aae"], rtol=1e-9)
    np.testing.assert_allclose(got["rase"], ref["rase"], rtol=1e-9)
    np.testing.assert_allclose(got["T_mean"], ref["T"].mean(axis=1), rtol=1e-12)
    assert got["best"] == ref["best"]


def test_cross_validation_errors_and_fp32_run():
    import torch

    from paper_1710_03038_amd import mpr as M
    z, known, fold = _cv_inputs(48, 40, seed=8, n_folds=4)
    dev = torch.device("cuda:0")
    zt, kt = torch.from_numpy(z).to(dev), torch.from_numpy(known).to(dev)
    qs = [0.25, 0.5]
    tables = [load_table(q=q)[:2] for q in qs]
    out = M.cv_select_q(zt, kt, torch.from_numpy(fold).to(dev), 4, qs, tables, 20, 20, 2,
                        params=M.default_params(dtype="fp32", seed=2))
    assert out["best"] in (0, 1) and np.all(np.isfinite(out["aae"])) and np.all(out["rase"] >= out["aae"])
    # a fold with no held-out sample
    empty = np.where(fold == 3, 0, fold).astype(np.uint8)
    with pytest.raises(M.MPRError) as ei:
        M.cv_select_q(zt, kt, torch.from_numpy(empty).to(dev), 4, qs, tables, 20, 20, 2)
    assert ei.value.status == M.MPR_E_DEGENERATE
