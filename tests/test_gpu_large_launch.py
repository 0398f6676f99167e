"""Launches whose work-item count passes 2^32 - 1, the most one launch
dimension counts: the kernels then run on rows of 65536 workgroups and skip
those past their count.  Both cases are compared with the oracle.

* 16384 x 16384 grid in 8 x 8 tiles, 1024-thread sweep workgroups (the
  FP32 default): 2^22 workgroups, 2^32 work-items (the sweep and nothing
  else on two rows).
* 2^24 + 5 chains of a 2 x 2 grid: one workgroup per chain in the hot
  start, the per-chain energy and its final sum, and the sweep, each on two
  rows, with chains in the ragged last row checked.
"""
import numpy as np
import pytest

from oracle import mpr as om
from tests.gpu_util import (TWO_PI, as_fp32_state, beta_of, chain_margins, explainable, fp32_cap, make_field,
                            mismatches, oracle_init)
from tests.test_gpu_fullsize import _oracle_window

pytestmark = pytest.mark.gpu


def test_sweep_of_2p32_work_items_16384_grid():
    ny = nx = 16384
    rng = np.random.default_rng(77)
    z = rng.normal(50.0, 10.0, (ny, nx))
    known = (rng.random((ny, nx)) < 0.5).astype(np.uint8)
    seed, T, a, sweep0 = 9, 0.3, 2.0, 3
    f = make_field([(z, known, 1)], dtype="fp32", seed=seed, tile_x=8, tile_y=8, sweeps_per_pass=1)
    f.set_chain_state(sweep0, np.full(1, a))
    f.sweep(1, [T])
    got_full = f.get_phi(0, 0).cpu().numpy()
    f.close()
    kn = known.astype(bool)
    bounds = (float(z[kn].min()), float(z[kn].max()))
    w = 48
    # first and last tiles of the launch, the centre, the last row's middle
    wins = [(0, w, 0, w), (ny - w, ny, nx - w, nx), (ny // 2, ny // 2 + w, nx // 2, nx // 2 + w),
            (ny - w, ny, nx // 2, nx // 2 + w)]
    bad = gaps = 0
    for win in wins:
        ref, expl, kw = _oracle_window(z, known, bounds, seed, 0, 0, T, a, sweep0, 1, win, "fp32")
        got = got_full[win[0]:win[1], win[2]:win[3]]
        n_bad, _, unexpl = mismatches(got, ref, expl, kw, 1e-3)
        assert len(unexpl) == 0, (win, unexpl[:4])
        bad += n_bad
        gaps += int((~kw).sum())
    assert bad <= fp32_cap(gaps), (bad, gaps)


def test_many_chains_past_2p32_work_items():
    C = (1 << 24) + 5
    z = np.array([[1.0, 2.0], [3.0, 4.0]])
    known = np.array([[1, 0], [0, 1]], dtype=np.uint8)
    seed, T, a, sweep0 = 4, 0.2, 1.5, 6
    f = make_field([(z, known, C)], dtype="fp32", seed=seed)
    # first chain, one at a row boundary of 65536 workgroups, the ragged row
    chains = [0, 1, 65536 * 256 - 1, 65536 * 256, C - 1]
    phi0 = {c: oracle_init(z, known, seed, c, 0, "fp32") for c in chains}
    for c in chains:
        assert np.array_equal(f.get_phi(0, c).cpu().numpy(), phi0[c]), c
    e, cnt = f.specific_energy(1)  # per chain, Eq. (5)
    assert cnt.shape == (C,) and np.all(cnt == 4)
    for c in chains:
        assert e[c] == pytest.approx(om.state_specific_energy(phi0[c][None], 0.5)[0][0], abs=1e-5), c
    f.set_chain_state(sweep0, np.full(C, a))
    f.sweep(1, [T])
    kn = known.astype(bool)
    for c in chains:
        margins = {}
        ref, _ = om.hybrid_sweep(phi0[c][None], kn, [beta_of(T)], [TWO_PI / a], 0.5, seed, sweep0, [c], 0,
                                 margins=margins)
        got = f.get_phi(0, c).cpu().numpy()
        _, _, unexpl = mismatches(got, as_fp32_state(ref[0], known), explainable([chain_margins(margins, 0)]), kn,
                                  1e-3)
        assert len(unexpl) == 0, (c, unexpl)
    f.close()
