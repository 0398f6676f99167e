"""Pins of the oracle's replicate-boundary option (Sec. 2.5): auxiliary
nodes around the grid copy their nearest grid sites, and the augmented grid
is swept with open boundaries.

The pin is that construction written out: pad the state with a ring of edge
copies, freeze the ring, run the open-boundary sweep on the padded grid with
the interior's own random stream, crop.  Padding once per sweep is enough:
a colour-1 site's copy taken before the sweep still holds its value before
the second half-sweep, because colour-1 sites do not move in the first.
The literal per-site loop, the all-frozen-edge case (which must equal the
open boundary bit for bit) and the corner count (two auxiliary neighbours)
complete the set."""
import math

import numpy as np
import pytest

from oracle import mpr

TWO_PI = 2.0 * math.pi
R = mpr.REPLICATE


def _setup(shape, seed, frac=0.4, chains=(0, 3)):
    rng = np.random.default_rng(seed)
    known = rng.random(shape) < frac
    known.flat[-1] = True
    phi_s, _, _ = mpr.transform(rng.normal(size=shape), known)
    phi = mpr.hot_start(phi_s, known, seed, list(chains), 0)
    return known, phi


def _augmented_sweep(phi, known, beta, alpha, q, seed, sweep, chains, or_step, model):
    """The paper's construction: an (ny + 2) x (nx + 2) grid whose ring holds
    copies of the nearest grid sites, frozen, with open boundaries."""
    ny, nx = known.shape
    pad = np.pad(phi, [(0, 0), (1, 1), (1, 1)], mode="edge")
    kpad = np.pad(known, 1, mode="constant", constant_values=True)
    out, acc = mpr.hybrid_sweep(pad, kpad, beta, alpha, q, seed, sweep, chains, 0, origin=(-1, -1),
                                gnx=nx, or_step=or_step, model=model)
    return out[:, 1:-1, 1:-1], acc


@pytest.mark.parametrize("model", [mpr.MPR, mpr.GMRF])
@pytest.mark.parametrize("shape", [(6, 8), (7, 9), (1, 7), (5, 1), (2, 2)])
def test_replicate_equals_augmented_grid(shape, model):
    chains = [0, 3]
    known, phi = _setup(shape, 11 + shape[0] * 7 + shape[1])
    q = 0.5
    for i, (T, a) in enumerate([(0.05, 1.0), (0.5, 3.0), (math.inf, 1.0), (0.01, 7.0)]):
        beta = 0.0 if T == math.inf else 1 / T
        for or_step in (True, False):
            want, acc_w = _augmented_sweep(phi, known, [beta, beta], [TWO_PI / a] * 2, q, 9, i, chains, or_step, model)
            got, acc_g = mpr.hybrid_sweep(phi, known, [beta, beta], [TWO_PI / a] * 2, q, 9, i, chains, 0,
                                          or_step=or_step, model=model, boundary=R)
            np.testing.assert_array_equal(got, want)
            np.testing.assert_array_equal(acc_g, acc_w)
        phi = got  # chain several sweeps through different states


def test_replicate_run_equals_augmented_run():
    # many sweeps in a row, so a stale ring (refreshed too rarely) would show
    known, phi = _setup((9, 10), 3, frac=0.2, chains=(1,))
    cur_r, cur_a = phi.copy(), phi.copy()
    for s in range(12):
        cur_r, _ = mpr.hybrid_sweep(cur_r, known, [20.0], [TWO_PI / 2], 0.5, 4, s, [1], 0, boundary=R)
        cur_a, _ = _augmented_sweep(cur_a, known, [20.0], [TWO_PI / 2], 0.5, 4, s, [1], True, mpr.MPR)
        np.testing.assert_array_equal(cur_r, cur_a)
    cur_o, _, _, _ = mpr.run_sweeps(phi, known, 0.05, 1.0, 0.5, 4, 0, 12, [1], 0)
    assert not np.array_equal(cur_o, cur_r)  # the option changes the chain


@pytest.mark.parametrize("model", [mpr.MPR, mpr.GMRF])
@pytest.mark.parametrize("shape", [(4, 5), (1, 6), (3, 3)])
def test_vectorised_replicate_matches_literal_loop(shape, model):
    known, phi = _setup(shape, 5 * shape[0] + shape[1], chains=(2,))
    for T, a in ((0.05, 1.0), (0.3, 4.0), (math.inf, 1.0)):
        beta = 0.0 if T == math.inf else 1 / T
        for or_step in (True, False):
            v, acc = mpr.hybrid_sweep(phi, known, [beta], [TWO_PI / a], 0.5, 6, 1, [2], 0, or_step=or_step,
                                      model=model, boundary=R)
            lit, acc_l = mpr.hybrid_sweep_literal(phi[0], known, beta, TWO_PI / a, 0.5, 6, 1, 2, 0,
                                                  or_step=or_step, model=model, boundary=R)
            np.testing.assert_allclose(v[0], lit, rtol=0, atol=1e-12)
            assert acc[0] == acc_l


@pytest.mark.parametrize("model", [mpr.MPR, mpr.GMRF])
def test_frozen_edges_make_replicate_open(model):
    # auxiliary nodes only neighbour edge sites; with every edge site a
    # sample they never enter an update
    ny, nx = 8, 9
    known, phi = _setup((ny, nx), 21, frac=0.3)
    known[0, :] = known[-1, :] = known[:, 0] = known[:, -1] = True
    a, _ = mpr.hybrid_sweep(phi, known, [15.0, 15.0], [2.0, 2.0], 0.5, 2, 0, [0, 3], 0, model=model, boundary=R)
    b, _ = mpr.hybrid_sweep(phi, known, [15.0, 15.0], [2.0, 2.0], 0.5, 2, 0, [0, 3], 0, model=model)
    np.testing.assert_array_equal(a, b)


def test_corner_has_two_auxiliary_neighbours():
    # 2 x 2 grid, only (0, 0) a gap: its field is 2 e^{iq phi} (auxiliary)
    # plus e^{iq phi_j} for the two grid neighbours; over-relaxation
    # reflects q phi about that field's direction
    q = 0.5
    phi = np.array([[[1.0, 2.5], [4.0, 0.7]]])
    known = np.array([[False, True], [True, True]])
    nbrs = mpr._neighbours(phi, R)
    vals = sorted(float(n[0, 0, 0]) for n in nbrs)
    assert vals == sorted([1.0, 1.0, 2.5, 4.0])
    hx = 2 * math.cos(q * 1.0) + math.cos(q * 2.5) + math.cos(q * 4.0)
    hy = 2 * math.sin(q * 1.0) + math.sin(q * 2.5) + math.sin(q * 4.0)
    star = (2 * math.atan2(hy, hx) - q * 1.0) / q
    got = mpr.over_relax(phi, nbrs, q)[0, 0, 0]
    assert got == pytest.approx(star if 0 <= star < TWO_PI else 1.0, abs=1e-14)
    # with alpha -> 0 and beta = 0 the proposal is the reflected angle, accepted
    out, _ = mpr.hybrid_sweep(phi, known, [0.0], [1e-300], q, 1, 0, [0], 0, boundary=R)
    assert out[0, 0, 0] == pytest.approx(got, abs=1e-12)


def test_energies_ignore_the_option():
    # Eqs. (4)-(5) count the grid's own pairs; the fill records them unchanged
    rng = np.random.default_rng(2)
    z = rng.normal(size=(10, 12))
    known = rng.random(z.shape) < 0.5
    o = mpr.fill(z, known, 0.02, 6, 6, 2, seed=3, chains=2)
    r = mpr.fill(z, known, 0.02, 6, 6, 2, seed=3, chains=2, boundary=R)
    np.testing.assert_array_equal(o["z_hat"][known], r["z_hat"][known])
    edge = np.zeros(z.shape, dtype=bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    assert not np.array_equal(o["z_hat"][edge & ~known], r["z_hat"][edge & ~known])
