"""The fill graph (mpr_set_graph) and mpr_reinit, through the C ABI.

A fill recorded into a hipGraph and replayed must give bitwise the results
of the plain fill from the same state; replays are checked one by one, with
the program's own eager work and synchronisations between them.  A context
set up again by mpr_reinit must behave bitwise like a fresh one.
"""
import numpy as np
import pytest

from tests.gpu_util import make_field, random_grid

pytestmark = pytest.mark.gpu

T = [0.05, 0.2]


def _grids():
    z1, k1 = random_grid(96, 80, 0.5, 11)
    z2, k2 = random_grid(40, 56, 0.7, 12)
    return [(z1, k1, 3), (z2, k2, 2)]


def _host(out):
    zh, zs, rep = out
    return ([h.cpu().numpy() for h in zh], [s.cpu().numpy() for s in zs],
            {k: np.array(v) for k, v in rep.items()})


def _assert_same(a, b):
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        assert np.array_equal(x, y)
    for k in a[2]:
        assert np.array_equal(a[2][k], b[2][k], equal_nan=True), k


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_reinit_behaves_like_a_fresh_context(dtype):
    fresh = make_field(_grids(), dtype=dtype, seed=5)
    ref = _host(fresh.fill(T, 12, 24, 3))
    fresh.close()
    f = make_field(_grids(), dtype=dtype, seed=5)
    f.sweep(9, T, adapt=True)
    f.fill(T, 5, 6, 2)
    f.reinit()
    assert f.chain_state()[0] == 0
    assert np.all(f.chain_state()[1] == 1.0)
    _assert_same(_host(f.fill(T, 12, 24, 3)), ref)
    f.close()


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_graph_replays_equal_the_plain_fill(dtype):
    import torch
    plain = make_field(_grids(), dtype=dtype, seed=5)
    ref = _host(plain.fill(T, 17, 40, 4))
    ref_next = _host(plain.fill(T, 17, 40, 4))   # continuing the chains
    plain.close()

    g = make_field(_grids(), dtype=dtype, seed=5)
    g.set_graph(True)
    g.set_timing(True)
    for rep in range(3):                          # record, then two replays
        _assert_same(_host(g.fill(T, 17, 40, 4)), ref)
        ms, launches, site_sweeps = g.timing()
        assert launches > 0 and ms > 0
        # every sweep of the fill covers every site of every chain once
        assert site_sweeps == (17 + 40) * sum(z.size * ch for z, _, ch in _grids())
        # eager work between replays
        g.specific_energy()
        x = torch.ones(1 << 16, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        assert float(x[-1]) == float(1 << 16)
        g.reinit()
    # a fill from another sweep counter records afresh and stays exact
    g.fill(T, 17, 40, 4)
    _assert_same(_host(g.fill(T, 17, 40, 4)), ref_next)
    g.close()


def test_graph_follows_a_new_launch_shape():
    ref = None
    for graph in (False, True):
        f = make_field(_grids(), dtype="fp32", seed=9)
        f.set_graph(graph)
        f.fill(T, 8, 16, 2)                       # records with the default shape
        f.reinit()
        f.autotune(T, 8)                          # may change sweeps per pass and workgroup size
        f.reinit()
        out = _host(f.fill(T, 8, 16, 2))
        if ref is None:
            ref = out
        else:
            _assert_same(out, ref)
        f.close()
