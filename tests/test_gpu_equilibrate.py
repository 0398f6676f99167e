"""Equilibrium detection (mpr_equilibrate, Algorithm 2, step 4) on the GPU
against the oracle, and the relaxation comparison of Sec. 2.4."""
import numpy as np
import pytest

from oracle import mpr as om
from tests.gpu_util import make_field, oracle_init, random_grid

pytestmark = pytest.mark.gpu


def _grid(n=24, p_gap=0.7, seed=3):
    z, known = random_grid(n, n + 4, p_gap, seed, smooth=True)
    return z, known


@pytest.mark.parametrize("adapt,over_relax", [(True, True), (True, False), (False, False)])
def test_equilibrate_matches_oracle_fp64(adapt, over_relax):
    z, known = _grid()
    kb = known.astype(bool)
    C, seed, T = 3, 41, 0.02
    f = make_field([(z, known, C)], dtype="fp64", seed=seed)
    n, at, tr = f.equilibrate([T], n_f=5, n_fit=20, i_max=150, adapt=adapt, over_relax=over_relax)
    tr = tr.cpu().numpy()
    phi0 = np.stack([oracle_init(z, known, seed, c, 0, "fp64") for c in range(C)])
    phi, a, n_ref, at_ref, e_ref, acc_ref = om.equilibrate(phi0, kb, T, np.ones(C), 0.5, seed, 0, np.arange(C), 0,
                                                           n_f=5, n_fit=20, i_max=150, adapt=adapt,
                                                           or_step=over_relax)
    assert np.abs(tr[:, :, 1] - e_ref[:n]).max() <= 1e-9
    assert np.abs(tr[:, :, 0] - acc_ref[:n]).max() <= 1e-12
    assert n == n_ref and np.array_equal(at, at_ref), (n, n_ref, at, at_ref)
    for c in range(C):
        assert np.abs(f.get_phi(0, c).cpu().numpy() - phi[c]).max() <= 1e-5
    idx, a_gpu = f.chain_state()
    assert idx == n and np.allclose(a_gpu, a, rtol=0, atol=0)
    f.close()


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_equilibrate_then_fill_equals_fill_with_those_sweeps(dtype):
    # mpr_equilibrate runs exactly the equilibration sweeps of Algorithm 2:
    # following it with a fill of n_eq = 0 gives bitwise the fill with
    # n_eq = the sweeps it ran.
    z, known = _grid(40, 0.6, 8)
    C, T = 2, 0.05
    f = make_field([(z, known, C)], dtype=dtype, seed=6)
    n, at, _ = f.equilibrate([T], i_max=200)
    zh1, zs1, rep1 = f.fill([T], 0, 30, 3)
    f.close()
    g = make_field([(z, known, C)], dtype=dtype, seed=6)
    zh2, zs2, rep2 = g.fill([T], n, 30, 3)
    g.close()
    assert np.array_equal(zh1[0].cpu().numpy(), zh2[0].cpu().numpy())
    assert np.array_equal(zs1[0].cpu().numpy(), zs2[0].cpu().numpy())
    assert np.array_equal(rep1["a_eq"], rep2["a_eq"])


def test_hybrid_equilibrates_where_standard_metropolis_lags():
    # Sec. 2.4: on a 128 x 128 field with 90 % gaps at its fitted (low)
    # temperature, the hybrid update passes the slope test within a few
    # hundred sweeps, and standard Metropolis (a = 1, no over-relaxation)
    # is still at a higher energy after as many sweeps.
    z, known = random_grid(128, 128, 0.9, 17, smooth=True)
    from oracle.etable import load_table
    tT, te, _ = load_table()
    f = make_field([(z, known, 2)], dtype="fp32", seed=2)
    e_s, _ = f.specific_energy(0)
    T, _ = om.match_T(e_s, tT, te)
    n, at, tr = f.equilibrate(T, i_max=1000)
    assert np.all(at > 0) and n <= 400, (n, at)
    e_h = tr.cpu().numpy()[-1, :, 1]
    f.close()
    g = make_field([(z, known, 2)], dtype="fp32", seed=2)
    tr_s = g.sweep(n, T, trace=True, trace_energy=True, over_relax=False).cpu().numpy()
    g.close()
    assert np.all(tr_s[-1, :, 1] > e_h), (tr_s[-1, :, 1], e_h)


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_equilibrate_is_bit_reproducible(dtype):
    # The per-sweep energies are summed over a chain's tiles in a fixed
    # order, so two identical runs give bit-equal traces and stop points
    # (Algorithm 2, steps 4.3-4.4), here on a batch of many tiles per chain.
    z, known = random_grid(256, 320, 0.8, 23, smooth=True)
    runs = []
    for _ in range(2):
        f = make_field([(z, known, 3)], dtype=dtype, seed=12, tile_x=32, tile_y=32)
        n, at, tr = f.equilibrate([0.01], n_f=5, n_fit=20, i_max=300)
        runs.append((n, at.copy(), tr.cpu().numpy().copy(), f.get_phi(0, 2).cpu().numpy()))
        f.close()
    (n1, at1, tr1, p1), (n2, at2, tr2, p2) = runs
    assert n1 == n2 and np.array_equal(at1, at2)
    assert np.array_equal(tr1, tr2)
    assert np.array_equal(p1, p2)
