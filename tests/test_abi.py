"""The C ABI on the CPU: the library loads, exports what include/mpr.h
declares, validates its arguments before touching the GPU, and its host-only
entry point (mpr_match_T) matches the oracle."""
import ctypes
import math

import numpy as np
import pytest

from oracle import mpr as om
from oracle.etable import load_table
from paper_1710_03038_amd import mpr as M


def test_library_exports_every_declared_symbol():
    L = M.lib()
    names = M.header_functions()
    assert len(names) == 24
    for n in names:
        assert hasattr(L, n), n


def test_default_params_are_the_papers():
    p = M.default_params()
    assert (p.q, p.a_targ, p.k_a, p.adapt_every, p.a_sample_keep) == (0.5, 0.3, 3.0, 1, 0)
    assert p.dtype == M.FP32 and p.seed == 0 and p.model == M.MODEL_MPR
    assert M.default_params(model="gmrf").model == M.MODEL_GMRF


@pytest.mark.parametrize("model,q", [("mpr", 0.5), ("mpr", 0.125), ("mpr", 0.25), ("mpr", 0.375), ("gmrf", 0.5)])
def test_match_T_matches_oracle_on_the_oracle_table(model, q):
    T, e, _ = load_table(model=model, q=q)
    es = np.concatenate([np.linspace(e[0], e[-1], 700), e, [e[0] - 1e-3, e[-1] + 1e-3, -1.0, -1.5]])
    a, sa = M.match_T(es, T, e)
    b, sb = om.match_T(es, T, e)
    np.testing.assert_allclose(a, b, rtol=1e-12)
    assert np.array_equal(sa == M.MPR_E_RANGE, sb == om.RANGE_CLAMPED)


def test_match_T_power_law_exact():
    T = np.logspace(-6, 0, 25)
    e = T / 4 - 1
    es = -1 + np.array([3e-6, 1e-4, 0.1, 0.2])
    out, st = M.match_T(es, T, e)
    # 1 + e_s near e_s = -1 carries ~1e-16 / 3e-6 relative rounding of its own
    np.testing.assert_allclose(out, 4 * (1 + es), rtol=1e-11)
    assert np.all(st == 0)


def test_match_T_validation():
    T = np.array([1e-3, 1e-2, 1e-1])
    with pytest.raises(M.MPRError) as ei:
        M.match_T([-0.9], T[::-1], np.array([-0.999, -0.99, -0.9]))
    assert ei.value.status == M.MPR_E_ARG
    with pytest.raises(M.MPRError):
        M.match_T([-0.9], T, np.array([-0.9, -0.99, -0.8]))        # not monotone
    with pytest.raises(M.MPRError):
        M.match_T([-0.9], T[:1], np.array([-0.9]))                  # one point
    with pytest.raises(M.MPRError) as ei:
        M.match_T([-0.5], T, np.array([-0.999, -0.99, -0.9]), raise_on_range=True)
    assert ei.value.status == M.MPR_E_RANGE


def test_nan_e_s_is_an_argument_error():
    T = np.array([1e-3, 1e-2, 1e-1])
    e = np.array([-0.999, -0.99, -0.9])
    es = np.array([math.nan, -0.995])
    Tout = np.empty(2)
    st = np.zeros(2, np.int32)
    rc = M.lib().mpr_match_T(M._dptr(es), 2, M._dptr(T), M._dptr(e), 3, M._dptr(Tout),
                             st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == M.MPR_E_ARG and st[0] == M.MPR_E_ARG and st[1] == M.MPR_OK
    assert math.isnan(Tout[0]) and 1e-3 < Tout[1] < 1e-2


def test_workspace_size_query_and_layout():
    p = M.default_params()
    n1 = M.workspace_bytes([(64, 64, 1)], p)
    n2 = M.workspace_bytes([(64, 64, 2)], p)
    assert n2 > n1 > 5 * 64 * 64 * 4            # 2 state buffers + 3 fill accumulators
    p64 = M.default_params(dtype="fp64")
    assert M.workspace_bytes([(64, 64, 1)], p64) > n1
    nb = M.workspace_bytes([(64, 64, 1), (3, 5, 7), (1, 2, 1)], p)
    assert nb > n1


@pytest.mark.parametrize("field,value,status", [
    ("q", 0.7, M.MPR_E_ARG), ("q", 0.0, M.MPR_E_ARG), ("a_targ", 1.5, M.MPR_E_ARG),
    ("k_a", 0.0, M.MPR_E_ARG), ("adapt_every", 0, M.MPR_E_ARG), ("dtype", 3, M.MPR_E_ARG),
    ("sweeps_per_pass", 17, M.MPR_E_ARG), ("tile_x", 7, M.MPR_E_ARG), ("tile_y", 194, M.MPR_E_ARG),
    ("a_sample_keep", 2, M.MPR_E_ARG), ("model", 2, M.MPR_E_ARG), ("boundary", 2, M.MPR_E_ARG),
    ("boundary", -1, M.MPR_E_ARG)])
def test_bad_params_rejected_before_any_launch(field, value, status):
    p = M.default_params(**{field: value})
    with pytest.raises(M.MPRError) as ei:
        M.workspace_bytes([(8, 8, 1)], p)
    assert ei.value.status == status


@pytest.mark.parametrize("shape,status", [((1, 1, 1), M.MPR_E_SHAPE), ((0, 5, 1), M.MPR_E_SHAPE),
                                          ((4, 4, 0), M.MPR_E_SHAPE), ((70000, 2, 1), M.MPR_E_SHAPE)])
def test_bad_shapes_rejected(shape, status):
    with pytest.raises(M.MPRError) as ei:
        M.workspace_bytes([shape], M.default_params())
    assert ei.value.status == status


def test_q_one_is_accepted_as_test_mode():
    assert M.workspace_bytes([(4, 4, 1)], M.default_params(q=1.0)) > 0


def test_null_context_calls_fail_cleanly():
    L = M.lib()
    T = np.array([1.0])
    assert L.mpr_sweep(None, 1, M._dptr(T), 0, None) == M.MPR_E_STATE
    e = np.empty(1)
    assert L.mpr_specific_energy(None, 0, M._dptr(e), None) == M.MPR_E_STATE
    assert L.mpr_fill(None, M._dptr(T), 1, 1, 1, None, None, None) == M.MPR_E_STATE
    assert L.mpr_get_phi(None, 0, 0, None) == M.MPR_E_STATE
    assert L.mpr_reinit(None) == M.MPR_E_STATE
    assert L.mpr_set_graph(None, 1) == M.MPR_E_STATE
    assert L.mpr_validation_measures(None, 0, None, None, M._dptr(e)) == M.MPR_E_STATE
    assert L.mpr_equilibrate(None, M._dptr(T), 5, 20, 10, 0, None, None, None) == M.MPR_E_STATE
    assert L.mpr_set_grid_q(None, M._dptr(T)) == M.MPR_E_STATE
    L.mpr_destroy(None)
    assert b"NULL" in L.mpr_last_error(None)


def _cv_query(n_folds=4, qs=(0.25, 0.5), model=0, n_samp=10, stride=2, shape=(32, 40), chains=1):
    L = M.lib()
    g = M.Grid()
    g.ny, g.nx = shape
    g.chains, g.reserved = chains, 0
    p = M.default_params(model=model)
    q = np.array(qs, dtype=np.float64)
    n = ctypes.c_size_t(0)
    best = ctypes.c_int32(-1)
    dp = ctypes.POINTER(ctypes.c_double)
    nq = len(qs)
    rc = L.mpr_cv_select_q(ctypes.byref(g), ctypes.byref(p), None, n_folds, M._dptr(q), nq, (dp * max(nq, 1))(),
                           (dp * max(nq, 1))(), (ctypes.c_int32 * max(nq, 1))(), 20, n_samp, stride, None,
                           ctypes.byref(n), None, None, ctypes.byref(best))
    return rc, n.value


def test_cv_select_q_workspace_query_and_validation():
    rc, n = _cv_query()
    assert rc == M.MPR_OK
    one = M.workspace_bytes([(32, 40, 1)], M.default_params())
    # eight fits, four fold masks and scoring fields, eight predictions
    assert n >= 8 * 32 * 40 * 8 + 4 * 32 * 40 * 9 + one
    assert _cv_query(qs=(0.25, 0.5, 0.125))[1] > n
    for kw in (dict(n_folds=1), dict(n_folds=255), dict(qs=(0.0, 0.5)), dict(qs=(0.6,)), dict(qs=()),
               dict(model=M.MODEL_GMRF), dict(n_samp=1, stride=2)):
        assert _cv_query(**kw)[0] == M.MPR_E_ARG, kw
    assert _cv_query(shape=(1, 1))[0] == M.MPR_E_SHAPE


def _tile_query(n_eq=20, n_samp=80, trial=16, shape=(32, 40), ws_bytes=True, **prm):
    L = M.lib()
    g = (M.Grid * 1)()
    g[0].ny, g[0].nx = shape
    g[0].chains, g[0].reserved = 1, 0
    p = M.default_params(**prm)
    T = np.array([1.0])
    n = ctypes.c_size_t(0)
    rc = L.mpr_autotune_tile(g, 1, ctypes.byref(p), M._dptr(T), n_eq, n_samp, trial, None,
                             ctypes.byref(n) if ws_bytes else None, None, None, None, None)
    return rc, L.mpr_last_error(None)


def test_autotune_tile_validates_before_touching_the_device():
    # every argument error is reported before the device query, which on a
    # machine without a GPU is the first thing to fail
    for kw in (dict(n_eq=-1), dict(n_eq=0, n_samp=0), dict(n_samp=-5), dict(trial=0), dict(ws_bytes=False),
               dict(q=0.7), dict(tile_x=7), dict(sweeps_per_pass=17)):
        assert _tile_query(**kw)[0] == M.MPR_E_ARG, kw
    assert _tile_query(shape=(1, 1))[0] == M.MPR_E_SHAPE
    assert _tile_query(shape=(0, 4))[0] == M.MPR_E_SHAPE


def test_workspace_too_small_or_misaligned_is_rejected_before_any_device_call():
    # the size and alignment checks come before the context touches the
    # device, so placeholder (never dereferenced) pointers suffice here
    L = M.lib()
    g = (M.Grid * 1)()
    g[0].ny, g[0].nx, g[0].chains, g[0].reserved = 16, 16, 1, 0
    g[0].z, g[0].known = 4096, 8192
    p = M.default_params()
    need = M.workspace_bytes([(16, 16, 1)], p)
    ctx = ctypes.c_void_p()
    for ws, size in ((1 << 20, need - 1), (256 + 1, need), (256 + 128, need)):
        n = ctypes.c_size_t(size)
        rc = L.mpr_init_field(ctypes.byref(ctx), g, 1, ctypes.byref(p), ctypes.c_void_p(ws), ctypes.byref(n), None)
        assert rc == M.MPR_E_WORKSPACE, (ws, size)
        assert b"workspace" in L.mpr_last_error(None)
    assert not ctx.value


def test_autotune_tile_without_a_device_reports_the_hip_error():
    import torch
    rc, msg = _tile_query()
    if torch.cuda.is_available():
        assert rc == M.MPR_OK
    else:
        assert rc == M.MPR_E_HIP and b"device query" in msg
