"""Precision policy: the FP32 sweeps sample the same equilibrium as FP64.

Unconditional 128 x 128 grids at six temperatures, from the frozen to the
nearly free regime, are run to equilibrium with 16 independent chains in
FP32 (bounded-argument sin, cos, atan2 and exp, FP32 state) and 16 in FP64
(library math), from independent seeds.  The equilibrium specific energy
e(T) of Eq. (5) of the two must agree within their combined statistical
error (4 sigma, each sigma from its 16 per-chain means), for both pair
interactions.  A bias of the fast functions would show as a systematic
offset."""
import numpy as np
import pytest

from paper_1710_03038_amd.etable import build_table, default_temperatures

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("model", ["mpr", "gmrf"])
def test_fp32_equilibrium_energy_equals_fp64(model):
    T = default_temperatures()[[0, 9, 18, 27, 36, 45]]
    kw = dict(temps=T, chains=16, n_eq=600, n_meas=2400, model=model)
    _, e32, err32, _ = build_table(seed=97531, dtype="fp32", **kw)
    _, e64, err64, _ = build_table(seed=13579, dtype="fp64", **kw)
    d = e32 - e64
    sig = np.sqrt(err32 ** 2 + err64 ** 2)
    assert np.all(np.abs(d) <= 4.0 * sig + 1e-9), (T, d, sig)
