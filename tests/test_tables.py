"""Both e(T) tables against what the mathematics fixes: monotone in T, the
low-temperature equipartition slope eps = (L + 1) T / (4 L) of an
unconditional L x L grid (harmonic limit of Eq. 3), and the infinite-
temperature limit e = -4/pi^2 for q = 1/2 as an upper bound."""
import math

import numpy as np
import pytest

from oracle.etable import load_table as load_oracle_table
from paper_1710_03038_amd.etable import load_table as load_product_table


@pytest.mark.parametrize("loader,L", [(load_oracle_table, 32), (load_product_table, 128)])
def test_table_shape_and_limits(loader, L):
    T, e, err = loader()
    assert np.all(np.diff(T) > 0) and np.all(np.diff(e) > 0)
    eps = 1.0 + e
    low = T < 3e-3
    ratio = eps[low] / ((L + 1) * T[low] / (4 * L))
    assert np.all(np.abs(ratio - 1.0) < 0.01), ratio
    assert np.all(e < -4.0 / math.pi ** 2)
    assert np.all(err < 5e-3 * eps + 1e-12)


@pytest.mark.parametrize("which,L", [("oracle", 32), ("product", 128)])
def test_gmrf_table_shape_and_limits(which, L):
    # The GMRF energy is exactly quadratic: the same equipartition slope at
    # low T, and at T = infinity 1 + e = E[dphi^2] / (2 pi^2) = 1/3 for
    # independent uniform angles, so e < -2/3 throughout.
    if which == "oracle":
        from oracle import mpr as om
        T, e, err = load_oracle_table(model=om.GMRF)
    else:
        T, e, err = load_product_table(model="gmrf")
    assert np.all(np.diff(T) > 0) and np.all(np.diff(e) > 0)
    eps = 1.0 + e
    low = T < 3e-3
    ratio = eps[low] / ((L + 1) * T[low] / (4 * L))
    assert np.all(np.abs(ratio - 1.0) < 0.01), ratio
    assert np.all(e < -2.0 / 3.0)
    assert np.all(err < 5e-3 * eps + 1e-12)


@pytest.mark.parametrize("q", [0.125, 0.25, 0.375])
def test_product_tables_of_other_q(q):
    # the same closed forms as for q = 1/2: the equipartition slope
    # (L + 1) T / (4 L) does not depend on q, and e stays below the
    # infinite-temperature value -(sin(pi q) / (pi q))^2
    T, e, err = load_product_table(q=q)
    L = 128
    assert np.all(np.diff(T) > 0) and np.all(np.diff(e) > 0)
    eps = 1.0 + e
    low = T < 3e-3
    ratio = eps[low] / ((L + 1) * T[low] / (4 * L))
    assert np.all(np.abs(ratio - 1.0) < 0.01), ratio
    e_inf = -(math.sin(math.pi * q) / (math.pi * q)) ** 2
    assert np.all(e < e_inf)
    assert np.all(err < 5e-3 * eps + 1e-12)
    # and it agrees with the oracle's L = 32 table where e depends little on L
    To, eo, _ = load_oracle_table(q=q)
    mid = (T > 1e-2) & (T < 0.3)
    np.testing.assert_allclose(1 + e[mid], 1 + eo[mid], rtol=0.05)
