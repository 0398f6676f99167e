"""mpr_validation_measures_static (the entry point that allocates nothing,
on the library's static device scratch) against mpr_validation_measures on
the same inputs: bit-equal measures, over two calls in a row, the second on
a smaller grid, and the size limit."""
import numpy as np
import pytest

from tests.gpu_util import make_field, random_grid

pytestmark = pytest.mark.gpu


def _case(ny, nx, seed):
    import torch
    from paper_1710_03038_amd import mpr as M
    z, known = random_grid(ny, nx, 0.6, seed)
    f = make_field([(z, known, 2)], dtype="fp32", seed=seed)
    e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
    zh, _, _ = f.fill([0.01], 20, 10, 2)
    ref = f.validation_measures(0, z, zh[0])
    dev = zh[0].device
    zt = torch.from_numpy(z).to(dev)
    kn = torch.from_numpy(known).to(dev)
    shift = float(z[known.astype(bool)].min())   # the context's z_min
    f.close()
    return zt, zh[0].contiguous(), kn, shift, ref


def test_static_measures_equal_the_context_ones_twice():
    import torch
    from paper_1710_03038_amd import mpr as M
    big = _case(300, 257, 5)
    small = _case(40, 33, 6)
    out = torch.full((8,), float("nan"), dtype=torch.float64, device=big[0].device)
    for zt, zh, kn, shift, ref in (big, small):
        M.validation_measures_static(zt, zh, kn, shift, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = np.array([ref["AAE"], ref["ARE"], ref["AARE"], ref["RASE"], ref["R"], ref["P"], ref["mean_z"],
                         ref["mean_zhat"]])
        assert np.array_equal(got, want), (got, want)


def test_static_measures_reject_sizes_beyond_the_scratch():
    import torch
    from paper_1710_03038_amd import mpr as M
    zt, zh, kn, shift, _ = _case(16, 16, 7)
    out = torch.empty(8, dtype=torch.float64, device=zt.device)
    L = M.lib()
    import ctypes
    rc = L.mpr_validation_measures_static(ctypes.c_void_p(zt.data_ptr()), ctypes.c_void_p(zh.data_ptr()),
                                          ctypes.c_void_p(kn.data_ptr()), M.STATIC_MAX_SITES + 1, shift,
                                          ctypes.c_void_p(out.data_ptr()), None)
    assert rc == M.MPR_E_ARG
    assert b"static scratch" in L.mpr_last_error(None)
