"""Helpers for the GPU tests (no test functions here)."""
import math

import numpy as np

from oracle import mpr as om

TWO_PI = 2.0 * math.pi


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm GPU")
    return torch.device("cuda:0")


def make_field(grids, **params):
    """grids: list of (z ndarray, known ndarray, chains)."""
    import torch
    from paper_1710_03038_amd import mpr as M
    dev = device()
    ts = [(torch.from_numpy(np.ascontiguousarray(z, dtype=np.float64)).to(dev),
           torch.from_numpy(np.ascontiguousarray(k, dtype=np.uint8)).to(dev), ch) for z, k, ch in grids]
    return M.Field(ts, M.default_params(**params))


def random_grid(ny, nx, p_gap, seed, smooth=True):
    import mprgen
    if smooth and min(ny, nx) >= 4:
        z = mprgen.gaussian_field(ny, nx, max(1.0, min(ny, nx) / 8), seed, 50.0, 10.0)
    else:
        z = np.random.default_rng(seed).normal(50.0, 10.0, (ny, nx))
    rng = np.random.default_rng(seed + 1)
    known = (rng.random((ny, nx)) >= p_gap).astype(np.uint8)
    known.flat[0] = 1
    known.flat[-1] = 1
    return z, known


def oracle_init(z, known, seed, chain, grid, dtype):
    phi_s, zmin, zmax = om.transform(z, known.astype(bool))
    phi = om.hot_start(phi_s, known.astype(bool), seed, [chain], grid)[0]
    if dtype == "fp32":
        phi = as_fp32_state(phi, known)
    return phi


def as_fp32_state(phi, known):
    """Round an oracle state as an FP32 context stores it: gaps kept below 2*pi."""
    f = np.asarray(phi, dtype=np.float32).astype(np.float64)
    gap = ~known.astype(bool)
    top = float(np.float32(TWO_PI))
    f[gap & (f >= top)] = float(np.nextafter(np.float32(TWO_PI), np.float32(0)))
    return f


def beta_of(T):
    return 0.0 if T == math.inf else (math.inf if T == 0 else 1.0 / T)


def explained_mismatches(phi_gpu, phi_ref, margins, known, tol, thr=1e-4):
    """Sites with |gpu - ref| > tol, split into those explained by a
    rounding-sensitive decision (near a threshold, or a colour-1 site next to
    a mismatched colour-0 site) and the unexplained rest."""
    diff = np.abs(phi_gpu - phi_ref)
    bad = (diff > tol) & ~known.astype(bool)
    ny, nx = bad.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    near = (margins["accept"] < thr) | (margins["or_edge"] < thr) | (margins["wrap"] < thr)
    expl = bad & near
    c0bad = bad & (((xx + yy) % 2) == 0)
    nb = np.zeros_like(bad)
    nb[:, 1:] |= c0bad[:, :-1]
    nb[:, :-1] |= c0bad[:, 1:]
    nb[1:, :] |= c0bad[:-1, :]
    nb[:-1, :] |= c0bad[1:, :]
    expl |= bad & (((xx + yy) % 2) == 1) & nb
    return int(bad.sum()), int(expl.sum()), np.argwhere(bad & ~expl)
