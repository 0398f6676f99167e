"""Seeded synthetic workloads for the MPR gap-filling path.

This module only draws inputs: Gaussian / lognormal random fields and
missing-data masks.  It holds none of the method's arithmetic and is shared
by the tests, the smoke check, the benchmark and the oracle's callers.

The paper validates on Gaussian fields with mean 50 and standard deviation 10
sampled by a spectral method, with sites removed by random thinning or as
solid blocks (Sec. 4.1), and on lognormal data (Sec. 4.3).  Its own fields
and the two real datasets are not available here; these generators stand in
for them.  The covariances are squared-exponential,
C(h) = sigma^2 exp(-h^2 / (2 l^2)), and the paper's Whittle-Matern family,
sampled on a periodic torus by circulant embedding and cropped.
"""
import math

import numpy as np


def _fft_size(n):
    """Smallest 2^a 3^b 5^c >= n (fast FFT lengths)."""
    best = None
    p2 = 1
    while p2 < 2 * n:
        p3 = p2
        while p3 < 2 * n:
            p5 = p3
            while p5 < 2 * n:
                if p5 >= n and (best is None or p5 < best):
                    best = p5
                p5 *= 5
            p3 *= 3
        p2 *= 2
    return best


def _circulant_field(ny, nx, corr_sq, margin, seed, mean, std):
    """Stationary Gaussian field with correlation corr_sq(h^2) (1 at 0).

    Circulant embedding on a torus ``margin`` sites larger than the grid:
    eigenvalues lambda = Re FFT2(c), clipped at 0;
    Y = Re IFFT2(sqrt(lambda) * FFT2(W)) with W iid N(0, 1); crop to ny x nx.
    """
    import scipy.fft as sfft

    my = _fft_size(ny + margin)
    mx = _fft_size(nx + margin)
    dy = np.minimum(np.arange(my), my - np.arange(my)).astype(np.float64)
    dx = np.minimum(np.arange(mx), mx - np.arange(mx)).astype(np.float64)
    cov = corr_sq(dy[:, None] ** 2 + dx[None, :] ** 2)
    lam = np.maximum(sfft.rfft2(cov, workers=-1).real, 0.0)
    del cov
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((my, mx))
    spec = sfft.rfft2(w, workers=-1)
    del w
    spec *= np.sqrt(lam)
    y = sfft.irfft2(spec, s=(my, mx), workers=-1)[:ny, :nx]
    return np.ascontiguousarray(mean + std * y)


def gaussian_field(ny, nx, corr_len, seed, mean=0.0, std=1.0):
    """Stationary Gaussian field with squared-exponential covariance
    sigma^2 exp(-h^2 / (2 l^2)), on a torus 4 correlation lengths larger."""
    return _circulant_field(ny, nx, lambda h2: np.exp(-h2 / (2.0 * corr_len ** 2)),
                            int(math.ceil(4 * corr_len)), seed, mean, std)


def matern_corr(h, kappa, nu):
    """Whittle-Matern correlation 2^(1-nu) / Gamma(nu) (kappa h)^nu
    K_nu(kappa h), 1 at h = 0 (the paper's WM(kappa, nu) covariance divided
    by sigma^2)."""
    from scipy.special import gamma, kv

    x = kappa * np.asarray(h, dtype=np.float64)
    out = np.ones_like(x)
    pos = x > 0
    out[pos] = (2.0 ** (1.0 - nu) / gamma(nu)) * x[pos] ** nu * kv(nu, x[pos])
    return out


def matern_field(ny, nx, kappa, nu, seed, mean=0.0, std=1.0):
    """Stationary Gaussian field with Whittle-Matern covariance WM(kappa, nu)
    (nu = 1/2 is the exponential model), on a torus 12 / kappa larger than
    the grid, where the correlation has fallen below 1e-4 for nu <= 1."""
    return _circulant_field(ny, nx, lambda h2: matern_corr(np.sqrt(h2), kappa, nu), int(math.ceil(12.0 / kappa)),
                            seed, mean, std)


def lognormal_field(ny, nx, corr_len, seed, log_std=0.5, log_mean=0.0):
    """exp of a Gaussian field with the given log-mean and log-std."""
    return np.exp(gaussian_field(ny, nx, corr_len, seed, mean=log_mean, std=log_std))


def mask_random(ny, nx, p, seed):
    """Exactly floor(p * N) gap sites chosen without replacement.

    Returns ``known`` as uint8 (1 = sample, 0 = gap).
    """
    n = ny * nx
    n_gap = int(math.floor(p * n))
    rng = np.random.Generator(np.random.PCG64(seed))
    known = np.ones(n, dtype=np.uint8)
    known[rng.choice(n, size=n_gap, replace=False)] = 0
    return known.reshape(ny, nx)


def mask_block(ny, nx, side, seed):
    """One solid side x side square of gaps at a uniform position (the
    paper's block removal, Sec. 4.1).  Returns ``known`` as uint8."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y0 = int(rng.integers(0, ny - side + 1))
    x0 = int(rng.integers(0, nx - side + 1))
    known = np.ones((ny, nx), dtype=np.uint8)
    known[y0:y0 + side, x0:x0 + side] = 0
    return known


def mask_blocks(ny, nx, p, seed, block=16):
    """Solid block x block squares at uniform positions until gaps >= p."""
    rng = np.random.Generator(np.random.PCG64(seed))
    known = np.ones((ny, nx), dtype=np.uint8)
    target = p * ny * nx
    gaps = 0
    while gaps < target:
        y0 = int(rng.integers(0, max(1, ny - block + 1)))
        x0 = int(rng.integers(0, max(1, nx - block + 1)))
        blk = known[y0:y0 + block, x0:x0 + block]
        gaps += int(blk.sum())
        blk[...] = 0
    return known


def cv_folds(known, n_folds, seed):
    """Fold ids for K-fold cross-validation: the sample sites (known != 0)
    in a seeded random order, dealt round-robin into n_folds folds (sizes
    differ by at most one).  Returns uint8 (ny, nx): the fold id at sample
    sites, 255 at gaps."""
    if not 2 <= n_folds <= 254:
        raise ValueError("n_folds must be in [2, 254]")
    known = np.asarray(known) != 0
    idx = np.flatnonzero(known)
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(idx.size)
    fold = np.full(known.size, 255, dtype=np.uint8)
    fold[idx[order]] = (np.arange(idx.size) % n_folds).astype(np.uint8)
    return fold.reshape(known.shape)


def mask_clouds(ny, nx, p, seed, a_min=16.0, a_max=512.0):
    """Elliptical clouds (log-uniform semi-axes, uniform orientation and
    centre) added until the gap fraction reaches p."""
    rng = np.random.Generator(np.random.PCG64(seed))
    known = np.ones((ny, nx), dtype=np.uint8)
    target = p * ny * nx
    gaps = 0
    while gaps < target:
        a = math.exp(rng.uniform(math.log(a_min), math.log(a_max)))
        b = math.exp(rng.uniform(math.log(a_min), math.log(a_max)))
        th = rng.uniform(0.0, math.pi)
        cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
        r = max(a, b)
        y0, y1 = max(0, int(cy - r)), min(ny, int(cy + r) + 1)
        x0, x1 = max(0, int(cx - r)), min(nx, int(cx + r) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dy, dx = yy - cy, xx - cx
        u = (dx * math.cos(th) + dy * math.sin(th)) / a
        v = (-dx * math.sin(th) + dy * math.cos(th)) / b
        inside = (u * u + v * v) <= 1.0
        sub = known[y0:y1, x0:x1]
        gaps += int((sub[inside] == 1).sum())
        sub[inside] = 0
    return known


# --------------------------------------------------------------------------
# The workloads: synthetic stand-ins with the paper's value ranges
# --------------------------------------------------------------------------
def single_grid(n, corr_len, gap_frac, seed_base, field="gaussian", mask="random"):
    """One n x n workload: (z_true, known).  Seeds: field seed_base+1, mask
    seed_base+2 (the Philox seed of the run is seed_base+3)."""
    if field == "gaussian":
        z = gaussian_field(n, n, corr_len, seed_base + 1, mean=50.0, std=10.0)
    else:
        z = lognormal_field(n, n, corr_len, seed_base + 1, log_std=0.5)
    if mask == "random":
        known = mask_random(n, n, gap_frac, seed_base + 2)
    elif mask == "blocks":
        known = mask_blocks(n, n, gap_frac, seed_base + 2)
    else:
        known = mask_clouds(n, n, gap_frac, seed_base + 2)
    return z, known


# name -> (n, corr_len, gap fraction, seed base, field, mask, chains,
#          n_eq, n_samp, stride)
WORKLOADS = {
    "grid64_fp64": (64, 8.0, 0.33, 100, "gaussian", "random", 1, 100, 100, 1),
    "grid1024": (1024, 16.0, 0.50, 200, "gaussian", "random", 1, 100, 900, 9),
    "grid512x512chains": (512, 10.0, 0.60, 300, "lognormal", "blocks", 512, 100, 100, 1),
    "grid8192x64chains": (8192, 64.0, 0.90, 500, "gaussian", "clouds", 64, 100, 1, 1),
}


def workload(name):
    """(z_true, known, spec dict) of a named single-grid workload."""
    n, ell, p, sb, field, mask, chains, n_eq, n_samp, stride = WORKLOADS[name]
    z, known = single_grid(n, ell, p, sb, field, mask)
    spec = dict(n=n, corr_len=ell, gap_frac=p, seed=sb + 3, field=field, mask=mask,
                chains=chains, n_eq=n_eq, n_samp=n_samp, stride=stride)
    return z, known, spec


def uneven_batch(n_grids, seed=401, l_min=32, l_max=2048):
    """Specs of a batch of grids of uneven size (sides log-uniform in
    [l_min, l_max], gap fraction U(0.1, 0.9), Gaussian or lognormal with
    probability 1/2, correlation length log-uniform in [4, 32] capped at
    side/4).  Returns a list of dicts; fields are drawn by ``batch_grid``."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    specs = []
    for k, child in enumerate(ss.spawn(n_grids)):
        side = int(round(math.exp(rng.uniform(math.log(l_min), math.log(l_max)))))
        p = float(rng.uniform(0.1, 0.9))
        field = "gaussian" if rng.random() < 0.5 else "lognormal"
        ell = min(math.exp(rng.uniform(math.log(4.0), math.log(32.0))), side / 4.0)
        s1, s2 = child.generate_state(2)
        specs.append(dict(n=side, gap_frac=p, field=field, corr_len=ell,
                          field_seed=int(s1), mask_seed=int(s2)))
    return specs


def batch_grid(spec):
    n = spec["n"]
    if spec["field"] == "gaussian":
        z = gaussian_field(n, n, spec["corr_len"], spec["field_seed"], mean=50.0, std=10.0)
    else:
        z = lognormal_field(n, n, spec["corr_len"], spec["field_seed"], log_std=0.5)
    known = mask_random(n, n, spec["gap_frac"], spec["mask_seed"])
    return z, known
