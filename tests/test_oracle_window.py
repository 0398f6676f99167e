"""The oracle run on a window of a larger grid (random stream keyed by the
full grid's coordinates) reproduces the full-grid run away from the
window's edges: k sweeps reach 2k sites in from an edge."""
import math

import numpy as np

from oracle import mpr as om


def test_window_matches_full_grid_away_from_edges():
    rng = np.random.default_rng(4)
    ny, nx = 40, 37
    z = rng.normal(size=(ny, nx))
    known = rng.random((ny, nx)) < 0.4
    phi_s, zmin, zmax = om.transform(z, known)
    seed, chain, grid = 99, 3, 2
    phi = om.hot_start(phi_s, known, seed, [chain], grid)
    k = 3
    full = phi
    for s in range(k):
        full, _ = om.hybrid_sweep(full, known, [1 / 0.05], [2 * math.pi / 2], 0.5, seed, 5 + s, [chain], grid)
    y0, y1, x0, x1 = 9, 30, 11, 27
    H = 2 * k + 1
    ey0, ey1, ex0, ex1 = y0 - H, y1 + H, x0 - H, x1 + H
    ws, _, _ = om.transform(z[ey0:ey1, ex0:ex1], known[ey0:ey1, ex0:ex1], bounds=(zmin, zmax))
    w = om.hot_start(ws, known[ey0:ey1, ex0:ex1], seed, [chain], grid, origin=(ey0, ex0), gnx=nx)
    assert np.array_equal(w[0], phi[0, ey0:ey1, ex0:ex1])
    for s in range(k):
        w, _ = om.hybrid_sweep(w, known[ey0:ey1, ex0:ex1], [1 / 0.05], [2 * math.pi / 2], 0.5, seed, 5 + s,
                               [chain], grid, origin=(ey0, ex0), gnx=nx)
    inner = w[0, y0 - ey0:y1 - ey0, x0 - ex0:x1 - ex0]
    assert np.array_equal(inner, full[0, y0:y1, x0:x1])
    # and the edge rings really do differ (the test has teeth)
    assert not np.array_equal(w[0], full[0, ey0:ey1, ex0:ex1])
