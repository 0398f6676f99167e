"""Equilibrium specific-energy table e(T) of the oracle (Sec. 2.3, Eq. 5).

TEST INFRASTRUCTURE (part of the CPU oracle).  The table is the input of
specific energy matching: e(T, L) = <H>/N_GP, evaluated by unconditional
simulation, i.e. the same hybrid sweeps with an empty sample set (Sec. 2.4),
computed once and stored (Sec. 2.3).  Running this module writes
``oracle/etable_L32.csv`` using the oracle alone:

    python -m oracle.etable

Procedure (a reading: the paper gives no table domain, resolution, start or
run lengths for this step): for every T on a log-spaced grid, ``chains``
unconditional L x L chains start from a uniform field (cold start, which
reaches the energy plateau fastest at low T), run ``n_eq`` sweeps with the
a-rule from a(0) = max(1, 0.3/sqrt(T)), then ``n_meas`` sweeps at the
adapted a, recording e after every sweep.  The table value is the mean over
all recorded sweeps and chains; the error column is the standard error of
the per-chain means.
"""
import math
import os
import sys

import numpy as np

from . import mpr

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "etable_L32.csv")
GMRF_PATH = os.path.join(HERE, "etable_gmrf_L32.csv")


def table_path(model=mpr.MPR, q=0.5):
    """File of the oracle's table for a model (and, for MPR, q)."""
    if model == mpr.GMRF:
        return GMRF_PATH
    return DEFAULT_PATH if q == 0.5 else os.path.join(HERE, f"etable_q{q:g}_L32.csv")


def default_temperatures():
    return np.logspace(-5.0, math.log10(3.0), 46)


def table_point(T, L=32, chains=8, n_eq=300, n_meas=900, q=0.5, seed=7, grid=0, model=mpr.MPR):
    known = np.zeros((L, L), dtype=bool)
    rng = np.random.Generator(np.random.PCG64(seed + grid))
    phi = np.broadcast_to(rng.uniform(0, 2 * math.pi, chains)[:, None, None],
                          (chains, L, L)).copy()
    a0 = max(1.0, 0.3 / math.sqrt(T))
    ids = np.arange(chains)
    phi, a, _, _ = mpr.run_sweeps(phi, known, T, a0, q, seed, 0, n_eq, ids, grid, adapt=True, model=model)
    _, _, _, e = mpr.run_sweeps(phi, known, T, a, q, seed, n_eq, n_meas, ids, grid,
                                trace_energy=True, model=model)
    per_chain = e.mean(axis=0)
    return float(per_chain.mean()), float(per_chain.std(ddof=1) / math.sqrt(chains))


def _point(args):
    k, T, kw = args
    return table_point(T, grid=k, **kw)


def build_table(temps=None, processes=8, **kw):
    temps = default_temperatures() if temps is None else np.asarray(temps)
    jobs = [(k, float(T), kw) for k, T in enumerate(temps)]
    if processes > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes) as pool:
            res = pool.map(_point, jobs)
    else:
        res = [_point(j) for j in jobs]
    e = np.array([r[0] for r in res])
    err = np.array([r[1] for r in res])
    return temps, e, err


def save_table(path, T, e, err, header):
    with open(path, "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        f.write("T,e,e_stderr\n")
        for t, v, s in zip(T, e, err):
            f.write(f"{t:.17g},{v:.17g},{s:.6g}\n")


def load_table(path=None, model=mpr.MPR, q=0.5):
    """Return (T, e, e_stderr) arrays of a table file (default: the model's
    at q)."""
    if path is None:
        path = table_path(model, q)
    rows = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or line.startswith("T,"):
                continue
            rows.append([float(v) for v in line.split(",")])
    a = np.array(rows)
    return a[:, 0], a[:, 1], a[:, 2]


if __name__ == "__main__":
    # python -m oracle.etable [processes] [mpr|gmrf] [q]
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    model = sys.argv[2] if len(sys.argv) > 2 else mpr.MPR
    q = float(sys.argv[3]) if len(sys.argv) > 3 else 0.5
    n_meas = 2400 if (model == mpr.GMRF or q != 0.5) else 900
    kw = dict(L=32, chains=8, n_eq=300, n_meas=n_meas, q=q, seed=7, model=model)
    T, e, err = build_table(processes=procs, **kw)
    order_ok = bool(np.all(np.diff(e) > 0))
    path = table_path(model, q)
    what = ("Equilibrium GMRF specific energy e(T) = <H>/N_GP, H_ij = 1 - dphi^2/(2 pi^2), open boundaries,"
            if model == mpr.GMRF else f"Equilibrium MPR specific energy e(T) = <H>/N_GP, q = {q:g}, open boundaries,")
    save_table(path, T, e, err, [
        what,
        "from unconditional CPU-oracle chains (oracle/etable.py): "
        + ", ".join(f"{k}={v}" for k, v in kw.items() if k != "model"),
        f"strictly increasing in T: {order_ok}",
    ])
    print("wrote", path, "monotone:", order_ok)
