"""Equilibrium specific-energy table e(T) computed with the library (Sec. 2.3).

Specific energy matching needs e(T, L) = <H>/N_GP (Eq. 5), which the paper
evaluates by unconditional simulation (the hybrid sweeps with an empty
sample set, Sec. 2.4) once and stores as a lookup table; e depends only
weakly on L.  This module runs that simulation on the GPU for a log-spaced
set of temperatures, one grid of the batch per temperature, and writes the
table that the benchmark and applications pass to mpr_match_T:

    python -m paper_1710_03038_amd.etable        # writes data/etable_L128.csv
    python -m paper_1710_03038_amd.etable gmrf   # the GMRF variant: data/etable_gmrf_L128.csv
    python -m paper_1710_03038_amd.etable q DIR 0.125 0.25   # MPR at other q: DIR/etable_q<q>_L128.csv

Tables of several q run as one batch, each grid with its own q
(mpr_set_grid_q).

Procedure (the paper leaves domain, resolution and run lengths open): every
chain starts from a uniform field at a random angle (cold start, the
fastest way onto the low-T energy plateau), runs n_eq sweeps with the a-rule
from a(0) = max(1, 0.3/sqrt(T)), then n_meas sweeps with the adapted a while
the library records e after every sweep.  The table value is the mean over
sweeps and chains, its error the standard error of the per-chain means.
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PATH = os.path.join(HERE, "data", "etable_L128.csv")
GMRF_PATH = os.path.join(HERE, "data", "etable_gmrf_L128.csv")


def table_path(model="mpr", q=0.5, folder=None):
    """File of the library's table for a model (and, for MPR, q)."""
    if model == "gmrf":
        return GMRF_PATH
    if q == 0.5 and folder is None:
        return DEFAULT_PATH
    return os.path.join(folder or os.path.join(HERE, "data"), f"etable_q{q:g}_L128.csv")


def default_temperatures():
    return np.logspace(-5.0, math.log10(3.0), 46)


def build_table(L=128, temps=None, chains=4, n_eq=600, n_meas=2400, seed=20171003, dtype="fp64", model="mpr"):
    import torch

    from .mpr import Field, default_params

    temps = default_temperatures() if temps is None else np.asarray(temps, dtype=np.float64)
    dev = torch.device("cuda:0")
    zero = torch.zeros((L, L), dtype=torch.float64, device=dev)
    none = torch.zeros((L, L), dtype=torch.uint8, device=dev)
    f = Field([(zero, none, chains) for _ in temps], default_params(dtype=dtype, seed=seed, model=model))
    rng = np.random.Generator(np.random.PCG64(seed))
    for g in range(len(temps)):
        for c in range(chains):
            f.set_phi(torch.full((L, L), float(rng.uniform(0.0, 2.0 * math.pi)), dtype=torch.float64), g, c)
    a0 = np.repeat([max(1.0, 0.3 / math.sqrt(T)) for T in temps], chains)
    f.set_chain_state(0, a0)
    f.sweep(n_eq, temps, adapt=True)
    tr = f.sweep(n_meas, temps, trace=True, trace_energy=True)[:, :, 1].cpu().numpy()
    per_chain = tr.mean(axis=0).reshape(len(temps), chains)
    e = per_chain.mean(axis=1)
    err = per_chain.std(axis=1, ddof=1) / math.sqrt(chains)
    f.close()
    return temps, e, err, dict(L=L, chains=chains, n_eq=n_eq, n_meas=n_meas, seed=seed, dtype=dtype, model=model)


def build_tables_q(qs, L=128, temps=None, chains=4, n_eq=600, n_meas=2400, seed=20171003, dtype="fp64"):
    """MPR tables of several q in one batch: grid (i, j) = q[i] at temps[j].
    Returns a list of (T, e, err, meta), one per q."""
    import torch

    from .mpr import Field, default_params

    temps = default_temperatures() if temps is None else np.asarray(temps, dtype=np.float64)
    nT = len(temps)
    dev = torch.device("cuda:0")
    zero = torch.zeros((L, L), dtype=torch.float64, device=dev)
    none = torch.zeros((L, L), dtype=torch.uint8, device=dev)
    f = Field([(zero, none, chains) for _ in qs for _ in temps], default_params(dtype=dtype, seed=seed))
    f.set_grid_q(np.repeat(np.asarray(qs, dtype=np.float64), nT))
    rng = np.random.Generator(np.random.PCG64(seed))
    for g in range(len(qs) * nT):
        for c in range(chains):
            f.set_phi(torch.full((L, L), float(rng.uniform(0.0, 2.0 * math.pi)), dtype=torch.float64), g, c)
    Tg = np.tile(temps, len(qs))
    f.set_chain_state(0, np.repeat([max(1.0, 0.3 / math.sqrt(T)) for T in Tg], chains))
    f.sweep(n_eq, Tg, adapt=True)
    tr = f.sweep(n_meas, Tg, trace=True, trace_energy=True)[:, :, 1].cpu().numpy()
    f.close()
    per_chain = tr.mean(axis=0).reshape(len(qs), nT, chains)
    out = []
    for i, q in enumerate(qs):
        e = per_chain[i].mean(axis=1)
        err = per_chain[i].std(axis=1, ddof=1) / math.sqrt(chains)
        out.append((temps, e, err, dict(L=L, chains=chains, n_eq=n_eq, n_meas=n_meas, seed=seed, dtype=dtype,
                                        model="mpr", q=float(q))))
    return out


def save_table(path, T, e, err, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        if meta.get("model") == "gmrf":
            f.write("# Equilibrium GMRF specific energy e(T) = <H>/N_GP, H_ij = 1 - dphi^2/(2 pi^2), "
                    "open boundaries,\n")
        else:
            q = meta.get("q", 0.5)
            f.write(f"# Equilibrium MPR specific energy e(T) = <H>/N_GP, q = {'1/2' if q == 0.5 else f'{q:g}'}, "
                    "open boundaries,\n")
        f.write("# from unconditional hybrid Monte Carlo chains run with libmpr (paper_1710_03038_amd/etable.py): "
                + ", ".join(f"{k}={v}" for k, v in meta.items()) + "\n")
        f.write(f"# strictly increasing in T: {bool(np.all(np.diff(e) > 0))}\n")
        f.write("T,e,e_stderr\n")
        for t, v, s in zip(T, e, err):
            f.write(f"{t:.17g},{v:.17g},{s:.6g}\n")


def load_table(path=None, model="mpr", q=0.5):
    """(T, e, e_stderr) arrays of a table file (default: the model's at q)."""
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
    if len(sys.argv) > 3 and sys.argv[1] == "q":
        folder, qs = sys.argv[2], [float(v) for v in sys.argv[3:]]
        for T, e, err, meta in build_tables_q(qs):
            out = table_path("mpr", meta["q"], folder)
            save_table(out, T, e, err, meta)
            print("wrote", out, "monotone:", bool(np.all(np.diff(e) > 0)), flush=True)
        sys.exit(0)
    model = sys.argv[1] if len(sys.argv) > 1 else "mpr"
    out = sys.argv[2] if len(sys.argv) > 2 else (GMRF_PATH if model == "gmrf" else DEFAULT_PATH)
    T, e, err, meta = build_table(model=model)
    save_table(out, T, e, err, meta)
    print("wrote", out, "monotone:", bool(np.all(np.diff(e) > 0)), flush=True)
