#!/usr/bin/env python3
"""Benchmark of the MPR gap-filling hot path on one MI355X.

One step = the whole path on one synthetic workload with inputs resident in
HBM: mpr_reinit (Eq. 2 bounds, gap-site plan, hot start), mpr_specific_energy
(Eq. 4), mpr_match_T (specific energy matching, Sec. 2.3, one T per grid),
mpr_autotune (a cached lookup after the first step) and mpr_fill
(Algorithm 2 with fixed counts: equilibration with the a-rule, sampling,
conditional mean and std; in the FP32 arm replayed from a hipGraph).  The
context and its workspace are set up once per arm, outside the timed steps;
before the FP32 arm's context is built, mpr_autotune_tile picks its tile
shape (set-up, untimed, skipped with --no-autotune or an explicit --tile).

Prints one JSON line.  value = spin-updates/s (hybrid updates of gap sites,
whole job); realisations/s is reported beside it.  The default workload is
the satellite-scale case: an 8192 x 8192 Gaussian field (squared-
exponential, correlation length 64, mean 50, std 10) with >= 90 % gaps as
random elliptical cloud masks and the truth held out, 64 conditional chains
in one batch, 100 equilibration sweeps with the a-rule and the final state
recorded (64 realisations), FP32.  The plain FP64 arm (one context per
grid, FP64 library math, one sweep per pass, no graph, no autotuning) runs
the same input, and its fill MAE is compared with the FP32 one; the FP64
CPU oracle is timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Workloads: grid64_fp64, grid1024, grid512x512chains,
grid8192x64chains (default), uneven2000.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-updates/sec + realisations/sec, batched FP32 vs plain FP64, equal MAE"
HBM_PEAK_GBS = 8000.0
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs at 2.4 GHz, one wave64
# instruction issued per SIMD at a time: 2.458e12 SIMD issue-cycles/s.
# Issue cycles per wave64 instruction on gfx950, measured with throughput
# probes (independent chains, 16 waves per SIMD): FP32 add/mul/fma/min/max,
# compares and selects, v_add_u32 and v_mov 2; other 32-bit integer and bit
# operations (xor, shifts, lshl_add, add3, mul_lo, cvt) and v_mad_u64_u32 4;
# transcendentals (v_sin, v_exp, v_sqrt, v_rcp) 8.  The published 157.3
# TFLOP/s FP32 is 1024 x 2.4 GHz x 64 lanes x 2 flops / 2 cycles.
VALU_PEAK_TCYC = 256 * 4 * 2.4e9 / 1e12
# Issue cycles of one FP32 gap-site update (q < 1) in the compiled sweep
# kernel, per lane: one step of k_sweep<float, 512> updates a pair of sites
# of one colour; the loop body (loop control included) is 296 VALU
# instructions for colour 0 (174 FP32/compare/select, 22 fast integer, 90
# other integer, 10 transcendental) = 832 cycles, and 312 = 878 cycles for
# colour 1, for 2 x 64 updates: 6.68 cycles per update, of which the pair's
# shared Philox4x32-10 call (20 v_mad_u64_u32, 40 v_xor_b32) is 1.88.
CYC_PER_UPDATE = (832 + 878) / 2 / 128


KERNEL_SOURCES = ("paper_1710_03038_amd/csrc/kernels.hip", "paper_1710_03038_amd/csrc/fastmath.h",
                  "paper_1710_03038_amd/csrc/internal.h")
# rocprofv3 summaries whose FETCH_SIZE / WRITE_SIZE give the measured HBM
# traffic of the sweep launches, per workload.
PROFILES = {"grid8192x64chains": "profiles/k_sweep_fp32_grid8192x64chains.md"}


def bytes_per_site_sweep(elem, p):
    """Algorithmic HBM bytes of one site in one pass (any number of sweeps
    in LDS): read the angle, write it back at gap sites, one mask bit."""
    return elem * (1.0 + p) + 0.125


def profiled_traffic(workload, shape, tile, single_only=False):
    """HBM bytes per sweep launch measured by rocprofv3 (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy) for this workload, or None when
    there is no profile for it, the kernel sources changed since it was
    taken, or this run's launch shape or tile differs from the profiled
    one.  With single_only (every pass of the fill is one sweep), only the
    single-sweep part of the shape (threads, persistent) has to match;
    speculative two-sweep a-rule passes run at the multi-sweep workgroup
    size, so then the whole shape has to."""
    import hashlib
    import re
    if workload not in PROFILES:
        return None
    try:
        text = open(os.path.join(ROOT, PROFILES[workload])).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+) kernel_sources_sha256: ([0-9a-f]+)"
                  r"(?: shape: (\d+) (\d+) (\d+) (\d+) tile: (\d+) (\d+))?", text)
    if not m or m.group(2) != h.hexdigest():
        return None
    if m.group(3) is not None:
        prof_shape = tuple(int(m.group(i)) for i in (3, 4, 5, 6))
        prof_tile = (int(m.group(7)), int(m.group(8)))
        run_shape = tuple(int(v or 0) for v in shape)
        same = run_shape[2:] == prof_shape[2:] if single_only else run_shape == prof_shape
        if not same or tuple(tile)[:2] not in (prof_tile, (0, 0)):
            return None
    return float(m.group(1))


def relaxation_study(L, p, sweeps, chains=4, seed=512, field="wm"):
    """Relaxation of the specific energy from the hot start under the three
    updates the paper compares (Sec. 2.4): hybrid (over-relaxation and the
    a-rule), restricted Metropolis (a-rule, no over-relaxation) and standard
    Metropolis (a = 1, no over-relaxation).  Input: WM(0.5, 0.5) field, mean
    50, std 10, on an L x L grid with floor(p L^2) random gaps, at the
    temperature fitted by specific energy matching (field="se16": a smooth
    squared-exponential field, length 16, instead).  Reports each update's
    Savitzky-Golay equilibration point (Algorithm 2, step 4: n_f = 5,
    n_fit = 20) and its mean energy at fixed sweep counts."""
    import torch

    import mprgen
    from paper_1710_03038_amd import mpr as M
    from paper_1710_03038_amd.etable import load_table

    table = load_table()
    if field == "wm":
        z = mprgen.matern_field(L, L, 0.5, 0.5, seed + 1, mean=50.0, std=10.0)
        desc = "WM(0.5, 0.5), mean 50, std 10 (synthetic)"
    else:
        z = mprgen.gaussian_field(L, L, 16.0, seed + 1, mean=50.0, std=10.0)
        desc = "squared-exponential, length 16, mean 50, std 10 (synthetic)"
    known = mprgen.mask_random(L, L, p, seed + 2)
    dev = torch.device("cuda:0")
    grids = [(torch.from_numpy(z).to(dev), torch.from_numpy(known).to(dev), chains)]
    f = M.Field(grids, M.default_params(dtype="fp32", seed=seed + 3))
    e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
    T, _ = M.match_T(e_s, table[0], table[1])
    marks = [m for m in (10, 20, 50, 100, 200, 500, 1000, 2000, 5000, 10000, 20000, 50000, 100000) if m <= sweeps]
    out = {"study": "relaxation", "grid": [L, L], "field": desc,
           "gap_fraction": p, "chains": chains, "T_hat": float(T[0]), "e_s": float(e_s[0]), "n_f": 5, "n_fit": 20,
           "updates": {}}
    for name, adapt, over_relax in (("hybrid", True, True), ("restricted", True, False), ("standard", False, False)):
        f.reinit()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_sg, at, tr_sg = f.equilibrate(T, n_f=5, n_fit=20, i_max=sweeps - 1, adapt=adapt, over_relax=over_relax)
        torch.cuda.synchronize()
        t_sg = time.perf_counter() - t0
        f.reinit()
        tr = f.sweep(sweeps, T, adapt=adapt, trace=True, trace_energy=True, over_relax=over_relax).cpu().numpy()
        e = tr[:, :, 1].mean(axis=1)
        out["updates"][name] = {"sg_equilibrated_at": [int(v) for v in at], "sg_sweeps_run": n_sg,
                                "sg_seconds": t_sg, "acceptance_last": float(tr[-1, :, 0].mean()),
                                "e_at": {str(m): float(e[m - 1]) for m in marks}}
    f.close()
    h = out["updates"]["hybrid"]["e_at"]
    ref = np.mean([h[str(m)] for m in marks[-3:]])  # hybrid's late level as the equilibrium energy
    out["e_equilibrium_hybrid"] = float(ref)
    for name, u in out["updates"].items():
        u["e_minus_equilibrium"] = {k: v - ref for k, v in u["e_at"].items()}
    print(json.dumps(out), flush=True)


PAPER_MPR = "tests/golden/paper_mpr_validation.txt"


def validation_study(Ls, S):
    """The paper's validation of the MPR method on synthetic data (Sec. 4):
    WM(0.2, nu) Gaussian fields, mean 50, std 10, on L x L grids; case a:
    33 % random gaps, b: 66 %, c: one 20 x 20 block.  Per configuration:
    mpr_reinit, e_s, T-hat by SEM, mpr_equilibrate (n_f = 5, n_fit = 20),
    mpr_fill with M = 100 recorded sweeps, mpr_validation_measures; timed on
    the device from reinit to the measures.  Prints one JSON line per row
    with the means over S configurations and the paper's printed values."""
    import torch

    import mprgen
    from paper_1710_03038_amd import mpr as M
    from paper_1710_03038_amd.etable import load_table

    table = load_table()
    paper = {}
    for line in open(os.path.join(ROOT, PAPER_MPR)):
        if line.startswith("#") or not line.strip():
            continue
        kappa, nu, L, case, *vals = line.split()
        paper[(float(nu), int(L), case)] = dict(zip(("MAAE", "MARE", "MAARE", "MRASE", "MR"), map(float, vals)))
    dev = torch.device("cuda:0")
    for L in Ls:
        n_cfg = S or (100 if L <= 256 else 40 if L <= 512 else 16 if L <= 1024 else 6)
        for nu in (0.5, 0.25):
            for case in ("a", "b", "c"):
                zt = torch.empty((L, L), dtype=torch.float64, device=dev)
                kt = torch.empty((L, L), dtype=torch.uint8, device=dev)
                f = None
                rows, secs, eqs = [], [], []
                for s in range(n_cfg):
                    base = 100000 * L + 1000 * int(nu * 100) + 10 * ord(case) + s
                    z = mprgen.matern_field(L, L, 0.2, nu, base, mean=50.0, std=10.0)
                    known = (mprgen.mask_block(L, L, 20, base + 1) if case == "c"
                             else mprgen.mask_random(L, L, {"a": 0.33, "b": 0.66}[case], base + 1))
                    zt.copy_(torch.from_numpy(z))
                    kt.copy_(torch.from_numpy(known))
                    if f is None:
                        f = M.Field([(zt, kt, 1)], M.default_params(dtype="fp32", seed=base + 2))
                        f.set_graph(True)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    f.reinit()
                    e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
                    T, _ = M.match_T(e_s, table[0], table[1])
                    n, _, _ = f.equilibrate(T, n_f=5, n_fit=20, i_max=2000)
                    zh, _, _ = f.fill(T, 0, 100, 1)
                    m = f.validation_measures(0, zt, zh[0])
                    secs.append(time.perf_counter() - t0)
                    eqs.append(n)
                    rows.append(m)
                f.close()
                mean = {k: float(np.mean([r[k] for r in rows])) for k in ("AAE", "ARE", "AARE", "RASE", "R")}
                out = {"study": "validation", "L": L, "kappa": 0.2, "nu": nu, "case": case, "S": n_cfg,
                       "MAAE": mean["AAE"], "MARE_pct": 100 * mean["ARE"], "MAARE_pct": 100 * mean["AARE"],
                       "MRASE": mean["RASE"], "MR_pct": 100 * mean["R"],
                       "MAAE_sd": float(np.std([r["AAE"] for r in rows])), "eq_sweeps_mean": float(np.mean(eqs)),
                       "ms_per_configuration": 1e3 * float(np.mean(secs)),
                       "paper": paper.get((nu, L, case))}
                print(json.dumps(out), flush=True)


def gmrf_study(S, L=32):
    """The paper's comparison of the MPR and GMRF pair interactions (Sec.
    4.4): S configurations of L x L WM(kappa, nu) data, Gaussian
    (mean 50, std 10) or lognormal (log Z with mean 5, std 1), case a: 33 %
    random gaps, b: 66 %, c: one 20 x 20 block; each model with its own e(T)
    table for SEM, Savitzky-Golay equilibration and M = 100 recorded sweeps.
    All S configurations of a row run as one batch (one grid each).  One
    JSON line per row, with the paper's values where printed."""
    import torch

    import mprgen
    from paper_1710_03038_amd import mpr as M
    from paper_1710_03038_amd.etable import load_table

    paper = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_mpr_gmrf.txt")):
        if line.startswith("#") or not line.strip():
            continue
        dist, nu, kappa, model, case, *vals = line.split()
        paper[(dist, float(nu), float(kappa), model, case)] = dict(
            zip(("MAAE", "MARE", "MAARE", "MRASE", "MR"), map(float, vals)))
    dev = torch.device("cuda:0")
    for dist in ("gaussian", "lognormal"):
        for nu in (0.5, 0.25):
            for kappa in (0.5, 0.2):
                for case in ("a", "b", "c"):
                    grids = []
                    for s in range(S):
                        base = 700000 + 1000 * s + 100 * int(kappa * 10) + int(nu * 100) + ord(case)
                        y = mprgen.matern_field(L, L, kappa, nu, base, mean=0.0, std=1.0)
                        z = 50.0 + 10.0 * y if dist == "gaussian" else np.exp(5.0 + y)
                        known = (mprgen.mask_block(L, L, 20, base + 1) if case == "c"
                                 else mprgen.mask_random(L, L, {"a": 0.33, "b": 0.66}[case], base + 1))
                        grids.append((torch.from_numpy(z).to(dev), torch.from_numpy(known).to(dev), 1))
                    for model in ("mpr", "gmrf"):
                        table = load_table(model=model)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        f = M.Field(grids, M.default_params(dtype="fp32", seed=991, model=model))
                        e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
                        T, _ = M.match_T(e_s, table[0], table[1])
                        n, _, _ = f.equilibrate(T, n_f=5, n_fit=20, i_max=2000)
                        zh, _, _ = f.fill(T, 0, 100, 1)
                        ms = [f.validation_measures(g, grids[g][0], zh[g]) for g in range(S)]
                        f.close()
                        dt = time.perf_counter() - t0
                        aae = np.array([m["AAE"] for m in ms])
                        out = {"study": "gmrf", "distribution": dist, "nu": nu, "kappa": kappa, "model": model,
                               "case": case, "L": L, "S": S,
                               "MAAE": float(aae.mean()), "MARE_pct": 100 * float(np.mean([m["ARE"] for m in ms])),
                               "MAARE_pct": 100 * float(np.mean([m["AARE"] for m in ms])),
                               "MRASE": float(np.mean([m["RASE"] for m in ms])),
                               "MR_pct": 100 * float(np.mean([m["R"] for m in ms])),
                               "AAE_quartiles": [float(v) for v in np.percentile(aae, [25, 50, 75])],
                               "eq_sweeps": n, "seconds_for_S": dt,
                               "paper": paper.get((dist, nu, kappa, model, case))}
                        print(json.dumps(out), flush=True)


def boundary_study(S, Ls, kappa=0.2, band=4, inner=8):
    """Replicate auxiliary nodes (Sec. 2.5) against open boundaries.  S
    configurations of L x L WM(kappa, nu) data (mean 50, std 10), case a:
    33 % random gaps, b: 66 %; all S as one batch (one grid each), run once
    with each boundary from the same seed: e_s, T-hat by SEM (open-boundary
    table), Savitzky-Golay equilibration (n_f = 5, n_fit = 20), M = 100
    recorded sweeps.  Errors (GPU validation measures) over all gaps, the
    gaps on the grid's edge, those within ``band`` sites of it, and those
    more than ``inner`` sites in.  One JSON line per (L, nu, case, boundary)."""
    import torch

    import mprgen
    from paper_1710_03038_amd import mpr as M
    from paper_1710_03038_amd.etable import load_table

    table = load_table()
    dev = torch.device("cuda:0")
    for L in Ls:
        yy, xx = np.mgrid[0:L, 0:L]
        dist = np.minimum(np.minimum(yy, L - 1 - yy), np.minimum(xx, L - 1 - xx))
        regions = {"all": np.ones((L, L), bool), "edge": dist == 0, "band": dist < band, "interior": dist >= inner}
        for nu in (0.5, 0.25):
            for case in ("a", "b"):
                grids, zs = [], []
                for s in range(S):
                    base = 400000 + 1000 * s + int(nu * 100) + ord(case) + 7 * L
                    z = mprgen.matern_field(L, L, kappa, nu, base, mean=50.0, std=10.0)
                    known = mprgen.mask_random(L, L, {"a": 0.33, "b": 0.66}[case], base + 1)
                    grids.append((torch.from_numpy(z).to(dev), torch.from_numpy(known).to(dev), 1))
                    zs.append(z)
                zsub = {r: [torch.from_numpy(np.where(m, z, np.nan)).to(dev) for z in zs]
                        for r, m in regions.items()}
                for bc in ("open", "replicate"):
                    f = M.Field(grids, M.default_params(dtype="fp32", seed=4242, boundary=bc))
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
                    T, _ = M.match_T(e_s, table[0], table[1])
                    n, _, _ = f.equilibrate(T, n_f=5, n_fit=20, i_max=2000)
                    zh, _, _ = f.fill(T, 0, 100, 1)
                    torch.cuda.synchronize()
                    secs = time.perf_counter() - t0
                    out = {"study": "boundary", "L": L, "kappa": kappa, "nu": nu, "case": case, "S": S,
                           "boundary": bc, "eq_sweeps": int(n), "ms_per_batch": 1e3 * secs}
                    for r in regions:
                        ms = [f.validation_measures(g, zsub[r][g], zh[g]) for g in range(S)]
                        out[r] = {"MAAE": float(np.mean([m["AAE"] for m in ms])),
                                  "MRASE": float(np.mean([m["RASE"] for m in ms])),
                                  "MR_pct": 100 * float(np.mean([m["R"] for m in ms])),
                                  "sites": int(np.mean([m["P"] for m in ms]))}
                    f.close()
                    print(json.dumps(out), flush=True)


def qcv_study(S, L=64, qs=(0.125, 0.25, 0.375, 0.5), n_folds=5):
    """Choice of q by cross-validation (the extension proposed in Sec. 6).
    Data: L x L fields, S configurations each, case a (33 % random gaps):
    Gaussian 50 + 10 WM(0.2, 0.5), rough Gaussian 50 + 10 WM(0.5, 0.25),
    and lognormal exp(5 + WM(0.5, 0.5)).  Per configuration: mpr_cv_select_q
    over the candidates with n_folds folds of the samples (FP32, 100 + 100
    sweeps per fit, every sweep recorded), timed; then the method at every
    candidate on the true gaps, all S x n_q fits as one batch with per-grid
    q (e_s, SEM on each q's table, Savitzky-Golay equilibration, M = 100).
    One JSON line per data kind: mean CV score and true AAE per q, how often
    CV picked each q, and the true AAE at the CV choice, at q = 1/2 and at
    the best q in hindsight."""
    import torch

    import mprgen
    from paper_1710_03038_amd import mpr as M
    from paper_1710_03038_amd.etable import load_table

    dev = torch.device("cuda:0")
    tables = [load_table(q=q)[:2] for q in qs]
    nq = len(qs)
    kinds = {"gaussian": (0.2, 0.5, lambda y: 50.0 + 10.0 * y), "rough": (0.5, 0.25, lambda y: 50.0 + 10.0 * y),
             "lognormal": (0.5, 0.5, lambda y: np.exp(5.0 + y))}
    for kind, (kappa, nu, tr) in kinds.items():
        data = []
        for s in range(S):
            base = 810000 + 1000 * s + 7 * len(kind)
            z = tr(mprgen.matern_field(L, L, kappa, nu, base, mean=0.0, std=1.0))
            known = mprgen.mask_random(L, L, 0.33, base + 1)
            fold = mprgen.cv_folds(known, n_folds, base + 2)
            data.append((torch.from_numpy(z).to(dev), torch.from_numpy(known).to(dev), torch.from_numpy(fold).to(dev)))
        cv, secs = [], []
        for s, (zt, kt, ft) in enumerate(data):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cv.append(M.cv_select_q(zt, kt, ft, n_folds, qs, tables, 100, 100, 1,
                                    params=M.default_params(dtype="fp32", seed=77 + s)))
            secs.append(time.perf_counter() - t0)
        grids = [(zt, kt, 1) for zt, kt, _ in data for _ in qs]
        f = M.Field(grids, M.default_params(dtype="fp32", seed=991))
        f.set_grid_q(np.tile(np.asarray(qs, dtype=np.float64), S))
        e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
        T = np.array([M.match_T(e_s[g:g + 1], *tables[g % nq])[0][0] for g in range(S * nq)])
        n, _, _ = f.equilibrate(T, n_f=5, n_fit=20, i_max=2000)
        zh, _, _ = f.fill(T, 0, 100, 1)
        true = np.array([f.validation_measures(g, data[g // nq][0], zh[g])["AAE"] for g in range(S * nq)]).reshape(S, nq)
        f.close()
        pick = np.array([c["best"] for c in cv])
        out = {"study": "qcv", "data": kind, "kappa": kappa, "nu": nu, "L": L, "S": S, "folds": n_folds,
               "q": list(qs), "cv_aae_mean": [float(np.mean([c["aae"][i] for c in cv])) for i in range(nq)],
               "picked": [int((pick == i).sum()) for i in range(nq)],
               "true_aae_mean": [float(v) for v in true.mean(axis=0)],
               "true_aae_at_cv_choice": float(true[np.arange(S), pick].mean()),
               "true_aae_at_q_half": float(true[:, qs.index(0.5)].mean()),
               "true_aae_at_best_q": float(true.min(axis=1).mean()),
               "T_hat_over_q2": [float(np.mean([c["T_mean"][i] for c in cv]) / qs[i] ** 2) for i in range(nq)],
               "eq_sweeps": int(n), "ms_per_cv": 1e3 * float(np.mean(secs)), "fits_per_cv": nq * n_folds}
        print(json.dumps(out), flush=True)


def copy_calibration(nbytes=256 << 20, reps=10):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters of rocprofv3 to bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
                      "GBps": 2 * nbytes / dt / 1e9}), flush=True)


def _batch_grid(spec):
    import mprgen
    return mprgen.batch_grid(spec)


def load_workload(name):
    """Host inputs of a named workload: grids [(z, known)], chains per grid,
    sweep counts, Philox seed and a description."""
    import mprgen
    if name == "uneven2000":
        specs = mprgen.uneven_batch(2000, seed=401)
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
            grids = pool.map(_batch_grid, specs, chunksize=8)
        return dict(grids=grids, chains=[1] * len(grids), n_eq=100, n_samp=100, stride=1, seed=403,
                    config={"grids": len(grids), "sides": "log-uniform [32, 2048]", "gap_fraction_per_grid":
                            "U(0.1, 0.9)", "field": "Gaussian or lognormal", "chains": 1})
    z, known, spec = mprgen.workload(name)
    return dict(grids=[(z, known)], chains=[spec["chains"]], n_eq=spec["n_eq"], n_samp=spec["n_samp"],
                stride=spec["stride"], seed=spec["seed"],
                config={"grid": [spec["n"], spec["n"]], "field": spec["field"], "corr_len": spec["corr_len"],
                        "mask": spec["mask"], "chains": spec["chains"]})


def one_step(M, f, W, table, tune, timing=False, shape=None):
    """One pass of the whole path on a set-up context: hot start from the
    resident inputs (mpr_reinit), e_s, T-hat by SEM, launch shape (cached
    after the first tuning), fill."""
    f.reinit()
    if timing:
        f.set_timing(True)
    e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
    T, _ = M.match_T(e_s, table[0], table[1])
    tuned = f.autotune(T, 16) if tune else (shape or (f.params.sweeps_per_pass, None, None, None))
    zh, zs, rep = f.fill(T, W["n_eq"], W["n_samp"], W["stride"])
    kt = f.timing() if timing else (0.0, 0, 0)
    return dict(zh=zh, zs=zs, rep=rep, T=T, e_s=e_s, kt=kt, tuned=tuned)


def run_arm(M, dev_grids, W, table, params, steps, warmup, graph, tune=True, shape=None):
    """Batched arm: one context over every grid and chain of the workload.
    Host set-up (context, workspace) once, outside the timed region; the
    timed steps run the whole path on the device."""
    import torch
    tune = tune and params.dtype == M.FP32
    f = M.Field(dev_grids, params)
    f.set_graph(graph)
    if shape:
        f.set_launch_shape(*shape)
        tune = False
    for _ in range(warmup):
        one_step(M, f, W, table, tune, shape=shape)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = kl = kss = 0
    out = None
    for _ in range(steps):
        out = one_step(M, f, W, table, tune, timing=True, shape=shape)
        kms += out["kt"][0]
        kl += out["kt"][1]
        kss += out["kt"][2]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    f.close()
    return dt, out, (kms, kl, kss)


def run_plain_arm(M, dev_grids, W, table, params, steps, warmup):
    """Plain per-grid arm: each grid in a context of its own (its chains
    together), run one after the other; the step time is the sum over the
    grids.  No graph and no autotuning; the caller's params fix the
    precision and sweeps per pass."""
    import torch
    dt = 0.0
    outs = []
    for g, grid in enumerate(dev_grids):
        wg = dict(W, grids=[W["grids"][g]])
        f = M.Field([grid], params)
        for _ in range(warmup):
            one_step(M, f, wg, table, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = None
        for _ in range(steps):
            out = one_step(M, f, wg, table, False)
        torch.cuda.synchronize()
        dt += (time.perf_counter() - t0) / steps
        outs.append(out)
        f.close()
        del f
    zh = [o["zh"][0] for o in outs]
    zs = [o["zs"][0] for o in outs]
    return dt, dict(zh=zh, zs=zs, rep=outs[0]["rep"], T=np.concatenate([o["T"] for o in outs]),
                    e_s=np.concatenate([o["e_s"] for o in outs]))


def fill_mae(W, zh, zs, chains):
    """Gap-fill MAE against the held-out truth, and a bound on its Monte
    Carlo standard error: the prediction at a gap site is a mean of R
    recorded states, so its error has standard deviation z_std / sqrt(R)
    for independent records, and the MAE moves by at most the mean of
    those errors; their root-mean-square over the gaps is reported as
    sigma (R = records per chain x chains)."""
    err = n = 0.0
    var = 0.0
    for (z, known), h, s, r in zip(W["grids"], zh, zs, chains):
        gap = known == 0
        err += float(np.abs(h.cpu().numpy()[gap] - z[gap]).sum())
        var += float((s.cpu().numpy()[gap] ** 2).sum()) / r
        n += int(gap.sum())
    return err / n, math.sqrt(var / n)


def cpu_baseline(W, T, budget_s=10.0, max_side=1024, boundary="open"):
    """The FP64 NumPy oracle timed on this host on a bounded sample of the
    same workload: hybrid sweeps (with the a-rule) of its grids in order,
    each cut to at most max_side x max_side, until budget_s has elapsed."""
    from oracle import mpr as om
    done = 0
    spent = 0.0
    used = []
    for g, (z, known) in enumerate(W["grids"]):
        kn = known.astype(bool)
        zc, kc = z[:max_side, :max_side], kn[:max_side, :max_side]
        phi_s, _, _ = om.transform(zc, kc, bounds=(float(z[kn].min()), float(z[kn].max())))
        phi = om.hot_start(phi_s, kc, W["seed"], [0], g)
        P = int((~kc).sum())
        s = 0
        t0 = time.perf_counter()
        while s < 2 or (time.perf_counter() - t0 < budget_s - spent and s < 1000):
            phi, _, _, _ = om.run_sweeps(phi, kc, T[g], 1.0, 0.5, W["seed"], s, 1, [0], g, adapt=True,
                                         boundary=boundary)
            s += 1
        spent += time.perf_counter() - t0
        done += s * P
        used.append((zc.shape, s))
        if spent >= budget_s:
            break
    return done / spent, spent, used


def oracle_scalars(W, table, max_grids=4):
    """Eq. (4) and T-hat by the FP64 oracle (NumPy pair sums, scipy PCHIP
    and Brent) on the first grids of the workload, for the error of the
    GPU results against it."""
    from oracle import mpr as om
    e_o, T_o = [], []
    for z, known in W["grids"][:max_grids]:
        kn = known.astype(bool)
        phi_s, _, _ = om.transform(z, kn)
        e, _, _ = om.sample_specific_energy(phi_s, kn, 0.5)
        e_o.append(e)
        T_o.append(float(om.match_T([e], table[0], table[1])[0][0]))
    return np.array(e_o), np.array(T_o)


# The paper's own timing (Sec. 4.1.3, table of MPR validation measures):
# Matlab on one desktop CPU, mean CPU time of one conditional simulation
# (SEM, about 50 hybrid equilibration sweeps, M = 100 recorded sampling
# sweeps) over S = 100 configurations of WM(0.2, 0.5) data.
PAPER_TIMING = {
    "hardware": "Intel Core i7-4790 3.60 GHz, 16 GB RAM, Matlab (Sec. 3)",
    "workload": "L = 2048, case (b): 66 % random gaps, WM(kappa = 0.2, nu = 0.5), one chain",
    "t_cpu_s_per_simulation": 149.11,
    "spin_updates_per_s_derived": 150 * 2768240 / 149.11,
    "derivation": "about 150 sweeps (50 equilibration + 100 sampling) x floor(0.66 * 2048^2) gap sites / t_cpu",
    "note": "another machine and a smaller workload: context, not a target",
}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid8192x64chains")
    ap.add_argument("--sweeps-per-pass", type=int, default=0)
    ap.add_argument("--tile", type=int, nargs=2, default=(0, 0))
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="timed steps of the plain FP64 arm (each several seconds on the default workload)")
    ap.add_argument("--fp64-warmup", type=int, default=1)
    ap.add_argument("--shape", type=int, nargs=4, default=None, metavar=("NSW", "THREADS", "THREADS1", "PERSIST1"),
                    help="fix the launch shape (sweeps per pass, workgroup size, workgroup size of single-sweep "
                         "passes, 1 for persistent single-sweep workgroups) instead of autotuning it, e.g. for "
                         "profiling runs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape (for profiling runs, whose timing would sway "
                         "the autotuner)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--boundary", choices=["open", "replicate"], default="open",
                    help="sweep boundary: open, or the replicate auxiliary nodes of Sec. 2.5")
    ap.add_argument("--study", choices=["relaxation", "validation", "gmrf", "boundary", "qcv"], default=None,
                    help="relaxation: energy relaxation of the hybrid, restricted and standard Metropolis updates "
                         "and their Savitzky-Golay equilibration points (L x L Whittle-Matern field, p gaps); "
                         "validation: the paper's MPR validation measures on WM(0.2, nu) data, one JSON line per "
                         "(L, nu, case); gmrf: MPR against the GMRF pair interaction on Gaussian and lognormal "
                         "WM data, L = 32; boundary: replicate auxiliary nodes against open boundaries, "
                         "errors at the edge and in the interior; qcv: the choice of q by cross-validation on "
                         "Gaussian, rough and lognormal data")
    ap.add_argument("--Ls", type=int, nargs="+", default=[256, 512, 1024])
    ap.add_argument("--S", type=int, default=0, help="configurations per row (0: 100 at L <= 256, then fewer)")
    ap.add_argument("--L", type=int, default=512)
    ap.add_argument("--p", type=float, default=0.9)
    ap.add_argument("--sweeps", type=int, default=20000)
    ap.add_argument("--field", choices=["wm", "se16"], default="wm",
                    help="relaxation study input: WM(0.5, 0.5) (the paper's) or squared-exponential, length 16")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the benchmark measures one GPU; chains and "
              "grids would shard across GPUs with no exchange during sweeps.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.study == "relaxation":
        relaxation_study(args.L, args.p, args.sweeps, field=args.field)
        return
    if args.study == "validation":
        validation_study(args.Ls, args.S)
        return
    if args.study == "gmrf":
        gmrf_study(args.S or 100)
        return
    if args.study == "boundary":
        boundary_study(args.S or 100, args.Ls)
        return
    if args.study == "qcv":
        qcv_study(args.S or 40)
        return

    import torch

    from paper_1710_03038_amd import mpr as M
    from paper_1710_03038_amd.etable import load_table

    M.lib()
    table = load_table()
    t_in = time.perf_counter()
    W = load_workload(args.workload)
    print("inputs drawn: %s in %.1f s" % (args.workload, time.perf_counter() - t_in), file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    dev_grids = [(torch.from_numpy(z).to(dev), torch.from_numpy(k).to(dev), c)
                 for (z, k), c in zip(W["grids"], W["chains"])]
    gaps = [int((k == 0).sum()) for _, k in W["grids"]]
    sites = [int(k.size) for _, k in W["grids"]]
    P = sum(g * c for g, c in zip(gaps, W["chains"]))
    p = sum(gaps) / sum(sites)
    sweeps = W["n_eq"] + W["n_samp"]
    updates = sweeps * P

    prm32 = M.default_params(dtype="fp32", seed=W["seed"], sweeps_per_pass=args.sweeps_per_pass,
                             tile_x=args.tile[0], tile_y=args.tile[1], boundary=args.boundary)
    tile_tuned = None
    if not args.no_autotune and tuple(args.tile) == (0, 0):
        # Set-up, untimed: the tile shape (and the depth its LDS allows) at
        # the workload's own T, chosen before the context is built.
        f0 = M.Field(dev_grids, prm32)
        T0, _ = M.match_T(f0.specific_energy(M.SAMPLE_PAIRS)[0], table[0], table[1])
        f0.close()
        del f0
        # trial runs of 16 sweeps on small batches, 8 on batches of 2.5e7
        # sites or more (shorter runs let one-off delays sway the choice)
        site_chains = sum(k.size * c for (_, k), c in zip(W["grids"], W["chains"]))
        trial = int(np.clip(16 * 1.25e7 / site_chains, 8, 16))
        tile_tuned = M.autotune_tile(dev_grids, T0, W["n_eq"], W["n_samp"], params=prm32, trial_sweeps=trial)
        prm32.tile_x, prm32.tile_y, prm32.sweeps_per_pass = tile_tuned
        print("tile autotuned: %d x %d, up to %d sweeps per pass" % tile_tuned, file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    dt32, out32, (kms, kl, kss) = run_arm(M, dev_grids, W, table, prm32, args.steps, args.warmup, graph=True,
                                          tune=not args.no_autotune, shape=args.shape)
    print("FP32 arm: %.1f ms per step" % (dt32 * 1e3), file=sys.stderr, flush=True)
    records_per_chain = out32["rep"]["records"]
    mae32, sig32 = fill_mae(W, out32["zh"], out32["zs"], [records_per_chain * c for c in W["chains"]])
    records = records_per_chain * sum(W["chains"])
    T_hat = out32["T"]
    e_s32 = out32["e_s"]
    tuned = out32["tuned"]
    del out32
    torch.cuda.empty_cache()

    # Plain FP64 arm: a context per grid, FP64 library math, one sweep per
    # pass, the library's default tile, no graph and no autotuning.
    fp64 = None
    e_s64 = T64 = None
    if args.fp64_steps > 0:
        prm64 = M.default_params(dtype="fp64", seed=W["seed"], sweeps_per_pass=1, boundary=args.boundary)
        dt64, out64 = run_plain_arm(M, dev_grids, W, table, prm64, args.fp64_steps, args.fp64_warmup)
        print("FP64 plain arm: %.1f ms per step" % (dt64 * 1e3), file=sys.stderr, flush=True)
        mae64, sig64 = fill_mae(W, out64["zh"], out64["zs"], [out64["rep"]["records"] * c for c in W["chains"]])
        sigma = math.sqrt(sig32 ** 2 + sig64 ** 2)
        e_s64, T64 = out64["e_s"], out64["T"]
        fp64 = {"spin_updates_per_s": updates / dt64, "realisations_per_s": records / dt64,
                "ms_per_step": dt64 * 1e3, "steps": args.fp64_steps, "warmup": args.fp64_warmup,
                "arm": "one context per grid, FP64, one sweep per pass, default tile, no graph, no autotuning",
                "mae": mae64, "mae_sigma": sig64,
                "mae_diff_over_sigma": abs(mae32 - mae64) / sigma if sigma > 0 else None,
                "equal_mae_3sigma": abs(mae32 - mae64) <= 3 * sigma,
                "speedup_fp32_over_fp64": dt64 / dt32}
        del out64
        torch.cuda.empty_cache()

    b_site = bytes_per_site_sweep(4, p)
    ksec = kms * 1e-3
    useful_updates = kss * p  # gap-site updates of the timed sweep launches (halo work excluded)
    cyc = CYC_PER_UPDATE
    achieved = useful_updates * cyc / ksec / 1e12 if kms > 0 else None
    avg_us = kms * 1e3 / kl if kl else None
    # algorithmic one-pass bytes per launch: each launch passes over every site once
    sites_all = sum(int(z.size) * c for (z, _), c in zip(W["grids"], W["chains"]))
    alg_bytes = sites_all * b_site if kl else None
    hbm_gbs = alg_bytes / (avg_us * 1e-6) / 1e9 if avg_us else None
    traffic = profiled_traffic(args.workload, tuple(tuned)[:4], tile_tuned or tuple(args.tile), False) \
        if args.boundary == "open" and "MPR_SWEEP_THREADS" not in os.environ else None
    cfg = dict(W["config"])
    cfg.update({"workload": args.workload, "boundary": args.boundary, "gap_fraction": p, "n_eq": W["n_eq"],
                "n_samp": W["n_samp"], "stride": W["stride"], "tile": [prm32.tile_x or 64, prm32.tile_y or 64],
                "tile_autotuned": tile_tuned is not None,
                "sweeps_per_pass_max": prm32.sweeps_per_pass or 8,
                "autotuned_shape": {"sweeps_per_pass": tuned[0], "threads": tuned[1],
                                    "threads_single_sweep_passes": tuned[2],
                                    "persistent_single_sweep_passes": tuned[3]}, "fill_graph": True,
                "T_hat": float(T_hat[0]) if len(T_hat) == 1 else [float(T_hat.min()), float(T_hat.max())],
                "e_s": float(e_s32[0]) if len(T_hat) == 1 else None})
    res = {
        "metric": METRIC,
        "value": updates / dt32,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (seeded Gaussian/lognormal random fields and gap masks; no dataset)",
        "config": cfg,
        "realisations_per_s": records / dt32,
        "fills_per_s": len(W["grids"]) / dt32,
        "mae_fp32": mae32,
        "mae_fp32_sigma": sig32,
        "fp64_plain": fp64,
        "roofline": {"bound": "alu", "kernel": "k_sweep<float> (every sweep launch of the fill)",
                     "achieved": achieved, "peak": VALU_PEAK_TCYC,
                     "unit": "T SIMD issue-cycles/s (useful updates x their VALU issue cycles)",
                     "frac": (achieved / VALU_PEAK_TCYC) if achieved else None,
                     "traffic": traffic,
                     "alu_frac": (achieved / VALU_PEAK_TCYC) if achieved else None,
                     "hbm_achieved_GBps": hbm_gbs, "hbm_peak_GBps": HBM_PEAK_GBS,
                     "hbm_frac": hbm_gbs / HBM_PEAK_GBS if hbm_gbs else None,
                     "hbm_measured_GBps": traffic / (avg_us * 1e-6) / 1e9 if traffic and avg_us else None,
                     "hbm_measured_frac": traffic / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS if traffic and avg_us else None,
                     "hbm_note": "hbm_frac: one-pass algorithmic bytes per launch over its time (effective bandwidth); "
                                 "hbm_measured_*: profiled FETCH_SIZE + WRITE_SIZE bytes per launch over the same time",

                     "hbm_algorithmic_bytes_per_launch": alg_bytes, "bytes_per_site_sweep": b_site,
                     "issue_cycles_per_update": cyc, "avg_launch_us": avg_us, "launches": kl,
                     "site_sweeps_per_launch": kss / kl if kl else None},
        "paper_timing": PAPER_TIMING,
    }
    if not args.no_cpu:
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        v, dt, used = cpu_baseline(W, T_hat, budget_s=args.cpu_seconds, boundary=args.boundary)
        desc = ", ".join(f"{s} sweeps of {sh[0]}x{sh[1]}" for sh, s in used[:4]) + (" ..." if len(used) > 4 else "")
        res["cpu_baseline"] = {"value": v, "unit": "spin-updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"{desc} (1 chain each, from the hot start, a-rule on), FP64 NumPy oracle, "
                                         f"one thread, {dt:.1f} s on {platform.processor() or platform.machine()}"}
        # Error of the GPU's Eq. (4) and T-hat against the FP64 oracle (the
        # oracle's pair sums and scipy root-find on the same table).
        e_o, T_o = oracle_scalars(W, table)
        k = len(e_o)
        errs = {"grids": k, "e_s_rel_err_fp32": float(np.max(np.abs(e_s32[:k] / e_o - 1))),
                "T_hat_rel_err_fp32": float(np.max(np.abs(T_hat[:k] / T_o - 1)))}
        if e_s64 is not None:
            errs["e_s_rel_err_fp64"] = float(np.max(np.abs(e_s64[:k] / e_o - 1)))
            errs["T_hat_rel_err_fp64"] = float(np.max(np.abs(T64[:k] / T_o - 1)))
        res["vs_fp64_oracle"] = errs
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
