#!/usr/bin/env python3
"""Benchmark of the MPR gap-filling hot path on one MI355X.

One step = the whole path on one synthetic workload with inputs resident in
HBM: mpr_init_field (Eq. 2, hot start), mpr_specific_energy (Eq. 4),
mpr_match_T (SEM, Sec. 2.3) and mpr_fill (Algorithm 2 with fixed counts:
equilibration with the a-rule, sampling, conditional mean and std).

Prints one JSON line.  value = spin-updates/s (hybrid updates of gap sites,
whole job); realisations/s is reported beside it.  The default workload is
a 1024 x 1024 Gaussian field (correlation length 16, mean 50, std 10) with
50 % random gaps, 1 chain, 1000 hybrid sweeps (100 equilibration + 900
sampling, every 9th recorded: 100 realisations), FP32.  The plain FP64 arm
(one sweep per pass) and the FP64 CPU oracle are timed on the same input.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
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
# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-
# instructions per second (the published 157.3 TFLOP/s FP32 counts a packed
# two-wide FMA, 4 flops, per lane-instruction).
VALU_PEAK_TINST = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane-instructions of one FP32 gap-site update in the compiled sweep
# kernel (the update loop of k_sweep<float>: 211 VALU instructions, of
# which 21 v_mad_u64_u32 for Philox and 6 transcendental).
VALU_INST_PER_UPDATE = 211


def bytes_per_site_sweep(elem, p):
    """Algorithmic HBM bytes of one site in one single-pass sweep: read the
    angle, write it back at gap sites, one mask bit."""
    return elem * (1.0 + p) + 0.125


def load_inputs(name):
    import torch

    import mprgen
    z, known, spec = mprgen.workload(name)
    dev = torch.device("cuda:0")
    zt = torch.from_numpy(z).to(dev)
    kt = torch.from_numpy(known).to(dev)
    return z, known, zt, kt, spec


def one_step(M, zt, kt, spec, table, params, timing=False):
    f = M.Field([(zt, kt, spec["chains"])], params)
    if timing:
        f.set_timing(True)
    e_s, _ = f.specific_energy(M.SAMPLE_PAIRS)
    T, _ = M.match_T(e_s, table[0], table[1])
    zh, zs, rep = f.fill(T, spec["n_eq"], spec["n_samp"], spec["stride"])
    kt_ = f.timing() if timing else (0.0, 0, 0)
    f.close()
    return zh[0], zs[0], rep, float(T[0]), float(e_s[0]), kt_


def run_arm(M, zt, kt, spec, table, params, steps, warmup):
    import torch
    for _ in range(warmup):
        one_step(M, zt, kt, spec, table, params)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = kl = kss = 0
    out = None
    for _ in range(steps):
        out = one_step(M, zt, kt, spec, table, params, timing=True)
        kms += out[5][0]
        kl += out[5][1]
        kss += out[5][2]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, out, (kms, kl, kss)


KERNEL_SOURCES = ("paper_1710_03038_amd/csrc/kernels.hip", "paper_1710_03038_amd/csrc/fastmath.h",
                  "paper_1710_03038_amd/csrc/internal.h")
PROFILE = "profiles/k_sweep_fp32_grid1024.md"


def profiled_traffic():
    """HBM bytes per sweep launch measured by rocprofv3 (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy) for the default configuration, or
    None when the kernel sources changed since that profile was taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, PROFILE)).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+) kernel_sources_sha256: ([0-9a-f]+)", text)
    if not m or m.group(2) != h.hexdigest():
        return None
    return float(m.group(1))


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


def cpu_baseline(z, known, T, spec, sweeps):
    """The FP64 NumPy oracle timed on this host on a bounded sample: the
    first ``sweeps`` hybrid sweeps of the same workload from the hot start."""
    from oracle import mpr as om
    kn = known.astype(bool)
    phi_s, _, _ = om.transform(z, kn)
    phi = om.hot_start(phi_s, kn, spec["seed"], [0], 0)
    t0 = time.perf_counter()
    phi, a, _, _ = om.run_sweeps(phi, kn, T, 1.0, 0.5, spec["seed"], 0, sweeps, [0], 0, adapt=True)
    dt = time.perf_counter() - t0
    P = int((~kn).sum())
    return sweeps * P / dt, dt


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid1024")
    ap.add_argument("--sweeps-per-pass", type=int, default=0)
    ap.add_argument("--tile", type=int, nargs=2, default=(0, 0))
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=12)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the MPR path here is a single-GPU build; "
              "chains and grids would shard across GPUs with no exchange during sweeps.", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    from paper_1710_03038_amd import mpr as M
    from paper_1710_03038_amd.etable import load_table

    M.lib()
    table = load_table()
    z, known, zt, kt, spec = load_inputs(args.workload)
    kn = known.astype(bool)
    P = int((~kn).sum())
    N = z.size
    p = P / N
    chains = spec["chains"]
    sweeps = spec["n_eq"] + spec["n_samp"]

    prm32 = M.default_params(dtype="fp32", seed=spec["seed"], sweeps_per_pass=args.sweeps_per_pass,
                             tile_x=args.tile[0], tile_y=args.tile[1])
    dt32, out32, (kms, kl, kss) = run_arm(M, zt, kt, spec, table, prm32, args.steps, args.warmup)
    zh32 = out32[0].cpu().numpy()
    mae32 = float(np.abs(zh32[~kn] - z[~kn]).mean())
    updates = sweeps * P * chains
    records = out32[2]["records"] * chains

    # plain FP64 arm: one sweep per pass, library default tiles, same input
    fp64 = None
    if args.fp64_steps > 0:
        prm64 = M.default_params(dtype="fp64", seed=spec["seed"], sweeps_per_pass=1)
        dt64, out64, _ = run_arm(M, zt, kt, spec, table, prm64, args.fp64_steps, 0)
        zh64 = out64[0].cpu().numpy()
        mae64 = float(np.abs(zh64[~kn] - z[~kn]).mean())
        fp64 = {"spin_updates_per_s": updates / dt64, "realisations_per_s": records / dt64,
                "ms_per_step": dt64 * 1e3, "mae": mae64, "speedup_fp32_over_fp64": dt64 / dt32}

    elem = 4
    b_site = bytes_per_site_sweep(elem, p)
    default_config = (args.workload == "grid1024" and args.sweeps_per_pass == 0 and tuple(args.tile) == (0, 0)
                      and "MPR_SWEEP_THREADS" not in os.environ)
    ksec = kms * 1e-3
    hbm_gbs = kss * b_site / ksec / 1e9 if kms > 0 else None
    useful_updates = kss * p  # gap-site updates of the timed sweep launches (halo work excluded)
    achieved = useful_updates * VALU_INST_PER_UPDATE / ksec / 1e12 if kms > 0 else None
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
        "data": "synthetic (seeded Gaussian random field and random gap mask; no dataset)",
        "config": {"workload": args.workload, "grid": [spec["n"], spec["n"]], "gap_fraction": p,
                   "field": spec["field"], "corr_len": spec["corr_len"], "mask": spec["mask"], "chains": chains,
                   "n_eq": spec["n_eq"], "n_samp": spec["n_samp"], "stride": spec["stride"],
                   "sweeps_per_pass": prm32.sweeps_per_pass or 8, "tile": [prm32.tile_x or 64, prm32.tile_y or 64],
                   "T_hat": out32[3], "e_s": out32[4]},
        "realisations_per_s": records / dt32,
        "mae_fp32": mae32,
        "fp64_plain": fp64,
        "roofline": {"bound": "alu", "kernel": "k_sweep<float>",
                     "achieved": achieved, "peak": VALU_PEAK_TINST, "unit": "Tinst/s (VALU lane-instructions)",
                     "frac": (achieved / VALU_PEAK_TINST) if achieved else None,
                     "traffic": profiled_traffic() if default_config else None,
                     "inst_per_update": VALU_INST_PER_UPDATE,
                     "avg_launch_us": kms * 1e3 / kl if kl else None, "launches": kl,
                     "site_sweeps_per_launch": kss / kl if kl else None,
                     "hbm_one_pass": {"achieved_GBps": hbm_gbs, "peak_GBps": HBM_PEAK_GBS,
                                      "frac": hbm_gbs / HBM_PEAK_GBS if hbm_gbs else None,
                                      "bytes_per_site_sweep": b_site}},
    }
    if not args.no_cpu:
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        v, dt = cpu_baseline(z, known, out32[3], spec, args.cpu_sweeps)
        res["cpu_baseline"] = {"value": v, "unit": "spin-updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.cpu_sweeps} hybrid sweeps of the {spec['n']}x{spec['n']} workload "
                                         f"(1 chain, {P} gap sites) from the hot start, FP64 NumPy oracle, "
                                         f"one thread, {dt:.1f} s on {platform.processor() or platform.machine()}"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
