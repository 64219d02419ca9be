"""Benchmark: radiance-cascades formal solve on one MI355X.

A step is one formal solve of the 1024 x 1024, 64-wavelength, 7-cascade line
medium (seed 2): prep, every cascade's fused march + merge, J. Inputs are
resident in HBM before the timed region. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ray-intervals/s + s per converged non-LTE solve, plain vs learned/FP16"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell step and wavelength: chi and S, FP32 each.
BYTES_PER_STEP = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--waves", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 1 GiB (known traffic) three times, "
                         "to scale hardware byte counters")
    ap.add_argument("--cpu-waves", type=int, default=1,
                    help="wavelengths of the same workload the FP64 oracle solves for the CPU baseline")
    return ap.parse_args()


def algorithmic_bytes(work, n_wave):
    """Bytes the fused march+merge kernels touch per solve: chi and S per cell
    step, the cascade above read once, the merged cascade written once."""
    b = 0
    n = work.n_cascades
    for i in range(n):
        if work.top_skipped and i == n - 1:
            continue
        b += work.level_steps[i] * n_wave * BYTES_PER_STEP
        b += work.level_rays[i] * n_wave * 4  # write merged cascade i
        up_read = i + 1 < n and not (work.top_skipped and i + 1 == n - 1)
        if up_read:
            b += work.level_rays[i + 1] * n_wave * 4
    return b


def measured_traffic(kernel_file: str, profile: str):
    """HBM bytes per launch of the march kernel from the committed rocprofv3
    counter summary, or None when the kernel source changed since."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        src = open(os.path.join(ROOT, "paper_2408_14425_amd", "csrc", kernel_file), "rb").read()
    except OSError:
        return None
    h = re.search(r"kernel_source_sha256: ([0-9a-f]+)", text)
    t = re.search(r"traffic_bytes_per_launch: ([0-9.eE+-]+)", text)
    if not h or not t or h.group(1) != hashlib.sha256(src).hexdigest():
        return None
    return float(t.group(1))


def cpu_baseline(inp, n_waves: int):
    import numpy as np

    import oracle
    sel = slice(inp.n_wave // 2 - n_waves // 2, inp.n_wave // 2 - n_waves // 2 + n_waves)
    chi = inp.chi[sel].astype(np.float64)
    eta = inp.eta[sel].astype(np.float64)
    t0 = time.perf_counter()
    r = oracle.formal_solve(chi, eta, inp.n_cascades)
    dt = time.perf_counter() - t0
    return {
        "value": r["nonempty"] / dt,
        "unit": "ray-intervals/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"FP64 oracle full formal solve of {n_waves} of the 64 wavelengths "
                  f"({r['nonempty']} non-empty ray intervals, {r['steps']} cell steps) in {dt:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the formal solve of one atmosphere is "
              f"single-GPU; --gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2408_14425_amd import rcx, workloads

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4, "repeats": 3}), flush=True)
        return

    inp = workloads.line_medium(args.n, args.waves, seed=2)
    dev = torch.device("cuda:0")
    chi = torch.from_numpy(inp.chi).to(dev)
    eta = torch.from_numpy(inp.eta).to(dev)
    J = torch.empty_like(chi)
    plan = rcx.Plan(inp.nx, inp.nz, inp.n_wave)
    work = plan.work()
    for _ in range(args.warmup):
        plan.formal_solve(chi, eta, J)
    torch.cuda.synchronize()
    plan.get_timing()  # discard anything pending
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.formal_solve(chi, eta, J)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.set_timing(False)
    ms_level, ms_other, n_launch, n_solves = plan.get_timing()
    ok = bool(torch.isfinite(J).all().item())
    plan.close()

    ms_step = dt / args.steps * 1e3
    rays = work.rays_nonempty * inp.n_wave
    value = rays / (dt / args.steps)
    march_ms = sum(ms_level)
    avg_launch_s = march_ms / 1e3 / max(n_launch, 1)
    bytes_per_launch = algorithmic_bytes(work, inp.n_wave) / max(n_launch // max(n_solves, 1), 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ray-intervals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"formal solve, {inp.nx}x{inp.nz} grid, {inp.n_wave} wavelengths, "
                        f"{work.n_cascades} cascades (line medium, seed 2)",
            "nx": inp.nx, "nz": inp.nz, "n_wave": inp.n_wave, "n_cascades": work.n_cascades,
            "ray_intervals_nonempty_per_step": rays,
            "ray_intervals_all_per_step": work.rays_all * inp.n_wave,
            "cell_steps_per_step": work.cell_steps * inp.n_wave,
            "cell_steps_per_s": work.cell_steps * inp.n_wave / (dt / args.steps),
            "kernel_ms_per_cascade": [m / max(n_solves, 1) for m in ms_level],
            "kernel_ms_prep_and_J": ms_other / max(n_solves, 1),
            "finite": ok,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_march_merge",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("fs_kernels.hip", "k_march_merge_line1024_w64.md"),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_waves)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
