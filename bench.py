"""Benchmark: radiance-cascades formal solve and non-LTE iteration on one MI355X.

A step is one formal solve of the 1024 x 1024, 64-wavelength, 7-cascade line
medium (seed 2): prep, every cascade's fused march + merge, J. Inputs are
resident in HBM before the timed region. The same line also reports the
FP16-storage variant of that solve and the seconds per converged non-LTE
solve (1024 x 1024, 160 wavelengths, max relative change < 1e-3) from the
LTE start with FP32 cascade storage and from the learned warm start with
FP16 storage (when a trained network is present). Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-nlte]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ray-intervals/s + s per converged non-LTE solve, plain vs learned/FP16"
HBM_PEAK_GBS = 8000.0
# Vector ALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12
# lane operations per second (78.6 TFLOP/s of unpacked FP32 FMA; the 157.3
# TFLOP/s figure counts two-wide packed FMAs, which this code does not use).
VALU_LANE_OPS = 39.3e12
# Algorithmic VALU operations per cell step and wavelength of the march:
# optical depth y = kappa ds, e = 2^-y, 1 - e, T S, I += T S (1 - e),
# T *= e.
ALU_OPS_PER_STEP = 6
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
    ap.add_argument("--no-nlte", action="store_true", help="skip the converged non-LTE solves")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage formal solve")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the sparse formal solve (a quarter of the cells flagged)")
    ap.add_argument("--no-fix", action="store_true",
                    help="skip the formal solve with the bilinear fix")
    ap.add_argument("--no-incl", action="store_true",
                    help="skip the 2D-invariant formal solve with 8 inclinations per flatland ray")
    ap.add_argument("--c4", action="store_true",
                    help="also run the batched formal solve of 16 uneven atmospheres (256^2..2048^2, "
                         "32..256 wavelengths; ~190 GB of device memory, a few minutes)")
    ap.add_argument("--nlte-only", action="store_true",
                    help="only the converged non-LTE solves (for profiling; prints their object)")
    ap.add_argument("--nlte-variants", default="plain_fp32,learned_fp16,ng_fp32,learned_ng_fp16",
                    help="comma-separated subset of the non-LTE runs")
    ap.add_argument("--nlte-n", type=int, default=1024)
    ap.add_argument("--nlte-corona", type=float, default=0.0,
                    help="fraction of the non-LTE atmosphere turned into 1e6 K corona (for sparse_fp32)")
    ap.add_argument("--nlte-max-iter", type=int, default=300)
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2408_14425_amd", "data", "warmstart_mlp.npz"),
                    help="trained warm-start network (skipped when absent)")
    return ap.parse_args()


def algorithmic_bytes(work, n_wave):
    """Bytes the fused march+merge kernels touch per solve: chi and S per cell
    step, the cascade above read once, the merged cascade written once
    (cascade 0 writes J instead: one value per cell, its 4 directions summed
    in the kernel)."""
    b = 0
    n = work.n_cascades
    for i in range(n):
        if work.top_skipped and i == n - 1:
            continue
        b += work.level_steps[i] * n_wave * BYTES_PER_STEP
        b += (work.level_rays[i] // 4 if i == 0 else work.level_rays[i]) * n_wave * 4  # cascade i or J
        up_read = i + 1 < n and not (work.top_skipped and i + 1 == n - 1)
        if up_read:
            b += work.level_rays[i + 1] * n_wave * 4
    return b


KERNEL_SOURCES = ("march_rows.h", "fs_kernels.hip", "rcx_internal.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2408_14425_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(profile: str):
    """HBM bytes per launch of the march kernel from the committed rocprofv3
    counter summary, or None when the kernel source changed since."""
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    h = re.search(r"kernel_source_sha256: ([0-9a-f]+)", text)
    t = re.search(r"traffic_bytes_per_launch: ([0-9.eE+-]+)", text)
    if not h or not t or h.group(1) != kernel_source_hash():
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


def time_solves(plan, chi, eta, J, steps: int, warmup: int):
    """Wall time of `steps` formal solves after `warmup`, and the per-cascade
    kernel times from the plan's HIP events over the timed solves."""
    import torch
    for _ in range(warmup):
        plan.formal_solve(chi, eta, J)
    torch.cuda.synchronize()
    plan.get_timing()  # discard anything pending
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.formal_solve(chi, eta, J)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.set_timing(False)
    return dt, plan.get_timing()


def nlte_solves(args):
    """Seconds to a converged non-LTE solve (max relative change < 1e-3)
    from the LTE start with FP32 and FP16 cascade storage, and from the
    learned warm start when trained weights are present."""
    import numpy as np
    import torch

    from paper_2408_14425_amd import rcx, warmstart, workloads
    inp = workloads.nlte_atmosphere(args.nlte_n, seed=3, n_line=64, n_cont=32, corona_frac=args.nlte_corona)
    corona = f", {args.nlte_corona:.0%} of the cells 1e6 K corona" if args.nlte_corona > 0 else ""
    out = {"workload": f"non-LTE iteration, {inp.nx}x{inp.nz} grid, {inp.n_wave} wavelengths "
                       f"(2 lines x 64 + 32 continuum), synthetic 3-level + continuum atom, seed 3{corona}, "
                       f"stop at max relative change < 1e-3",
           "tol": 1e-3}
    net = None
    if os.path.exists(args.weights):
        net, fn, tn = warmstart.load(args.weights)
    runs = [("plain_fp32", rcx.RCX_STORE_F32, False), ("plain_fp16", rcx.RCX_STORE_F16_SCALED, False),
            ("ng_fp32", rcx.RCX_STORE_F32, False), ("charge_fp32", rcx.RCX_STORE_F32, False),
            ("sparse_fp32", rcx.RCX_STORE_F32, False)]
    if net is not None:
        runs += [("learned_fp32", rcx.RCX_STORE_F32, True), ("learned_fp16", rcx.RCX_STORE_F16_SCALED, True),
                 ("learned_ng_fp16", rcx.RCX_STORE_F16_SCALED, True)]
    wanted = set(args.nlte_variants.split(","))
    runs = [r for r in runs if r[0] in wanted]
    final = {}
    for name, storage, learned in runs:
        s = rcx.Nlte(inp, storage=storage)
        # one untimed iteration from LTE warms the kernels up
        p = s.lte()
        s.iterate(p, 1, 0.0)
        torch.cuda.synchronize()
        if "ng_" in name:
            # Ng acceleration (not in the paper): order 2, first after 4
            # iterations, then every 4
            s.set_acceleration(2, 4, 4)
        if "sparse" in name:
            # sparsity: cells below 250 kK flagged, the corona left out
            out.setdefault("flagged_probes_per_cascade", s.set_temperature_cut(2.5e5))
        if "charge" in name:
            # charge conservation: a Newton-Raphson step on the populations
            # and n_e after each equilibrium step
            s.set_charge_conservation(True)
        t0 = time.perf_counter()
        p = s.warm_start(net, fn, tn) if learned else s.lte()
        it, rc, ch = 0, 1, float("inf")
        hist = []  # (iterations, change) after each chunk
        while rc != 0 and it < args.nlte_max_iter:
            # chunks of the same iteration, so that progress is visible
            rc, k, ch = s.iterate(p, min(5, args.nlte_max_iter - it), 1e-3)
            it += k
            hist.append((it, ch))
            print(f"[bench] non-LTE {name}: {it} iterations, change {ch:.3e}, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        final[name] = p
        if name == "plain_fp32":
            # emergent spectra of the converged atmosphere along a beam of
            # parallel long characteristics
            n_em = int(math.ceil(inp.nx * 0.6 + inp.nz * 0.8)) + 2
            s.emergent(p, 0.8, 0.6, n_em)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(5):
                s.emergent(p, 0.8, 0.6, n_em)
            torch.cuda.synchronize()
            out["emergent_spectra"] = {"direction": [0.8, 0.6], "rays": n_em,
                                       "ms_per_image": (time.perf_counter() - t1) / 5 * 1e3}
        s.close()
        out[name] = {"seconds": dt, "iterations": it, "last_change": ch, "converged": rc == 0,
                     "s_per_iteration": dt / max(it, 1)}
        # distance to the fixed point estimated from the contraction rate of
        # the last chunks: rho per iteration, error ~ change * rho / (1 - rho)
        if len(hist) >= 3 and hist[-3][1] > 0 and ch > 0:
            rho = (ch / hist[-3][1]) ** (1.0 / max(it - hist[-3][0], 1))
            if rho < 1.0:
                out[name]["contraction_per_iteration"] = rho
                out[name]["error_estimate"] = ch * rho / (1.0 - rho)
        print(f"[bench] non-LTE {name}: {it} iterations, {dt:.2f} s", file=sys.stderr, flush=True)
    ref = final.get("plain_fp32")
    for name in final:
        if ref is not None and name != "plain_fp32":
            out[name]["max_rel_diff_vs_plain_fp32"] = float(((final[name] - ref).abs() / ref.abs()).max())
    if "plain_fp32" in out:
        for name in final:
            if name != "plain_fp32":
                out[name]["speedup_vs_plain_fp32"] = out["plain_fp32"]["seconds"] / out[name]["seconds"]
    if net is not None:
        net.close()
    return out


def c4_batched(args):
    """The 16-atmosphere uneven batch in one batched solve (HIP graph), FP32
    and FP16 cascade storage: time per solve, ray intervals per second, and
    J at sampled cells of a wing and a core wavelength of every atmosphere
    against the FP64 oracle (through the cells' dependency cones)."""
    import numpy as np
    import torch

    import oracle
    from paper_2408_14425_amd import rcx, workloads
    specs = workloads.uneven_batch()
    rng = np.random.default_rng(7)
    chi, eta, J, samples = [], [], [], []
    t0 = time.perf_counter()
    for side, nw, seed in specs:
        inp = workloads.line_medium(side, nw, seed=seed)
        chi.append(torch.from_numpy(inp.chi).cuda())
        eta.append(torch.from_numpy(inp.eta).cuda())
        J.append(torch.empty_like(chi[-1]))
        lam = [0, nw // 2]  # line wing and line core
        cells = [(0, 0), (side - 1, side - 1)] + [tuple(int(c) for c in rng.integers(0, side, 2)) for _ in range(2)]
        samples.append((inp.chi[lam].copy(), inp.eta[lam].copy(), lam, cells, inp.n_cascades))
        del inp
        print(f"[bench] c4 atmosphere {side}^2 x {nw} ready ({time.perf_counter() - t0:.0f} s)", file=sys.stderr,
              flush=True)
    out = {"workload": "16 line-medium atmospheres, sides " + ",".join(str(s_[0]) for s_ in specs)
                       + "; wavelengths " + ",".join(str(s_[1]) for s_ in specs),
           "atmospheres": len(specs)}
    got = {}
    for name, storage in (("fp32", rcx.RCX_STORE_F32), ("fp16", rcx.RCX_STORE_F16_SCALED)):
        B = rcx.Batch([(s_[0], s_[0]) for s_ in specs], [s_[1] for s_ in specs], storage=storage)
        B.solve(chi, eta, J)  # builds the schedule and captures the graph
        torch.cuda.synchronize()
        reps = 2
        t1 = time.perf_counter()
        for _ in range(reps):
            B.solve(chi, eta, J)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        rays, steps = B.work()
        B.close()
        got[name] = [[J[a][l, z, x].item() for l in smp[2] for (x, z) in smp[3]] for a, smp in enumerate(samples)]
        out[name] = {"s_per_solve": dt, "ray_intervals_per_s": rays / dt, "cell_steps_per_s": steps / dt}
        print(f"[bench] c4 {name}: {dt:.2f} s per batched solve", file=sys.stderr, flush=True)
    del chi, eta, J
    torch.cuda.empty_cache()
    ref = []
    for c_, e_, lam, cells, nc in samples:
        side = c_.shape[-1]
        need = np.zeros((side, side), np.uint8)
        for x, z in cells:
            need[z, x] = 1
        vals = []
        for i in range(len(lam)):
            Jo = oracle.formal_solve(c_[i:i + 1], e_[i:i + 1], nc, need=need)["J"][0]
            vals += [Jo[z, x] for (x, z) in cells]
        ref.append(vals)
    for name in ("fp32", "fp16"):
        rel = [abs(g - o) / o for ga, ra in zip(got[name], ref) for g, o in zip(ga, ra)]
        out[name]["max_rel_error_vs_oracle"] = max(rel)
        out[name]["samples"] = len(rel)
    out["rays_per_solve"] = rays
    return out


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

    if args.nlte_only:
        print(json.dumps(nlte_solves(args)), flush=True)
        return

    inp = workloads.line_medium(args.n, args.waves, seed=2)
    dev = torch.device("cuda:0")
    chi = torch.from_numpy(inp.chi).to(dev)
    eta = torch.from_numpy(inp.eta).to(dev)
    J = torch.empty_like(chi)
    plan = rcx.Plan(inp.nx, inp.nz, inp.n_wave)
    work = plan.work()
    dt, (ms_level, ms_other, n_launch, n_solves) = time_solves(plan, chi, eta, J, args.steps, args.warmup)
    ok = bool(torch.isfinite(J).all().item())
    plan.close()

    fp16 = None
    if not args.no_fp16:
        # the same solve with FP16 cascade storage
        plan16 = rcx.Plan(inp.nx, inp.nz, inp.n_wave, storage=rcx.RCX_STORE_F16_SCALED)
        J16 = torch.empty_like(chi)
        dt16, _ = time_solves(plan16, chi, eta, J16, args.steps, args.warmup)
        plan16.close()
        fp16 = {
            "ms_per_step": dt16 / args.steps * 1e3,
            "value": work.rays_nonempty * inp.n_wave / (dt16 / args.steps),
            "max_rel_diff_vs_fp32": float(((J16 - J).abs() / J.abs()).max().item()),
        }

    incl = None
    if not args.no_incl:
        # the same solve with the paper's 8 inclinations per flatland ray
        # (2D invariance): 8 x the ray intervals, J the hemisphere average
        planI = rcx.Plan(inp.nx, inp.nz, inp.n_wave, n_incl=8)
        workI = planI.work()
        JI = torch.empty_like(chi)
        stepsI = max(1, min(args.steps, 3))
        dtI, _ = time_solves(planI, chi, eta, JI, stepsI, 1)
        planI.close()
        incl = {
            "n_incl": 8,
            "ms_per_step": dtI / stepsI * 1e3,
            "value": workI.rays_nonempty * inp.n_wave / (dtI / stepsI),
            "unit": "ray-intervals/s",
            "ray_intervals_nonempty_per_step": workI.rays_nonempty * inp.n_wave,
            "steps": stepsI,
        }

    fix = None
    if not args.no_fix:
        # the same solve with the bilinear fix: 4 traced rays per interval on
        # every cascade below the top
        planF = rcx.Plan(inp.nx, inp.nz, inp.n_wave, bilinear_fix=True)
        JF = torch.empty_like(chi)
        stepsF = max(1, min(args.steps, 5))
        dtF, (msF, _, _, nF) = time_solves(planF, chi, eta, JF, stepsF, 1)
        planF.close()
        top = work.n_cascades - 1
        traced = (4 * sum(work.level_rays[:top]) + (0 if work.top_skipped else work.level_rays[top])) * inp.n_wave
        fix = {
            "ms_per_step": dtF / stepsF * 1e3,
            "ray_intervals_traced_per_step": traced,
            "traced_per_s": traced / (dtF / stepsF),
            "kernel_ms_per_cascade": [m / max(nF, 1) for m in msF],
            "max_rel_diff_vs_basic": float(((JF - J).abs() / J.abs()).max().item()),
            "steps": stepsF,
        }

    sparse = None
    if not args.no_sparse:
        # the same solve with a quarter of the cells flagged (cool structure
        # in a hot corona); the rest transparent and empty
        act = workloads.active_cells(inp.nx, inp.nz, seed=7, frac=0.25)
        planS = rcx.Plan(inp.nx, inp.nz, inp.n_wave)
        counts = planS.set_active(act)
        JS = torch.empty_like(chi)
        stepsS = max(1, min(args.steps, 5))
        dtS, (msS, _, _, nS) = time_solves(planS, chi, eta, JS, stepsS, 1)
        planS.close()
        dense_probes = [L // (4 << (2 * i)) for i, L in enumerate(work.level_rays)]
        sparse = {
            "active_cells": float(act.mean()),
            "flagged_share_per_cascade": [c / d for c, d in zip(counts, dense_probes)],
            "ms_per_step": dtS / stepsS * 1e3,
            "speedup_vs_dense": (dt / args.steps) / (dtS / stepsS),
            "kernel_ms_per_cascade": [m / max(nS, 1) for m in msS],
            "steps": stepsS,
        }

    # emergent intensity along a beam of parallel long characteristics (light
    # direction (0.8, 0.6), one ray per cell across the beam)
    planE = rcx.Plan(inp.nx, inp.nz, inp.n_wave)
    n_em = int(math.ceil(inp.nx * 0.6 + inp.nz * 0.8)) + 2
    planE.emergent(chi, eta, 0.8, 0.6, n_em)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        planE.emergent(chi, eta, 0.8, 0.6, n_em)
    torch.cuda.synchronize()
    emergent = {"direction": [0.8, 0.6], "rays": n_em, "ms_per_image": (time.perf_counter() - t0) / 10 * 1e3}
    planE.close()

    ms_step = dt / args.steps * 1e3
    rays = work.rays_nonempty * inp.n_wave
    value = rays / (dt / args.steps)
    march_ms = sum(ms_level)
    avg_launch_s = march_ms / 1e3 / max(n_launch, 1)
    launches_per_solve = max(n_launch // max(n_solves, 1), 1)
    # ALU roofline (the bound the counters show): algorithmic lane operations
    # per launch over the average launch duration
    ops_per_launch = work.cell_steps * inp.n_wave * ALU_OPS_PER_STEP / launches_per_solve
    alu_achieved = ops_per_launch / avg_launch_s / 1e12
    # the cacheless byte count and the measured HBM traffic, for comparison
    bytes_per_launch = algorithmic_bytes(work, inp.n_wave) / launches_per_solve
    traffic = measured_traffic("k_march_rows_line1024_w64.md")
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
        "fp16_storage": fp16,
        "inclined": incl,
        "bilinear_fix": fix,
        "sparse": sparse,
        "emergent": emergent,
        "roofline": {
            "bound": "alu",
            "kernel": "k_march_rows",
            "achieved": alu_achieved,
            "peak": VALU_LANE_OPS / 1e12,
            "unit": "T VALU lane-ops/s",
            "frac": alu_achieved / (VALU_LANE_OPS / 1e12),
            "ops_per_cell_step": ALU_OPS_PER_STEP,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "hbm_GBs": traffic / avg_launch_s / 1e9 if traffic else None,
            "hbm_frac": traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS if traffic else None,
            "cacheless_bytes_GBs": bytes_per_launch / avg_launch_s / 1e9,
            "cacheless_frac": bytes_per_launch / avg_launch_s / 1e9 / HBM_PEAK_GBS,
        },
    }
    if not args.no_nlte:
        out["nonlte"] = nlte_solves(args)
    if args.c4:
        out["batched"] = c4_batched(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_waves)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
