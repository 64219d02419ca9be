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
# Vector ALU peak: MI355X's FP32 vector rate, 157.3 TFLOP/s = 78.6e12 FMA
# lane slots per second (256 CUs x 4 SIMDs x 2.4 GHz x 32 lanes). An issue
# probe of independent FMA chains reaches 0.76 of it without packed
# instructions (0.38 wave64 FMAs per SIMD cycle), so it is the rate full-rate
# FP32 instructions run at here; v_exp_f32 issues at 0.29 of the FMA rate
# (a quarter-rate transcendental).
VALU_SLOTS = 78.6e12
# Algorithmic work per cell step and wavelength of the march, in those
# slots: the optical depth (1), e^-dtau (4: quarter rate), 1 - e (1), the
# intensity FMA (1) and the accumulated optical depth or transmission
# update (1).
ALU_OPS_PER_STEP = 8
# Algorithmic bytes per cell step and wavelength: chi and S, FP32 each.
BYTES_PER_STEP = 8
# The non-LTE line march adds the line profile per step (expansion in the
# damping parameter a): x = |u w + v| (1), x^2 (1), e^{-x^2} (1 + 4), the
# Dawson term from its table (4: scale, clamp, fraction, interpolation),
# H = e (1 + a^2 (1 - 2x^2)) - (2a/sqrt(pi)) g (4) and chi = chi_0 H (1):
# 16 slots, plus the radiative update's 8.
LINE_OPS_PER_STEP = 24
# Dense BF16 MFMA peak of MI355X (FLOP/s).
MFMA_BF16_PEAK = 2.5e15


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
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the batched formal solve of 16 uneven atmospheres (256^2..2048^2, "
                         "32..256 wavelengths; ~190 GB of device memory, about two minutes)")
    ap.add_argument("--c4-reps", type=int, default=1, help="timed batched solves per storage")
    ap.add_argument("--c4-per-plan", action="store_true",
                    help="also time the 16 atmospheres one plan after another (FP32)")
    ap.add_argument("--nlte-only", action="store_true",
                    help="only the converged non-LTE solves (prints their object)")
    ap.add_argument("--nlte-profile", type=int, default=0,
                    help="only this many plain FP32 non-LTE iterations from LTE (for profiling the line march)")
    ap.add_argument("--mlp-profile", type=int, default=0,
                    help="only this many warm-start network training steps and forward passes on seeded data "
                         "(batch 65536; for profiling the BF16 MFMA products)")
    ap.add_argument("--nlte-variants", default="plain_fp32,plain_fp16,learned_fp32,learned_fp16",
                    help="comma-separated subset of the non-LTE runs (also ng_fp32, learned_ng_fp16, "
                         "charge_fp32, sparse_fp32)")
    ap.add_argument("--nlte-n", type=int, default=1024)
    ap.add_argument("--nlte-seed", type=int, default=3, help="seed of the non-LTE atmosphere")
    ap.add_argument("--nlte-corona", type=float, default=0.0,
                    help="fraction of the non-LTE atmosphere turned into 1e6 K corona (for sparse_fp32)")
    ap.add_argument("--nlte-max-iter", type=int, default=300)
    ap.add_argument("--nlte-ref-max-iter", type=int, default=200)
    ap.add_argument("--nlte-ref-tol", type=float, default=1e-7,
                    help="the reference stops when its max relative change drops below this")
    ap.add_argument("--nlte-ref-start", choices=("lte", "learned"), default="lte",
                    help="start of the reference iteration (the same fixed point either way)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2408_14425_amd", "data", "warmstart_mlp.npz"),
                    help="trained warm-start network (skipped when absent)")
    ap.add_argument("--orders", default=os.path.join(ROOT, "paper_2408_14425_amd", "data", "launch_orders.jsonl"),
                    help="launch-order cache of the autotuner (rcx_autotune); a miss tunes and appends")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch orders")
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
    """Hash of the march kernel's sources with comments and blank space
    removed (a comment change leaves the counters valid)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2408_14425_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(" ".join(text.split()).encode())
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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inp, n_waves: int):
    """The FP64 oracle (C, OpenMP, -O3 for x86-64-v3) on the host: the full
    formal solve of n_waves of the workload's wavelengths on all host
    threads, and the dependency cone of a central 64 x 64 block of cells of
    one wavelength on one thread."""
    import numpy as np

    import oracle
    sel = slice(inp.n_wave // 2 - n_waves // 2, inp.n_wave // 2 - n_waves // 2 + n_waves)
    chi = inp.chi[sel].astype(np.float64)
    eta = inp.eta[sel].astype(np.float64)
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    r = oracle.formal_solve(chi, eta, inp.n_cascades)
    dt = time.perf_counter() - t0
    # all threads first: a one-thread call leaves OpenMP at one thread
    nlte = nlte_cpu_baseline(r["steps"] // max(n_waves, 1))
    need = np.zeros((inp.nz, inp.nx), np.uint8)
    need[inp.nz // 2 - 32:inp.nz // 2 + 32, inp.nx // 2 - 32:inp.nx // 2 + 32] = 1
    t1 = time.perf_counter()
    r1 = oracle.formal_solve(chi[:1], eta[:1], inp.n_cascades, need=need, n_threads=1)
    dt1 = time.perf_counter() - t1
    return {
        "value": r["nonempty"] / dt,
        "unit": "ray-intervals/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"FP64 oracle full formal solve of {n_waves} of the 64 wavelengths "
                  f"({r['nonempty']} non-empty ray intervals, {r['steps']} cell steps) in {dt:.1f} s on "
                  f"{threads} threads",
        "one_thread": {"value": r1["nonempty"] / dt1, "unit": "ray-intervals/s",
                       "sample": f"dependency cone of the central 64x64 cells, 1 wavelength: {r1['nonempty']} "
                                 f"non-empty ray intervals in {dt1:.1f} s on 1 thread"},
        "nonlte_iteration": nlte,
    }


def nlte_cpu_baseline(steps_per_wave: int):
    """One iteration of the FP64 non-LTE oracle on the 1024^2, 160-wavelength
    atmosphere, estimated from a bounded sample: the dependency cones of the
    central 64 x 64 and 192 x 192 cells at one line-core wavelength (formal
    solution with the cascade-0 radiance, local opacities and profiles) on
    all host threads; the straight line through (cell steps, seconds)
    extrapolated to the full grid (the formal solve's steps per wavelength
    on the same grid) and multiplied by the 160 wavelengths."""
    import numpy as np

    import oracle
    from oracle import nlte
    from paper_2408_14425_amd import workloads
    inp = workloads.nlte_atmosphere(1024, seed=3, n_line=64, n_cont=32)
    P = nlte.Problem(inp)
    pts = []
    for h in (32, 96):
        need = np.zeros((inp.nz, inp.nx), np.uint8)
        need[inp.nz // 2 - h:inp.nz // 2 + h, inp.nx // 2 - h:inp.nx // 2 + h] = 1
        t0 = time.perf_counter()
        st = P.formal_solve(P.lte, lams=[32], need=need)[4]
        pts.append((int(st[2]), time.perf_counter() - t0))
    # seconds = a + b steps (a: the per-wavelength work on every cell)
    (s0, t0_), (s1, t1_) = pts
    b = (t1_ - t0_) / max(s1 - s0, 1)
    a = max(t0_ - b * s0, 0.0)
    est = (a + b * steps_per_wave) * inp.n_wave
    return {"seconds_per_iteration_estimated": est, "unit": "s per iteration", "cores": oracle.num_threads(),
            "sample": f"dependency cones of the central 64x64 and 192x192 cells at 1 line-core wavelength: "
                      f"{s0} and {s1} cell steps in {t0_:.1f} and {t1_:.1f} s on {oracle.num_threads()} threads; "
                      f"the line through them extrapolated to {steps_per_wave} cell steps per wavelength, times "
                      f"{inp.n_wave} wavelengths"}


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
    """Seconds to a converged non-LTE solve at equal accuracy (Sec. 4.2's
    criterion, and the true error against a converged reference).

    The reference is the plain FP32 iteration with Ng acceleration from the
    LTE start, iterated until its max relative change stops falling (the
    FP32 floor) or drops below --nlte-ref-tol (1e-7). Each variant then iterates one step at
    a time from its start (LTE, or the learned warm start: features, network
    inference and populations inside the timed region) with FP32 or 16-bit
    cascade storage; after each step its true error, the max relative
    difference of the populations from the reference, is measured outside
    the timed region. Reported per variant: the iterations and seconds at
    which the paper's criterion (max relative change < 1e-3) first holds and
    the true error then, and the iterations and seconds at which the true
    error first drops to 1e-3 (equal accuracy for every variant)."""
    import torch

    from paper_2408_14425_amd import rcx, warmstart, workloads
    inp = workloads.nlte_atmosphere(args.nlte_n, seed=args.nlte_seed, n_line=64, n_cont=32,
                                    corona_frac=args.nlte_corona)
    corona = f", {args.nlte_corona:.0%} of the cells 1e6 K corona" if args.nlte_corona > 0 else ""
    out = {"workload": f"non-LTE iteration, {inp.nx}x{inp.nz} grid, {inp.n_wave} wavelengths "
                       f"(2 lines x 64 + 32 continuum), synthetic 3-level + continuum atom, seed {args.nlte_seed}"
                       f"{corona}",
           "criterion": "max relative change < 1e-3 (Sec. 4.2); equal accuracy: true error <= 1e-3 against "
                        "the reference"}
    net = None
    if os.path.exists(args.weights):
        net, fn, tn = warmstart.load(args.weights)

    def err(p, ref):
        return float(((p - ref).abs() / ref.abs()).max().item())

    def tune(s):
        # launch orders of the marches from the autotuner's cache (results do
        # not depend on them)
        if not args.no_autotune:
            s.autotune(args.orders)

    # reference: Ng-accelerated FP32 iteration to the FP32 floor
    t0 = time.perf_counter()
    s = rcx.Nlte(inp)
    tune(s)
    s.set_acceleration(2, 4, 4)
    ref = s.warm_start(net, fn, tn) if args.nlte_ref_start == "learned" and net is not None else s.lte()
    it_r, best, since, ch = 0, float("inf"), 0, float("inf")
    while it_r < args.nlte_ref_max_iter and ch > args.nlte_ref_tol and since < 12:
        _, k, ch = s.iterate(ref, 1, 0.0)
        it_r += k
        if ch < 0.9 * best:
            best, since = ch, 0
        else:
            since += 1
        if it_r % 10 == 0:
            print(f"[bench] non-LTE reference: {it_r} iterations, change {ch:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    s.close()
    out["reference"] = {"iterations": it_r, "last_change": ch, "best_change": best, "ng": [2, 4, 4],
                        "tolerance": args.nlte_ref_tol, "start": args.nlte_ref_start,
                        "seconds": time.perf_counter() - t0}

    runs = [("plain_fp32", rcx.RCX_STORE_F32, False, False), ("plain_fp16", rcx.RCX_STORE_F16_SCALED, False, False),
            ("learned_fp32", rcx.RCX_STORE_F32, True, False), ("learned_fp16", rcx.RCX_STORE_F16_SCALED, True, False),
            ("ng_fp32", rcx.RCX_STORE_F32, False, True), ("learned_ng_fp16", rcx.RCX_STORE_F16_SCALED, True, True),
            ("charge_fp32", rcx.RCX_STORE_F32, False, False), ("sparse_fp32", rcx.RCX_STORE_F32, False, False)]
    wanted = set(args.nlte_variants.split(","))
    runs = [r for r in runs if r[0] in wanted and (net is not None or not r[2])]
    for name, storage, learned, ng in runs:
        s = rcx.Nlte(inp, storage=storage)
        tune(s)
        p = s.lte()
        s.iterate(p, 1, 0.0)  # one untimed iteration warms the kernels up
        torch.cuda.synchronize()
        if ng:
            # Ng acceleration (not in the paper): order 2, first after 4
            # iterations, then every 4
            s.set_acceleration(2, 4, 4)
        if "sparse" in name:
            out.setdefault("flagged_probes_per_cascade", s.set_temperature_cut(2.5e5))
        if "charge" in name:
            s.set_charge_conservation(True)
        t0 = time.perf_counter()
        p = s.warm_start(net, fn, tn) if learned else s.lte()
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t0
        rec = {"start_error": err(p, ref)}
        it, ch = 0, float("inf")
        while it < args.nlte_max_iter:
            t1 = time.perf_counter()
            _, k, ch = s.iterate(p, 1, 0.0)  # synchronises
            t_run += time.perf_counter() - t1
            it += k
            e = err(p, ref)
            if ch < 1e-3 and "criterion" not in rec:
                rec["criterion"] = {"iterations": it, "seconds": t_run, "true_error": e}
            if e <= 1e-3:
                rec["equal_accuracy"] = {"iterations": it, "seconds": t_run, "true_error": e}
                break
            if it % 10 == 0:
                print(f"[bench] non-LTE {name}: {it} iterations, change {ch:.3e}, error {e:.3e}, {t_run:.1f} s",
                      file=sys.stderr, flush=True)
        rec.update({"iterations_run": it, "seconds_run": t_run, "last_change": ch, "s_per_iteration": t_run / it})
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
        out[name] = rec
        print(f"[bench] non-LTE {name}: {json.dumps(rec)}", file=sys.stderr, flush=True)
    base = out.get("plain_fp32", {}).get("equal_accuracy")
    for name, _, _, _ in runs:
        ea = out[name].get("equal_accuracy")
        if base and ea and name != "plain_fp32":
            out[name]["speedup_vs_plain_fp32_at_equal_accuracy"] = base["seconds"] / ea["seconds"]
    # the march kernels' ALU rooflines (2 plain FP32 iterations with timing)
    s = rcx.Nlte(inp)
    tune(s)
    out["roofline"] = line_march_roofline(s, 2)
    s.close()
    if net is not None:
        out["network"] = {"weights": os.path.relpath(args.weights, ROOT)}
        net.close()
    return out


def line_march_roofline(s, iters: int):
    """ALU roofline of the non-LTE march from `iters` iterations with kernel
    timing: algorithmic slots (LINE_OPS_PER_STEP per line cell step and
    wavelength, ALU_OPS_PER_STEP per continuum one) over the summed event
    time of the launches."""
    p = s.lte()
    s.iterate(p, 1, 0.0)
    s.get_timing()
    s.set_timing(True)
    s.iterate(p, iters, 0.0)
    t = s.get_timing()
    s.set_timing(False)
    out = {}
    for kind, ops in (("line", LINE_OPS_PER_STEP), ("continuum", ALU_OPS_PER_STEP)):
        ms, n, steps = t[kind]
        if n == 0:
            continue
        achieved = ops * steps / (ms / 1e3) / 1e12
        out[kind] = {"bound": "alu", "kernel": "k_march_rows<LineOpT>" if kind == "line" else "k_march_rows<FieldOp>",
                     "achieved": achieved, "peak": VALU_SLOTS / 1e12,
                     "unit": "T VALU lane slots/s (FP32 FMA = 1, v_exp_f32 = 4)",
                     "frac": achieved / (VALU_SLOTS / 1e12), "ops_per_cell_step": ops,
                     "launches": n, "avg_launch_ms": ms / n, "cell_steps_x_wavelengths": steps,
                     "iterations": iters}
    return out


def nlte_profile(args):
    """Plain FP32 non-LTE iterations from LTE (one untimed first), with the
    seconds per iteration: the command the line march's profiles run."""
    import torch

    from paper_2408_14425_amd import rcx, workloads
    inp = workloads.nlte_atmosphere(args.nlte_n, seed=args.nlte_seed, n_line=64, n_cont=32)
    s = rcx.Nlte(inp)
    if not args.no_autotune:
        s.autotune(args.orders)
    p = s.lte()
    s.iterate(p, 1, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it, ch = s.iterate(p, args.nlte_profile, 0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    roof = line_march_roofline(s, 2)
    s.close()
    return {"workload": f"non-LTE iteration, {inp.nx}x{inp.nz}, {inp.n_wave} wavelengths, seed {args.nlte_seed}",
            "iterations": it, "s_per_iteration": dt / max(it, 1), "last_change": ch, "roofline": roof}


def nlte_inclined(args, n_incl: int = 8, iters: int = 2):
    """The non-LTE iteration with the paper's 8 Gauss-Radau inclinations per
    flatland ray (Sec. 3.1; Sec. 4.5 iterates with 8): one pass per
    inclination, velocities projected; one untimed iteration from LTE, then
    `iters` timed, and the march rooflines of one more (default launch
    orders)."""
    import torch

    from paper_2408_14425_amd import rcx, workloads
    inp = workloads.nlte_atmosphere(args.nlte_n, seed=args.nlte_seed, n_line=64, n_cont=32)
    s = rcx.Nlte(inp, n_incl=n_incl)
    p = s.lte()
    s.iterate(p, 1, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it, ch = s.iterate(p, iters, 0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    roof = line_march_roofline(s, 1)
    s.close()
    return {"workload": f"non-LTE iteration, {inp.nx}x{inp.nz}, {inp.n_wave} wavelengths, seed {args.nlte_seed}, "
                        f"{n_incl} inclinations", "n_incl": n_incl,
            "iterations": it, "s_per_iteration": dt / max(it, 1), "last_change": ch, "roofline": roof}


def mlp_profile(args):
    """Training steps and forward passes of the warm-start network
    (6 -> 4 x 128 -> 4, BF16 MFMA) on seeded data, batch 65536: the command
    the MLP kernels' profiles run. FLOP per sample: 2 x 50,432 multiply-adds
    forward, 3 x that for a training step (forward, input and weight
    gradients)."""
    import numpy as np
    import torch

    from paper_2408_14425_amd import rcx, workloads
    batch = 65536
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal((batch, 6)).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.standard_normal((batch, 4)).astype(np.float32)).cuda()
    net = rcx.Mlp(6, 128, 4, 4, max_batch=batch)
    net.set_params(workloads.mlp_init_params(6, 128, 4, 4, seed=0))
    net.train_step(x, y, 1e-3)
    net.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.mlp_profile):
        net.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / args.mlp_profile
    t0 = time.perf_counter()
    for _ in range(args.mlp_profile):
        net.forward(x)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / args.mlp_profile
    net.close()
    macs = 6 * 128 + 3 * 128 * 128 + 128 * 4
    train = 3 * 2 * macs * batch / t_train / 1e12
    fwd = 2 * macs * batch / t_fwd / 1e12
    return {"batch": batch, "steps": args.mlp_profile, "ms_per_train_step": t_train * 1e3,
            "ms_per_forward": t_fwd * 1e3, "train_TFLOPs": train, "forward_TFLOPs": fwd,
            # whole training step (every kernel of it) against the dense BF16 MFMA peak
            "roofline": {"bound": "mfma", "kernel": "training step (k_gemm_nt and its epilogues)",
                         "achieved": train, "peak": MFMA_BF16_PEAK / 1e12, "unit": "TFLOP/s",
                         "frac": train / (MFMA_BF16_PEAK / 1e12)}}


def c4_batched(args):
    """The 16-atmosphere uneven batch in one batched solve (HIP graph), FP32
    and FP16 cascade storage: time per solve, ray intervals per second, and
    J at sampled cells of a wing and a core wavelength of every atmosphere,
    which the cpu_baseline leg compares with the FP64 oracle
    (c4_oracle_check)."""
    import numpy as np
    import torch

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
        reps = max(args.c4_reps, 1)
        t1 = time.perf_counter()
        for _ in range(reps):
            B.solve(chi, eta, J)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        rays, steps = B.work()
        n_march, n_all = B.launches()
        B.close()
        got[name] = [[J[a][l, z, x].item() for l in smp[2] for (x, z) in smp[3]] for a, smp in enumerate(samples)]
        out[name] = {"s_per_solve": dt, "ray_intervals_per_s": rays / dt, "cell_steps_per_s": steps / dt,
                     "march_launches": n_march, "launches": n_all}
        print(f"[bench] c4 {name}: {dt:.2f} s per batched solve", file=sys.stderr, flush=True)
    if args.c4_per_plan:
        # the same atmospheres one plan after another (FP32, one untimed solve each first)
        t_pp = 0.0
        for a, (side, nw, _) in enumerate(specs):
            P = rcx.Plan(side, side, nw)
            P.formal_solve(chi[a], eta[a], J[a])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            P.formal_solve(chi[a], eta[a], J[a])
            torch.cuda.synchronize()
            t_pp += time.perf_counter() - t1
            P.close()
        out["fp32"]["per_plan_s"] = t_pp
        out["fp32"]["batched_speedup_vs_per_plan"] = t_pp / out["fp32"]["s_per_solve"]
        print(f"[bench] c4 per plan: {t_pp:.2f} s", file=sys.stderr, flush=True)
    del chi, eta, J
    torch.cuda.empty_cache()
    # the sampled cells' oracle values are computed by the cpu_baseline leg
    # (c4_oracle_check), the only leg that runs the oracle
    out["_oracle_samples"] = (samples, got)
    out["rays_per_solve"] = rays
    return out


def c4_oracle_check(batched: dict, samples, got) -> None:
    """Part of the cpu_baseline leg: the FP64 oracle's J at the batch's
    sampled cells (through their dependency cones), and the batched solve's
    FP32 and FP16 errors against it."""
    import numpy as np

    import oracle
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
        batched[name]["max_rel_error_vs_oracle"] = max(rel)
        batched[name]["samples"] = len(rel)


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
    if args.nlte_profile:
        print(json.dumps(nlte_profile(args)), flush=True)
        return
    if args.mlp_profile:
        print(json.dumps(mlp_profile(args)), flush=True)
        return

    inp = workloads.line_medium(args.n, args.waves, seed=2)
    dev = torch.device("cuda:0")
    chi = torch.from_numpy(inp.chi).to(dev)
    eta = torch.from_numpy(inp.eta).to(dev)
    J = torch.empty_like(chi)
    def tuned(plan):
        """The plan with its launch orders from the autotuner (cached)."""
        if not args.no_autotune:
            plan.autotune(args.orders)
        return plan

    plan = tuned(rcx.Plan(inp.nx, inp.nz, inp.n_wave))
    work = plan.work()
    orders = [plan.get_order(i) for i in range(work.n_cascades)]
    dt, (ms_level, ms_other, n_launch, n_solves) = time_solves(plan, chi, eta, J, args.steps, args.warmup)
    ok = bool(torch.isfinite(J).all().item())
    plan.close()

    fp16 = None
    if not args.no_fp16:
        # the same solve with FP16 cascade storage
        plan16 = tuned(rcx.Plan(inp.nx, inp.nz, inp.n_wave, storage=rcx.RCX_STORE_F16_SCALED))
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
        planI = tuned(rcx.Plan(inp.nx, inp.nz, inp.n_wave, n_incl=8))
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
        planF = tuned(rcx.Plan(inp.nx, inp.nz, inp.n_wave, bilinear_fix=True))
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
        tuned(planS)
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
    # ALU roofline: algorithmic lane slots per launch over the average
    # launch duration
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
            "launch_orders": {"per_cascade_tile_p_tile_d_xcd_chunk_shared_walk": orders,
                              "source": "defaults" if args.no_autotune else os.path.relpath(args.orders, ROOT)},
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
            "kernel": "k_march_rows and k_march_shared (every march launch of the solve)",
            "achieved": alu_achieved,
            "peak": VALU_SLOTS / 1e12,
            "unit": "T VALU lane slots/s (FP32 FMA = 1, v_exp_f32 = 4)",
            "frac": alu_achieved / (VALU_SLOTS / 1e12),
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
        out["nonlte_inclined"] = nlte_inclined(args)
        # the warm-start network's training step (20 steps, batch 65536)
        args.mlp_profile = 20
        out["mlp"] = mlp_profile(args)
    if not args.no_c4:
        out["batched"] = c4_batched(args)
    c4_samples = out["batched"].pop("_oracle_samples", None) if out.get("batched") else None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_waves)
        if c4_samples:
            c4_oracle_check(out["batched"], *c4_samples)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
