"""Learned warm start for the non-LTE iteration: training data from
converged runs of the method itself, training of the network on the GPU, and
the comparison of iterations and wall time to convergence from the LTE start
and from the network's prediction. Every numerical step runs in librcx
(formal solutions, iterations, features, network training and inference);
this module only orchestrates and keeps the bookkeeping.

    python -m paper_2408_14425_amd.warmstart --train-n 256 --train-runs 16 --eval-n 512
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import rcx, workloads as W


def converged_run(n: int, seed: int, n_line: int, n_cont: int, tol: float, max_iter: int, ng: bool = False,
                  keep: int = 1):
    """Features at LTE and converged log departure coefficients of one seeded
    atmosphere; ng: iterate with Ng acceleration (order 2, first after 4
    iterations, then every 4; the same fixed point, reached in fewer
    iterations); keep: every keep-th cell (a seeded random subset) only."""
    inp = W.nlte_atmosphere(n, seed=seed, n_line=n_line, n_cont=n_cont)
    s = rcx.Nlte(inp)
    if ng:
        s.set_acceleration(2, 4, 4)
    pops = s.lte()
    feat = s.features(pops).cpu().numpy()
    rc, it, ch = s.iterate(pops, max_iter, tol)
    targ = s.log_departures(pops).cpu().numpy()
    s.close()
    if keep > 1:
        sel = np.sort(np.random.default_rng(seed).choice(len(feat), len(feat) // keep, replace=False))
        feat, targ = feat[sel], targ[sel]
    return feat, targ, it, ch


def dataset(n: int, seeds, n_line: int, n_cont: int, tol: float = 1e-3, max_iter: int = 500, ng: bool = False,
            keep: int = 1):
    X, Y, info = [], [], []
    t0 = time.perf_counter()
    for seed in seeds:
        f, t, it, ch = converged_run(n, seed, n_line, n_cont, tol, max_iter, ng=ng, keep=keep)
        X.append(f)
        Y.append(t)
        info.append({"seed": int(seed), "iterations": it, "last_change": ch})
        print(f"converged run {n}^2 seed {seed}: {it} iterations (change {ch:.2e}), "
              f"{time.perf_counter() - t0:.0f} s", flush=True)
    return np.concatenate(X), np.concatenate(Y), info


def norms(a: np.ndarray) -> np.ndarray:
    mu = a.mean(axis=0)
    sd = a.std(axis=0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    return np.stack([mu, sd]).astype(np.float32)


def train(X, Y, epochs: int = 20, batch: int = 8192, lr: float = 2e-3, seed: int = 0, width: int = 128,
          depth: int = 4, verbose: bool = False):
    import torch
    fn, tn = norms(X), norms(Y)
    Xs = ((X - fn[0]) / fn[1]).astype(np.float32)
    Ys = ((Y - tn[0]) / tn[1]).astype(np.float32)
    net = rcx.Mlp(X.shape[1], width, depth, Y.shape[1], max_batch=batch)
    net.set_params(W.mlp_init_params(X.shape[1], width, depth, Y.shape[1], seed=seed))
    rng = np.random.default_rng(seed)
    xt = torch.from_numpy(Xs).cuda()
    yt = torch.from_numpy(Ys).cuda()
    losses = []
    n = len(Xs)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        tot = 0.0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            tot += net.train_step(xt[idx].contiguous(), yt[idx].contiguous(), lr_ep)
        losses.append(tot / max(1, n // batch))
        if verbose and (ep % 5 == 0 or ep == epochs - 1):
            print(f"epoch {ep}: loss {losses[-1]:.4g}", flush=True)
    return net, fn, tn, losses


def save(net, fn, tn, path: str, info: dict | None = None):
    """Trained parameters and the feature/target standardisation, as a
    plain npz (no pickled objects)."""
    import os
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=net.get_params(), feat_norm=fn, targ_norm=tn,
             shape=np.array([net.n_in, net.width, net.depth, net.n_out], np.int64),
             info=np.array(json.dumps(info or {})))


def load(path: str, max_batch: int = 65536):
    """(net, feat_norm, targ_norm) from a file written by save()."""
    d = np.load(path)  # allow_pickle stays False
    n_in, width, depth, n_out = (int(v) for v in d["shape"])
    net = rcx.Mlp(n_in, width, depth, n_out, max_batch=max_batch)
    net.set_params(d["params"])
    return net, d["feat_norm"].astype(np.float32), d["targ_norm"].astype(np.float32)


def evaluate(net, fn, tn, n: int, seeds, n_line: int, n_cont: int, tol: float = 1e-3, max_iter: int = 1000,
             ref_tol: float = 1e-6, ref_max_iter: int = 2000, storage: int = rcx.RCX_STORE_F32,
             accuracy: float = 1e-3):
    """For each seed: iterations and wall time to max change < tol from the
    LTE start and from the warm start, the largest relative difference of
    the starting guesses and of both converged results from a reference
    iterated further (with Ng acceleration to a change below ref_tol, or
    ref_max_iter iterations), the difference between the two converged
    results, and the iterations each start needs until its largest relative
    difference from the reference first drops to `accuracy` (equal
    accuracy)."""
    import torch
    out = []
    err = lambda p, r: float(((p - r).abs() / r.abs()).max())
    for seed in seeds:
        inp = W.nlte_atmosphere(n, seed=seed, n_line=n_line, n_cont=n_cont)
        s = rcx.Nlte(inp, storage=storage)
        s.set_acceleration(2, 4, 4)
        ref = s.lte()
        it_r, rc_r, ch_r = 0, 1, float("inf")
        while rc_r != 0 and it_r < ref_max_iter:
            rc_r, k, ch_r = s.iterate(ref, min(50, ref_max_iter - it_r), ref_tol)
            it_r += k
            print(f"reference {n}^2 seed {seed}: {it_r} iterations, change {ch_r:.2e}", flush=True)
        s.set_acceleration(0)
        torch.cuda.synchronize()
        to_acc = {}
        for name in ("lte", "warm"):
            p = s.lte() if name == "lte" else s.warm_start(net, fn, tn)
            k = 0
            while k < max_iter and err(p, ref) > accuracy:
                s.iterate(p, 1, 0.0)
                k += 1
            to_acc[name] = (k, err(p, ref))
        t0 = time.perf_counter()
        p_lte = s.lte()
        rc0, it0, ch0 = s.iterate(p_lte, max_iter, tol)
        torch.cuda.synchronize()
        t_lte = time.perf_counter() - t0
        t0 = time.perf_counter()
        p_ws = s.warm_start(net, fn, tn)
        p_pred = p_ws.clone()
        rc1, it1, ch1 = s.iterate(p_ws, max_iter, tol)
        torch.cuda.synchronize()
        t_ws = time.perf_counter() - t0
        med = lambda p, r=ref: float(((p - r).abs() / r.abs()).median())
        p_lte0 = s.lte()
        out.append({
            "seed": int(seed), "n": n, "reference_iterations": it_r, "reference_change": ch_r,
            "lte_iterations": it0, "lte_seconds": t_lte, "lte_error_vs_reference": err(p_lte, ref),
            "warm_iterations": it1, "warm_seconds": t_ws, "warm_error_vs_reference": err(p_ws, ref),
            "lte_start_error_vs_reference": err(p_lte0, ref), "lte_start_median_error": med(p_lte0),
            "prediction_error_vs_reference": err(p_pred, ref), "prediction_median_error": med(p_pred),
            "warm_vs_lte_converged": err(p_ws, p_lte),
            "converged": bool(rc0 == 0 and rc1 == 0),
            "accuracy": accuracy,
            "lte_iterations_to_accuracy": to_acc["lte"][0], "lte_error_at_accuracy": to_acc["lte"][1],
            "warm_iterations_to_accuracy": to_acc["warm"][0], "warm_error_at_accuracy": to_acc["warm"][1],
        })
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-n", type=int, default=128)
    ap.add_argument("--train-runs", type=int, default=16)
    ap.add_argument("--train-n2", type=int, default=0, help="a second training size (0: none)")
    ap.add_argument("--train-runs2", type=int, default=0, help="converged runs at the second size (seeds 5100..)")
    ap.add_argument("--eval-n", type=int, default=256)
    ap.add_argument("--eval-seeds", type=int, nargs="+", default=[6000, 6001])
    ap.add_argument("--n-line", type=int, default=64)
    ap.add_argument("--n-cont", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None, help="write the trained network (npz)")
    ap.add_argument("--ref-max-iter", type=int, default=300)
    ap.add_argument("--tol", type=float, default=1e-3, help="stopping change of the training runs")
    ap.add_argument("--ng", action="store_true", help="training runs with Ng acceleration")
    ap.add_argument("--keep", type=int, default=1, help="keep every keep-th cell of each training run")
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--max-iter", type=int, default=500, help="iteration cap of the training runs")
    a = ap.parse_args()
    t0 = time.perf_counter()
    X, Y, info = dataset(a.train_n, range(5000, 5000 + a.train_runs), a.n_line, a.n_cont, tol=a.tol, ng=a.ng,
                         keep=a.keep, max_iter=a.max_iter)
    if a.train_n2 > 0 and a.train_runs2 > 0:
        X2, Y2, info2 = dataset(a.train_n2, range(5100, 5100 + a.train_runs2), a.n_line, a.n_cont)
        X, Y = np.concatenate([X, X2]), np.concatenate([Y, Y2])
        info += [dict(i, n=a.train_n2) for i in info2]
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    print(f"training on {len(X)} samples", flush=True)
    net, fn, tn, losses = train(X, Y, epochs=a.epochs, verbose=True)
    t_train = time.perf_counter() - t0
    print(f"trained on {len(X)} samples in {t_train:.1f} s, loss {losses[0]:.4g} -> {losses[-1]:.4g}", flush=True)
    if a.save:
        save(net, fn, tn, a.save, {"train_n": a.train_n, "train_runs": a.train_runs, "train_n2": a.train_n2,
                                   "train_runs2": a.train_runs2, "epochs": a.epochs, "tol": a.tol, "ng": a.ng,
                                   "keep": a.keep, "samples": len(X), "max_iter": a.max_iter,
                                   "n_line": a.n_line, "n_cont": a.n_cont, "loss_last": losses[-1]})
    ev = [] if a.no_eval else evaluate(net, fn, tn, a.eval_n, a.eval_seeds, a.n_line, a.n_cont,
                                       ref_max_iter=a.ref_max_iter)
    for e in ev:
        print(json.dumps(e), flush=True)
    rep = {"train": {"n": a.train_n, "runs": a.train_runs, "n2": a.train_n2, "runs2": a.train_runs2,
                     "samples": len(X), "data_seconds": t_data,
                     "train_seconds": t_train, "epochs": a.epochs, "loss_first": losses[0], "loss_last": losses[-1],
                     "runs_info": info},
           "eval": ev}
    s = json.dumps(rep)
    print(s, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(s + "\n")


if __name__ == "__main__":
    main()
