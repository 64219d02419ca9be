"""Batched formal solve (list-scheduled launches in a HIP graph) vs the FP64 oracle and vs per-atmosphere
plan solves, through the C ABI.

Tolerances: 1e-4 relative on J against the oracle (FP32 path, as for the
single-plan solve); against the single-plan GPU solve 1e-6 relative (the
same per-ray arithmetic; only the order of the four cascade-0 direction sums
differs); bitwise across launch orders, graph on/off and repeated replays (the
per-ray arithmetic does not depend on which workgroup computes it).
"""
import numpy as np
import pytest

import oracle
from paper_2408_14425_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-4


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rand_atm(nx, nz, nw, seed):
    rng = np.random.default_rng(seed)
    chi = (10 ** rng.uniform(-2, 2, (nw, nz, nx))).astype(np.float32)
    eta = (chi * rng.uniform(0.2, 3.0, (nw, nz, nx))).astype(np.float32)
    return chi, eta


# uneven sizes (ragged against the probe spacing, wavelength counts that do
# not fill a 16-wide batch, more batches than buffer slots)
CASES = [(64, 64, 3, 1), (37, 53, 20, 2), (128, 96, 1, 3), (1, 1, 2, 4), (200, 256, 70, 5)]


def _inputs(cases):
    torch = _torch()
    host = [_rand_atm(nx, nz, nw, sd) for nx, nz, nw, sd in cases]
    chi = [torch.from_numpy(c).cuda() for c, _ in host]
    eta = [torch.from_numpy(e).cuda() for _, e in host]
    return host, chi, eta


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def test_uneven_batch_matches_oracle_and_plans():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    print("[gpu] batch uneven", CASES, flush=True)
    host, chi, eta = _inputs(CASES)
    B = rcx.Batch([(nx, nz) for nx, nz, _, _ in CASES], [nw for _, _, nw, _ in CASES])
    B.set_graph(False)
    assert B.launches() == (0, 0)
    J = B.solve(chi, eta)
    torch.cuda.synchronize()
    print("[gpu] batch solve done (direct launch)", flush=True)
    # one march launch advances every active chain by a cascade: at least the
    # longest chain, at most every (atmosphere, 16-wavelength batch) chain in turn
    n_march, n_all = B.launches()
    chains = [(-(-nw // 16), W.n_cascades_for(nx, nz)) for nx, nz, nw, _ in CASES]
    assert max(nc for _, nc in chains) - 1 <= n_march <= sum(nb * nc for nb, nc in chains)
    assert n_all == n_march + len(CASES)
    for a, (nx, nz, nw, _) in enumerate(CASES):
        Jg = J[a].cpu().numpy().astype(np.float64)
        plan = rcx.Plan(nx, nz, nw)
        Jp = plan.formal_solve(chi[a], eta[a]).cpu().numpy().astype(np.float64)
        plan.close()
        assert _rel(Jg, Jp) <= 1e-6, (a, _rel(Jg, Jp))
        lam = np.unique(np.linspace(0, nw - 1, min(nw, 4)).astype(int))
        Jo = oracle.formal_solve(host[a][0][lam], host[a][1][lam], W.n_cascades_for(nx, nz))["J"]
        r = _rel(Jg[lam], Jo)
        print(f"atm {a} {nx}x{nz} w{nw}: vs plan {_rel(Jg, Jp):.2e} vs oracle {r:.2e}")
        assert r <= RTOL
    B.close()


def test_launch_order_and_graph_do_not_change_results():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    host, chi, eta = _inputs(CASES)
    B = rcx.Batch([(nx, nz) for nx, nz, _, _ in CASES], [nw for _, _, nw, _ in CASES])
    ref = [j.cpu().numpy() for j in B.solve(chi, eta)]
    J = [torch.empty_like(c) for c in chi]
    for order, dirs in ((0, 32), (2, 32), (8, 32), (4, 16), (4, 64)):
        for graph in (False, True):
            print(f"[gpu] batch order {order} x {dirs} graph {graph}", flush=True)
            B.set_order(order, dirs)
            B.set_graph(graph)
            for rep in range(3):  # graph replays with eager work in between
                for j in J:
                    j.fill_(-1.0)
                B.solve(chi, eta, J)
                torch.cuda.synchronize()
                for a in range(len(CASES)):
                    assert np.array_equal(J[a].cpu().numpy(), ref[a]), (order, dirs, graph, rep, a)
                _ = (chi[0] * 2.0).sum().item()
    B.close()


def test_fp16_batch_error_is_bounded():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    cases = [(64, 64, 3, 1), (100, 80, 33, 7)]
    print("[gpu] batch fp16", cases, flush=True)
    host, chi, eta = _inputs(cases)
    B = rcx.Batch([(nx, nz) for nx, nz, _, _ in cases], [nw for _, _, nw, _ in cases],
                  storage=rcx.RCX_STORE_F16_SCALED)
    J = B.solve(chi, eta)
    torch.cuda.synchronize()
    for a, (nx, nz, nw, _) in enumerate(cases):
        Jg = J[a].cpu().numpy().astype(np.float64)
        lam = np.array([0, nw - 1])
        Jo = oracle.formal_solve(host[a][0][lam], host[a][1][lam], W.n_cascades_for(nx, nz))["J"]
        r = _rel(Jg[lam], Jo)
        print(f"fp16 batch atm {a}: max rel {r:.3e}")
        assert r < 1e-3
    B.close()


def test_autotune_and_cache(tmp_path):
    torch = _torch()
    from paper_2408_14425_amd import rcx
    cases = CASES[:3]
    host, chi, eta = _inputs(cases)
    B = rcx.Batch([(nx, nz) for nx, nz, _, _ in cases], [nw for _, _, nw, _ in cases])
    ref = [j.cpu().numpy() for j in B.solve(chi, eta)]
    path = str(tmp_path / "tiles.jsonl")
    print("[gpu] batch autotune", flush=True)
    best = B.autotune(chi, eta, cache_path=path)
    assert best in (0, 2032, 4016, 4032, 4064, 8032)
    assert open(path).read().count("\n") == 1
    assert B.autotune(chi, eta, cache_path=path) == best  # cache hit: no new line
    assert open(path).read().count("\n") == 1
    J = B.solve(chi, eta)
    torch.cuda.synchronize()
    for a in range(len(cases)):
        assert np.array_equal(J[a].cpu().numpy(), ref[a])
    B.close()


def test_line_medium_batch_sampled_against_oracle():
    """Three line-medium atmospheres (config-2 type) at 256^2, 384^2 and
    512^2 with 32, 48 and 64 wavelengths in one launch; sampled cells checked
    against the oracle through their dependency cones."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    specs = [(256, 32, 11), (384, 48, 12), (512, 64, 13)]
    inps = [W.line_medium(side, nw, seed=sd) for side, nw, sd in specs]
    print("[gpu] batch line media", specs, flush=True)
    chi = [torch.from_numpy(i.chi).cuda() for i in inps]
    eta = [torch.from_numpy(i.eta).cuda() for i in inps]
    B = rcx.Batch([(i.nx, i.nz) for i in inps], [i.n_wave for i in inps])
    J = [j.cpu().numpy() for j in B.solve(chi, eta)]
    B.close()
    rng = np.random.default_rng(5)
    for inp, Jg in zip(inps, J):
        n = inp.nx
        cells = [(0, 0), (n - 1, n - 1)] + [tuple(rng.integers(0, n, 2)) for _ in range(3)]
        need = np.zeros((n, n), np.uint8)
        for x, z in cells:
            need[z, x] = 1
        for lam in (0, inp.n_wave // 2, inp.n_wave - 1):
            Jo = oracle.formal_solve(inp.chi[lam:lam + 1], inp.eta[lam:lam + 1], inp.n_cascades, need=need)["J"][0]
            for x, z in cells:
                assert abs(float(Jg[lam, z, x]) - Jo[z, x]) <= RTOL * Jo[z, x], (inp.name, lam, x, z)


def test_sparse_atmospheres_in_a_batch():
    """Sparse atmospheres inside a batch (Sec. 3.5): two of four atmospheres
    flagged (one with nothing flagged), solved under the graph twice (the
    second a replay); flagged cells against the oracle's sparse solve to
    1e-4, J = 0 at unflagged cells, the dense atmospheres as before; then
    flags cleared, the batch is dense again."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    cases = [(64, 64, 3, 1), (37, 53, 20, 2), (128, 96, 17, 3), (40, 40, 2, 6)]
    print("[gpu] batch sparse", cases, flush=True)
    host, chi, eta = _inputs(cases)
    act = {0: W.active_cells(64, 64, seed=3, frac=0.3), 2: W.active_cells(128, 96, seed=4, frac=0.25),
           3: np.zeros((40, 40), bool)}
    B = rcx.Batch([(nx, nz) for nx, nz, _, _ in cases], [nw for _, _, nw, _ in cases])
    dense = [j.cpu().numpy() for j in B.solve(chi, eta)]
    for a, m in act.items():
        B.set_active(a, m)
    for rep in range(2):
        J = [j.cpu().numpy().astype(np.float64) for j in B.solve(chi, eta)]
        for a, (nx, nz, nw, _) in enumerate(cases):
            if a not in act:
                assert np.array_equal(J[a], dense[a]), a
                continue
            m = act[a]
            assert np.all(J[a][:, ~m] == 0.0), a
            if m.any():
                Jo = oracle.formal_solve_sparse(host[a][0], host[a][1], W.n_cascades_for(nx, nz), m)["J"]
                r = _rel(J[a][:, m], Jo[:, m])
                print(f"replay {rep} atm {a}: flagged {m.mean():.2f}, vs oracle {r:.2e}")
                assert r <= RTOL
    for a in act:
        B.set_active(a, None)
    again = [j.cpu().numpy() for j in B.solve(chi, eta)]
    B.close()
    for a in range(len(cases)):
        assert np.array_equal(again[a], dense[a]), a


def test_large_atmosphere_runs_through_its_plan_inside_the_batch():
    """An atmosphere whose every cascade holds at least 2^19 rays (512^2)
    runs through its plan's own solve inside the batch's captured sequence:
    its J equals a separate plan's bit for bit (the same launches) and
    stays so over graph replays, next to list-scheduled small atmospheres;
    sampled cells of it agree with the FP64 oracle. 20 wavelengths: a
    pair of batches (the second partly filled) shares the walks on the
    cascades with at most 256 directions."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    cases = [(512, 512, 20, 11), (40, 24, 5, 12), (32, 32, 18, 13)]
    print("[gpu] batch with a 512^2 atmosphere", cases, flush=True)
    host, chi, eta = _inputs(cases)
    B = rcx.Batch([(nx, nz) for nx, nz, _, _ in cases], [nw for _, _, nw, _ in cases])
    J = B.solve(chi, eta)
    torch.cuda.synchronize()
    first = [j.cpu().numpy() for j in J]
    n_march, n_all = B.launches()
    for _ in range(2):
        B.solve(chi, eta, J)  # graph replays
    torch.cuda.synchronize()
    again = [j.cpu().numpy() for j in J]
    B.close()
    for a in range(len(cases)):
        assert np.array_equal(first[a], again[a])
    plan = rcx.Plan(512, 512, 20)
    Jp = plan.formal_solve(chi[0], eta[0]).cpu().numpy()
    w = plan.work()
    plan.close()
    assert np.array_equal(first[0], Jp)
    # the plan's launches (cascades of two batches, paired below 256
    # directions) plus at least one per small atmosphere's cascade
    assert n_march > w.n_cascades and n_all == n_march + len(cases)
    for a, (nx, nz, nw, _) in enumerate(cases[1:], start=1):
        plan = rcx.Plan(nx, nz, nw)
        Jq = plan.formal_solve(chi[a], eta[a]).cpu().numpy().astype(np.float64)
        plan.close()
        assert _rel(first[a].astype(np.float64), Jq) <= 1e-6
    rng = np.random.default_rng(5)
    cells = [(0, 0), (511, 511)] + [tuple(int(c) for c in rng.integers(0, 512, 2)) for _ in range(2)]
    need = np.zeros((512, 512), np.uint8)
    for x, z in cells:
        need[z, x] = 1
    for lam in (0, 19):
        Jo = oracle.formal_solve(host[0][0][lam:lam + 1], host[0][1][lam:lam + 1], W.n_cascades_for(512, 512),
                                 need=need)["J"][0]
        for x, z in cells:
            assert abs(float(first[0][lam, z, x]) - Jo[z, x]) <= RTOL * Jo[z, x], (lam, x, z)
