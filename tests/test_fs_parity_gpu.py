"""GPU formal solve vs the FP64 oracle, element by element, through the C ABI.

Tolerance: 1e-4 relative per cell on J for the FP32 path (every term of the
march and merge is non-negative once 1 - e^{-x} is evaluated stably, so FP32
error grows at most linearly in the number of steps: ~1e-5 for the longest
rays here).
"""
import math

import os

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


def _gpu_solve(inp, n_cascades=0, t_rule=0, workspace=False, n_incl=1, storage=0, bilinear_fix=False):
    torch = _torch()
    from paper_2408_14425_amd import rcx
    print(f"[gpu] formal solve {inp.name} n_cascades={n_cascades or inp.n_cascades} t_rule={t_rule} "
          f"n_incl={n_incl} storage={storage} bilinear_fix={bilinear_fix}", flush=True)
    plan = rcx.Plan(inp.nx, inp.nz, inp.n_wave, voxel_scale=inp.voxel_scale, n_cascades=n_cascades,
                    t_rule=t_rule, n_incl=n_incl, storage=storage, bilinear_fix=bilinear_fix)
    chi = torch.from_numpy(inp.chi).cuda()
    eta = torch.from_numpy(inp.eta).cuda()
    ws = None
    if workspace:
        ws = torch.empty(plan.workspace_bytes(inp.n_wave), dtype=torch.uint8, device="cuda")
    J = plan.formal_solve(chi, eta, workspace=ws)
    torch.cuda.synchronize()
    out = J.cpu().numpy().astype(np.float64)
    plan.close()
    return out


def _assert_rel(Jg, Jo, rtol=RTOL):
    rel = np.abs(Jg - Jo) / np.maximum(np.abs(Jo), 1e-300)
    worst = np.unravel_index(np.argmax(rel), rel.shape)
    assert rel.max() <= rtol, f"max rel err {rel.max():.3e} at {worst}: gpu {Jg[worst]} oracle {Jo[worst]}"
    return rel.max()


def test_blobs_64_single_wavelength_full_field():
    """64^2, 1 wavelength, 5 cascades: every cell."""
    inp = W.blobs_medium(64, seed=1)
    Jg = _gpu_solve(inp)
    Jo = oracle.formal_solve(inp.chi, inp.eta, inp.n_cascades)["J"]
    print("max rel", _assert_rel(Jg, Jo))


def test_line_medium_256_eight_wavelengths_full_field():
    """Reduced multi-wavelength workload: 256^2, 8 wavelengths spanning the
    line profile (0.1 .. 1e4 opacity contrast), 6 cascades, every cell."""
    inp = W.line_medium(256, 64, seed=2, wave_subset=np.arange(0, 64, 8))
    Jg = _gpu_solve(inp)
    Jo = oracle.formal_solve(inp.chi, inp.eta, inp.n_cascades)["J"]
    _assert_rel(Jg, Jo)


@pytest.mark.parametrize("nx,nz,nw,seed", [(37, 53, 3, 1), (100, 64, 67, 2), (1, 1, 1, 3), (2, 7, 5, 4)])
def test_ragged_grids_and_wavelength_counts(nx, nz, nw, seed):
    """Sizes that are not multiples of the probe spacing (probes outside the
    domain, clamped taps) and wavelength counts that do not fill a wavefront."""
    rng = np.random.default_rng(seed)
    chi = (10 ** rng.uniform(-2, 2, (nw, nz, nx))).astype(np.float32)
    eta = (chi * rng.uniform(0.2, 3.0, (nw, nz, nx))).astype(np.float32)
    inp = W.FormalSolveInput(chi, eta, 1.0, W.n_cascades_for(nx, nz), f"rand{nx}x{nz}w{nw}")
    Jg = _gpu_solve(inp, workspace=True)
    Jo = oracle.formal_solve(chi, eta, inp.n_cascades)["J"]
    _assert_rel(Jg, Jo)


def test_vacuum_disc_zero_opacity_cells():
    """chi = eta = 0 outside an opaque disc: exercises the chi -> 0 limit."""
    inp = W.disc_in_vacuum(128, 4.0)
    Jg = _gpu_solve(inp)
    Jo = oracle.formal_solve(inp.chi, inp.eta, inp.n_cascades)["J"]
    _assert_rel(Jg, Jo)


def test_voxel_scale_and_interval_rule():
    inp = W.blobs_medium(48, seed=6)
    inp.chi[...] = (inp.chi * 1e-3).astype(np.float32)
    inp.eta[...] = (inp.eta * 1e-3).astype(np.float32)
    inp.voxel_scale = 250.0
    for t_rule in (0, 1):
        Jg = _gpu_solve(inp, t_rule=t_rule)
        Jo = oracle.formal_solve(inp.chi, inp.eta, inp.n_cascades, voxel=250.0, t_rule=t_rule)["J"]
        _assert_rel(Jg, Jo)


def test_single_and_two_cascades():
    inp = W.blobs_medium(32, seed=8)
    for nc in (1, 2):
        Jg = _gpu_solve(inp, n_cascades=nc)
        Jo = oracle.formal_solve(inp.chi, inp.eta, nc)["J"]
        _assert_rel(Jg, Jo)


def test_deterministic_bitwise():
    inp = W.line_medium(128, 64, seed=3, wave_subset=np.arange(0, 64, 4))
    a = _gpu_solve(inp)
    b = _gpu_solve(inp)
    assert np.array_equal(a, b)


def test_full_size_1024_64_wavelengths_sampled(tmp_path):
    """The benchmark workload (1024^2, 64 wavelengths, 7 cascades) in the
    benchmark's launch configuration (the launch orders of the committed
    autotuner cache, read from a copy); J compared at sampled (cell,
    wavelength) points that the oracle computes through their dependency
    cones."""
    import shutil
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.line_medium(1024, 64, seed=2)
    print("[gpu] full-size 1024^2 x 64 formal solve", flush=True)
    plan = rcx.Plan(1024, 1024, 64)
    cache = tmp_path / "launch_orders.jsonl"
    shutil.copy(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2408_14425_amd",
                             "data", "launch_orders.jsonl"), cache)
    plan.autotune(str(cache))
    print("launch orders:", [plan.get_order(i) for i in range(7)], flush=True)
    chi = torch.from_numpy(inp.chi).cuda()
    eta = torch.from_numpy(inp.eta).cuda()
    J = plan.formal_solve(chi, eta)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy()
    plan.close()
    assert np.all(np.isfinite(Jg)) and Jg.min() > 0
    rng = np.random.default_rng(123)
    cells = [(0, 0), (1023, 1023), (0, 1023), (511, 512)] + [tuple(rng.integers(0, 1024, 2)) for _ in range(2)]
    need = np.zeros((1024, 1024), np.uint8)
    for x, z in cells:
        need[z, x] = 1
    for lam in (0, 21, 31, 32, 47, 63):
        Jo = oracle.formal_solve(inp.chi[lam:lam + 1], inp.eta[lam:lam + 1], 7, need=need)["J"][0]
        for x, z in cells:
            g, o = float(Jg[lam, z, x]), Jo[z, x]
            assert abs(g - o) <= RTOL * o, (lam, x, z, g, o)


@pytest.mark.parametrize("which", ["blobs64", "line256", "line96_w40"])
def test_fp16_storage_error_is_bounded(which):
    """16-bit cascade storage (FP16's 10-bit significand, the exponent
    rebased per wavelength below its largest source function): each stored
    value carries at most 2^-11 relative rounding error, accumulated over at
    most 6 stored cascades and averaged over taps and directions; the error
    against the FP64 oracle is reported and bounded by 1e-3."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    if which == "blobs64":
        inp = W.blobs_medium(64, seed=1)
    elif which == "line256":
        inp = W.line_medium(256, 64, seed=2, wave_subset=np.arange(0, 64, 8))
    else:
        # three 16-wavelength batches: a pair marched together, then one alone
        inp = W.line_medium(96, 64, seed=5, wave_subset=np.arange(0, 40))
    print(f"[gpu] fp16 storage {inp.name}", flush=True)
    plan = rcx.Plan(inp.nx, inp.nz, inp.n_wave, storage=rcx.RCX_STORE_F16_SCALED)
    J = plan.formal_solve(torch.from_numpy(inp.chi).cuda(), torch.from_numpy(inp.eta).cuda())
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().astype(np.float64)
    plan.close()
    Jo = oracle.formal_solve(inp.chi, inp.eta, inp.n_cascades)["J"]
    rel = np.abs(Jg - Jo) / Jo
    print(f"fp16 storage {which}: max rel {rel.max():.3e} mean {rel.mean():.3e}")
    assert rel.max() < 1e-3


@pytest.mark.parametrize("case", ["blobs64_incl8", "ragged_w20_incl3", "ragged_w20_incl8", "line96_w40_incl8_fp16"])
def test_inclined_formal_solve_matches_oracle(case):
    """2D invariance (Sec. 3.1): n_incl rays per flatland ray on a
    Gauss-Radau rule in mu = cos(inclination to y), each with the path per
    projected cell 1/sqrt(1 - mu^2) times longer; J the weighted sum. Cases:
    the paper's 8 inclinations on the 64^2 blobs, 3 on a ragged grid with a
    pair and an odd 16-wavelength batch (one pass per inclination), 8 on it
    (the 8 inclinations as slots of one march), and 8 with FP16 cascade
    storage (one pass per inclination; bounded as in the FP16 test)."""
    if case == "blobs64_incl8":
        inp, ni, st, tol = W.blobs_medium(64, seed=1), 8, 0, RTOL
    elif case.startswith("ragged_w20"):
        rng = np.random.default_rng(11)
        nx, nz, nw = 37, 53, 20
        chi = (10 ** rng.uniform(-2, 2, (nw, nz, nx))).astype(np.float32)
        eta = (chi * rng.uniform(0.2, 3.0, (nw, nz, nx))).astype(np.float32)
        ni = 3 if case.endswith("incl3") else 8
        inp, st, tol = W.FormalSolveInput(chi, eta, 1.0, W.n_cascades_for(nx, nz), "rand37x53w20"), 0, RTOL
    else:
        inp, ni, st, tol = W.line_medium(96, 64, seed=5, wave_subset=np.arange(0, 40)), 8, 1, 2e-3
    Jg = _gpu_solve(inp, n_incl=ni, storage=st)
    Jo = oracle.formal_solve_inclined(inp.chi, inp.eta, inp.n_cascades, ni, voxel=inp.voxel_scale)
    print(f"inclined {case}: max rel {_assert_rel(Jg, Jo, tol):.3e}")


def _ragged_w20():
    rng = np.random.default_rng(11)
    nx, nz, nw = 37, 53, 20
    chi = (10 ** rng.uniform(-2, 2, (nw, nz, nx))).astype(np.float32)
    eta = (chi * rng.uniform(0.2, 3.0, (nw, nz, nx))).astype(np.float32)
    return W.FormalSolveInput(chi, eta, 1.0, W.n_cascades_for(nx, nz), "rand37x53w20")


@pytest.mark.parametrize("case", ["blobs64", "ragged_w20", "blobs32_nc2", "blobs32_nc3", "disc128",
                                  "line96_w40_fp16", "blobs64_incl8", "ragged_w20_incl3"])
def test_bilinear_fix_matches_oracle(case):
    """Bilinear fix (Sec. 2.5): each interval of the cascades below the top
    traced once per bilinear probe, to the start of that probe's child cone.
    Cases: the 64^2 blobs; a ragged 37 x 53 grid with 20 wavelengths (two
    batches, the last one partial; its top cascade lies outside the domain,
    so the cascade below traces its four rays with nothing above); 2 and 3
    cascades (the top cascade marched and merged); the opaque disc in vacuum
    (zero-opacity cells); FP16 cascade storage (bounded as in the FP16
    test); the 8 inclinations as slots, and 3 inclinations as passes over a
    pair of batches."""
    tol, nc, st, ni = RTOL, 0, 0, 1
    if case == "blobs64":
        inp = W.blobs_medium(64, seed=1)
    elif case == "ragged_w20":
        inp = _ragged_w20()
    elif case == "blobs64_incl8":
        inp, ni = W.blobs_medium(64, seed=1), 8
    elif case == "ragged_w20_incl3":
        inp, ni = _ragged_w20(), 3
    elif case.startswith("blobs32_nc"):
        inp, nc = W.blobs_medium(32, seed=8), int(case[-1])
    elif case == "disc128":
        inp = W.disc_in_vacuum(128, 4.0)
    else:
        inp, st, tol = W.line_medium(96, 64, seed=5, wave_subset=np.arange(0, 40)), 1, 2e-3
    Jg = _gpu_solve(inp, n_cascades=nc, storage=st, bilinear_fix=True, n_incl=ni)
    if ni > 1:
        Jo = oracle.formal_solve_inclined(inp.chi, inp.eta, inp.n_cascades, ni, voxel=inp.voxel_scale,
                                          bilinear_fix=True)
    else:
        Jo = oracle.formal_solve(inp.chi, inp.eta, nc or inp.n_cascades, voxel=inp.voxel_scale,
                                 bilinear_fix=True)["J"]
    if case == "disc128":
        # cells no ray of any cascade reaches from the disc are exactly 0 on both sides
        assert np.array_equal(Jg == 0, Jo == 0)
        m = Jo > 0
        print(f"bilinear fix {case}: max rel {_assert_rel(Jg[m], Jo[m], tol):.3e}")
        return
    print(f"bilinear fix {case}: max rel {_assert_rel(Jg, Jo, tol):.3e}")


def test_bilinear_fix_thin_wall_is_opaque():
    """Behind a one-cell opaque wall the fix lets nothing through: the GPU's
    J there is exactly zero, like the oracle's, and the lit side agrees with
    the oracle."""
    n, x0 = 64, 30
    chi = np.zeros((1, n, n), np.float32)
    eta = np.zeros((1, n, n), np.float32)
    chi[0, :, :x0 - 4] = 0.3
    eta[0, :, :x0 - 4] = 0.3
    chi[0, :, x0] = 1e4
    inp = W.FormalSolveInput(chi, eta, 1.0, W.n_cascades_for(n, n), "wall64")
    Jg = _gpu_solve(inp, bilinear_fix=True)[0]
    Jo = oracle.formal_solve(chi, eta, inp.n_cascades, bilinear_fix=True)["J"][0]
    assert np.all(Jg[:, x0 + 1:] == 0.0)
    _assert_rel(Jg[:, :x0], Jo[:, :x0])


def test_bilinear_fix_full_size_sampled():
    """The benchmark workload (1024^2, 64 wavelengths, 7 cascades) with the
    fix, sampled (cell, wavelength) points against the oracle's dependency
    cones."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.line_medium(1024, 64, seed=2)
    print("[gpu] full-size 1024^2 x 64 formal solve, bilinear fix", flush=True)
    plan = rcx.Plan(1024, 1024, 64, bilinear_fix=True)
    J = plan.formal_solve(torch.from_numpy(inp.chi).cuda(), torch.from_numpy(inp.eta).cuda())
    torch.cuda.synchronize()
    Jg = J.cpu().numpy()
    plan.close()
    assert np.all(np.isfinite(Jg)) and Jg.min() > 0
    cells = [(0, 0), (1023, 1023), (511, 512), (700, 90)]
    need = np.zeros((1024, 1024), np.uint8)
    for x, z in cells:
        need[z, x] = 1
    for lam in (0, 31, 63):
        Jo = oracle.formal_solve(inp.chi[lam:lam + 1], inp.eta[lam:lam + 1], 7, need=need, bilinear_fix=True)["J"][0]
        for x, z in cells:
            g, o = float(Jg[lam, z, x]), Jo[z, x]
            assert abs(g - o) <= RTOL * o, (lam, x, z, g, o)


def _gpu_sparse(inp, active, storage=0, bilinear_fix=False, also_dense=False, n_incl=1):
    torch = _torch()
    from paper_2408_14425_amd import rcx
    print(f"[gpu] sparse formal solve {inp.name} active {active.mean():.3f} storage={storage} "
          f"bilinear_fix={bilinear_fix}", flush=True)
    plan = rcx.Plan(inp.nx, inp.nz, inp.n_wave, voxel_scale=inp.voxel_scale, storage=storage,
                    bilinear_fix=bilinear_fix, n_incl=n_incl)
    chi = torch.from_numpy(inp.chi).cuda()
    eta = torch.from_numpy(inp.eta).cuda()
    dense = None
    if also_dense:
        dense = plan.formal_solve(chi, eta).cpu().numpy()
    counts = plan.set_active(active)
    J = plan.formal_solve(chi, eta)
    torch.cuda.synchronize()
    out = J.cpu().numpy().astype(np.float64)
    again = None
    if also_dense:
        plan.set_active(None)
        again = plan.formal_solve(chi, eta).cpu().numpy()
    plan.close()
    return out, counts, dense, again


@pytest.mark.parametrize("case", ["blobs64", "ragged_w20", "line96_w40_fp16", "line256_w16_fix", "one_cell",
                                  "blobs64_incl8"])
def test_sparse_matches_oracle(case):
    """Sparse solve (Sec. 3.5): only the flagged probes' rays (the flagged
    cells and their bilinear parents up to the top) are marched, unflagged
    cells are transparent and empty, J is zero there. Cases: 30% of the 64^2
    blobs; a ragged grid with two batches; FP16 cascades with a pair of
    batches; 256^2 with the bilinear fix (its wide cascades launch the
    flagged probes tile by tile); a single flagged cell; the 8 inclinations
    as slots of one march."""
    tol, st, fix, ni = RTOL, 0, False, 1
    if case == "blobs64":
        inp = W.blobs_medium(64, seed=1)
        act = W.active_cells(64, 64, seed=1, frac=0.3)
    elif case == "ragged_w20":
        inp = _ragged_w20()
        act = W.active_cells(inp.nx, inp.nz, seed=2, frac=0.4)
    elif case == "line96_w40_fp16":
        inp, st, tol = W.line_medium(96, 64, seed=5, wave_subset=np.arange(0, 40)), 1, 2e-3
        act = W.active_cells(96, 96, seed=3, frac=0.25)
    elif case == "line256_w16_fix":
        inp, fix = W.line_medium(256, 64, seed=2, wave_subset=np.arange(0, 64, 4)), True
        act = W.active_cells(256, 256, seed=4, frac=0.25)
    elif case == "one_cell":
        inp = W.blobs_medium(64, seed=1)
        act = np.zeros((64, 64), bool)
        act[40, 17] = True
    else:
        inp, ni = W.blobs_medium(64, seed=1), 8
        act = W.active_cells(64, 64, seed=5, frac=0.3)
    Jg, counts, _, _ = _gpu_sparse(inp, act, storage=st, bilinear_fix=fix, n_incl=ni)
    if ni == 1:
        ref = oracle.formal_solve_sparse(inp.chi, inp.eta, inp.n_cascades, act, voxel=inp.voxel_scale,
                                         bilinear_fix=fix)
        Jo = ref["J"]
        # the library's flagged probes per cascade give the oracle's ray count
        top = inp.n_cascades - 1
        rays = sum(c * (4 << (2 * i)) * (4 if fix and i < top else 1) for i, c in enumerate(counts))
        assert rays * inp.n_wave == ref["rays"], (counts, ref["rays"])
    else:
        mu, wt = oracle.radau_inclinations(ni)
        Jo = sum(wt[m] * oracle.formal_solve_sparse(inp.chi, inp.eta, inp.n_cascades, act,
                                                    voxel=inp.voxel_scale / np.sqrt(1.0 - mu[m] ** 2))["J"]
                 for m in range(ni))
    assert counts[0] == act.sum()
    assert np.all(Jg[:, ~act] == 0.0)
    rel = _assert_rel(Jg[:, act], Jo[:, act], tol)
    print(f"sparse {case}: flagged per cascade {counts}, max rel {rel:.3e}")


def test_sparse_all_flagged_and_reset_equal_dense():
    """Every cell flagged gives the dense result bit for bit, and clearing
    the flags returns to it."""
    inp = W.line_medium(128, 64, seed=3, wave_subset=np.arange(0, 64, 4))
    Jg, counts, dense, again = _gpu_sparse(inp, np.ones((128, 128), bool), also_dense=True)
    assert np.array_equal(Jg, dense.astype(np.float64))
    assert np.array_equal(again, dense)


def test_sparse_full_size_sampled():
    """The benchmark workload (1024^2, 64 wavelengths) with a quarter of the
    cells flagged, in the benchmark's launch configuration; J at sampled
    flagged cells against the oracle's dependency cones of the medium with
    the unflagged cells emptied."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.line_medium(1024, 64, seed=2)
    act = W.active_cells(1024, 1024, seed=7, frac=0.25)
    print("[gpu] full-size 1024^2 x 64 sparse formal solve", flush=True)
    plan = rcx.Plan(1024, 1024, 64)
    counts = plan.set_active(act)
    J = plan.formal_solve(torch.from_numpy(inp.chi).cuda(), torch.from_numpy(inp.eta).cuda())
    torch.cuda.synchronize()
    Jg = J.cpu().numpy()
    plan.close()
    assert np.all(Jg[:, ~act] == 0.0) and np.all(Jg[:, act] > 0.0)
    zs, xs = np.nonzero(act)
    rng = np.random.default_rng(5)
    pick = rng.choice(len(zs), 6, replace=False)
    need = np.zeros((1024, 1024), np.uint8)
    need[zs[pick], xs[pick]] = 1
    for lam in (0, 31, 63):
        chi = np.where(act, inp.chi[lam], 0.0)[None]
        eta = np.where(act, inp.eta[lam], 0.0)[None]
        Jo = oracle.formal_solve(chi, eta, 7, need=need)["J"][0]
        for z, x in zip(zs[pick], xs[pick]):
            g, o = float(Jg[lam, z, x]), Jo[z, x]
            assert abs(g - o) <= RTOL * o, (lam, x, z, g, o)
    print("flagged per cascade", counts)


@pytest.mark.parametrize("t_rule, c0_dirs", [(1, 4), (0, 8)])
def test_bilinear_fix_interval_rule_and_directions(t_rule, c0_dirs):
    """The fix with the lengths-x4 interval rule, and with 8 cascade-0
    directions (cascade 0 stored and averaged by the J kernel), on 20
    wavelengths (a pair of batches)."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    rng = np.random.default_rng(12)
    nx, nz, nw = 48, 40, 20
    chi = (10 ** rng.uniform(-1.5, 1.5, (nw, nz, nx))).astype(np.float32)
    eta = (chi * rng.uniform(0.2, 3.0, (nw, nz, nx))).astype(np.float32)
    ncas = W.n_cascades_for(nx, nz)
    print(f"[gpu] bilinear fix t_rule={t_rule} c0_dirs={c0_dirs}", flush=True)
    plan = rcx.Plan(nx, nz, nw, t_rule=t_rule, c0_dirs=c0_dirs, bilinear_fix=True)
    J = plan.formal_solve(torch.from_numpy(chi).cuda(), torch.from_numpy(eta).cuda())
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().astype(np.float64)
    plan.close()
    Jo = oracle.formal_solve(chi, eta, ncas, t_rule=t_rule, c0_dirs=c0_dirs, bilinear_fix=True)["J"]
    print(f"fix t_rule={t_rule} c0_dirs={c0_dirs}: max rel {_assert_rel(Jg, Jo):.3e}")


def test_sparse_nothing_flagged_gives_zero_then_dense_again():
    """No flagged cell: J is 0 everywhere and nothing is marched; clearing
    the flags restores the dense result."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.blobs_medium(32, seed=8)
    print("[gpu] sparse formal solve, nothing flagged", flush=True)
    plan = rcx.Plan(inp.nx, inp.nz, inp.n_wave)
    chi = torch.from_numpy(inp.chi).cuda()
    eta = torch.from_numpy(inp.eta).cuda()
    dense = plan.formal_solve(chi, eta).cpu().numpy()
    counts = plan.set_active(np.zeros((32, 32), bool))
    J0 = plan.formal_solve(chi, eta).cpu().numpy()
    plan.set_active(None)
    J1 = plan.formal_solve(chi, eta).cpu().numpy()
    plan.close()
    assert all(c == 0 for c in counts)
    assert np.all(J0 == 0.0)
    assert np.array_equal(J1, dense)


@pytest.mark.parametrize("case, wx, wz", [("blobs64", 0.8, 0.6), ("blobs64", -0.26, 0.97), ("blobs64", -0.6, -0.8),
                                          ("ragged_w20", 0.5, -0.866), ("line96_w40", 0.9, 0.3)])
def test_emergent_matches_oracle(case, wx, wz):
    """Emergent intensity of a beam of parallel long characteristics (Sec.
    3.9) against the oracle's, ray by ray; rays that miss the domain are 0
    on both sides."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    if case == "blobs64":
        inp = W.blobs_medium(64, seed=1)
    elif case == "ragged_w20":
        inp = _ragged_w20()
    else:
        inp = W.line_medium(96, 64, seed=5, wave_subset=np.arange(0, 40))
    n = math.hypot(wx, wz)
    n_rays = int(math.ceil(abs(inp.nx * wz / n) + abs(inp.nz * wx / n))) + 6
    print(f"[gpu] emergent {inp.name} w=({wx}, {wz}) rays {n_rays}", flush=True)
    plan = rcx.Plan(inp.nx, inp.nz, inp.n_wave, voxel_scale=inp.voxel_scale)
    I = plan.emergent(torch.from_numpy(inp.chi).cuda(), torch.from_numpy(inp.eta).cuda(), wx, wz, n_rays)
    torch.cuda.synchronize()
    Ig = I.cpu().numpy().astype(np.float64)
    plan.close()
    Io = oracle.emergent(inp.chi, inp.eta, wx, wz, n_rays, voxel=inp.voxel_scale)
    hit = Io > 0
    assert np.all(Ig[~hit] == 0.0) and hit.sum() > 0
    print(f"emergent {case}: {hit[0].sum()} of {n_rays} rays hit, max rel {_assert_rel(Ig[hit], Io[hit]):.3e}")


def test_emergent_on_a_sparse_plan_sees_the_emptied_medium():
    """A sparse plan's emergent image treats unflagged cells as empty: it
    equals the oracle's image of the medium with those cells emptied."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.blobs_medium(64, seed=1)
    act = W.active_cells(64, 64, seed=9, frac=0.35)
    print("[gpu] emergent on a sparse plan", flush=True)
    plan = rcx.Plan(64, 64, inp.n_wave)
    plan.set_active(act)
    I = plan.emergent(torch.from_numpy(inp.chi).cuda(), torch.from_numpy(inp.eta).cuda(), 0.6, 0.8, 96)
    torch.cuda.synchronize()
    Ig = I.cpu().numpy().astype(np.float64)
    plan.close()
    Io = oracle.emergent(np.where(act, inp.chi, 0.0), np.where(act, inp.eta, 0.0), 0.6, 0.8, 96)
    hit = Io > 0
    assert np.all(Ig[~hit] == 0.0)
    print(f"sparse emergent: max rel {_assert_rel(Ig[hit], Io[hit]):.3e}")
