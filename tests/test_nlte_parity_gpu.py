"""GPU non-LTE iteration vs the FP64 oracle, through the C ABI.

Tolerances: populations 1e-3 relative (compared after the same number of
iterations, the oracle's stopping count for converged runs); J 1e-4
relative (the FP32 march, whose rounding is ~1e-6 to 1e-5 over these path
lengths, plus the march's Voigt profile, within 2e-5 of the oracle's);
rate coefficients 1e-4 of the sum of the magnitudes of their terms (the
preconditioned sums cancel in optically thick cells, so their relative
error is measured against the scale the FP32 terms carry); LTE populations
1e-12 (FP64 on both sides). Stored oracle results (tests/golden, written by
make_nlte_goldens.py from the oracle alone) stand in where the oracle would
need minutes: the converged 128^2 run and the sampled cells of the 1024^2,
160-wavelength atmosphere."""
import json
import math
import os

import numpy as np
import pytest

from paper_2408_14425_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def case32():
    inp = W.nlte_atmosphere(32, seed=3, n_line=32, n_cont=16)
    from oracle import nlte
    return inp, nlte.Problem(inp)


def _solver(inp, line_profile=0):
    from paper_2408_14425_amd import rcx
    print(f"[gpu] nlte solver {inp.name} profile {line_profile}", flush=True)
    return rcx.Nlte(inp, line_profile=line_profile)


# the line march's profile: the expansion about a = 0 (chosen automatically
# for this atmosphere's small damping) and the compact (a, x) table
PROFILES = [pytest.param(0, id="auto"), pytest.param(1, id="table")]


def test_voigt_table_matches_reference(case32):
    torch = _torch()
    from oracle import nlte
    inp, P = case32
    s = _solver(inp)
    rng = np.random.default_rng(1)
    a = rng.uniform(0, P.adamp.max(), 200000)
    x = np.concatenate([rng.uniform(0, 8, 100000), rng.uniform(8, 40, 100000)])
    got = s.voigt(torch.tensor(a, dtype=torch.float32, device="cuda"),
                  torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy().astype(np.float64)
    s.close()
    ref = nlte.voigt_H(a.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64))
    rel = np.abs(got - ref) / ref
    print("voigt table max rel", rel.max())
    assert rel.max() < 5e-5


@pytest.mark.parametrize("profile", PROFILES)
def test_march_profile_table_matches_reference(case32, profile):
    """The line march's profile (the expansion about a = 0 with Dawson's
    function from its LDS table, or the compact LDS table, Hermite in x and
    linear in a) against the oracle's Voigt function over the atmosphere's
    damping range, in the core and across the table/series boundary at
    x = 8."""
    torch = _torch()
    from oracle import nlte
    inp, P = case32
    s = _solver(inp, profile)
    rng = np.random.default_rng(2)
    a = rng.uniform(0, P.adamp.max(), 200000)
    x = np.concatenate([rng.uniform(0, 8, 100000), rng.uniform(7.9, 40, 100000)])
    got = s.voigt(torch.tensor(a, dtype=torch.float32, device="cuda"),
                  torch.tensor(x, dtype=torch.float32, device="cuda"), march=True).cpu().numpy().astype(np.float64)
    s.close()
    ref = nlte.voigt_H(a.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64))
    rel = np.abs(got - ref) / ref
    print("march profile table max rel", rel.max())
    assert rel.max() < 2e-5


def test_lte_populations(case32):
    _torch()
    inp, P = case32
    s = _solver(inp)
    pops = s.lte().cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    np.testing.assert_allclose(pops, P.lte, rtol=1e-12)


def test_formal_solve_J_and_first_update(case32):
    torch = _torch()
    inp, P = case32
    s = _solver(inp)
    pops = s.lte()
    rates, J = s.formal_solve_rates(pops, want_J=True)
    ch = s.stat_eq(rates, pops)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().reshape(inp.n_wave, -1).astype(np.float64)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    po = P.lte.copy()
    Jo, I0, chi_loc, H_loc, _ = P.formal_solve(po)
    Rup, Rdn = P.rates(po, I0, chi_loc, H_loc)
    new, cho = P.stat_eq(po, Rup, Rdn)
    relJ = np.abs(Jg - Jo) / np.abs(Jo)
    print("J max rel", relJ.max(), "first change gpu/oracle", ch, cho)
    assert relJ.max() < 1e-4
    relp = np.abs(pg - new) / np.abs(new)
    print("pops after one update max rel", relp.max())
    assert relp.max() < 1e-3
    assert abs(ch / cho - 1) < 1e-3


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rates_vs_oracle(rg, P, pops, I0, chi_loc, H_loc):
    """Max over transitions and cells of |R_gpu - R_oracle| / (magnitude
    sum), for the upward and downward coefficients."""
    Rup, Rdn = P.rates(pops, I0, chi_loc, H_loc)
    Aup, Adn = P.rate_magnitudes(pops, I0, chi_loc, H_loc)
    rg = rg.reshape(len(P.atom.trans), 2, -1).astype(np.float64)
    return float(np.max(np.abs(rg[:, 0] - Rup) / Aup)), float(np.max(np.abs(rg[:, 1] - Rdn) / Adn))


@pytest.mark.parametrize("profile", PROFILES)
def test_rates_elementwise(case32, profile):
    """The preconditioned rate coefficients of one formal solution at LTE,
    cell by cell and transition by transition, against the oracle's."""
    torch = _torch()
    inp, P = case32
    s = _solver(inp, profile)
    pops = s.lte()
    rates, _ = s.formal_solve_rates(pops)
    torch.cuda.synchronize()
    rg = rates.cpu().numpy()
    s.close()
    _, I0, chi_loc, H_loc, _ = P.formal_solve(P.lte)
    eu, ed = _rates_vs_oracle(rg, P, P.lte, I0, chi_loc, H_loc)
    print(f"rates vs oracle ({profile}): up {eu:.3e}, down {ed:.3e} of the magnitude sums")
    assert eu < 1e-4 and ed < 1e-4


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_cool_atmosphere_far_uv_continuum(storage):
    """An atmosphere at 5000 K everywhere (16^2: its blobs cover the grid),
    whose Lyman continuum at half the edge wavelength has J ~ 1e-31 (17
    orders below the lines): alpha (n_i*/n_c*) e^{-h nu / kT} is then below
    FP32's range, so the rate epilogue must not form it on its own. J at LTE
    for every wavelength and the rates (of their magnitude sums) to 1e-4 with
    FP32 cascades and 1e-3 with 16-bit ones, the populations after one
    iteration to 1e-3; a continuum batch of 8 wavelengths (half a batch)."""
    torch = _torch()
    from oracle import nlte
    from paper_2408_14425_amd import rcx
    inp = W.nlte_atmosphere(16, seed=5, n_line=16, n_cont=8)
    assert inp.T.max() <= 5000.0 + 1e-9
    P = nlte.Problem(inp)
    print(f"[gpu] nlte cool atmosphere {inp.name} {storage}", flush=True)
    s = rcx.Nlte(inp, storage=rcx.RCX_STORE_F32 if storage == "f32" else rcx.RCX_STORE_F16_SCALED)
    pops = s.lte()
    rates, J = s.formal_solve_rates(pops, want_J=True)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().reshape(inp.n_wave, -1).astype(np.float64)
    rg = rates.cpu().numpy()
    s.iterate(pops, 1, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    Jo, I0, chi_loc, H_loc, _ = P.formal_solve(P.lte)
    relJ = np.abs(Jg - Jo) / np.abs(Jo)
    eu, ed = _rates_vs_oracle(rg, P, P.lte, I0, chi_loc, H_loc)
    po, _ = P.iterate(P.lte.copy(), 1)
    relp = np.abs(pg - po) / np.abs(po)
    print(f"{storage}: J max rel {relJ.max():.3e} (smallest J {Jo.min():.2e}), rates {eu:.3e} / {ed:.3e}, "
          f"pops {relp.max():.3e}")
    tol = 1e-4 if storage == "f32" else 1e-3
    assert relJ.max() < tol
    assert eu < tol and ed < tol
    assert relp.max() < 1e-3


def test_two_continuum_batches():
    """32 continuum wavelengths: two continuum batches, which the march pairs
    per lane on the cascades with at most 256 directions. J to 1e-4, the
    rates to 1e-4 of their magnitude sums, populations after 3 iterations
    to 1e-3."""
    torch = _torch()
    from oracle import nlte
    inp = W.nlte_atmosphere(32, seed=6, n_line=16, n_cont=32)
    P = nlte.Problem(inp)
    s = _solver(inp)
    pops = s.lte()
    rates, J = s.formal_solve_rates(pops, want_J=True)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().reshape(inp.n_wave, -1).astype(np.float64)
    rg = rates.cpu().numpy()
    rc, it, ch = s.iterate(pops, 3, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    Jo, I0, chi_loc, H_loc, _ = P.formal_solve(P.lte)
    relJ = np.abs(Jg - Jo) / np.abs(Jo)
    eu, ed = _rates_vs_oracle(rg, P, P.lte, I0, chi_loc, H_loc)
    po, _ = P.iterate(P.lte.copy(), 3)
    relp = np.abs(pg - po) / np.abs(po)
    cont = inp.trans == inp.trans.max()
    print(f"two continuum batches: J max rel {relJ.max():.3e} (continuum {relJ[cont].max():.3e}), "
          f"rates {eu:.3e} / {ed:.3e}, pops after 3 iterations {relp.max():.3e}")
    assert cont.sum() == 32
    assert relJ.max() < 1e-4
    assert eu < 1e-4 and ed < 1e-4
    assert relp.max() < 1e-3


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_line_batch_groups(storage):
    """112 wavelengths per line: 7 batches, which the march groups as 4 + 2
    + 1 (the 4 and the 2 share their cascades above 0, each batch takes its
    own cascade 0). One launch per group and marched cascade above 0 and one
    per batch at cascade 0; J to 1e-4 (16-bit cascades 1e-3), the rates to
    the same bar of their magnitude sums, the populations after one
    iteration to 1e-3."""
    torch = _torch()
    from oracle import nlte
    from paper_2408_14425_amd import rcx
    inp = W.nlte_atmosphere(32, seed=4, n_line=112, n_cont=16)
    P = nlte.Problem(inp)
    print(f"[gpu] nlte line batch groups {inp.name} {storage}", flush=True)
    s = rcx.Nlte(inp, storage=rcx.RCX_STORE_F32 if storage == "f32" else rcx.RCX_STORE_F16_SCALED)
    pops = s.lte()
    s.set_timing(True)
    rates, J = s.formal_solve_rates(pops, want_J=True)
    torch.cuda.synchronize()
    t = s.get_timing()
    s.set_timing(False)
    Jg = J.cpu().numpy().reshape(inp.n_wave, -1).astype(np.float64)
    rg = rates.cpu().numpy()
    s.iterate(pops, 1, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    plan = rcx.Plan(inp.nx, inp.nz, 1)
    w = plan.work()
    plan.close()
    marched = w.n_cascades - (1 if w.top_skipped else 0)
    assert marched >= 2
    n_lines = len(inp.atom["lines"])
    assert list(np.bincount(inp.trans)[:n_lines]) == [112] * n_lines
    assert t["line"][1] == n_lines * ((marched - 1 + 4) + (marched - 1 + 2) + marched)
    Jo, I0, chi_loc, H_loc, _ = P.formal_solve(P.lte)
    relJ = np.abs(Jg - Jo) / np.abs(Jo)
    eu, ed = _rates_vs_oracle(rg, P, P.lte, I0, chi_loc, H_loc)
    po, _ = P.iterate(P.lte.copy(), 1)
    relp = np.abs(pg - po) / np.abs(po)
    print(f"line batch groups {storage}: J max rel {relJ.max():.3e}, rates {eu:.3e} / {ed:.3e}, "
          f"pops {relp.max():.3e}")
    tol = 1e-4 if storage == "f32" else 1e-3
    assert relJ.max() < tol
    assert eu < tol and ed < tol
    assert relp.max() < 1e-3


def test_converged_128_at_oracle_iteration_count():
    """The 128^2 atmosphere (6 cascades) iterated for the oracle's count K
    (stored: the oracle needs minutes for it) agrees with the oracle's
    populations to 1e-3, and the GPU's own stopping test fires within one
    iteration of K."""
    _torch()
    g = np.load(os.path.join(GOLDEN, "nlte128_s4.npz"))
    K = int(g["K"])
    inp = W.nlte_atmosphere(128, seed=4, n_line=32, n_cont=16)
    s = _solver(inp)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, K, 0.0)
    pg = pops.cpu().numpy().reshape(g["pops"].shape)
    pops2 = s.lte()
    rc2, it2, ch2 = s.iterate(pops2, K + 2, 1e-3)
    s.close()
    relp = np.abs(pg - g["pops"]) / np.abs(g["pops"])
    print(f"128^2 converged: oracle {K} iterations (last change {g['changes'][-1]:.3e}); gpu after {it} "
          f"({ch:.3e}): max rel {relp.max():.3e}; gpu stopping test rc {rc2} at {it2}")
    assert it == K
    assert relp.max() < 1e-3
    assert rc2 == 0 and abs(it2 - K) <= 1


def test_full_size_atmosphere_sampled_cells():
    """The 1024^2, 160-wavelength atmosphere (7 cascades, two continuum
    batches, the tiled launch order and XCD-chunked workgroups of the full
    size) at LTE: J at four sampled cells for every wavelength to 1e-4, the
    rate coefficients there to 1e-4 of their magnitude sums, and the
    populations after one equilibrium step to 1e-3, against the oracle's
    dependency-cone solve of those cells (stored)."""
    torch = _torch()
    with open(os.path.join(GOLDEN, "nlte1024_s3_cells.json")) as f:
        g = json.load(f)
    cells = np.array(g["cells"])
    inp = W.nlte_atmosphere(1024, seed=3, n_line=64, n_cont=32)
    s = _solver(inp)
    pops = s.lte()
    rates, J = s.formal_solve_rates(pops, want_J=True)
    lte = pops.cpu().numpy().reshape(4, -1)[:, cells]
    s.stat_eq(rates, pops)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().reshape(inp.n_wave, -1)[:, cells].astype(np.float64)
    rg = rates.cpu().numpy().reshape(3, 2, -1)[:, :, cells].astype(np.float64)
    pg = pops.cpu().numpy().reshape(4, -1)[:, cells]
    s.close()
    relJ = np.abs(Jg - np.array(g["J"])) / np.abs(np.array(g["J"]))
    eu = np.max(np.abs(rg[:, 0] - np.array(g["Rup"])) / np.array(g["Aup"]))
    ed = np.max(np.abs(rg[:, 1] - np.array(g["Rdn"])) / np.array(g["Adn"]))
    relp = np.abs(pg - np.array(g["pops1"])) / np.abs(np.array(g["pops1"]))
    print(f"1024^2 sampled cells {cells.tolist()}: J max rel {relJ.max():.3e}, rates {eu:.3e} / {ed:.3e}, "
          f"pops after one step {relp.max():.3e}")
    np.testing.assert_allclose(lte, np.array(g["lte"]), rtol=1e-12)
    assert relJ.max() < 1e-4
    assert eu < 1e-4 and ed < 1e-4
    assert relp.max() < 1e-3


@pytest.mark.parametrize("n_incl", [2, 8])
def test_inclinations(case32, n_incl):
    """2D invariance in the non-LTE iteration (Sec. 3.1; the paper iterates
    with 8 inclinations): J (the Gauss-Radau sum over inclinations) to 1e-4,
    the rate coefficients to 1e-4 of their magnitude sums, and the
    populations after 3 iterations to 1e-3, against the oracle with the same
    inclinations."""
    torch = _torch()
    from oracle import nlte
    from paper_2408_14425_amd import rcx
    inp, _ = case32
    P = nlte.Problem(inp, n_incl=n_incl)
    print(f"[gpu] nlte {inp.name} with {n_incl} inclinations", flush=True)
    s = rcx.Nlte(inp, n_incl=n_incl)
    pops = s.lte()
    rates, J = s.formal_solve_rates(pops, want_J=True)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy().reshape(inp.n_wave, -1).astype(np.float64)
    rg = rates.cpu().numpy()
    rc, it, ch = s.iterate(pops, 3, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    Jo, I0, chi_loc, H_loc, _ = P.formal_solve(P.lte)
    relJ = np.abs(Jg - Jo) / np.abs(Jo)
    eu, ed = _rates_vs_oracle(rg, P, P.lte, I0, chi_loc, H_loc)
    po, _ = P.iterate(P.lte.copy(), 3)
    relp = np.abs(pg - po) / np.abs(po)
    Jflat = nlte.Problem(inp).formal_solve(P.lte)[0]
    print(f"{n_incl} inclinations: J max rel {relJ.max():.3e} (differs from flatland by up to "
          f"{np.max(np.abs(Jo - Jflat) / Jflat):.2e}), rates {eu:.3e} / {ed:.3e}, pops after 3 iterations "
          f"{relp.max():.3e}")
    assert relJ.max() < 1e-4
    assert eu < 1e-4 and ed < 1e-4
    assert relp.max() < 1e-3


def test_march_timing_counts(case32):
    """Kernel timing of the non-LTE march: one formal solution with 2
    inclinations records one launch per (batch, marched cascade,
    inclination), except that 4 (or 2) consecutive batches of one line share
    their launches of the cascades above 0; the cell steps x wavelengths of the line and
    continuum launches equal the plan's dense per-cascade counts times the
    batches' wavelengths; the records are dropped after reading."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp, _ = case32
    print(f"[gpu] nlte timing {inp.name}", flush=True)
    s = rcx.Nlte(inp, n_incl=2)
    pops = s.lte()
    s.set_timing(True)
    s.formal_solve_rates(pops)
    t = s.get_timing()
    s.set_timing(False)
    s.formal_solve_rates(pops)
    torch.cuda.synchronize()
    t2 = s.get_timing()
    s.close()
    plan = rcx.Plan(inp.nx, inp.nz, 1)
    w = plan.work()
    plan.close()
    marched = w.n_cascades - (1 if w.top_skipped else 0)
    # batches of <= 16 wavelengths per transition; transitions below the
    # number of lines are lines, the rest continua
    n_lines = len(inp.atom["lines"])
    counts = np.bincount(inp.trans)
    line_batches = sum(-(-int(c) // 16) for c in counts[:n_lines])
    cont_batches = sum(-(-int(c) // 16) for c in counts[n_lines:])
    n_lw = int(counts[:n_lines].sum())
    n_cont = int(counts[n_lines:].sum())
    assert line_batches > 0 and cont_batches > 0
    # a line's batches march in groups of 4, then 2 (when a cascade above 0
    # is marched): a group of G takes one launch per cascade above 0 and one
    # per batch at 0
    line_launches = 0
    for c in counts[:n_lines]:
        nb, b = -(-int(c) // 16), 0
        while b < nb:
            G = next(g for g in (4, 2, 1) if nb - b >= g) if marched >= 2 else 1
            line_launches += (marched - 1 + G) if G > 1 else marched
            b += G
    assert t["line"][1] == line_launches * 2
    assert t["continuum"][1] == cont_batches * marched * 2
    assert t["line"][2] == n_lw * w.cell_steps * 2
    assert t["continuum"][2] == n_cont * w.cell_steps * 2
    assert t["line"][0] > 0 and t["continuum"][0] > 0
    assert t2 == {"line": (0.0, 0, 0), "continuum": (0.0, 0, 0)}


def test_inclinations_converged_at_oracle_iteration_count(case32):
    """With 3 inclinations the GPU iterated for the oracle's stopping count
    agrees with the oracle's populations to 1e-3."""
    _torch()
    from oracle import nlte
    from paper_2408_14425_amd import rcx
    inp, _ = case32
    P = nlte.Problem(inp, n_incl=3)
    po, changes = P.iterate(P.lte.copy(), 200, tol=1e-3)
    K = len(changes)
    s = rcx.Nlte(inp, n_incl=3)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, K, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    relp = np.abs(pg - po) / np.abs(po)
    print(f"3 inclinations converged: oracle {K} iterations; gpu max rel {relp.max():.3e}")
    assert it == K
    assert relp.max() < 1e-3


@pytest.mark.parametrize("profile", PROFILES)
def test_three_iterations(case32, profile):
    _torch()
    inp, P = case32
    s = _solver(inp, profile)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, 3, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    po, changes = P.iterate(P.lte.copy(), 3)
    relp = np.abs(pg - po) / np.abs(po)
    print("3 iterations: max rel", relp.max(), "changes", ch, changes[-1])
    assert it == 3 and rc == 1
    assert relp.max() < 1e-3


def test_converged_at_oracle_iteration_count(case32):
    """The oracle iterates to max change < 1e-3 (K iterations). The GPU run
    for exactly K iterations agrees with it to 1e-3 in the populations, and
    the GPU's own stopping test fires within one iteration of K: the change
    it tests (max relative difference of successive populations, about 1e-3
    here) is formed from FP32 radiances, and differences at the 1e-4 level,
    inside the population bar, move its crossing of the threshold by up to
    one iteration."""
    _torch()
    inp, P = case32
    po, changes = P.iterate(P.lte.copy(), 200, tol=1e-3)
    K = len(changes)
    s = _solver(inp)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, K, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    pops2 = s.lte()
    rc2, it2, ch2 = s.iterate(pops2, K + 2, 1e-3)
    s.close()
    relp = np.abs(pg - po) / np.abs(po)
    print(f"converged: oracle {K} iterations (last change {changes[-1]:.3e}); gpu after {it}: change {ch:.3e}, "
          f"max rel {relp.max():.3e}; gpu stopping test: rc {rc2} at {it2} ({ch2:.3e})")
    assert it == K
    assert relp.max() < 1e-3
    assert rc2 == 0 and abs(it2 - K) <= 1 and ch2 < 1e-3


def test_ng_accelerated_iteration_matches_oracle(case32):
    """Ng acceleration (order 2, first after 4 iterations, then every 4):
    the oracle converges in fewer iterations than the plain iteration; the
    GPU run for the same count agrees with it to 1e-3 and its own stopping
    test fires within one iteration of that count."""
    _torch()
    inp, P = case32
    _, plain = P.iterate(P.lte.copy(), 200, tol=1e-3)
    po, changes = P.iterate(P.lte.copy(), 200, tol=1e-3, ng=(2, 4, 4))
    K = len(changes)
    s = _solver(inp)
    s.set_acceleration(2, 4, 4)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, K, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.set_acceleration(2, 4, 4)
    pops2 = s.lte()
    rc2, it2, ch2 = s.iterate(pops2, K + 2, 1e-3)
    s.close()
    relp = np.abs(pg - po) / np.abs(po)
    print(f"ng: oracle {K} iterations (plain {len(plain)}); gpu after {it}: max rel {relp.max():.3e}; "
          f"gpu stopping test: rc {rc2} at {it2} ({ch2:.3e})")
    assert K < len(plain)
    assert it == K
    assert relp.max() < 1e-3
    assert rc2 == 0 and abs(it2 - K) <= 1


def test_fp16_storage_converged_populations(case32):
    """16-bit cascade storage inside the non-LTE iteration: cascades >= 1
    stored as FP16-precision codes (10-bit significand, relative rounding
    2^-11) whose 6-bit exponent is rebased per wavelength below its largest
    source function, so the 2^43 dynamic range of the Lyman continuum
    between hot and cool cells stays inside the format. J of every
    transition agrees with the FP64 oracle to 1e-3 relative, element by
    element (at most ~6 stored cascades of 2^-11 each, averaged over taps
    and directions); the rate coefficients (cascade 0 is FP32, but its
    merged radiance carries the stored cascades' rounding) agree with the
    oracle to 1e-3 of their magnitude sums, the bound of J; the converged
    populations (same iteration count as the oracle) to 1e-3."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp, P = case32
    po, changes = P.iterate(P.lte.copy(), 200, tol=1e-3)
    K = len(changes)
    print(f"[gpu] nlte fp16 {inp.name}", flush=True)
    res = {}
    for st in (rcx.RCX_STORE_F32, rcx.RCX_STORE_F16_SCALED):
        s = rcx.Nlte(inp, storage=st)
        pops = s.lte()
        r, J = s.formal_solve_rates(pops, want_J=True)
        torch.cuda.synchronize()
        res[st] = (r.cpu().numpy(), J.cpu().numpy().reshape(inp.n_wave, -1).astype(np.float64))
        if st == rcx.RCX_STORE_F16_SCALED:
            rc, it, ch = s.iterate(pops, K, 1e-3)
            pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
        s.close()
    Jo, I0, chi_loc, H_loc, _ = P.formal_solve(P.lte.copy())
    J16 = res[rcx.RCX_STORE_F16_SCALED][1]
    rel = np.abs(J16 - Jo) / np.abs(Jo)
    worst = 0.0
    for t in range(int(inp.trans.max()) + 1):
        sel = inp.trans == t
        print(f"fp16 J, transition {t}: max rel {rel[sel].max():.3e}, median {np.median(rel[sel]):.3e}")
        worst = max(worst, float(rel[sel].max()))
    eu, ed = _rates_vs_oracle(res[rcx.RCX_STORE_F16_SCALED][0], P, P.lte, I0, chi_loc, H_loc)
    relp = np.abs(pg - po) / np.abs(po)
    print(f"fp16: rates vs oracle {eu:.3e} / {ed:.3e} of the magnitude sums; after {it} iterations pops max rel "
          f"{relp.max():.3e}")
    assert np.all(np.isfinite(J16))
    assert worst < 1e-3
    assert eu < 1e-3 and ed < 1e-3
    assert relp.max() < 1e-3


def test_converged_64_at_oracle_iteration_count():
    """The same at 64^2 (the oracle's iteration count, populations to 1e-3)."""
    _torch()
    from oracle import nlte
    inp = W.nlte_atmosphere(64, seed=4, n_line=32, n_cont=16)
    P = nlte.Problem(inp)
    po, changes = P.iterate(P.lte.copy(), 200, tol=1e-3)
    K = len(changes)
    s = _solver(inp)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, K, 0.0)  # exactly the oracle's iteration count
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    relp = np.abs(pg - po) / np.abs(po)
    print(f"64^2 converged: oracle {K} iterations (last change {changes[-1]:.3e}); gpu {it} ({ch:.3e}); "
          f"max rel {relp.max():.3e}")
    assert it == K
    assert relp.max() < 1e-3


def test_charge_conservation_matches_oracle(case32):
    """Charge conservation (Sec. 3.3): one Newton-Raphson step on the
    populations and n_e after each equilibrium step. After 5 iterations the
    GPU's populations and electron density agree with the oracle's to 1e-3,
    and the converged run stops within one iteration of the oracle's
    count."""
    torch = _torch()
    inp, P = case32
    po, changes = P.iterate(P.lte.copy(), 5, charge=True)
    ne_o = P.last_ne.copy()
    pc, ch_c = P.iterate(P.lte.copy(), 200, tol=1e-3, charge=True)
    K = len(ch_c)
    s = _solver(inp)
    s.set_charge_conservation(True)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, 5, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    ne_g = s.electron_density().cpu().numpy()
    s.close()
    s = _solver(inp)
    s.set_charge_conservation(True)
    pops2 = s.lte()
    rc2, it2, ch2 = s.iterate(pops2, K + 2, 1e-3)
    s.close()
    relp = np.abs(pg - po) / np.abs(po)
    rele = np.abs(ne_g - ne_o) / ne_o
    print(f"charge: after 5 iterations pops max rel {relp.max():.3e}, n_e max rel {rele.max():.3e}, "
          f"n_e moved {np.abs(ne_o / P.ne - 1).max():.3e}; oracle converges in {K}, gpu rc {rc2} at {it2}")
    assert it == 5
    assert relp.max() < 1e-3 and rele.max() < 1e-3
    assert rc2 == 0 and abs(it2 - K) <= 1


def test_pressure_conservation_matches_oracle(case32):
    """Pressure conservation with charge conservation (Sec. 3.3): n_Htot
    rescaled after each charge step to hold the starting pressure; after 5
    iterations the populations (and so n_Htot, their sum) and n_e agree with
    the oracle's to 1e-3."""
    _torch()
    inp, P = case32
    po, _ = P.iterate(P.lte.copy(), 5, charge=True, pressure=True)
    ne_o = P.last_ne.copy()
    s = _solver(inp)
    s.set_charge_conservation(True)
    s.set_pressure_conservation(True)
    pops = s.lte()
    rc, it, ch = s.iterate(pops, 5, 0.0)
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    ne_g = s.electron_density().cpu().numpy()
    s.close()
    relp = np.abs(pg - po) / np.abs(po)
    rele = np.abs(ne_g - ne_o) / ne_o
    print(f"pressure: pops max rel {relp.max():.3e}, n_e max rel {rele.max():.3e}, "
          f"n_Htot moved {np.abs(po.sum(axis=0) / P.ntot - 1).max():.3e}")
    assert relp.max() < 1e-3 and rele.max() < 1e-3
    np.testing.assert_allclose(pg.sum(axis=0) + ne_g, P.ntot + P.ne, rtol=1e-12)


def test_collisional_starting_n_e_matches_oracle(case32):
    """The starting n_e from the collisional rates alone (Sec. 3.3): 20
    equilibrium + charge steps with the radiative rates off, FP64 on both
    sides: n_e and the LTE populations at it agree to 1e-10."""
    _torch()
    inp, P = case32
    Q = P.collisional_ne(20)
    s = _solver(inp)
    s.collisional_ne(20)
    ne_g = s.electron_density().cpu().numpy()
    lte_g = s.lte().cpu().numpy().reshape(P.atom.n_levels, -1)
    s.close()
    print(f"collisional n_e: max rel {np.abs(ne_g / Q.ne - 1).max():.3e}, moved {np.abs(Q.ne / P.ne - 1).max():.3e}")
    np.testing.assert_allclose(ne_g, Q.ne, rtol=1e-10)
    np.testing.assert_allclose(lte_g, Q.lte, rtol=1e-10)


def test_sparse_nlte_matches_oracle():
    """Sparse non-LTE iteration (Sec. 3.5): a 32^2 atmosphere with 1e6 K
    corona in about 45% of the cells and a 250 kK cut. After 5 iterations
    the flagged cells' populations agree with the oracle's to 1e-3, the
    coronal populations are still their LTE start and their rates are 0;
    the converged run stops within one iteration of the oracle's count."""
    torch = _torch()
    from oracle import nlte
    inp = W.nlte_atmosphere(32, seed=3, n_line=32, n_cont=16, corona_frac=0.45)
    P = nlte.Problem(inp, t_cut=2.5e5)
    act = P.active
    assert 0.3 < (~act).mean() < 0.6
    po, _ = P.iterate(P.lte.copy(), 5)
    _, ch = P.iterate(P.lte.copy(), 200, tol=1e-3)
    K = len(ch)
    s = _solver(inp)
    counts = s.set_temperature_cut(2.5e5)
    pops = s.lte()
    lte0 = pops.clone()
    rc, it, chg = s.iterate(pops, 5, 0.0)
    rates, _ = s.formal_solve_rates(pops)
    torch.cuda.synchronize()
    pg = pops.cpu().numpy().reshape(P.atom.n_levels, -1)
    l0 = lte0.cpu().numpy().reshape(P.atom.n_levels, -1)
    rg = rates.cpu().numpy()
    s.close()
    s = _solver(inp)
    s.set_temperature_cut(2.5e5)
    p2 = s.lte()
    rc2, it2, ch2 = s.iterate(p2, K + 2, 1e-3)
    s.close()
    relp = np.abs(pg[:, act] - po[:, act]) / np.abs(po[:, act])
    print(f"sparse nlte: flagged cells {act.mean():.2f}, probes per cascade {counts}; after 5 iterations "
          f"max rel {relp.max():.3e}; oracle converges in {K}, gpu rc {rc2} at {it2}")
    assert relp.max() < 1e-3
    assert np.array_equal(pg[:, ~act], l0[:, ~act])
    assert np.all(rg.reshape(rg.shape[0], 2, -1)[:, :, ~act] == 0.0)
    assert rc2 == 0 and abs(it2 - K) <= 1


@pytest.mark.parametrize("wx, wz", [(0.8, 0.6), (-0.45, -0.9)])
def test_emergent_spectra_match_oracle(case32, wx, wz):
    """Emergent spectra (Sec. 3.9) along a beam of parallel long
    characteristics at the oracle's populations after two iterations (given
    to both sides): 1e-4 relative (the FP32 march and the march's Voigt
    profile, as for J)."""
    torch = _torch()
    inp, P = case32
    po, _ = P.iterate(P.lte.copy(), 2)
    s = _solver(inp)
    pops = torch.from_numpy(np.ascontiguousarray(po).reshape(P.atom.n_levels, inp.nz, inp.nx)).to("cuda:0")
    n_rays = int(math.ceil(abs(inp.nx * wz) + abs(inp.nz * wx))) + 4
    I = s.emergent(pops, wx, wz, n_rays)
    torch.cuda.synchronize()
    Ig = I.cpu().numpy().astype(np.float64)
    s.close()
    Io = P.emergent(po, wx, wz, n_rays)
    hit = Io > 0
    rel = np.abs(Ig[hit] - Io[hit]) / Io[hit]
    print(f"emergent spectra w=({wx}, {wz}): {hit[0].sum()} of {n_rays} rays hit, max rel {rel.max():.3e}")
    assert np.all(Ig[~hit] == 0.0)
    assert rel.max() < 1e-4


def test_emergent_spectra_of_a_sparse_solver():
    """With a temperature cut the emergent spectra see the corona as empty:
    they equal the oracle's for the sparse problem (the coronal fields
    emptied) at the same populations."""
    torch = _torch()
    from oracle import nlte
    inp = W.nlte_atmosphere(32, seed=3, n_line=16, n_cont=8, corona_frac=0.45)
    P = nlte.Problem(inp, t_cut=2.5e5)
    s = _solver(inp)
    s.set_temperature_cut(2.5e5)
    pops = s.lte()
    I = s.emergent(pops, 0.8, -0.6, 48)
    torch.cuda.synchronize()
    Ig = I.cpu().numpy().astype(np.float64)
    s.close()
    Io = P.emergent(P.lte, 0.8, -0.6, 48)
    hit = Io > 0
    rel = np.abs(Ig[hit] - Io[hit]) / Io[hit]
    print(f"sparse emergent spectra: max rel {rel.max():.3e}")
    assert np.all(Ig[~hit] == 0.0)
    assert rel.max() < 1e-4


def test_autotune_keeps_the_iteration_bitwise(tmp_path):
    """rcx_nlte_autotune changes only the launch orders of the solver's
    marches (each ray's arithmetic does not depend on where it runs): one
    iteration from LTE gives bitwise the same populations with the tuned
    orders as with the defaults, and the tuner appends one cache line."""
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.nlte_atmosphere(64, seed=4, n_line=16, n_cont=8)
    print(f"[gpu] nlte autotune {inp.name}", flush=True)
    out = []
    for tuned in (False, True):
        s = rcx.Nlte(inp)
        if tuned:
            s.autotune(tmp_path / "orders.jsonl")
        p = s.lte()
        s.iterate(p, 1, 0.0)
        torch.cuda.synchronize()
        out.append(p.clone())
        s.close()
    assert (tmp_path / "orders.jsonl").read_text().count("\n") == 1
    assert torch.equal(out[0], out[1])
