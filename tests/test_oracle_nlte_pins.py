"""Pins of the FP64 non-LTE oracle (no GPU) against what physics and the
paper fix: textbook atomic constants, Kirchhoff / detailed balance at LTE,
the collision-dominated limit, profile normalisation, the cascade-0 operator
as the derivative of the march, rate-matrix conservation and the fixed point
of the preconditioned iteration."""
import math

import numpy as np
import pytest
from scipy.special import wofz

import oracle
from oracle import nlte
from paper_2408_14425_amd import workloads as W


@pytest.fixture(scope="module")
def small():
    inp = W.nlte_atmosphere(16, seed=5, n_line=24, n_cont=8)
    return nlte.Problem(inp)


def test_voigt_matches_faddeeva():
    """H(a, x) = Re w(x + i a) against scipy's Faddeeva function."""
    rng = np.random.default_rng(0)
    a = 10 ** rng.uniform(-5, 0.5, 50000)
    x = rng.uniform(-30, 30, 50000)
    ref = wofz(x + 1j * a).real
    np.testing.assert_allclose(nlte.voigt_H(a, x), ref, rtol=1e-7)


def test_einstein_A_textbook_values():
    """Oscillator strengths 0.4164 (Ly-alpha) and 0.6407 (H-alpha) give the
    textbook n-averaged hydrogen rates 4.699e8 and 4.410e7 1/s."""
    atom = nlte.Atom(W.SYNTH_ATOM)
    assert abs(atom.lines[0].A / 4.699e8 - 1) < 2e-3
    assert abs(atom.lines[1].A / 4.410e7 - 1) < 2e-3
    # Einstein relation between spontaneous and stimulated emission:
    # A_ji = (2 h nu^3 / c^2) B_ji with B_ji = (g_i/g_j) 4 pi sigma / (h nu)
    for t in atom.lines:
        Bji = atom.g[t.i] / atom.g[t.j] * 4 * math.pi * t.sigma / (nlte.H_PLANCK * t.nu0)
        assert abs(t.A / (2 * nlte.H_PLANCK * t.nu0 ** 3 / nlte.C_LIGHT ** 2 * Bji) - 1) < 1e-12


def test_saha_boltzmann_constants():
    """Boltzmann ratio of level 1 to 0 is (g1/g0) e^{-E1/kT} (E1 = hc / 121.57 nm); the Saha
    factor (2 pi m_e k T / h^2)^{3/2} is 2.4147e21 T^{3/2} m^-3."""
    atom = nlte.Atom(W.SYNTH_ATOM)
    T = np.array([6000.0, 2e4])
    ne = np.array([1e16, 1e17])
    n = nlte.lte_populations(atom, T, ne, np.array([1.0, 1.0]))
    kT_eV = nlte.K_BOLTZ * T / nlte.EV
    np.testing.assert_allclose(n[1] / n[0], 4.0 * np.exp(-1239.8419843320025 / 121.57 / kT_eV), rtol=1e-9)
    saha = 2.4147e21 * T ** 1.5 / ne * 2 * (1.0 / 2.0) * np.exp(-1239.8419843320025 / 91.18 / kT_eV)
    np.testing.assert_allclose(n[3] / n[0], saha, rtol=2e-4)
    np.testing.assert_allclose(n.sum(axis=0), 1.0, rtol=1e-14)


def test_line_profile_normalised_on_grid(small):
    """sum_lambda phi dnu over a line's sub-grid is 1 up to the truncated
    far wings (phi = H / (sqrt(pi) dnu_D))."""
    P = small
    for li, tr in enumerate(P.atom.lines):
        lams = np.where(P.line_index == li)[0]
        # on a fine uniform grid the normalisation is exact to the wings
        u = np.linspace(-150e3, 150e3, 20001)
        for c in (0, P.ncell // 2):
            x = u / P.vth[c]
            H = nlte.voigt_H(P.adamp[li][c], x)
            integral = np.trapezoid(H / math.sqrt(math.pi), x)
            assert abs(integral - 1) < 5e-3
        assert len(lams) > 0


def test_rates_vanish_at_lte_for_planck_field(small):
    """Kirchhoff: with LTE populations and the LTE source function in every
    direction (B at the line centre for line wavelengths, complete
    redistribution; B_nu for the continuum), every transition's
    preconditioned net rate vanishes (eta_t = chi_t S, Psi* terms cancel), so
    the statistical-equilibrium solve returns the LTE populations."""
    P = small
    pops = P.lte.copy()
    nu_eval = P.nu.copy()
    for lam, t in enumerate(P.trans_of):
        if P.atom.trans[t].kind == "line":
            nu_eval[lam] = P.atom.trans[t].nu0
    nu = nu_eval[:, None]
    B = 2 * nlte.H_PLANCK * nu ** 3 / nlte.C_LIGHT ** 2 / np.expm1(nlte.H_PLANCK * nu / (nlte.K_BOLTZ * P.T[None, :]))
    I0 = np.repeat(B[:, :, None], P.n0, axis=2)
    _, _, chi_loc, H_loc, _ = P.formal_solve(pops)
    Rup, Rdn = P.rates(pops, I0, chi_loc, H_loc)
    for t, tr in enumerate(P.atom.trans):
        lams = np.where(P.trans_of == t)[0]
        gross = np.zeros(P.ncell)
        for lam in lams:
            if tr.kind == "line":
                _, Vij, _, _ = P.line_coeffs(lam, H_loc[lam])
            else:
                _, Vic, _, _ = P.cont_coeffs(lam)
                Vij = Vic[:, None]
            gross += P.W[lam] / P.n0 * np.sum(Vij * I0[lam], axis=1) * pops[tr.i]
        net = pops[tr.i] * Rup[t] - pops[tr.j] * Rdn[t]
        assert np.max(np.abs(net) / gross) < 1e-8, t
    new, ch = P.stat_eq(pops, Rup, Rdn)
    assert ch < 1e-7


def _planck(nu, T):
    """B_nu(T) = (2 h nu^3 / c^2) / (e^{h nu / k T} - 1)."""
    return 2 * nlte.H_PLANCK * nu ** 3 / nlte.C_LIGHT ** 2 / np.expm1(nlte.H_PLANCK * nu / (nlte.K_BOLTZ * T))


def test_line_source_function_is_planck_at_lte(small):
    """Kirchhoff for the synthesised line fields: at LTE populations the
    line's emissivity over its opacity (the same profile multiplies both
    under complete redistribution) is B_nu(nu0, T) in every cell. A
    dropped g_i/g_j or a wrong population index fails this."""
    P = small
    _, _, kappa, eps = P.fields(P.lte)
    for li, tr in enumerate(P.atom.lines):
        np.testing.assert_allclose(eps[li] / kappa[li], _planck(tr.nu0, P.T), rtol=1e-10)


def test_continuum_source_function_is_planck_at_lte(small):
    """At LTE the continuum's emissivity over its opacity (stimulated
    emission included) is B_nu(nu, T) at every continuum wavelength."""
    P = small
    chi_c, eta_c, _, _ = P.fields(P.lte)
    for lam, t in enumerate(P.trans_of):
        if P.atom.trans[t].kind == "cont":
            assert np.all(chi_c[lam] > 0)
            np.testing.assert_allclose(eta_c[lam] / chi_c[lam], _planck(P.nu[lam], P.T), rtol=1e-10)


def test_thick_isothermal_atmosphere_has_planck_mean_intensity():
    """A homogeneous isothermal atmosphere at rest at LTE populations, dense
    enough that every cell is optically thick at the Lyman-alpha core and
    across the Lyman continuum: the formal solution gives J = B_nu(T) (at
    the line's rest frequency for line wavelengths) wherever the medium is
    thick, the cells more than 8 cells from the edge."""
    n = 32
    inp = W.nlte_atmosphere(n, seed=9, n_line=16, n_cont=8)
    T = np.full((n, n), 6000.0)
    ntot = np.full((n, n), 5e19)
    inp = W.NlteInput(T, 0.2 * ntot, ntot, np.zeros((2, n, n), np.float32), inp.lambda_nm, inp.trans, inp.dnu,
                      inp.voxel, inp.atom, "isothermal")
    P = nlte.Problem(inp)
    chi_c, _, kappa, _ = P.fields(P.lte)
    J = P.formal_solve(P.lte)[0]
    inner = np.zeros((n, n), bool)
    inner[8:-8, 8:-8] = True
    inner = inner.ravel()
    checked = 0
    for lam, t in enumerate(P.trans_of):
        tr = P.atom.trans[t]
        if tr.kind == "line":
            li = P.line_index[lam]
            H = nlte.voigt_H(P.adamp[li], np.abs(P.u[lam]) / P.vth)
            tau_cell = kappa[li] * H * inp.voxel
            B = _planck(tr.nu0, P.T)
        else:
            tau_cell = chi_c[lam] * inp.voxel
            B = _planck(P.nu[lam], P.T)
        if tau_cell.min() < 5.0:
            continue
        checked += 1
        np.testing.assert_allclose(J[lam][inner], B[inner], rtol=1e-10)
    # the Lyman-alpha core and every Lyman-continuum wavelength are checked
    assert checked >= 8 + 2


def test_inclined_static_atmosphere_matches_the_inclined_formal_solve():
    """2D invariance in the non-LTE oracle (Sec. 3.1): in an atmosphere at
    rest the fields are isotropic, so its J with 3 inclinations equals the
    formal-solve oracle's inclined solve (a separate code path: isotropic
    chi and eta arrays, the path scaled through the voxel size) of the same
    fields, wavelength by wavelength."""
    inp = W.nlte_atmosphere(24, seed=7, n_line=12, n_cont=8)
    inp.vel[...] = 0.0
    P = nlte.Problem(inp, n_incl=3)
    J = P.formal_solve(P.lte)[0]
    chi_c, eta_c, kappa, eps = P.fields(P.lte)
    chi = chi_c.copy()
    eta = eta_c.copy()
    for lam in range(len(P.nu)):
        li = P.line_index[lam]
        if li >= 0:
            H = nlte.voigt_H(P.adamp[li], np.abs(P.u[lam]) / P.vth)
            chi[lam] += kappa[li] * H
            eta[lam] += eps[li] * H
    ref = oracle.formal_solve_inclined(chi.reshape(-1, 24, 24), eta.reshape(-1, 24, 24), P.n_casc, 3,
                                       voxel=inp.voxel).reshape(len(P.nu), -1)
    np.testing.assert_allclose(J, ref, rtol=1e-11)


def test_inclined_rays_are_flatland_rays_with_projected_velocity_and_longer_paths():
    """Inclination m of the non-LTE oracle equals the flatland problem whose
    cells are 1/sin(theta_m) longer and whose velocities are sin(theta_m)
    times the in-plane ones: the cascade-0 radiances, the local opacities and
    profiles, and the rates summed with the Gauss-Radau weights."""
    inp = W.nlte_atmosphere(16, seed=8, n_line=12, n_cont=8)
    P = nlte.Problem(inp, n_incl=3)
    J, I0, chi_loc, H_loc, _ = P.formal_solve(P.lte)
    Rup, Rdn = P.rates(P.lte, I0, chi_loc, H_loc)
    mu, w = oracle.radau_inclinations(3)
    Jsum = np.zeros_like(J)
    Usum = np.zeros_like(Rup)
    Dsum = np.zeros_like(Rdn)
    for m in range(3):
        sm = math.sqrt(1.0 - mu[m] ** 2)
        q = W.NlteInput(inp.T, inp.ne, inp.ntot, (inp.vel.astype(np.float64) * sm).astype(np.float32),
                        inp.lambda_nm, inp.trans, inp.dnu, inp.voxel / sm, inp.atom, "scaled")
        Q = nlte.Problem(q)
        # the velocity is rounded to FP32 again after scaling: compare the
        # opacities at the precision that leaves
        Jm, I0m, chim, Hm, _ = Q.formal_solve(Q.lte)
        np.testing.assert_allclose(I0[m], I0m, rtol=1e-6)
        np.testing.assert_allclose(chi_loc[m], chim, rtol=1e-6)
        u, d = Q.rates(Q.lte, I0m, chim, Hm)
        Jsum += w[m] * Jm
        Usum += w[m] * u
        Dsum += w[m] * d
    np.testing.assert_allclose(J, Jsum, rtol=1e-6)
    np.testing.assert_allclose(Rup, Usum, rtol=1e-5, atol=1e-6 * np.abs(Rup).max())
    np.testing.assert_allclose(Rdn, Dsum, rtol=1e-5, atol=1e-6 * np.abs(Rdn).max())


def test_thick_isothermal_atmosphere_with_inclinations_has_planck_mean_intensity():
    """J = B_nu(T) deep in a thick isothermal atmosphere for any quadrature
    of inclinations (every inclined ray sees the same source function)."""
    n = 24
    base = W.nlte_atmosphere(n, seed=9, n_line=12, n_cont=8)
    T = np.full((n, n), 6000.0)
    ntot = np.full((n, n), 5e19)
    inp = W.NlteInput(T, 0.2 * ntot, ntot, np.zeros((2, n, n), np.float32), base.lambda_nm, base.trans, base.dnu,
                      base.voxel, base.atom, "isothermal")
    P = nlte.Problem(inp, n_incl=8)
    chi_c, _, _, _ = P.fields(P.lte)
    J = P.formal_solve(P.lte)[0]
    inner = np.zeros((n, n), bool)
    inner[6:-6, 6:-6] = True
    inner = inner.ravel()
    for lam, t in enumerate(P.trans_of):
        tr = P.atom.trans[t]
        if tr.kind == "cont":
            np.testing.assert_allclose(J[lam][inner], _planck(P.nu[lam], P.T)[inner], rtol=1e-10)


def test_collision_dominated_limit_is_lte():
    """Collisions far above radiative rates force Saha-Boltzmann populations."""
    d = dict(W.SYNTH_ATOM)
    d["q_coll"] = [q * 1e12 for q in W.SYNTH_ATOM["q_coll"]]
    inp = W.nlte_atmosphere(16, seed=6, n_line=16, n_cont=8)
    inp.atom = d
    P = nlte.Problem(inp)
    pops, changes = P.iterate(P.lte.copy(), 3)
    np.testing.assert_allclose(pops, P.lte, rtol=1e-6)


def test_gamma_columns_sum_to_zero_and_solution_unique(small):
    P = small
    pops = P.lte.copy()
    J, I0, chi_loc, H_loc, _ = P.formal_solve(pops)
    Rup, Rdn = P.rates(pops, I0, chi_loc, H_loc)
    G = P.gamma(Rup, Rdn)
    colsum = np.abs(G.sum(axis=1)).max(axis=1) / np.abs(G).max(axis=(1, 2))
    assert colsum.max() < 1e-13
    new, _ = P.stat_eq(pops, Rup, Rdn)
    np.testing.assert_allclose(new.sum(axis=0), P.ntot, rtol=1e-12)
    # The solution of Gamma n = 0, sum n = ntot does not depend on which
    # equation the conservation row replaces: check against the
    # least-squares solution of the full over-determined system.
    for c in range(0, P.ncell, 37):
        A = np.vstack([G[c], np.ones(P.atom.n_levels)])
        b = np.zeros(P.atom.n_levels + 1)
        b[-1] = P.ntot[c]
        sol, *_ = np.linalg.lstsq(A, b, rcond=None)
        np.testing.assert_allclose(new[:, c], sol, rtol=1e-8, atol=1e-12 * P.ntot[c])


def test_cascade0_operator_is_derivative_of_march():
    """Psi*(k) = (1 - e^{-chi l_k}) / chi equals dI_0(k)/d eta of the cell
    itself, l_k the distance from the cell centre to its edge along w_k (one
    cascade, so no other interval passes the cell)."""
    rng = np.random.default_rng(2)
    n = 9
    chi = 10 ** rng.uniform(-2, 1.5, (1, n, n))
    eta = chi * rng.uniform(0.5, 2.0, (1, n, n))
    c = (4, 5)
    base = oracle.formal_solve(chi, eta, 1, want_I0=True)["I0"][0, c[0], c[1]]
    h = 1e-3 * eta[0, c[0], c[1]]
    eta2 = eta.copy()
    eta2[0, c[0], c[1]] += h
    pert = oracle.formal_solve(chi, eta2, 1, want_I0=True)["I0"][0, c[0], c[1]]
    fd = (pert - base) / h
    ell = math.sqrt(0.5)
    psi = -math.expm1(-chi[0, c[0], c[1]] * ell) / chi[0, c[0], c[1]]
    np.testing.assert_allclose(fd, psi, rtol=1e-7)


def test_fixed_point_balances_unpreconditioned_rates():
    """At convergence the preconditioning terms cancel: the plain rates
    (I, no Psi*) balance the populations to about the stopping tolerance."""
    inp = W.nlte_atmosphere(16, seed=5, n_line=24, n_cont=8)
    P = nlte.Problem(inp)
    pops, changes = P.iterate(P.lte.copy(), 200, tol=1e-9)
    assert changes[-1] < 1e-9
    J, I0, chi_loc, H_loc, _ = P.formal_solve(pops)
    nt = len(P.atom.trans)
    Rup = np.zeros((nt, P.ncell))
    Rdn = np.zeros((nt, P.ncell))
    for lam in range(len(P.nu)):
        t = P.trans_of[lam]
        tr = P.atom.trans[t]
        if tr.kind == "line":
            _, Vij, Vji, Uji = P.line_coeffs(lam, H_loc[lam])
        else:
            _, Vic, Vci, Uci = P.cont_coeffs(lam)
            Vij, Vji, Uji = Vic[:, None], Vci[:, None], Uci[:, None]
        Rup[t] += P.W[lam] / P.n0 * np.sum(Vij * I0[lam], axis=1)
        Rdn[t] += P.W[lam] / P.n0 * np.sum(Uji + Vji * I0[lam], axis=1)
    G = P.gamma(Rup, Rdn)
    res = np.einsum("cij,jc->ic", G, pops)
    scale = np.einsum("cij,jc->ic", np.abs(G), pops)
    assert np.max(np.abs(res) / scale) < 1e-6


@pytest.mark.parametrize("M,rates", [(1, (0.9,)), (2, (0.93, 0.6)), (3, (0.95, 0.7, -0.4))])
def test_ng_extrapolation_recovers_fixed_point_of_linear_iteration(M, rates):
    """Ng of order M is exact when the error of the iterates spans M
    geometric modes, x_k = x* + sum_m a_m r_m^k (minimal-polynomial
    extrapolation): from the M + 2 newest iterates it returns x*."""
    from oracle.nlte import ng_extrapolate
    rng = np.random.default_rng(M)
    xstar = rng.uniform(1.0, 2.0, (3, 40))
    modes = [rng.normal(0.0, 0.05, xstar.shape) for _ in rates]
    xs = [xstar + sum(a * r ** k for a, r in zip(modes, rates)) for k in range(6, 6 + M + 2)]
    got = ng_extrapolate(xs[::-1], M)
    np.testing.assert_allclose(got, xstar, rtol=1e-9, atol=0)


def test_ng_extrapolation_of_converged_iterates_is_identity():
    """Iterates that no longer change give a singular system: no step."""
    from oracle.nlte import ng_extrapolate
    x = np.full((2, 5), 1.5)
    assert ng_extrapolate([x, x, x, x], 2) is None


# ------------------------------------------------------ charge conservation


def test_charge_conservation_collisional_limit_is_saha():
    """Sec. 3.3 (charge conservation by a Newton-Raphson step, also used for
    a self-consistent starting n_e from the collisional rates alone): with
    the radiative rates switched off the equilibrium is LTE at the current
    n_e, and repeated steps drive n_e to the Saha solution of a plasma whose
    only electron donor is this atom, n_e^2 = Phi (n_tot - n_e) / U, with
    Phi = n_c n_e / n_1 from the Saha equation and U the bound partition
    function relative to the ground level; the convergence is quadratic, as
    a Newton step with the right derivative must be."""
    from oracle.nlte import H_PLANCK, K_BOLTZ, M_ELEC
    inp = W.nlte_atmosphere(8, seed=3, n_line=8, n_cont=4)
    P = nlte.Problem(inp)
    A = P.atom
    kT = K_BOLTZ * P.T
    cl = A.n_levels - 1
    U = sum(A.g[l] / A.g[0] * np.exp(-(A.E[l] - A.E[0]) / kT) for l in range(cl))
    Phi = A.g[cl] / A.g[0] * 2.0 * (2.0 * np.pi * M_ELEC * kT / H_PLANCK ** 2) ** 1.5 * np.exp(-(A.E[cl] - A.E[0]) / kT)
    Pp = Phi / U
    ne_true = 0.5 * (-Pp + np.sqrt(Pp * Pp + 4.0 * Pp * P.ntot))
    zero = np.zeros((len(A.trans), P.ncell))
    Q = P.with_ne(1.3 * ne_true)
    pops = Q.lte
    errs = []
    for _ in range(7):
        pops, _ = Q.stat_eq(pops, zero, zero)
        pops, ne = Q.charge_step(pops, zero, zero)
        Q = P.with_ne(ne)
        errs.append(float(np.max(np.abs(ne / ne_true - 1.0))))
    assert errs[-1] < 1e-12, errs
    k = next(i for i, e in enumerate(errs) if e < 1e-3)
    assert errs[k + 1] < 10 * errs[k] ** 2 + 1e-14, errs       # quadratic
    np.testing.assert_allclose(pops[cl], ne_true, rtol=1e-10)
    pops_eq, _ = Q.stat_eq(pops, zero, zero)
    np.testing.assert_allclose(pops_eq, Q.lte, rtol=1e-10)


def test_charge_step_at_a_solution_is_zero():
    """At populations in equilibrium with n_e = n_c the Newton-Raphson step
    changes nothing."""
    inp = W.nlte_atmosphere(8, seed=3, n_line=8, n_cont=4)
    P = nlte.Problem(inp)
    zero = np.zeros((len(P.atom.trans), P.ncell))
    Q = P.with_ne(P.ne)
    pops = Q.lte
    for _ in range(8):
        pops, _ = Q.stat_eq(pops, zero, zero)
        pops, ne = Q.charge_step(pops, zero, zero)
        Q = P.with_ne(ne)
    pops, _ = Q.stat_eq(pops, zero, zero)
    new, ne2 = Q.charge_step(pops, zero, zero)
    np.testing.assert_allclose(new, pops, rtol=1e-12)
    np.testing.assert_allclose(ne2, Q.ne, rtol=1e-12)


def test_charge_conserving_iteration_converges_with_n_e_equal_n_c():
    """The full iteration with charge conservation (radiation on) converges
    to populations with n_e = n_c in every cell, in a number of iterations
    comparable to the iteration at fixed n_e."""
    inp = W.nlte_atmosphere(16, seed=3, n_line=16, n_cont=8)
    P = nlte.Problem(inp)
    _, plain = P.iterate(P.lte.copy(), 200, tol=1e-3)
    pops, ch = P.iterate(P.lte.copy(), 200, tol=1e-3, charge=True)
    cl = P.atom.n_levels - 1
    assert ch[-1] < 1e-3 and len(ch) < 3 * len(plain)
    np.testing.assert_allclose(P.last_ne, pops[cl], rtol=5e-3)


def test_collisional_starting_n_e_is_saha():
    """Sec. 3.3: the starting n_e from the collisional rates alone is the
    Saha n_e of the pure plasma (the same closed form as above)."""
    from oracle.nlte import H_PLANCK, K_BOLTZ, M_ELEC
    inp = W.nlte_atmosphere(8, seed=4, n_line=8, n_cont=4)
    P = nlte.Problem(inp)
    A = P.atom
    kT = K_BOLTZ * P.T
    cl = A.n_levels - 1
    U = sum(A.g[l] / A.g[0] * np.exp(-(A.E[l] - A.E[0]) / kT) for l in range(cl))
    Pp = A.g[cl] / A.g[0] * 2.0 * (2.0 * np.pi * M_ELEC * kT / H_PLANCK ** 2) ** 1.5 \
        * np.exp(-(A.E[cl] - A.E[0]) / kT) / U
    ne_true = 0.5 * (-Pp + np.sqrt(Pp * Pp + 4.0 * Pp * P.ntot))
    Q = P.collisional_ne(20)
    np.testing.assert_allclose(Q.ne, ne_true, rtol=1e-10)


def test_pressure_conservation_holds_the_starting_pressure():
    """Sec. 3.3 (pressure conservation, with charge conservation): every
    iteration leaves n_Htot + n_e at its starting value (A_tot = 1) and the
    iteration converges; with radiation off its fixed point is the Saha
    solution under that pressure, n_e = -Phi' + sqrt(Phi'^2 + Phi' P/kT)."""
    from oracle.nlte import H_PLANCK, K_BOLTZ, M_ELEC
    inp = W.nlte_atmosphere(16, seed=3, n_line=16, n_cont=8)
    P = nlte.Problem(inp)
    p_kt = P.ntot + P.ne
    pops, ch = P.iterate(P.lte.copy(), 200, tol=1e-3, charge=True, pressure=True)
    assert ch[-1] < 1e-3
    np.testing.assert_allclose(P.last_ntot + P.last_ne, p_kt, rtol=1e-12)
    np.testing.assert_allclose(pops.sum(axis=0), P.last_ntot, rtol=1e-9)
    # collisional limit under constant pressure
    A = P.atom
    kT = K_BOLTZ * P.T
    cl = A.n_levels - 1
    U = sum(A.g[l] / A.g[0] * np.exp(-(A.E[l] - A.E[0]) / kT) for l in range(cl))
    Pp = A.g[cl] / A.g[0] * 2.0 * (2.0 * np.pi * M_ELEC * kT / H_PLANCK ** 2) ** 1.5 \
        * np.exp(-(A.E[cl] - A.E[0]) / kT) / U
    ne_true = -Pp + np.sqrt(Pp * Pp + Pp * p_kt)
    zero = np.zeros((len(A.trans), P.ncell))
    Q = P
    pops = Q.lte
    for _ in range(30):
        pops, _ = Q.stat_eq(pops, zero, zero)
        pops, ne = Q.charge_step(pops, zero, zero)
        nt = p_kt - ne
        pops = pops * (nt / Q.ntot)[None, :]
        Q = P.with_ne(ne, nt)
    np.testing.assert_allclose(Q.ne, ne_true, rtol=1e-9)


# ------------------------------------------------------------ sparsity


def test_sparse_nlte_cut_above_every_cell_is_dense():
    """Sec. 3.5: a temperature cut above every cell flags everything."""
    inp = W.nlte_atmosphere(16, seed=3, n_line=8, n_cont=4)
    P, Ps = nlte.Problem(inp), nlte.Problem(inp, t_cut=2.5e5)
    a, _ = P.iterate(P.lte.copy(), 3)
    b, _ = Ps.iterate(Ps.lte.copy(), 3)
    np.testing.assert_array_equal(a, b)


def test_sparse_nlte_ignores_coronal_cells():
    """Sec. 3.5: with a 250 kK cut the coronal cells are transparent, empty
    and held: the flagged cells' populations after a few iterations do not
    depend on the corona's temperature or density, and the coronal
    populations stay at their starting values."""
    import dataclasses
    inp = W.nlte_atmosphere(48, seed=3, n_line=8, n_cont=4, corona_frac=0.6)
    hot = inp.T >= 2.5e5
    assert 0.5 < hot.mean() < 0.7
    inp2 = dataclasses.replace(inp, T=np.where(hot, 3e6, inp.T), ntot=np.where(hot, 7.0 * inp.ntot, inp.ntot))
    P, P2 = nlte.Problem(inp, t_cut=2.5e5), nlte.Problem(inp2, t_cut=2.5e5)
    a, ch = P.iterate(P.lte.copy(), 4)
    b, _ = P2.iterate(P2.lte.copy(), 4)
    act = ~hot.reshape(-1)
    np.testing.assert_allclose(a[:, act], b[:, act], rtol=1e-12)
    np.testing.assert_array_equal(a[:, ~act], P.lte[:, ~act])


# -------------------------------------------------------- emergent spectra


def test_nlte_emergent_without_lines_is_the_given_fields_solver():
    """Sec. 3.9: at continuum wavelengths the non-LTE emergent intensity is
    the given-fields beam solver's on the synthesised continuum opacity and
    emissivity (the two share only the ray layout)."""
    inp = W.nlte_atmosphere(24, seed=3, n_line=8, n_cont=4)
    P = nlte.Problem(inp)
    chi_c, eta_c, _, _ = P.fields(P.lte)
    I = P.emergent(P.lte, 0.6, -0.8, 40)
    cont = np.nonzero(P.line_index < 0)[0]
    ref = oracle.emergent(chi_c[cont].reshape(-1, 24, 24), eta_c[cont].reshape(-1, 24, 24), 0.6, -0.8, 40,
                          voxel=inp.voxel)
    np.testing.assert_allclose(I[cont], ref, rtol=1e-12, atol=0)


def test_nlte_emergent_line_follows_the_flow():
    """Sec. 3.9 with Sec. 3.2's Doppler shifts: a uniform flow of 20 km/s
    along +x shifts the emergent line to the blue for an observer on the +x
    side and to the red for one on the -x side (the intensity-weighted
    velocity centroid of the line against the same atmosphere at rest; on
    the coarse, non-uniform wavelength grid the centroid moves by 0.4-1 x
    the flow speed, so the bound is loose and the sign is the pin)."""
    import dataclasses
    inp = W.nlte_atmosphere(24, seed=3, n_line=32, n_cont=4)
    v0 = 20e3
    still = dataclasses.replace(inp, vel=np.zeros_like(inp.vel))
    vel = np.zeros_like(inp.vel)
    vel[0] = v0
    flow = dataclasses.replace(inp, vel=vel)
    P0, P1 = nlte.Problem(still), nlte.Problem(flow)
    line0 = np.nonzero(P0.line_index == 0)[0]
    u = P0.u[line0]

    def centroid(P, wx):
        I = P.emergent(P0.lte, wx, 0.0, 24)[line0].mean(axis=1)
        e = I - I.min()
        return float(np.sum(u * e) / np.sum(e))

    for wx, sign in ((1.0, 1.0), (-1.0, -1.0)):
        shift = centroid(P1, wx) - centroid(P0, wx)
        assert 0.2 * v0 < sign * shift < 1.5 * v0, (wx, shift)
