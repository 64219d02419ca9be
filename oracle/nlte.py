"""FP64 CPU oracle of the non-LTE iteration (arXiv:2408.14425, Sec. 3.3).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's CPU
baseline, never by the product path; shares no code with the HIP library.

One iteration, in the paper's order:
  1. opacities and emissivities from the current populations (lines with
     Doppler-shifted Voigt profiles evaluated per ray step, Sec. 3.2);
  2. the radiance-cascades formal solution per wavelength (``rc_oracle.c``);
  3. at cascade 0: the diagonal operator Psi* of the piecewise-constant
     solver, the effective intensity I_eff = I - Psi* eta_t and the
     preconditioned rates of the "same-preconditioning" MALI scheme, where
     only a transition's own emissivity is treated implicitly (Sec. 3.3);
  4. the rate matrix Gamma: off-diagonal terms from radiative + collisional
     rates, the diagonal from conservation (column sums vanish), one row
     replaced by particle conservation, solved in FP64 (Sec. 3.3, 3.5);
  5. the maximum relative change of the populations (Sec. 4.2);
  6. optionally, charge conservation: one Newton-Raphson step on the
     populations and the electron density after the equilibrium step,
     hydrogen (this atom) the only electron donor (Sec. 3.3).

Readings (listed in the design notes):
  - The directional operator is Lambda* = 1 - exp(-tau), with tau the
    optical depth from the cell centre to its edge along the ray, and
    Psi* = Lambda* / chi (the printed exp(-tau) makes Psi* diverge as
    chi -> 0). Psi* is exactly dI_probe / d eta_cell of the march.
  - I_eff = I - Psi* n_j U_ji (the population factor makes it an
    emissivity); the downward coefficient is
    sum W w [V_ji I_eff + U_ji (1 - chi_t Psi*)], chi_t the transition's own
    opacity at the previous populations.
  - The conservation row replaces the equation of the most populated level.
  - Convergence: max over cells and levels of |n_new - n_old| / n_new.
  - Rate integrals: W = 4 pi dnu / (h nu) with the input frequency weights;
    flatland angular weights 1/N_0.
  - Charge conservation: unknowns (n, n_e) per cell; equations Gamma(n_e) n
    = 0 with the conservation row, and n_e = n_c (the continuum level). The
    rates proportional to n_e are the collisional downward rates, the
    bound-bound collisional upward rates (detailed balance with a Boltzmann
    ratio) and the radiative recombination rates (through n_i*/n_c*, which
    is proportional to n_e); dGamma/dn_e = (those rates) / n_e, all other
    rates held fixed. The step is taken only if it leaves every population
    and n_e positive. The change metric includes |dn_e| / n_e.
  - Pressure conservation (needs charge conservation): the gas pressure
    P = (A_tot n_Htot + n_e) k T of the starting atmosphere is held, with
    A_tot = 1 (this atom is the only species); after the charge step n_Htot
    becomes P/(kT) - n_e and every population is scaled by its ratio to the
    old n_Htot; the change metric includes |dn_Htot| / n_Htot.
  - Starting n_e from the collisional rates alone: equilibrium and charge
    steps with the radiative rates set to zero, from the given n_e.
  - Sparsity (Sec. 3.5): with a temperature cut, cells at or above it are
    not flagged: transparent with no emission in the formal solution, and
    their populations (and n_e) are held; the change metric covers the
    flagged cells. The formal solution here is the dense one of the medium
    with those cells emptied, which at flagged cells equals the sparse one.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np

from . import _dp, default_cascades, lib, make_geom, radau_inclinations

# CODATA 2018, SI
H_PLANCK = 6.62607015e-34
C_LIGHT = 2.99792458e8
K_BOLTZ = 1.380649e-23
M_ELEC = 9.1093837015e-31
Q_ELEC = 1.602176634e-19
EPS0 = 8.8541878128e-12
AMU = 1.66053906660e-27
EV = Q_ELEC


class NlteFields(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("nz", C.c_int32), ("n_wave", C.c_int32), ("n_lines", C.c_int32),
        ("line", C.c_void_p), ("u", C.c_void_p), ("chi_c", C.c_void_p), ("eta_c", C.c_void_p),
        ("kappa", C.c_void_p), ("eps", C.c_void_p), ("adamp", C.c_void_p), ("inv_vth", C.c_void_p),
        ("vx", C.c_void_p), ("vz", C.c_void_p), ("vscale", C.c_double),
    ]


def _bind():
    L = lib()
    if not hasattr(L, "_nlte_bound"):
        L.ora_voigt_H_vec.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ora_voigt_H_vec.restype = None
        L.ora_nlte_formal_solve.argtypes = [C.c_void_p, C.POINTER(NlteFields), C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_int32]
        L.ora_nlte_formal_solve.restype = C.c_int32
        L.ora_nlte_local.argtypes = [C.c_void_p, C.POINTER(NlteFields), C.c_void_p, C.c_void_p]
        L.ora_nlte_local.restype = None
        L.ora_nlte_emergent.argtypes = [C.c_void_p, C.POINTER(NlteFields), C.c_double, C.c_double, C.c_int32,
                                        C.c_void_p]
        L.ora_nlte_emergent.restype = C.c_int32
        L._nlte_bound = True
    return L


def voigt_H(a, x):
    """Voigt function H(a, x) = Re w(x + i a) (Weideman's series, FP64)."""
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), np.broadcast(a, x).shape))
    x = np.ascontiguousarray(np.broadcast_to(np.asarray(x, np.float64), a.shape))
    out = np.empty_like(a)
    _bind().ora_voigt_H_vec(a.size, a.ctypes.data, x.ctypes.data, out.ctypes.data)
    return out


# ------------------------------------------------------------------- atom


@dataclass
class Transition:
    kind: str      # "line" or "cont"
    i: int         # lower level
    j: int         # upper level
    nu0: float     # line centre or edge frequency [Hz]
    sigma: float   # line: integrated cross-section [m^2 Hz]; cont: cross-section at the edge [m^2]
    A: float       # line: spontaneous emission rate [1/s]
    q: float       # collisional de-excitation coefficient [m^3/s]


class Atom:
    """The model atom, with the line quantities of classical radiation theory:
    integrated cross-section sigma = e^2 f / (4 eps0 m_e c), Einstein
    A_ji = 2 pi e^2 nu^2 g_i f / (eps0 m_e c^3 g_j), natural damping
    Gamma = sum of A out of the upper and lower levels."""

    def __init__(self, d: dict):
        self.E = np.array(d["E_eV"], np.float64) * EV
        self.g = np.array(d["g"], np.float64)
        self.mass = d["mass_amu"] * AMU
        self.n_levels = len(self.E)
        self.trans: list[Transition] = []
        for (i, j, lam0, f), q in zip(d["lines"], d["q_coll"]):
            nu0 = C_LIGHT / (lam0 * 1e-9)
            sigma = Q_ELEC ** 2 * f / (4.0 * EPS0 * M_ELEC * C_LIGHT)
            A = 2.0 * math.pi * Q_ELEC ** 2 * nu0 ** 2 * self.g[i] * f / (EPS0 * M_ELEC * C_LIGHT ** 3 * self.g[j])
            self.trans.append(Transition("line", i, j, nu0, sigma, A, q))
        for (i, j, ledge, a0), q in zip(d["continua"], d["q_coll"][len(d["lines"]):]):
            self.trans.append(Transition("cont", i, j, C_LIGHT / (ledge * 1e-9), a0, 0.0, q))
        self.lines = [t for t in self.trans if t.kind == "line"]
        # natural damping of each line
        self.gamma = []
        for t in self.lines:
            out_up = sum(s.A for s in self.lines if s.j == t.j)
            out_lo = sum(s.A for s in self.lines if s.j == t.i)
            self.gamma.append(out_up + out_lo)


def lte_populations(atom: Atom, T, ne, ntot):
    """Saha-Boltzmann populations [n_levels][cells]: bound levels relative to
    the ground level by Boltzmann, the continuum (last level) by Saha with the
    free-electron partition factor 2 (2 pi m_e k T / h^2)^{3/2} / n_e;
    normalised to ntot."""
    T = np.asarray(T, np.float64)
    kT = K_BOLTZ * T
    rel = np.empty((atom.n_levels,) + T.shape)
    for l in range(atom.n_levels - 1):
        rel[l] = atom.g[l] / atom.g[0] * np.exp(-(atom.E[l] - atom.E[0]) / kT)
    saha = 2.0 * (2.0 * math.pi * M_ELEC * kT / H_PLANCK ** 2) ** 1.5 / ne
    c = atom.n_levels - 1
    rel[c] = atom.g[c] / atom.g[0] * saha * np.exp(-(atom.E[c] - atom.E[0]) / kT)
    return rel / rel.sum(axis=0) * ntot


# -------------------------------------------------------------- problem


def ng_extrapolate(xs, M: int):
    """Ng acceleration (Ng 1974; least-squares form of Auer 1987) from the
    iterates xs[0] (newest) .. xs[M + 1]: with d_k = x_k - x_{k+1} and
    w = 1 / x_0^2, minimise sum w (d_0 - sum_j c_j (d_0 - d_j))^2 over c and
    return (1 - sum c) x_0 + sum_j c_j x_j (None if the normal equations are
    singular)."""
    x = [np.asarray(v, dtype=np.float64).ravel() for v in xs]
    d = [x[k] - x[k + 1] for k in range(M + 1)]
    w = 1.0 / x[0] ** 2
    e = [d[0] - d[j] for j in range(1, M + 1)]
    A = np.array([[np.sum(w * e[a] * e[b]) for b in range(M)] for a in range(M)])
    b = np.array([np.sum(w * d[0] * e[a]) for a in range(M)])
    try:
        c = np.linalg.solve(A, b)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(c)):
        return None
    out = (1.0 - c.sum()) * x[0] + sum(c[j - 1] * x[j] for j in range(1, M + 1))
    return out.reshape(np.shape(xs[0]))


class Problem:
    """Static (population-independent) data of one non-LTE problem."""

    def __init__(self, inp, n_casc: int | None = None, t_cut: float | None = None, n_incl: int = 1):
        self.inp = inp
        self.atom = Atom(inp.atom)
        self.nx, self.nz = inp.nx, inp.nz
        self.ncell = inp.nx * inp.nz
        self.T = inp.T.reshape(-1).astype(np.float64)
        self.ne = inp.ne.reshape(-1).astype(np.float64)
        self.ntot = inp.ntot.reshape(-1).astype(np.float64)
        # sparsity: flagged cells (None = all)
        self.active = None if t_cut is None else self.T < t_cut
        self.vx = inp.vel[0].reshape(-1).astype(np.float64)
        self.vz = inp.vel[1].reshape(-1).astype(np.float64)
        self.nu = C_LIGHT / (inp.lambda_nm.astype(np.float64) * 1e-9)
        self.trans_of = inp.trans.astype(np.int32)
        self.W = 4.0 * math.pi * inp.dnu / (H_PLANCK * self.nu)
        self.n_casc = default_cascades(self.nx, self.nz) if n_casc is None else n_casc
        self.geom = make_geom(self.nx, self.nz, self.n_casc, voxel=inp.voxel)
        # 2D invariance (Sec. 3.1): n_incl rays per flatland ray, inclined to
        # the invariant y axis at mu = cos(theta) on the Gauss-Radau rule
        # with the in-plane node mu = 0 fixed; ray m has the flatland ray's
        # projection, a path sin(theta_m)^-1 times longer per projected cell
        # and sin(theta_m) of the in-plane velocity along it; J and the
        # rates are the weighted sums over m. n_incl = 1 is flatland.
        self.n_incl = n_incl
        mu, wmu = radau_inclinations(n_incl)
        self.incl_sin = np.sqrt(1.0 - mu ** 2)
        self.incl_w = wmu
        self.incl_geom = [make_geom(self.nx, self.nz, self.n_casc, voxel=inp.voxel / sm) for sm in self.incl_sin]
        self.n0 = 4
        self.lte = lte_populations(self.atom, self.T, self.ne, self.ntot)
        # thermal speed and line quantities per cell
        self.vth = np.sqrt(2.0 * K_BOLTZ * self.T / self.atom.mass)
        self.line_index = np.full(len(self.nu), -1, np.int32)
        self.u = np.zeros(len(self.nu))
        for lam, t in enumerate(self.trans_of):
            tr = self.atom.trans[t]
            if tr.kind == "line":
                self.line_index[lam] = self.atom.lines.index(tr)
                self.u[lam] = C_LIGHT * (self.nu[lam] - tr.nu0) / tr.nu0
        self.dnuD = [t.nu0 * self.vth / C_LIGHT for t in self.atom.lines]
        self.adamp = np.array([g / (4.0 * math.pi * d) for g, d in zip(self.atom.gamma, self.dnuD)])
        # collisional rates: down C_ji = ne q (T/1e4)^-1/2, up by detailed balance
        self.Cdown = np.array([self.ne * t.q * (self.T / 1e4) ** -0.5 for t in self.atom.trans])
        self.Cup = np.array([cd * self.lte[t.j] / self.lte[t.i] for cd, t in zip(self.Cdown, self.atom.trans)])
        # c0 directions and the distance from the cell centre to its edge along each
        self.dirs = [(math.cos(2 * math.pi * (k + 0.5) / self.n0), math.sin(2 * math.pi * (k + 0.5) / self.n0))
                     for k in range(self.n0)]
        self.ell = np.array([0.5 / max(abs(wx), abs(wz)) for wx, wz in self.dirs]) * inp.voxel

    # -- per-transition coefficients at wavelength index lam
    def cont_coeffs(self, lam: int):
        """Bound-free V_ic, V_ci, U_ci per cell: alpha (nu_edge/nu)^3, times the
        LTE ratio n_i*/n_c* and exp(-h nu / k T) for the downward terms."""
        tr = self.atom.trans[self.trans_of[lam]]
        nu = self.nu[lam]
        alpha = tr.sigma * (tr.nu0 / nu) ** 3 if nu >= tr.nu0 else 0.0
        Vic = np.full(self.ncell, alpha)
        Vci = alpha * self.lte[tr.i] / self.lte[tr.j] * np.exp(-H_PLANCK * nu / (K_BOLTZ * self.T))
        Uci = 2.0 * H_PLANCK * nu ** 3 / C_LIGHT ** 2 * Vci
        return tr, Vic, Vci, Uci

    def line_coeffs(self, lam: int, H):
        """Line V_ij, V_ji, U_ji for profile values H (same shape as cells x ...):
        phi = H / (sqrt(pi) dnu_D)."""
        li = self.line_index[lam]
        tr = self.atom.lines[li]
        phi = H / (math.sqrt(math.pi) * self.dnuD[li][:, None])
        Vij = tr.sigma * phi
        Vji = self.atom.g[tr.i] / self.atom.g[tr.j] * Vij
        Uji = 2.0 * H_PLANCK * tr.nu0 ** 3 / C_LIGHT ** 2 * Vji
        return tr, Vij, Vji, Uji

    def fields(self, pops, lams=None):
        """Opacity fields for the formal solve at populations pops [levels][cells]:
        continuum chi, eta [wavelengths][cells] of the wavelength indices lams
        (all if None), and the line opacity and emissivity per unit profile
        [lines][cells]."""
        lams = np.arange(len(self.nu)) if lams is None else np.asarray(lams)
        nw = len(lams)
        chi_c = np.zeros((nw, self.ncell))
        eta_c = np.zeros((nw, self.ncell))
        nl = len(self.atom.lines)
        kappa = np.zeros((nl, self.ncell))
        eps = np.zeros((nl, self.ncell))
        for q, lam in enumerate(lams):
            tr = self.atom.trans[self.trans_of[lam]]
            if tr.kind == "cont":
                _, Vic, Vci, Uci = self.cont_coeffs(lam)
                chi_c[q] = pops[tr.i] * Vic - pops[tr.j] * Vci
                eta_c[q] = pops[tr.j] * Uci
        for li, tr in enumerate(self.atom.lines):
            norm = tr.sigma / (math.sqrt(math.pi) * self.dnuD[li])
            gr = self.atom.g[tr.i] / self.atom.g[tr.j]
            kappa[li] = norm * (pops[tr.i] - gr * pops[tr.j])
            eps[li] = norm * gr * pops[tr.j] * 2.0 * H_PLANCK * tr.nu0 ** 3 / C_LIGHT ** 2
        if self.active is not None:
            off = ~self.active
            for a in (chi_c, eta_c, kappa, eps):
                a[:, off] = 0.0
        return chi_c, eta_c, kappa, eps

    def _cfields(self, chi_c, eta_c, kappa, eps, lams=None, vscale: float = 1.0):
        lams = np.arange(len(self.nu)) if lams is None else np.asarray(lams)
        keep = [np.ascontiguousarray(a, dtype=np.float64) for a in
                (self.u[lams], chi_c, eta_c, kappa, eps, self.adamp, 1.0 / self.vth, self.vx, self.vz)]
        line = np.ascontiguousarray(self.line_index[lams], dtype=np.int32)
        keep.append(line)
        f = NlteFields(self.nx, self.nz, len(lams), len(self.atom.lines), line.ctypes.data,
                       *[k.ctypes.data for k in keep[:9]], vscale)
        return f, keep

    def formal_solve(self, pops, lams=None, need=None):
        """J [n_wave][cells] and merged cascade-0 radiance I0 [n_wave][cells][N_0],
        plus the local directional opacity chi [n_wave][cells][N_0] and line
        profile H at each cell. lams: wavelength indices to solve (all if
        None; the outputs then cover those only); need: [cells] mask of the
        cells whose J is wanted (only their dependency cone is solved, the
        other cells' J and I0 are 0). With inclinations J is the weighted sum
        over them, and I0, chi and H carry a leading inclination axis."""
        lams = np.arange(len(self.nu)) if lams is None else np.asarray(lams)
        chi_c, eta_c, kappa, eps = self.fields(pops, lams)
        nw = len(lams)
        L = _bind()
        nm = None if need is None else np.ascontiguousarray(np.asarray(need).reshape(-1), dtype=np.uint8)
        Js, I0s, chis, Hs = [], [], [], []
        st = np.zeros(3, np.int64)
        for m in range(self.n_incl):
            f, keep = self._cfields(chi_c, eta_c, kappa, eps, lams, float(self.incl_sin[m]))
            J = np.zeros((nw, self.ncell))
            I0 = np.zeros((nw, self.ncell, self.n0))
            rc = L.ora_nlte_formal_solve(C.byref(self.incl_geom[m]), C.byref(f),
                                         None if nm is None else nm.ctypes.data, J.ctypes.data, I0.ctypes.data,
                                         st.ctypes.data, 0)
            if rc != 0:
                raise RuntimeError("ora_nlte_formal_solve failed")
            chi_loc = np.zeros((nw, self.ncell, self.n0))
            H_loc = np.zeros((nw, self.ncell, self.n0))
            L.ora_nlte_local(C.byref(self.incl_geom[m]), C.byref(f), chi_loc.ctypes.data, H_loc.ctypes.data)
            del keep
            Js.append(J)
            I0s.append(I0)
            chis.append(chi_loc)
            Hs.append(H_loc)
        if self.n_incl == 1:
            return Js[0], I0s[0], chis[0], Hs[0], st
        J = sum(w * Jm for w, Jm in zip(self.incl_w, Js))
        return J, np.array(I0s), np.array(chis), np.array(Hs), st

    def emergent(self, pops, wx: float, wz: float, n_rays: int):
        """Emergent intensity [n_wave][n_rays] at populations pops along the
        beam of parallel long characteristics of light direction (wx, wz)
        (Sec. 3.9; the ray layout of ``oracle.emergent``), line profiles
        Doppler-shifted along the rays."""
        f, keep = self._cfields(*self.fields(pops))
        I = np.zeros((len(self.nu), n_rays))
        L = _bind()
        rc = L.ora_nlte_emergent(C.byref(self.geom), C.byref(f), wx, wz, n_rays, I.ctypes.data)
        del keep
        if rc != 0:
            raise RuntimeError("ora_nlte_emergent failed")
        return I

    def _incl_parts(self, I0, chi_loc, H_loc):
        """(weight, path factor 1/sin, I0, chi, H) per inclination."""
        if self.n_incl == 1:
            return [(1.0, 1.0, I0, chi_loc, H_loc)]
        return [(self.incl_w[m], 1.0 / self.incl_sin[m], I0[m], chi_loc[m], H_loc[m]) for m in range(self.n_incl)]

    def rates(self, pops, I0, chi_loc, H_loc):
        """Preconditioned radiative rate coefficients per transition and cell:
        Rup (multiplies n_i) and Rdown (multiplies n_j); with inclinations
        the weighted sum over them, each with its longer path through the
        cell (l / sin theta) in Psi*."""
        nt = len(self.atom.trans)
        Rup = np.zeros((nt, self.ncell))
        Rdn = np.zeros((nt, self.ncell))
        for wm, pf, I0m, chim, Hm in self._incl_parts(I0, chi_loc, H_loc):
            u, d = self._rates_one(pops, I0m, chim, Hm, self.ell * pf)
            Rup += wm * u
            Rdn += wm * d
        return Rup, Rdn

    def _rates_one(self, pops, I0, chi_loc, H_loc, ell):
        nt = len(self.atom.trans)
        Rup = np.zeros((nt, self.ncell))
        Rdn = np.zeros((nt, self.ncell))
        w = 1.0 / self.n0
        for lam in range(len(self.nu)):
            t = self.trans_of[lam]
            tr = self.atom.trans[t]
            chi = chi_loc[lam]                                   # [cells][k]
            # Psi* = (1 - e^{-chi l}) / chi, and its limit l where chi = 0
            with np.errstate(invalid="ignore", divide="ignore"):
                psi = np.where(chi > 0, -np.expm1(-chi * ell[None, :]) / chi, ell[None, :])
            if tr.kind == "line":
                _, Vij, Vji, Uji = self.line_coeffs(lam, H_loc[lam])
            else:
                _, Vic, Vci, Uci = self.cont_coeffs(lam)
                Vij, Vji, Uji = Vic[:, None], Vci[:, None], Uci[:, None]
            eta_t = pops[tr.j][:, None] * Uji
            chi_t = pops[tr.i][:, None] * Vij - pops[tr.j][:, None] * Vji
            Ieff = I0[lam] - psi * eta_t
            Rup[t] += self.W[lam] * w * np.sum(Vij * Ieff, axis=1)
            Rdn[t] += self.W[lam] * w * np.sum(Vji * Ieff + Uji * (1.0 - chi_t * psi), axis=1)
        return Rup, Rdn

    def rate_magnitudes(self, pops, I0, chi_loc, H_loc):
        """The sums of ``rates`` with every term replaced by its magnitude,
        sum W w |V_ij| (|I| + |Psi* eta_t|) and
        sum W w [|V_ji| (|I| + |Psi* eta_t|) + |U_ji| (1 + |chi_t Psi*|)]: the
        scale against which rounding in the rate sums is measured (the
        preconditioned sums cancel where a cell is optically thick)."""
        nt = len(self.atom.trans)
        Aup = np.zeros((nt, self.ncell))
        Adn = np.zeros((nt, self.ncell))
        for wm, pf, I0m, chim, Hm in self._incl_parts(I0, chi_loc, H_loc):
            u, d = self._rate_magnitudes_one(pops, I0m, chim, Hm, self.ell * pf)
            Aup += wm * u
            Adn += wm * d
        return Aup, Adn

    def _rate_magnitudes_one(self, pops, I0, chi_loc, H_loc, ell):
        nt = len(self.atom.trans)
        Aup = np.zeros((nt, self.ncell))
        Adn = np.zeros((nt, self.ncell))
        w = 1.0 / self.n0
        for lam in range(len(self.nu)):
            t = self.trans_of[lam]
            tr = self.atom.trans[t]
            chi = chi_loc[lam]
            with np.errstate(invalid="ignore", divide="ignore"):
                psi = np.where(chi > 0, -np.expm1(-chi * ell[None, :]) / chi, ell[None, :])
            if tr.kind == "line":
                _, Vij, Vji, Uji = self.line_coeffs(lam, H_loc[lam])
            else:
                _, Vic, Vci, Uci = self.cont_coeffs(lam)
                Vij, Vji, Uji = Vic[:, None], Vci[:, None], Uci[:, None]
            eta_t = pops[tr.j][:, None] * Uji
            chi_t = pops[tr.i][:, None] * Vij - pops[tr.j][:, None] * Vji
            mag = np.abs(I0[lam]) + np.abs(psi * eta_t)
            Aup[t] += self.W[lam] * w * np.sum(np.abs(Vij) * mag, axis=1)
            Adn[t] += self.W[lam] * w * np.sum(np.abs(Vji) * mag + np.abs(Uji) * (1.0 + np.abs(chi_t * psi)), axis=1)
        return Aup, Adn

    def gamma(self, Rup, Rdn):
        """Rate matrix [cells][levels][levels]: Gamma[j][i] = rate i -> j
        (i != j), diagonal = minus the column sum (conservation)."""
        nlv = self.atom.n_levels
        G = np.zeros((self.ncell, nlv, nlv))
        for t, tr in enumerate(self.atom.trans):
            G[:, tr.j, tr.i] += Rup[t] + self.Cup[t]
            G[:, tr.i, tr.j] += Rdn[t] + self.Cdown[t]
        for l in range(nlv):
            G[:, l, l] = -(G.sum(axis=1)[:, l] - G[:, l, l])
        return G

    def at_cells(self, idx):
        """The cell-local part of the problem restricted to the cells idx
        (the rates, the rate matrix and the equilibrium solve of those cells
        only; no formal solve on the result)."""
        import copy
        idx = np.asarray(idx)
        P = copy.copy(self)
        P.ncell = len(idx)
        for name in ("T", "ne", "ntot", "vx", "vz", "vth"):
            setattr(P, name, getattr(self, name)[idx].copy())
        P.lte = self.lte[:, idx].copy()
        P.Cdown = self.Cdown[:, idx].copy()
        P.Cup = self.Cup[:, idx].copy()
        P.dnuD = [d[idx].copy() for d in self.dnuD]
        P.adamp = self.adamp[:, idx].copy()
        P.active = None if self.active is None else self.active[idx].copy()
        P.geom = None
        return P

    def with_ne(self, ne, ntot=None):
        """A copy of the problem at electron density ne (and hydrogen
        density ntot): the LTE populations, collisional rates and continuum
        coefficients follow them."""
        import copy
        P = copy.copy(self)
        P.ne = np.asarray(ne, np.float64).copy()
        if ntot is not None:
            P.ntot = np.asarray(ntot, np.float64).copy()
        P.lte = lte_populations(self.atom, self.T, P.ne, P.ntot)
        P.Cdown = np.array([P.ne * t.q * (P.T / 1e4) ** -0.5 for t in self.atom.trans])
        P.Cup = np.array([cd * P.lte[t.j] / P.lte[t.i] for cd, t in zip(P.Cdown, self.atom.trans)])
        return P

    def charge_step(self, pops, Rup, Rdn):
        """One Newton-Raphson step for charge conservation at the populations
        of the equilibrium step (readings in the module notes). Returns the
        new populations, n_e and the max relative change of both."""
        G = self.gamma(Rup, Rdn)
        nlv = self.atom.n_levels
        cl = nlv - 1
        nc = self.ncell
        ne = self.ne
        # dGamma/dn_e applied to the populations
        D = np.zeros((nc, nlv))
        for t, tr in enumerate(self.atom.trans):
            up = self.Cup[t] if tr.kind == "line" else np.zeros(nc)
            dn = self.Cdown[t] + (Rdn[t] if tr.kind == "cont" else 0.0)
            D[:, tr.j] += up / ne * pops[tr.i]
            D[:, tr.i] -= up / ne * pops[tr.i]
            D[:, tr.i] += dn / ne * pops[tr.j]
            D[:, tr.j] -= dn / ne * pops[tr.j]
        M = np.zeros((nc, nlv + 1, nlv + 1))
        rhs = np.zeros((nc, nlv + 1))
        M[:, :nlv, :nlv] = G
        M[:, :nlv, nlv] = D
        rhs[:, :nlv] = -np.einsum("clm,mc->cl", G, pops)
        r = np.argmax(pops, axis=0)
        idx = np.arange(nc)
        M[idx, r, :] = 0.0
        M[idx, r, :nlv] = 1.0
        rhs[idx, r] = self.ntot - pops.sum(axis=0)
        M[:, nlv, cl] = -1.0
        M[:, nlv, nlv] = 1.0
        rhs[:, nlv] = pops[cl] - ne
        d = np.linalg.solve(M, rhs[..., None])[..., 0]
        new = pops + d[:, :nlv].T
        ne_new = ne + d[:, nlv]
        ok = np.all(new > 0, axis=0) & (ne_new > 0)
        if self.active is not None:
            ok &= self.active
        new = np.where(ok[None, :], new, pops)
        ne_new = np.where(ok, ne_new, ne)
        return new, ne_new

    def stat_eq(self, pops, Rup, Rdn):
        """Solve Gamma n = 0 with the most populated level's row replaced by
        sum(n) = ntot. Returns new populations and max |dn| / n_new."""
        G = self.gamma(Rup, Rdn)
        nlv = self.atom.n_levels
        r = np.argmax(pops, axis=0)
        A = G.copy()
        b = np.zeros((self.ncell, nlv))
        A[np.arange(self.ncell), r, :] = 1.0
        b[np.arange(self.ncell), r] = self.ntot
        new = np.linalg.solve(A, b[..., None])[..., 0].T
        if self.active is not None:
            new[:, ~self.active] = pops[:, ~self.active]
        change = float(np.max(np.abs(new - pops) / np.abs(new)))
        return new, change

    def collisional_ne(self, n_iter: int = 20):
        """Starting n_e from the collisional rates alone (radiative rates
        zero): n_iter equilibrium + charge steps from the given n_e, LTE
        start. Returns the problem at that n_e."""
        zero = np.zeros((len(self.atom.trans), self.ncell))
        P = self
        pops = P.lte
        for _ in range(n_iter):
            pops, _ = P.stat_eq(pops, zero, zero)
            pops, ne = P.charge_step(pops, zero, zero)
            P = self.with_ne(ne)
        return P

    def iterate(self, pops, n_iter: int, tol: float | None = None, ng: tuple | None = None,
                charge: bool = False, pressure: bool = False):
        """The iteration of Sec. 3.3: formal solution with rates, then the
        equilibrium step. Stops after n_iter iterations or once the max
        relative change drops below tol. ng = (order M, delay, period) adds Ng
        acceleration after the equilibrium step (not used by the paper).
        charge: one Newton-Raphson charge-conservation step after each
        equilibrium step, n_e carried from iteration to iteration (the final
        n_e is left in ``self.last_ne``); pressure (with charge): n_Htot
        rescaled to hold the starting pressure after each charge step (the
        final n_Htot in ``self.last_ntot``)."""
        changes = []
        hist = []  # newest last
        P = self
        p_kt = self.ntot + self.ne  # P / (k T), A_tot = 1
        for it in range(1, n_iter + 1):
            J, I0, chi_loc, H_loc, _ = P.formal_solve(pops)
            Rup, Rdn = P.rates(pops, I0, chi_loc, H_loc)
            old = pops
            pops, ch = P.stat_eq(pops, Rup, Rdn)
            if charge:
                pops, ne_new = P.charge_step(pops, Rup, Rdn)
                nt_new = P.ntot
                if pressure:
                    nt_new = p_kt - ne_new
                    ok = nt_new > 0
                    nt_new = np.where(ok, nt_new, P.ntot)
                    pops = pops * (nt_new / P.ntot)[None, :]
                ch = max(float(np.max(np.abs(pops - old) / np.abs(pops))),
                         float(np.max(np.abs(ne_new - P.ne) / ne_new)),
                         float(np.max(np.abs(nt_new - P.ntot) / nt_new)))
                P = self.with_ne(ne_new, nt_new)
                self.last_ne = P.ne
                self.last_ntot = P.ntot
            changes.append(ch)
            if tol is not None and ch < tol:
                break
            if ng is not None and ng[0] > 0:
                M, delay, period = ng
                hist = (hist + [pops.copy()])[-(M + 2):]
                if len(hist) == M + 2 and it >= delay and (it - delay) % period == 0:
                    acc = ng_extrapolate(hist[::-1], M)
                    if acc is not None:
                        pops = acc
                        hist = [pops.copy()]
        return pops, changes
