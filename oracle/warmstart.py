"""FP64 CPU oracle of the learned warm start's data transforms: the per-cell
features the network reads, its targets (log departure coefficients), and
the populations rebuilt from a prediction. These belong to the learned
warm-start growth pattern of the non-LTE iteration (Sec. 3.3); the paper
fixes none of them, so they follow the definitions stated here.

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path;
shares no code with the HIP library.

Definitions, per cell c (the Problem's atmosphere and atom):
  f0 = log10 T
  f1 = log10 n_e
  f2 = |v| in km/s (the in-plane velocity's length)
  f3 = log10 kappa_0, kappa_0 = sigma_0 (n_i - (g_i/g_j) n_j) / (sqrt(pi) dnu_D)
       the opacity of line 0 per unit Voigt function [1/m] at the given
       populations (its centre opacity is kappa_0 H(a, 0))
  f4, f5 = log10 Jbar_t for lines t = 0, 1, with
       Jbar_t = sum_l H(a_t, |u_l| / v_th) dnu_l J_l / sum_l H(a_t, |u_l| / v_th) dnu_l
       over the wavelengths l of line t (u_l their velocity offsets from
       the line centre): the mean intensity weighted by the line's profile
       at rest in the cell
  targets: log10 (n_l / n_l^LTE) for every level l
  populations from a prediction y (standardised targets, norm = (means,
  stds)): b_l = 10^(y_l std_l + mean_l), n_l = ntot b_l n_l^LTE /
  sum_m b_m n_m^LTE (particle conservation restored).
"""
from __future__ import annotations

import math

import numpy as np

from . import nlte


def jbar(P: "nlte.Problem", J, line: int):
    """Profile-weighted mean intensity of line ``line`` per cell from
    J [n_wave][cells] (FP64)."""
    J = np.asarray(J, np.float64).reshape(len(P.nu), P.ncell)
    lams = np.where(P.line_index == line)[0]
    num = np.zeros(P.ncell)
    den = np.zeros(P.ncell)
    for lam in lams:
        H = nlte.voigt_H(P.adamp[line], np.abs(P.u[lam]) / P.vth)
        w = H * P.inp.dnu[lam]
        num += w * J[lam]
        den += w
    return num / den


def features(P: "nlte.Problem", pops, J):
    """Raw features [cells][6] at populations pops [levels][cells] and mean
    intensity J [n_wave][cells] (the definitions in the module notes)."""
    pops = np.asarray(pops, np.float64).reshape(P.atom.n_levels, P.ncell)
    out = np.zeros((P.ncell, 6))
    out[:, 0] = np.log10(P.T)
    out[:, 1] = np.log10(P.ne)
    out[:, 2] = np.hypot(P.vx, P.vz) * 1e-3
    tr = P.atom.lines[0]
    kappa0 = tr.sigma * (pops[tr.i] - P.atom.g[tr.i] / P.atom.g[tr.j] * pops[tr.j]) / (math.sqrt(math.pi) * P.dnuD[0])
    out[:, 3] = np.log10(kappa0)
    for t in range(2):
        out[:, 4 + t] = np.log10(jbar(P, J, t)) if t < len(P.atom.lines) else 0.0
    return out


def standardise(a, norm):
    """(a - mean) / std with norm = [means, stds] (rows of a are samples)."""
    norm = np.asarray(norm, np.float64).reshape(2, -1)
    return (np.asarray(a, np.float64) - norm[0]) / norm[1]


def log_departures(P: "nlte.Problem", pops):
    """Targets [cells][levels]: log10 (n_l / n_l^LTE)."""
    pops = np.asarray(pops, np.float64).reshape(P.atom.n_levels, P.ncell)
    return np.log10(pops / P.lte).T


def pops_from_prediction(P: "nlte.Problem", y, norm):
    """Populations [levels][cells] from standardised predicted targets
    y [cells][levels]: de-standardise, exponentiate the departure
    coefficients, scale the LTE populations and renormalise to ntot."""
    norm = np.asarray(norm, np.float64).reshape(2, -1)
    z = np.asarray(y, np.float64) * norm[1] + norm[0]
    n = P.lte * (10.0 ** z).T
    return P.ntot * n / n.sum(axis=0)
