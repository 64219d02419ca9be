"""Pins of the FP64 oracle of the warm start's data transforms (features,
targets, populations from a prediction; no GPU) against identities that
fix each of them independently of the oracle's own code: a profile-weighted
mean of a constant is that constant, the weights against scipy's Faddeeva
function, the line opacity against its textbook form at LTE, LTE departure
coefficients of one, and the round trip populations -> targets ->
populations. A wrong line index, a dropped g_i/g_j, a transposed
[cells][levels] layout or a missing renormalisation fails one of them."""
import math

import numpy as np
import pytest
from scipy.special import wofz

from oracle import nlte
from oracle import warmstart as WSO
from paper_2408_14425_amd import workloads as W


@pytest.fixture(scope="module")
def small():
    inp = W.nlte_atmosphere(16, seed=5, n_line=24, n_cont=8)
    return nlte.Problem(inp)


def test_jbar_of_constant_is_the_constant(small):
    """A weighted mean of a constant is that constant; line t reads only its
    own wavelengths (J = t + 1 on line t's wavelengths, 100 elsewhere)."""
    P = small
    J = np.full((len(P.nu), P.ncell), 100.0)
    cell_scale = np.linspace(0.5, 3.0, P.ncell)
    for t in range(2):
        J[P.line_index == t] = (t + 1.0) * cell_scale
    f = WSO.features(P, P.lte, J)
    np.testing.assert_allclose(f[:, 4], np.log10(cell_scale), rtol=0, atol=1e-14)
    np.testing.assert_allclose(f[:, 5], np.log10(2.0 * cell_scale), rtol=0, atol=1e-14)


def test_jbar_weights_follow_the_voigt_profile(small):
    """J = 1 on one wavelength of line 0 and 0 elsewhere: Jbar is that
    wavelength's profile weight H(a, |u|/v_th) dnu over the sum of all of
    them, with H from scipy's Faddeeva function (not the oracle's)."""
    P = small
    lams = np.where(P.line_index == 0)[0]
    pick = lams[len(lams) // 2 - 3]
    J = np.zeros((len(P.nu), P.ncell))
    J[pick] = 1.0
    got = WSO.jbar(P, J, 0)
    a = P.adamp[0]
    H = np.array([wofz(np.abs(P.u[l]) / P.vth + 1j * a).real for l in lams])  # [lams][cells]
    w = H * P.inp.dnu[lams][:, None]
    ref = w[list(lams).index(pick)] / w.sum(axis=0)
    np.testing.assert_allclose(got, ref, rtol=1e-6)


def test_kappa_feature_is_the_textbook_line_opacity_at_lte(small):
    """At LTE the lower-minus-stimulated population factor is
    n_i (1 - e^{-h nu0 / k T}) (Boltzmann with the level energies of the
    line), so kappa_0 = (e^2 / (4 eps0 m_e c)) f n_i (1 - e^{-h nu0/kT}) /
    (sqrt(pi) nu0 v_th / c), v_th = sqrt(2 k T / m)."""
    P = small
    f = WSO.features(P, P.lte, np.ones((len(P.nu), P.ncell)))
    tr = W.SYNTH_ATOM["lines"][0]
    lam0 = tr[2] * 1e-9
    nu0 = nlte.C_LIGHT / lam0
    e, eps0, me, c, h, k = (nlte.Q_ELEC, nlte.EPS0, nlte.M_ELEC, nlte.C_LIGHT, nlte.H_PLANCK, nlte.K_BOLTZ)
    vth = np.sqrt(2 * k * P.T / (W.SYNTH_ATOM["mass_amu"] * nlte.AMU))
    dnuD = nu0 * vth / c
    kappa = e * e / (4 * eps0 * me * c) * tr[3] * P.lte[tr[0]] * -np.expm1(-h * nu0 / (k * P.T)) / (math.sqrt(math.pi) * dnuD)
    np.testing.assert_allclose(f[:, 3], np.log10(kappa), rtol=0, atol=1e-9)


def test_state_features_are_the_inputs(small):
    P = small
    f = WSO.features(P, P.lte, np.ones((len(P.nu), P.ncell)))
    inp = P.inp
    np.testing.assert_allclose(f[:, 0], np.log10(inp.T.ravel()), rtol=1e-15)
    np.testing.assert_allclose(f[:, 1], np.log10(inp.ne.ravel()), rtol=1e-15)
    v = np.sqrt(inp.vel[0].astype(np.float64) ** 2 + inp.vel[1].astype(np.float64) ** 2).ravel() / 1e3
    np.testing.assert_allclose(f[:, 2], v, rtol=1e-14)


def test_departures_vanish_at_lte(small):
    P = small
    d = WSO.log_departures(P, P.lte)
    assert d.shape == (P.ncell, P.atom.n_levels)
    assert np.max(np.abs(d)) < 1e-14


def test_prediction_of_zero_departures_is_lte(small):
    """b_l = 1 for every level gives back the LTE populations."""
    P = small
    nl = P.atom.n_levels
    norm = np.concatenate([np.zeros(nl), np.ones(nl)])
    n = WSO.pops_from_prediction(P, np.zeros((P.ncell, nl)), norm)
    np.testing.assert_allclose(n, P.lte, rtol=1e-14)


def test_round_trip_populations_targets_populations(small):
    """Populations that sum to ntot survive targets -> standardise ->
    prediction unchanged; a common factor on every b_l is removed by the
    renormalisation; the level order is kept ([cells][levels] targets)."""
    P = small
    rng = np.random.default_rng(3)
    nl = P.atom.n_levels
    n = P.lte * 10.0 ** rng.uniform(-2, 2, P.lte.shape)
    n = n / n.sum(axis=0) * P.ntot
    d = WSO.log_departures(P, n)
    norm = np.concatenate([d.mean(axis=0), d.std(axis=0)])
    y = WSO.standardise(d, norm)
    np.testing.assert_allclose(WSO.pops_from_prediction(P, y, norm), n, rtol=1e-12)
    shifted = np.concatenate([norm[:nl] + 0.7, norm[nl:]])
    np.testing.assert_allclose(WSO.pops_from_prediction(P, y, shifted), n, rtol=1e-12)
    np.testing.assert_allclose(WSO.pops_from_prediction(P, y, norm).sum(axis=0), P.ntot, rtol=1e-14)
