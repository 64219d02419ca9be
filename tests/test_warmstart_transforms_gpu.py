"""The warm start's data transforms on the GPU against their FP64 oracle
(oracle/warmstart.py), element by element, through the C ABI:

  rcx_nlte_features       raw features at LTE: log10 T, log10 n_e and
                          log10 kappa_0 to 4 FP32 ulps of the value (FP32
                          logarithms of FP64 inputs rounded to FP32), |v| to
                          1e-6 relative, log10 Jbar_t to 1e-4 / ln 10 plus 4
                          ulps (J is FP32 to 1e-4 relative; the profile
                          weights come from the device Voigt table, within
                          5e-5);
                          standardisation (f - mean) / std applied exactly
  rcx_nlte_log_departures log10 (n / n^LTE) in FP64 rounded to FP32
  rcx_nlte_pops_from_prediction
                          populations from seeded predictions, FP64 on
                          both sides: 1e-12 relative
"""
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
def case():
    from oracle import nlte
    inp = W.nlte_atmosphere(48, seed=8, n_line=24, n_cont=16)
    return inp, nlte.Problem(inp)


def test_features_match_oracle(case):
    torch = _torch()
    from oracle import warmstart as WSO
    from paper_2408_14425_amd import rcx
    inp, P = case
    print(f"[gpu] features {inp.name}", flush=True)
    s = rcx.Nlte(inp)
    pops = s.lte()
    raw = s.features(pops).cpu().numpy().astype(np.float64)
    norm = np.array([3.9, 15.0, 10.0, -2.0, 1.0, 2.0, 0.5, 1.5, 5.0, 1.0, 2.0, 3.0], np.float32)
    std = s.features(pops, norm).cpu().numpy().astype(np.float64)
    s.close()
    J = P.formal_solve(P.lte)[0]
    ref = WSO.features(P, P.lte, J)
    err = np.abs(raw - ref)
    ulp4 = 4.0 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    print("feature max abs error per column:", " ".join(f"{e:.2e}" for e in err.max(axis=0)))
    assert np.all(err[:, [0, 1, 3]] <= ulp4[:, [0, 1, 3]])
    assert np.max(err[:, 2] / np.maximum(ref[:, 2], 1e-3)) < 1e-6
    assert np.all(err[:, 4:] <= 1e-4 / np.log(10.0) + ulp4[:, 4:])
    ref_std = WSO.standardise(ref, norm.astype(np.float64))
    assert np.max(np.abs(std - ref_std)) < 1e-4


def test_log_departures_match_oracle(case):
    torch = _torch()
    from oracle import warmstart as WSO
    from paper_2408_14425_amd import rcx
    inp, P = case
    rng = np.random.default_rng(4)
    n = P.lte * 10.0 ** rng.uniform(-1.5, 1.5, P.lte.shape)
    n = n / n.sum(axis=0) * P.ntot
    s = rcx.Nlte(inp)
    d = s.log_departures(torch.from_numpy(n.reshape(4, inp.nz, inp.nx)).to("cuda:0")).cpu().numpy()
    s.close()
    ref = WSO.log_departures(P, n)
    err = np.abs(d.astype(np.float64) - ref)
    print(f"log departures max abs error {err.max():.2e}")
    assert err.max() < 4e-7


def test_pops_from_prediction_match_oracle(case):
    """Seeded standardised predictions (the network's output range) through
    rcx_nlte_pops_from_prediction against the oracle's definition."""
    torch = _torch()
    from oracle import warmstart as WSO
    from paper_2408_14425_amd import rcx
    inp, P = case
    rng = np.random.default_rng(5)
    y = rng.normal(0.0, 1.0, (P.ncell, 4)).astype(np.float32)
    norm = np.array([0.1, -0.5, 0.8, -1.2, 0.3, 1.1, 0.7, 2.0], np.float32)
    s = rcx.Nlte(inp)
    got = s.pops_from_prediction(torch.from_numpy(y).to("cuda:0"), norm).cpu().numpy().reshape(4, -1)
    s.close()
    ref = WSO.pops_from_prediction(P, y.astype(np.float64), norm.astype(np.float64))
    rel = np.abs(got - ref) / ref
    print(f"populations from prediction max rel {rel.max():.2e}")
    assert rel.max() < 1e-12
    np.testing.assert_allclose(got.sum(axis=0), P.ntot, rtol=1e-13)
