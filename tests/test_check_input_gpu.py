"""RCX_FLAG_CHECK_INPUT through the C ABI: values forced from the host (a
NaN, an infinity, a negative opacity or emissivity, a zero temperature, a
non-finite velocity) make the call return RCX_E_NONFINITE before anything
is computed; valid inputs give the same result as an unchecked call, bit for
bit. Every kernel runs to completion: the check is a reduction over the
inputs, read back by the host."""
import numpy as np
import pytest

from paper_2408_14425_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _expect_nonfinite(fn, words):
    from paper_2408_14425_amd import rcx
    with pytest.raises(rcx.RcxError) as e:
        fn()
    assert e.value.code == rcx.RCX_E_NONFINITE
    code, msg = rcx.rcx_last_error()
    assert code == rcx.RCX_E_NONFINITE
    for w in words:
        assert w in msg, msg


def test_formal_solve_input_check():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.line_medium(48, 64, seed=5, wave_subset=np.arange(0, 20))
    print(f"[gpu] input check {inp.name}", flush=True)
    chi = torch.from_numpy(inp.chi).cuda()
    eta = torch.from_numpy(inp.eta).cuda()
    plain = rcx.Plan(inp.nx, inp.nz, inp.n_wave)
    checked = rcx.Plan(inp.nx, inp.nz, inp.n_wave, check_input=True)
    J0 = plain.formal_solve(chi, eta)
    J1 = checked.formal_solve(chi, eta)
    torch.cuda.synchronize()
    assert torch.equal(J0, J1)
    bad = chi.clone()
    bad[7, 11, 3] = float("nan")
    _expect_nonfinite(lambda: checked.formal_solve(bad, eta), ["chi or eta", "not finite"])
    bad = eta.clone()
    bad[19, 47, 47] = float("inf")
    _expect_nonfinite(lambda: checked.formal_solve(chi, bad), ["not finite"])
    bad = eta.clone()
    bad[0, 0, 0] = -1.0
    _expect_nonfinite(lambda: checked.formal_solve(chi, bad), ["out of range"])
    _expect_nonfinite(lambda: checked.emergent(bad, eta, 0.6, 0.8, 40), ["rcx_emergent"])
    # the same plan still solves valid inputs afterwards
    J2 = checked.formal_solve(chi, eta)
    torch.cuda.synchronize()
    assert torch.equal(J0, J2)
    plain.close()
    checked.close()


def test_batch_input_check():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    shapes, nw = [(40, 24), (32, 32)], [5, 18]
    rng = np.random.default_rng(2)
    chi = [torch.from_numpy(rng.uniform(0.01, 3.0, (w, nz, nx)).astype(np.float32)).cuda() for (nx, nz), w in
           zip(shapes, nw)]
    eta = [c * 0.5 for c in chi]
    B = rcx.Batch(shapes, nw, check_input=True)
    J = B.solve(chi, eta)
    torch.cuda.synchronize()
    assert all(torch.isfinite(j).all() for j in J)
    bad = [c.clone() for c in chi]
    bad[1][17, 31, 0] = float("nan")
    _expect_nonfinite(lambda: B.solve(bad, eta), ["rcx_batch_solve"])
    B.close()


def test_nlte_atmosphere_input_check():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    inp = W.nlte_atmosphere(16, seed=5, n_line=16, n_cont=8)
    s = rcx.Nlte(inp, check_input=True, set_atmosphere=False)
    T = torch.from_numpy(inp.T.copy()).cuda()
    ne = torch.from_numpy(inp.ne.copy()).cuda()
    ntot = torch.from_numpy(inp.ntot.copy()).cuda()
    vel = torch.from_numpy(inp.vel.copy()).cuda()
    s.set_atmosphere(T, ne, ntot, vel)  # valid (negative velocities included)
    assert (vel < 0).any()
    bad = T.clone()
    bad[3, 4] = 0.0
    _expect_nonfinite(lambda: s.set_atmosphere(bad, ne, ntot, vel), ["T", "out of range"])
    bad = ntot.clone()
    bad[15, 15] = float("nan")
    _expect_nonfinite(lambda: s.set_atmosphere(T, ne, bad, vel), ["ntot", "not finite"])
    bad = vel.clone()
    bad[1, 2, 2] = float("-inf")
    _expect_nonfinite(lambda: s.set_atmosphere(T, ne, ntot, bad), ["vel", "not finite"])
    s.close()
