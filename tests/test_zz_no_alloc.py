"""rcx_formal_solve_noalloc (the formal solve in the library's scratch, no
allocation) against rcx_formal_solve on the same plan, through the C ABI:
two calls in a row, the second with a smaller input, each bit for bit equal
to the allocating entry point's J (the same kernels on the same inputs) and
within the FP32 parity bar (1e-4) of the FP64 oracle; a solve whose
workspace exceeds the scratch is rejected before anything runs."""
import numpy as np
import pytest

import oracle
from paper_2408_14425_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_matches_allocating_solve_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_14425_amd import rcx
    big = W.line_medium(96, 64, seed=5, wave_subset=np.arange(0, 40))   # three batches: a pair, then one
    small = W.line_medium(96, 64, seed=6, wave_subset=np.arange(0, 7))  # one ragged batch
    plan = rcx.Plan(96, 96, 40)
    print(f"[gpu] no-alloc formal solve: workspace {plan.workspace_bytes(40)} B for 40 wavelengths", flush=True)
    for inp in (big, small):
        chi = torch.from_numpy(inp.chi).cuda()
        eta = torch.from_numpy(inp.eta).cuda()
        J_ref = plan.formal_solve(chi, eta)
        J = torch.full_like(chi, float("nan"))
        plan.formal_solve_noalloc(chi, eta, J)
        torch.cuda.synchronize()
        assert torch.equal(J, J_ref), inp.name
        Jo = oracle.formal_solve(inp.chi, inp.eta, oracle.default_cascades(96, 96))["J"]
        rel = np.abs(J.cpu().numpy().astype(np.float64) - Jo) / Jo
        print(f"no-alloc {inp.name}: bitwise equal to rcx_formal_solve, max rel vs oracle {rel.max():.3e}", flush=True)
        assert rel.max() < 1e-4
    plan.close()


def test_noalloc_rejects_solves_beyond_the_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_14425_amd import rcx
    plan = rcx.Plan(1024, 1024, 16)
    assert plan.workspace_bytes(16) > 64 << 20
    chi = torch.ones((16, 1024, 1024), dtype=torch.float32, device="cuda")
    J = torch.zeros_like(chi)
    with pytest.raises(rcx.RcxError) as e:
        plan.formal_solve_noalloc(chi, chi, J)
    assert e.value.code == rcx.RCX_E_WORKSPACE
    torch.cuda.synchronize()
    assert torch.count_nonzero(J).item() == 0
    plan.set_timing(True)
    small = rcx.Plan(32, 32, 1)
    small.set_timing(True)
    c = torch.ones((1, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(rcx.RcxError) as e:
        small.formal_solve_noalloc(c, c, torch.zeros_like(c))
    assert e.value.code == rcx.RCX_E_INVALID
    plan.close()
    small.close()
