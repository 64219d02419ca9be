"""GPU BF16-MFMA MLP vs the FP64 oracle through the C ABI: forward values,
gradients (cosine >= 0.999, max abs difference <= 2e-2 of the largest
gradient: BF16 operands carry ~4e-3 relative rounding), and training."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2408_14425_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _params_list(flat, n_in, width, depth, n_out):
    return omlp.unflatten(flat.astype(np.float64), n_in, width, depth, n_out)


@pytest.mark.parametrize("batch", [1, 1000, 4096])
def test_forward_matches_oracle(batch):
    torch = _torch()
    from paper_2408_14425_amd import rcx
    print(f"[gpu] mlp forward batch={batch}", flush=True)
    flat = W.mlp_init_params(6, 128, 4, 4, seed=1)
    net = rcx.Mlp(6, 128, 4, 4, max_batch=4096)
    net.set_params(flat)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(batch, 6)).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    net.close()
    yo, _, _ = omlp.forward(_params_list(flat, 6, 128, 4, 4), x.astype(np.float64))
    err = np.abs(y - yo).max() / np.abs(yo).max()
    print("forward max err / max |y|", err)
    assert err < 3e-2


def test_gradients_match_oracle():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    flat = W.mlp_init_params(6, 128, 4, 4, seed=3)
    net = rcx.Mlp(6, 128, 4, 4, max_batch=2048)
    net.set_params(flat)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(1500, 6)).astype(np.float32)
    yr = rng.normal(size=(1500, 4)).astype(np.float32)
    loss, g = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(yr).cuda())
    g = g.cpu().numpy().astype(np.float64)
    net.close()
    lo, go = omlp.loss_and_grads(_params_list(flat, 6, 128, 4, 4), x.astype(np.float64), yr.astype(np.float64))
    gflat = np.concatenate([np.concatenate([gW.ravel(), gb.ravel()]) for gW, gb in go])
    cos = g @ gflat / (np.linalg.norm(g) * np.linalg.norm(gflat))
    maxd = np.abs(g - gflat).max() / np.abs(gflat).max()
    print(f"loss gpu {loss:.6f} oracle {lo:.6f}; grad cosine {cos:.6f}, max diff / max |g| {maxd:.3e}")
    assert abs(loss - lo) <= 1e-2 * lo
    assert cos >= 0.999
    assert maxd <= 2e-2


def test_training_reduces_loss():
    torch = _torch()
    from paper_2408_14425_amd import rcx
    rng = np.random.default_rng(5)
    x = rng.normal(size=(4096, 6)).astype(np.float32)
    y = np.stack([np.sin(x[:, 0]), x[:, 1] * x[:, 2], np.tanh(x[:, 3]), x[:, 4] - x[:, 5]], 1).astype(np.float32)
    net = rcx.Mlp(6, 128, 4, 4, max_batch=4096)
    net.set_params(W.mlp_init_params(6, 128, 4, 4, seed=6))
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    losses = [net.train_step(xt, yt, 2e-3) for _ in range(300)]
    net.close()
    print("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.1 * losses[0]
