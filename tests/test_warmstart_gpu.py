"""The learned warm start, end to end on the GPU: converged runs of the
method as training data, GPU training, and the test that the trained network
starts the plain iteration closer to the fixed point, so it needs fewer
iterations, while converging to the same populations. Equal accuracy: a
reference iterated with Ng acceleration to a change below 1e-6 stands for
the fixed point, and each start iterates until its largest relative
difference from it first drops to 1e-3; the warm start must get there in
fewer iterations. The paper's stopping rule (max relative change < 1e-3)
is checked too: the warm start meets it sooner."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_saves_iterations_and_reaches_same_fixed_point():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_14425_amd import warmstart as WS
    print("[gpu] warm start: training data 8 x 32^2", flush=True)
    X, Y, info = WS.dataset(32, range(5000, 5008), n_line=32, n_cont=16)
    net, fn, tn, losses = WS.train(X, Y, epochs=60, batch=1024, lr=3e-3)
    print("training loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.2 * losses[0]
    ev = WS.evaluate(net, fn, tn, 64, [6000], n_line=32, n_cont=16)
    net.close()
    e = ev[0]
    print(e)
    assert e["converged"]
    assert e["warm_iterations"] < e["lte_iterations"]
    # equal accuracy: both within 1e-3 of the fixed point, the warm start in
    # fewer iterations
    assert e["warm_error_at_accuracy"] <= 1e-3 and e["lte_error_at_accuracy"] <= 1e-3
    assert e["warm_iterations_to_accuracy"] < e["lte_iterations_to_accuracy"]
    # the prediction starts closer than LTE does where LTE is far off (most
    # cells are collision-dominated and start at LTE within 1e-4)
    assert e["prediction_error_vs_reference"] < e["lte_start_error_vs_reference"]
