"""What the trained warm-start network gains over the method without it, on held-out
potentials: a small instance of the whole loop (targets from the method's own batched
solves, training by the device kernels, start blocks for new problems)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_trained_network_saves_iterations_on_held_out_problems():
    from paper_2306_10379_amd import warmstart as W
    print("warm start: 32 x 32 grids, 8 wells, p = 8, 256 training / 32 held-out problems", flush=True)
    r = W.run_experiment(N=32, p=8, ntrain=256, ntest=32, modes=12, width=16, layers=3, epochs=40, batch=16,
                         lr=3e-3, tol=1e-8, seed=1, nsingle=4, log=lambda s: print(s, flush=True))
    b = r["batched_held_out"]
    # the network's subspaces are closer than the prior's (the V = 0 eigenvectors) ...
    assert r["held_out_loss"]["trained"] < 0.25 * r["held_out_loss"]["prior"]
    # ... and the solves from them take fewer iterations than from the prior and than from
    # random blocks (the fallback), all to the same residual tolerance
    assert b["network"]["iters_mean"] < b["prior"]["iters_mean"]
    assert b["network"]["iters_mean"] < 0.5 * b["random"]["iters_mean"]
    assert b["network"]["fallbacks"] == 0
    assert r["single_fp64"]["network"]["iters_mean"] < r["single_fp64"]["random"]["iters_mean"]
