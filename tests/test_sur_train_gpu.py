"""End to end on a small scale: solver trajectories -> training with the
library kernels (the loss must fall) -> judged inference with fallback."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_train_and_evaluate_small():
    from paper_2105_09671_amd import sur_train as T
    data = T.make_trajectories(list(range(16)), blocks=3)
    assert data.shape == (16, 4, 256, 256)
    # snapshots are the stepper's own states: block 0 is the initial field
    assert torch.isfinite(data).all() and float(data.abs().max()) <= 1.0 + 1e-6
    net, hist, _ = T.train(data, steps=60, batch=8, lr=2e-3, log_every=59)
    val = T.validate(net, data, ["circle"] * 16)
    assert len(val["circle"]) == 3 and all(v >= 0 for v in val["circle"])
    assert hist[-1][1] < hist[0][1]
    res = T.evaluate(net, list(range(100000, 100016)), T_blocks=3, sample_every=4)
    assert res["grid_blocks"] == 48 and 0 <= res["surrogate_grid_blocks"] <= 36
    assert 0.0 <= res["final_ok_fraction"] <= 1.0
    # a grid never advanced by the surrogate ends exactly on the plain result
    if res["surrogate_grid_blocks"] == 0:
        assert res["final_ok_fraction"] == 1.0 and res["final_l2_median"] == 0.0
    net.close()
