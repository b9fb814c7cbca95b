"""Pins of the FP64 surrogate oracle (sur_oracle.c).

* its backward pass equals central finite differences of its own loss;
* each building block equals an independent library routine: the 3x3 replicate-
  padded cross-correlation is scipy.ndimage.correlate with mode='nearest', the
  2x2 average pool is a reshape-mean, the nearest upsample is np.repeat;
* structural facts: zero weights leave phi + head bias, and a spatially
  constant input gives a spatially constant output (replicate, not zero,
  padding all the way through the U-Net).
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import surrogate as S
from paper_2105_09671_amd import inputs

TINY = (2, 3, 4)


def _rand(shape, seed, amp=1.0):
    return inputs.random_field(shape, seed, amp=amp)


def test_param_count_matches_layer_table():
    assert S.num_params() == 241473
    n = sum(co * k * k * ci + co for _, ci, co, k in S.layer_table())
    assert n == 241473
    assert S.num_params(TINY) == sum(co * k * k * ci + co for _, ci, co, k in S.layer_table(TINY))


def test_backward_matches_finite_differences():
    n = S.num_params(TINY)
    w = _rand((n,), 1, amp=0.6)
    phi = _rand((2, 8, 8), 2, amp=0.9)
    tgt = _rand((2, 8, 8), 3, amp=0.9)
    loss, g = S.loss_grad(w, phi, tgt, TINY)
    step = 1e-6
    fd = np.empty(n)
    for i in range(n):
        wp, wm = w.copy(), w.copy()
        wp[i] += step
        wm[i] -= step
        fd[i] = (S.loss_grad(wp, phi, tgt, TINY)[0] - S.loss_grad(wm, phi, tgt, TINY)[0]) / (2 * step)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)
    assert np.max(np.abs(fd - g)) <= 1e-5 * np.max(np.abs(g))
    out = S.forward(w, phi, TINY)
    assert abs(loss - np.mean((out - tgt) ** 2)) <= 1e-15 * max(1.0, loss)


@pytest.mark.parametrize("k", [3, 1])
def test_conv_equals_scipy_correlate(k):
    x = _rand((2, 3, 9, 7), 4)
    w = _rand((4, k, k, 3), 5)
    b = _rand((4,), 6)
    y = S.conv(x, w, b, k)
    for bi in range(2):
        for co in range(4):
            ref = np.full((9, 7), b[co])
            for ci in range(3):
                ref += ndimage.correlate(x[bi, ci], w[co, :, :, ci], mode="nearest")
            assert np.max(np.abs(y[bi, co] - ref)) <= 1e-13


def test_pool_and_upsample_equal_numpy():
    x = _rand((2, 3, 8, 6), 7)
    p = S.pool(x)
    assert np.max(np.abs(p - x.reshape(2, 3, 4, 2, 3, 2).mean(axis=(3, 5)))) <= 1e-15
    u = S.up(x)
    assert np.array_equal(u, np.repeat(np.repeat(x, 2, axis=2), 2, axis=3))


def test_zero_weights_give_phi_plus_head_bias():
    w = np.zeros(S.num_params())
    w[-1] = 0.125
    phi = _rand((1, 16, 12), 8)
    assert np.array_equal(S.forward(w, phi), phi + 0.125)


def test_constant_input_stays_constant():
    w = S.init_weights(9, TINY)
    w += _rand(w.shape, 10, amp=0.05)      # non-zero biases too
    phi = np.full((2, 16, 16), 0.3)
    out = S.forward(w, phi, TINY)
    for b in range(2):
        assert np.max(out[b]) - np.min(out[b]) <= 1e-14
