"""GPU surrogate kernels (BF16 MFMA, FP32 accumulate) against the FP64 oracle.

The oracle is fed the same BF16-rounded weights and a BF16-representable input,
so the remaining difference is the BF16 rounding of the GPU's intermediate
activations and gradients (8-bit significand, 2^-8 = 3.9e-3) compounded over
the layers, plus FP32 summation order.  Bars: output update U within 1e-2
relative L2; per-layer weight gradients within 5e-2 relative L2.
"""
import numpy as np
import pytest
import torch

from oracle import surrogate as S
from paper_2105_09671_amd import inputs

pytestmark = pytest.mark.gpu


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


@pytest.fixture(scope="module")
def sur():
    assert torch.cuda.is_available()
    from paper_2105_09671_amd import surrogate
    return surrogate


def _case(seed, B, hw):
    w = S.init_weights(seed)
    w = w + inputs.random_field(w.shape, seed + 1, amp=0.02)      # non-zero biases
    w = bf16_round(w).astype(np.float64)
    phi = bf16_round(inputs.random_field((B, hw, hw), seed + 2, amp=0.9)).astype(np.float64)
    tgt = inputs.random_field((B, hw, hw), seed + 3, amp=0.9)
    return w, phi, tgt


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("B,hw", [(2, 32), (3, 16)])
def test_forward_matches_oracle(sur, B, hw):
    w, phi, _ = _case(60, B, hw)
    net = sur.Surrogate(B, hw)
    net.set_weights(w.astype(np.float32))
    x = torch.from_numpy(phi.astype(np.float32)).cuda()
    out = net.forward(x).cpu().numpy().astype(np.float64)
    ref = S.forward(w, phi)
    U, Ur = out - phi, ref - phi
    assert _rel(U, Ur) <= 1e-2
    assert np.max(np.abs(U - Ur)) <= 5e-2 * np.max(np.abs(Ur))
    net.close()


@pytest.mark.parametrize("B,hw", [(3, 20), (2, 32), (1, 64), (1, 136)])
def test_infer_matches_forward_and_oracle(sur, B, hw):
    """The inference path (decoder 1x1 outputs kept at low resolution and
    upsampled inside the next 3x3 layer's patch load; head and residual in the
    last layer's epilogue; the first skip tensor dense) against the training
    forward, which also stores the 3x3 outputs, copies the upsampled 1x1 maps
    into the concatenations and runs the head as its own kernel: the same
    products in the same order, so bit for bit equal; and against the oracle
    to the forward's own bar.  Sizes cover grids narrower than a 64-wide tile,
    odd sizes at the coarse levels (20 -> 10 -> 5) and ragged tiles (136)."""
    w, phi, _ = _case(62, B, hw)
    net = sur.Surrogate(B, hw)
    net.set_weights(w.astype(np.float32))
    x = torch.from_numpy(phi.astype(np.float32)).cuda()
    a = net.forward(x).cpu().numpy().astype(np.float64)
    y = torch.full_like(x, float("nan"))
    b = net.infer(x, y).cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(b))
    assert np.array_equal(a, b)
    ref = S.forward(w, phi)
    U, Ur = b - phi, ref - phi
    assert _rel(U, Ur) <= 1e-2
    assert np.max(np.abs(U - Ur)) <= 5e-2 * np.max(np.abs(Ur))
    # a smaller batch on the same handle, and no backward state left behind
    b1 = net.infer(x[:1].contiguous()).cpu().numpy().astype(np.float64)
    assert np.array_equal(b1, b[:1])
    from paper_2105_09671_amd import _lib as L
    with pytest.raises(L.AcError):
        net.loss(x)
    with pytest.raises(ValueError):
        net.infer(x, x)
    net.close()


def test_zero_weights_give_phi(sur):
    net = sur.Surrogate(2, 16)
    x = torch.from_numpy(inputs.random_field((2, 16, 16), 61).astype(np.float32)).cuda()
    assert torch.equal(net.forward(x), x)
    assert torch.equal(net.infer(x), x)
    net.close()


@pytest.mark.parametrize("B,hw", [(2, 32), (1, 64)])
def test_gradients_match_oracle(sur, B, hw):
    w, phi, tgt = _case(70, B, hw)
    net = sur.Surrogate(B, hw)
    net.set_weights(w.astype(np.float32))
    x = torch.from_numpy(phi.astype(np.float32)).cuda()
    t = torch.from_numpy(tgt.astype(np.float32)).cuda()
    net.forward(x)
    loss = float(net.loss(t).item())
    net.backward(B)
    g = net.grads().astype(np.float64)
    lref, gref = S.loss_grad(w, phi, tgt)
    assert abs(loss - lref) <= 1e-2 * lref
    off = 0
    for name, cin, cout, k in S.layer_table():
        nw = cout * k * k * cin
        for part, n in (("w", nw), ("b", cout)):
            err = _rel(g[off:off + n], gref[off:off + n])
            assert err <= 5e-2, "%s.%s rel L2 %.3g" % (name, part, err)
            off += n
    net.close()


def test_adam_matches_reference_update(sur):
    w, phi, tgt = _case(80, 2, 16)
    net = sur.Surrogate(2, 16)
    net.set_weights(w.astype(np.float32))
    x = torch.from_numpy(phi.astype(np.float32)).cuda()
    t = torch.from_numpy(tgt.astype(np.float32)).cuda()
    net.forward(x)
    net.loss(t)
    net.backward(2)
    g = net.grads().astype(np.float64)
    net.adam(1e-3)
    w1 = net.get_weights().astype(np.float64)
    # Adam (Kingma & Ba) first step: m = (1-b1) g, v = (1-b2) g^2, bias-corrected
    m, v = 0.1 * g, 0.001 * g * g
    expect = w - 1e-3 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    assert np.max(np.abs(w1 - expect)) <= 1e-6
    net.close()


def test_backward_of_external_output_gradient(sur):
    """ac_sur_backward with a caller's d loss / d out: fed the mean-squared-error
    gradient 2 (out - target) / n it gives the gradients of the stored-loss
    path (to FP32 summation order) and of the oracle (BF16 bar); the map is
    linear in d loss / d out (x2, exact in BF16 and FP32, gives 2x the
    gradients up to the order of the FP32 atomic sums)."""
    B, hw = 2, 32
    w, phi, tgt = _case(71, B, hw)
    net = sur.Surrogate(B, hw)
    net.set_weights(w.astype(np.float32))
    x = torch.from_numpy(phi.astype(np.float32)).cuda()
    t = torch.from_numpy(tgt.astype(np.float32)).cuda()
    out = net.forward(x).clone()
    net.loss(t)
    net.backward(B)
    g_loss = net.grads().astype(np.float64)
    dU = (out - t) * np.float32(2.0 / out.numel())
    net.forward(x)
    net.backward(B, dU)
    g_ext = net.grads().astype(np.float64)
    assert _rel(g_ext, g_loss) <= 1e-5
    _, gref = S.loss_grad(w, phi, tgt)
    assert _rel(g_ext, gref) <= 5e-2
    net.forward(x)
    net.backward(B, (2.0 * dU).contiguous())
    assert _rel(net.grads().astype(np.float64), 2.0 * g_ext) <= 1e-5
    from paper_2105_09671_amd import _lib as L
    net.infer(x, torch.empty_like(x))               # no activations kept: refused
    with pytest.raises(L.AcError):
        net.backward(B, dU)
    with pytest.raises(ValueError):
        net.backward(1, dU)                         # wrong batch for the gradient tensor
    net.close()


def test_infer_full_batch_sampled_against_oracle(sur):
    """The benchmarked launch: 256 grids of 256^2 in one inference call with
    the stored trained weights.  One sampled grid against the FP64 oracle (fed
    the same BF16-rounded weights and input) to the forward's bar, and equal
    bit for bit to the same grid inferred alone (no result depends on the
    batch or on where a tile lands)."""
    import os
    B, hw, k = 256, 256, 137
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2105_09671_amd", "weights", "sur256.npz")
    w = bf16_round(np.load(path)["weights"]).astype(np.float64)
    phi = bf16_round(inputs.random_field((B, hw, hw), 71, amp=0.9))
    net = sur.Surrogate(B, hw)
    net.set_weights(w.astype(np.float32))
    x = torch.from_numpy(phi).cuda()
    out = net.infer(x).cpu().numpy()
    one = net.infer(x[k:k + 1].contiguous()).cpu().numpy()
    net.close()
    assert np.all(np.isfinite(out))
    assert np.array_equal(out[k], one[0])
    ref = S.forward(w, phi[k:k + 1].astype(np.float64))[0]
    U, Ur = out[k].astype(np.float64) - phi[k], ref - phi[k]
    assert _rel(U, Ur) <= 1e-2
    assert np.max(np.abs(U - Ur)) <= 5e-2 * np.max(np.abs(Ur))
