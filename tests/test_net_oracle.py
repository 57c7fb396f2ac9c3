"""Pins of the float64 proposal-network reference (oracle/net.py) against
library routines, adjoint identities and finite differences."""
import numpy as np
import pytest
import scipy.signal

from oracle import net
from paper_1002_1168_amd import synth


def test_bf16_matches_torch_conversion():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 2000), rng.normal(0, 1e-3, 500),
                        # exact ties between two bfloat16 neighbours
                        (np.arange(1, 200) * 2 + 1) * 2.0 ** -8 + 1.0])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16(x), want)


@pytest.mark.parametrize("stride,H,Ci,Co", [(1, 24, 2, 5), (2, 24, 3, 4), (2, 12, 32, 2)])
def test_conv_matches_scipy_correlate(stride, H, Ci, Co):
    rng = np.random.default_rng(stride * 100 + H)
    x = rng.normal(size=(H, H, Ci))
    w = rng.normal(size=(Co, 3, 3, Ci))
    b = rng.normal(size=Co)
    got = net.conv(x, w, b, stride)
    for co in range(Co):
        full = sum(scipy.signal.correlate2d(x[:, :, ci], w[co, :, :, ci], mode="same") for ci in range(Ci))
        want = full[::stride, ::stride] + b[co]
        assert np.allclose(got[:, :, co], want, atol=1e-10)


@pytest.mark.parametrize("stride,H,Ci,Co", [(1, 24, 2, 32), (2, 24, 32, 32), (2, 12, 32, 2)])
def test_gradient_adjoints(stride, H, Ci, Co):
    """<conv(x, w), y> = <x, dX(y, w)> = <w, dW(x, y)> (no bias)."""
    rng = np.random.default_rng(H + Ci)
    x = rng.normal(size=(H, H, Ci))
    w = rng.normal(size=(Co, 3, 3, Ci))
    y = net.conv(x, w, np.zeros(Co), stride)
    r = rng.normal(size=y.shape)
    lhs = float((y * r).sum())
    assert np.isclose(lhs, float((x * net.conv_input_grad(r, w, stride, x.shape)).sum()), rtol=1e-10)
    assert np.isclose(lhs, float((w * net.conv_weight_grad(x, r, stride)).sum()), rtol=1e-10)


def test_prep_box_average_and_edge_clamp():
    rng = np.random.default_rng(5)
    H, W = 48, 64
    cur = rng.integers(0, 256, (H, W), dtype=np.uint8)
    ref = rng.integers(0, 256, (H, W), dtype=np.uint8)
    for x0, y0 in [(0, 0), (48, 32), (16, 16)]:
        got = net.prep(cur, ref, x0, y0, rnd=False)
        c = cur[y0:y0 + 16, x0:x0 + 16].astype(float).reshape(8, 2, 8, 2).mean(axis=(1, 3))
        assert np.allclose(got[8:16, 8:16, 0], (c - 128) / 128)
        assert not got[:8, :, 0].any() and not got[16:, :, 0].any() and not got[:, :8, 0].any()
        padded = np.pad(ref.astype(float), 16, mode="edge")
        win = padded[y0:y0 + 48, x0:x0 + 48].reshape(24, 2, 24, 2).mean(axis=(1, 3))
        assert np.allclose(got[:, :, 1], (win - 128) / 128)
        assert np.array_equal(net.prep(cur, ref, x0, y0), net.bf16(got))


def test_prep_scale_four_box_average_and_edge_clamp():
    # window scale 4: the 96-pixel window [-40, 56) in 4 x 4 means, the
    # current MB as 4 x 4 means in the canvas centre [10, 14)
    rng = np.random.default_rng(6)
    H, W = 64, 80
    cur = rng.integers(0, 256, (H, W), dtype=np.uint8)
    ref = rng.integers(0, 256, (H, W), dtype=np.uint8)
    for x0, y0 in [(0, 0), (64, 48), (32, 16)]:
        got = net.prep(cur, ref, x0, y0, rnd=False, scale=4)
        c = cur[y0:y0 + 16, x0:x0 + 16].astype(float).reshape(4, 4, 4, 4).mean(axis=(1, 3))
        assert np.allclose(got[10:14, 10:14, 0], (c - 128) / 128)
        mask = np.ones((24, 24), bool)
        mask[10:14, 10:14] = False
        assert not got[:, :, 0][mask].any()
        padded = np.pad(ref.astype(float), 40, mode="edge")
        win = padded[y0:y0 + 96, x0:x0 + 96].reshape(24, 4, 24, 4).mean(axis=(1, 3))
        assert np.allclose(got[:, :, 1], (win - 128) / 128)
    assert net.half_width(2) == 16 and net.half_width(4) == 40


def test_finite_difference_gradient():
    """The analytic backward of the float64 network against central
    differences of the loss, on a sample of parameters of every tensor."""
    rng = np.random.default_rng(11)
    P = synth.net_init(3).astype(np.float64) * 1.5
    P[net.NPARAM - 2:] = [0.3, -0.2]
    xs = [rng.normal(0, 0.5, (24, 24, 2)) for _ in range(2)]
    ys = np.array([[3.0, -2.0], [-1.0, 4.0]])
    _, g, _ = net.loss_and_grad(xs, ys, P, rnd=False)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in net.SHAPES])
    idx = np.concatenate([rng.choice(np.arange(offs[t], offs[t + 1]), size=min(12, offs[t + 1] - offs[t]),
                                     replace=False) for t in range(len(net.SHAPES))])
    eps = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += eps
        Pm[i] -= eps
        fd = (net.loss_and_grad(xs, ys, Pp, rnd=False)[0] - net.loss_and_grad(xs, ys, Pm, rnd=False)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_rounded_forward_activations_are_bf16():
    rng = np.random.default_rng(2)
    f = net.forward(net.prep(rng.integers(0, 256, (48, 48), dtype=np.uint8),
                             rng.integers(0, 256, (48, 48), dtype=np.uint8), 16, 16), synth.net_init(1))
    for k in ("x0", "a1", "a2"):
        assert np.array_equal(net.bf16(f[k]), f[k])
    assert f["a1"].shape == (24, 24, 32) and f["a2"].shape == (12, 12, 32) and f["z3"].shape == (6, 6, 2)
    assert np.allclose(f["p"], f["z3"].reshape(-1, 2).mean(axis=0))


def test_sgd_closed_form():
    P, V = np.array([1.0, -2.0]), np.zeros(2)
    g = np.array([0.5, 0.25])
    P1, V1 = net.sgd(P, V, g, lr=0.1, mu=0.9)
    P2, V2 = net.sgd(P1, V1, g, lr=0.1, mu=0.9)
    assert np.allclose(V2, 1.9 * g) and np.allclose(P2, P - 0.1 * g - 0.1 * 1.9 * g)


def test_seed_rounding_and_clip():
    p = np.array([[0.5, 1.5], [-2.5, 2.4999], [17.2, -30.0]])
    assert net.seed_of(p).tolist() == [[0, 4], [-4, 4], [32, -32]]
    p4 = np.array([[17.2, -30.0], [40.4, -41.0]])
    assert net.seed_of(p4, scale=4).tolist() == [[34, -60], [80, -80]]


def test_parameter_count():
    assert net.NPARAM == 10434 and synth.net_init(0).shape == (10434,)
