"""Float64 reference of the learned motion-vector proposal network (test
infrastructure: only the tests, ``__graft_entry__.smoke()`` and the bench's
``cpu_baseline`` leg use it; the GPU library never does).

The paper has no network: the proposal that seeds its pel-recursive search
(Section 3.2 starts from the block-recursive winner) is an addition of this
project.  What it computes, per 16x16 macroblock (MB) at (x0, y0):

  input   2 x 24 x 24, for a window scale f (2 or 4): channel 0 = the
          current MB box-averaged f x f ((16/f) x (16/f)), centred in a zero
          24 x 24 canvas; channel 1 = the reference window of rows/columns
          [-(12f - 8), 12f + 8) around the MB (24f pixels, frame-clamped),
          box-averaged f x f.  An f x f sum s maps to (s - 128 f^2) / (128 f^2).
          f = 2 is the window [-16, 32) with (s - 512) / 512.
  conv1   3x3, 2 -> 32 channels, stride 1, zero padding 1, ReLU   (24 x 24)
  conv2   3x3, 32 -> 32, stride 2, padding 1, ReLU                (12 x 12)
  conv3   3x3, 32 -> 2, stride 2, padding 1                       (6 x 6)
  output  p = the mean of conv3 over its 36 positions: the predicted
          full-pel vector (x, y); the seed is 2 * clip(rint(p), -w, w) in
          half-pel units, w = 12f - 8 the window's half-width (16 at f = 2).
  loss    sum over a batch of B MBs of |p - y|^2 / (2B), y = the plain
          method's full-pel vector (labels).
  update  momentum SGD on float32 master weights: v <- mu v + g, w <- w - lr v.

Rounding points (``rnd=True``), the ones the GPU kernels take: the input
values, every weight used in a product and the post-ReLU activations are
rounded to bfloat16 (round to nearest even); the conv2 and conv1
pre-activation gradients are rounded to bfloat16 before they enter the
weight-gradient and the next input-gradient products; biases, bias
gradients, conv3 and every sum stay wide.  ``rnd=False`` is the same
function in plain float64 (used by the finite-difference check).

Tensors are (H, W, C) arrays; weights (Co, 3, 3, Ci).  Parameter vector
layout (float32 master copy): W1 (32,3,3,2) | b1 (32) | W2 (32,3,3,32) |
b2 (32) | W3 (2,3,3,32) | b3 (2): 10434 values.
"""
from __future__ import annotations

import numpy as np

SHAPES = (("W1", (32, 3, 3, 2)), ("b1", (32,)), ("W2", (32, 3, 3, 32)), ("b2", (32,)),
          ("W3", (2, 3, 3, 32)), ("b3", (2,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
WINDOW = 16  # reference window half-width in full pels at window scale 2


def half_width(scale: int) -> int:
    """Reference window half-width (full pels) at window scale f: 12 f - 8."""
    return 12 * scale - 8


def unpack(P: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(P[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via the float32 bit pattern:
    keep the upper 16 bits after adding 0x7FFF plus the lowest kept bit."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, rnd):
    return bf16(x) if rnd else np.asarray(x, dtype=np.float64)


def prep(cur: np.ndarray, ref: np.ndarray, x0: int, y0: int, rnd=True, scale: int = 2) -> np.ndarray:
    """Network input (24, 24, 2) of the MB at (x0, y0) at window scale f."""
    f = scale
    H, W = cur.shape
    n, hw, norm = 16 // f, half_width(f), 128 * f * f
    o = (24 - n) // 2
    x = np.zeros((24, 24, 2))
    c = cur[y0:y0 + 16, x0:x0 + 16].astype(np.int64)
    x[o:o + n, o:o + n, 0] = (c.reshape(n, f, n, f).sum(axis=(1, 3)) - norm) / float(norm)
    ys = np.clip(np.arange(y0 - hw, y0 + 16 + hw), 0, H - 1)
    xs = np.clip(np.arange(x0 - hw, x0 + 16 + hw), 0, W - 1)
    w = ref[np.ix_(ys, xs)].astype(np.int64)
    x[:, :, 1] = (w.reshape(24, f, 24, f).sum(axis=(1, 3)) - norm) / float(norm)
    return _r(x, rnd)


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """out[oy, ox, co] = b[co] + sum over taps (ky, kx) and ci of
    w[co, ky, kx, ci] * x[stride*oy + ky - 1, stride*ox + kx - 1, ci]
    (zero outside x)."""
    H, W, _ = x.shape
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    xp = np.zeros((H + 2, W + 2, x.shape[2]))
    xp[1:H + 1, 1:W + 1] = x
    out = np.zeros((Ho, Wo, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            patch = xp[ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            out += patch @ w[:, ky, kx, :].T
    return out


def conv_input_grad(dy: np.ndarray, w: np.ndarray, stride: int, in_shape) -> np.ndarray:
    """Adjoint of ``conv`` in its input: dx[iy, ix, ci] = sum of
    dy[oy, ox, co] * w[co, ky, kx, ci] over stride*oy + ky - 1 = iy,
    stride*ox + kx - 1 = ix."""
    H, W, Ci = in_shape
    Ho, Wo, _ = dy.shape
    dxp = np.zeros((H + 2, W + 2, Ci))
    for ky in range(3):
        for kx in range(3):
            dxp[ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride] += dy @ w[:, ky, kx, :]
    return dxp[1:H + 1, 1:W + 1]


def conv_weight_grad(x: np.ndarray, dy: np.ndarray, stride: int) -> np.ndarray:
    """gw[co, ky, kx, ci] = sum over (oy, ox) of dy[oy, ox, co] *
    x[stride*oy + ky - 1, stride*ox + kx - 1, ci]."""
    H, W, Ci = x.shape
    Ho, Wo, Co = dy.shape
    xp = np.zeros((H + 2, W + 2, Ci))
    xp[1:H + 1, 1:W + 1] = x
    gw = np.zeros((Co, 3, 3, Ci))
    d2 = dy.reshape(-1, Co)
    for ky in range(3):
        for kx in range(3):
            patch = xp[ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            gw[:, ky, kx, :] = d2.T @ patch.reshape(-1, Ci)
    return gw


def forward(x0: np.ndarray, P: np.ndarray, rnd=True) -> dict:
    w = unpack(P)
    W1, W2, W3 = (_r(w[k], rnd) for k in ("W1", "W2", "W3"))
    a1 = _r(np.maximum(conv(x0, W1, w["b1"], 1), 0.0), rnd)
    a2 = _r(np.maximum(conv(a1, W2, w["b2"], 2), 0.0), rnd)
    z3 = conv(a2, W3, w["b3"], 2)
    return {"x0": x0, "a1": a1, "a2": a2, "z3": z3, "p": z3.mean(axis=(0, 1)), "W1": W1, "W2": W2, "W3": W3}


def backward(f: dict, dp: np.ndarray, rnd=True) -> np.ndarray:
    """Gradient of the parameters for an upstream gradient dp = dL/dp (2,)."""
    dz3 = np.broadcast_to(np.asarray(dp, dtype=np.float64) / 36.0, f["z3"].shape)
    gW3 = conv_weight_grad(f["a2"], dz3, 2)
    gb3 = dz3.sum(axis=(0, 1))
    da2 = conv_input_grad(dz3, f["W3"], 2, f["a2"].shape)
    dpre2 = da2 * (f["a2"] > 0)
    gb2 = dpre2.sum(axis=(0, 1))
    dpre2 = _r(dpre2, rnd)
    gW2 = conv_weight_grad(f["a1"], dpre2, 2)
    da1 = conv_input_grad(dpre2, f["W2"], 2, f["a1"].shape)
    dpre1 = da1 * (f["a1"] > 0)
    gb1 = dpre1.sum(axis=(0, 1))
    dpre1 = _r(dpre1, rnd)
    gW1 = conv_weight_grad(f["x0"], dpre1, 1)
    return pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3})


def loss_and_grad(inputs, labels, P, rnd=True):
    """inputs: list of (24, 24, 2) arrays; labels: (B, 2) full-pel vectors.
    -> (loss, gradient, predictions (B, 2))."""
    B = len(inputs)
    g = np.zeros(NPARAM)
    loss = 0.0
    preds = np.zeros((B, 2))
    for i, (x0, y) in enumerate(zip(inputs, np.asarray(labels, dtype=np.float64))):
        f = forward(x0, P, rnd)
        d = f["p"] - y
        loss += 0.5 * float(d @ d) / B
        g += backward(f, d / B, rnd)
        preds[i] = f["p"]
    return loss, g, preds


def sgd(P, V, g, lr, mu):
    """Momentum SGD: -> (P', V')."""
    V2 = mu * np.asarray(V, dtype=np.float64) + g
    return np.asarray(P, dtype=np.float64) - lr * V2, V2


def seed_of(p, scale: int = 2) -> np.ndarray:
    """Half-pel seed of predictions p (..., 2): 2 * clip(rint(p), -w, w),
    w the window half-width at scale f (16 at f = 2)."""
    w = half_width(scale)
    return (2 * np.clip(np.rint(np.asarray(p, dtype=np.float64)), -w, w)).astype(np.int16)


def opaque_mbs(cls):
    """(v, h) of the MBs the proposal serves: opaque ones (all when cls is None)."""
    if cls is None:
        return None
    return [tuple(x) for x in np.argwhere(np.asarray(cls) == 1)]
