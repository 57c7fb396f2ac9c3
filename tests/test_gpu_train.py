"""What training gains: the network trained by the library's own kernels on
generated CIF sequences (labels = the plain method's vectors) against the
zero predictor, the untrained network and the plain method, on held-out
sequences: prediction error, PSNR, distortion, recursion iterations and
compared blocks per MB, each printed for plain, untrained and trained."""
import numpy as np
import pytest

import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    me.lib()
    return torch


def test_trained_network_gains(torch_cuda):
    from paper_1002_1168_amd import train as T
    tr, ho = T.training_sets(120, 10, 16)
    p = me.me_default_params(search_range=16)
    dtr, dho = T.label(tr, p), T.label(ho, p)
    untrained = me.Net(synth.net_init(1))
    try:
        e0 = T.prediction_error(untrained, dho)
        ev_u = T.evaluate(dho, p, untrained)
    finally:
        untrained.close()
    net = me.Net(synth.net_init(1))
    try:
        hist = T.train(net, dtr, steps=2500, pairs_per_step=64, lr=0.03, momentum=0.9, seed=0)
        e1 = T.prediction_error(net, dho)
        ev_l = T.evaluate(dho, p, net)
    finally:
        net.close()
    ev_p = T.evaluate(dho, p, None)
    say("loss", np.mean(hist[:200]), "->", np.mean(hist[-200:]))
    say("held-out MAE: zero", e1["mae_zero"], "untrained", e0["mae_net"], "trained", e1["mae_net"])
    for name, ev in (("plain", ev_p), ("untrained seeds", ev_u), ("trained seeds", ev_l)):
        say(f"{name:16s} PSNR {ev['psnr_db']:.4f} dB  cost/MB {ev['cost_per_mb']:.2f}  "
            f"iters/MB {ev['iters_per_mb']:.4f}  points/MB {ev['points_per_mb']:.3f}")
    assert np.mean(hist[-200:]) < 0.5 * np.mean(hist[:200])
    # the trained proposal predicts the plain method's vectors far better than no motion
    assert e1["mae_net"] < 0.6 * e1["mae_zero"] and e1["mae_net"] < 0.6 * e0["mae_net"]
    # its seeds start the recursion closer: fewer iterations than the untrained seeds
    assert ev_l["iters_per_mb"] < 0.75 * ev_u["iters_per_mb"]
    # the learned form stays within the admitted PSNR loss of the plain method
    # (it gains a little here) at no higher distortion
    assert ev_l["psnr_db"] >= ev_p["psnr_db"] - 0.05
    assert ev_l["cost_per_mb"] <= ev_p["cost_per_mb"]
    # What does not hold: fewer iterations than the plain method.  The plain
    # recursion starts from the best of A, B, C and T, which already sits at
    # its fixed point for most MBs (about 0.2 iterations per MB here); the
    # seeded recursion runs whenever the rounded seed misses that point, and
    # the fallback adds the plain recursion on top.  The measured figures are
    # printed above; nothing is asserted about them.
