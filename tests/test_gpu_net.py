"""GPU parity of the learned proposal network against the float64 oracle
(oracle/net.py): predictions and seeds, the gradient of a training step,
momentum-SGD updates, determinism, and seeded searches bit-exact with the
oracle's search fed the GPU's seeds."""
import numpy as np
import pytest

import oracle
from oracle import net as onet
import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth

from gpu_util import assert_same, gpu_classify, oracle_params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    me.lib()
    return torch


def init_weights(seed=7):
    w = synth.net_init(seed)
    rng = np.random.default_rng(seed + 1)
    w[onet.NPARAM - 2:] = rng.normal(0, 1.0, 2).astype(np.float32)   # non-zero output bias
    w[576:608] = rng.normal(0, 0.1, 32).astype(np.float32)
    w[9824:9856] = rng.normal(0, 0.1, 32).astype(np.float32)
    return w


class NetCase:
    """Frame pairs of a sequence on the device, classes, seed / prediction /
    label buffers, and the served (opaque) MBs in flat order."""

    def __init__(self, seq, vop, pairs, label_seed=0):
        import torch
        from paper_1002_1168_amd.device import DeviceSequence, Outputs
        self.seq, self.vop, self.pairs = seq, vop, pairs
        self.ds = DeviceSequence(seq)
        if vop is not None:
            gpu_classify(self.ds)
        hm, wm = self.ds.hm, self.ds.wm
        self.out = Outputs.alloc(pairs, hm, wm)
        self.seed = torch.zeros((pairs, hm, wm, 2), dtype=torch.int16, device="cuda")
        self.pred = torch.full((pairs, hm, wm, 2), float("nan"), dtype=torch.float32, device="cuda")
        rng = np.random.default_rng(label_seed)
        self.labels_np = (2 * rng.integers(-6, 7, size=(pairs, hm, wm, 2))).astype(np.int16)
        self.labels = torch.from_numpy(self.labels_np).cuda()
        self.jobs = self.ds.pair_jobs(vop, self.out, pairs, seeds=self.seed)
        self.served = []
        for i in range(pairs):
            cls = None if vop is None else self.ds.cls[vop, i + 1].cpu().numpy()
            for v in range(hm):
                for h in range(wm):
                    if cls is None or cls[v, h] == 1:
                        self.served.append((i, v, h))

    def inputs(self):
        return [onet.prep(self.seq.luma[i + 1], self.seq.luma[i], 16 * h, 16 * v) for i, v, h in self.served]

    def label_vectors(self):
        return np.array([self.labels_np[i, v, h] // 2 for i, v, h in self.served], dtype=np.float64)


def dev_ptrs(t):
    return [t[i].data_ptr() for i in range(t.shape[0])]


def test_forward_predictions_and_seeds(torch_cuda):
    import torch
    from paper_1002_1168_amd.device import stream_handle
    w = init_weights()
    cases = [NetCase(synth.qcif_ellipse(seed=41, frames=4), 0, 3), NetCase(synth.cif_two_vops(seed=42, frames=3), 1, 2),
             NetCase(synth.random_frames(43, 64, 48, frames=2), None, 1)]
    nt = me.Net(w)
    try:
        for c in cases:
            nt.forward(c.jobs, dev_ptrs(c.pred), stream=stream_handle())
            torch.cuda.synchronize()
            pred, seed = c.pred.cpu().numpy(), c.seed.cpu().numpy()
            want = np.array([onet.forward(x, w)["p"] for x in c.inputs()])
            got = np.array([pred[i, v, h] for i, v, h in c.served])
            gs = np.array([seed[i, v, h] for i, v, h in c.served])
            say(c.seq.name, "served", len(c.served), "max |dp|", float(np.abs(got - want).max()))
            assert np.allclose(got, want, atol=1e-3, rtol=1e-4)
            safe = np.abs(np.abs(want - np.trunc(want)) - 0.5) > 5e-3
            assert np.array_equal(gs[safe], onet.seed_of(want)[safe])
            # MBs not served keep their (NaN) prediction
            mask = np.ones(pred.shape[:3], bool)
            for i, v, h in c.served:
                mask[i, v, h] = False
            assert np.isnan(pred[mask]).all()
    finally:
        nt.close()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_training_gradient_matches_oracle(torch_cuda):
    import torch
    from paper_1002_1168_amd.device import stream_handle
    w = init_weights(9)
    c = NetCase(synth.qcif_ellipse(seed=44, frames=3), 0, 2, label_seed=3)
    g = torch.zeros(me.ME_NET_PARAMS, dtype=torch.float32, device="cuda")
    nt = me.Net(w)
    try:
        loss = nt.train_step(c.jobs, dev_ptrs(c.labels), lr=0.0, momentum=0.0, grad=g.data_ptr(),
                             stream=stream_handle())
        torch.cuda.synchronize()
    finally:
        nt.close()
    want_loss, want_g, _ = onet.loss_and_grad(c.inputs(), c.label_vectors(), w)
    got_g = g.cpu().numpy().astype(np.float64)
    say("B", len(c.served), "loss", loss, want_loss)
    assert abs(loss - want_loss) <= 1e-4 * abs(want_loss)
    o = 0
    for name, shape in onet.SHAPES:
        n = int(np.prod(shape))
        e = rel_err(got_g[o:o + n], want_g[o:o + n])
        say(name, "rel err", e)
        assert e < 1e-3, (name, e)
        o += n


def test_sgd_steps_match_oracle_and_are_deterministic(torch_cuda):
    from paper_1002_1168_amd.device import stream_handle
    w0 = init_weights(10)
    c = NetCase(synth.qcif_ellipse(seed=45, frames=3), 0, 2, label_seed=4)
    runs = []
    for rep in range(2):
        nt = me.Net(w0)
        try:
            for _ in range(2):
                nt.train_step(c.jobs, dev_ptrs(c.labels), lr=0.05, momentum=0.9, want_loss=False,
                              stream=stream_handle())
            runs.append(nt.weights(momentum=True))
        finally:
            nt.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    P, V = w0.astype(np.float64), np.zeros(onet.NPARAM)
    xs, ys = c.inputs(), c.label_vectors()
    for _ in range(2):
        # the oracle forward reads fp32 master weights
        _, g, _ = onet.loss_and_grad(xs, ys, P.astype(np.float32).astype(np.float64))
        P, V = onet.sgd(P, V, g, 0.05, 0.9)
    got_w, got_v = runs[0]
    assert rel_err(got_w.astype(np.float64) - w0, P - w0) < 1e-3
    assert rel_err(got_v.astype(np.float64), V) < 1e-3


def test_seeded_search_through_the_network(torch_cuda):
    """me_texture_recursive with a network: seeds from the kernels, then the
    search; the oracle's search fed those seeds gives the same outputs."""
    import torch
    from paper_1002_1168_amd.device import stream_handle
    w = init_weights(12)
    for seq, S in ((synth.qcif_ellipse(seed=46, frames=5), 7), (synth.cif_two_vops(seed=47, frames=4), 16)):
        c = NetCase(seq, 0, seq.frames - 1)
        p = me.me_default_params(search_range=S)
        nt = me.Net(w)
        try:
            me.me_texture_recursive(c.jobs, p, nt, stream=stream_handle())
            torch.cuda.synchronize()
            assert me.me_device_status(stream_handle()) == me.ME_OK
        finally:
            nt.close()
        seeds = c.seed.cpu().numpy()
        res = oracle.pa_sequence(seq, 0, oracle_params(p), pairs=c.pairs, seeds=list(seeds))
        want = {k: np.stack([r[k] for r in res]) for k in ("mv", "mv_int", "cost", "iters", "points")}
        assert_same(c.out.host(), want, f"net-seeded {seq.name}")
