"""GPU parity of the learned proposal network against the float64 oracle
(oracle/net.py), at window scales 2 and 4: predictions and seeds, the
gradient (me_net_backward) element by element, momentum-SGD updates element
by element, the split backward + SGD step against the fused step, checkpoint
round trips, determinism, and seeded searches (half-pel at S=32 included)
bit-exact with the oracle's search fed the GPU's seeds.

Tolerances (derived from the arithmetic): the GPU and the oracle round to
bfloat16 at the same points, so they differ by the order of fp32 sums
(against fp64) over at most 576 terms of bounded bf16 products - relative
error about 1e-6 - and, rarely, by a one-ulp bf16 flip (2^-8) of a single
activation or pre-activation gradient among thousands.  Such a flip moves a
gradient element by about 2^-8 of one of the ~100 terms of its sum.  The
element-wise bound |g - r| <= 2e-3 max|r| + 1e-2 |r| (per tensor) holds with
a wide margin; predictions use 1e-3 absolute."""
import numpy as np
import pytest

import oracle
from oracle import net as onet
import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth

from gpu_util import assert_same, gpu_classify, oracle_params, say
from test_checkpoint_files import parse as parse_checkpoint

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

    def __init__(self, seq, vop, pairs, label_seed=0, scale=2):
        import torch
        from paper_1002_1168_amd.device import DeviceSequence, Outputs
        self.seq, self.vop, self.pairs, self.scale = seq, vop, pairs, scale
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
        return [onet.prep(self.seq.luma[i + 1], self.seq.luma[i], 16 * h, 16 * v, scale=self.scale)
                for i, v, h in self.served]

    def label_vectors(self):
        return np.array([self.labels_np[i, v, h] // 2 for i, v, h in self.served], dtype=np.float64)


def dev_ptrs(t):
    return [t[i].data_ptr() for i in range(t.shape[0])]


@pytest.mark.parametrize("scale", [2, 4])
def test_forward_predictions_and_seeds(torch_cuda, scale):
    import torch
    from paper_1002_1168_amd.device import stream_handle
    w = init_weights()
    if scale == 4:   # a larger output bias, so that seeds reach past +-16
        w[onet.NPARAM - 2:] = [21.3, -33.6]
    cases = [NetCase(synth.qcif_ellipse(seed=41, frames=4), 0, 3, scale=scale),
             NetCase(synth.cif_two_vops(seed=42, frames=3), 1, 2, scale=scale),
             NetCase(synth.random_frames(43, 64, 48, frames=2), None, 1, scale=scale)]
    nt = me.Net(w, scale=scale)
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
            assert np.array_equal(gs[safe], onet.seed_of(want, scale)[safe])
            # MBs not served keep their (NaN) prediction
            mask = np.ones(pred.shape[:3], bool)
            for i, v, h in c.served:
                mask[i, v, h] = False
            assert np.isnan(pred[mask]).all()
    finally:
        nt.close()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def check_elementwise(got, want, what, atol=2e-3, rtol=1e-2):
    """|got - want| <= atol * max|want| + rtol * |want|, tensor by tensor."""
    o = 0
    for name, shape in onet.SHAPES:
        n = int(np.prod(shape))
        g, w = got[o:o + n], want[o:o + n]
        bound = atol * float(np.abs(w).max()) + rtol * np.abs(w)
        worst = float((np.abs(g - w) / np.maximum(bound, 1e-30)).max())
        say(what, name, "worst / bound", worst, "rel L2", rel_err(g, w))
        assert (np.abs(g - w) <= bound).all(), (what, name, worst)
        o += n


@pytest.mark.parametrize("scale", [2, 4])
def test_training_gradient_matches_oracle(torch_cuda, scale):
    import torch
    from paper_1002_1168_amd.device import stream_handle
    w = init_weights(9)
    c = NetCase(synth.qcif_ellipse(seed=44, frames=3), 0, 2, label_seed=3, scale=scale)
    g = torch.zeros(me.ME_NET_PARAMS, dtype=torch.float32, device="cuda")
    nt = me.Net(w, scale=scale)
    try:
        loss = nt.backward(c.jobs, dev_ptrs(c.labels), g.data_ptr(), stream=stream_handle())
        torch.cuda.synchronize()
        assert np.array_equal(nt.weights(), w)   # backward leaves the weights alone
    finally:
        nt.close()
    want_loss, want_g, _ = onet.loss_and_grad(c.inputs(), c.label_vectors(), w)
    got_g = g.cpu().numpy().astype(np.float64)
    say("B", len(c.served), "loss", loss, want_loss)
    assert abs(loss - want_loss) <= 1e-4 * abs(want_loss)
    check_elementwise(got_g, want_g, f"gradient scale {scale}")


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
    check_elementwise(got_w.astype(np.float64) - w0, P - w0, "two SGD steps: weight change")
    check_elementwise(got_v.astype(np.float64), V, "two SGD steps: momentum")


def test_backward_then_sgd_step_is_the_fused_step(torch_cuda):
    """me_net_backward + me_net_sgd_step give bit for bit the weights,
    momentum and gradient of me_net_train_step."""
    import torch
    from paper_1002_1168_amd.device import stream_handle
    w0 = init_weights(13)
    c = NetCase(synth.cif_two_vops(seed=48, frames=3), 0, 2, label_seed=5)
    g1 = torch.zeros(me.ME_NET_PARAMS, dtype=torch.float32, device="cuda")
    g2 = torch.zeros_like(g1)
    a, b = me.Net(w0), me.Net(w0)
    try:
        for _ in range(3):
            la = a.train_step(c.jobs, dev_ptrs(c.labels), lr=0.02, momentum=0.8, grad=g1.data_ptr(),
                              stream=stream_handle())
            lb = b.backward(c.jobs, dev_ptrs(c.labels), g2.data_ptr(), stream=stream_handle())
            b.sgd_step(g2.data_ptr(), lr=0.02, momentum=0.8, stream=stream_handle())
            torch.cuda.synchronize()
            assert la == lb and torch.equal(g1, g2)
        wa, va = a.weights(momentum=True)
        wb, vb = b.weights(momentum=True)
        assert np.array_equal(wa, wb) and np.array_equal(va, vb)
        with pytest.raises(me.MeError):
            b.sgd_step(g2.data_ptr(), lr=0.02, momentum=1.0)
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("scale", [2, 4])
def test_checkpoint_round_trip(torch_cuda, scale, tmp_path):
    """me_net_save / me_net_load: weights, momentum and window scale come back
    bit for bit and give the same predictions; a flipped byte is refused."""
    import torch
    from paper_1002_1168_amd.device import stream_handle
    c = NetCase(synth.qcif_ellipse(seed=49, frames=3), 0, 2, label_seed=6, scale=scale)
    net = me.Net(init_weights(14), scale=scale)
    path = str(tmp_path / "net.menet")
    try:
        net.train_step(c.jobs, dev_ptrs(c.labels), lr=0.01, momentum=0.9, want_loss=False, stream=stream_handle())
        net.save(path)
        back = me.Net.load(path)
        try:
            assert back.scale == scale
            w1, v1 = net.weights(momentum=True)
            w2, v2 = back.weights(momentum=True)
            assert np.array_equal(w1, w2) and np.array_equal(v1, v2) and np.abs(v1).max() > 0
            p1 = torch.full_like(c.pred, float("nan"))
            p2 = torch.full_like(c.pred, float("nan"))
            net.forward(c.jobs, dev_ptrs(p1), stream=stream_handle())
            back.forward(c.jobs, dev_ptrs(p2), stream=stream_handle())
            torch.cuda.synchronize()
            assert torch.equal(torch.nan_to_num(p1, 1e9), torch.nan_to_num(p2, 1e9))
        finally:
            back.close()
    finally:
        net.close()
    # the file read back with plain Python: header, standard FNV-1a 64 checksum, payload
    fscale, fw, fv = parse_checkpoint(path)
    assert fscale == scale and np.array_equal(fw, w1) and np.array_equal(fv, v1)
    raw = bytearray(open(path, "rb").read())
    raw[24 + 4 * 100] ^= 0x01
    bad = tmp_path / "bad.menet"
    bad.write_bytes(bytes(raw))
    with pytest.raises(me.MeError) as e:
        me.Net.load(str(bad))
    assert e.value.code == me.ME_EFORMAT


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


def hd_crop(frames=3, vops=3):
    seq = synth.hd_streams(frames=frames, streams=1)[0]
    ys, xs = np.nonzero(seq.alpha[0, 1])
    y0 = int(np.clip((ys.mean() - 160) // 16 * 16, 0, seq.height - 320))
    x0 = int(np.clip((xs.mean() - 192) // 16 * 16, 0, seq.width - 384))
    seq.luma = np.ascontiguousarray(seq.luma[:, y0:y0 + 320, x0:x0 + 384])
    seq.alpha = np.ascontiguousarray(seq.alpha[:vops, :, y0:y0 + 320, x0:x0 + 384])
    return seq


@pytest.mark.parametrize("scale", [2, 4])
def test_seeded_half_pel_search_s32(torch_cuda, scale):
    """The network-seeded search with half-sample refinement at S=32 (the
    setting of the 1920x1088 workload) on a crop of a 1920x1088 stream: the
    oracle's search fed the GPU's seeds gives the same outputs."""
    import torch
    from paper_1002_1168_amd.device import stream_handle
    seq = hd_crop()
    w = init_weights(15)
    w[onet.NPARAM - 2:] = [9.4, -14.2] if scale == 2 else [23.6, -28.3]
    p = me.me_default_params(search_range=32, half_pel=1)
    for v in range(seq.vops):
        c = NetCase(seq, v, seq.frames - 1, scale=scale)
        nt = me.Net(w, scale=scale)
        try:
            me.me_texture_recursive(c.jobs, p, nt, stream=stream_handle())
            torch.cuda.synchronize()
            assert me.me_device_status(stream_handle()) == me.ME_OK
        finally:
            nt.close()
        seeds = c.seed.cpu().numpy()
        served = [seeds[i, vv, h] for i, vv, h in c.served]
        if scale == 4 and served:
            assert np.abs(np.array(served)).max() > 32   # seeds past the scale-2 clamp
        res = oracle.pa_sequence(seq, v, oracle_params(p), pairs=c.pairs, seeds=list(seeds))
        want = {k: np.stack([r[k] for r in res]) for k in ("mv", "mv_int", "cost", "iters", "points")}
        assert_same(c.out.host(), want, f"net-seeded half-pel S=32 scale {scale} vop {v}")
