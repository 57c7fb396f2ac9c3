"""GPU parity of the batched frame step (``me_batch_*``): many streams of
mixed sizes, one graph launch per frame step, against the CPU oracle run
stream by stream, VOP by VOP, pair by pair (bit-exact vectors, costs,
iteration and point counts, classes, SSE and pixel counts)."""
import numpy as np
import pytest

import oracle
import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth

from gpu_util import assert_same, oracle_params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    me.lib()
    return torch


class Streams:
    """Device copies of several sequences, per-(stream, VOP) outputs for every
    pair and a zero T field for the first step.  ``rect`` adds a rectangular
    (no alpha) job on the luma of each listed stream."""

    def __init__(self, seqs, pairs, rect=()):
        import torch
        from paper_1002_1168_amd.device import DeviceSequence, Outputs
        self.seqs, self.pairs = seqs, pairs
        self.ds = [DeviceSequence(s) for s in seqs]
        self.units = [(si, v) for si, s in enumerate(seqs) for v in range(s.vops)] + [(si, None) for si in rect]
        self.out = [Outputs.alloc(pairs, self.ds[si].hm, self.ds[si].wm) for si, _ in self.units]
        self.zero = [torch.zeros((self.ds[si].hm, self.ds[si].wm, 2), dtype=torch.int16, device="cuda")
                     for si, _ in self.units]

    def jobs(self, i, outs=None):
        """Jobs of frame step i (pair (i, i+1)); T = the previous step's mv_int."""
        from paper_1002_1168_amd.device import job
        outs = self.out if outs is None else outs
        js = []
        for u, (si, v) in enumerate(self.units):
            d = self.ds[si]
            t = i + 1
            tf = outs[u].mv_int[i - 1] if i > 0 else self.zero[u]
            if v is None:
                js.append(job(d.luma[t], d.luma[t - 1], None, None, None, tf, outs[u], i))
            else:
                js.append(job(d.luma[t], d.luma[t - 1], d.alpha[v, t], d.alpha[v, t - 1], d.cls[v, t], tf,
                              outs[u], i))
        return js

    def oracle(self, params, shape_only=False):
        want = []
        for si, v in self.units:
            res = oracle.pa_sequence(self.seqs[si], v, oracle_params(params), shape_only=shape_only,
                                     pairs=self.pairs)
            want.append(res)
        return want


def check_step(st: Streams, i, want, sums, label):
    sse, npx, _, _ = sums
    for u, (si, v) in enumerate(st.units):
        got = {k: a[i:i + 1] for k, a in st.out[u].host().items()}
        w = {k: want[u][i][k][None] for k in ("mv", "mv_int", "cost", "iters", "points")}
        assert_same(got, w, f"{label} step {i} stream {si} vop {v}")
        if v is not None:
            cls = st.ds[si].cls[v, i + 1].cpu().numpy()
            assert np.array_equal(cls, want[u][i]["cls"]), f"{label} step {i} stream {si} vop {v}: classes"
        assert sse[u] == want[u][i]["sse"] and npx[u] == want[u][i]["npix"], f"{label} step {i} unit {u}: SSE"


def run_batch(st: Streams, params, flags=0, label="batch"):
    import torch
    from paper_1002_1168_amd.device import stream_handle
    want = st.oracle(params, shape_only=bool(flags & me.ME_BATCH_SHAPE))
    s = stream_handle()
    b = me.Batch(st.jobs(0), params, flags, stream=s)
    try:
        say(label, "config", b.config())
        for i in range(st.pairs):
            say(label, "step", i)
            b.step(st.jobs(i))
            sums = b.results(check=False)
            assert sums[3] in (me.ME_OK, me.ME_EEMPTY), sums[3]
            check_step(st, i, want, sums, label)
    finally:
        b.close()
    torch.cuda.synchronize()
    return want


def test_batch_mixed_streams_plain(torch_cuda):
    seqs = synth.mixed_streams(seed=21, frames=5, counts=(2, 2, 1))
    st = Streams(seqs, 4, rect=(0, 2))
    run_batch(st, me.me_default_params(search_range=16), label="mixed")


def test_batch_autotuned_same_results(torch_cuda):
    seqs = synth.mixed_streams(seed=22, frames=4, counts=(1, 2, 1))
    st = Streams(seqs, 3)
    run_batch(st, me.me_default_params(search_range=16), me.ME_BATCH_AUTOTUNE, label="tuned")


def test_batch_shape_mode(torch_cuda):
    seqs = synth.mixed_streams(seed=23, frames=4, counts=(2, 1, 0))
    st = Streams(seqs, 3)
    run_batch(st, me.me_default_params(search_range=16), me.ME_BATCH_SHAPE, label="shape")


def test_batch_small_range_half_pel(torch_cuda):
    seqs = [synth.qcif_ellipse(seed=24, frames=5), synth.cif_two_vops(seed=25, frames=5)]
    p = me.me_default_params(search_range=7, half_pel=1)
    st = Streams(seqs, 4, rect=(1,))
    run_batch(st, p, label="s7-half")


def test_batch_replays_with_eager_work_between(torch_cuda):
    """Every replay of the graph against the eager entry points on the same
    step, with eager launches and synchronisations between the replays."""
    import torch
    from paper_1002_1168_amd.device import Outputs, stream_handle
    seqs = synth.mixed_streams(seed=26, frames=6, counts=(1, 1, 1))
    st = Streams(seqs, 5)
    p = me.me_default_params(search_range=16)
    eager_out = [Outputs.alloc(st.pairs, st.ds[si].hm, st.ds[si].wm) for si, _ in st.units]
    s = stream_handle()
    b = me.Batch(st.jobs(0), p, 0, stream=s)
    try:
        for i in range(st.pairs):
            b.step(st.jobs(i))
            bsum = b.results(check=False)
            # eager: the same step into separate outputs (classes already written)
            ej = st.jobs(i, eager_out)
            me.me_texture_recursive(ej, p, None, stream=s)
            esum = me.me_motion_compensate_psnr(ej, stream=s, check=False)
            assert bsum[3] == esum[3]
            torch.cuda.synchronize()
            for u in range(len(st.units)):
                g = {k: a[i:i + 1] for k, a in st.out[u].host().items()}
                e = {k: a[i:i + 1] for k, a in eager_out[u].host().items()}
                assert_same(g, e, f"replay {i} unit {u}")
            assert bsum[0] == esum[0] and bsum[1] == esum[1], f"replay {i}: SSE"
    finally:
        b.close()


def test_batch_rejects_other_structure(torch_cuda):
    seqs = synth.mixed_streams(seed=27, frames=3, counts=(1, 1, 0))
    st = Streams(seqs, 2)
    p = me.me_default_params(search_range=16)
    from paper_1002_1168_amd.device import stream_handle
    b = me.Batch(st.jobs(0), p, 0, stream=stream_handle())
    try:
        js = st.jobs(1)
        assert b.step(js[:-1], check=False) == me.ME_EINVAL          # fewer jobs
        js2 = st.jobs(1)
        js2[0].t_field = None                                         # T presence differs
        assert b.step(js2, check=False) == me.ME_EINVAL
        assert b.step(st.jobs(1), check=False) == me.ME_OK
        assert b.results(check=False)[3] in (me.ME_OK, me.ME_EEMPTY)   # a VOP may be empty in a frame
    finally:
        b.close()


@pytest.mark.parametrize("S,half,scale", [(16, 0, 2), (32, 1, 4)])
def test_batch_with_proposal_network(torch_cuda, S, half, scale):
    """A network attached to the batch: every step's seeds and results equal
    the eager network-seeded search, and the oracle's search fed those seeds
    (S=16 with the default window; S=32 with half-sample refinement and the
    scale-4 window, the setting of the 1920x1088 workload)."""
    import torch
    from paper_1002_1168_amd.device import Outputs, job, stream_handle
    seqs = synth.mixed_streams(seed=28, frames=4, counts=(1, 1, 1))
    st = Streams(seqs, 3)
    p = me.me_default_params(search_range=S, half_pel=half)
    w = synth.net_init(5)
    w[-2:] = [0.7, -1.3] if scale == 2 else [19.6, -27.2]
    seeds = [torch.zeros((st.pairs, st.ds[si].hm, st.ds[si].wm, 2), dtype=torch.int16, device="cuda")
             for si, _ in st.units]
    eager_out = [Outputs.alloc(st.pairs, st.ds[si].hm, st.ds[si].wm) for si, _ in st.units]
    eager_seeds = [torch.zeros_like(x) for x in seeds]

    def jobs(i, outs, sd):
        js = st.jobs(i, outs)
        for u, j in enumerate(js):
            j.seed = sd[u][i].data_ptr()
        return js

    s = stream_handle()
    net = me.Net(w, scale=scale)
    b = me.Batch(jobs(0, st.out, seeds), p, 0, stream=s)
    try:
        b.set_net(net)
        for i in range(st.pairs):
            b.step(jobs(i, st.out, seeds))
            b.results(check=False)
            me.me_texture_recursive(jobs(i, eager_out, eager_seeds), p, net, stream=s)
            torch.cuda.synchronize()
            for u in range(len(st.units)):
                assert torch.equal(seeds[u][i], eager_seeds[u][i]), f"step {i} unit {u}: seeds"
                g = {k: a[i:i + 1] for k, a in st.out[u].host().items()}
                e = {k: a[i:i + 1] for k, a in eager_out[u].host().items()}
                assert_same(g, e, f"net batch step {i} unit {u}")
    finally:
        b.close()
        net.close()
    for u, (si, v) in enumerate(st.units):
        res = oracle.pa_sequence(st.seqs[si], v, oracle_params(p), pairs=st.pairs,
                                 seeds=list(seeds[u].cpu().numpy()))
        want = {k: np.stack([r[k] for r in res]) for k in ("mv", "mv_int", "cost", "iters", "points")}
        assert_same(st.out[u].host(), want, f"net batch unit {u} vs oracle")


def forced_configs(nlines, cap16, plan_ok, rows_cap=0):
    """Every launch configuration the autotuner can pick for a batch of
    `nlines` lines: line workers with waves 1 / 2 / 4, workers cap, cap/2,
    cap/4 (at least 1), staging plan / generic, poll back-off 1 / 2 / 4
    (one-wave workers only); row workers (rows_cap > 0: the resident
    workgroup count) with cap, cap/2 and a single workgroup, both stagings,
    back-off 1 / 2."""
    out = []
    stagings = ("plan", "generic") if plan_ok else ("generic",)
    for waves in (1, 2, 4):
        cap = min(nlines, cap16 // waves)
        for w in sorted({cap, max(cap // 2, 1), max(cap // 4, 1)}, reverse=True):
            for staging in stagings:
                for sleep in ((1, 2, 4) if waves == 1 else (1,)):
                    out.append({"workers": w, "staging": staging, "poll_sleep": sleep, "flat_per_cu": 8,
                                "waves_per_line": waves, "search": "lines"})
    if rows_cap:
        for w in sorted({rows_cap, max(rows_cap // 2, 1), 1}, reverse=True):
            for staging in stagings:
                for sleep in (1, 2):
                    out.append({"workers": w, "staging": staging, "poll_sleep": sleep, "flat_per_cu": 8,
                                "waves_per_line": 4, "search": "rows"})
    return out


def test_batch_every_forced_config_matches_oracle(torch_cuda):
    # the configurations the autotuner chooses between, each forced and
    # checked against the oracle on the same mixed-size streams (the generic
    # staging loop and the reduced worker counts included)
    import torch
    from paper_1002_1168_amd.device import stream_handle
    seqs = synth.mixed_streams(seed=26, frames=3, counts=(1, 1, 1))
    st = Streams(seqs, 2, rect=(1,))
    p = me.me_default_params(search_range=16)
    want = st.oracle(p)
    s = stream_handle()
    b = me.Batch(st.jobs(0), p, 0, stream=s)
    try:
        cap16 = torch.cuda.get_device_properties(0).multi_processor_count * 16
        nlines = sum(st.ds[si].hm * st.ds[si].wm for si, _ in st.units)
        cfg0 = b.config()
        assert cfg0["search"] == "rows"          # the default for a set without chains
        cfgs = forced_configs(nlines, cap16, plan_ok=True, rows_cap=cfg0["workers"])
        assert len(cfgs) >= 30
        for cfg in cfgs:
            say("forced config", cfg)
            b.set_config(cfg)
            assert b.config() == cfg
            for i in range(st.pairs):
                for o in st.out:   # a stale result must not pass (pair i only: i-1 is this step's T)
                    o.mv[i].fill_(0x5555)
                    o.mv_int[i].fill_(0x5555)
                b.step(st.jobs(i))
                sums = b.results(check=False)
                assert sums[3] in (me.ME_OK, me.ME_EEMPTY), (cfg, sums[3])
                check_step(st, i, want, sums, f"forced {cfg}")
        bad = dict(cfgs[0], waves_per_line=3)
        assert b.set_config(bad, check=False) == me.ME_EINVAL
        bad = dict(cfgs[0], workers=0)
        assert b.set_config(bad, check=False) == me.ME_EINVAL
    finally:
        b.close()
    torch.cuda.synchronize()


def test_batch_graph_kernel_timing(torch_cuda):
    # with timing on at capture, every replay records the search and MC
    # kernels' events inside the graph; the sums count every replay
    import torch
    from paper_1002_1168_amd.device import stream_handle
    seqs = synth.mixed_streams(seed=27, frames=3, counts=(1, 1, 0))
    st = Streams(seqs, 2)
    p = me.me_default_params(search_range=16)
    s = stream_handle()
    me.me_kernel_timing(True, kinds=[me.ME_KT_SEARCH, me.ME_KT_MC])
    try:
        b = me.Batch(st.jobs(0), p, 0, stream=s)
    finally:
        me.me_kernel_timing(False)
    try:
        for r in range(5):
            b.step(st.jobs(r % st.pairs))
        ms, cnt = b.kernel_time_ms(me.ME_KT_SEARCH)
        ms_mc, cnt_mc = b.kernel_time_ms(me.ME_KT_MC)
        assert cnt == 5 and cnt_mc == 5, (cnt, cnt_mc)
        assert 0 < ms < 1000 and 0 < ms_mc < 1000
        assert b.kernel_time_ms(me.ME_KT_CLASSIFY) == (0.0, 0)   # not timed
        assert b.kernel_time_ms(me.ME_KT_SEARCH) == (0.0, 0)     # restarted
        # results are unchanged by the timing nodes
        want = st.oracle(p)
        for i in range(st.pairs):
            b.step(st.jobs(i))
            sums = b.results(check=False)
            check_step(st, i, want, sums, "timed graph")
        assert b.kernel_time_ms(me.ME_KT_SEARCH)[1] == st.pairs
        # re-capture without timing: one graph, nothing recorded
        b.set_config(b.config())
        b.step(st.jobs(0))
        assert b.kernel_time_ms(me.ME_KT_SEARCH) == (0.0, 0)
    finally:
        b.close()
    torch.cuda.synchronize()


def test_batch_masked_prs(torch_cuda):
    # the masked-luma recursion of boundary MBs in the batched frame step
    # (row workers), with and without T on texture
    seqs = synth.mixed_streams(seed=29, frames=4, counts=(1, 2, 1))
    st = Streams(seqs, 3)
    for flags in (me.ME_FLAG_MASKED_PRS, me.ME_FLAG_MASKED_PRS | me.ME_FLAG_T_TEXTURE):
        run_batch(st, me.me_default_params(search_range=16, flags=flags), label=f"masked prs {flags}")


def test_batch_t_on_texture(torch_cuda):
    # the Section 3.1 text reading in the batched frame step (row workers)
    seqs = synth.mixed_streams(seed=28, frames=4, counts=(1, 2, 1))
    st = Streams(seqs, 3)
    run_batch(st, me.me_default_params(search_range=16, flags=me.ME_FLAG_T_TEXTURE), label="t-texture")
