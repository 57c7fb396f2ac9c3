#!/usr/bin/env python3
"""Throughput of the shape-adaptive motion estimator on one MI355X.

Workload (default): CIF 352x288, 300 frames, two VOPs (a polygon and an
ellipse with occlusion over a panning background), search range +-16,
seeded synthetic data resident in HBM.  One timed step is one pass of the
paper's path over the whole sequence: MB classification of every VOP frame,
the proposed block/pel-recursive search for all 2 x 299 frame pairs (one
pipelined launch), and motion compensation + PSNR.  `value` counts grid MBs
of every (VOP, frame pair) per second.  The baselines (ES, TSS, DS) run on
the same frames and are timed the same way, reported under "baselines".

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
CUS, CLOCK_GHZ = 256, 2.4
PEAK_INT_TOPS = CUS * 4 * 16 * CLOCK_GHZ / 1000.0   # 32-bit VALU lane-ops/s (T), 39.3

PEAK_BF16_TFLOPS = 2500.0   # dense bf16 MFMA
# proposal network forward per MB: conv1 24x24x32x18, conv2 12x12x32x288, conv3 6x6x2x288 multiply-adds
NET_FWD_FLOP = 2 * (576 * 32 * 18 + 144 * 32 * 288 + 36 * 2 * 288)

# algorithmic VALU lane-ops of the proposed method per searched MB
SAD_OPS = 64          # 256 absolute differences, 4 per v_sad_u8 lane-op
PASS_OPS = 256 * 12   # gradient pass: e, gx, gy, two reciprocal lookups, two products, two counts, ...


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel: str, sources, summary: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 PMC
    summary, or None when the kernel's sources changed since it was taken."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in sources:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        with open(os.path.join(ROOT, summary)) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    for ln in lines:
        t = ln.split()
        if len(t) == 4 and t[0] == "traffic" and t[1] == kernel:
            kv = dict(x.split("=", 1) for x in t[2:])
            if kv.get("source_sha256") == h.hexdigest():
                return int(kv["bytes_per_launch"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-baselines", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-stream batched frame-step measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-seed measurement")
    ap.add_argument("--no-hd", action="store_true",
                    help="skip the 8-stream 1920x1088 batched measurement (plain and network-seeded)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the 64-stream batched measurement (for profiling) and print it")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 3 device copies of this many MiB (calibrates the HBM byte counters) and exit")
    return ap.parse_args()


class Workload:
    """Device buffers and job lists of the CIF two-VOP sequence."""

    def __init__(self, frames: int):
        import paper_1002_1168_amd as me
        from paper_1002_1168_amd import device as dv
        from paper_1002_1168_amd import synth
        self.me, self.dv = me, dv
        t0 = time.time()
        self.seq = synth.cif_two_vops(seed=2, frames=frames)
        log(f"generated {self.seq.name} {self.seq.width}x{self.seq.height} x{frames} in {time.time() - t0:.1f}s")
        self.ds = dv.DeviceSequence(self.seq)
        self.S = self.seq.search_range
        self.params = me.me_default_params(search_range=self.S)
        self.pairs = frames - 1
        self.V = self.seq.vops
        fr, cp, bp = self.ds.classify_frames()
        self.cls_frames = (me.me_frame * len(fr))(*fr)
        self.cls_ptrs = (C.c_void_p * len(cp))(*cp)
        self.bab_ptrs = (C.c_void_p * len(bp))(*bp)
        self.out = [dv.Outputs.alloc(self.pairs, self.ds.hm, self.ds.wm) for _ in range(self.V)]
        self.jobs = me.job_array([j for v in range(self.V) for j in self.ds.pair_jobs(v, self.out[v], self.pairs)])
        self.base_out = {m: [dv.Outputs.alloc(self.pairs, self.ds.hm, self.ds.wm) for _ in range(self.V)]
                         for m in (me.ME_ES, me.ME_TSS, me.ME_DS)}
        self.base_jobs = {m: me.job_array([j for v in range(self.V)
                                           for j in self.ds.pair_jobs(v, o[v], self.pairs, chained=False)])
                          for m, o in self.base_out.items()}
        self.grid_mbs = self.V * self.pairs * self.ds.hm * self.ds.wm

    def step(self, stream, ring, slot):
        """classify -> proposed search -> MC/SSE (sums read back by `ring`)."""
        me = self.me
        me.me_classify_babs(self.cls_frames, self.cls_ptrs, self.bab_ptrs, stream=stream)
        me.me_texture_recursive(self.jobs, self.params, None, stream=stream)
        ring.queue(self.jobs, slot, stream)

    def baseline_step(self, method, stream, ring, slot):
        me = self.me
        me.me_full_search(method, self.base_jobs[method], self.params, stream=stream)
        ring.queue(self.base_jobs[method], slot, stream)


class SumsRing:
    """Per-job (SSE, pixel count) sums of two frame steps, written by
    me_motion_compensate_sse straight into pinned host memory, so that one
    step's PSNR is read while the next step runs (no copy kernel)."""

    def __init__(self, torch, me, n):
        self.me = me
        self.host = [torch.zeros(2 * n, dtype=torch.int64, pin_memory=True) for _ in range(2)]
        self.ev = [torch.cuda.Event() for _ in range(2)]

    def queue(self, jobs, slot, stream):
        """MC/SSE of `jobs` on `stream`, which must be torch's current stream
        (the event follows it there)."""
        self.me.me_motion_compensate_sse(jobs, self.host[slot].data_ptr(), stream=stream)
        self.ev[slot].record()

    def result(self, slot):
        """-> (sse list, npix list, psnr_db list, status) of the step in `slot`."""
        self.ev[slot].synchronize()
        s = self.host[slot].numpy().view(np.uint64)
        sse, npx = s[0::2].copy(), s[1::2].copy()
        with np.errstate(divide="ignore", invalid="ignore"):
            ps = 10.0 * np.log10(255.0 * 255.0 * npx.astype(np.float64) / sse.astype(np.float64))
        ps[npx == 0] = np.nan
        rc = self.me.ME_EEMPTY if (npx == 0).any() else self.me.ME_OK
        return [int(x) for x in sse], [int(x) for x in npx], [float(x) for x in ps], rc


class MixedWorkload:
    """64 streams (24 QCIF, 24 CIF, 16 4CIF 704x576), 1-4 VOPs each, S=16:
    one batched frame step = every (stream, VOP) pair of one frame step."""

    def __init__(self, frames=31, counts=(24, 24, 16)):
        import torch
        import paper_1002_1168_amd as me
        from paper_1002_1168_amd import device as dv
        from paper_1002_1168_amd import synth
        self.me, self.dv = me, dv
        t0 = time.time()
        self.seqs = synth.mixed_streams(seed=3, frames=frames, counts=counts)
        log(f"generated {len(self.seqs)} mixed streams x{frames} frames in {time.time() - t0:.1f}s")
        self.pairs = frames - 1
        self.ds = [dv.DeviceSequence(q) for q in self.seqs]
        self.units = [(si, v) for si, q in enumerate(self.seqs) for v in range(q.vops)]
        self.out = [dv.Outputs.alloc(self.pairs, self.ds[si].hm, self.ds[si].wm) for si, _ in self.units]
        self.zero = [torch.zeros((self.ds[si].hm, self.ds[si].wm, 2), dtype=torch.int16, device="cuda")
                     for si, _ in self.units]
        self.params = me.me_default_params(search_range=16)
        self.steps = [me.job_array(self.jobs(i)) for i in range(self.pairs)]
        self.grid_mbs = sum(self.ds[si].hm * self.ds[si].wm for si, _ in self.units)
        self.layer_mbs = sum(d.hm * d.wm for d in self.ds)

    def jobs(self, i, chained_in_call=False):
        """Jobs of frame step i; T = the previous step's mv_int (zero at step 0)."""
        js = []
        for u, (si, v) in enumerate(self.units):
            d, t = self.ds[si], i + 1
            tf = self.out[u].mv_int[i - 1] if i > 0 else (None if chained_in_call else self.zero[u])
            js.append(self.dv.job(d.luma[t], d.luma[t - 1], d.alpha[v, t], d.alpha[v, t - 1], d.cls[v, t], tf,
                                  self.out[u], i))
        return js


def learned_measurement(wl, torch, steps, warmup, plain_psnr, plain_iters):
    """The same CIF step with the proposal network seeding the recursion
    (weights trained by paper_1002_1168_amd.train on generated CIF
    sequences): classification, network forward, seeded search, MC/PSNR."""
    me, dv = wl.me, wl.dv
    path = os.path.join(ROOT, "paper_1002_1168_amd", "weights", "proposal_cif_s16.npy")
    if not os.path.exists(path):
        return None
    net = me.Net(np.load(path, allow_pickle=False))
    stream = dv.stream_handle()
    outs = [dv.Outputs.alloc(wl.pairs, wl.ds.hm, wl.ds.wm) for _ in range(wl.V)]
    seeds = [torch.zeros((wl.pairs, wl.ds.hm, wl.ds.wm, 2), dtype=torch.int16, device="cuda") for _ in range(wl.V)]
    jobs = me.job_array([j for v in range(wl.V) for j in wl.ds.pair_jobs(v, outs[v], wl.pairs, seeds=seeds[v])])

    ring = SumsRing(torch, me, len(jobs))

    def step(slot):
        me.me_classify_babs(wl.cls_frames, wl.cls_ptrs, wl.bab_ptrs, stream=stream)
        me.me_texture_recursive(jobs, wl.params, net, stream=stream)
        ring.queue(jobs, slot, stream)

    dt, net_ms, res = timed(step, ring, steps, warmup, torch, me, stream, me.ME_KT_NET)
    assert me.me_device_status(stream) == me.ME_OK
    net.close()
    classes = wl.ds.cls[:, 1:].cpu().numpy()
    served = int((classes == 1).sum())
    tflops = served * NET_FWD_FLOP / (net_ms * 1e-3) / 1e12
    pts, its, n = summarize(outs, classes)
    psnr = float(np.mean(res[2]))
    out = {"mb_per_s": wl.grid_mbs * steps / dt, "ms_per_step": 1000.0 * dt / steps, "psnr_db": psnr,
           "psnr_delta_vs_plain_db": psnr - plain_psnr, "iters_per_mb": its / max(n, 1),
           "iters_per_mb_plain": plain_iters, "points_per_mb": pts / max(n, 1),
           "admitted": bool(psnr >= plain_psnr - 0.05), "weights": "paper_1002_1168_amd/weights/proposal_cif_s16.npy",
           "network_forward": {"kernel_ms": net_ms, "mbs": served, "bound": "mfma", "achieved": tflops,
                               "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": tflops / PEAK_BF16_TFLOPS}}
    log(f"learned seeds: {out['mb_per_s'] / 1e6:.1f} M MB/s, PSNR {psnr:.3f} dB ({out['psnr_delta_vs_plain_db']:+.4f}), "
        f"iters/MB {out['iters_per_mb']:.3f}; network forward {net_ms:.3f} ms for {served} MBs = {tflops:.1f} TFLOP/s")
    return out


def batched_measurement(torch, steps, warmup):
    """Per-frame-step graph launches over the mixed streams, and the same
    frames as one pipelined launch over all steps."""
    me = __import__("paper_1002_1168_amd")
    mw = MixedWorkload()
    stream = mw.dv.stream_handle()
    b = me.Batch(mw.steps[0], mw.params, me.ME_BATCH_AUTOTUNE, stream=stream)
    cfg = b.config()
    n = len(mw.steps)
    for i in range(max(warmup, n)):   # one pass over every step's job table first
        b.step(mw.steps[i % n])
    torch.cuda.synchronize()
    k = max(steps, 3 * n)
    t0 = time.perf_counter()
    for i in range(k):
        b.step(mw.steps[i % n])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    status = b.results(check=False)[3]
    assert status in (me.ME_OK, me.ME_EEMPTY), status
    b.close()
    per_step = {"mb_per_s": mw.grid_mbs * k / dt, "ms_per_frame_step": 1000.0 * dt / k, "frame_steps": k,
                "config": cfg}
    # all frame steps of all streams in one pipelined launch (T chained in the call)
    allj = me.job_array([j for i in range(n) for j in mw.jobs(i, chained_in_call=True)])
    for _ in range(2):
        me.me_texture_recursive(allj, mw.params, None, stream=stream)
    torch.cuda.synchronize()
    reps = max(steps // 4, 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        me.me_texture_recursive(allj, mw.params, None, stream=stream)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    assert me.me_device_status(stream) == me.ME_OK
    pipelined = {"mb_per_s": mw.grid_mbs * n * reps / dtp, "ms_per_launch": 1000.0 * dtp / reps,
                 "frame_steps_per_launch": n, "search_only": True}
    log(f"batched mixed streams: {per_step['mb_per_s'] / 1e6:.1f} M MB/s per-step graph "
        f"({per_step['ms_per_frame_step']:.3f} ms/step, cfg {cfg}); pipelined search over {n} steps "
        f"{pipelined['mb_per_s'] / 1e6:.1f} M MB/s")
    return {"workload": f"mixed64_{len(mw.seqs)}streams_{len(mw.units)}vops_S16", "grid_mbs_per_frame_step": mw.grid_mbs,
            "grid_mbs_per_vop_layer": mw.layer_mbs, "per_step_graph": per_step, "pipelined_all_steps": pipelined}


class HDWorkload:
    """8 streams of 1920x1088, 3-6 VOPs each (sub-pixel motion up to 24 px
    per frame), S=32 with half-pel: one batched frame step = every
    (stream, VOP) pair of one frame step, plain or with seed buffers."""

    def __init__(self, frames=6, streams=8):
        import torch
        import paper_1002_1168_amd as me
        from paper_1002_1168_amd import device as dv
        from paper_1002_1168_amd import synth
        self.me, self.dv, self.torch = me, dv, torch
        t0 = time.time()
        self.seqs = synth.hd_streams(seed=5, frames=frames, streams=streams)
        log(f"generated {len(self.seqs)} 1920x1088 streams x{frames} frames in {time.time() - t0:.1f}s")
        self.pairs = frames - 1
        self.ds = [dv.DeviceSequence(q) for q in self.seqs]
        self.units = [(si, v) for si, q in enumerate(self.seqs) for v in range(q.vops)]
        self.params = me.me_default_params(search_range=32, half_pel=1)
        self.grid_mbs = sum(self.ds[si].hm * self.ds[si].wm for si, _ in self.units)

    def outputs(self):
        return [self.dv.Outputs.alloc(self.pairs, self.ds[si].hm, self.ds[si].wm) for si, _ in self.units]

    def jobs(self, i, out, zero, seeds=None):
        """Jobs of frame step i; T = the previous step's mv_int (zero at step 0)."""
        js = []
        for u, (si, v) in enumerate(self.units):
            d, t = self.ds[si], i + 1
            tf = out[u].mv_int[i - 1] if i > 0 else zero[u]
            js.append(self.dv.job(d.luma[t], d.luma[t - 1], d.alpha[v, t], d.alpha[v, t - 1], d.cls[v, t], tf,
                                  out[u], i, None if seeds is None else seeds[u]))
        return js


def hd_measurement(torch, steps):
    """The batched frame step on the 1920x1088 streams, plain and with the
    proposal network attached (weights trained on CIF at S=16; the seed is
    clamped to +-16 and refined by the recursion at S=32): MB/s, PSNR,
    recursion iterations per searched MB."""
    me = __import__("paper_1002_1168_amd")
    hw = HDWorkload()
    stream = hw.dv.stream_handle()
    zero = [torch.zeros((hw.ds[si].hm, hw.ds[si].wm, 2), dtype=torch.int16, device="cuda") for si, _ in hw.units]
    path = os.path.join(ROOT, "paper_1002_1168_amd", "weights", "proposal_cif_s16.npy")
    net = me.Net(np.load(path, allow_pickle=False)) if os.path.exists(path) else None
    res = {}
    for form in ("plain", "learned"):
        if form == "learned" and net is None:
            break
        out = hw.outputs()
        seeds = None
        if form == "learned":
            seeds = [torch.zeros((hw.ds[si].hm, hw.ds[si].wm, 2), dtype=torch.int16, device="cuda")
                     for si, _ in hw.units]
        step_jobs = [me.job_array(hw.jobs(i, out, zero, seeds)) for i in range(hw.pairs)]
        b = me.Batch(step_jobs[0], hw.params, 0, stream=stream)
        if form == "learned":
            b.set_net(net)
        # one pass with the per-step results: quality
        psnr = []
        for i in range(hw.pairs):
            b.step(step_jobs[i])
            sse, npx, ps, status = b.results(check=False)
            assert status in (me.ME_OK, me.ME_EEMPTY), status
            psnr += [x for x, n in zip(ps, npx) if n > 0 and np.isfinite(x)]
        torch.cuda.synchronize()
        its = n = 0
        for u, (si, v) in enumerate(hw.units):
            h = out[u].host()
            m = hw.ds[si].cls[v, 1:].cpu().numpy() != 0
            its += int(h["iters"][m].astype(np.int64).sum())
            n += int(m.sum())
        # timed passes
        k = max(steps // hw.pairs, 2) * hw.pairs
        t0 = time.perf_counter()
        for i in range(k):
            b.step(step_jobs[i % hw.pairs])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        res[form] = {"mb_per_s": hw.grid_mbs * k / dt, "ms_per_frame_step": 1000.0 * dt / k, "frame_steps": k,
                     "psnr_db": float(np.mean(psnr)), "iters_per_mb": its / max(n, 1), "searched_mbs_per_pass": n}
    if net is not None:
        net.close()
        res["psnr_delta_db"] = res["learned"]["psnr_db"] - res["plain"]["psnr_db"]
        res["admitted"] = bool(res["psnr_delta_db"] >= -0.05)
    log("hd batched: " + "; ".join(f"{f} {r['mb_per_s'] / 1e6:.1f} M MB/s, {r['ms_per_frame_step']:.3f} ms/step, "
                                     f"PSNR {r['psnr_db']:.3f} dB, iters/MB {r['iters_per_mb']:.3f}"
                                     for f, r in res.items() if isinstance(r, dict)))
    return {"workload": f"hd1920x1088_{len(hw.seqs)}streams_{len(hw.units)}vops_S32_halfpel",
            "grid_mbs_per_frame_step": hw.grid_mbs, **res}


def timed(fn, ring, steps, warmup, torch, me, stream, kind):
    """Wall time of `steps` frame steps fn(slot), and the mean duration of
    the main kernel of call kind `kind` over the same steps (HIP events
    recorded by the library on `stream` around that kernel).  Step i is
    queued before the host waits for step i-1's sums and computes its PSNR,
    so the GPU does not idle while the host reads results back; every
    step's PSNR is still computed.  Returns the last step's results."""
    def run(n):
        for i in range(n):
            fn(i & 1)
            if i:
                ring.result((i - 1) & 1)
        return ring.result((n - 1) & 1)

    run(warmup)
    torch.cuda.synchronize()
    me.me_kernel_timing(True, kinds=[kind])  # events around this kind's kernel only
    me.me_kernel_time_ms(kind, stream)  # restart the sums
    t0 = time.perf_counter()
    res = run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    total, count = me.me_kernel_time_ms(kind, stream)
    me.me_kernel_timing(False)
    assert count == steps, (count, steps)
    return dt, total / count, res


def summarize(out_list, classes, searched_only=True):
    pts = its = n = 0
    for v, o in enumerate(out_list):
        h = o.host()
        m = classes[v] != 0
        pts += int(h["points"][m].astype(np.int64).sum())
        its += int(h["iters"][m].astype(np.int64).sum())
        n += int(m.sum())
    return pts, its, n


def cpu_baseline(wl, gpu_hosts, min_seconds=10.0):
    """The oracle on the whole workload, single thread, repeated until
    `min_seconds` have passed; also checks the GPU result of the last timed
    step bit-exactly.  -> (seconds per pass, passes, exact)."""
    import oracle
    seq, p = wl.seq, wl.params
    op = oracle.Params(p.search_range, p.theta, p.eps_q12, p.max_step, p.k_max, p.half_pel)
    t0 = time.perf_counter()
    reps = 0
    while True:
        res = [oracle.pa_sequence(seq, v, op, pairs=wl.pairs) for v in range(wl.V)]
        reps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = (time.perf_counter() - t0) / reps
    exact = True
    for v in range(wl.V):
        for i, r in enumerate(res[v]):
            for k in ("mv", "mv_int", "cost", "iters", "points"):
                if not np.array_equal(gpu_hosts[v][k][i], r[k]):
                    exact = False
    return dt, reps, exact


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if a.copy_mib:
        src = torch.randint(0, 255, (a.copy_mib << 20,), dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {a.copy_mib} MiB x3")
        return
    if a.only_batched:
        print(json.dumps({"batched": batched_measurement(torch, a.steps, a.warmup)}), flush=True)
        return
    wl = Workload(a.frames)
    me = wl.me
    stream = wl.dv.stream_handle()

    ring = SumsRing(torch, me, len(wl.jobs))
    dt, kern_ms, res = timed(lambda slot: wl.step(stream, ring, slot), ring, a.steps, a.warmup, torch, me, stream,
                             me.ME_KT_SEARCH)
    assert me.me_device_status(stream) == me.ME_OK
    sse, npx, ps, _ = res
    ms = 1000.0 * dt / a.steps
    value = wl.grid_mbs * a.steps / dt
    classes = wl.ds.cls[:, 1:].cpu().numpy()
    pts, its, nsearch = summarize(wl.out, classes)
    psnr = float(np.mean(ps))
    # roofline of the dominant kernel (the pipelined search): integer VALU
    ops = SAD_OPS * pts + PASS_OPS * (nsearch + its)   # one pass at the BRS winner + one per iteration
    achieved = ops / (kern_ms * 1e-3) / 1e12
    log(f"step {ms:.3f} ms, search kernel {kern_ms:.3f} ms, {value / 1e6:.1f} M MB/s, PSNR {psnr:.2f} dB, "
        f"iters/MB {its / max(nsearch, 1):.3f}, points/MB {pts / max(nsearch, 1):.3f}")

    baselines = {}
    if not a.no_baselines:
        for m, name in ((me.ME_ES, "es"), (me.ME_TSS, "tss"), (me.ME_DS, "ds")):
            bdt, bk, bres = timed(lambda slot, m=m: wl.baseline_step(m, stream, ring, slot), ring,
                                  max(a.steps // 2, 1), 1, torch, me, stream,
                                  me.ME_KT_FULL)
            bpts, _, bn = summarize(wl.base_out[m], classes)
            steps_b = max(a.steps // 2, 1)
            entry = {"mb_per_s": wl.grid_mbs * steps_b / bdt, "ms_per_step": 1000.0 * bdt / steps_b,
                     "search_kernel_ms": bk, "psnr_db": float(np.mean(bres[2])),
                     "points_per_mb": bpts / max(bn, 1)}
            if m == me.ME_ES:
                es_ops = SAD_OPS * bpts
                ach = es_ops / (bk * 1e-3) / 1e12
                entry["roofline"] = {"bound": "alu", "achieved": ach, "peak": PEAK_INT_TOPS, "unit": "Tops/s",
                                     "frac": ach / PEAK_INT_TOPS}
            baselines[name] = entry
            log(f"{name}: {entry['mb_per_s'] / 1e6:.1f} M MB/s, kernel {bk:.3f} ms, PSNR {entry['psnr_db']:.2f}, "
                f"points/MB {entry['points_per_mb']:.2f}")
        assert me.me_device_status(stream) == me.ME_OK

    learned = None
    if not a.no_learned:
        learned = learned_measurement(wl, torch, a.steps, a.warmup, psnr, its / max(nsearch, 1))

    batched = None
    if not a.no_batched:
        batched = batched_measurement(torch, a.steps, a.warmup)

    hd = None
    if not a.no_hd:
        hd = hd_measurement(torch, a.steps)

    cpu = None
    if not a.no_cpu_baseline:
        hosts = [o.host() for o in wl.out]
        cdt, reps, exact = cpu_baseline(wl, hosts)
        cpu = {"value": wl.grid_mbs / cdt, "unit": "MB/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole workload ({wl.V} VOPs x {wl.pairs} pairs: classification, proposed search, "
                         f"MC/SSE) {reps}x back to back, mean per pass (single thread, C oracle built -O2)",
               "parity_vs_gpu": "bit-exact" if exact else "MISMATCH"}
        log(f"oracle: {cdt:.2f}s -> {cpu['value'] / 1e6:.3f} M MB/s, GPU parity {'ok' if exact else 'MISMATCH'}")

    line = {
        "metric": "macroblocks/sec estimated at <=0.05 dB PSNR vs plain; mean iterations/MB",
        "value": value, "unit": "MB/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"cif352x288_{wl.V}vop_{a.frames}f_S{wl.S}_plain", "frames": a.frames,
                   "vops": wl.V, "frame_pairs_per_vop": wl.pairs, "search_range": wl.S,
                   "grid_mbs_per_step": wl.grid_mbs, "searched_mbs_per_step": nsearch},
        "psnr_db": psnr, "iters_per_mb": its / max(nsearch, 1), "points_per_mb": pts / max(nsearch, 1),
        "searched_mb_per_s": nsearch * a.steps / dt,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS, "unit": "Tops/s",
                     "frac": achieved / PEAK_INT_TOPS,
                     "traffic": measured_traffic("pa2_kernel", ("paper_1002_1168_amd/csrc/k_pa.hip",
                                                                "paper_1002_1168_amd/csrc/me_internal.h"),
                                                 "profiles/pa2_kernel_traffic_cif352x288_2vop_300f_S16.md"),
                     "kernel": "pa2_kernel", "kernel_ms": kern_ms},
        "cpu_baseline": cpu,
        "baselines": baselines,
        "learned": learned,
        "batched": batched,
        "hd_batched": hd,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
