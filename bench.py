#!/usr/bin/env python3
"""Throughput of the shape-adaptive motion estimator on one MI355X.

Headline workload: 8 concurrent 1920x1088 streams, 3-6 VOPs each (37 VOP
layers) with occlusion and sub-pixel motion up to 24 px per frame, 60
frames, search range +-32 with half-sample refinement; seeded synthetic data
resident in HBM.  One timed step is one pass of the paper's path over the
whole workload: 59 batched frame steps, each one HIP-graph replay of MB
classification, (optionally) the learned proposal network, the
block/pel-recursive search and motion compensation + SSE for every
(stream, VOP) pair of that frame step.  `value` counts grid MBs of every
(VOP, frame pair) per second, for the fastest form admitted by the metric
(the plain method, or the network-seeded form when its PSNR is within
0.05 dB of plain).

Also reported (under "extras"): the CIF two-VOP sequence (300 frames, +-16)
as one pipelined launch with the ES / TSS / 4SS / DS baselines, the QCIF
sequence in the paper's geometry (+-7: VOP mode, rectangular mode and the
Section 4 protocol with frame distance 2, unrestricted vectors and the
MPEG-4-padded reference) and CIF in rectangular mode with every method's
PSNR, points per MB and figure of merit (Eq. 6), and the 64-stream
mixed-size batch.

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits.
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

METRIC = "macroblocks/sec estimated at <=0.05 dB PSNR vs plain; mean iterations/MB"
KIND_NAMES = {0: "classify_kernel", 1: "search_kernel", 3: "mc_kernel", 4: "net_kernel"}


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


def figure_of_merit(psnr_db, points_per_mb, S):
    """Eq. 6: I = PSNR (2S+1)^2 / C with the PSNR averaged in linear scale
    (10^(dB/10) per frame and VOP) and C the mean compared blocks per MB."""
    ps = [x for x in psnr_db if np.isfinite(x)]
    if not ps or points_per_mb <= 0:
        return None
    lin = float(np.mean([10.0 ** (x / 10.0) for x in ps]))
    return lin * (2 * S + 1) ** 2 / points_per_mb


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed passes over the headline workload")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=60, help="frames per 1920x1088 stream")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only (for profiling)")
    ap.add_argument("--no-learned", action="store_true", help="skip the network-seeded forms")
    ap.add_argument("--only-cif", action="store_true",
                    help="only the CIF pipelined step (for profiling its search kernel) and print it")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the 64-stream batched measurement (for profiling) and print it")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 3 device copies of this many MiB (calibrates the HBM byte counters) and exit")
    return ap.parse_args()


def net_weights(name):
    path = os.path.join(ROOT, "paper_1002_1168_amd", "weights", name)
    return (np.load(path, allow_pickle=False), os.path.relpath(path, ROOT)) if os.path.exists(path) else (None, None)


# ------------------------------------------------------------------ headline
class HDWorkload:
    """8 streams of 1920x1088, 3-6 VOPs each, S=32 with half-pel: one frame
    step = every (stream, VOP) pair of one frame pair; a pass = every frame
    step of the sequences."""

    def __init__(self, seqs):
        import torch
        import paper_1002_1168_amd as me
        from paper_1002_1168_amd import device as dv
        self.me, self.dv, self.torch = me, dv, torch
        self.seqs = seqs
        self.frames = seqs[0].frames
        self.pairs = self.frames - 1
        self.ds = [dv.DeviceSequence(q) for q in self.seqs]
        self.units = [(si, v) for si, q in enumerate(self.seqs) for v in range(q.vops)]
        self.params = me.me_default_params(search_range=32, half_pel=1)
        self.grid_mbs = sum(self.ds[si].hm * self.ds[si].wm for si, _ in self.units)   # per frame step
        self.zero = [torch.zeros((self.ds[si].hm, self.ds[si].wm, 2), dtype=torch.int16, device="cuda")
                     for si, _ in self.units]

    def outputs(self):
        return [self.dv.Outputs.alloc(self.pairs, self.ds[si].hm, self.ds[si].wm) for si, _ in self.units]

    def jobs(self, i, out, seeds=None):
        """Jobs of frame step i; T = the previous step's mv_int (zero at step 0)."""
        js = []
        for u, (si, v) in enumerate(self.units):
            d, t = self.ds[si], i + 1
            tf = out[u].mv_int[i - 1] if i > 0 else self.zero[u]
            js.append(self.dv.job(d.luma[t], d.luma[t - 1], d.alpha[v, t], d.alpha[v, t - 1], d.cls[v, t], tf,
                                  out[u], i, None if seeds is None else seeds[u][i]))
        return js


def hd_form(hw, form, net, steps, warmup):
    """One form (plain / learned) of the headline: a quality pass with every
    frame step's PSNR and a per-kernel breakdown (events inside the graph),
    then `steps` timed passes with events around the dominant kernel only."""
    me, torch, dv = hw.me, hw.torch, hw.dv
    stream = dv.stream_handle()
    out = hw.outputs()
    seeds = None
    if form == "learned":
        seeds = [torch.zeros((hw.pairs, hw.ds[si].hm, hw.ds[si].wm, 2), dtype=torch.int16, device="cuda")
                 for si, _ in hw.units]
    step_jobs = [me.job_array(hw.jobs(i, out, seeds)) for i in range(hw.pairs)]
    kinds = [me.ME_KT_CLASSIFY, me.ME_KT_SEARCH, me.ME_KT_MC] + ([me.ME_KT_NET] if net is not None else [])
    me.me_kernel_timing(True, kinds=kinds)
    try:
        b = me.Batch(step_jobs[0], hw.params, 0, stream=stream)
        if net is not None:
            b.set_net(net)
    finally:
        me.me_kernel_timing(False)
    cfg = b.config()
    # quality pass: per-step results
    psnr, jobs_db = [], []
    for i in range(hw.pairs):
        b.step(step_jobs[i])
        sse, npx, ps, status = b.results(check=False)
        assert status in (me.ME_OK, me.ME_EEMPTY), status
        jobs_db += [x for x, n in zip(ps, npx) if n > 0 and np.isfinite(x)]
    torch.cuda.synchronize()
    breakdown = {}
    for k in kinds:
        ms, cnt = b.kernel_time_ms(k)
        breakdown[KIND_NAMES[k]] = ms / max(cnt, 1)
    dom_kind = max(kinds, key=lambda k: breakdown[KIND_NAMES[k]])
    pts = its = n = 0
    for u, (si, v) in enumerate(hw.units):
        h = out[u].host()
        m = hw.ds[si].cls[v, 1:].cpu().numpy() != 0
        pts += int(h["points"][m].astype(np.int64).sum())
        its += int(h["iters"][m].astype(np.int64).sum())
        n += int(m.sum())
    # timed passes: events around the dominant kernel only
    me.me_kernel_timing(True, kinds=[dom_kind])
    try:
        b.set_config(cfg)
    finally:
        me.me_kernel_timing(False)
    for _ in range(warmup):
        for i in range(hw.pairs):
            b.step(step_jobs[i])
    torch.cuda.synchronize()
    b.kernel_time_ms(dom_kind)   # restart the sums
    t0 = time.perf_counter()
    for _ in range(steps):
        for i in range(hw.pairs):
            b.step(step_jobs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, kcnt = b.kernel_time_ms(dom_kind)
    assert kcnt == steps * hw.pairs, (kcnt, steps * hw.pairs)
    status = b.results(check=False)[3]
    assert status in (me.ME_OK, me.ME_EEMPTY), status
    b.close()
    grid = hw.grid_mbs * hw.pairs
    res = {"mb_per_s": grid * steps / dt, "ms_per_step": 1000.0 * dt / steps,
           "ms_per_frame_step": 1000.0 * dt / (steps * hw.pairs), "psnr_db": float(np.mean(jobs_db)),
           "iters_per_mb": its / max(n, 1), "points_per_mb": pts / max(n, 1), "searched_mbs_per_step": n,
           "searched_mb_per_s": n * steps / dt, "launch_config": cfg,
           "kernel_ms_per_frame_step": breakdown, "dominant_kernel": KIND_NAMES[dom_kind],
           "dominant_kernel_ms": kms / kcnt, "outputs": out, "pts": pts, "its": its, "n": n}
    if net is not None:
        served = int(sum(int((hw.ds[si].cls[v, 1:] == 1).sum()) for si, v in hw.units))
        net_ms = breakdown["net_kernel"] * hw.pairs
        tf = served * NET_FWD_FLOP / (net_ms * 1e-3) / 1e12
        res["network_forward"] = {"mbs_per_step": served, "kernel_ms_per_frame_step": breakdown["net_kernel"],
                                  "bound": "mfma", "achieved": tf, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tf / PEAK_BF16_TFLOPS}
    log(f"hd {form}: {res['mb_per_s'] / 1e6:.1f} M MB/s, {res['ms_per_step']:.2f} ms/pass "
        f"({res['ms_per_frame_step']:.3f} ms/frame step), PSNR {res['psnr_db']:.3f} dB, "
        f"iters/MB {res['iters_per_mb']:.3f}, points/MB {res['points_per_mb']:.2f}; "
        f"kernels/frame step {({k: round(v, 4) for k, v in breakdown.items()})}, cfg {cfg}")
    return res


def search_roofline(r, kernel, traffic=None):
    """Integer-VALU roofline of the pipelined search from its algorithmic
    work: one SAD per compared block, one gradient pass at the block-recursive
    winner and one per pel-recursion candidate."""
    ops = SAD_OPS * r["pts"] + PASS_OPS * (r["n"] + r["its"])
    launches_ops = ops  # per pass
    ach = launches_ops / (r["dominant_kernel_ms"] * 1e-3 * r["frame_steps"]) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK_INT_TOPS, "unit": "Tops/s", "frac": ach / PEAK_INT_TOPS,
            "traffic": traffic, "kernel": kernel, "kernel_ms": r["dominant_kernel_ms"],
            "work_per_launch": ops / r["frame_steps"], "work_unit": "int lane-ops"}


def cpu_baseline_hd(hw, plain_out, nsteps, threads):
    """The oracle on the first `nsteps` frame steps of every (stream, VOP)
    (classification, the proposed search, MC/SSE per pair; T chained), once
    on one thread and once on `threads` threads (one task per (stream, VOP)
    chain); checks the GPU's plain results of those steps bit-exactly."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    p = hw.params
    op = oracle.Params(p.search_range, p.theta, p.eps_q12, p.max_step, p.k_max, p.half_pel)

    def task(u):
        si, v = hw.units[u]
        return oracle.pa_sequence(hw.seqs[si], v, op, pairs=nsteps)

    t0 = time.perf_counter()
    res1 = [task(u) for u in range(len(hw.units))]
    t1 = time.perf_counter() - t0
    reps = 0
    t0 = time.perf_counter()
    while True:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            resn = list(ex.map(task, range(len(hw.units))))
        reps += 1
        if time.perf_counter() - t0 >= 3.0:
            break
    tn = (time.perf_counter() - t0) / reps
    exact = True
    for u in range(len(hw.units)):
        h = plain_out[u].host()
        for i in range(nsteps):
            for k in ("mv", "mv_int", "cost", "iters", "points"):
                if not (np.array_equal(h[k][i], res1[u][i][k]) and np.array_equal(h[k][i], resn[u][i][k])):
                    exact = False
    return t1, tn, exact


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# --------------------------------------------------------------------- extras
class CifWorkload:
    """Device buffers and job lists of the CIF two-VOP sequence (300 frames)."""

    def __init__(self, frames=300):
        import paper_1002_1168_amd as me
        from paper_1002_1168_amd import device as dv
        from paper_1002_1168_amd import synth
        self.me, self.dv = me, dv
        self.seq = synth.cif_two_vops(seed=2, frames=frames)
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
        self.grid_mbs = self.V * self.pairs * self.ds.hm * self.ds.wm

    def step(self, stream, ring, slot):
        """classify -> proposed search -> MC/SSE (sums read back by `ring`)."""
        me = self.me
        me.me_classify_babs(self.cls_frames, self.cls_ptrs, self.bab_ptrs, stream=stream)
        me.me_texture_recursive(self.jobs, self.params, None, stream=stream)
        ring.queue(self.jobs, slot, stream)


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


def timed(fn, ring, steps, warmup, torch, me, stream, kind):
    """Wall time of `steps` steps fn(slot), and the mean duration of the main
    kernel of call kind `kind` over the same steps (HIP events recorded by
    the library on `stream` around that kernel).  Step i is queued before the
    host waits for step i-1's sums, so the GPU does not idle while the host
    reads results back.  Returns the last step's results."""
    def run(n):
        for i in range(n):
            fn(i & 1)
            if i:
                ring.result((i - 1) & 1)
        return ring.result((n - 1) & 1)

    run(warmup)
    torch.cuda.synchronize()
    me.me_kernel_timing(True, kinds=[kind])
    me.me_kernel_time_ms(kind, stream)
    t0 = time.perf_counter()
    res = run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    total, count = me.me_kernel_time_ms(kind, stream)
    me.me_kernel_timing(False)
    assert count == steps, (count, steps)
    return dt, total / count, res


def summarize(out_list, classes):
    pts = its = n = 0
    for v, o in enumerate(out_list):
        h = o.host()
        m = classes[v] != 0
        pts += int(h["points"][m].astype(np.int64).sum())
        its += int(h["iters"][m].astype(np.int64).sum())
        n += int(m.sum())
    return pts, its, n


def cif_measurement(torch, steps, warmup, learned=True):
    """CIF two-VOP sequence, 300 frames, +-16: the proposed search for all 598
    pairs in one pipelined launch, the baselines, and the network-seeded form."""
    import paper_1002_1168_amd as me
    wl = CifWorkload()
    stream = wl.dv.stream_handle()
    ring = SumsRing(torch, me, len(wl.jobs))
    dt, kern_ms, res = timed(lambda slot: wl.step(stream, ring, slot), ring, steps, warmup, torch, me, stream,
                             me.ME_KT_SEARCH)
    assert me.me_device_status(stream) == me.ME_OK
    classes = wl.ds.cls[:, 1:].cpu().numpy()
    pts, its, nsearch = summarize(wl.out, classes)
    psnr_list = res[2]
    psnr = float(np.mean(psnr_list))
    ops = SAD_OPS * pts + PASS_OPS * (nsearch + its)
    ach = ops / (kern_ms * 1e-3) / 1e12
    out = {"workload": f"cif352x288_{wl.V}vop_300f_S{wl.S}", "mb_per_s": wl.grid_mbs * steps / dt,
           "ms_per_step": 1000.0 * dt / steps, "grid_mbs_per_step": wl.grid_mbs, "searched_mbs_per_step": nsearch,
           "searched_mb_per_s": nsearch * steps / dt, "psnr_db": psnr, "iters_per_mb": its / max(nsearch, 1),
           "points_per_mb": pts / max(nsearch, 1),
           "figure_of_merit": figure_of_merit(psnr_list, pts / max(nsearch, 1), wl.S),
           "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_INT_TOPS, "unit": "Tops/s",
                        "frac": ach / PEAK_INT_TOPS, "kernel": "pa2_kernel", "kernel_ms": kern_ms,
                        "traffic": measured_traffic("pa2_kernel", ("paper_1002_1168_amd/csrc/k_pa.hip",
                                                                   "paper_1002_1168_amd/csrc/me_internal.h"),
                                                    "profiles/pa2_kernel_traffic_cif352x288_2vop_300f_S16.md")}}
    log(f"cif: step {out['ms_per_step']:.3f} ms, search kernel {kern_ms:.3f} ms, {out['mb_per_s'] / 1e6:.1f} M MB/s, "
        f"PSNR {psnr:.2f} dB, iters/MB {out['iters_per_mb']:.3f}, points/MB {out['points_per_mb']:.3f}")
    baselines = {}
    for m, name in ((me.ME_ES, "es"), (me.ME_TSS, "tss"), (me.ME_4SS, "4ss"), (me.ME_DS, "ds")):
        bout = [wl.dv.Outputs.alloc(wl.pairs, wl.ds.hm, wl.ds.wm) for _ in range(wl.V)]
        bj = me.job_array([j for v in range(wl.V) for j in wl.ds.pair_jobs(v, bout[v], wl.pairs, chained=False)])
        bsteps = max(steps // 2, 1)

        def bstep(slot, bj=bj, m=m):
            me.me_full_search(m, bj, wl.params, stream=stream)
            ring.queue(bj, slot, stream)

        bdt, bk, bres = timed(bstep, ring, bsteps, 1, torch, me, stream, me.ME_KT_FULL)
        bpts, _, bn = summarize(bout, classes)
        entry = {"mb_per_s": wl.grid_mbs * bsteps / bdt, "ms_per_step": 1000.0 * bdt / bsteps, "search_kernel_ms": bk,
                 "psnr_db": float(np.mean(bres[2])), "points_per_mb": bpts / max(bn, 1),
                 "figure_of_merit": figure_of_merit(bres[2], bpts / max(bn, 1), wl.S)}
        if m == me.ME_ES:
            a2 = SAD_OPS * bpts / (bk * 1e-3) / 1e12
            entry["roofline"] = {"bound": "alu", "achieved": a2, "peak": PEAK_INT_TOPS, "unit": "Tops/s",
                                 "frac": a2 / PEAK_INT_TOPS,
                                 "kernel": f"es_fixed_kernel<{wl.S}>" if wl.S in (7, 16, 32) else "es_kernel"}
        baselines[name] = entry
        log(f"cif {name}: {entry['mb_per_s'] / 1e6:.1f} M MB/s, kernel {bk:.3f} ms, PSNR {entry['psnr_db']:.2f}, "
            f"points/MB {entry['points_per_mb']:.2f}")
    assert me.me_device_status(stream) == me.ME_OK
    out["baselines"] = baselines
    w, wpath = net_weights("proposal_cif_s16.npy")
    if learned and w is not None:
        net = me.Net(w)
        outs = [wl.dv.Outputs.alloc(wl.pairs, wl.ds.hm, wl.ds.wm) for _ in range(wl.V)]
        seeds = [torch.zeros((wl.pairs, wl.ds.hm, wl.ds.wm, 2), dtype=torch.int16, device="cuda") for _ in range(wl.V)]
        jobs = me.job_array([j for v in range(wl.V) for j in wl.ds.pair_jobs(v, outs[v], wl.pairs, seeds=seeds[v])])

        def lstep(slot):
            me.me_classify_babs(wl.cls_frames, wl.cls_ptrs, wl.bab_ptrs, stream=stream)
            me.me_texture_recursive(jobs, wl.params, net, stream=stream)
            ring.queue(jobs, slot, stream)

        ldt, net_ms, lres = timed(lstep, ring, steps, warmup, torch, me, stream, me.ME_KT_NET)
        assert me.me_device_status(stream) == me.ME_OK
        net.close()
        served = int((classes == 1).sum())
        tflops = served * NET_FWD_FLOP / (net_ms * 1e-3) / 1e12
        lp, li, ln = summarize(outs, classes)
        lps = float(np.mean(lres[2]))
        out["learned"] = {"mb_per_s": wl.grid_mbs * steps / ldt, "ms_per_step": 1000.0 * ldt / steps, "psnr_db": lps,
                          "psnr_delta_vs_plain_db": lps - psnr, "iters_per_mb": li / max(ln, 1),
                          "points_per_mb": lp / max(ln, 1), "admitted": bool(lps >= psnr - 0.05), "weights": wpath,
                          "network_forward": {"kernel_ms": net_ms, "mbs": served, "bound": "mfma", "achieved": tflops,
                                              "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                                              "frac": tflops / PEAK_BF16_TFLOPS}}
        log(f"cif learned: {out['learned']['mb_per_s'] / 1e6:.1f} M MB/s, PSNR {lps:.3f} "
            f"({lps - psnr:+.4f}), iters/MB {out['learned']['iters_per_mb']:.3f}")
    return out


def quality_grid(seq, S, rect, torch, protocol=False):
    """Every method on one sequence (VOP mode, or rectangular mode with no
    alpha): mean per-frame PSNR, points and iterations per searched MB and
    the figure of merit (Eq. 6), as in Tables 1-2.  ``protocol`` (VOP mode):
    Section 4's setting as read here - frame distance 2, unrestricted
    vectors and the MPEG-4-padded reference VOP for search and MC."""
    import paper_1002_1168_amd as me
    from paper_1002_1168_amd import device as dv
    ds = dv.DeviceSequence(seq)
    s = dv.stream_handle()
    dist = 2 if protocol else 1
    pairs = seq.frames - dist
    vops = [None] if rect else list(range(seq.vops))
    if not rect:
        fr, cp, bp = ds.classify_frames()
        me.me_classify_babs(fr, cp, bp, stream=s)
    refs = ds.padded_refs(stream=s) if protocol else None
    p = me.me_default_params(search_range=S, half_pel=int(seq.half_pel),
                             flags=me.ME_FLAG_UNRESTRICTED if protocol else 0)
    res = {}
    for name, m in (("pa", None), ("es", me.ME_ES), ("tss", me.ME_TSS), ("4ss", me.ME_4SS), ("ds", me.ME_DS)):
        outs = [dv.Outputs.alloc(pairs, ds.hm, ds.wm) for _ in vops]
        jobs = [j for v, o in zip(vops, outs)
                for j in ds.pair_jobs(v, o, pairs, chained=m is None, distance=dist, refs=refs)]
        if m is None:
            me.me_texture_recursive(jobs, p, None, stream=s)
        else:
            me.me_full_search(m, jobs, p, stream=s)
        _, npx, ps, rc = me.me_motion_compensate_psnr(jobs, stream=s, check=False)
        assert rc in (me.ME_OK, me.ME_EEMPTY), rc
        assert me.me_device_status(s) == me.ME_OK
        db = [x for x, n in zip(ps, npx) if n > 0]
        pts = its = n = 0
        for v, o in zip(vops, outs):
            h = o.host()
            msk = np.ones(h["points"].shape, bool) if v is None else ds.cls[v, dist:].cpu().numpy() != 0
            pts += int(h["points"][msk].astype(np.int64).sum())
            its += int(h["iters"][msk].astype(np.int64).sum())
            n += int(msk.sum())
        res[name] = {"psnr_db": float(np.mean(db)), "points_per_mb": pts / max(n, 1),
                     "iters_per_mb": its / max(n, 1), "figure_of_merit": figure_of_merit(db, pts / max(n, 1), S)}
    torch.cuda.synchronize()
    log(f"{seq.name} {'rect' if rect else ('protocol' if protocol else 'vop')} S={S}: " + "; ".join(
        f"{k} {v['psnr_db']:.2f} dB {v['points_per_mb']:.2f} pts" for k, v in res.items()))
    return res


def batched_measurement(torch, steps, warmup):
    """64 mixed-size streams: per-frame-step graph launches, autotuned."""
    import paper_1002_1168_amd as me
    from paper_1002_1168_amd import device as dv
    from paper_1002_1168_amd import synth
    seqs = synth.mixed_streams(seed=3, frames=31)
    pairs = 30
    ds = [dv.DeviceSequence(q) for q in seqs]
    units = [(si, v) for si, q in enumerate(seqs) for v in range(q.vops)]
    out = [dv.Outputs.alloc(pairs, ds[si].hm, ds[si].wm) for si, _ in units]
    zero = [torch.zeros((ds[si].hm, ds[si].wm, 2), dtype=torch.int16, device="cuda") for si, _ in units]
    params = me.me_default_params(search_range=16)

    def jobs(i):
        js = []
        for u, (si, v) in enumerate(units):
            d, t = ds[si], i + 1
            tf = out[u].mv_int[i - 1] if i > 0 else zero[u]
            js.append(dv.job(d.luma[t], d.luma[t - 1], d.alpha[v, t], d.alpha[v, t - 1], d.cls[v, t], tf, out[u], i))
        return me.job_array(js)

    step_jobs = [jobs(i) for i in range(pairs)]
    stream = dv.stream_handle()
    b = me.Batch(step_jobs[0], params, me.ME_BATCH_AUTOTUNE, stream=stream)
    cfg = b.config()
    for i in range(max(warmup, pairs)):
        b.step(step_jobs[i % pairs])
    torch.cuda.synchronize()
    k = max(steps, 3 * pairs)
    t0 = time.perf_counter()
    for i in range(k):
        b.step(step_jobs[i % pairs])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    status = b.results(check=False)[3]
    assert status in (me.ME_OK, me.ME_EEMPTY), status
    b.close()
    grid = sum(ds[si].hm * ds[si].wm for si, _ in units)
    log(f"batched mixed streams: {grid * k / dt / 1e6:.1f} M MB/s ({1000 * dt / k:.3f} ms/step, cfg {cfg})")
    return {"workload": f"mixed64_{len(seqs)}streams_{len(units)}vops_S16", "grid_mbs_per_frame_step": grid,
            "mb_per_s": grid * k / dt, "ms_per_frame_step": 1000.0 * dt / k, "frame_steps": k, "config": cfg}


# ----------------------------------------------------------------------- main
def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    hd_seqs = None
    if not (a.copy_mib or a.only_batched or a.only_cif):
        # rendered in forked processes before anything touches the GPU
        from paper_1002_1168_amd import synth
        t0 = time.time()
        hd_seqs = synth.hd_streams(seed=5, frames=a.frames, streams=8, workers=min(8, threads))
        log(f"generated 8 1920x1088 streams x{a.frames} frames in {time.time() - t0:.1f}s")
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    import paper_1002_1168_amd as me
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
    if a.only_cif:
        print(json.dumps({"cif": cif_measurement(torch, a.steps, a.warmup, learned=False)}), flush=True)
        return

    hw = HDWorkload(hd_seqs)
    forms = {"plain": hd_form(hw, "plain", None, a.steps, a.warmup)}
    # the network trained on 1920x1088 streams (scale-4 window), else the CIF one
    ck = os.path.join(ROOT, "paper_1002_1168_amd", "weights", "proposal_hd_s32.menet")
    net = None
    if os.path.exists(ck):
        wpath = os.path.relpath(ck, ROOT)
        if not a.no_learned:
            net = me.Net.load(ck)
    else:
        w, wpath = net_weights("proposal_cif_s16.npy")
        if not a.no_learned and w is not None:
            net = me.Net(w)
    if net is not None:
        forms["learned"] = hd_form(hw, "learned", net, a.steps, a.warmup)
        net.close()
        lf = forms["learned"]
        lf["psnr_delta_vs_plain_db"] = lf["psnr_db"] - forms["plain"]["psnr_db"]
        lf["admitted"] = bool(lf["psnr_delta_vs_plain_db"] >= -0.05)
        lf["weights"] = wpath
    admitted = ["plain"] + [f for f in ("learned",) if f in forms and forms[f]["admitted"]]
    best = max(admitted, key=lambda f: forms[f]["mb_per_s"])
    r = forms[best]
    r["frame_steps"] = hw.pairs
    kern = r["dominant_kernel"]
    if kern == "search_kernel":
        # the search kernel that ran: row workers (pr_kernel) or line workers
        # (pa_kernel), with the window staging instantiated for S = 32 (28
        # elements per lane) or the generic one (0)
        cfg = r["launch_config"]
        name = ("pr_kernel" if cfg["search"] == "rows" else "pa_kernel") + \
            ("<28>" if cfg["staging"] == "plan" else "<0>")
        summary = {"pr_kernel<28>": "profiles/pr_kernel_hd1920x1088_8streams_S32_halfpel.md",
                   "pa_kernel<28>": "profiles/pa_kernel_hd1920x1088_8streams_S32_halfpel.md"}.get(name, "")
        roof = search_roofline(r, name, measured_traffic(
            name, ("paper_1002_1168_amd/csrc/k_pa.hip", "paper_1002_1168_amd/csrc/me_internal.h"), summary))
    else:
        roof = {"kernel": kern, "kernel_ms": r["dominant_kernel_ms"], "bound": None, "achieved": None,
                "peak": None, "unit": None, "frac": None, "traffic": None}

    cpu = None
    if not a.no_cpu_baseline:
        nsteps = min(10, hw.pairs)
        t1, tn, exact = cpu_baseline_hd(hw, forms["plain"]["outputs"], nsteps, threads)
        sample_mbs = hw.grid_mbs * nsteps
        cpu = {"value": sample_mbs / tn, "unit": "MB/s", "cores": threads, "kind": "oracle",
               "sample": f"the first {nsteps} of {hw.pairs} frame steps of all 8 streams and {len(hw.units)} VOP "
                         f"layers ({sample_mbs} grid MBs: classification, the proposed search with half-pel, "
                         f"MC/SSE; T chained); C oracle built -O2, one thread per (stream, VOP) chain",
               "single_thread_value": sample_mbs / t1, "host_cpus_visible": len(os.sched_getaffinity(0)),
               "cpu_model": cpu_model(), "parity_vs_gpu": "bit-exact" if exact else "MISMATCH"}
        log(f"oracle: {nsteps} frame steps, 1 thread {t1:.2f}s ({cpu['single_thread_value'] / 1e6:.3f} M MB/s), "
            f"{threads} threads {tn:.2f}s ({cpu['value'] / 1e6:.3f} M MB/s), GPU parity {'ok' if exact else 'MISMATCH'}")

    extras = {}
    if not a.no_extras:
        from paper_1002_1168_amd import synth
        extras["cif"] = cif_measurement(torch, a.steps, a.warmup, learned=not a.no_learned)
        extras["qcif_vop"] = quality_grid(synth.qcif_ellipse(seed=1, frames=10), 7, False, torch)
        extras["qcif_rect"] = quality_grid(synth.qcif_ellipse(seed=1, frames=10), 7, True, torch)
        extras["qcif_protocol"] = quality_grid(synth.qcif_ellipse(seed=1, frames=10), 7, False, torch, protocol=True)
        extras["cif_rect"] = quality_grid(synth.cif_two_vops(seed=2, frames=60), 16, True, torch)
        extras["batched_mixed64"] = batched_measurement(torch, a.steps, a.warmup)

    for f in forms.values():
        for k in ("outputs", "pts", "its", "n"):
            f.pop(k, None)
    line = {
        "metric": METRIC, "value": r["mb_per_s"], "unit": "MB/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"hd1920x1088_8streams_{len(hw.units)}vops_{hw.frames}f_S32_halfpel",
                   "form": best, "streams": 8, "vop_layers": len(hw.units), "frames": hw.frames,
                   "frame_steps_per_step": hw.pairs, "search_range": 32, "half_pel": True,
                   "grid_mbs_per_step": hw.grid_mbs * hw.pairs, "searched_mbs_per_step": r["searched_mbs_per_step"]},
        "iters_per_mb": r["iters_per_mb"], "psnr_db": r["psnr_db"], "points_per_mb": r["points_per_mb"],
        "searched_mb_per_s": r["searched_mb_per_s"],
        "forms": forms,
        "roofline": roof,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
