"""Training and evaluation of the learned motion-vector proposal network.

Labels are the plain method's own full-pel vectors (``mv_int`` of
``me_texture_recursive`` without a network) on generated sequences; every
step of both the labelling and the training runs in the library's kernels.
Evaluation runs the plain and the network-seeded search on held-out
sequences and compares prediction quality (PSNR of the motion-compensated
frames over the VOP), distortion, recursion iterations and compared blocks.
"""
from __future__ import annotations

import argparse
import json
import os
import time
from dataclasses import dataclass

import numpy as np
import torch

import paper_1002_1168_amd as me
from paper_1002_1168_amd import device as dv
from paper_1002_1168_amd import synth


@dataclass
class Labelled:
    """One sequence on the device with its classes and, per VOP, the plain
    method's results for every frame pair."""
    ds: dv.DeviceSequence
    plain: list          # per VOP: dv.Outputs

    @property
    def pairs(self) -> int:
        return self.ds.F - 1


def label(seqs, params: me.me_params, stream=None) -> list:
    """Classes and plain-method results (all pairs of a VOP in one launch)."""
    s = dv.stream_handle() if stream is None else stream
    out = []
    for q in seqs:
        ds = dv.DeviceSequence(q)
        fr, cp, bp = ds.classify_frames()
        me.me_classify_babs(fr, cp, bp, stream=s)
        plain = []
        for v in range(ds.V):
            o = dv.Outputs.alloc(ds.F - 1, ds.hm, ds.wm)
            me.me_texture_recursive(ds.pair_jobs(v, o), params, None, stream=s)
            plain.append(o)
        out.append(Labelled(ds, plain))
    torch.cuda.synchronize()
    return out


def _pair_job(L: Labelled, v: int, i: int):
    d = L.ds
    t = i + 1
    return dv.job(d.luma[t], d.luma[t - 1], d.alpha[v, t], d.alpha[v, t - 1], d.cls[v, t], None, L.plain[v], i)


def train(net: me.Net, data: list, steps: int, pairs_per_step: int, lr: float, momentum: float = 0.9,
          seed: int = 0, stream=None, log_every: int = 0, log=print) -> list:
    """SGD steps, each on the opaque MBs of `pairs_per_step` frame pairs drawn
    (seeded) from `data`.  -> loss before each step."""
    s = dv.stream_handle() if stream is None else stream
    units = [(li, v, i) for li, L in enumerate(data) for v in range(L.ds.V) for i in range(L.pairs)]
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.time()
    for step in range(steps):
        pick = rng.choice(len(units), size=min(pairs_per_step, len(units)), replace=False)
        jobs, labels = [], []
        for u in pick:
            li, v, i = units[u]
            jobs.append(_pair_job(data[li], v, i))
            labels.append(data[li].plain[v].mv_int[i].data_ptr())
        hist.append(net.train_step(jobs, labels, lr, momentum, stream=s))
        if not np.isfinite(hist[-1]):
            raise FloatingPointError(f"training diverged at step {step} (lr {lr})")
        if log_every and (step % log_every == 0 or step == steps - 1):
            log(f"step {step}: loss {hist[-1]:.4f} ({time.time() - t0:.1f}s)")
    return hist


def evaluate(data: list, params: me.me_params, net: me.Net | None, stream=None) -> dict:
    """Plain or network-seeded search on every pair of `data`, with MC/PSNR.
    -> mean per-frame PSNR (dB), mean distortion, iterations and compared
    blocks per searched MB, searched MBs."""
    s = dv.stream_handle() if stream is None else stream
    psnr, cost, its, pts, nmb = [], 0, 0, 0, 0
    for L in data:
        d = L.ds
        for v in range(d.V):
            o = dv.Outputs.alloc(L.pairs, d.hm, d.wm)
            seeds = torch.zeros((L.pairs, d.hm, d.wm, 2), dtype=torch.int16, device="cuda") if net else None
            jobs = d.pair_jobs(v, o, seeds=seeds)
            me.me_texture_recursive(jobs, params, net, stream=s)
            sse, npx, ps, _ = me.me_motion_compensate_psnr(jobs, stream=s, check=False)
            psnr += [p for p, n in zip(ps, npx) if n > 0 and np.isfinite(p)]
            h = o.host()
            m = d.cls[v, 1:].cpu().numpy() != 0
            cost += int(h["cost"][m].astype(np.int64).sum())
            its += int(h["iters"][m].astype(np.int64).sum())
            pts += int(h["points"][m].astype(np.int64).sum())
            nmb += int(m.sum())
    n = max(nmb, 1)
    return {"psnr_db": float(np.mean(psnr)) if psnr else float("nan"), "cost_per_mb": cost / n,
            "iters_per_mb": its / n, "points_per_mb": pts / n, "searched_mbs": nmb}


def prediction_error(net: me.Net, data: list, stream=None) -> dict:
    """Mean |p - label| (full pels) of the network over the opaque MBs of
    `data`, beside the same error of the zero vector."""
    s = dv.stream_handle() if stream is None else stream
    err = zero = 0.0
    n = 0
    for L in data:
        d = L.ds
        for v in range(d.V):
            pred = torch.full((L.pairs, d.hm, d.wm, 2), float("nan"), dtype=torch.float32, device="cuda")
            jobs = [_pair_job(L, v, i) for i in range(L.pairs)]
            net.forward(jobs, [pred[i].data_ptr() for i in range(L.pairs)], stream=s)
            torch.cuda.synchronize()
            p = pred.cpu().numpy()
            lab = L.plain[v].mv_int.cpu().numpy().astype(np.float64) / 2.0
            m = ~np.isnan(p[..., 0])
            err += float(np.abs(p[m] - lab[m]).sum())
            zero += float(np.abs(lab[m]).sum())
            n += int(m.sum())
    n = max(n, 1)
    return {"mae_net": err / (2 * n), "mae_zero": zero / (2 * n), "mbs": n}


def training_sets(train_count: int, held_count: int, frames: int, seed: int = 4):
    """Generated CIF sequences in the two-VOP style with 1-4 VOPs: the
    training set and a held-out set from disjoint seeds."""
    return (synth.cif_training_set(seed, train_count, frames),
            synth.cif_training_set(seed + 1000, held_count, frames))


def hd_training_sets(train_count: int, held_count: int, frames: int, seed: int = 104, workers: int = 16):
    """1920x1088 streams in the style of the batched high-definition workload
    (3-6 VOPs, sub-pixel velocities up to 24 px per frame), from seeds
    disjoint from each other and from the workload's own streams."""
    return (synth.hd_streams(seed=seed, frames=frames, streams=train_count, workers=workers),
            synth.hd_streams(seed=seed + 1000, frames=frames, streams=held_count, workers=workers))


# Presets: (training-set maker, search range, half-sample refinement, window scale, output name)
PRESETS = {
    "cif": (training_sets, 16, 0, 2, "proposal_cif_s16"),
    "hd": (hd_training_sets, 32, 1, 4, "proposal_hd_s32"),
}


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def main(argv=None):
    """Train on generated sequences (labels: the plain method), evaluate on
    held-out ones, write the weights (.npy, float32), a checkpoint (.menet,
    with the window scale) and a JSON record."""
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--preset", choices=sorted(PRESETS), default="cif",
                    help="cif: 352x288, S=16, scale 2; hd: 1920x1088, S=32 with half-pel, scale 4")
    ap.add_argument("--train", type=int, default=None)
    ap.add_argument("--held", type=int, default=None)
    ap.add_argument("--frames", type=int, default=None)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--pairs-per-step", type=int, default=64)
    ap.add_argument("--lr", type=float, default=None)
    ap.add_argument("--momentum", type=float, default=0.9)
    ap.add_argument("--init-seed", type=int, default=1)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    make, S, half, scale, name = PRESETS[a.preset]
    hd = a.preset == "hd"
    ntrain = a.train if a.train is not None else (32 if hd else 200)
    nheld = a.held if a.held is not None else (8 if hd else 50)
    frames = a.frames if a.frames is not None else (12 if hd else 30)
    lr = a.lr if a.lr is not None else (0.003 if hd else 0.03)
    out = a.out or os.path.join(WEIGHTS, name)
    torch.cuda.set_device(0)
    t0 = time.time()
    tr, ho = make(ntrain, nheld, frames)
    p = me.me_default_params(search_range=S, half_pel=half)
    dtr, dho = label(tr, p), label(ho, p)
    del tr, ho
    print(f"generated and labelled {ntrain} + {nheld} sequences in {time.time() - t0:.1f}s", flush=True)
    net = me.Net(synth.net_init(a.init_seed), scale=scale)
    t1 = time.time()
    hist = train(net, dtr, a.steps, a.pairs_per_step, lr, a.momentum, log_every=500,
                 log=lambda m: print(m, flush=True))
    torch.cuda.synchronize()
    ttrain = time.time() - t1
    rec = {"preset": a.preset, "train_sequences": ntrain, "held_out_sequences": nheld, "frames": frames,
           "steps": a.steps, "pairs_per_step": a.pairs_per_step, "lr": lr, "momentum": a.momentum,
           "init_seed": a.init_seed, "search_range": S, "half_pel": half, "window_scale": scale,
           "train_seconds": ttrain,
           "loss_first100": float(np.mean(hist[:100])), "loss_last100": float(np.mean(hist[-100:])),
           "held_out": {"prediction": prediction_error(net, dho), "plain": evaluate(dho, p, None),
                        "learned": evaluate(dho, p, net)}}
    w = net.weights()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    net.save(out + ".menet")
    net.close()
    np.save(out + ".npy", w, allow_pickle=False)
    with open(out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
