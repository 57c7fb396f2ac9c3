"""Device-memory plumbing for the C ABI: torch CUDA tensors for frames and
results, and the me_job lists that point into them.  Nothing here computes
any part of the method; it only allocates and fills descriptor structs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import me_frame, me_job

_NULL = None


def stream_handle(stream: torch.cuda.Stream | None = None):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def ptr(t: torch.Tensor | None):
    return _NULL if t is None else t.data_ptr()


@dataclass
class Outputs:
    """Per-pair result planes for P frame pairs on an hm x wm MB grid."""
    mv: torch.Tensor       # (P, hm, wm, 2) int16, half-pel
    mv_int: torch.Tensor   # (P, hm, wm, 2) int16
    cost: torch.Tensor     # (P, hm, wm) int32 (uint32 values)
    iters: torch.Tensor    # (P, hm, wm) uint8
    points: torch.Tensor   # (P, hm, wm) int16 (uint16 values)

    @classmethod
    def alloc(cls, P: int, hm: int, wm: int, device="cuda") -> "Outputs":
        return cls(torch.zeros((P, hm, wm, 2), dtype=torch.int16, device=device),
                   torch.zeros((P, hm, wm, 2), dtype=torch.int16, device=device),
                   torch.zeros((P, hm, wm), dtype=torch.int32, device=device),
                   torch.zeros((P, hm, wm), dtype=torch.uint8, device=device),
                   torch.zeros((P, hm, wm), dtype=torch.int16, device=device))

    def host(self) -> dict:
        return dict(mv=self.mv.cpu().numpy(), mv_int=self.mv_int.cpu().numpy(),
                    cost=self.cost.cpu().numpy().view(np.uint32), iters=self.iters.cpu().numpy(),
                    points=self.points.cpu().numpy().view(np.uint16))


def frame(luma: torch.Tensor, alpha: torch.Tensor | None = None) -> me_frame:
    H, W = luma.shape[-2:]
    return me_frame(ptr(luma), ptr(alpha), W, H, luma.stride(-2))


def job(cur, ref, cur_alpha, ref_alpha, mb_class, t_field, out: Outputs, i: int, seed=None) -> me_job:
    return me_job(frame(cur, cur_alpha), frame(ref, ref_alpha), ptr(mb_class), ptr(t_field), ptr(seed),
                  ptr(out.mv[i]), ptr(out.mv_int[i]), ptr(out.cost[i]), ptr(out.iters[i]),
                  ptr(out.points[i]))


def mc_job(cur, ref, cur_alpha, mb_class, mv) -> me_job:
    """A job for me_motion_compensate_psnr: only frames, classes and ``mv``."""
    return me_job(frame(cur, cur_alpha), frame(ref, None), ptr(mb_class), None, None, ptr(mv), ptr(mv),
                  None, None, None)


class DeviceSequence:
    """A synthetic sequence resident in HBM: luma (F, H, W) and alpha
    (V, F, H, W) uint8, plus per-frame MB classes of each VOP."""

    def __init__(self, seq, device="cuda"):
        self.seq = seq
        self.luma = torch.from_numpy(np.ascontiguousarray(seq.luma)).to(device)
        self.alpha = torch.from_numpy(np.ascontiguousarray(seq.alpha)).to(device)
        self.F, self.H, self.W = seq.luma.shape
        self.V = seq.alpha.shape[0]
        self.hm, self.wm = self.H // 16, self.W // 16
        self.cls = torch.zeros((max(self.V, 1), self.F, self.hm, self.wm), dtype=torch.uint8, device=device)
        self.bab = torch.zeros((max(self.V, 1), self.F, self.hm * self.wm * 8), dtype=torch.int32, device=device)

    def classify_frames(self):
        """(frames, class pointers, BAB pointers) for every (VOP, frame)."""
        fr, cp, bp = [], [], []
        for v in range(self.V):
            for t in range(self.F):
                fr.append(frame(self.luma[t], self.alpha[v, t]))
                cp.append(ptr(self.cls[v, t]))
                bp.append(ptr(self.bab[v, t]))
        return fr, cp, bp

    def padded_refs(self, stream=None) -> torch.Tensor:
        """Every (VOP, frame) luma after MPEG-4 reference VOP padding
        (``me_pad_vops``, one call): (V, F, H, W) uint8 on the device."""
        from . import me_pad_vops
        out = torch.empty((self.V, self.F, self.H, self.W), dtype=torch.uint8, device=self.luma.device)
        frames = [frame(self.luma[t], self.alpha[v, t]) for v in range(self.V) for t in range(self.F)]
        me_pad_vops(frames, [out[v, t].data_ptr() for v in range(self.V) for t in range(self.F)],
                    stream=stream_handle() if stream is None else stream)
        return out

    def pair_jobs(self, vop: int | None, out: Outputs, pairs=None, chained=True, use_class=True,
                  seeds: torch.Tensor | None = None, distance: int = 1,
                  refs: torch.Tensor | None = None) -> list[me_job]:
        """Jobs for frame pairs (t - distance, t), t = distance .. distance + P - 1
        (reference ``distance`` frames back).  ``chained``: each pair's T field
        is the previous pair's mv_int (the first pair gets none).  ``refs``
        (V, F, H, W), e.g. from ``padded_refs``: the reference luma of VOP v at
        frame r is refs[v, r] instead of the frame's luma."""
        P = self.F - distance if pairs is None else pairs
        jobs = []
        for i in range(P):
            t = i + distance
            r = t - distance
            ca = ra = cls = None
            if vop is not None:
                ca, ra = self.alpha[vop, t], self.alpha[vop, r]
                cls = self.cls[vop, t] if use_class else None
            tf = out.mv_int[i - 1] if (chained and i > 0) else None
            sd = None if seeds is None else seeds[i]
            rl = refs[vop, r] if (refs is not None and vop is not None) else self.luma[r]
            jobs.append(job(self.luma[t], rl, ca, ra, cls, tf, out, i, sd))
        return jobs
