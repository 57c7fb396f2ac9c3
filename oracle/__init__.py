"""CPU oracle of the shape-adaptive motion estimator (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the GPU library never does.  The C
routines in ``me_oracle.c`` are the plain definition of every step of the
method (Fig. 1, Eqs. 3-5 of the paper); this module only marshals numpy
arrays into them.  ``net.py`` holds the float64 reference of the learned
proposal network.

Frames are numpy ``uint8`` arrays of shape (H, W); motion vectors are int16
(x, y) pairs in half-pel units with shape (H/16, W/16, 2).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "me_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TRANSPARENT, OPAQUE, BOUNDARY = 0, 1, 2
ES, TSS, DS, FSS = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vector intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Pair(C.Structure):
    _fields_ = [("cur_luma", C.c_void_p), ("ref_luma", C.c_void_p),
                ("cur_alpha", C.c_void_p), ("ref_alpha", C.c_void_p),
                ("width", C.c_int), ("height", C.c_int), ("stride", C.c_int)]


class _Params(C.Structure):
    _fields_ = [("search_range", C.c_int), ("theta", C.c_int), ("eps_q12", C.c_int),
                ("max_step", C.c_int), ("k_max", C.c_int), ("half_pel", C.c_int),
                ("unrestricted", C.c_int), ("t_texture", C.c_int), ("masked_prs", C.c_int)]


@dataclass
class Params:
    search_range: int = 16
    theta: int = 3
    eps_q12: int = 4096
    max_step: int = 1
    k_max: int = 8
    half_pel: int = 0
    unrestricted: int = 0
    t_texture: int = 0
    masked_prs: int = 0

    def _c(self) -> _Params:
        return _Params(self.search_range, self.theta, self.eps_q12, self.max_step,
                       self.k_max, int(self.half_pel), int(self.unrestricted), int(self.t_texture),
                       int(self.masked_prs))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, i, u32 = C.c_void_p, C.c_int, C.c_uint32
        L.or_classify.argtypes = [vp, i, i, i, vp, vp]
        L.or_classify.restype = i
        for f in (L.or_sad, L.or_mismatch):
            f.argtypes = [C.POINTER(_Pair), i, i, i, i]
            f.restype = u32
        L.or_sad_half.argtypes = [C.POINTER(_Pair), i, i, i, i]
        L.or_sad_half.restype = u32
        L.or_recip.argtypes = [i, i]
        L.or_recip.restype = C.c_int32
        L.or_step.argtypes = [C.c_int32, i, i]
        L.or_step.restype = i
        L.or_prs_pass.argtypes = [C.POINTER(_Pair), i, i, i, i, i, i,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.or_prs_pass.restype = None
        L.or_pa.argtypes = [C.POINTER(_Pair), vp, vp, vp, C.POINTER(_Params), i,
                            vp, vp, vp, vp, vp]
        L.or_pa.restype = i
        L.or_pa_order.argtypes = [C.POINTER(_Pair), vp, vp, vp, C.POINTER(_Params), i, vp,
                                  vp, vp, vp, vp, vp]
        L.or_pa_order.restype = i
        L.or_search.argtypes = [i, C.POINTER(_Pair), vp, C.POINTER(_Params), vp, vp, vp, vp]
        L.or_search.restype = i
        L.or_mc_sse.argtypes = [C.POINTER(_Pair), vp, vp, vp,
                                C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.or_mc_sse.restype = i
        L.or_prs8.argtypes = [C.POINTER(_Pair), vp, vp, vp, C.POINTER(_Params), vp, vp, vp, vp]
        L.or_prs8.restype = i
        L.or_mc4_sse.argtypes = [C.POINTER(_Pair), vp, vp, vp,
                                 C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.or_mc4_sse.restype = i
        L.or_pad_vop.argtypes = [vp, vp, i, i, i, vp, i]
        L.or_pad_vop.restype = i
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def _pair(cur, ref, cur_alpha=None, ref_alpha=None):
    cur, ref = _u8(cur), _u8(ref)
    cur_alpha, ref_alpha = _u8(cur_alpha), _u8(ref_alpha)
    H, W = cur.shape
    p = _Pair(_ptr(cur), _ptr(ref), _ptr(cur_alpha), _ptr(ref_alpha), W, H, W)
    return p, (cur, ref, cur_alpha, ref_alpha)   # keep the arrays alive


def classify(alpha):
    """-> (classes (H/16, W/16) u8, BAB words (H/16, W/16, 8) u32)."""
    a = _u8(alpha)
    H, W = a.shape
    cls = np.zeros((H // 16, W // 16), dtype=np.uint8)
    bab = np.zeros((H // 16, W // 16, 8), dtype=np.uint32)
    rc = lib().or_classify(_ptr(a), W, H, W, _ptr(cls), _ptr(bab))
    if rc:
        raise ValueError("or_classify rejected its arguments")
    return cls, bab


def sad(cur, ref, x0, y0, dx, dy):
    p, keep = _pair(cur, ref)
    return int(lib().or_sad(C.byref(p), x0, y0, dx, dy))


def mismatch(cur_alpha, ref_alpha, x0, y0, dx, dy):
    p, keep = _pair(cur_alpha, ref_alpha, cur_alpha, ref_alpha)
    return int(lib().or_mismatch(C.byref(p), x0, y0, dx, dy))


def sad_half(cur, ref, x0, y0, hx, hy):
    p, keep = _pair(cur, ref)
    return int(lib().or_sad_half(C.byref(p), x0, y0, hx, hy))


def recip(g, theta):
    return int(lib().or_recip(int(g), int(theta)))


def step(u, eps_q12, max_step):
    return int(lib().or_step(int(u), int(eps_q12), int(max_step)))


def prs_pass(cur, ref, x0, y0, dx, dy, theta=3, shape=False, cur_alpha=None, ref_alpha=None):
    p, keep = _pair(cur, ref, cur_alpha, ref_alpha)
    ux, uy = C.c_int32(), C.c_int32()
    lib().or_prs_pass(C.byref(p), int(shape), theta, x0, y0, dx, dy, C.byref(ux), C.byref(uy))
    return int(ux.value), int(uy.value)


def _outputs(H, W):
    hm, wm = H // 16, W // 16
    return dict(mv=np.zeros((hm, wm, 2), np.int16), mv_int=np.zeros((hm, wm, 2), np.int16),
                cost=np.zeros((hm, wm), np.uint32), iters=np.zeros((hm, wm), np.uint8),
                points=np.zeros((hm, wm), np.uint16))


def pa(cur, ref, params: Params, cur_alpha=None, ref_alpha=None, cls=None, t_field=None,
       seed=None, shape_only=False):
    """The proposed algorithm (Fig. 1) on one frame pair of one VOP."""
    p, keep = _pair(cur, ref, cur_alpha, ref_alpha)
    H, W = keep[0].shape
    out = _outputs(H, W)
    cls = _u8(cls)
    tf = None if t_field is None else np.ascontiguousarray(t_field, dtype=np.int16)
    sd = None if seed is None else np.ascontiguousarray(seed, dtype=np.int16)
    prm = params._c()
    rc = lib().or_pa(C.byref(p), _ptr(cls), _ptr(tf), _ptr(sd), C.byref(prm), int(shape_only),
                     _ptr(out["mv"]), _ptr(out["mv_int"]), _ptr(out["cost"]),
                     _ptr(out["iters"]), _ptr(out["points"]))
    if rc:
        raise ValueError("or_pa rejected its arguments")
    return out


def pa_order(cur, ref, params: Params, order, cur_alpha=None, ref_alpha=None, cls=None, t_field=None,
             seed=None, shape_only=False):
    """The proposed algorithm with the MBs visited in ``order`` (flat MB
    indices, each once) instead of the raster scan."""
    p, keep = _pair(cur, ref, cur_alpha, ref_alpha)
    H, W = keep[0].shape
    out = _outputs(H, W)
    cls = _u8(cls)
    tf = None if t_field is None else np.ascontiguousarray(t_field, dtype=np.int16)
    sd = None if seed is None else np.ascontiguousarray(seed, dtype=np.int16)
    od = np.ascontiguousarray(order, dtype=np.int32)
    if od.shape != ((H // 16) * (W // 16),):
        raise ValueError("order must list every MB once")
    prm = params._c()
    rc = lib().or_pa_order(C.byref(p), _ptr(cls), _ptr(tf), _ptr(sd), C.byref(prm), int(shape_only), _ptr(od),
                           _ptr(out["mv"]), _ptr(out["mv_int"]), _ptr(out["cost"]),
                           _ptr(out["iters"]), _ptr(out["points"]))
    if rc:
        raise ValueError("or_pa_order rejected its arguments")
    return out


def search(method, cur, ref, params: Params, cls=None):
    """Baseline search (ES / TSS / DS / FSS) on one frame pair."""
    p, keep = _pair(cur, ref)
    H, W = keep[0].shape
    out = _outputs(H, W)
    cls = _u8(cls)
    prm = params._c()
    rc = lib().or_search(int(method), C.byref(p), _ptr(cls), C.byref(prm), _ptr(out["mv"]),
                         _ptr(out["mv_int"]), _ptr(out["cost"]), _ptr(out["points"]))
    if rc:
        raise ValueError("or_search rejected its arguments")
    return out


def mc_sse(cur, ref, mv, cur_alpha=None, cls=None, want_pred=False):
    """-> (sse, npix, pred or None)."""
    p, keep = _pair(cur, ref, cur_alpha, None)
    H, W = keep[0].shape
    mvv = np.ascontiguousarray(mv, dtype=np.int16)
    cls = _u8(cls)
    pred = np.zeros((H, W), np.uint8) if want_pred else None
    s, n = C.c_uint64(), C.c_uint64()
    rc = lib().or_mc_sse(C.byref(p), _ptr(cls), _ptr(mvv), _ptr(pred), C.byref(s), C.byref(n))
    if rc:
        raise ValueError("or_mc_sse rejected its arguments")
    return int(s.value), int(n.value), pred


def prs8(cur, ref, params: Params, mv, mv_int, cls=None):
    """Four-vector mode: the pel-recursive refinement on each 8 x 8 block of
    the texture MBs from the MB vectors (mv, mv_int: an or_pa result).
    -> dict mv4 (H/16, W/16, 4, 2), cost4 / iters4 / points4 (H/16, W/16, 4)."""
    p, keep = _pair(cur, ref)
    H, W = keep[0].shape
    hm, wm = H // 16, W // 16
    out = dict(mv4=np.zeros((hm, wm, 4, 2), np.int16), cost4=np.zeros((hm, wm, 4), np.uint32),
               iters4=np.zeros((hm, wm, 4), np.uint8), points4=np.zeros((hm, wm, 4), np.uint16))
    cls = _u8(cls)
    mvv = np.ascontiguousarray(mv, dtype=np.int16)
    mvi = np.ascontiguousarray(mv_int, dtype=np.int16)
    prm = params._c()
    rc = lib().or_prs8(C.byref(p), _ptr(cls), _ptr(mvv), _ptr(mvi), C.byref(prm), _ptr(out["mv4"]),
                       _ptr(out["cost4"]), _ptr(out["iters4"]), _ptr(out["points4"]))
    if rc:
        raise ValueError("or_prs8 rejected its arguments")
    return out


def mc4_sse(cur, ref, mv4, cur_alpha=None, cls=None, want_pred=False):
    """MC with four vectors per MB -> (sse, npix, pred or None)."""
    p, keep = _pair(cur, ref, cur_alpha, None)
    H, W = keep[0].shape
    mvv = np.ascontiguousarray(mv4, dtype=np.int16)
    cls = _u8(cls)
    pred = np.zeros((H, W), np.uint8) if want_pred else None
    s, n = C.c_uint64(), C.c_uint64()
    rc = lib().or_mc4_sse(C.byref(p), _ptr(cls), _ptr(mvv), _ptr(pred), C.byref(s), C.byref(n))
    if rc:
        raise ValueError("or_mc4_sse rejected its arguments")
    return int(s.value), int(n.value), pred


def pad_vop(luma, alpha):
    """MPEG-4 padding of a reference VOP (boundary MBs: repetitive padding,
    transparent MBs: extended padding) -> padded luma (H, W) u8."""
    lu, al = _u8(luma), _u8(alpha)
    H, W = lu.shape
    out = np.zeros((H, W), np.uint8)
    rc = lib().or_pad_vop(_ptr(lu), _ptr(al), W, H, W, _ptr(out), W)
    if rc:
        raise ValueError("or_pad_vop rejected its arguments")
    return out


def psnr_db(sse: int, npix: int) -> float:
    """10 log10(255^2 N / SSE); +inf for a perfect prediction."""
    if npix == 0:
        raise ValueError("PSNR over zero pixels")
    if sse == 0:
        return float("inf")
    return 10.0 * np.log10(255.0 * 255.0 * npix / sse)


def pa_sequence(seq, vop: int | None, params: Params, shape_only=False, pairs=None, seeds=None, distance=1,
                padded=False):
    """Run the proposed algorithm over the frame pairs (t - distance, t),
    t = distance, distance + 1, ... of a synthetic sequence (Section 4 uses a
    distance of two), feeding each pair's full-pel field forward as the
    temporal candidate of the next.  ``vop=None`` treats frames as
    rectangular.  ``padded``: the reference luma is the reference VOP after
    MPEG-4 padding (``pad_vop``), for search and MC alike.  Returns a list of
    per-pair dicts (with classes and SSE)."""
    n = seq.frames - distance if pairs is None else pairs
    res = []
    t_field = None
    for i in range(n):
        t = i + distance
        cur, ref = seq.luma[t], seq.luma[t - distance]
        ca = ra = cls = None
        if vop is not None:
            ca, ra = seq.alpha[vop, t], seq.alpha[vop, t - distance]
            cls, _ = classify(ca)
            if padded:
                ref = pad_vop(ref, ra)
        sd = None if seeds is None else seeds[i]
        out = pa(cur, ref, params, ca, ra, cls, t_field, sd, shape_only)
        out["cls"] = cls
        sse, npx, _ = mc_sse(cur, ref, out["mv"], ca, cls)
        out["sse"], out["npix"] = sse, npx
        res.append(out)
        t_field = out["mv_int"]
    return res
