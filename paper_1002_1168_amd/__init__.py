"""Python binding of the gfx950 shape-adaptive motion-estimation library.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libme.so`` (C ABI in ``include/me.h``).  The functions below carry the
C names and take ctypes structs whose pointer fields are device addresses
(e.g. ``torch.Tensor.data_ptr()`` of CUDA tensors).  If the library is not
built, every call raises ``MeError``: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libme.so")

ME_OK, ME_EINVAL, ME_EALIGN, ME_EHIP, ME_ENOMEM, ME_EEMPTY, ME_EDEVICE, ME_ENODEV = 0, -1, -2, -3, -4, -5, -6, -7
ME_EFORMAT, ME_EIO = -8, -9
ME_MB_TRANSPARENT, ME_MB_OPAQUE, ME_MB_BOUNDARY = 0, 1, 2
ME_ES, ME_TSS, ME_DS, ME_4SS = 0, 1, 2, 3
ME_KT_CLASSIFY, ME_KT_SEARCH, ME_KT_FULL, ME_KT_MC, ME_KT_NET, ME_KT_NET_TRAIN, ME_KT_REFINE8 = 0, 1, 2, 3, 4, 5, 6
ME_BATCH_SHAPE, ME_BATCH_AUTOTUNE = 1, 2
ME_FLAG_UNRESTRICTED, ME_FLAG_T_TEXTURE, ME_FLAG_MASKED_PRS, ME_FLAG_LINE_WORKERS = 0x1, 0x2, 0x4, 0x100
ME_NET_PARAMS = 10434

EXPORTED = ("me_default_params", "me_status_str", "me_shutdown", "me_classify_babs", "me_pad_vops",
            "me_texture_recursive",
            "me_shape_search", "me_full_search", "me_motion_compensate_psnr", "me_motion_compensate_sse",
            "me_motion_compensate_sse_noalloc", "me_refine_8x8", "me_motion_compensate4_sse", "me_device_status",
            "me_kernel_timing", "me_kernel_time_ms", "me_batch_create", "me_batch_step", "me_batch_results",
            "me_batch_config", "me_batch_set_config", "me_batch_kernel_time_ms", "me_batch_set_net", "me_batch_destroy", "me_net_create", "me_net_forward", "me_net_backward",
            "me_net_sgd_step", "me_net_train_step", "me_net_weights", "me_net_scale", "me_net_save", "me_net_load",
            "me_net_destroy", "me_search_schedule")


class MeError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {status_str(code)} ({code})" if what else f"{status_str(code)} ({code})")


class me_frame(C.Structure):
    _fields_ = [("luma", C.c_void_p), ("alpha", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32), ("stride", C.c_int32)]


class me_params(C.Structure):
    _fields_ = [("search_range", C.c_int32), ("theta", C.c_int32), ("eps_q12", C.c_int32),
                ("max_step", C.c_int32), ("k_max", C.c_int32), ("half_pel", C.c_int32),
                ("flags", C.c_uint32)]


class me_job(C.Structure):
    _fields_ = [("cur", me_frame), ("ref", me_frame), ("mb_class", C.c_void_p),
                ("t_field", C.c_void_p), ("seed", C.c_void_p), ("mv", C.c_void_p),
                ("mv_int", C.c_void_p), ("cost", C.c_void_p), ("iters", C.c_void_p),
                ("points", C.c_void_p)]


_lib = None


def lib():
    """The loaded ``libme.so`` (raises MeError when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MeError(ME_ENODEV, f"HIP library missing at {LIB_PATH}; run `python -m paper_1002_1168_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i = C.c_void_p, C.c_int
        L.me_default_params.argtypes = [C.POINTER(me_params)]
        L.me_default_params.restype = None
        L.me_status_str.argtypes = [i]
        L.me_status_str.restype = C.c_char_p
        L.me_shutdown.argtypes = []
        L.me_shutdown.restype = None
        L.me_classify_babs.argtypes = [C.POINTER(me_frame), i, C.POINTER(vp), C.POINTER(vp), vp]
        L.me_classify_babs.restype = i
        L.me_pad_vops.argtypes = [C.POINTER(me_frame), i, C.POINTER(vp), vp]
        L.me_pad_vops.restype = i
        L.me_texture_recursive.argtypes = [C.POINTER(me_job), i, C.POINTER(me_params), vp, vp]
        L.me_texture_recursive.restype = i
        L.me_shape_search.argtypes = [C.POINTER(me_job), i, C.POINTER(me_params), vp]
        L.me_shape_search.restype = i
        L.me_full_search.argtypes = [i, C.POINTER(me_job), i, C.POINTER(me_params), vp]
        L.me_full_search.restype = i
        L.me_motion_compensate_psnr.argtypes = [C.POINTER(me_job), i, C.POINTER(vp), C.POINTER(C.c_uint64),
                                                C.POINTER(C.c_uint64), C.POINTER(C.c_double), vp]
        L.me_motion_compensate_psnr.restype = i
        L.me_motion_compensate_sse.argtypes = [C.POINTER(me_job), i, C.POINTER(vp), vp, vp]
        L.me_motion_compensate_sse.restype = i
        L.me_refine_8x8.argtypes = [C.POINTER(me_job), i, C.POINTER(me_params), C.POINTER(vp), C.POINTER(vp),
                                    C.POINTER(vp), C.POINTER(vp), vp]
        L.me_refine_8x8.restype = i
        L.me_motion_compensate4_sse.argtypes = [C.POINTER(me_job), i, C.POINTER(vp), C.POINTER(vp), vp, vp]
        L.me_motion_compensate4_sse.restype = i
        L.me_motion_compensate_sse_noalloc.argtypes = [C.POINTER(me_job), i, C.POINTER(vp), vp, vp]
        L.me_motion_compensate_sse_noalloc.restype = i
        L.me_device_status.argtypes = [vp]
        L.me_device_status.restype = i
        L.me_kernel_timing.argtypes = [i]
        L.me_kernel_timing.restype = i
        L.me_kernel_time_ms.argtypes = [i, vp, C.POINTER(C.c_double), C.POINTER(i)]
        L.me_kernel_time_ms.restype = i
        L.me_batch_create.argtypes = [C.POINTER(me_job), i, C.POINTER(me_params), C.c_uint32, vp, C.POINTER(vp)]
        L.me_batch_create.restype = i
        L.me_batch_step.argtypes = [vp, C.POINTER(me_job), i]
        L.me_batch_step.restype = i
        L.me_batch_results.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_double), i]
        L.me_batch_results.restype = i
        L.me_batch_config.argtypes = [vp, C.POINTER(C.c_int32), i]
        L.me_batch_config.restype = i
        L.me_batch_set_config.argtypes = [vp, C.POINTER(C.c_int32), i]
        L.me_batch_set_config.restype = i
        L.me_batch_kernel_time_ms.argtypes = [vp, i, C.POINTER(C.c_double), C.POINTER(i)]
        L.me_batch_kernel_time_ms.restype = i
        L.me_batch_set_net.argtypes = [vp, vp]
        L.me_batch_set_net.restype = i
        L.me_batch_destroy.argtypes = [vp]
        L.me_batch_destroy.restype = None
        L.me_net_create.argtypes = [C.POINTER(C.c_float), C.c_int32, C.POINTER(vp)]
        L.me_net_create.restype = i
        L.me_net_backward.argtypes = [vp, C.POINTER(me_job), i, C.POINTER(vp), vp, C.POINTER(C.c_double), vp]
        L.me_net_backward.restype = i
        L.me_net_sgd_step.argtypes = [vp, vp, C.c_float, C.c_float, vp]
        L.me_net_sgd_step.restype = i
        L.me_net_scale.argtypes = [vp]
        L.me_net_scale.restype = i
        L.me_net_save.argtypes = [vp, C.c_char_p]
        L.me_net_save.restype = i
        L.me_net_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.me_net_load.restype = i
        L.me_net_forward.argtypes = [vp, C.POINTER(me_job), i, C.POINTER(vp), vp]
        L.me_net_forward.restype = i
        L.me_net_train_step.argtypes = [vp, C.POINTER(me_job), i, C.POINTER(vp), C.c_float, C.c_float, vp,
                                        C.POINTER(C.c_double), vp]
        L.me_net_train_step.restype = i
        L.me_net_weights.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.me_net_weights.restype = i
        L.me_search_schedule.argtypes = [C.POINTER(me_job), i, vp, vp, i, C.POINTER(i)]
        L.me_search_schedule.restype = i
        L.me_net_destroy.argtypes = [vp]
        L.me_net_destroy.restype = None
        _lib = L
    return _lib


def status_str(code: int) -> str:
    try:
        return lib().me_status_str(int(code)).decode()
    except MeError:
        return {0: "ok"}.get(code, f"status {code}")


def _check(rc: int, what: str) -> int:
    if rc != ME_OK:
        raise MeError(rc, what)
    return rc


def _arr(ctype, items):
    """ctypes array of `items`; a ctypes array of `ctype` is used as is."""
    if isinstance(items, C.Array) and items._type_ is ctype:
        return items, len(items)
    items = list(items)
    return (ctype * max(len(items), 1))(*items), len(items)


def job_array(jobs) -> C.Array:
    """Prebuilt me_job array: pass it instead of a list to skip per-call
    marshalling when the same job set is launched repeatedly."""
    jobs = list(jobs)
    return (me_job * len(jobs))(*jobs)


def me_default_params(**over) -> me_params:
    p = me_params()
    lib().me_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, int(v))
    return p


def me_shutdown() -> None:
    lib().me_shutdown()


def me_classify_babs(frames, mb_class, bab_bits=None, stream=None, check=True) -> int:
    """``frames``: me_frame list; ``mb_class`` / ``bab_bits``: device addresses."""
    fa, n = _arr(me_frame, frames)
    ca, _ = _arr(C.c_void_p, mb_class)
    ba = None if bab_bits is None else _arr(C.c_void_p, bab_bits)[0]
    rc = lib().me_classify_babs(fa, n, ca, ba, stream)
    return _check(rc, "me_classify_babs") if check else rc


def me_pad_vops(frames, padded, stream=None, check=True) -> int:
    """``frames``: me_frame list (reference luma + VOP alpha); ``padded``:
    device addresses of the padded planes (same stride as each frame)."""
    fa, n = _arr(me_frame, frames)
    pa, _ = _arr(C.c_void_p, padded)
    rc = lib().me_pad_vops(fa, n, pa, stream)
    return _check(rc, "me_pad_vops") if check else rc


def me_texture_recursive(jobs, params: me_params, net=None, stream=None, check=True) -> int:
    """``net``: None (plain method) or a :class:`Net` whose proposals are
    written into the jobs' seed buffers first."""
    ja, n = _arr(me_job, jobs)
    h = net.handle if isinstance(net, Net) else net
    rc = lib().me_texture_recursive(ja, n, C.byref(params), h, stream)
    return _check(rc, "me_texture_recursive") if check else rc


def me_shape_search(jobs, params: me_params, stream=None, check=True) -> int:
    ja, n = _arr(me_job, jobs)
    rc = lib().me_shape_search(ja, n, C.byref(params), stream)
    return _check(rc, "me_shape_search") if check else rc


def me_full_search(method: int, jobs, params: me_params, stream=None, check=True) -> int:
    ja, n = _arr(me_job, jobs)
    rc = lib().me_full_search(int(method), ja, n, C.byref(params), stream)
    return _check(rc, "me_full_search") if check else rc


def me_motion_compensate_psnr(jobs, pred=None, stream=None, check=True):
    """-> (sse list, npix list, psnr_db list, status)."""
    ja, n = _arr(me_job, jobs)
    pa = None if pred is None else _arr(C.c_void_p, pred)[0]
    sse = (C.c_uint64 * max(n, 1))()
    npx = (C.c_uint64 * max(n, 1))()
    ps = (C.c_double * max(n, 1))()
    rc = lib().me_motion_compensate_psnr(ja, n, pa, sse, npx, ps, stream)
    if check and rc not in (ME_OK,):
        raise MeError(rc, "me_motion_compensate_psnr")
    return list(sse)[:n], list(npx)[:n], list(ps)[:n], rc


def me_motion_compensate_sse(jobs, sums, pred=None, stream=None, check=True) -> int:
    """``sums``: device address of 2n uint64 receiving (SSE, pixel count)
    per job when the stream gets there; returns without waiting."""
    ja, n = _arr(me_job, jobs)
    pa = None if pred is None else _arr(C.c_void_p, pred)[0]
    rc = lib().me_motion_compensate_sse(ja, n, pa, sums, stream)
    return _check(rc, "me_motion_compensate_sse") if check else rc


def me_refine_8x8(jobs, params: me_params, mv4, cost4=None, iters4=None, points4=None, stream=None,
                  check=True) -> int:
    """Four vectors per MB: ``mv4`` (and the optional per-block outputs) are
    lists of device addresses, one per job."""
    ja, n = _arr(me_job, jobs)
    m4 = _arr(C.c_void_p, mv4)[0]
    c4 = None if cost4 is None else _arr(C.c_void_p, cost4)[0]
    i4 = None if iters4 is None else _arr(C.c_void_p, iters4)[0]
    p4 = None if points4 is None else _arr(C.c_void_p, points4)[0]
    rc = lib().me_refine_8x8(ja, n, C.byref(params), m4, c4, i4, p4, stream)
    return _check(rc, "me_refine_8x8") if check else rc


def me_motion_compensate4_sse(jobs, mv4, sums, pred=None, stream=None, check=True) -> int:
    """MC with four vectors per MB (``mv4``: per-job device addresses)."""
    ja, n = _arr(me_job, jobs)
    m4 = _arr(C.c_void_p, mv4)[0]
    pa = None if pred is None else _arr(C.c_void_p, pred)[0]
    rc = lib().me_motion_compensate4_sse(ja, n, m4, pa, sums, stream)
    return _check(rc, "me_motion_compensate4_sse") if check else rc


def me_motion_compensate_sse_noalloc(jobs, sums, pred=None, stream=None, check=True) -> int:
    """As me_motion_compensate_sse, with no allocation (fixed device scratch)."""
    ja, n = _arr(me_job, jobs)
    pa = None if pred is None else _arr(C.c_void_p, pred)[0]
    rc = lib().me_motion_compensate_sse_noalloc(ja, n, pa, sums, stream)
    return _check(rc, "me_motion_compensate_sse_noalloc") if check else rc


def me_device_status(stream=None) -> int:
    return lib().me_device_status(stream)


def me_kernel_timing(on: bool, kinds=None) -> int:
    """Timing on for every call kind, or only for the ME_KT_* in ``kinds``."""
    mask = (sum(2 << k for k in set(kinds)) if kinds else 1) if on else 0
    return _check(lib().me_kernel_timing(mask), "me_kernel_timing")


def me_kernel_time_ms(kind: int, stream=None):
    """-> (total ms, launches) of the main kernel of `kind` (ME_KT_*) over the
    timed calls since the previous read."""
    ms, cnt = C.c_double(), C.c_int()
    _check(lib().me_kernel_time_ms(int(kind), stream, C.byref(ms), C.byref(cnt)), "me_kernel_time_ms")
    return float(ms.value), int(cnt.value)


class Batch:
    """A batched frame step (``me_batch_*``): created from one job set,
    stepped with job sets of the same structure, one graph launch per step."""

    def __init__(self, jobs, params: me_params, flags: int = 0, stream=None):
        ja, n = _arr(me_job, jobs)
        h = C.c_void_p()
        _check(lib().me_batch_create(ja, n, C.byref(params), int(flags), stream, C.byref(h)), "me_batch_create")
        self.handle, self.n = h, n

    def step(self, jobs, check=True) -> int:
        ja, n = _arr(me_job, jobs)
        rc = lib().me_batch_step(self.handle, ja, n)
        return _check(rc, "me_batch_step") if check else rc

    def results(self, check=True):
        """-> (sse list, npix list, psnr_db list, status) of the last step."""
        n = self.n
        sse, npx, ps = (C.c_uint64 * n)(), (C.c_uint64 * n)(), (C.c_double * n)()
        rc = lib().me_batch_results(self.handle, sse, npx, ps, n)
        if check and rc != ME_OK:
            raise MeError(rc, "me_batch_results")
        return list(sse), list(npx), list(ps), rc

    def set_net(self, net) -> None:
        """Seed every step's search with proposal network ``net`` (None: plain)."""
        _check(lib().me_batch_set_net(self.handle, None if net is None else net.handle), "me_batch_set_net")
        self._net = net   # keep it alive while attached

    def config(self) -> dict:
        c = (C.c_int32 * 6)()
        _check(lib().me_batch_config(self.handle, c, 6), "me_batch_config")
        return {"workers": c[0], "staging": "plan" if c[1] else "generic", "poll_sleep": c[2], "flat_per_cu": c[3],
                "waves_per_line": c[4], "search": "rows" if c[5] else "lines"}

    def set_config(self, cfg: dict, check=True) -> int:
        """Force the launch configuration (keys as returned by config())."""
        c = (C.c_int32 * 6)(int(cfg["workers"]), 1 if cfg["staging"] == "plan" else 0, int(cfg["poll_sleep"]),
                            int(cfg["flat_per_cu"]), int(cfg["waves_per_line"]),
                            1 if cfg.get("search", "lines") == "rows" else 0)
        rc = lib().me_batch_set_config(self.handle, c, 6)
        return _check(rc, "me_batch_set_config") if check else rc

    def kernel_time_ms(self, kind: int):
        """-> (total ms, replays) of the kernel of ``kind`` inside the graph."""
        ms, cnt = C.c_double(), C.c_int()
        _check(lib().me_batch_kernel_time_ms(self.handle, int(kind), C.byref(ms), C.byref(cnt)),
               "me_batch_kernel_time_ms")
        return float(ms.value), int(cnt.value)

    def close(self) -> None:
        if self.handle:
            lib().me_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The learned motion-vector proposal network (``me_net_*``); ``scale``:
    window scale 2 (reference window [-16, 32)) or 4 ([-40, 56))."""

    def __init__(self, init, scale: int = 2):
        import numpy as np
        w = np.ascontiguousarray(init, dtype=np.float32)
        if w.shape != (ME_NET_PARAMS,):
            raise MeError(ME_EINVAL, "Net: init must hold ME_NET_PARAMS floats")
        h = C.c_void_p()
        _check(lib().me_net_create(w.ctypes.data_as(C.POINTER(C.c_float)), int(scale), C.byref(h)), "me_net_create")
        self.handle = h

    @classmethod
    def load(cls, path: str) -> "Net":
        """A network from a checkpoint written by save() (me_net_load)."""
        h = C.c_void_p()
        _check(lib().me_net_load(os.fsencode(path), C.byref(h)), f"me_net_load {path}")
        obj = cls.__new__(cls)
        obj.handle = h
        return obj

    def save(self, path: str) -> None:
        _check(lib().me_net_save(self.handle, os.fsencode(path)), f"me_net_save {path}")

    @property
    def scale(self) -> int:
        return int(lib().me_net_scale(self.handle))

    def backward(self, jobs, labels, grad, want_loss=True, stream=None):
        """Gradient into ``grad`` (device address of ME_NET_PARAMS floats);
        -> loss (None unless want_loss).  The weights are unchanged."""
        ja, n = _arr(me_job, jobs)
        la, _ = _arr(C.c_void_p, labels)
        loss = C.c_double()
        _check(lib().me_net_backward(self.handle, ja, n, la, grad, C.byref(loss) if want_loss else None, stream),
               "me_net_backward")
        return float(loss.value) if want_loss else None

    def sgd_step(self, grad, lr: float, momentum: float, stream=None) -> None:
        """Momentum SGD from the gradient at device address ``grad``."""
        _check(lib().me_net_sgd_step(self.handle, grad, float(lr), float(momentum), stream), "me_net_sgd_step")

    def forward(self, jobs, pred=None, stream=None, check=True) -> int:
        """Seeds into the jobs' seed buffers; ``pred``: per-job device
        pointers (or None) receiving the raw predictions."""
        ja, n = _arr(me_job, jobs)
        pa = None if pred is None else _arr(C.c_void_p, pred)[0]
        rc = lib().me_net_forward(self.handle, ja, n, pa, stream)
        return _check(rc, "me_net_forward") if check else rc

    def train_step(self, jobs, labels, lr: float, momentum: float, grad=None, want_loss=True, stream=None):
        """One SGD step; -> loss before the step (None unless want_loss)."""
        ja, n = _arr(me_job, jobs)
        la, _ = _arr(C.c_void_p, labels)
        loss = C.c_double()
        _check(lib().me_net_train_step(self.handle, ja, n, la, float(lr), float(momentum), grad,
                                       C.byref(loss) if want_loss else None, stream), "me_net_train_step")
        return float(loss.value) if want_loss else None

    def weights(self, momentum=False):
        import numpy as np
        w = np.empty(ME_NET_PARAMS, np.float32)
        v = np.empty(ME_NET_PARAMS, np.float32) if momentum else None
        _check(lib().me_net_weights(self.handle, w.ctypes.data_as(C.POINTER(C.c_float)),
                                    None if v is None else v.ctypes.data_as(C.POINTER(C.c_float))),
               "me_net_weights")
        return (w, v) if momentum else w

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().me_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
