"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/me.h, and rejects invalid arguments with the documented
codes before touching the device."""
import ctypes as C
import os
import re

import pytest

import paper_1002_1168_amd as me

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "me.h")

pytestmark = pytest.mark.skipif(not os.path.exists(me.LIB_PATH), reason="libme.so not built")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(me_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    L = C.CDLL(me.LIB_PATH)
    names = declared_functions()
    assert "me_texture_recursive" in names and "me_classify_babs" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(me.EXPORTED) <= set(names)


def test_status_strings_and_defaults():
    assert me.status_str(0) == "ok"
    assert "alignment" in me.status_str(me.ME_EALIGN)
    p = me.me_default_params()
    assert (p.search_range, p.theta, p.eps_q12, p.max_step, p.k_max, p.half_pel, p.flags) == (16, 3, 4096, 1, 8, 0, 0)


FAKE = 0x10000  # never dereferenced: validation fails before any HIP call


def frame(w=64, h=48, stride=None, luma=FAKE, alpha=None):
    return me.me_frame(luma, alpha, w, h, w if stride is None else stride)


def job(**kw):
    j = me.me_job(frame(), frame(), None, None, None, FAKE, FAKE + 4096, None, None, None)
    for k, v in kw.items():
        setattr(j, k, v)
    return j


@pytest.mark.parametrize("over,code", [
    (dict(search_range=0), me.ME_EINVAL), (dict(search_range=65), me.ME_EINVAL),
    (dict(theta=0), me.ME_EINVAL), (dict(eps_q12=-1), me.ME_EINVAL),
    (dict(max_step=0), me.ME_EINVAL), (dict(max_step=17), me.ME_EINVAL),
    (dict(k_max=256), me.ME_EINVAL), (dict(half_pel=2), me.ME_EINVAL), (dict(flags=8), me.ME_EINVAL),
    (dict(flags=0x200), me.ME_EINVAL)])
def test_bad_params(over, code):
    p = me.me_default_params(**over)
    assert me.me_texture_recursive([job()], p, check=False) == code
    assert me.me_full_search(me.ME_ES, [job()], p, check=False) == code


@pytest.mark.parametrize("cur,code", [
    (frame(w=60), me.ME_EALIGN), (frame(h=40), me.ME_EALIGN), (frame(stride=62), me.ME_EALIGN),
    (frame(stride=66), me.ME_EALIGN), (frame(luma=FAKE + 1), me.ME_EALIGN), (frame(luma=None), me.ME_EINVAL),
    (frame(w=0), me.ME_EINVAL), (frame(w=4112), me.ME_EINVAL)])
def test_bad_frames(cur, code):
    p = me.me_default_params()
    j = job(cur=cur, ref=cur)
    assert me.me_texture_recursive([j], p, check=False) == code
    assert me.me_classify_babs([frame(luma=cur.luma, alpha=FAKE, w=cur.width, h=cur.height, stride=cur.stride)],
                               [FAKE], check=False) in (code, me.ME_EINVAL)


def test_bad_jobs():
    p = me.me_default_params()
    assert me.me_texture_recursive([job(mv=None)], p, check=False) == me.ME_EINVAL
    assert me.me_texture_recursive([job(ref=frame(w=48))], p, check=False) == me.ME_EINVAL
    assert me.me_texture_recursive([job(cur=frame(alpha=FAKE))], p, check=False) == me.ME_EINVAL  # alpha one-sided
    assert me.me_shape_search([job()], p, check=False) == me.ME_EINVAL                          # needs alpha
    assert me.me_texture_recursive([job(mv=FAKE + 2)], p, check=False) == me.ME_EALIGN
    j = job()
    j.t_field = j.mv_int
    assert me.me_texture_recursive([j], p, check=False) == me.ME_EINVAL                         # reads own output
    a, b = job(), job(mv=FAKE + 8192, mv_int=FAKE + 12288)
    a.t_field = b.mv_int                                                                            # written later
    assert me.me_texture_recursive([a, b], p, check=False) == me.ME_EINVAL
    c = job(mv=FAKE + 8192)
    assert me.me_texture_recursive([job(), c], p, check=False) == me.ME_EINVAL                  # shared mv_int
    assert me.me_full_search(4, [job()], p, check=False) == me.ME_EINVAL
    assert me.me_texture_recursive([job()], p, net=C.c_void_p(FAKE), check=False) == me.ME_EINVAL


def test_seeded_search_caps_k_max():
    # a dropped seed counts both recursions in the byte-wide iteration count,
    # so seeded calls take k_max <= 127 (plain calls keep 0..255)
    p = me.me_default_params(k_max=128)
    assert me.me_texture_recursive([job(seed=FAKE + 8192)], p, check=False) == me.ME_EINVAL
    assert me.me_shape_search([job(seed=FAKE + 8192, cur=frame(alpha=FAKE), ref=frame(alpha=FAKE))], p,
                              check=False) == me.ME_EINVAL
    assert me.me_texture_recursive([job(seed=FAKE + 8192)], p, net=C.c_void_p(FAKE), check=False) == me.ME_EINVAL
    L = me.lib()
    h = C.c_void_p()
    ja = (me.me_job * 1)(job(seed=FAKE + 8192))
    assert L.me_batch_create(ja, 1, C.byref(p), 0, None, C.byref(h)) == me.ME_EINVAL
    # at 127 validation passes (the call then fails only for want of a device)
    p127 = me.me_default_params(k_max=127)
    assert me.me_texture_recursive([job(seed=FAKE + 8192)], p127, check=False) != me.ME_EINVAL


def test_empty_calls_are_ok_without_device():
    p = me.me_default_params()
    assert me.me_texture_recursive([], p, check=False) == me.ME_OK
    assert me.me_full_search(me.ME_DS, [], p, check=False) == me.ME_OK
    assert me.me_classify_babs([], [], check=False) == me.ME_OK
    assert me.me_motion_compensate_psnr([], check=False)[3] == me.ME_OK


def test_psnr_requires_host_outputs():
    L = me.lib()
    ja = (me.me_job * 1)(job())
    assert L.me_motion_compensate_psnr(ja, 1, None, None, None, None, None) == me.ME_EINVAL


def test_async_sse_argument_validation():
    """The queued MC/SSE call checks its arguments on the host first."""
    L = me.lib()
    ja = (me.me_job * 1)(job())
    assert L.me_motion_compensate_sse(ja, 1, None, None, None) == me.ME_EINVAL      # no sums
    assert L.me_motion_compensate_sse(ja, 1, None, FAKE + 4, None) == me.ME_EALIGN  # sums not 8-aligned
    assert L.me_motion_compensate_sse(ja, -1, None, FAKE, None) == me.ME_EINVAL
    assert me.me_motion_compensate_sse([job(mv=None)], FAKE, check=False) == me.ME_EINVAL
    assert me.me_motion_compensate_sse([job(ref=frame(w=48))], FAKE, check=False) == me.ME_EINVAL
    assert me.me_motion_compensate_sse([job(mv=FAKE + 2)], FAKE, check=False) == me.ME_EALIGN
    assert me.me_motion_compensate_sse([], FAKE, check=False) == me.ME_OK


def test_kernel_timing_validation():
    L = me.lib()
    assert L.me_kernel_timing(3) == me.ME_EINVAL      # "every kind" with kind bits
    assert L.me_kernel_timing(2 << 7) == me.ME_EINVAL  # no such kind
    assert L.me_kernel_timing(-1) == me.ME_EINVAL
    assert L.me_kernel_timing((2 << 1) | (2 << 4)) == me.ME_OK  # search and network only
    assert L.me_kernel_timing(0) == me.ME_OK
    ms, cnt = C.c_double(), C.c_int()
    assert L.me_kernel_time_ms(7, None, C.byref(ms), C.byref(cnt)) == me.ME_EINVAL
    assert L.me_kernel_time_ms(-1, None, C.byref(ms), C.byref(cnt)) == me.ME_EINVAL
    assert L.me_kernel_time_ms(me.ME_KT_SEARCH, None, None, C.byref(cnt)) == me.ME_EINVAL


def test_batch_argument_validation():
    L = me.lib()
    p = me.me_default_params()
    h = C.c_void_p(1)
    ja = (me.me_job * 1)(job())
    assert L.me_batch_create(ja, 1, C.byref(p), 0, None, None) == me.ME_EINVAL          # no handle out
    assert L.me_batch_create(ja, 0, C.byref(p), 0, None, C.byref(h)) == me.ME_EINVAL    # empty
    assert h.value is None                                                              # cleared on error
    assert L.me_batch_create(ja, 1, C.byref(p), 8, None, C.byref(h)) == me.ME_EINVAL    # unknown flag
    assert L.me_batch_create(ja, 1, None, 0, None, C.byref(h)) == me.ME_EINVAL          # no params
    bad = (me.me_job * 1)(job(mv=None))
    assert L.me_batch_create(bad, 1, C.byref(p), 0, None, C.byref(h)) == me.ME_EINVAL
    noalpha = (me.me_job * 1)(job())
    assert L.me_batch_create(noalpha, 1, C.byref(p), me.ME_BATCH_SHAPE, None, C.byref(h)) == me.ME_EINVAL
    assert L.me_batch_step(None, ja, 1) == me.ME_EINVAL
    s, n_, d = (C.c_uint64 * 1)(), (C.c_uint64 * 1)(), (C.c_double * 1)()
    assert L.me_batch_results(None, s, n_, d, 1) == me.ME_EINVAL
    cfg = (C.c_int32 * 4)()
    assert L.me_batch_config(None, cfg, 4) == me.ME_EINVAL
    L.me_batch_destroy(None)


def test_net_argument_validation():
    L = me.lib()
    h = C.c_void_p(1)
    w = (C.c_float * me.ME_NET_PARAMS)()
    assert L.me_net_create(w, 2, None) == me.ME_EINVAL
    assert L.me_net_create(None, 2, C.byref(h)) == me.ME_EINVAL and h.value is None
    assert L.me_net_create(w, 3, C.byref(h)) == me.ME_EINVAL and h.value is None   # scale 2 or 4 only
    w[5] = float("nan")
    assert L.me_net_create(w, 2, C.byref(h)) == me.ME_EINVAL
    ja = (me.me_job * 1)(job())
    assert L.me_net_forward(None, ja, 1, None, None) == me.ME_EINVAL
    labels = (C.c_void_p * 1)(FAKE)
    assert L.me_net_train_step(None, ja, 1, labels, 0.1, 0.9, None, None, None) == me.ME_EINVAL
    assert L.me_net_backward(None, ja, 1, labels, FAKE, None, None) == me.ME_EINVAL
    assert L.me_net_sgd_step(None, FAKE, 0.1, 0.9, None) == me.ME_EINVAL
    s = (C.c_float * me.ME_NET_PARAMS)()
    assert L.me_net_weights(None, s, None) == me.ME_EINVAL
    assert L.me_net_scale(None) == me.ME_EINVAL
    assert L.me_net_save(None, b"/tmp/x") == me.ME_EINVAL
    assert L.me_net_load(b"/tmp/x", None) == me.ME_EINVAL
    L.me_net_destroy(None)


def test_net_checkpoint_errors_before_any_device_call(tmp_path):
    # file checks run on the host before a network is created
    L = me.lib()
    h = C.c_void_p(1)
    assert L.me_net_load(str(tmp_path / "missing.menet").encode(), C.byref(h)) == me.ME_EIO and h.value is None
    bad = tmp_path / "short.menet"
    bad.write_bytes(b"ME-NET\0\0" + b"\0" * 100)
    assert L.me_net_load(str(bad).encode(), C.byref(h)) == me.ME_EFORMAT and h.value is None
    n = 24 + 8 * me.ME_NET_PARAMS + 8
    wrong = tmp_path / "magic.menet"
    wrong.write_bytes(b"X" * n)
    assert L.me_net_load(str(wrong).encode(), C.byref(h)) == me.ME_EFORMAT
    assert "checkpoint" in me.status_str(me.ME_EFORMAT) and "file" in me.status_str(me.ME_EIO)


def test_pad_argument_validation():
    """me_pad_vops rejects bad frames, outputs and counts before any device call."""
    ok = frame(alpha=FAKE + 4096)
    out = FAKE + 8192
    assert me.me_pad_vops([], [], check=False) == me.ME_OK
    assert me.me_pad_vops([frame()], [out], check=False) == me.ME_EINVAL          # no alpha
    assert me.me_pad_vops([ok], [None], check=False) == me.ME_EINVAL              # no output
    assert me.me_pad_vops([ok], [FAKE], check=False) == me.ME_EINVAL              # output is the luma
    assert me.me_pad_vops([ok], [out + 1], check=False) == me.ME_EALIGN           # unaligned output
    assert me.me_pad_vops([frame(w=40, alpha=FAKE)], [out], check=False) == me.ME_EALIGN
    assert me.me_pad_vops([frame(stride=66, alpha=FAKE)], [out], check=False) == me.ME_EALIGN
    assert me.lib().me_pad_vops(None, 1, None, None) == me.ME_EINVAL
    assert me.lib().me_pad_vops(None, -1, None, None) == me.ME_EINVAL
