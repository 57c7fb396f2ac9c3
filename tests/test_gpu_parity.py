"""GPU parity: every entry point of the C ABI against the CPU oracle on the
same seeded inputs, bit-exact (classes, BAB words, vectors, costs, iteration
and point counts, SSE, pixel counts; PSNR within 1e-6 dB)."""
import math

import numpy as np
import pytest

import oracle
import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth

from gpu_util import assert_same, gpu_classify, gpu_pa, oracle_pa, oracle_params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    me.lib()
    return torch


def dseq(seq):
    from paper_1002_1168_amd.device import DeviceSequence
    return DeviceSequence(seq)


# ------------------------------------------------------------ classification
@pytest.mark.parametrize("maker", ["qcif", "cif", "random"])
def test_classify_parity(torch_cuda, maker):
    say("classify", maker)
    seq = {"qcif": lambda: synth.qcif_ellipse(frames=4), "cif": lambda: synth.cif_two_vops(frames=4),
           "random": lambda: synth.random_frames(5, 96, 64, frames=3, vops=2)}[maker]()
    if maker == "random":   # non-binary alpha: inside <=> != 0
        rng = np.random.default_rng(1)
        nz = seq.alpha != 0
        seq.alpha[nz] = rng.integers(1, 256, size=int(nz.sum()))
    ds = dseq(seq)
    gpu_classify(ds)
    cls = ds.cls.cpu().numpy()
    bab = ds.bab.cpu().numpy().view(np.uint32)
    for v in range(seq.vops):
        for t in range(seq.frames):
            c, b = oracle.classify(seq.alpha[v, t])
            np.testing.assert_array_equal(cls[v, t], c)
            np.testing.assert_array_equal(bab[v, t].reshape(c.shape + (8,)), b)


# ----------------------------------------------------------- proposed method
def check_pa(seq, vops, params, pairs, shape_only=False, one_call=True, chained=True, label="", distance=1):
    say("pa", label, seq.name, seq.width, seq.height, "vops", vops, "pairs", pairs, "shape_only", shape_only)
    ds = dseq(seq)
    gpu_classify(ds)
    got = gpu_pa(ds, vops, params, pairs, shape_only, one_call, chained, distance=distance)
    for v in vops:
        want = oracle_pa(seq, v, params, pairs, shape_only, distance=distance)
        assert_same(got[v], want, f"{label} vop {v}")
    return got


def test_pa_qcif_ellipse_full(torch_cuda):
    seq = synth.qcif_ellipse()
    check_pa(seq, [0], me.me_default_params(search_range=7), seq.frames - 1, label="qcif")


def test_pa_qcif_rectangular(torch_cuda):
    seq = synth.qcif_ellipse()
    check_pa(seq, [None], me.me_default_params(search_range=7), seq.frames - 1, label="qcif-rect")


def test_pa_shape_only(torch_cuda):
    seq = synth.cif_two_vops(frames=8)
    check_pa(seq, [0, 1], me.me_default_params(search_range=16), 7, shape_only=True, label="shape")


def test_pa_cif_two_vops_chained_one_launch(torch_cuda):
    seq = synth.cif_two_vops(frames=25)
    check_pa(seq, [0, 1], me.me_default_params(search_range=16), 24, label="cif-chain")


def test_pa_one_call_per_pair_matches(torch_cuda):
    seq = synth.cif_two_vops(frames=6)
    check_pa(seq, [0, 1], me.me_default_params(search_range=16), 5, one_call=False, label="cif-per-pair")


# one call per pair: no chain inside a call, so the row workers run (the line
# workers when forced), T read from the previous call's output
@pytest.mark.parametrize("flags", [0, me.ME_FLAG_LINE_WORKERS])
@pytest.mark.parametrize("case", ["qcif", "qcif-rect", "shape", "hd-halfpel", "cif-halfpel", "qcif-halfpel",
                                  "noise-halfpel", "w4096", "noise", "tiny"])
def test_pa_per_pair_rows_and_lines(torch_cuda, case, flags):
    # the half-pel cases run the row workers with two windows each (each MB's
    # half-sample step one MB late) at S = 32, 16 and 7
    if case == "qcif":
        seq, vops, p, P, so = synth.qcif_ellipse(), [0], dict(search_range=7), 5, False
    elif case == "cif-halfpel":
        seq, vops, p, P, so = synth.cif_two_vops(frames=5), [0, 1, None], dict(search_range=16, half_pel=1), 4, False
    elif case == "qcif-halfpel":
        seq, vops, p, P, so = synth.qcif_ellipse(frames=6), [0, None], dict(search_range=7, half_pel=1), 5, False
    elif case == "noise-halfpel":
        seq, vops, p, P, so = synth.random_frames(8, 96, 64, frames=4, vops=1, search_range=7), [0, None], \
            dict(search_range=7, half_pel=1, k_max=255), 3, False
    elif case == "qcif-rect":
        seq, vops, p, P, so = synth.qcif_ellipse(), [None], dict(search_range=7, k_max=255, max_step=3), 4, False
    elif case == "shape":
        seq, vops, p, P, so = synth.cif_two_vops(frames=5), [0, 1], dict(search_range=16), 4, True
    elif case == "hd-halfpel":
        seq, vops, p, P, so = synth.hd_streams(frames=3, streams=1)[0], [0, 1, 2], dict(search_range=32, half_pel=1), \
            2, False
    elif case == "w4096":
        seq, vops, p, P, so = synth.random_frames(6, 4096, 48, frames=3, vops=1, search_range=16), [0, None], \
            dict(search_range=16), 2, False
    elif case == "noise":
        seq, vops, p, P, so = synth.random_frames(3, 48, 32, frames=5, vops=1, search_range=4), [0, None], \
            dict(search_range=4, k_max=255), 4, False
    else:
        seq, vops, p, P, so = synth.random_frames(4, 16, 16, frames=3, vops=1, search_range=2), [0, None], \
            dict(search_range=2), 2, False
    check_pa(seq, vops, me.me_default_params(flags=flags, **p), P, shape_only=so, one_call=False,
             label=f"per-pair {case} flags {flags}")


# unrestricted vectors (reference padding, Section 4 protocol): the chained
# launch (line workers), one call per pair (row workers, and line workers
# forced), shape-only, half-pel at S=32
@pytest.mark.parametrize("mode", ["chained", "rows", "lines", "shape", "hd-halfpel"])
def test_pa_unrestricted(torch_cuda, mode):
    U = me.ME_FLAG_UNRESTRICTED
    if mode == "hd-halfpel":
        seq = synth.hd_streams(frames=3, streams=1)[0]
        check_pa(seq, [0, 1], me.me_default_params(search_range=32, half_pel=1, flags=U), 2, one_call=False,
                 label="unrestricted hd")
        return
    seq = synth.qcif_ellipse(frames=6)
    p = me.me_default_params(search_range=7, flags=U | (me.ME_FLAG_LINE_WORKERS if mode == "lines" else 0))
    if mode == "shape":
        check_pa(synth.cif_two_vops(frames=4), [0, 1], me.me_default_params(search_range=16, flags=U), 3,
                 shape_only=True, label="unrestricted shape")
    else:
        check_pa(seq, [0, None], p, 5, one_call=mode == "chained", label=f"unrestricted {mode}")


# the Section 3.1 text reading (a boundary MB's T scored on texture): the
# chained launch (one-wave line workers), one call per pair (row workers, and
# line workers forced), with unrestricted vectors, half-pel at S=32
@pytest.mark.parametrize("mode", ["chained", "rows", "lines", "unrestricted", "hd-halfpel"])
def test_pa_t_on_texture(torch_cuda, mode):
    T = me.ME_FLAG_T_TEXTURE
    if mode == "hd-halfpel":
        seq = synth.hd_streams(frames=3, streams=1)[0]
        check_pa(seq, [0, 1, 2], me.me_default_params(search_range=32, half_pel=1, flags=T), 2, one_call=False,
                 label="t-texture hd")
        return
    seq = synth.cif_two_vops(frames=6)
    flags = T | (me.ME_FLAG_LINE_WORKERS if mode == "lines" else 0) | \
        (me.ME_FLAG_UNRESTRICTED if mode == "unrestricted" else 0)
    check_pa(seq, [0, 1], me.me_default_params(search_range=16, flags=flags), 5, one_call=mode == "chained",
             label=f"t-texture {mode}")


# the masked-luma reading of a boundary MB's recursion, alone and with T on
# texture: the chained launch (one-wave line workers), one call per pair (row
# workers, and line workers forced), unrestricted vectors, half-pel at S=32
@pytest.mark.parametrize("mode", ["chained", "rows", "lines", "unrestricted", "with-t-texture", "hd-halfpel"])
def test_pa_masked_prs(torch_cuda, mode):
    M = me.ME_FLAG_MASKED_PRS
    if mode == "hd-halfpel":
        seq = synth.hd_streams(frames=3, streams=1)[0]
        check_pa(seq, [0, 1, 2], me.me_default_params(search_range=32, half_pel=1, flags=M), 2, one_call=False,
                 label="masked prs hd")
        return
    seq = synth.cif_two_vops(frames=6)
    flags = M | (me.ME_FLAG_LINE_WORKERS if mode == "lines" else 0) | \
        (me.ME_FLAG_UNRESTRICTED if mode == "unrestricted" else 0) | \
        (me.ME_FLAG_T_TEXTURE if mode == "with-t-texture" else 0)
    check_pa(seq, [0, 1], me.me_default_params(search_range=16, flags=flags), 5, one_call=mode == "chained",
             label=f"masked prs {mode}")


# the Section 4 protocol: reference frame two back, T from the previous pair
@pytest.mark.parametrize("one_call", [True, False])
@pytest.mark.parametrize("flags", [0, me.ME_FLAG_UNRESTRICTED])
def test_pa_frame_distance_two(torch_cuda, one_call, flags):
    seq = synth.qcif_ellipse(frames=8)
    check_pa(seq, [0, None], me.me_default_params(search_range=7, flags=flags), 6, one_call=one_call,
             label=f"distance 2 flags {flags}", distance=2)


@pytest.mark.parametrize("method", [me.ME_ES, me.ME_TSS, me.ME_DS, me.ME_4SS])
def test_search_unrestricted(torch_cuda, method):
    import torch
    from paper_1002_1168_amd import device as dv
    for seq, S, vop in ((synth.qcif_ellipse(frames=3), 7, None), (synth.cif_two_vops(frames=3), 16, 0)):
        say("search unrestricted", method, seq.name, S)
        ds = dseq(seq)
        if vop is not None:
            gpu_classify(ds)
        out = dv.Outputs.alloc(2, ds.hm, ds.wm)
        p = me.me_default_params(search_range=S, flags=me.ME_FLAG_UNRESTRICTED)
        me.me_full_search(method, ds.pair_jobs(vop, out, 2, chained=False), p, stream=dv.stream_handle())
        torch.cuda.synchronize()
        assert me.me_device_status(dv.stream_handle()) == me.ME_OK
        got = out.host()
        for i in range(2):
            t = i + 1
            cls = oracle.classify(seq.alpha[vop, t])[0] if vop is not None else None
            want = oracle.search(method, seq.luma[t], seq.luma[t - 1], oracle_params(p), cls)
            assert_same({k: got[k][i] for k in got}, want, f"unrestricted method {method} pair {i}",
                        keys=("mv", "mv_int", "cost", "points"))


def test_pa_rows_bad_class_raises_status(torch_cuda):
    """The row workers (a single unchained job): a class byte outside 0..2
    raises the status word, that MB gets the transparent result."""
    import torch
    from paper_1002_1168_amd import device as dv
    seq = synth.qcif_ellipse(frames=3)
    ds = dseq(seq)
    gpu_classify(ds)
    cls = ds.cls[0, 1]
    opaque = (cls == me.ME_MB_OPAQUE).nonzero()
    v, h = (int(x) for x in opaque[len(opaque) // 2])
    cls[v, h] = 9
    out = dv.Outputs.alloc(1, ds.hm, ds.wm)
    s = dv.stream_handle()
    me.me_texture_recursive(ds.pair_jobs(0, out, 1), me.me_default_params(search_range=7), None, stream=s)
    torch.cuda.synchronize()
    assert me.me_device_status(s) == me.ME_EDEVICE
    assert me.me_device_status(s) == me.ME_OK
    got = out.host()
    assert (got["mv"][0][v, h] == 0).all() and got["points"][0][v, h] == 0
    assert (got["points"][0][cls.cpu().numpy() == me.ME_MB_OPAQUE] > 0).all()


@pytest.mark.parametrize("over", [dict(eps_q12=2048), dict(max_step=3), dict(theta=2), dict(k_max=0),
                                  dict(k_max=1), dict(k_max=255, max_step=7), dict(eps_q12=65536, theta=1)])
def test_pa_parameter_variants(torch_cuda, over):
    seq = synth.qcif_ellipse()
    check_pa(seq, [0, None], me.me_default_params(search_range=7, **over), seq.frames - 1, label=str(over))


def test_pa_half_pel_hd(torch_cuda):
    seq = synth.hd_streams(frames=3, streams=1)[0]
    check_pa(seq, [0, 1, 2], me.me_default_params(search_range=32, half_pel=1), 2, label="hd-halfpel")


def test_pa_random_noise_small_frames(torch_cuda):
    # unstructured texture: long recursions, many infeasible candidates
    seq = synth.random_frames(3, 48, 32, frames=5, vops=1, search_range=4)
    check_pa(seq, [0, None], me.me_default_params(search_range=4, k_max=255), 4, label="noise")


def test_pa_single_mb_and_empty_masks(torch_cuda):
    seq = synth.random_frames(4, 16, 16, frames=3, vops=1, search_range=2)
    seq.alpha[:] = 0
    check_pa(seq, [0, None], me.me_default_params(search_range=2), 2, label="single-mb")


def test_pa_bad_class_raises_status(torch_cuda):
    """A class byte outside 0..2 sets the device status word (ME_EDEVICE on
    the next status read, which clears it); that MB is given the transparent
    result and the other MBs of the pair are still solved."""
    import torch
    from paper_1002_1168_amd import device as dv
    seq = synth.qcif_ellipse(frames=3)
    say("pa bad class", seq.name)
    ds = dseq(seq)
    gpu_classify(ds)
    cls = ds.cls[0, 1]
    opaque = (cls == me.ME_MB_OPAQUE).nonzero()
    v, h = (int(x) for x in opaque[len(opaque) // 2])
    cls[v, h] = 7
    out = dv.Outputs.alloc(2, ds.hm, ds.wm)
    s = dv.stream_handle()
    me.me_texture_recursive(ds.pair_jobs(0, out, 2), me.me_default_params(search_range=7), None, stream=s)
    torch.cuda.synchronize()
    assert me.me_device_status(s) == me.ME_EDEVICE
    assert me.me_device_status(s) == me.ME_OK
    got = out.host()
    assert (got["mv"][0][v, h] == 0).all() and (got["mv_int"][0][v, h] == 0).all()
    assert got["cost"][0][v, h] == 0 and got["iters"][0][v, h] == 0 and got["points"][0][v, h] == 0
    assert (got["points"][0][cls.cpu().numpy() == me.ME_MB_OPAQUE] > 0).all()


def test_pa_max_width(torch_cuda):
    seq = synth.random_frames(6, 4096, 32, frames=3, vops=0, search_range=16)
    check_pa(seq, [None], me.me_default_params(search_range=16), 2, label="w4096")


def test_pa_mixed_sizes_one_launch(torch_cuda):
    import torch
    from paper_1002_1168_amd import device as dv
    streams = synth.mixed_streams(frames=4, counts=(2, 2, 1))
    p = me.me_default_params(search_range=16)
    say("pa mixed streams", [s.name for s in streams])
    jobs, keep = [], []
    for s in streams:
        ds = dseq(s)
        gpu_classify(ds)
        for v in range(s.vops):
            out = dv.Outputs.alloc(3, ds.hm, ds.wm)
            jobs += ds.pair_jobs(v, out, 3)
            keep.append((s, v, out, ds))
    me.me_texture_recursive(jobs, p, None, stream=dv.stream_handle())
    torch.cuda.synchronize()
    assert me.me_device_status(dv.stream_handle()) == me.ME_OK
    for s, v, out, _ in keep:
        assert_same(out.host(), oracle_pa(s, v, p, 3), f"{s.name} vop {v}")


# -------------------------------------------------------------- baselines
def check_search(seq, method, S, pairs, vop=0):
    import torch
    from paper_1002_1168_amd import device as dv
    say("search", method, seq.name, seq.width, seq.height, "S", S, "pairs", pairs)
    ds = dseq(seq)
    if vop is not None:
        gpu_classify(ds)
    out = dv.Outputs.alloc(pairs, ds.hm, ds.wm)
    p = me.me_default_params(search_range=S)
    jobs = ds.pair_jobs(vop, out, pairs, chained=False)
    me.me_full_search(method, jobs, p, stream=dv.stream_handle())
    torch.cuda.synchronize()
    assert me.me_device_status(dv.stream_handle()) == me.ME_OK
    got = out.host()
    for i in range(pairs):
        t = i + 1
        cls = oracle.classify(seq.alpha[vop, t])[0] if vop is not None else None
        want = oracle.search(method, seq.luma[t], seq.luma[t - 1], oracle_params(p), cls)
        assert_same({k: got[k][i] for k in got}, want, f"method {method} pair {i}",
                    keys=("mv", "mv_int", "cost", "points"))
        assert (got["iters"][i] == 0).all()


@pytest.mark.parametrize("method", [me.ME_ES, me.ME_TSS, me.ME_DS, me.ME_4SS])
def test_search_qcif(torch_cuda, method):
    seq = synth.qcif_ellipse()
    check_search(seq, method, 7, seq.frames - 1)
    check_search(seq, method, 7, 3, vop=None)


@pytest.mark.parametrize("method", [me.ME_ES, me.ME_TSS, me.ME_DS, me.ME_4SS])
def test_search_cif(torch_cuda, method):
    check_search(synth.cif_two_vops(frames=4), method, 16, 3, vop=None)


@pytest.mark.parametrize("method", [me.ME_ES, me.ME_TSS, me.ME_DS, me.ME_4SS])
@pytest.mark.parametrize("S", [1, 4, 13])
def test_search_random_tiny(torch_cuda, method, S):
    check_search(synth.random_frames(8, 64, 48, frames=3, vops=1), method, S, 2)


@pytest.mark.parametrize("method", [me.ME_ES, me.ME_TSS, me.ME_DS, me.ME_4SS])
def test_search_s32_crop(torch_cuda, method):
    seq = synth.hd_streams(frames=2, streams=1)[0]
    seq.luma = np.ascontiguousarray(seq.luma[:, 256:512, 640:960])
    seq.alpha = np.ascontiguousarray(seq.alpha[:, :, 256:512, 640:960])
    check_search(seq, method, 32, 1, vop=None)


# ------------------------------------------------------- MC, SSE, PSNR
@pytest.mark.parametrize("half", [0, 1])
def test_mc_psnr_parity(torch_cuda, half):
    import torch
    from paper_1002_1168_amd import device as dv
    seq = synth.hd_streams(frames=3, streams=1)[0] if half else synth.cif_two_vops(frames=5)
    S = 32 if half else 16
    vops = list(range(seq.vops))
    p = me.me_default_params(search_range=S, half_pel=half)
    say("mc", seq.name, "half", half)
    ds = dseq(seq)
    gpu_classify(ds)
    pairs = seq.frames - 1
    got = gpu_pa(ds, vops, p, pairs)
    for v in vops + [None]:
        if v is None:  # rectangular prediction with the VOP's vectors
            out = got[0]
        else:
            out = got[v]
        mvt = torch.from_numpy(out["mv"]).cuda()
        jobs = []
        for i in range(pairs):
            t = i + 1
            ca = None if v is None else ds.alpha[v, t]
            cls = None if v is None else ds.cls[v, t]
            jobs.append(dv.mc_job(ds.luma[t], ds.luma[t - 1], ca, cls, mvt[i]))
        preds = [torch.zeros((seq.height, seq.width), dtype=torch.uint8, device="cuda") for _ in range(pairs)]
        sse, npx, ps, rc = me.me_motion_compensate_psnr(jobs, [x.data_ptr() for x in preds],
                                                        stream=dv.stream_handle())
        assert rc == me.ME_OK
        # without prediction frames (transparent MBs skipped by class): the same sums
        sse2, npx2, ps2, rc2 = me.me_motion_compensate_psnr(jobs, stream=dv.stream_handle())
        assert rc2 == me.ME_OK and list(sse2) == list(sse) and list(npx2) == list(npx)
        for i in range(pairs):
            t = i + 1
            ca = None if v is None else seq.alpha[v, t]
            cls = None if v is None else oracle.classify(ca)[0]
            ws, wn, wp = oracle.mc_sse(seq.luma[t], seq.luma[t - 1], out["mv"][i], ca, cls, want_pred=True)
            assert (sse[i], npx[i]) == (ws, wn)
            want_db = oracle.psnr_db(ws, wn)
            assert (ps[i] == want_db) or abs(ps[i] - want_db) < 1e-6
            np.testing.assert_array_equal(preds[i].cpu().numpy(), wp)


def test_classify_mc_five_thousand_one_mb_jobs(torch_cuda):
    """5,000 one-MB frames (16x16 windows of one wide plane): finding a
    unit's job takes three 64-way rounds, and every unit spans 8 or 16 jobs."""
    import torch
    from paper_1002_1168_amd import device as dv
    rng = np.random.default_rng(7)
    n = 5000
    say("classify+mc 5000 one-MB jobs")
    W = 16 * n
    cur = rng.integers(0, 256, size=(16, W), dtype=np.uint8)
    ref = rng.integers(0, 256, size=(16, W), dtype=np.uint8)
    alpha = (rng.random((16, W)) < 0.6).astype(np.uint8) * 255
    alpha[:, 16 * np.arange(0, n, 5)[:, None] + np.arange(16)] = 0      # some transparent MBs
    alpha[:, 16 * np.arange(1, n, 5)[:, None] + np.arange(16)] = 255    # some opaque MBs
    mv = rng.integers(-6, 7, size=(n, 1, 1, 2)).astype(np.int16)
    tc, tr, ta = (torch.from_numpy(x).cuda() for x in (cur, ref, alpha))
    tmv = torch.from_numpy(mv).cuda()
    cls = torch.full((n, 1, 1), 9, dtype=torch.uint8, device="cuda")
    bab = torch.zeros((n, 8), dtype=torch.int32, device="cuda")
    pred = torch.zeros((16, W), dtype=torch.uint8, device="cuda")
    win = lambda t, i: t[:, 16 * i:16 * i + 16]
    s = dv.stream_handle()
    me.me_classify_babs([dv.frame(win(tc, i), win(ta, i)) for i in range(n)], [cls[i].data_ptr() for i in range(n)],
                        [bab[i].data_ptr() for i in range(n)], stream=s)
    jobs = [dv.mc_job(win(tc, i), win(tr, i), win(ta, i), cls[i], tmv[i]) for i in range(n)]
    sse, npx, ps, rc = me.me_motion_compensate_psnr(jobs, [win(pred, i).data_ptr() for i in range(n)], stream=s,
                                                    check=False)
    torch.cuda.synchronize()
    assert rc == me.ME_EEMPTY
    # the sums alone: units of 64 one-MB jobs, transparent ones skipped by class
    sse2, npx2, _, rc2 = me.me_motion_compensate_psnr(jobs, stream=s, check=False)
    assert rc2 == me.ME_EEMPTY and list(sse2) == list(sse) and list(npx2) == list(npx)
    gc, gb, gp = cls.cpu().numpy(), bab.cpu().numpy().view(np.uint32), pred.cpu().numpy()
    for i in range(n):
        sl = slice(16 * i, 16 * i + 16)
        c, b = oracle.classify(np.ascontiguousarray(alpha[:, sl]))
        assert gc[i, 0, 0] == c[0, 0] and (gb[i] == b[0, 0]).all(), f"job {i}"
        ws, wn, wp = oracle.mc_sse(np.ascontiguousarray(cur[:, sl]), np.ascontiguousarray(ref[:, sl]), mv[i],
                                   np.ascontiguousarray(alpha[:, sl]), c, want_pred=True)
        assert (sse[i], npx[i]) == (ws, wn), f"job {i}"
        np.testing.assert_array_equal(gp[:, sl], wp, err_msg=f"job {i}")


def test_mc_empty_mask_reports_eempty(torch_cuda):
    import torch
    from paper_1002_1168_amd import device as dv
    seq = synth.random_frames(2, 32, 32, frames=2, vops=1)
    seq.alpha[:] = 0
    ds = dseq(seq)
    mv = torch.zeros((2, 2, 2), dtype=torch.int16, device="cuda")
    jobs = [dv.mc_job(ds.luma[1], ds.luma[0], ds.alpha[0, 1], None, mv)]
    sse, npx, ps, rc = me.me_motion_compensate_psnr(jobs, stream=dv.stream_handle(), check=False)
    assert rc == me.ME_EEMPTY and npx[0] == 0 and math.isnan(ps[0])


@pytest.mark.parametrize("seed", [0, 1])
def test_classify_mc_many_small_jobs(torch_cuda, seed):
    """150 frames of 1 to 12 MBs each, padded strides, in one call each of
    classification and MC: the kernels' units of 16 and 8 consecutive MBs
    straddle many jobs, and finding a unit's job takes two 64-way rounds."""
    import torch
    from paper_1002_1168_amd import device as dv
    rng = np.random.default_rng(seed)
    say("classify+mc many small jobs, seed", seed)
    n = 150
    host, dev = [], []
    for i in range(n):
        W, H = 16 * int(rng.integers(1, 5)), 16 * int(rng.integers(1, 4))
        st = W + 4 * int(rng.integers(0, 5))
        cur = rng.integers(0, 256, size=(H, st), dtype=np.uint8)
        ref = rng.integers(0, 256, size=(H, st), dtype=np.uint8)
        kind = i % 3   # all inside, all outside, mixed
        alpha = np.full((H, st), 255 if kind == 0 else 0, np.uint8)
        if kind == 2:
            alpha = (rng.random((H, st)) < 0.5).astype(np.uint8) * rng.integers(1, 256, size=(H, st), dtype=np.uint8)
        mv = rng.integers(-9, 10, size=(H // 16, W // 16, 2)).astype(np.int16)
        host.append((cur[:, :W], ref[:, :W], alpha[:, :W], mv))
        t = [torch.from_numpy(x).cuda() for x in (cur, ref, alpha)]
        d = dict(cur=t[0][:, :W], ref=t[1][:, :W], alpha=t[2][:, :W], mv=torch.from_numpy(mv).cuda(),
                 cls=torch.full((H // 16, W // 16), 7, dtype=torch.uint8, device="cuda"),
                 bab=torch.zeros((H // 16, W // 16, 8), dtype=torch.int32, device="cuda"),
                 pred=torch.zeros((H, st), dtype=torch.uint8, device="cuda"))
        assert d["cur"].stride(0) == st
        dev.append(d)
    s = dv.stream_handle()
    me.me_classify_babs([dv.frame(d["cur"], d["alpha"]) for d in dev], [d["cls"].data_ptr() for d in dev],
                        [d["bab"].data_ptr() for d in dev], stream=s)
    jobs = [dv.mc_job(d["cur"], d["ref"], d["alpha"], d["cls"], d["mv"]) for d in dev]
    sse, npx, ps, rc = me.me_motion_compensate_psnr(jobs, [d["pred"].data_ptr() for d in dev], stream=s,
                                                    check=False)
    torch.cuda.synchronize()
    for i, ((cur, ref, alpha, mv), d) in enumerate(zip(host, dev)):
        c, b = oracle.classify(alpha)
        np.testing.assert_array_equal(d["cls"].cpu().numpy(), c, err_msg=f"job {i}")
        np.testing.assert_array_equal(d["bab"].cpu().numpy().view(np.uint32), b, err_msg=f"job {i}")
        ws, wn, wp = oracle.mc_sse(cur, ref, mv, alpha, c, want_pred=True)
        assert (sse[i], npx[i]) == (ws, wn), f"job {i}"
        np.testing.assert_array_equal(d["pred"].cpu().numpy()[:, :cur.shape[1]], wp, err_msg=f"job {i}")
    # every third job has no pixel inside: the call reports it
    assert rc == me.ME_EEMPTY
    # the queued form leaves the same sums in device memory (no ME_EEMPTY)
    sums = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
    assert me.me_motion_compensate_sse(jobs, sums.data_ptr(), stream=s) == me.ME_OK
    torch.cuda.synchronize()
    got = sums.cpu().numpy().view(np.uint64)
    assert [int(x) for x in got[0::2]] == list(sse) and [int(x) for x in got[1::2]] == list(npx)
    # ... or in pinned host memory, readable once the stream has passed it
    hsums = torch.full((2 * n,), -1, dtype=torch.int64, pin_memory=True)
    assert me.me_motion_compensate_sse(jobs, hsums.data_ptr(), stream=s) == me.ME_OK
    torch.cuda.synchronize()
    got = hsums.numpy().view(np.uint64)
    assert [int(x) for x in got[0::2]] == list(sse) and [int(x) for x in got[1::2]] == list(npx)


# ------------------------------------------- full size, repeated launches
def test_pa_full_bench_workload(torch_cuda):
    """The benchmark's workload and launch (CIF, 300 frames, two VOPs, all
    598 pairs in one pipelined call), every output against the oracle."""
    seq = synth.cif_two_vops(seed=2, frames=300)
    check_pa(seq, [0, 1], me.me_default_params(search_range=16), 299, label="bench-full")


def test_pa_repeat_launches_identical(torch_cuda):
    """Schedule perturbation: the worker interleaving differs run to run; the
    result must not."""
    seq = synth.mixed_streams(seed=11, frames=40, counts=(1, 1, 1))[2]
    p = me.me_default_params(search_range=16)
    ds = dseq(seq)
    gpu_classify(ds)
    want = {v: oracle_pa(seq, v, p, 39) for v in range(seq.vops)}
    for rep in range(4):
        say("repeat", rep, seq.name)
        got = gpu_pa(ds, list(range(seq.vops)), p, 39)
        for v in range(seq.vops):
            assert_same(got[v], want[v], f"rep {rep} vop {v}")


def test_kernel_timing_counts_each_launch(torch_cuda):
    """The library's kernel events: one duration per timed call, positive,
    and the timed results still equal the oracle's."""
    seq = synth.qcif_ellipse(seed=1, frames=4)
    p = me.me_default_params(search_range=7)
    ds = dseq(seq)
    gpu_classify(ds)
    from paper_1002_1168_amd.device import stream_handle
    s = stream_handle()
    me.me_kernel_timing(True)
    try:
        me.me_kernel_time_ms(me.ME_KT_SEARCH, s)
        got = None
        for _ in range(3):
            got = gpu_pa(ds, [0], p, 3)
        total, count = me.me_kernel_time_ms(me.ME_KT_SEARCH, s)
    finally:
        me.me_kernel_timing(False)
    assert count == 3 and total > 0.0
    assert_same(got[0], oracle_pa(seq, 0, p, 3), "timed")
    assert me.me_kernel_time_ms(me.ME_KT_SEARCH, s) == (0.0, 0)


def test_kernel_timing_selected_kinds_only(torch_cuda):
    """With ME_KT_ONLY bits only the selected call kinds record events."""
    seq = synth.qcif_ellipse(seed=1, frames=3)
    p = me.me_default_params(search_range=7)
    ds = dseq(seq)
    from paper_1002_1168_amd.device import stream_handle
    s = stream_handle()
    me.me_kernel_timing(True, kinds=[me.ME_KT_SEARCH])
    try:
        for k in (me.ME_KT_CLASSIFY, me.ME_KT_SEARCH):
            me.me_kernel_time_ms(k, s)
        gpu_classify(ds)
        gpu_pa(ds, [0], p, 2)
        cls_total, cls_count = me.me_kernel_time_ms(me.ME_KT_CLASSIFY, s)
        total, count = me.me_kernel_time_ms(me.ME_KT_SEARCH, s)
    finally:
        me.me_kernel_timing(False)
    assert (cls_total, cls_count) == (0.0, 0)
    assert count == 1 and total > 0.0


@pytest.mark.parametrize("maker,S", [("qcif", 7), ("cif", 16)])
def test_pa_seeded_start_parity(torch_cuda, maker, S):
    """Learned-seed start with the 5 % fallback (seeds = random vectors,
    half of them near the plain result) against the oracle."""
    import torch
    from paper_1002_1168_amd.device import Outputs, stream_handle
    seq = synth.qcif_ellipse(seed=31, frames=6) if maker == "qcif" else synth.cif_two_vops(seed=32, frames=6)
    p = me.me_default_params(search_range=S)
    ds = dseq(seq)
    gpu_classify(ds)
    P = 5
    plain = oracle_pa(seq, 0, p, P)
    rng = np.random.default_rng(S)
    seeds = rng.integers(-S, S + 1, size=(P, ds.hm, ds.wm, 2)).astype(np.int16) * 2
    near = rng.random((P, ds.hm, ds.wm)) < 0.5
    jitter = rng.integers(-1, 2, size=(P, ds.hm, ds.wm, 2)).astype(np.int16) * 2
    seeds[near] = (plain["mv_int"] + jitter)[near]
    seeds = np.clip(seeds, -2 * S, 2 * S).astype(np.int16)
    want = oracle.pa_sequence(seq, 0, oracle_params(p), pairs=P, seeds=list(seeds))
    want = {k: np.stack([r[k] for r in want]) for k in ("mv", "mv_int", "cost", "iters", "points")}
    out = Outputs.alloc(P, ds.hm, ds.wm)
    sd = torch.from_numpy(seeds).cuda()
    me.me_texture_recursive(ds.pair_jobs(0, out, P, seeds=sd), p, None, stream=stream_handle())
    torch.cuda.synchronize()
    assert me.me_device_status(stream_handle()) == me.ME_OK
    assert_same(out.host(), want, f"seeded {maker}")


def test_pa_many_lines_one_wave_per_line(torch_cuda):
    """More lines than half the worker budget: the one-wave-per-line worker
    (the four-wave worker runs every case up to a quarter of it, the two-wave
    one the cases up to half), against the oracle."""
    import torch
    from paper_1002_1168_amd import device as dv
    streams = synth.mixed_streams(seed=33, frames=3, counts=(0, 0, 3))
    p = me.me_default_params(search_range=16)
    jobs, keep, alive, lines = [], [], [], 0
    for s in streams:
        ds = dseq(s)
        alive.append(ds)  # the jobs point into these device frames
        gpu_classify(ds)
        for v in range(s.vops):
            out = dv.Outputs.alloc(2, ds.hm, ds.wm)
            jobs += ds.pair_jobs(v, out, 2)
            keep.append((s, v, out))
            lines += ds.hm * ds.wm
    say("lines", lines)
    assert lines > 256 * 16 // 2
    me.me_texture_recursive(jobs, p, None, stream=dv.stream_handle())
    torch.cuda.synchronize()
    assert me.me_device_status(dv.stream_handle()) == me.ME_OK
    for s, v, out in keep:
        assert_same(out.host(), oracle_pa(s, v, p, 2), f"{s.name} vop {v}")


def test_pa_two_waves_per_line(torch_cuda):
    """Between a quarter and half the worker budget in lines (one 4CIF VOP
    layer: 1584 lines): the two-wave worker, against the oracle."""
    import torch
    from paper_1002_1168_amd import device as dv
    s = synth.mixed_streams(seed=34, frames=4, counts=(0, 0, 1))[0]
    p = me.me_default_params(search_range=16)
    ds = dseq(s)
    gpu_classify(ds)
    lines = ds.hm * ds.wm
    say("lines", lines)
    assert 256 * 16 // 4 < lines <= 256 * 16 // 2
    out = dv.Outputs.alloc(3, ds.hm, ds.wm)
    me.me_texture_recursive(ds.pair_jobs(0, out, 3), p, None, stream=dv.stream_handle())
    torch.cuda.synchronize()
    assert me.me_device_status(dv.stream_handle()) == me.ME_OK
    assert_same(out.host(), oracle_pa(s, 0, p, 3), f"{s.name} vop 0")


@pytest.mark.parametrize("method", [me.ME_ES, me.ME_TSS, me.ME_DS, me.ME_4SS])
@pytest.mark.parametrize("S", [20, 24, 26, 64])
def test_search_wide_ranges(torch_cuda, method, S):
    """Ranges that take the general ES kernel with G = 8, 5, 6 and 4 rows per
    task (S = 64: the largest range, a window of 147 rows of 256 bytes in
    four byte-shifted copies, 151 KB of LDS)."""
    check_search(synth.random_frames(9, 96, 80, frames=3, vops=1), method, S, 2)


@pytest.mark.parametrize("S", [20, 40, 64])
@pytest.mark.parametrize("mode", ["lines", "rows"])
def test_pa_wide_ranges(torch_cuda, S, mode):
    """The proposed search at ranges whose windows take the general staging
    loop (no per-range staging plan), up to S = 64: line workers (pairs
    chained in one call) and row workers (one call per pair), with and
    without half-sample refinement, VOP and rectangular."""
    seq = synth.random_frames(10 + S, 112, 96, frames=4, vops=1, search_range=S)
    for half in (0, 1):
        p = me.me_default_params(search_range=S, half_pel=half, k_max=255, max_step=min(S, 3))
        check_pa(seq, [0, None], p, 3, one_call=mode == "lines", label=f"S={S} half={half} {mode}")
