"""GPU parity of the MPEG-4 reference VOP padding (me_pad_vops; Section 4
protocol) against the oracle: every padded byte equal, bytes past each row's
width untouched, and searches over a padded reference equal to the oracle's
search over the oracle's padded reference."""
import numpy as np
import pytest

import oracle
import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth
from gpu_util import assert_same, oracle_params, say

pytestmark = pytest.mark.gpu

GUARD = 7  # byte value of the output buffer before the call


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    me.lib()
    return torch


def run_pad(planes):
    """planes: list of (luma (H, W) u8, alpha (H, W) u8, row stride).  Pads
    all of them in one call; returns the output buffers (H, stride)."""
    import torch
    from paper_1002_1168_amd import device as dv
    keep, frames, outs = [], [], []
    for lu, al, stride in planes:
        H, W = lu.shape
        L = torch.zeros((H, stride), dtype=torch.uint8, device="cuda")
        A = torch.zeros((H, stride), dtype=torch.uint8, device="cuda")
        L[:, :W] = torch.from_numpy(np.ascontiguousarray(lu))
        A[:, :W] = torch.from_numpy(np.ascontiguousarray(al))
        O = torch.full((H, stride), GUARD, dtype=torch.uint8, device="cuda")
        frames.append(me.me_frame(L.data_ptr(), A.data_ptr(), W, H, stride))
        outs.append(O.data_ptr())
        keep.append((L, A, O))
    me.me_pad_vops(frames, outs, stream=dv.stream_handle())
    torch.cuda.synchronize()
    assert me.me_device_status(dv.stream_handle()) == me.ME_OK
    return [o.cpu().numpy() for _, _, o in keep]


def check(planes, label):
    got = run_pad(planes)
    for i, ((lu, al, stride), g) in enumerate(zip(planes, got)):
        W = lu.shape[1]
        want = oracle.pad_vop(lu, al)
        bad = np.argwhere(g[:, :W] != want)
        assert bad.size == 0, f"{label} plane {i}: {len(bad)} samples differ, first at (y, x) {tuple(bad[0])}"
        assert (g[:, W:] == GUARD).all(), f"{label} plane {i}: bytes past the width were written"


def blob_alpha(rng, H, W, density):
    a = (rng.random((H, W)) < density).astype(np.uint8)
    # a few solid rectangles so that opaque and transparent MBs both occur
    for _ in range(3):
        y, x = rng.integers(0, H), rng.integers(0, W)
        a[y:y + rng.integers(8, 40), x:x + rng.integers(8, 40)] = rng.integers(0, 2) * 255
    return a


def test_pad_synthetic_vops(torch_cuda):
    seq = synth.cif_two_vops(frames=3)
    planes = [(seq.luma[t], seq.alpha[v, t], seq.luma.shape[2]) for v in range(seq.vops) for t in range(3)]
    say("pad cif", len(planes), "VOP planes")
    check(planes, "cif")


def test_pad_qcif_ellipse(torch_cuda):
    seq = synth.qcif_ellipse(frames=2)
    check([(seq.luma[t], seq.alpha[0, t], 176) for t in range(2)], "qcif")


@pytest.mark.parametrize("density", [0.01, 0.3, 0.7, 0.99])
def test_pad_random_shapes(torch_cuda, density):
    rng = np.random.default_rng(int(density * 1000) + 5)
    planes = []
    for H, W, extra in ((48, 64, 0), (80, 96, 12), (16, 16, 4), (16, 112, 0), (112, 16, 8)):
        lu = rng.integers(0, 256, (H, W), dtype=np.uint8)
        planes.append((lu, blob_alpha(rng, H, W, density), W + extra))
    say("pad random density", density)
    check(planes, f"density {density}")


def test_pad_degenerate(torch_cuda):
    rng = np.random.default_rng(11)
    lu = rng.integers(0, 256, (48, 48), dtype=np.uint8)
    one = np.zeros((16, 16), np.uint8)
    one[9, 4] = 1
    centre = np.zeros((48, 48), np.uint8)
    centre[16:32, 16:32] = 1
    planes = [
        (lu, np.zeros((48, 48), np.uint8), 48),        # all transparent: 128
        (lu, np.full((48, 48), 255, np.uint8), 52),    # all opaque: copy
        (lu[:16, :16], one, 16),                       # one inside pixel
        (lu, centre, 48),                              # corners without a padded neighbour
    ]
    check(planes, "degenerate")
    got = run_pad(planes[:2])
    assert (got[0][:, :48] == 128).all()
    assert np.array_equal(got[1][:, :48], lu)


def test_pad_many_vops_one_call(torch_cuda):
    rng = np.random.default_rng(12)
    planes = []
    for i in range(40):
        H, W = 16 * int(rng.integers(1, 6)), 16 * int(rng.integers(1, 8))
        lu = rng.integers(0, 256, (H, W), dtype=np.uint8)
        planes.append((lu, blob_alpha(rng, H, W, float(rng.random())), W + 4 * int(rng.integers(0, 3))))
    say("pad 40 planes")
    check(planes, "batch")


@pytest.mark.parametrize("method", [None, me.ME_ES, me.ME_DS])
def test_search_on_padded_reference(torch_cuda, method):
    """The proposed search (method None) and two baselines over a padded
    reference equal the oracle's over the oracle's padded reference."""
    import torch
    from paper_1002_1168_amd import device as dv
    seq = synth.cif_two_vops(frames=3)
    v, t = 0, 2
    cur, ref = seq.luma[t], seq.luma[t - 1]
    ca, ra = seq.alpha[v, t], seq.alpha[v, t - 1]
    want_ref = oracle.pad_vop(ref, ra)
    H, W = cur.shape
    padded = run_pad([(ref, ra, W)])[0]
    assert np.array_equal(padded, want_ref)
    cls, _ = oracle.classify(ca)
    p = me.me_default_params(search_range=16)
    dcur = torch.from_numpy(np.ascontiguousarray(cur)).cuda()
    dref = torch.from_numpy(np.ascontiguousarray(padded)).cuda()
    dca = torch.from_numpy(np.ascontiguousarray(ca)).cuda()
    dra = torch.from_numpy(np.ascontiguousarray(ra)).cuda()
    dcls = torch.from_numpy(cls).cuda()
    out = dv.Outputs.alloc(1, H // 16, W // 16)
    s = dv.stream_handle()
    say("search on padded reference", method)
    if method is None:
        j = dv.job(dcur, dref, dca, dra, dcls, None, out, 0)
        me.me_texture_recursive([j], p, None, stream=s)
        torch.cuda.synchronize()
        want = oracle.pa(cur, want_ref, oracle_params(p), cur_alpha=ca, ref_alpha=ra, cls=cls)
    else:
        j = dv.job(dcur, dref, None, None, dcls, None, out, 0)
        me.me_full_search(method, [j], p, stream=s)
        torch.cuda.synchronize()
        want = oracle.search(method, cur, want_ref, oracle_params(p), cls)
    assert me.me_device_status(s) == me.ME_OK
    got = out.host()
    assert_same({k: got[k][0] for k in got}, want, f"padded reference, method {method}",
                keys=("mv", "mv_int", "cost", "points"))


@pytest.mark.parametrize("case", ["qcif-one-call", "qcif-per-pair", "cif-two-vops"])
def test_pa_section4_protocol(torch_cuda, case):
    """Section 4 protocol assembled: frame distance 2, unrestricted vectors
    and the MPEG-4-padded reference VOP (padded by me_pad_vops, one call for
    every VOP and frame), against the oracle under the same protocol; SSE and
    pixel counts of MC over the padded reference too."""
    import torch
    from paper_1002_1168_amd import device as dv
    from gpu_util import gpu_classify, gpu_pa, oracle_pa
    if case.startswith("qcif"):
        seq, S, vops = synth.qcif_ellipse(frames=6), 7, [0]
    else:
        seq, S, vops = synth.cif_two_vops(frames=5), 16, [0, 1]
    ds = dv.DeviceSequence(seq)
    gpu_classify(ds)
    refs = ds.padded_refs()
    torch.cuda.synchronize()
    for v in vops:
        for t in range(seq.frames):
            assert np.array_equal(refs[v, t].cpu().numpy(), oracle.pad_vop(seq.luma[t], seq.alpha[v, t])), (v, t)
    p = me.me_default_params(search_range=S, half_pel=1, flags=me.ME_FLAG_UNRESTRICTED)
    pairs = seq.frames - 2
    say("section 4 protocol", case)
    got = gpu_pa(ds, vops, p, pairs, one_call=case != "qcif-per-pair", distance=2, refs=refs)
    for v in vops:
        res = oracle.pa_sequence(seq, v, oracle_params(p), pairs=pairs, distance=2, padded=True)
        want = {k: np.stack([r[k] for r in res]) for k in ("mv", "mv_int", "cost", "iters", "points")}
        assert_same(got[v], want, f"{case} vop {v}")
        # MC over the padded reference with the GPU's vectors
        out = dv.Outputs.alloc(pairs, ds.hm, ds.wm)
        out.mv.copy_(torch.from_numpy(got[v]["mv"]).cuda())
        jobs = [dv.mc_job(ds.luma[i + 2], refs[v, i], ds.alpha[v, i + 2], ds.cls[v, i + 2], out.mv[i])
                for i in range(pairs)]
        sse, npx, _, rc = me.me_motion_compensate_psnr(jobs, stream=dv.stream_handle(), check=False)
        assert rc in (me.ME_OK, me.ME_EEMPTY), rc
        assert [int(x) for x in sse] == [r["sse"] for r in res]
        assert [int(x) for x in npx] == [r["npix"] for r in res]
