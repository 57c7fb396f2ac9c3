"""The allocation-free MC/SSE entry point against the allocating one, through
the C ABI: the same per-job sums and predicted frames on two calls in a row,
the second with a smaller input (stale scratch contents must not leak)."""
import numpy as np
import pytest

import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth

from gpu_util import gpu_classify, gpu_pa, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    me.lib()
    return torch


def mc_jobs(ds, res, vops, pairs):
    from paper_1002_1168_amd.device import mc_job
    import torch
    jobs, keep = [], []
    for v in vops:
        for i in range(pairs):
            t = i + 1
            mv = torch.from_numpy(np.ascontiguousarray(res[v]["mv"][i])).cuda()
            keep.append(mv)
            if v is None:
                jobs.append(mc_job(ds.luma[t], ds.luma[t - 1], None, None, mv))
            else:
                jobs.append(mc_job(ds.luma[t], ds.luma[t - 1], ds.alpha[v, t], ds.cls[v, t], mv))
    return jobs, keep


def both(torch, jobs, H, W, half):
    """(sums, preds) from the allocating call and from the allocation-free one."""
    from paper_1002_1168_amd.device import stream_handle
    s = stream_handle()
    n = len(jobs)
    out = {}
    for name, fn in (("alloc", me.me_motion_compensate_sse), ("noalloc", me.me_motion_compensate_sse_noalloc)):
        sums = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
        preds = torch.full((n, H, W), 7, dtype=torch.uint8, device="cuda")
        fn(jobs, sums.data_ptr(), pred=[preds[i].data_ptr() for i in range(n)], stream=s)
        torch.cuda.synchronize()
        out[name] = (sums.cpu().numpy(), preds.cpu().numpy())
    assert me.me_device_status(s) == me.ME_OK
    return out


def test_noalloc_mc_matches_allocating_call_twice(torch_cuda):
    torch = torch_cuda
    from paper_1002_1168_amd.device import DeviceSequence
    # call 1: a 352 x 288 crop of a 1920 x 1088 stream, two VOPs and the rectangular frame, 3 pairs each,
    # half-pel vectors
    seq = synth.hd_streams(frames=4, streams=1)[0]
    # a 352 x 288 crop centred on VOP 0 in frame 1, with the two VOPs that
    # have the most pixels there
    ys, xs = np.nonzero(seq.alpha[0, 1])
    y0 = int(np.clip((ys.mean() - 144) // 16 * 16, 0, seq.height - 288))
    x0 = int(np.clip((xs.mean() - 176) // 16 * 16, 0, seq.width - 352))
    crop = seq.alpha[:, :, y0:y0 + 288, x0:x0 + 352]
    keepv = np.argsort([-(crop[v] != 0).sum() for v in range(seq.vops)])[:2]
    seq.luma = np.ascontiguousarray(seq.luma[:, y0:y0 + 288, x0:x0 + 352])
    seq.alpha = np.ascontiguousarray(crop[keepv])
    ds = DeviceSequence(seq)
    gpu_classify(ds)
    p = me.me_default_params(search_range=32, half_pel=1)
    res = gpu_pa(ds, [0, 1, None], p, 3)
    jobs, keep = mc_jobs(ds, res, [0, 1, None], 3)
    say("noalloc call 1:", len(jobs), "jobs", seq.width, "x", seq.height)
    r = both(torch, jobs, seq.height, seq.width, True)
    assert np.array_equal(r["alloc"][0], r["noalloc"][0]), (r["alloc"][0], r["noalloc"][0])
    assert np.array_equal(r["alloc"][1], r["noalloc"][1])
    assert (r["noalloc"][0][1::2] > 0).all()
    # call 2: a smaller input (QCIF, one VOP, 2 pairs) right after
    q = synth.qcif_ellipse(frames=3)
    dq = DeviceSequence(q)
    gpu_classify(dq)
    pq = me.me_default_params(search_range=7)
    rq = gpu_pa(dq, [0], pq, 2)
    jobs2, keep2 = mc_jobs(dq, rq, [0], 2)
    say("noalloc call 2:", len(jobs2), "jobs", q.width, "x", q.height)
    r2 = both(torch, jobs2, q.height, q.width, False)
    assert np.array_equal(r2["alloc"][0], r2["noalloc"][0]), (r2["alloc"][0], r2["noalloc"][0])
    assert np.array_equal(r2["alloc"][1], r2["noalloc"][1])


def test_noalloc_limits_rejected_on_host(torch_cuda):
    torch = torch_cuda
    from paper_1002_1168_amd.device import mc_job
    luma = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    mv = torch.zeros((1, 1, 2), dtype=torch.int16, device="cuda")
    sums = torch.zeros(2 * 1025, dtype=torch.int64, device="cuda")
    j = mc_job(luma, luma, None, None, mv)
    assert me.me_motion_compensate_sse_noalloc([j] * 1025, sums.data_ptr(), check=False) == me.ME_EINVAL
    big = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")   # 65536 MBs per job
    mvb = torch.zeros((256, 256, 2), dtype=torch.int16, device="cuda")
    jb = mc_job(big, big, None, None, mvb)
    assert me.me_motion_compensate_sse_noalloc([jb] * 9, sums.data_ptr(), check=False) == me.ME_EINVAL
    assert me.me_motion_compensate_sse_noalloc([jb] * 8, sums.data_ptr(), check=False) == me.ME_OK
    assert me.me_motion_compensate_sse_noalloc([j], sums.data_ptr() + 4, check=False) == me.ME_EALIGN
    torch.cuda.synchronize()
