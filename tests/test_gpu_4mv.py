"""GPU parity of the four-vector mode: me_refine_8x8 (the pel-recursive
refinement on the 8 x 8 blocks of texture MBs, Section 3.2) and
me_motion_compensate4_sse against the oracle fed the same MB vectors,
bit-exact (vectors, costs, iteration and point counts, SSE, pixel counts,
predicted frames)."""
import numpy as np
import pytest

import oracle
import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth

from gpu_util import gpu_classify, gpu_pa, oracle_params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    me.lib()
    return torch


def hd_crop(vops=3):
    seq = synth.hd_streams(frames=3, streams=1)[0]
    ys, xs = np.nonzero(seq.alpha[0, 1])
    y0 = int(np.clip((ys.mean() - 160) // 16 * 16, 0, seq.height - 320))
    x0 = int(np.clip((xs.mean() - 192) // 16 * 16, 0, seq.width - 384))
    seq.luma = np.ascontiguousarray(seq.luma[:, y0:y0 + 320, x0:x0 + 384])
    seq.alpha = np.ascontiguousarray(seq.alpha[:vops, :, y0:y0 + 320, x0:x0 + 384])
    return seq


CASES = {
    "qcif": (lambda: synth.qcif_ellipse(frames=5), [0, None], dict(search_range=7), 4),
    "cif": (lambda: synth.cif_two_vops(frames=4), [0, 1, None], dict(search_range=16), 3),
    "hd-halfpel": (lambda: hd_crop(), [0, 1, None], dict(search_range=32, half_pel=1), 2),
    "noise-kmax": (lambda: synth.random_frames(7, 64, 48, frames=3, vops=1, search_range=4), [0, None],
                   dict(search_range=4, k_max=255, max_step=2), 2),
    "eps-half": (lambda: synth.qcif_ellipse(frames=3), [0], dict(search_range=7, eps_q12=2048, k_max=0), 2),
    "unrestricted": (lambda: synth.qcif_ellipse(frames=4), [0, None],
                     dict(search_range=7, half_pel=1, flags=me.ME_FLAG_UNRESTRICTED), 3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_refine_8x8_and_mc4_parity(torch_cuda, case):
    torch = torch_cuda
    from paper_1002_1168_amd import device as dv
    make, vops, over, P = CASES[case]
    seq = make()
    p = me.me_default_params(**over)
    say("4mv", case, seq.width, seq.height, vops, over)
    ds = dv.DeviceSequence(seq)
    gpu_classify(ds)
    res = gpu_pa(ds, vops, p, P)
    s = dv.stream_handle()
    for v in vops:
        # the search's outputs on the device, then the four-vector refinement
        out = dv.Outputs.alloc(P, ds.hm, ds.wm)
        out.mv.copy_(torch.from_numpy(res[v]["mv"]))
        out.mv_int.copy_(torch.from_numpy(res[v]["mv_int"]))
        jobs = ds.pair_jobs(v, out, P, chained=False)
        mv4 = torch.full((P, ds.hm, ds.wm, 4, 2), 0x3333, dtype=torch.int16, device="cuda")
        c4 = torch.full((P, ds.hm, ds.wm, 4), -1, dtype=torch.int32, device="cuda")
        i4 = torch.full((P, ds.hm, ds.wm, 4), 77, dtype=torch.uint8, device="cuda")
        p4 = torch.full((P, ds.hm, ds.wm, 4), -1, dtype=torch.int16, device="cuda")
        me.me_refine_8x8(jobs, p, [mv4[i].data_ptr() for i in range(P)], [c4[i].data_ptr() for i in range(P)],
                         [i4[i].data_ptr() for i in range(P)], [p4[i].data_ptr() for i in range(P)], stream=s)
        sums = torch.zeros(2 * P, dtype=torch.int64, device="cuda")
        pred = torch.zeros((P, ds.H, ds.W), dtype=torch.uint8, device="cuda")
        me.me_motion_compensate4_sse(jobs, [mv4[i].data_ptr() for i in range(P)], sums.data_ptr(),
                                     pred=[pred[i].data_ptr() for i in range(P)], stream=s)
        torch.cuda.synchronize()
        assert me.me_device_status(s) == me.ME_OK
        g4, gc, gi, gp = (mv4.cpu().numpy(), c4.cpu().numpy().view(np.uint32), i4.cpu().numpy(),
                          p4.cpu().numpy().view(np.uint16))
        gs, gpred = sums.cpu().numpy(), pred.cpu().numpy()
        for i in range(P):
            t = i + 1
            ca = None if v is None else seq.alpha[v, t]
            cls = None if v is None else oracle.classify(ca)[0]
            want = oracle.prs8(seq.luma[t], seq.luma[t - 1], oracle_params(p), res[v]["mv"][i],
                               res[v]["mv_int"][i], cls)
            for key, got in (("mv4", g4[i]), ("cost4", gc[i]), ("iters4", gi[i]), ("points4", gp[i])):
                if not np.array_equal(got, want[key]):
                    bad = np.argwhere(got != want[key])[0]
                    raise AssertionError(f"{case} vop {v} pair {i} {key} at {tuple(bad)}: gpu "
                                         f"{got[tuple(bad)]} oracle {want[key][tuple(bad)]}")
            sse, npx, wp = oracle.mc4_sse(seq.luma[t], seq.luma[t - 1], want["mv4"], ca, cls, want_pred=True)
            assert (int(gs[2 * i]), int(gs[2 * i + 1])) == (sse, npx), (case, v, i)
            assert np.array_equal(gpred[i], wp), (case, v, i)


def test_refine_8x8_rejects_bad_arguments(torch_cuda):
    torch = torch_cuda
    from paper_1002_1168_amd.device import Outputs, job
    f = torch.zeros((32, 32), dtype=torch.uint8, device="cuda")
    out = Outputs.alloc(1, 2, 2)
    j = job(f, f, None, None, None, None, out, 0)
    p = me.me_default_params(search_range=4)
    mv4 = torch.zeros((2, 2, 4, 2), dtype=torch.int16, device="cuda")
    assert me.me_refine_8x8([j], p, [None], check=False) == me.ME_EINVAL
    assert me.me_refine_8x8([j], p, [mv4.data_ptr() + 2], check=False) == me.ME_EALIGN
    bad = me.me_default_params(search_range=0)
    assert me.me_refine_8x8([j], bad, [mv4.data_ptr()], check=False) == me.ME_EINVAL
    sums = torch.zeros(2, dtype=torch.int64, device="cuda")
    assert me.me_motion_compensate4_sse([j], [None], sums.data_ptr(), check=False) == me.ME_EINVAL
    assert me.me_refine_8x8([j], p, [mv4.data_ptr()], check=False) == me.ME_OK
    torch.cuda.synchronize()
