"""Shared helpers of the GPU parity tests: run a workload through the C ABI
and the same workload through the oracle, on the same seeded bytes."""
import sys

import numpy as np

import oracle
import paper_1002_1168_amd as me
from paper_1002_1168_amd import device as dv


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_params(p: me.me_params) -> oracle.Params:
    return oracle.Params(p.search_range, p.theta, p.eps_q12, p.max_step, p.k_max, p.half_pel,
                         int(bool(p.flags & me.ME_FLAG_UNRESTRICTED)), int(bool(p.flags & me.ME_FLAG_T_TEXTURE)),
                         int(bool(p.flags & me.ME_FLAG_MASKED_PRS)))


def gpu_classify(ds: dv.DeviceSequence):
    import torch
    fr, cp, bp = ds.classify_frames()
    me.me_classify_babs(fr, cp, bp, stream=dv.stream_handle())
    torch.cuda.synchronize()
    assert me.me_device_status(dv.stream_handle()) == me.ME_OK


def gpu_pa(ds: dv.DeviceSequence, vops, params, pairs, shape_only=False, one_call=True, chained=True, distance=1,
           refs=None):
    """PA for the listed VOPs (None = rectangular) over `pairs` pairs
    (reference `distance` frames back).  Returns {vop: host outputs}.  With
    one_call every VOP chain is solved in a single launch; otherwise one
    call per pair (T read from memory)."""
    import torch
    outs, jobs = {}, []
    for v in vops:
        out = dv.Outputs.alloc(pairs, ds.hm, ds.wm)
        outs[v] = out
        jobs.append(ds.pair_jobs(v, out, pairs, chained=chained, distance=distance, refs=refs))
    fn = me.me_shape_search if shape_only else me.me_texture_recursive
    s = dv.stream_handle()
    if one_call:
        flat = [j for js in jobs for j in js]
        if shape_only:
            fn(flat, params, stream=s)
        else:
            fn(flat, params, None, stream=s)
    else:
        for i in range(pairs):
            for js in jobs:
                if shape_only:
                    fn([js[i]], params, stream=s)
                else:
                    fn([js[i]], params, None, stream=s)
    torch.cuda.synchronize()
    assert me.me_device_status(s) == me.ME_OK
    return {v: o.host() for v, o in outs.items()}


def oracle_pa(seq, vop, params, pairs, shape_only=False, distance=1, padded=False):
    res = oracle.pa_sequence(seq, vop, oracle_params(params), shape_only=shape_only, pairs=pairs,
                             distance=distance, padded=padded)
    return {k: np.stack([r[k] for r in res]) for k in ("mv", "mv_int", "cost", "iters", "points")}


def assert_same(got: dict, want: dict, what: str, keys=("mv", "mv_int", "cost", "iters", "points")):
    for k in keys:
        g, w = np.asarray(got[k]), np.asarray(want[k])
        if not np.array_equal(g, w):
            bad = np.argwhere(g != w)
            idx = tuple(bad[0])
            raise AssertionError(f"{what}: {k} differs at {len(bad)} places, first {idx}: gpu {g[idx]} oracle {w[idx]}")
