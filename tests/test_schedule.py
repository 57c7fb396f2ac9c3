"""Legality of the parallel schedule, checked on the CPU.

The GPU search does not visit MBs in the raster order of Fig. 1: it hands
out MB "lines" (one MB position of one chain of frame pairs) in the order
(h + 2v, chain), and runs every line as soon as its left, upper and
upper-right neighbours (A, B, C) and its temporal candidate T are done.
Two facts make that legal:

* any order in which each MB follows A, B and C gives the raster result
  (shown here with the oracle visiting MBs on anti-diagonals and in random
  topological orders);
* the library's ticket table is a topological order of the A/B/C/T
  dependencies (shown here on the table the library builds, read through
  me_search_schedule, which touches no device).
"""
import ctypes as C

import numpy as np
import pytest

import paper_1002_1168_amd as me
from paper_1002_1168_amd import synth


def antidiagonal_order(wm, hm):
    ks = [(h + 2 * v, v, h) for v in range(hm) for h in range(wm)]
    return np.array([v * wm + h for _, v, h in sorted(ks)], np.int32)


def random_topological_order(wm, hm, rng):
    """Kahn's algorithm over the A/B/C edges with a random ready pick."""
    deps = {}
    for v in range(hm):
        for h in range(wm):
            d = []
            if h > 0:
                d.append((h - 1, v))
            if v > 0:
                d.append((h, v - 1))
                if h + 1 < wm:
                    d.append((h + 1, v - 1))
            deps[(h, v)] = set(d)
    done, order = set(), []
    ready = [m for m, d in deps.items() if not d]
    while ready:
        m = ready.pop(int(rng.integers(len(ready))))
        order.append(m[1] * wm + m[0])
        done.add(m)
        for x, d in deps.items():
            if x not in done and x not in ready and m in d and d <= done:
                ready.append(x)
    assert len(order) == wm * hm
    return np.array(order, np.int32)


@pytest.mark.parametrize("shape_only", [False, True])
def test_oracle_order_independence(orc, shape_only):
    seq = synth.cif_two_vops(seed=2, frames=4)
    H, W = seq.height, seq.width
    wm, hm = W // 16, H // 16
    p = orc.Params(search_range=16)
    rng = np.random.default_rng(11)
    orders = [antidiagonal_order(wm, hm), random_topological_order(wm, hm, rng)]
    for vop in range(seq.vops):
        tf = None
        for t in range(1, seq.frames):
            ca, ra = seq.alpha[vop, t], seq.alpha[vop, t - 1]
            cls, _ = orc.classify(ca)
            want = orc.pa(seq.luma[t], seq.luma[t - 1], p, ca, ra, cls, tf, shape_only=shape_only)
            for od in orders:
                got = orc.pa_order(seq.luma[t], seq.luma[t - 1], p, od, ca, ra, cls, tf, shape_only=shape_only)
                for k in ("mv", "mv_int", "cost", "iters", "points"):
                    np.testing.assert_array_equal(got[k], want[k], err_msg=f"{k} vop {vop} t {t}")
            tf = want["mv_int"]


def test_order_dependence_is_real(orc):
    """Control: a reversed scan (which breaks A/B/C) changes the result on
    the same data, so the check above is not vacuous."""
    seq = synth.cif_two_vops(seed=2, frames=3)
    wm, hm = seq.width // 16, seq.height // 16
    p = orc.Params(search_range=16)
    ca, ra = seq.alpha[0, 2], seq.alpha[0, 1]
    cls, _ = orc.classify(ca)
    want = orc.pa(seq.luma[2], seq.luma[1], p, ca, ra, cls)
    rev = np.arange(wm * hm, dtype=np.int32)[::-1].copy()
    got = orc.pa_order(seq.luma[2], seq.luma[1], p, rev, ca, ra, cls)
    assert not all(np.array_equal(got[k], want[k]) for k in ("mv_int", "points"))


FAKE = 0x100000


def fake_job(i, w, h, t_from=None, stride=None):
    """A job whose pointers are never dereferenced (the schedule is computed
    on the host); mv_int addresses are distinct so chains are recognised."""
    fr = me.me_frame(FAKE, None, w, h, w if stride is None else stride)
    mvi = FAKE + (1 << 24) + i * (1 << 16)
    tf = None if t_from is None else FAKE + (1 << 24) + t_from * (1 << 16)
    return me.me_job(fr, fr, None, tf, None, mvi + 8192, mvi, None, None, None)


def schedule(jobs):
    L = me.lib()
    ja = (me.me_job * len(jobs))(*jobs)
    info = (C.c_int32 * (3 * len(jobs)))()
    nl = C.c_int()
    rc = L.me_search_schedule(ja, len(jobs), info, None, 0, C.byref(nl))
    assert rc == me.ME_EINVAL and nl.value > 0      # capacity too small: count only
    lines = (C.c_uint32 * nl.value)()
    assert L.me_search_schedule(ja, len(jobs), info, lines, nl.value, C.byref(nl)) == me.ME_OK
    inf = np.array(info, np.int32).reshape(-1, 3)
    return inf, [(int(x) >> 16, (int(x) >> 8) & 0xFF, int(x) & 0xFF) for x in lines]


@pytest.mark.parametrize("case", ["one_chain", "two_vops", "mixed_sizes", "forked"])
def test_ticket_table_is_topological(case):
    if case == "one_chain":        # 5 pairs, T from the previous pair of the same chain
        jobs = [fake_job(i, 64, 48, i - 1 if i else None) for i in range(5)]
    elif case == "two_vops":       # two interleaved chains
        jobs = [fake_job(i, 96, 64, i - 2 if i >= 2 else None) for i in range(8)]
    elif case == "mixed_sizes":    # chains of different frame sizes
        jobs = [fake_job(0, 176, 144), fake_job(1, 352, 288), fake_job(2, 176, 144, 0), fake_job(3, 352, 288, 1),
                fake_job(4, 64, 32)]
    else:                          # two pairs take T from the same producer: a second chain depends on the first
        jobs = [fake_job(0, 64, 48), fake_job(1, 64, 48, 0), fake_job(2, 64, 48, 0), fake_job(3, 64, 48, 2)]
    info, lines = schedule(jobs)
    pos = {ln: i for i, ln in enumerate(lines)}
    assert len(pos) == len(lines)
    # every MB position of every chain is a line, exactly once
    dims = {}
    for j, (c, p, prod) in enumerate(info):
        w, h = jobs[j].cur.width // 16, jobs[j].cur.height // 16
        assert dims.setdefault(c, (w, h)) == (w, h)
    assert sorted(lines) == sorted((c, v, h) for c, (w, hh) in dims.items() for v in range(hh) for h in range(w))
    # producer chains of T (another chain's line at the same MB position)
    tdep = {}
    for j, (c, p, prod) in enumerate(info):
        if prod >= 0:
            pc = info[prod][0]
            if pc != c:
                tdep.setdefault(c, set()).add(int(pc))
            else:
                assert info[prod][1] == p - 1          # same chain: the previous position
    for (c, v, h), i in pos.items():
        w, _ = dims[c]
        before = []
        if h > 0:
            before.append((c, v, h - 1))
        if v > 0:
            before.append((c, v - 1, h))
            if h + 1 < w:
                before.append((c, v - 1, h + 1))
        for pc in tdep.get(c, ()):
            before.append((pc, v, h))
        for b in before:
            assert pos[b] < i, (case, (c, v, h), b)
