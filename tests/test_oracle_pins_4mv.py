"""Pins of the oracle's four-vector mode (Section 3.2: the pel-recursive
search on the 8 x 8 blocks of a macroblock) and of motion compensation with
four vectors per MB.  Expectations are closed forms worked out by hand on
ramps, numpy indexing, and reductions to the one-vector path."""
import numpy as np
import pytest

from paper_1002_1168_amd import synth


def block_shift_pair(shifts, axis, W=64, H=64):
    """ref = 20 + 3 * (x or y); in every MB, block b of cur is ref displaced
    by shifts[b] along `axis` (a linear ramp, so the 8 x 8 SAD at offset d is
    64 * 3 * |shift - d| away from the edges)."""
    y, x = np.mgrid[0:H, 0:W]
    base = x if axis == 0 else y
    ref = (20 + 3 * base).astype(np.uint8)
    cur = np.empty_like(ref)
    for by in (0, 1):
        for bx in (0, 1):
            m = ((y % 16) // 8 == by) & ((x % 16) // 8 == bx)
            cur[m] = (20 + 3 * (base[m] + shifts[2 * by + bx])).astype(np.uint8)
    return cur, ref


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("shifts", [(1, -2, 3, 0), (-3, 2, 0, 1)])
def test_prs8_ramp_per_block_closed_form(orc, axis, shifts):
    # from a zero MB vector, each block walks one pixel per accepted step to
    # its own shift (Eq. 3 mean 4095 (shift - d) in Q.12, one pel per step
    # at max_step 1): iters = |shift|, final SAD 0, the other axis untouched
    cur, ref = block_shift_pair(shifts, axis)
    z = np.zeros((4, 4, 2), np.int16)
    out = orc.prs8(cur, ref, orc.Params(search_range=7), z, z)
    for v, h in [(1, 1), (1, 2), (2, 1), (2, 2)]:
        for b in range(4):
            d = shifts[b]
            want = (2 * d, 0) if axis == 0 else (0, 2 * d)
            assert tuple(out["mv4"][v, h, b]) == want, (v, h, b, out["mv4"][v, h, b])
            assert out["cost4"][v, h, b] == 0
            assert out["iters4"][v, h, b] == abs(d) and out["points4"][v, h, b] == abs(d)


def test_prs8_jump_step_one_iteration(orc):
    # max_step >= |shift|: one step lands on the shift
    cur, ref = block_shift_pair((3, -2, 1, -3), 0)
    z = np.zeros((4, 4, 2), np.int16)
    out = orc.prs8(cur, ref, orc.Params(search_range=7, max_step=7), z, z)
    for b, d in enumerate((3, -2, 1, -3)):
        assert tuple(out["mv4"][2, 2, b]) == (2 * d, 0) and out["iters4"][2, 2, b] == 1


def test_prs8_starts_from_the_mb_vector(orc):
    # a start vector equal to a block's shift costs 0 there: no iteration
    cur, ref = block_shift_pair((2, 2, -1, 2), 0)
    start = np.zeros((4, 4, 2), np.int16)
    start[..., 0] = 4   # full-pel (2, 0)
    out = orc.prs8(cur, ref, orc.Params(search_range=7), start, start)
    assert tuple(out["iters4"][2, 2]) == (0, 0, 3, 0)
    assert tuple(out["mv4"][2, 2, 2]) == (-2, 0)


def test_prs8_identical_frames_and_classes(orc):
    f = synth.qcif_ellipse(frames=1)
    luma, alpha = f.luma[0], f.alpha[0, 0]
    cls, _ = orc.classify(alpha)
    mv = np.zeros((9, 11, 2), np.int16)
    mv[..., 0] = 6
    mv[..., 1] = -3     # a half-pel shape vector: kept as is on boundary MBs
    mvi = np.zeros_like(mv)
    out = orc.prs8(luma, luma, orc.Params(search_range=7), mv, mvi, cls)
    op, bd, tr = cls == 1, cls == 2, cls == 0
    assert (out["mv4"][op] == 0).all() and (out["iters4"][op] == 0).all() and (out["cost4"][op] == 0).all()
    assert (out["mv4"][bd] == np.array([6, -3])).all() and (out["points4"][bd] == 0).all()
    assert (out["mv4"][tr] == 0).all()


def test_prs8_cost_never_above_start_and_half_pel_points(orc):
    seq = synth.cif_two_vops(frames=3)
    p = orc.Params(search_range=16, half_pel=1)
    cls, _ = orc.classify(seq.alpha[0, 1])
    r = orc.pa(seq.luma[1], seq.luma[0], p, seq.alpha[0, 1], seq.alpha[0, 0], cls)
    out = orc.prs8(seq.luma[1], seq.luma[0], p, r["mv"], r["mv_int"], cls)
    cur = seq.luma[1].astype(np.int64)
    ref = seq.luma[0].astype(np.int64)
    for v, h in zip(*np.nonzero(cls == 1)):
        dx, dy = r["mv_int"][v, h] // 2
        for b in range(4):
            y0, x0 = 16 * v + 8 * (b >> 1), 16 * h + 8 * (b & 1)
            start = np.abs(cur[y0:y0 + 8, x0:x0 + 8] - ref[y0 + dy:y0 + dy + 8, x0 + dx:x0 + dx + 8]).sum()
            assert out["cost4"][v, h, b] <= start
            # recursion candidates plus at most 8 half-sample ones
            assert out["iters4"][v, h, b] <= out["points4"][v, h, b] <= out["iters4"][v, h, b] + 8


def test_mc4_equal_vectors_is_mc(orc):
    # four equal vectors per MB reduce to the one-vector prediction
    seq = synth.cif_two_vops(frames=2)
    rng = np.random.default_rng(5)
    mv = rng.integers(-6, 7, size=(18, 22, 2)).astype(np.int16)
    mv4 = np.repeat(mv[:, :, None, :], 4, axis=2)
    cls, _ = orc.classify(seq.alpha[1, 1])
    a = orc.mc_sse(seq.luma[1], seq.luma[0], mv, seq.alpha[1, 1], cls, want_pred=True)
    b = orc.mc4_sse(seq.luma[1], seq.luma[0], mv4, seq.alpha[1, 1], cls, want_pred=True)
    assert a[:2] == b[:2] and np.array_equal(a[2], b[2])


def test_mc4_integer_vectors_vs_numpy(orc):
    # whole-pel vectors, one per 8 x 8 block, away from the frame edges: the
    # prediction is plain indexing
    rng = np.random.default_rng(6)
    H, W = 64, 80
    cur = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    ref = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    mv4 = np.zeros((4, 5, 4, 2), np.int16)
    mv4[1:3, 1:4] = 2 * rng.integers(-3, 4, size=(2, 3, 4, 2))
    s, n, pred = orc.mc4_sse(cur, ref, mv4, want_pred=True)
    want = ref.copy()
    for v in range(1, 3):
        for h in range(1, 4):
            for b in range(4):
                dx, dy = mv4[v, h, b] // 2
                y0, x0 = 16 * v + 8 * (b >> 1), 16 * h + 8 * (b & 1)
                want[y0:y0 + 8, x0:x0 + 8] = ref[y0 + dy:y0 + dy + 8, x0 + dx:x0 + dx + 8]
    assert np.array_equal(pred, want)
    assert n == H * W and s == int(((cur.astype(np.int64) - want) ** 2).sum())
