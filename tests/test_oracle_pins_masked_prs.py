"""Pins of the masked-luma reading of a boundary MB's recursion (Section 3.1
says a boundary MB's temporal candidate is evaluated on texture; in this
reading its pel recursion, Section 3.2, refines on texture too, over the
current VOP's pixels only).  Closed forms on a horizontal luma ramp: every
gradient pass sees g = 2a, so U = e / a per VOP pixel, and with max_step 1
the recursion walks one pixel per candidate until e = 0.  Built so that a
pass or a distortion that forgot the VOP mask, or the BAB reading, gives a
different answer."""
import numpy as np
import pytest

A = 4      # ramp slope (luma per pixel)
SHIFT = 3  # inside the VOP, cur is the reference three pixels to the right


def frames():
    """48 x 32 frame; the VOP is the column band 16 <= x < 24 in both frames,
    so MBs (1, 0) and (1, 1) are boundary MBs and columns 0 and 2 are
    transparent.  The reference is the ramp 40 + A x.  Inside the VOP, cur is
    the reference SHIFT pixels to the right; outside, SHIFT pixels to the
    left, so that a pass over the whole block sees opposite errors that
    cancel (it would not move)."""
    W, H = 48, 32
    y, x = np.mgrid[0:H, 0:W]
    ref = (40 + A * x).astype(np.uint8)
    inside = (x >= 16) & (x < 24)
    cur = np.where(inside, 40 + A * np.minimum(x + SHIFT, W - 1), 40 + A * np.maximum(x - SHIFT, 0)).astype(np.uint8)
    alpha = np.where(inside, 255, 0).astype(np.uint8)
    return cur, ref, alpha


def run(orc, masked_prs, k_max=8, cur=None, shape_only=False):
    c, ref, alpha = frames()
    cur = c if cur is None else cur
    cls, _ = orc.classify(alpha)
    assert cls[0, 1] == 2 and cls[1, 1] == 2 and cls[0, 0] == 0 and cls[0, 2] == 0
    return orc.pa(cur, ref, orc.Params(search_range=7, k_max=k_max, masked_prs=masked_prs), alpha, alpha, cls,
                  np.zeros((2, 3, 2), np.int16), shape_only=shape_only)


def test_masked_recursion_walks_to_the_vop_motion(orc):
    # MB (1, 0): one candidate (0, 0); its masked SAD (one more block) starts
    # the recursion, which steps (1, 0), (2, 0), (3, 0) and stops at U = 0
    out = run(orc, 1)
    assert tuple(out["mv"][0, 1]) == (2 * SHIFT, 0) and tuple(out["mv_int"][0, 1]) == (2 * SHIFT, 0)
    assert out["iters"][0, 1] == SHIFT and out["cost"][0, 1] == 0
    assert out["points"][0, 1] == 1 + 1 + SHIFT
    # MB (1, 1): B = (3, 0) joins the list but loses on the BABs (its shifted
    # band mismatches 3 columns), so the walk starts at (0, 0) again
    assert tuple(out["mv"][1, 1]) == (2 * SHIFT, 0) and out["iters"][1, 1] == SHIFT
    assert out["points"][1, 1] == 2 + 1 + SHIFT


def test_bab_reading_does_not_move(orc):
    # the same VOP in both frames: the shape passes see e = 0
    out = run(orc, 0)
    assert tuple(out["mv"][0, 1]) == (0, 0) and out["iters"][0, 1] == 0 and out["cost"][0, 1] == 0


@pytest.mark.parametrize("k_max, d", [(0, 0), (1, 1), (2, 2)])
def test_capped_walk_reports_the_masked_sad(orc, k_max, d):
    # 128 VOP pixels, each off by A (SHIFT - d) at (d, 0)
    out = run(orc, 1, k_max=k_max)
    assert tuple(out["mv_int"][0, 1]) == (2 * d, 0) and out["iters"][0, 1] == d
    assert out["cost"][0, 1] == 128 * A * (SHIFT - d)
    assert out["points"][0, 1] == 2 + d


def test_pixels_outside_the_vop_are_never_read(orc):
    cur, _, alpha = frames()
    other = cur.copy()
    other[alpha == 0] = 255 - other[alpha == 0]
    a, b = run(orc, 1), run(orc, 1, cur=other)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_other_modes_are_unchanged(orc):
    # shape-only search, and opaque / rectangular MBs
    for k, v in run(orc, 1, shape_only=True).items():
        assert np.array_equal(v, run(orc, 0, shape_only=True)[k]), k
    cur, ref, _ = frames()
    a = orc.pa(cur, ref, orc.Params(search_range=7, masked_prs=1))
    b = orc.pa(cur, ref, orc.Params(search_range=7))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
