"""Pins of the Section 3.1 text reading (a boundary MB's temporal candidate
is evaluated on texture): the spatial candidates are scored on the BABs, and
T replaces their winner when its luma SAD over the VOP pixels is strictly
lower.  Built by hand so that the two readings, and a texture SAD that
forgot the VOP mask, give different answers."""
import numpy as np
import pytest


def frames():
    """48 x 32 frame; the VOP is the column band 16 <= x < 24 in both frames
    (MB (1, 0) is a boundary MB; the MBs of column 0 are transparent, so A,
    B and C of MB (1, 0) are all (0, 0)).  Inside the VOP, cur is the
    reference three rows down (T = (0, 3) matches exactly) on a low-contrast
    texture; outside, cur equals the reference (d = 0 matches there) and the
    reference has full-contrast row stripes (a shift by three rows costs
    255 per pixel outside the VOP)."""
    W, H = 48, 32
    y, x = np.mgrid[0:H + 3, 0:W]
    ref_ext = np.where((x >= 16) & (x < 24), 100 + (x + 2 * y) % 7, 255 * (y % 2)).astype(np.uint8)
    ref = ref_ext[:H].copy()
    cur = ref.copy()
    inside = np.zeros((H, W), bool)
    inside[:, 16:24] = True
    cur[inside] = ref_ext[3:H + 3][inside]
    alpha = np.where(inside, 255, 0).astype(np.uint8)
    return cur, ref, alpha


def run(orc, t_texture, shape_only=False):
    cur, ref, alpha = frames()
    cls, _ = orc.classify(alpha)
    assert cls[0, 1] == 2 and cls[0, 0] == 0
    t = np.zeros((2, 3, 2), np.int16)
    t[0, 1] = (0, 6)   # T of MB (1, 0): (0, 3) in half-pel units
    return orc.pa(cur, ref, orc.Params(search_range=7, t_texture=t_texture), alpha, alpha, cls, t,
                  shape_only=shape_only)


def test_bab_reading_keeps_the_first_minimum(orc):
    # both candidates have zero BAB mismatch (the VOP is the same in every
    # row): the listing's first minimum, A = (0, 0), wins; no recursion step
    out = run(orc, 0)
    assert tuple(out["mv"][0, 1]) == (0, 0) and out["cost"][0, 1] == 0
    assert out["points"][0, 1] == 2 and out["iters"][0, 1] == 0


def test_text_reading_takes_t_on_texture(orc):
    # masked luma SAD: T = 0 inside the VOP, A > 0 -> T; its BAB mismatch is
    # the recursion's start (0: no step); one more compared block
    out = run(orc, 1)
    assert tuple(out["mv"][0, 1]) == (0, 6) and out["cost"][0, 1] == 0
    assert out["points"][0, 1] == 3 and out["iters"][0, 1] == 0


def test_text_reading_masks_the_texture(orc):
    # the full-block SADs favour A (the stripes outside the VOP): only the
    # masked comparison picks T, as the previous pin requires
    cur, ref, _ = frames()
    a = int(np.abs(cur[0:16, 16:32].astype(int) - ref[0:16, 16:32]).sum())
    big = np.pad(ref, 8, mode="edge")
    t = int(np.abs(cur[0:16, 16:32].astype(int) - big[8 + 3:8 + 19, 8 + 16:8 + 32]).sum())
    assert a < t


def test_text_reading_leaves_other_modes_alone(orc):
    # shape-only search and opaque / rectangular MBs are unchanged
    assert np.array_equal(run(orc, 1, shape_only=True)["mv"], run(orc, 0, shape_only=True)["mv"])
    cur, ref, _ = frames()
    a = orc.pa(cur, ref, orc.Params(search_range=7, t_texture=1))
    b = orc.pa(cur, ref, orc.Params(search_range=7))
    for k in a:
        assert np.array_equal(a[k], b[k])
