"""Pins of the oracle's vertical gradient axis and of the half-sample
frame-edge rule.

Section 3.2 gives Eqs. 4-5 for the x component and obtains u_y "by
exchanging the index"; these pins fix the y component on its own: vertical
ramps (interior closed form, top- and bottom-edge clamps in frames whose
width differs from their height, so that a clamp taken against the wrong
dimension shows), a plane with different slopes along x and y (so that the
two components cannot be swapped or share a gradient), and the recursion's
iteration count along y.  The half-sample rule (Section 4, half-sample
accuracy; MPEG-4 bilinear interpolation) is pinned at every kind of frame
edge against an independent formulation on the 2x upsampled grid.

Every expected value is worked out by hand in the comments or computed by
numpy from the definition, never by the oracle.
"""
import numpy as np
import pytest


def vramp_pair(delta, W=48, H=64, slope=3, base=20):
    """ref(x, y) = base + slope*y, cur(x, y) = ref(x, y + delta)."""
    y = np.arange(H)[:, None]
    ref = np.broadcast_to(base + slope * y, (H, W)).astype(np.uint8)
    cur = np.broadcast_to(base + slope * (y + delta), (H, W)).astype(np.uint8)
    return np.ascontiguousarray(cur), np.ascontiguousarray(ref)


def hramp_pair(delta, W=64, H=48, slope=3, base=20):
    x = np.arange(W)[None, :]
    ref = np.broadcast_to(base + slope * x, (H, W)).astype(np.uint8)
    cur = np.broadcast_to(base + slope * (x + delta), (H, W)).astype(np.uint8)
    return np.ascontiguousarray(cur), np.ascontiguousarray(ref)


# ------------------------------------------------------------ vertical axis
@pytest.mark.parametrize("delta", [-3, -1, 0, 2, 3])
def test_prs_pass_vertical_ramp_interior(orc, delta):
    # e = 3 delta at every pixel, g_y = ref(y+1) - ref(y-1) = 6 -> R[6] = 1365
    # (Theta 3), g_x = 0 -> no x term: U = (0, 1365 * 3 delta) = (0, 4095 delta)
    cur, ref = vramp_pair(delta)
    assert orc.prs_pass(cur, ref, 16, 16, 0, 0, theta=3) == (0, 4095 * delta)


@pytest.mark.parametrize("delta,want", [(1, 4351), (-1, -4351), (2, 8702)])
def test_prs_pass_vertical_ramp_top_edge_clamped(orc, delta, want):
    # Theta 1, MB at y0 = 0: the top row's central difference is clamped to
    # ref(1) - ref(0) = 3 -> R[3] = floor(16387 / 6) = 2731; the other 15 rows
    # have g = 6 -> R[6] = floor(16390 / 12) = 1365.  Per column
    # (15 * 3 * 1365 + 3 * 2731) * delta = 69618 delta over 16 pixels
    # = 4351.125 delta, truncated toward zero.
    cur, ref = vramp_pair(delta)
    ux, uy = orc.prs_pass(cur, ref, 16, 0, 0, 0, theta=1)
    assert (ux, uy) == (0, want)


@pytest.mark.parametrize("W,H", [(48, 64), (80, 64)])
@pytest.mark.parametrize("delta,want", [(-1, -4351), (-2, -8702), (1, 4351)])
def test_prs_pass_vertical_ramp_bottom_edge_clamped(orc, W, H, delta, want):
    # the bottom MB (y0 = H - 16): its last row is clamped to
    # ref(H-1) - ref(H-2) = 3, the mirror image of the top edge.  W != H, so a
    # clamp bound taken from the width reads other rows (W < H) or runs past
    # the frame (W > H) and fails.  delta > 0 shifts cur past the ramp's top
    # row, which still fits a byte: 20 + 3 * 64 = 212.
    cur, ref = vramp_pair(delta, W=W, H=H)
    ux, uy = orc.prs_pass(cur, ref, 16, H - 16, 0, 0, theta=1)
    assert (ux, uy) == (0, want)


@pytest.mark.parametrize("W,H", [(64, 48), (64, 80)])
@pytest.mark.parametrize("delta,want", [(1, 4351), (-1, -4351)])
def test_prs_pass_horizontal_ramp_right_edge_clamped(orc, W, H, delta, want):
    # the x mirror of the bottom-edge case, with H != W
    cur, ref = hramp_pair(delta, W=W, H=H)
    ux, uy = orc.prs_pass(cur, ref, W - 16, 16, 0, 0, theta=1)
    assert (ux, uy) == (want, 0)


@pytest.mark.parametrize("dx,dy", [(1, -1), (-1, 2), (2, 1), (0, -2)])
def test_prs_pass_plane_sets_both_components(orc, dx, dy):
    # ref = 10 + 2x + 3y on 48 x 48 (at most 10 + 94 + 141 = 245), cur = ref
    # displaced by (dx, dy): e = 2 dx + 3 dy everywhere.  With Theta 2:
    # g_x = 4 -> R[4] = floor(16388 / 8) = 2048, g_y = 6 -> R[6] =
    # floor(16390 / 12) = 1365.  So U = (2048 e, 1365 e): different gains on
    # the two axes, each signed like e.
    W = H = 48
    y, x = np.mgrid[0:H, 0:W]
    ref = (10 + 2 * x + 3 * y).astype(np.uint8)
    cur = np.clip(10 + 2 * (x + dx) + 3 * (y + dy), 0, 255).astype(np.uint8)
    e = 2 * dx + 3 * dy
    assert orc.prs_pass(cur, ref, 16, 16, 0, 0, theta=2) == (2048 * e, 1365 * e)


def one_mb_alpha(W, H, h=1, v=1):
    a = np.zeros((H, W), np.uint8)
    a[16 * v:16 * v + 16, 16 * h:16 * h + 16] = 255
    return a


@pytest.mark.parametrize("delta", [-3, -1, 0, 2, 3])
@pytest.mark.parametrize("max_step", [1, 3])
def test_pa_vertical_ramp_iterations_closed_form(orc, delta, max_step):
    # the recursion's update is 4095 delta / 4096 -> one pixel per step toward
    # delta (max_step 1: |delta| accepted steps and no further candidate; a
    # step of min(|delta|, 3) with max_step 3), ending on SAD 0 at (0, delta)
    cur, ref = vramp_pair(delta, W=48, H=64)
    a = one_mb_alpha(48, 64, 1, 1)
    cls, _ = orc.classify(a)
    out = orc.pa(cur, ref, orc.Params(search_range=7, theta=3, max_step=max_step), a, a, cls)
    want_iters = abs(delta) if max_step == 1 else (1 if delta else 0)
    assert tuple(out["mv_int"][1, 1]) == (0, 2 * delta)
    assert out["cost"][1, 1] == 0
    assert out["iters"][1, 1] == want_iters
    assert out["points"][1, 1] == 1 + want_iters


# --------------------------------------------------- half-sample frame edges
def np_half_grid(ref):
    """The 2x upsampled reference of MPEG-4 bilinear interpolation with
    rounding control 0: even/even samples are the pixels, the others the
    rounded means of their 2 or 4 neighbours (size (2H-1) x (2W-1))."""
    r = ref.astype(np.int64)
    H, W = r.shape
    g = np.zeros((2 * H - 1, 2 * W - 1), np.int64)
    g[0::2, 0::2] = r
    g[0::2, 1::2] = (r[:, :-1] + r[:, 1:] + 1) >> 1
    g[1::2, 0::2] = (r[:-1, :] + r[1:, :] + 1) >> 1
    g[1::2, 1::2] = (r[:-1, :-1] + r[:-1, 1:] + r[1:, :-1] + r[1:, 1:] + 2) >> 2
    return g


def np_half_feasible(W, H, S, x0, y0, hx, hy):
    """A half-sample block is admissible when its 16 x 16 samples lie on the
    upsampled grid (every pixel the interpolation reads is in the frame) and
    |h| <= 2S: rows 2*y0 + hy .. 2*(y0 + 15) + hy inside 0 .. 2H - 2."""
    return (abs(hx) <= 2 * S and abs(hy) <= 2 * S and 2 * x0 + hx >= 0 and 2 * (x0 + 15) + hx <= 2 * W - 2
            and 2 * y0 + hy >= 0 and 2 * (y0 + 15) + hy <= 2 * H - 2)


OFFS = [(-1, -1), (0, -1), (1, -1), (-1, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]


def test_half_feasible_closed_form_counts():
    # the independent formulation itself, against counts worked out by hand:
    # corner MBs keep 3 of the 8 offsets, edge MBs 5, interior MBs 8
    W, H = 64, 48
    cnt = lambda x0, y0: sum(np_half_feasible(W, H, 7, x0, y0, ox, oy) for ox, oy in OFFS)
    assert cnt(0, 0) == 3 and cnt(W - 16, 0) == 3 and cnt(0, H - 16) == 3 and cnt(W - 16, H - 16) == 3
    assert cnt(16, 0) == 5 and cnt(0, 16) == 5 and cnt(W - 16, 16) == 5 and cnt(16, H - 16) == 5
    assert cnt(16, 16) == 8
    assert not np_half_feasible(W, H, 7, W - 16, 16, 1, 0)
    assert not np_half_feasible(W, H, 7, 0, 16, -1, 0)
    assert not np_half_feasible(W, H, 7, 16, 0, 0, -1)
    assert not np_half_feasible(W, H, 7, 16, H - 16, 0, 1)


@pytest.mark.parametrize("W,H", [(64, 48), (48, 64)])
def test_half_pel_points_at_frame_edges(orc, W, H):
    # identical constant frames: the integer search stops at (0, 0) with SAD 0
    # (one compared block, no recursion), every half-sample candidate ties and
    # loses, so points = 1 + the number of admissible half-sample offsets
    f = np.full((H, W), 77, np.uint8)
    out = orc.pa(f, f, orc.Params(search_range=7, half_pel=1))
    for v in range(H // 16):
        for h in range(W // 16):
            want = 1 + sum(np_half_feasible(W, H, 7, 16 * h, 16 * v, ox, oy) for ox, oy in OFFS)
            assert out["points"][v, h] == want, (h, v)
            assert tuple(out["mv"][v, h]) == (0, 0)


@pytest.mark.parametrize("W,H", [(64, 48), (48, 64)])
def test_half_pel_best_offset_outside_frame_is_not_taken(orc, W, H):
    # cur(x, y) = ref(x + 1/2, y + 1/2) exactly on a plane ref = 20 + 2x + 2y
    # (the 4-tap mean (4 ref + 8 + 2) >> 2 = ref + 2, cur = 22 + 2x + 2y), so
    # the half-sample offset (+1, +1) has SAD 0 wherever it is admissible.  At
    # Theta 3 the gradient (|g| = 4 < 6) gives no integer step, so each MB
    # compares (0, 0) and then the admissible half-sample offsets.  Where
    # (+1, +1) is admissible it wins with SAD 0; elsewhere the winner is the
    # best admissible offset on the numpy half grid.
    y, x = np.mgrid[0:H, 0:W]
    ref = (20 + 2 * x + 2 * y).astype(np.uint8)
    cur = (22 + 2 * x + 2 * y).astype(np.uint8)
    g = np_half_grid(ref)
    out = orc.pa(cur, ref, orc.Params(search_range=7, half_pel=1))
    for v in range(H // 16):
        for h in range(W // 16):
            x0, y0 = 16 * h, 16 * v
            blk = cur[y0:y0 + 16, x0:x0 + 16].astype(np.int64)
            best, bsad = (0, 0), int(np.abs(blk - ref[y0:y0 + 16, x0:x0 + 16]).sum())
            for ox, oy in OFFS:
                if not np_half_feasible(W, H, 7, x0, y0, ox, oy):
                    continue
                p = g[2 * y0 + oy:2 * (y0 + 15) + oy + 1:2, 2 * x0 + ox:2 * (x0 + 15) + ox + 1:2]
                s = int(np.abs(blk - p).sum())
                if s < bsad:
                    best, bsad = (ox, oy), s
            assert tuple(out["mv"][v, h]) == best, (h, v)
            assert out["cost"][v, h] == bsad, (h, v)
            inside = x0 + 16 < W and y0 + 16 < H
            assert (best == (1, 1)) == inside and (bsad == 0) == inside
