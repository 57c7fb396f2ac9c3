"""Pins of the oracle's unrestricted-vector reading (MPEG-4 reference
padding, the Section 4 protocol): with the reference extended by repeating
its edge pixels, a vector is admissible when |dx|, |dy| <= S, wherever the
displaced block lands.  Expectations: closed-form point counts, and
translations across the frame edge built with numpy's edge padding."""
import numpy as np
import pytest

from paper_1002_1168_amd import synth


def edge_shifted(ref, d):
    """cur(x, y) = ref(clamp(x + dx), clamp(y + dy)): numpy edge padding."""
    m = 40
    big = np.pad(ref, m, mode="edge")
    H, W = ref.shape
    return big[m + d[1]:m + d[1] + H, m + d[0]:m + d[0] + W].copy()


@pytest.mark.parametrize("S", [4, 7])
def test_es_unrestricted_points_closed_form(orc, S):
    f = synth.qcif_ellipse(frames=2).luma
    out = orc.search(orc.ES, f[1], f[0], orc.Params(search_range=S, unrestricted=1))
    assert (out["points"] == (2 * S + 1) ** 2).all()


@pytest.mark.parametrize("method", [0, 1, 2, 3])
def test_baselines_unrestricted_identical_frames(orc, method):
    f = synth.qcif_ellipse(frames=1).luma[0]
    out = orc.search(method, f, f, orc.Params(search_range=7, unrestricted=1))
    assert (out["mv"] == 0).all() and (out["cost"] == 0).all()
    # corner MBs see the full patterns: TSS 25, DS 13, 4SS 17 points
    want = {0: 225, 1: 25, 2: 13, 3: 17}[method]
    assert (out["points"] == want).all()


@pytest.mark.parametrize("d", [(-3, -2), (5, 4), (-7, 6)])
def test_es_recovers_translation_across_the_edge(orc, d):
    rng = np.random.default_rng(8)
    ref = rng.integers(0, 256, size=(64, 80), dtype=np.uint8)
    cur = edge_shifted(ref, d)
    free = orc.search(orc.ES, cur, ref, orc.Params(search_range=7, unrestricted=1))
    tight = orc.search(orc.ES, cur, ref, orc.Params(search_range=7))
    # every MB, corners included: the true shift with zero SAD
    assert (free["mv_int"] == np.array([2 * d[0], 2 * d[1]])).all()
    assert (free["cost"] == 0).all()
    # restricted: the corner MB toward the shift cannot reach it
    v = 0 if d[1] < 0 else -1
    h = 0 if d[0] < 0 else -1
    assert tuple(tight["mv_int"][v, h]) != (2 * d[0], 2 * d[1])


def test_pa_unrestricted_translation_with_true_temporal(orc):
    rng = np.random.default_rng(9)
    ref = rng.integers(0, 256, size=(48, 64), dtype=np.uint8)
    d = (-4, 3)
    cur = edge_shifted(ref, d)
    t = np.tile(np.array([2 * d[0], 2 * d[1]], np.int16), (3, 4, 1))
    out = orc.pa(cur, ref, orc.Params(search_range=7, unrestricted=1), t_field=t)
    assert (out["mv_int"] == t).all() and (out["cost"] == 0).all() and (out["iters"] == 0).all()


def test_half_pel_unrestricted_every_offset_admissible(orc):
    # identical frames: the integer vector stays, and every MB compares all
    # eight half-sample offsets (the restricted corner MBs compare fewer)
    f = synth.qcif_ellipse(frames=1).luma[0]
    free = orc.pa(f, f, orc.Params(search_range=7, half_pel=1, unrestricted=1))
    tight = orc.pa(f, f, orc.Params(search_range=7, half_pel=1))
    assert (free["mv"] == 0).all() and (free["points"] == 1 + 8).all()
    assert tight["points"][0, 0] == 1 + 3 and tight["points"][4, 5] == 1 + 8


def test_prs_ramp_beyond_the_edge_saturates(orc):
    # ref = 20 + 3x extended by its edge: left of x = 0 it is flat (g = 0
    # gives no update there), so the MB at the left edge with cur a shift of
    # ref by -3 still converges to the shift with zero cost
    W, H = 64, 32
    y, x = np.mgrid[0:H, 0:W]
    ref = (20 + 3 * x).astype(np.uint8)
    cur = edge_shifted(ref, (-3, 0))
    out = orc.pa(cur, ref, orc.Params(search_range=7, unrestricted=1))
    assert (out["mv_int"] == np.array([-6, 0])).all() and (out["cost"] == 0).all()
    # the first MB walks there one pel per step; the rest inherit it from A or B
    assert out["iters"][0, 0] == 3 and out["iters"].sum() == 3
    # restricted at the left edge: x0 + dx >= 0 keeps d = 0
    tight = orc.pa(cur, ref, orc.Params(search_range=7))
    assert tuple(tight["mv_int"][1, 0]) == (0, 0)
