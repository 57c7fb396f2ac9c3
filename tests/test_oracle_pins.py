"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each check derives its expectation without the oracle: closed forms worked
out by hand, numpy brute force on tiny inputs, invariants, or special cases
that reduce to textbook behaviour.  A plausible slip in the oracle (a sign,
an index, a transposed operand, the wrong rounding) fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1002_1168_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ----------------------------------------------------------- classification
def np_classes(alpha):
    H, W = alpha.shape
    b = (alpha != 0).reshape(H // 16, 16, W // 16, 16).transpose(0, 2, 1, 3).reshape(H // 16, W // 16, 256)
    cls = np.where(b.all(-1), 1, np.where(b.any(-1), 2, 0))
    return cls.astype(np.uint8), b


def test_classify_all_zero_and_all_set(orc):
    z = np.zeros((48, 64), np.uint8)
    c, bab = orc.classify(z)
    assert (c == orc.TRANSPARENT).all() and (bab == 0).all()
    f = np.full((48, 64), 255, np.uint8)
    c, bab = orc.classify(f)
    assert (c == orc.OPAQUE).all() and (bab == 0xFFFFFFFF).all()


def test_classify_matches_numpy_and_bab_bits(orc):
    seq = synth.random_frames(7, 96, 80, frames=3, vops=1)
    for t in range(3):
        a = seq.alpha[0, t].copy()
        a[a != 0] = np.random.default_rng(t).integers(1, 256, size=int((a != 0).sum()))  # non-binary alpha
        c, bab = orc.classify(a)
        ref, bits = np_classes(a)
        np.testing.assert_array_equal(c, ref)
        assert c.size == (c == 0).sum() + (c == 1).sum() + (c == 2).sum()
        # bit (j % 2) * 16 + i of word j // 2 is pixel (i, j) of the block
        for (v, h) in [(0, 0), (2, 3), (4, 5)]:
            blk = bits[v, h].reshape(16, 16)
            for j in range(16):
                for i in range(16):
                    got = (int(bab[v, h, j // 2]) >> ((j % 2) * 16 + i)) & 1
                    assert got == int(blk[j, i])


def test_classify_grid_aligned_rectangle_has_no_boundary(orc):
    a = np.zeros((64, 96), np.uint8)
    a[16:48, 32:80] = 255
    c, _ = orc.classify(a)
    assert (c != orc.BOUNDARY).all()
    assert (c == orc.OPAQUE).sum() == 2 * 3


# ------------------------------------------------------------- block costs
def test_sad_and_mismatch_vs_numpy(orc):
    rng = np.random.default_rng(3)
    cur = rng.integers(0, 256, (64, 64), dtype=np.uint8)
    ref = rng.integers(0, 256, (64, 64), dtype=np.uint8)
    ca = np.where(rng.random((64, 64)) < 0.5, 255, 0).astype(np.uint8)
    ra = np.where(rng.random((64, 64)) < 0.5, 7, 0).astype(np.uint8)
    for (x0, y0, dx, dy) in [(16, 16, 0, 0), (16, 32, -16, 5), (32, 16, 16, -3), (0, 0, 3, 7)]:
        want = np.abs(cur[y0:y0 + 16, x0:x0 + 16].astype(int)
                      - ref[y0 + dy:y0 + dy + 16, x0 + dx:x0 + dx + 16].astype(int)).sum()
        assert orc.sad(cur, ref, x0, y0, dx, dy) == want
        mm = np.count_nonzero((ca[y0:y0 + 16, x0:x0 + 16] != 0)
                              != (ra[y0 + dy:y0 + dy + 16, x0 + dx:x0 + dx + 16] != 0))
        assert orc.mismatch(ca, ra, x0, y0, dx, dy) == mm
        # symmetric, and SAD on the 0/255 plane is 255 times the count
        assert orc.mismatch(ra, ca, x0 + dx, y0 + dy, -dx, -dy) == mm
        bc = np.where(ca != 0, 255, 0).astype(np.uint8)
        br = np.where(ra != 0, 255, 0).astype(np.uint8)
        assert orc.sad(bc, br, x0, y0, dx, dy) == 255 * mm
    assert orc.sad(cur, cur, 16, 16, 0, 0) == 0


# ------------------------------------------------ Eqs. 4-5 reciprocal table
def test_recip_table_closed_form(orc):
    g = golden("recip_theta3.json")
    for k, v in g["values"].items():
        assert orc.recip(int(k), 3) == v, k
    for a in range(1, 256):
        assert orc.recip(-a, 3) == -orc.recip(a, 3)
        # u = 2/g in Q.12 rounded half up: |R - 8192/a| <= 1/2
        r = orc.recip(a, 3)
        if a >= 6:
            assert abs(r - 8192.0 / a) <= 0.5
        else:
            assert r == 0
    assert orc.recip(0, 1) == 0
    assert orc.recip(2, 1) == 4096 and orc.recip(1, 1) == 0


def test_step_rounding(orc):
    # eps * U in Q.24 rounded half away from zero, clamped to +-max_step
    assert orc.step(2048, 4096, 5) == 1      # exactly 0.5 -> 1
    assert orc.step(-2048, 4096, 5) == -1
    assert orc.step(2047, 4096, 5) == 0
    assert orc.step(4095 * 3, 4096, 5) == 3  # 2.9993 -> 3
    assert orc.step(4095 * 3, 4096, 1) == 1
    assert orc.step(4095 * 3, 2048, 5) == 1  # eps 0.5: 1.4996 -> 1
    assert orc.step(4095, 2048, 5) == 0      # 0.49988 -> 0
    assert orc.step(0, 4096, 5) == 0


# ------------------------------------------------------ ramp closed forms
def ramp_pair(delta, W=64, H=64, slope=3, base=20):
    x = np.arange(W)
    ref = np.tile((base + slope * x).astype(np.uint8), (H, 1))
    cur = np.tile((base + slope * (x + delta)).astype(np.uint8), (H, 1))
    return cur, ref


@pytest.mark.parametrize("delta", [-3, -1, 0, 2, 3])
def test_prs_pass_ramp_interior(orc, delta):
    cur, ref = ramp_pair(delta)
    # interior MB: gx = 6 everywhere, R[6] = 1365, e = 3 delta
    ux, uy = orc.prs_pass(cur, ref, 16, 16, 0, 0, theta=3)
    assert (ux, uy) == (4095 * delta, 0)


@pytest.mark.parametrize("delta,want", [(1, 4351), (-1, -4351), (2, 8702)])
def test_prs_pass_ramp_left_edge_clamped(orc, delta, want):
    # theta 1: the clamped left-edge pixel has g = ref(1) - ref(0) = 3,
    # R[3] = 2731, the 15 interior pixels R[6] = 1365.  Per row
    # (15 * 4095 + 8193) * delta over 16 pixels -> 4351.125 * delta,
    # truncated toward zero.
    cur, ref = ramp_pair(delta)
    ux, _ = orc.prs_pass(cur, ref, 0, 16, 0, 0, theta=1)
    assert ux == want


def one_mb_alpha(W=64, H=64, h=1, v=1):
    a = np.zeros((H, W), np.uint8)
    a[16 * v:16 * v + 16, 16 * h:16 * h + 16] = 255
    return a


@pytest.mark.parametrize("delta", [-3, -1, 0, 2, 3])
@pytest.mark.parametrize("max_step", [1, 3])
def test_pa_ramp_iterations_closed_form(orc, delta, max_step):
    cur, ref = ramp_pair(delta)
    a = one_mb_alpha()
    cls, _ = orc.classify(a)
    p = orc.Params(search_range=7, theta=3, max_step=max_step, k_max=8)
    out = orc.pa(cur, ref, p, a, a, cls)
    k = (1, 1)
    want_iters = abs(delta) if max_step == 1 else (1 if delta else 0)
    assert tuple(out["mv_int"][k]) == (2 * delta, 0)
    assert out["cost"][k] == 0
    assert out["iters"][k] == want_iters
    assert out["points"][k] == 1 + want_iters
    # every other MB is transparent
    m = np.ones(cls.shape, bool)
    m[k] = False
    assert (out["mv"][m] == 0).all() and (out["points"][m] == 0).all()


def test_pa_k_max_caps_recursion(orc):
    cur, ref = ramp_pair(3)
    a = one_mb_alpha()
    cls, _ = orc.classify(a)
    out = orc.pa(cur, ref, orc.Params(search_range=7, k_max=2), a, a, cls)
    assert out["iters"][1, 1] == 2
    assert tuple(out["mv_int"][1, 1]) == (4, 0)
    assert out["cost"][1, 1] == 256 * 3


def test_pa_half_eps_stalls_on_small_offsets(orc):
    # eps 0.5: one-pixel offset gives a 0.4999-pixel update -> no step
    cur, ref = ramp_pair(1)
    a = one_mb_alpha()
    cls, _ = orc.classify(a)
    out = orc.pa(cur, ref, orc.Params(search_range=7, eps_q12=2048), a, a, cls)
    assert out["iters"][1, 1] == 0 and tuple(out["mv_int"][1, 1]) == (0, 0)
    cur, ref = ramp_pair(3)
    out = orc.pa(cur, ref, orc.Params(search_range=7, eps_q12=2048), a, a, cls)
    # 3 -> step 1 (1.4996), then 2 -> step 1 (0.9998), then 1 -> 0: stop
    assert out["iters"][1, 1] == 2 and tuple(out["mv_int"][1, 1]) == (4, 0)


# --------------------------------------------------- proposed algorithm
def test_pa_identical_frames(orc):
    seq = synth.qcif_ellipse(frames=2)
    f = seq.luma[0]
    out = orc.pa(f, f, orc.Params(search_range=7))
    assert (out["mv"] == 0).all() and (out["cost"] == 0).all()
    assert (out["iters"] == 0).all() and (out["points"] == 1).all()


def crafted_candidates(case):
    """Frames where each MB before X = (1, 1) in raster order matches its
    temporal candidate exactly, so the neighbours' vectors are known, and
    X's block is placed so that two named candidates tie at SAD 0."""
    rng = np.random.default_rng(11)
    W = H = 96
    ref = rng.integers(0, 256, (H, W), dtype=np.uint8)
    wm = hm = W // 16
    vec = {}
    for v in range(hm):
        for h in range(wm):
            dx = int(np.clip(rng.integers(-4, 5), -16 * h, W - 16 - 16 * h))
            dy = int(np.clip(rng.integers(-4, 5), -16 * v, H - 16 - 16 * v))
            vec[(h, v)] = (dx, dy)
    a, b, c = vec[(0, 1)], vec[(1, 0)], vec[(2, 0)]
    t = (5, -5)
    X = (1, 1)
    x0 = y0 = 16

    def blk(ref, d):
        return ref[y0 + d[1]:y0 + d[1] + 16, x0 + d[0]:x0 + d[0] + 16]

    pair = {"AB": (a, b), "BC": (b, c), "CT": (c, t), "T": (t, None)}[case]
    src = blk(ref, pair[0]).copy()
    if pair[1] is not None:
        ref[y0 + pair[1][1]:y0 + pair[1][1] + 16, x0 + pair[1][0]:x0 + pair[1][0] + 16] = src
    cur = np.zeros_like(ref)
    tf = np.zeros((hm, wm, 2), np.int16)
    for (h, v), d in vec.items():
        dd = d if (h, v) != X else pair[0]
        cur[16 * v:16 * v + 16, 16 * h:16 * h + 16] = ref[16 * v + dd[1]:16 * v + dd[1] + 16,
                                                          16 * h + dd[0]:16 * h + dd[0] + 16]
        tf[v, h] = (2 * d[0], 2 * d[1])
    tf[1, 1] = (2 * t[0], 2 * t[1])
    return cur, ref, tf, {"A": a, "B": b, "C": c, "T": t}


@pytest.mark.parametrize("case,winner", [("AB", "A"), ("BC", "B"), ("CT", "C"), ("T", "T")])
def test_pa_candidate_order_first_minimum(orc, case, winner):
    cur, ref, tf, named = crafted_candidates(case)
    out = orc.pa(cur, ref, orc.Params(search_range=7), t_field=tf)
    # the MBs before X picked their exact temporal candidates
    assert tuple(out["mv_int"][0, 1]) == (2 * named["B"][0], 2 * named["B"][1])
    assert tuple(out["mv_int"][0, 2]) == (2 * named["C"][0], 2 * named["C"][1])
    assert tuple(out["mv_int"][1, 0]) == (2 * named["A"][0], 2 * named["A"][1])
    w = named[winner]
    assert tuple(out["mv_int"][1, 1]) == (2 * w[0], 2 * w[1])
    assert out["cost"][1, 1] == 0 and out["iters"][1, 1] == 0


def test_pa_translation_recovered_with_true_temporal(orc):
    rng = np.random.default_rng(5)
    big = synth.smoothed_noise(rng, 160, 208)
    d = (3, -2)
    ref = big[16:16 + 128, 16:16 + 176].copy()
    cur = big[16 + d[1]:16 + d[1] + 128, 16 + d[0]:16 + d[0] + 176].copy()
    tf = np.zeros((8, 11, 2), np.int16)
    tf[..., 0], tf[..., 1] = 2 * d[0], 2 * d[1]
    out = orc.pa(cur, ref, orc.Params(search_range=7), t_field=tf)
    wm, hm = 11, 8
    for v in range(hm):
        for h in range(wm):
            x0, y0 = 16 * h, 16 * v
            if 0 <= x0 + d[0] <= 176 - 16 and 0 <= y0 + d[1] <= 128 - 16:
                assert tuple(out["mv_int"][v, h]) == (2 * d[0], 2 * d[1])
                assert out["cost"][v, h] == 0 and out["iters"][v, h] == 0


def np_brs(cur, ref, mv_int, tf, cls, ca, ra, S, v, h):
    """Independent numpy restatement of the block-recursive stage of Fig. 1
    for MB (h, v): returns (list, first-minimum vector, its cost)."""
    hm, wm = mv_int.shape[:2]
    H, W = cur.shape
    x0, y0 = 16 * h, 16 * v
    z = np.zeros(2, np.int16)
    cands = [mv_int[v, h - 1] if h > 0 else z,
             mv_int[v - 1, h] if v > 0 else z,
             mv_int[v - 1, h + 1] if (v > 0 and h + 1 < wm) else z,
             tf[v, h] if tf is not None else z]
    lst = []
    for cnd in cands:
        d = (int(cnd[0]) // 2, int(cnd[1]) // 2)
        ok = abs(d[0]) <= S and abs(d[1]) <= S and 0 <= x0 + d[0] <= W - 16 and 0 <= y0 + d[1] <= H - 16
        if ok and d not in lst:
            lst.append(d)
    if not lst:
        lst = [(0, 0)]
    shape = cls is not None and cls[v, h] == 2
    costs = []
    for d in lst:
        if shape:
            a = ca[y0:y0 + 16, x0:x0 + 16] != 0
            b = ra[y0 + d[1]:y0 + d[1] + 16, x0 + d[0]:x0 + d[0] + 16] != 0
            costs.append(int(np.count_nonzero(a != b)))
        else:
            a = cur[y0:y0 + 16, x0:x0 + 16].astype(int)
            b = ref[y0 + d[1]:y0 + d[1] + 16, x0 + d[0]:x0 + d[0] + 16].astype(int)
            costs.append(int(np.abs(a - b).sum()))
    i = int(np.argmin(costs))   # numpy argmin: first minimum
    return lst, lst[i], costs[i]


def final_cost(cur, ref, ca, ra, shape, v, h, d):
    x0, y0 = 16 * h, 16 * v
    if shape:
        a = ca[y0:y0 + 16, x0:x0 + 16] != 0
        b = ra[y0 + d[1]:y0 + d[1] + 16, x0 + d[0]:x0 + d[0] + 16] != 0
        return int(np.count_nonzero(a != b))
    a = cur[y0:y0 + 16, x0:x0 + 16].astype(int)
    b = ref[y0 + d[1]:y0 + d[1] + 16, x0 + d[0]:x0 + d[0] + 16].astype(int)
    return int(np.abs(a - b).sum())


@pytest.mark.parametrize("shape_only", [False, True])
def test_pa_invariants_on_vop_sequence(orc, shape_only):
    seq = synth.qcif_ellipse(frames=5)
    p = orc.Params(search_range=7, k_max=8)
    res = orc.pa_sequence(seq, 0, p, shape_only=shape_only)
    tf = None
    for t, out in enumerate(res, start=1):
        cur, ref = seq.luma[t], seq.luma[t - 1]
        ca, ra = seq.alpha[0, t], seq.alpha[0, t - 1]
        cls = out["cls"]
        np.testing.assert_array_equal(cls, np_classes(ca)[0])
        hm, wm = cls.shape
        for v in range(hm):
            for h in range(wm):
                if cls[v, h] == 0:
                    assert (out["mv"][v, h] == 0).all() and out["points"][v, h] == 0
                    continue
                shape = shape_only or cls[v, h] == 2
                c2 = cls.copy()
                if shape_only:
                    c2[c2 == 1] = 2
                lst, d0, c0 = np_brs(cur, ref, out["mv_int"], tf, c2, ca, ra, 7, v, h)
                d = (int(out["mv_int"][v, h, 0]) // 2, int(out["mv_int"][v, h, 1]) // 2)
                assert out["mv_int"][v, h, 0] % 2 == 0 and out["mv_int"][v, h, 1] % 2 == 0
                assert abs(d[0]) <= 7 and abs(d[1]) <= 7
                assert 0 <= 16 * h + d[0] <= 176 - 16 and 0 <= 16 * v + d[1] <= 144 - 16
                c = int(out["cost"][v, h])
                assert c == final_cost(cur, ref, ca, ra, shape, v, h, d)
                it = int(out["iters"][v, h])
                assert it <= p.k_max
                assert out["points"][v, h] == len(lst) + it
                # iters counts every evaluated recursion candidate, the
                # rejected last one included: the cost never rises, an equal
                # cost means no move, and unit steps travel at most `it`
                assert c <= c0
                if it == 0 or c == c0:
                    assert d == d0 and c == c0
                assert max(abs(d[0] - d0[0]), abs(d[1] - d0[1])) <= it
        tf = out["mv_int"]


# ---------------------------------------------------------------- baselines
def np_es(cur, ref, S, x0, y0):
    H, W = cur.shape
    blk = cur[y0:y0 + 16, x0:x0 + 16].astype(int)
    best = None
    n = 0
    for dy in range(-S, S + 1):
        for dx in range(-S, S + 1):
            if not (0 <= x0 + dx <= W - 16 and 0 <= y0 + dy <= H - 16):
                continue
            n += 1
            s = int(np.abs(blk - ref[y0 + dy:y0 + dy + 16, x0 + dx:x0 + dx + 16].astype(int)).sum())
            key = (s, abs(dx) + abs(dy), dy, dx)
            best = key if best is None or key < best else best
    return best, n


def test_es_brute_force_tiny(orc):
    for seed in range(3):
        rng = np.random.default_rng(seed)
        cur = rng.integers(0, 256, (48, 48), dtype=np.uint8)
        ref = rng.integers(0, 256, (48, 48), dtype=np.uint8)
        # plant equal-cost ties: an exact copy at two offsets of one block
        ref[20:36, 19:35] = cur[16:32, 16:32]
        ref[14:30, 13:29] = cur[16:32, 16:32]
        out = orc.search(orc.ES, cur, ref, orc.Params(search_range=4))
        for v in range(3):
            for h in range(3):
                key, n = np_es(cur, ref, 4, 16 * h, 16 * v)
                assert out["cost"][v, h] == key[0]
                assert tuple(out["mv_int"][v, h]) == (2 * key[3], 2 * key[2])
                assert out["points"][v, h] == n
        # the second planted copy overwrites part of the first: only the
        # offset (-3, -2) still matches exactly
        assert tuple(out["mv"][1, 1]) == (-6, -4) and out["cost"][1, 1] == 0


def test_es_tie_break_by_l1_then_dy_then_dx(orc):
    rng = np.random.default_rng(9)
    cur = rng.integers(0, 256, (48, 48), dtype=np.uint8)
    ref = rng.integers(0, 256, (48, 48), dtype=np.uint8)
    src = cur[16:32, 16:32]
    for (dx, dy) in [(2, -1), (-1, 2), (1, -2), (-2, 1)]:   # all L1 3
        ref[16 + dy:32 + dy, 16 + dx:32 + dx] = src
    out = orc.search(orc.ES, cur, ref, orc.Params(search_range=4))
    # overlapping copies overwrite each other; recompute who still matches
    exact = [(dx, dy) for (dx, dy) in [(2, -1), (-1, 2), (1, -2), (-2, 1)]
             if (ref[16 + dy:32 + dy, 16 + dx:32 + dx] == src).all()]
    want = min(exact, key=lambda d: (abs(d[0]) + abs(d[1]), d[1], d[0]))
    assert tuple(out["mv_int"][1, 1]) == (2 * want[0], 2 * want[1])
    assert out["cost"][1, 1] == 0


@pytest.mark.parametrize("W,H,S,want", [(176, 144, 7, 18271 / 99), (352, 288, 16, 390028 / 396),
                                        (704, 576, 16, None)])
def test_es_points_closed_form(orc, W, H, S, want):
    def per_axis(n_mb, size):
        return sum(min(S, size - 16 - 16 * i) - max(-S, -16 * i) + 1 for i in range(n_mb))
    total = per_axis(W // 16, W) * per_axis(H // 16, H)
    mean = total / ((W // 16) * (H // 16))
    if want is not None:
        assert abs(mean - want) < 1e-9
    g = golden("es_points.json")["points_per_mb"]
    assert abs(mean - g[f"{W}x{H}_S{S}"]) < 5e-4
    if W * H <= 352 * 288:
        rng = np.random.default_rng(0)
        f = rng.integers(0, 256, (H, W), dtype=np.uint8)
        out = orc.search(orc.ES, f, f, orc.Params(search_range=S))
        assert int(out["points"].sum()) == total
        assert (out["mv"] == 0).all() and (out["cost"] == 0).all()


def test_es_1088_points_closed_form():
    g = golden("es_points.json")["points_per_mb"]
    S, W, H = 32, 1920, 1088

    def per_axis(n_mb, size):
        return sum(min(S, size - 16 - 16 * i) - max(-S, -16 * i) + 1 for i in range(n_mb))
    mean = per_axis(W // 16, W) * per_axis(H // 16, H) / ((W // 16) * (H // 16))
    assert abs(mean - g["1920x1088_S32"]) < 5e-4


def test_tss_ds_identical_frames_point_counts(orc):
    f = synth.qcif_ellipse(frames=1).luma[0]
    tss = orc.search(orc.TSS, f, f, orc.Params(search_range=7))
    ds = orc.search(orc.DS, f, f, orc.Params(search_range=7))
    assert (tss["mv"] == 0).all() and (ds["mv"] == 0).all()
    # interior MBs: 1 + 3 rounds x 8 = 25 (the paper's TSS bound at +-7);
    # diamond: 1 + 8 (large) + 4 (small) = 13
    assert (tss["points"][1:-1, 1:-1] == 25).all() and tss["points"].max() <= 25
    assert (ds["points"][1:-1, 1:-1] == 13).all() and ds["points"].max() <= 13


def bowl_pair(d, W=96, H=96):
    """A smooth paraboloid image: the SAD surface over offsets is unimodal
    with its minimum at the true shift d."""
    y, x = np.mgrid[0:H + 40, 0:W + 40].astype(np.float64)
    img = 20 + 0.02 * ((x - 68) ** 2 + (y - 68) ** 2)
    img = np.clip(img, 0, 255).astype(np.uint8)
    ref = img[20:20 + H, 20:20 + W].copy()
    cur = img[20 + d[1]:20 + d[1] + H, 20 + d[0]:20 + d[0] + W].copy()
    return cur, ref


@pytest.mark.parametrize("method,d", [(1, (1, 0)), (1, (0, -1)), (1, (-1, 1)), (1, (1, 1)),
                                      (2, (1, 0)), (2, (0, -1)), (2, (-1, 1)), (2, (1, 1)),
                                      (2, (3, -2)), (2, (-3, 1)), (2, (2, 2))])
def test_tss_ds_recover_smooth_translation(orc, method, d):
    # both recover one-pixel shifts of a smooth image; the diamond descent
    # also walks the unimodal bowl to larger shifts (three-step search may
    # legitimately pick a wrong quadrant on its coarse first step)
    cur, ref = bowl_pair(d)
    out = orc.search(method, cur, ref, orc.Params(search_range=7))
    es = orc.search(orc.ES, cur, ref, orc.Params(search_range=7))
    # centre MBs of the bowl: the global minimum is the true shift
    for (v, h) in [(2, 2), (2, 3), (3, 2), (3, 3)]:
        assert tuple(es["mv_int"][v, h]) == (2 * d[0], 2 * d[1])
        assert tuple(out["mv_int"][v, h]) == (2 * d[0], 2 * d[1]), (v, h)
        assert out["cost"][v, h] == 0


def test_tss_step_sizes_and_bound(orc):
    # S = 16: steps 16, 8, 4, 2, 1 -> at most 1 + 5 * 8 = 41 points
    f = synth.cif_two_vops(frames=2).luma
    out = orc.search(orc.TSS, f[1], f[0], orc.Params(search_range=16))
    assert out["points"].max() <= 41
    assert (orc.search(orc.TSS, f[0], f[0], orc.Params(search_range=16))["points"][2:-2, 2:-2] == 41).all()


def test_fss_identical_frames_point_counts(orc):
    # four-step search [6] on identical frames: the centre wins the first
    # 5 x 5 square at once, then the 3 x 3 square: 1 + 8 + 8 = 17 points
    for S in (7, 16):
        f = synth.qcif_ellipse(frames=1).luma[0]
        out = orc.search(orc.FSS, f, f, orc.Params(search_range=S))
        assert (out["mv"] == 0).all() and (out["cost"] == 0).all()
        assert (out["points"][2:-2, 2:-2] == 17).all() and out["points"].max() <= 17


def stripe_pair(d, axis, W=128, H=96):
    """cur = ref shifted by d on a ramp along one axis (ref = 20 + x, or
    20 + y): the SAD of a candidate is 256 |d - d'| along that axis and does
    not depend on the other, so every search move is decided by the
    row-order tie rule across the other axis."""
    y, x = np.mgrid[0:H, 0:W]
    if axis == 0:
        return (20 + x + d).astype(np.uint8), (20 + x).astype(np.uint8)
    return (20 + y + d).astype(np.uint8), (20 + y).astype(np.uint8)


# (S, axis, shift, final vector, points), worked by hand from the four-step
# rules: a square whose best column (row) lies 2 away moves to the first
# point of that column (row) in row order, i.e. a corner: 5 new points; a tie
# with the centre keeps it; the step-1 square adds 8 new points.
@pytest.mark.parametrize("S,axis,shift,final,pts", [
    (7, 0, 6, (6, -6), 9 + 5 + 5 + 8),     # three corner moves up-right, centre column wins the 3x3
    (7, 0, -3, (-3, -3), 9 + 5 + 8),       # one corner move, tie keeps the centre, 3x3 picks (-3, -3)
    (7, 1, 6, (-6, 6), 9 + 5 + 5 + 8),     # ties across x go to the first (leftmost) column
    (7, 0, 1, (1, -1), 9 + 8),             # centre wins the first square
    (16, 0, 11, (11, -11), 9 + 4 * 5 + 5 + 8),  # five moves: more than the textbook's three squares
])
def test_fss_stripe_closed_form(orc, S, axis, shift, final, pts):
    cur, ref = stripe_pair(shift, axis)
    out = orc.search(orc.FSS, cur, ref, orc.Params(search_range=S))
    for v in (1, 2, 3):
        for h in range(1, 6):
            assert tuple(out["mv_int"][v, h]) == (2 * final[0], 2 * final[1]), (v, h, out["mv_int"][v, h])
            assert out["cost"][v, h] == 0
            assert out["points"][v, h] == pts, (v, h, out["points"][v, h])


def test_fss_bound_at_s7(orc):
    # at most 9 + 5 + 5 + 8 = 27 distinct points per MB at +-7
    f = synth.qcif_ellipse(frames=3).luma
    for t in (1, 2):
        assert orc.search(orc.FSS, f[t], f[t - 1], orc.Params(search_range=7))["points"].max() <= 27


# ----------------------------------------------------------- half-sample
def test_half_pel_constant_image_keeps_integer_vector(orc):
    f = np.full((64, 64), 77, np.uint8)
    a = one_mb_alpha()
    cls, _ = orc.classify(a)
    out = orc.pa(f, f, orc.Params(search_range=7, half_pel=1), a, a, cls)
    assert tuple(out["mv"][1, 1]) == (0, 0) and out["cost"][1, 1] == 0
    assert out["points"][1, 1] == 1 + 8


def test_half_pel_ramp_closed_form(orc):
    # ref(x) = 2x, cur(x) = 2x + 1 = ref(x + 1/2).  The integer stage stays
    # at 0 (|g| = 4 < 2 theta); among the half-sample offsets (1,-1) is the
    # first with SAD 0: (4 * (2x) + 4 + 2) >> 2 = 2x + 1.
    x = np.arange(64)
    ref = np.tile((2 * x).astype(np.uint8), (64, 1))
    cur = np.tile((2 * x + 1).astype(np.uint8), (64, 1))
    a = one_mb_alpha()
    cls, _ = orc.classify(a)
    out = orc.pa(cur, ref, orc.Params(search_range=7, half_pel=1), a, a, cls)
    assert tuple(out["mv"][1, 1]) == (1, -1) and out["cost"][1, 1] == 0
    assert tuple(out["mv_int"][1, 1]) == (0, 0)
    assert orc.sad_half(cur, ref, 16, 16, 1, 0) == 0
    assert orc.sad_half(cur, ref, 16, 16, 0, 0) == 256
    assert orc.sad_half(cur, ref, 16, 16, -1, -1) == 512   # (8x - 2) >> 2 = 2x - 1


def np_pred_half(ref, x0, y0, hx, hy):
    ix, iy = hx // 2, hy // 2
    fx, fy = hx - 2 * ix, hy - 2 * iy
    r = ref.astype(int)
    A = r[y0 + iy:y0 + iy + 16, x0 + ix:x0 + ix + 16]
    B = r[y0 + iy:y0 + iy + 16, x0 + ix + 1:x0 + ix + 17]
    Cc = r[y0 + iy + 1:y0 + iy + 17, x0 + ix:x0 + ix + 16]
    D = r[y0 + iy + 1:y0 + iy + 17, x0 + ix + 1:x0 + ix + 17]
    if fx and fy:
        return (A + B + Cc + D + 2) >> 2
    if fx:
        return (A + B + 1) >> 1
    if fy:
        return (A + Cc + 1) >> 1
    return A


def test_mc_sse_vs_numpy_with_half_pel(orc):
    rng = np.random.default_rng(4)
    cur = rng.integers(0, 256, (64, 80), dtype=np.uint8)
    ref = rng.integers(0, 256, (64, 80), dtype=np.uint8)
    ca = np.where(rng.random((64, 80)) < 0.7, 255, 0).astype(np.uint8)
    cls, _ = orc.classify(ca)
    mv = rng.integers(-6, 7, size=(4, 5, 2)).astype(np.int16)
    # keep every footprint in frame for the numpy restatement
    for v in range(4):
        for h in range(5):
            for ax, (lo, hi) in enumerate([(-16 * h, 80 - 17 - 16 * h), (-16 * v, 64 - 17 - 16 * v)]):
                mv[v, h, ax] = np.clip(mv[v, h, ax], 2 * lo, 2 * hi)
    sse, n, pred = orc.mc_sse(cur, ref, mv, ca, cls, want_pred=True)
    want_sse, want_n = 0, 0
    for v in range(4):
        for h in range(5):
            m = mv[v, h] if cls[v, h] != 0 else (0, 0)
            pr = np_pred_half(ref, 16 * h, 16 * v, int(m[0]), int(m[1]))
            np.testing.assert_array_equal(pred[16 * v:16 * v + 16, 16 * h:16 * h + 16], pr)
            msk = ca[16 * v:16 * v + 16, 16 * h:16 * h + 16] != 0
            dd = cur[16 * v:16 * v + 16, 16 * h:16 * h + 16].astype(np.int64) - pr
            want_sse += int((dd[msk] ** 2).sum())
            want_n += int(msk.sum())
    assert (sse, n) == (want_sse, want_n)


@pytest.mark.parametrize("c", [1, 3, 17])
def test_psnr_constant_offset(orc, c):
    ref = np.full((32, 48), 100, np.uint8)
    cur = ref + np.uint8(c)
    sse, n, _ = orc.mc_sse(cur, ref, np.zeros((2, 3, 2), np.int16))
    assert (sse, n) == (c * c * 32 * 48, 32 * 48)
    assert abs(orc.psnr_db(sse, n) - 20 * math.log10(255 / c)) < 1e-9
    assert orc.psnr_db(0, n) == float("inf")


# ------------------------------------------------------- learned-seed start
def translated_pair(d, H=128, W=176, seed=5):
    rng = np.random.default_rng(seed)
    big = synth.smoothed_noise(rng, H + 32, W + 32)
    ref = big[16:16 + H, 16:16 + W].copy()
    cur = big[16 + d[1]:16 + d[1] + H, 16 + d[0]:16 + d[0] + W].copy()
    return cur, ref


def test_pa_true_seed_is_taken(orc):
    """A seed at the true translation costs 0: the seeded start is kept (no
    fallback), the vector is exact, and the seed adds one compared block."""
    d = (5, -4)
    cur, ref = translated_pair(d)
    seed = np.zeros((8, 11, 2), np.int16)
    seed[..., 0], seed[..., 1] = 2 * d[0], 2 * d[1]
    p = orc.Params(search_range=7)
    plain = orc.pa(cur, ref, p)
    got = orc.pa(cur, ref, p, seed=seed)
    for v in range(8):
        for h in range(11):
            x0, y0 = 16 * h, 16 * v
            if 0 <= x0 + d[0] <= 176 - 16 and 0 <= y0 + d[1] <= 128 - 16:
                assert tuple(got["mv_int"][v, h]) == (2 * d[0], 2 * d[1]) and got["cost"][v, h] == 0
                assert got["cost"][v, h] <= plain["cost"][v, h]
                # the BRS list of this run's own neighbours, plus the seed;
                # the seed's recursion stops at once (cost 0)
                lst, _, _ = np_brs(cur, ref, got["mv_int"], None, None, None, None, 7, v, h)
                assert got["points"][v, h] == len(lst) + 1 and got["iters"][v, h] == 0


def test_pa_bad_seed_falls_back_to_plain(orc):
    """Identical frames: the BRS minimum is 0 at (0, 0), so any seed with a
    positive cost fails the 5 % test and the plain result stands."""
    seq = synth.qcif_ellipse(frames=2)
    f = seq.luma[0]
    seed = np.full((9, 11, 2), 2 * 6, np.int16)
    out = orc.pa(f, f, orc.Params(search_range=7), seed=seed)
    assert (out["mv"] == 0).all() and (out["cost"] == 0).all()
    assert (out["points"] >= 2).all()


@pytest.mark.parametrize("k_max,its,pts", [(5, 5 + 3, 1 + 1 + 5 + 3), (127, 10, 1 + 1 + 10)])
def test_pa_seed_iteration_count_closed_form(orc, k_max, its, pts):
    """Ramp ref = 20 + 3x, cur displaced by +3, one opaque MB at (16, 16),
    S 7.  The block-recursive list is the single zero vector (SAD 9 * 256).
    A seed at -7 walks one pixel per recursion step toward +3.  With k_max 5
    it stops at -2 (SAD 15 * 256): 20 * 3840 > 21 * 2304, so the seed is
    dropped and the plain recursion from 0 takes 3 more steps; iterations
    count both recursions and points add the seed.  With k_max 127 the seed
    reaches +3 in 10 steps with SAD 0 and is kept."""
    cur, ref = ramp_pair(3)
    a = one_mb_alpha()
    cls, _ = orc.classify(a)
    seed = np.zeros((4, 4, 2), np.int16)
    seed[1, 1] = (-14, 0)
    out = orc.pa(cur, ref, orc.Params(search_range=7, k_max=k_max), a, a, cls, seed=seed)
    assert tuple(out["mv_int"][1, 1]) == (6, 0) and out["cost"][1, 1] == 0
    assert out["iters"][1, 1] == its and out["points"][1, 1] == pts


def test_pa_seeded_k_max_above_127_rejected(orc):
    cur, ref = ramp_pair(3)
    a = one_mb_alpha()
    cls, _ = orc.classify(a)
    seed = np.zeros((4, 4, 2), np.int16)
    with pytest.raises(ValueError):
        orc.pa(cur, ref, orc.Params(search_range=7, k_max=128), a, a, cls, seed=seed)
    orc.pa(cur, ref, orc.Params(search_range=7, k_max=255), a, a, cls)   # plain: the full range
