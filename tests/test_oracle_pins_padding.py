"""Pins of the oracle's MPEG-4 reference VOP padding (Section 4 protocol: the
reference is an MPEG-4 VOP; boundary MBs take repetitive padding, transparent
MBs extended padding).  Each case is a closed form written from the
definition, independent of the oracle's loops: a one-sided row or column is a
copy of its nearest inside sample, a gap between two inside samples is their
rounded-up mean, rows with no inside sample take the column rule, and a
transparent MB copies the border of its first non-transparent neighbour in
the order left, above, right, below, else 128."""
import numpy as np
import pytest

import oracle


def rnd(shape, seed):
    return np.random.default_rng(seed).integers(0, 256, shape, dtype=np.uint8)


def test_opaque_is_copied():
    lu = rnd((32, 48), 1)
    assert np.array_equal(oracle.pad_vop(lu, np.full(lu.shape, 255, np.uint8)), lu)


def test_transparent_everywhere_is_128():
    lu = rnd((32, 32), 2)
    assert (oracle.pad_vop(lu, np.zeros(lu.shape, np.uint8)) == 128).all()


def test_single_inside_column_fills_each_row():
    lu = rnd((16, 16), 3)
    al = np.zeros((16, 16), np.uint8)
    al[:, 5] = 1
    want = np.repeat(lu[:, 5:6], 16, axis=1)
    assert np.array_equal(oracle.pad_vop(lu, al), want)


def test_gap_between_two_columns_is_their_rounded_up_mean():
    lu = rnd((16, 16), 4)
    al = np.zeros((16, 16), np.uint8)
    al[:, 2] = al[:, 9] = 7
    a, b = lu[:, 2].astype(int), lu[:, 9].astype(int)
    want = np.empty((16, 16), int)
    want[:, :3] = a[:, None]
    want[:, 3:9] = ((a + b + 1) // 2)[:, None]
    want[:, 9:] = b[:, None]
    assert np.array_equal(oracle.pad_vop(lu, al), want.astype(np.uint8))


def test_single_inside_row_fills_each_column():
    lu = rnd((16, 16), 5)
    al = np.zeros((16, 16), np.uint8)
    al[3, :] = 1
    want = np.repeat(lu[3:4, :], 16, axis=0)
    assert np.array_equal(oracle.pad_vop(lu, al), want)


def test_open_rows_between_two_rows_take_the_column_mean():
    lu = rnd((16, 16), 6)
    al = np.zeros((16, 16), np.uint8)
    al[2, :] = al[10, :] = 1
    a, b = lu[2].astype(int), lu[10].astype(int)
    want = np.empty((16, 16), int)
    want[:3] = a
    want[3:10] = (a + b + 1) // 2
    want[10:] = b
    assert np.array_equal(oracle.pad_vop(lu, al), want.astype(np.uint8))


def test_one_inside_pixel_fills_the_block():
    lu = rnd((16, 16), 7)
    al = np.zeros((16, 16), np.uint8)
    al[4, 7] = 1
    assert (oracle.pad_vop(lu, al) == lu[4, 7]).all()


def test_rows_first_then_columns():
    """Inside: row 3 at columns 0 and 15, and pixel (12, 6).  Row 3 becomes
    the mean of its two ends between them; row 12 becomes its single pixel;
    the open rows then take the column rule over rows 3 and 12."""
    lu = rnd((16, 16), 8)
    al = np.zeros((16, 16), np.uint8)
    al[3, 0] = al[3, 15] = al[12, 6] = 1
    r3 = np.full(16, (int(lu[3, 0]) + int(lu[3, 15]) + 1) // 2)
    r3[0], r3[15] = lu[3, 0], lu[3, 15]
    r12 = np.full(16, int(lu[12, 6]))
    want = np.empty((16, 16), int)
    want[:4] = r3
    want[4:12] = (r3 + r12 + 1) // 2
    want[12:] = r12
    assert np.array_equal(oracle.pad_vop(lu, al), want.astype(np.uint8))


def test_outside_texture_is_never_read():
    lu = rnd((48, 48), 9)
    al = (rnd((48, 48), 10) > 200).astype(np.uint8)
    al[16:32, 16:32] = 0
    al[20, 20] = 1
    lu2 = lu.copy()
    lu2[al == 0] = 255 - lu2[al == 0]
    assert np.array_equal(oracle.pad_vop(lu, al), oracle.pad_vop(lu2, al))


def test_extended_padding_takes_the_left_or_right_neighbour():
    """Three MBs in a row, the middle one boundary (inside: its column 0 and
    column 15): the left MB repeats the middle one's first column, the right
    MB its last column."""
    lu = rnd((16, 48), 11)
    al = np.zeros((16, 48), np.uint8)
    al[:, 16] = al[:, 31] = 1
    out = oracle.pad_vop(lu, al)
    assert np.array_equal(out[:, :16], np.repeat(lu[:, 16:17], 16, axis=1))
    assert np.array_equal(out[:, 32:], np.repeat(lu[:, 31:32], 16, axis=1))


def test_extended_padding_priority():
    """2 x 2 MBs.  MB (0,0) and MB (1,1) transparent, (1,0) and (0,1) opaque.
    MB (0,0): no left or upper MB, so its right neighbour (1,0) wins over
    the lower one (0,1).  MB (1,1): its left neighbour (0,1) wins over the
    upper one (1,0)."""
    lu = rnd((32, 32), 12)
    al = np.zeros((32, 32), np.uint8)
    al[0:16, 16:32] = 1
    al[16:32, 0:16] = 1
    out = oracle.pad_vop(lu, al)
    assert np.array_equal(out[0:16, 0:16], np.repeat(lu[0:16, 16:17], 16, axis=1))
    assert np.array_equal(out[16:32, 16:32], np.repeat(lu[16:32, 15:16], 16, axis=1))


def test_extended_padding_from_above_and_below():
    """A column of three MBs, the middle one opaque: the top MB repeats its
    first row (lower neighbour), the bottom MB its last row (upper
    neighbour)."""
    lu = rnd((48, 16), 13)
    al = np.zeros((48, 16), np.uint8)
    al[16:32, :] = 1
    out = oracle.pad_vop(lu, al)
    assert np.array_equal(out[:16], np.repeat(lu[16:17], 16, axis=0))
    assert np.array_equal(out[32:], np.repeat(lu[31:32], 16, axis=0))


def test_mb_without_a_padded_neighbour_is_128():
    """3 x 3 MBs with only the centre MB inside: the four edge-adjacent MBs
    copy its border, the four corners (diagonal only) take 128."""
    lu = rnd((48, 48), 14)
    al = np.zeros((48, 48), np.uint8)
    al[16:32, 16:32] = 1
    out = oracle.pad_vop(lu, al)
    for y, x in ((0, 0), (0, 32), (32, 0), (32, 32)):
        assert (out[y:y + 16, x:x + 16] == 128).all()
    assert np.array_equal(out[16:32, 0:16], np.repeat(lu[16:32, 16:17], 16, axis=1))
    assert np.array_equal(out[0:16, 16:32], np.repeat(lu[16:17, 16:32], 16, axis=0))
    assert np.array_equal(out[16:32, 32:48], np.repeat(lu[16:32, 31:32], 16, axis=1))
    assert np.array_equal(out[32:48, 16:32], np.repeat(lu[31:32, 16:32], 16, axis=0))


def test_extended_padding_reads_the_padded_boundary_mb():
    """The left neighbour is a boundary MB with one inside pixel: its
    repetitive padding makes it constant, and the transparent MB to its
    right copies that constant."""
    lu = rnd((16, 32), 15)
    al = np.zeros((16, 32), np.uint8)
    al[9, 4] = 1
    out = oracle.pad_vop(lu, al)
    assert (out == lu[9, 4]).all()


@pytest.mark.parametrize("bad", [dict(W=24), dict(H=8)])
def test_rejects_frames_off_the_mb_grid(bad):
    H, W = bad.get("H", 16), bad.get("W", 16)
    with pytest.raises(ValueError):
        oracle.pad_vop(np.zeros((H, W), np.uint8), np.zeros((H, W), np.uint8))
