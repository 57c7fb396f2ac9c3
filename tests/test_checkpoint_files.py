"""The committed network checkpoints parse as the library's checkpoint format
(magic, version, parameter count, window scale, fp32 weights and momentum,
FNV-1a 64 checksum over everything before it), read with plain Python - no
GPU, nothing executed from the file."""
import json
import os
import struct

import numpy as np
import pytest

import paper_1002_1168_amd as me

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1002_1168_amd",
                       "weights")


def fnv1a64(data: bytes) -> int:
    h = 0xCBF29CE484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def parse(path):
    raw = open(path, "rb").read()
    assert raw[:8] == b"ME-NET\0\0"
    version, nparams, scale, zero = struct.unpack_from("<4I", raw, 8)
    assert (version, nparams, zero) == (1, me.ME_NET_PARAMS, 0)
    assert len(raw) == 24 + 8 * nparams + 8
    (check,) = struct.unpack_from("<Q", raw, len(raw) - 8)
    assert check == fnv1a64(raw[:-8])
    w = np.frombuffer(raw, dtype="<f4", count=nparams, offset=24)
    v = np.frombuffer(raw, dtype="<f4", count=nparams, offset=24 + 4 * nparams)
    return scale, w, v


@pytest.mark.parametrize("name", ["proposal_hd_s32"])
def test_committed_checkpoint_is_well_formed(name):
    scale, w, v = parse(os.path.join(WEIGHTS, name + ".menet"))
    rec = json.load(open(os.path.join(WEIGHTS, name + ".json")))
    assert scale == rec["window_scale"] == 4 and rec["search_range"] == 32 and rec["half_pel"] == 1
    assert np.isfinite(w).all() and np.isfinite(v).all() and np.abs(w).max() > 0
