"""Pins of the oracle's coefficient quantiser and of stream coefficient format
1 (uniform quantiser; the paper's encoder step (ii) is lossy and names no
quantiser, so this is a stated reading).  Hand-worked values in
tests/golden/quant_cases.txt, golden bytes of a hand-built tree, the
reconstruction error bound, and planted mistakes."""
import os
import struct

import numpy as np
import pytest

from oracle import aqmp_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cases():
    out = []
    with open(os.path.join(GOLDEN, "quant_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                c, st, q, _ = [v.strip() for v in line.split("|")]
                out.append((float(c), float(st), int(q)))
    return out


def pin_quant(fn=None) -> bool:
    fn = fn or O.quantize
    return all(int(fn([c], st)[0]) == q for c, st, q in _cases())


def _node(x0, y0, n, idx, coef, split):
    return O.Node(x0, y0, n, O.MPResult(idx=list(idx), coef=list(coef)), split, 0.0, 0.0)


def _tree():
    return [_node(0, 0, 16, [5], [0.5], True),
            _node(0, 0, 8, [3], [1.0], False), _node(8, 0, 8, [], [], False),
            _node(0, 8, 8, [7, 130], [-2.0, 0.25], False), _node(8, 8, 8, [0], [4.0], False)]


def test_quantiser_hand_values():
    assert len(_cases()) >= 9
    assert pin_quant()


def test_format1_bytes_of_a_hand_built_tree():
    """Step 0.5: coefficients 1, -2, 0.25, 4 of the leaves -> q = 2, -4, 0 (0.5
    is a tie, even neighbour 0), 8, as int16; the step 0.5 as binary32 after
    the 20-byte header; the header's last byte gives the integer width."""
    raw = O.pack_stream([_tree()], 16, 16, 8, 16, step=0.5)
    want = (b"AQMP" + bytes([1, 3, 1, 1]) + struct.pack("<II", 16, 16) + bytes([3, 4, 1, 2])
            + struct.pack("<f", 0.5)
            + struct.pack("<III", 5, 4, 4) + bytes([0b1]) + bytes([1, 0, 2, 1])
            + struct.pack("<4H", 3, 7, 130, 0)
            + struct.pack("<4h", 2, -4, 0, 8))
    assert raw == want
    back = O.unpack_stream(raw)
    assert back["step"] == 0.5
    assert back["channels"][0] == [(0, 0, 8, [3], [1.0]), (8, 0, 8, [], []), (0, 8, 8, [7, 130], [-2.0, 0.0]),
                                   (8, 8, 8, [0], [4.0])]


def test_wide_values_use_four_bytes():
    nodes = [_node(0, 0, 4, [1, 2], [40000.0, -1.0], False)]
    raw = O.pack_stream([nodes], 4, 4, 4, 4, step=1.0)
    assert raw[19] == 4
    assert O.unpack_stream(raw)["channels"][0][0][4] == [40000.0, -1.0]


def test_reconstruction_error_is_at_most_half_a_step():
    rng = np.random.default_rng(3)
    c = rng.normal(scale=5.0, size=10000)
    for st in (0.01, 0.1, 0.37, 2.0):
        d = float(np.float32(st))
        err = np.abs(c - O.dequantize(O.quantize(c, st), st))
        assert err.max() <= d / 2 * (1 + 1e-12)


def test_rejects_a_non_positive_step():
    with pytest.raises(ValueError):
        O.quantize([1.0], 0.0)


@pytest.mark.parametrize("bad", [
    lambda c, st: np.floor(np.asarray(c) / float(np.float32(st)) + 0.5).astype(np.int64),   # planted: ties away upward
    lambda c, st: np.trunc(np.asarray(c) / float(np.float32(st))).astype(np.int64),         # planted: truncation
    lambda c, st: np.rint(np.asarray(c) / float(st)).astype(np.int64),                      # planted: step not rounded to binary32
    lambda c, st: np.rint(np.asarray(c) * float(np.float32(st))).astype(np.int64),          # planted: multiplies by the step
])
def test_planted_quantiser_mistakes_caught(bad):
    assert not pin_quant(bad)
