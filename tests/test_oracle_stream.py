"""Pins of the oracle's bitstream, DEFLATE pass and compression rate (Section
2.3 step (iii) and decoder step (i); Section 3's CR)."""
import struct
import zlib

import numpy as np

from oracle import aqmp_oracle as O
from workloads import piecewise_image


def _node(x0, y0, n, idx, coef, split):
    return O.Node(x0, y0, n, O.MPResult(idx=list(idx), coef=list(coef)), split, 0.0, 0.0)


def test_stream_bytes_of_a_hand_built_tree():
    """Golden bytes: a 16 x 16 plane, N 8..16, one channel.  The top block is
    split; its children are leaves with 1, 0, 2 and 1 atoms."""
    nodes = [_node(0, 0, 16, [5], [0.5], True),
             _node(0, 0, 8, [3], [1.0], False), _node(8, 0, 8, [], [], False),
             _node(0, 8, 8, [7, 130], [-2.0, 0.25], False), _node(8, 8, 8, [0], [4.0], False)]
    raw = O.pack_stream([nodes], 16, 16, 8, 16)
    want = (b"AQMP" + bytes([1, 3, 0, 1]) + struct.pack("<II", 16, 16) + bytes([3, 4, 1, 0])
            + struct.pack("<III", 5, 4, 4) + bytes([0b1])            # one split flag (the 16 x 16 node)
            + bytes([1, 0, 2, 1])                                     # atom counts of the leaves
            + struct.pack("<4H", 3, 7, 130, 0)
            + struct.pack("<4f", 1.0, -2.0, 0.25, 4.0))
    assert raw == want
    back = O.unpack_stream(raw)
    assert back["channels"][0] == [(0, 0, 8, [3], [1.0]), (8, 0, 8, [], []), (0, 8, 8, [7, 130], [-2.0, 0.25]),
                                   (8, 8, 8, [0], [4.0])]


def test_stream_round_trip_of_an_encode():
    img = piecewise_image(96, 80, seed=3)         # not a multiple of N_max: padded plane
    p = O.Params(tol=0.02, max_atoms=12, n_min=4, n_max=32)
    chans = [O.encode_channel(img, p), O.encode_channel(img.T.copy()[:80, :96], p)]
    raw = O.pack_stream(chans, 80, 96, 4, 32)
    back = O.unpack_stream(raw)
    assert (back["w"], back["h"], back["n_min"], back["n_max"]) == (80, 96, 4, 32)
    for nodes, got in zip(chans, back["channels"]):
        lv = O.leaves(nodes)
        assert [(nd.x0, nd.y0, nd.n, nd.mp.idx) for nd in lv] == [(g[0], g[1], g[2], g[3]) for g in got]
        for nd, g in zip(lv, got):
            assert np.array_equal(np.array(nd.mp.coef, dtype=np.float32).astype(np.float64), np.array(g[4]))
    z = O.compress_stream(raw)
    assert zlib.decompress(z) == raw and len(z) < len(raw)
    cr = O.compression_rate(len(z), 80, 96, 2)
    assert abs(cr - 80 * 96 * 2 / len(z)) < 1e-12


def test_counts_above_255_use_two_bytes():
    nodes = [_node(0, 0, 4, list(range(300)), [0.0] * 300, False)]
    raw = O.pack_stream([nodes], 4, 4, 4, 4)
    assert raw[18] == 2
    assert O.unpack_stream(raw)["channels"][0][0][3] == list(range(300))
