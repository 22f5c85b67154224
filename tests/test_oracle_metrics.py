"""Pins of the oracle's PSNR and compression rate against hand-worked values.

``tests/golden/psnr_cases.txt``: planes with hand-computed MSE and PSNR (the
textbook PSNR; the paper reports quality in SSIM).  ``tests/golden/cr_cases.txt``:
streams whose byte counts are worked out by hand from the v1 layout, and the
compression rate of Section 3 (bytes of the 8-bit original over bytes of the
compressed file).  Planted mistakes in either function must fail a pin.
"""
import math
import os

import numpy as np
import pytest

from oracle import aqmp_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _samples(text: str) -> list[float]:
    out = []
    for tok in text.split():
        if "*" in tok:
            v, n = tok.split("*")
            out += [float(v)] * int(n)
        else:
            out.append(float(tok))
    return out


def _cases(name: str) -> list[list[str]]:
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([c.strip() for c in line.split("|")])
    return rows


def psnr_cases():
    out = []
    for name, shape, ref, rec, peak, want in _cases("psnr_cases.txt"):
        r, c = (int(v) for v in shape.split())
        a = np.array(_samples(ref)).reshape(r, c)
        b = np.array(_samples(rec)).reshape(r, c)
        out.append((name, a, b, float(peak), float(want)))
    return out


def pin_psnr(fn=None) -> bool:
    fn = fn or O.psnr
    for name, a, b, peak, want in psnr_cases():
        got = fn(a, b, peak=peak)
        if math.isinf(want):
            if not math.isinf(got):
                return False
        elif not abs(got - want) <= 1e-12 * max(1.0, abs(want)):
            return False
    return True


def _node(x0, y0, n, k, split):
    idx = list(range(1, k + 1))
    return O.Node(x0, y0, n, O.MPResult(idx=idx, coef=[0.5] * k), split, 0.0, 0.0)


def cr_trees() -> dict:
    leaf2 = [_node(0, 0, 64, 2, False)]
    split = [_node(0, 0, 64, 3, True), _node(0, 0, 32, 1, False), _node(32, 0, 32, 0, False),
             _node(0, 32, 32, 3, False), _node(32, 32, 32, 2, False)]
    return {"single_leaf": [leaf2], "three_channels": [leaf2, leaf2, leaf2], "split_tree": [split]}


def pin_cr(fn=None) -> bool:
    fn = fn or O.compression_rate
    trees = cr_trees()
    for name, dims, size, want in _cases("cr_cases.txt"):
        w, h, ch = (int(v) for v in dims.split())
        raw = O.pack_stream(trees[name], w, h, 32, 64)
        if len(raw) != int(size):            # the hand count of the stream layout
            return False
        got = fn(len(raw), w, h, ch)
        if not abs(got - float(want)) <= 1e-12 * float(want):
            return False
    return True


def test_psnr_hand_values():
    assert len(psnr_cases()) >= 6
    assert pin_psnr()


def test_psnr_does_not_clip_and_is_symmetric():
    # the reconstruction is not clipped to [0, peak]: a sample at -0.1
    # against 0 costs the same as one at +0.1
    a = np.zeros((2, 5))
    b = a.copy()
    b[0, 0] = -0.1
    c = a.copy()
    c[0, 0] = 0.1
    assert O.psnr(a, b) == O.psnr(a, c) == O.psnr(b, a)
    # MSE 0.01 / 10 = 0.001 -> 30 dB, worked out by hand
    assert abs(O.psnr(a, b) - 30.0) < 1e-12


def test_compression_rate_hand_sized_streams():
    assert pin_cr()


# -- planted mistakes -------------------------------------------------------

def _bad_psnr_unsquared_peak(ref, rec, peak=1.0):
    d = np.asarray(ref, float) - np.asarray(rec, float)
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else 10 * np.log10(peak / mse)      # planted: peak not squared


def _bad_psnr_sum(ref, rec, peak=1.0):
    d = np.asarray(ref, float) - np.asarray(rec, float)
    mse = float(np.sum(d * d))                                          # planted: sum, not mean
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)


def _bad_psnr_row_mean(ref, rec, peak=1.0):
    d = np.asarray(ref, float) - np.asarray(rec, float)
    mse = float(np.mean(np.sum(d * d, axis=0)))                        # planted: mean over one axis only
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)


def _bad_psnr_20log(ref, rec, peak=1.0):
    d = np.asarray(ref, float) - np.asarray(rec, float)
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else 20 * np.log10(peak * peak / mse)   # planted: 20 log10 of a power ratio


def _bad_psnr_clipped(ref, rec, peak=1.0):
    rec = np.clip(np.asarray(rec, float), 0.0, peak)                   # planted: clips the reconstruction
    d = np.asarray(ref, float) - rec
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else 10 * np.log10(peak * peak / mse)


@pytest.mark.parametrize("bad", [_bad_psnr_unsquared_peak, _bad_psnr_sum, _bad_psnr_row_mean, _bad_psnr_20log])
def test_planted_psnr_mistakes_caught(bad):
    assert not pin_psnr(bad)


def test_planted_psnr_clipping_caught(monkeypatch):
    monkeypatch.setattr(O, "psnr", _bad_psnr_clipped)
    with pytest.raises(AssertionError):
        test_psnr_does_not_clip_and_is_symmetric()


@pytest.mark.parametrize("bad", [
    lambda size, w, h, ch: float(w * h) / float(size),                # planted: channels ignored
    lambda size, w, h, ch: float(w * h * ch * 8) / float(size),       # planted: original counted in bits
    lambda size, w, h, ch: float(size) / float(w * h * ch),           # planted: inverted ratio
    lambda size, w, h, ch: float(w * h * ch * 4) / float(size),       # planted: original as binary32 samples
])
def test_planted_cr_mistakes_caught(bad):
    assert not pin_cr(bad)


def test_planted_stream_size_mistake_caught(monkeypatch):
    orig = O.pack_stream

    def bad_pack(*a, **k):          # planted: the coefficients written as binary64
        raw = orig(*a, **k)
        return raw + bytes(4 * sum(nd.mp.t for nodes in a[0] for nd in nodes if not nd.split))
    monkeypatch.setattr(O, "pack_stream", bad_pack)
    assert not pin_cr()
