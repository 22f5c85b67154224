"""Pins of the oracle's SSIM (Section 3): closed forms and a brute-force
scalar evaluation on tiny planes."""
import math

import numpy as np
import pytest

from oracle import aqmp_oracle as O


def _brute(x, y, mode):
    """Scalar loops over the windows (or the whole plane), written without
    array reductions."""
    c1, c2 = (0.01) ** 2, (0.03) ** 2
    h, w = len(x), len(x[0])

    def one(px, py, sample):
        n = len(px)
        mx = sum(px) / n
        my = sum(py) / n
        d = n - 1 if sample else n
        vx = sum((a - mx) ** 2 for a in px) / d
        vy = sum((b - my) ** 2 for b in py) / d
        cxy = sum((a - mx) * (b - my) for a, b in zip(px, py)) / d
        return ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))

    if mode == "global":
        return one([v for r in x for v in r], [v for r in y for v in r], False)
    vals = []
    for i in range(h - 6):
        for j in range(w - 6):
            px = [x[i + a][j + b] for a in range(7) for b in range(7)]
            py = [y[i + a][j + b] for a in range(7) for b in range(7)]
            vals.append(one(px, py, True))
    return sum(vals) / len(vals)


@pytest.mark.parametrize("mode", ["global", "window7"])
def test_ssim_matches_brute_force(mode):
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(11, 13))
    y = np.clip(x + rng.normal(0, 0.05, size=x.shape), 0, 1)
    assert abs(O.ssim(x, y, mode) - _brute(x.tolist(), y.tolist(), mode)) < 1e-12


@pytest.mark.parametrize("mode", ["global", "window7"])
def test_ssim_identity_and_symmetry(mode):
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(20, 24))
    y = rng.uniform(size=(20, 24))
    assert abs(O.ssim(x, x, mode) - 1.0) < 1e-15
    assert abs(O.ssim(x, y, mode) - O.ssim(y, x, mode)) < 1e-15
    assert O.ssim(x, y, mode) < 0.5


def test_ssim_global_closed_form_for_constants():
    """Two constant planes a and b: SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    c1 = 1e-4
    assert abs(O.ssim(np.full((9, 9), a), np.full((9, 9), b), "global") - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-15


def test_ssim_window_contrast_term():
    """y = x + c (a shift) leaves the structure and contrast terms at 1: each
    window's SSIM is the luminance term of its means."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0.2, 0.6, size=(10, 10))
    y = x + 0.1
    from numpy.lib.stride_tricks import sliding_window_view as swv
    mx = swv(x, (7, 7)).mean(axis=(2, 3))
    my = mx + 0.1
    lum = ((2 * mx * my + 1e-4) / (mx * mx + my * my + 1e-4)).mean()
    assert math.isclose(O.ssim(x, y, "window7"), lum, rel_tol=1e-12)
