"""Seeded synthetic images and the parameter sets of the measured workloads.

The paper evaluates on public photographs and document scans (USC-SIPI,
DIBCO, DIV2K; Section 3) that are not available here.  These generators stand
in for them with the same resolutions and the same kinds of content: smooth
regions, sharp edges, filled shapes, periodic texture and sensor noise.

Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed order, works in float64 and clips to [0, 1].  ``as_f32=True`` rounds the
result to float32-representable values so that a float32 device copy and the
float64 host copy hold identical numbers.

Nothing here belongs to the encoder: colour conversion (``rgb_to_ycbcr``) is
the codec's pre-processing step (i) of Section 2.3.1, applied before the
channels are handed to the encoder.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gradient_edges_image", "piecewise_image", "rgb_to_ycbcr", "workload",
    "C4_SIZES", "sweep_trials", "WORKLOADS",
]


def _finish(img: np.ndarray, rng: np.random.Generator, sigma: float, as_f32: bool) -> np.ndarray:
    img = img + rng.normal(0.0, sigma, size=img.shape)
    img = np.clip(img, 0.0, 1.0)
    if as_f32:
        img = img.astype(np.float32).astype(np.float64)
    return np.ascontiguousarray(img)


def gradient_edges_image(h: int, w: int, seed: int, as_f32: bool = True) -> np.ndarray:
    """Linear gradient + 3 random step edges + 2 random discs + N(0, 0.01^2) noise.

    Gradient ``a0 + ax*x/W + ay*y/H`` with a0 ~ U(0.2, 0.4), ax, ay ~ U(-0.2, 0.2).
    Each edge is a line through a uniform point with angle U(0, pi); one side
    is raised by h ~ U(-0.3, 0.3).  Each disc has radius U(4, 16) px, a uniform
    centre and adds U(-0.4, 0.4) inside.
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    a0 = rng.uniform(0.2, 0.4)
    ax, ay = rng.uniform(-0.2, 0.2, size=2)
    img = a0 + ax * xx / w + ay * yy / h
    for _ in range(3):
        px, py = rng.uniform(0, w), rng.uniform(0, h)
        th = rng.uniform(0, np.pi)
        step = rng.uniform(-0.3, 0.3)
        side = (xx - px) * np.sin(th) - (yy - py) * np.cos(th) > 0
        img = img + step * side
    for _ in range(2):
        r = rng.uniform(4, 16)
        cx, cy = rng.uniform(0, w), rng.uniform(0, h)
        v = rng.uniform(-0.4, 0.4)
        img = img + v * (((xx - cx) ** 2 + (yy - cy) ** 2) <= r * r)
    return _finish(img, rng, 0.01, as_f32)


def piecewise_image(h: int, w: int, seed: int, as_f32: bool = True,
                    n_regions: int = 8, n_ellipses: int = 20, n_gratings: int = 8,
                    sigma: float = 0.005) -> np.ndarray:
    """Piecewise-smooth quadratics + filled ellipses + grating patches + noise.

    * ``n_regions`` Voronoi cells (uniform seeds).  Cell ``j`` holds the
      quadratic ``c_j . (1, u, v, u^2, uv, v^2)`` in normalised coordinates
      u = x/W, v = y/H with c_j ~ N(0, 1); it is mapped affinely so that its
      range over the whole image is [lo_j, hi_j], lo_j < hi_j drawn from
      U(0.1, 0.9).
    * ``n_ellipses`` filled ellipses: semi-axes U(0.02, 0.15)*min(W, H),
      angle U(0, pi), uniform centre, fill value U(0, 1) (replaces pixels).
    * ``n_gratings`` square patches of side U(0.05, 0.2)*min(W, H), uniform
      position, adding ``amp*sin(2*pi*(x cos t + y sin t)/period)`` with
      period U(3, 16) px, t ~ U(0, pi), amp ~ U(0.1, 0.3).
    * Gaussian noise of standard deviation ``sigma``, then clipping to [0, 1].

    Geometry scales with the image size; grating periods stay in pixels.
    """
    rng = np.random.default_rng(seed)
    m = float(min(h, w))
    xs = np.arange(w, dtype=np.float64)
    ys = np.arange(h, dtype=np.float64)
    u = xs / w
    v = ys / h
    # Voronoi labels, computed row-block by row-block to bound memory.
    sx = rng.uniform(0, w, size=n_regions)
    sy = rng.uniform(0, h, size=n_regions)
    coef = rng.normal(0.0, 1.0, size=(n_regions, 6))
    lohi = np.sort(rng.uniform(0.1, 0.9, size=(n_regions, 2)), axis=1)
    # Each cell's quadratic is mapped affinely so that its range over the
    # full image (sampled on a 65 x 65 grid) becomes [lo, hi].
    gu = np.linspace(0.0, 1.0, 65)[None, :]
    gv = np.linspace(0.0, 1.0, 65)[:, None]
    a_lo = np.empty(n_regions)
    a_sc = np.empty(n_regions)
    q_lo = np.empty(n_regions)
    for j in range(n_regions):
        c = coef[j]
        g = c[0] + c[1] * gu + c[2] * gv + c[3] * gu * gu + c[4] * gu * gv + c[5] * gv * gv
        q_lo[j] = g.min()
        a_sc[j] = (lohi[j, 1] - lohi[j, 0]) / max(float(g.max() - g.min()), 1e-12)
        a_lo[j] = lohi[j, 0]
    img = np.empty((h, w), dtype=np.float64)
    uu = u[None, :]
    for r0 in range(0, h, 128):
        r1 = min(h, r0 + 128)
        yb = ys[r0:r1, None]
        vb = v[r0:r1, None]
        best = np.full((r1 - r0, w), np.inf)
        lab = np.zeros((r1 - r0, w), dtype=np.int64)
        for j in range(n_regions):
            d2 = (xs[None, :] - sx[j]) ** 2 + (yb - sy[j]) ** 2
            closer = d2 < best
            best = np.where(closer, d2, best)
            lab = np.where(closer, j, lab)
        c = coef[lab]  # [rows, w, 6]
        q = (c[..., 0] + c[..., 1] * uu + c[..., 2] * vb + c[..., 3] * uu * uu
             + c[..., 4] * uu * vb + c[..., 5] * vb * vb)
        img[r0:r1] = a_lo[lab] + (q - q_lo[lab]) * a_sc[lab]
    # Ellipses (replace), each restricted to its bounding box.
    for _ in range(n_ellipses):
        a, b = rng.uniform(0.02, 0.15, size=2) * m
        th = rng.uniform(0, np.pi)
        cx, cy = rng.uniform(0, w), rng.uniform(0, h)
        fill = rng.uniform(0, 1)
        rr = max(a, b)
        x0, x1 = max(0, int(cx - rr) - 1), min(w, int(cx + rr) + 2)
        y0, y1 = max(0, int(cy - rr) - 1), min(h, int(cy + rr) + 2)
        if x0 >= x1 or y0 >= y1:
            continue
        dx = xs[None, x0:x1] - cx
        dy = ys[y0:y1, None] - cy
        ct, st = np.cos(th), np.sin(th)
        p = (dx * ct + dy * st) / a
        q = (-dx * st + dy * ct) / b
        inside = p * p + q * q <= 1.0
        img[y0:y1, x0:x1][inside] = fill
    # Grating patches (add).
    for _ in range(n_gratings):
        side = rng.uniform(0.05, 0.2) * m
        px, py = rng.uniform(0, w - side), rng.uniform(0, h - side)
        period = rng.uniform(3, 16)
        th = rng.uniform(0, np.pi)
        amp = rng.uniform(0.1, 0.3)
        x0, x1 = int(px), min(w, int(px + side))
        y0, y1 = int(py), min(h, int(py + side))
        gx = xs[None, x0:x1]
        gy = ys[y0:y1, None]
        img[y0:y1, x0:x1] += amp * np.sin(2 * np.pi * (gx * np.cos(th) + gy * np.sin(th)) / period)
    return _finish(img, rng, sigma, as_f32)


def rgb_to_ycbcr(rgb: np.ndarray) -> np.ndarray:
    """Full-range BT.601 (JFIF) colour conversion, channels last -> channels first.

    Pre-processing step (i) of the codec (Section 2.3.1 and Appendix A name
    YCbCr without fixing the matrix).  Cb and Cr carry the +0.5 offset so
    that every channel lies in [0, 1].  Returns ``[3, H, W]`` float64.
    """
    r, g, b = rgb[..., 0], rgb[..., 1], rgb[..., 2]
    y = 0.299 * r + 0.587 * g + 0.114 * b
    cb = -0.168736 * r - 0.331264 * g + 0.5 * b + 0.5
    cr = 0.5 * r - 0.418688 * g - 0.081312 * b + 0.5
    return np.stack([y, cb, cr], axis=0)


# Image sizes (W x H) of the 16-image hyperparameter sweep; all multiples of 64.
C4_SIZES = [
    (256, 256), (320, 256), (512, 384), (512, 512), (640, 512), (768, 576),
    (1024, 768), (1024, 1024), (1280, 768), (1536, 1024), (1600, 1216),
    (2048, 1536), (2048, 2048), (2560, 1920), (3072, 2304), (4096, 3072),
]


def sweep_trials(n_trials: int = 32, seed: int = 7) -> list[dict]:
    """Seeded random-search trials over the encoder's hyperparameters.

    RMS tolerance log-uniform in [0.005, 0.06], max atoms uniform in {8..64},
    minimum block in {4, 8}, maximum block in {32, 64} (the paper's search
    space of Section 2.4, restricted to the parameters this encoder takes).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_trials):
        tau = float(np.exp(rng.uniform(np.log(0.005), np.log(0.06))))
        k = int(rng.integers(8, 65))
        n_min = int(rng.choice([4, 8]))
        n_max = int(rng.choice([32, 64]))
        out.append(dict(tol=tau, tol_mode="rms", max_atoms=k, n_min=n_min, n_max=n_max))
    return out


def _c0():
    img = gradient_edges_image(64, 64, seed=0)
    return dict(name="gradient-edges 64x64 grey, blocks 32->8, k=16, rms 0.02",
                channels=[img],
                params=[dict(tol=0.02, tol_mode="rms", max_atoms=16, n_min=8, n_max=32)],
                jobs=[(0, 0)])


def _c1(tau=0.02):
    img = piecewise_image(512, 512, seed=1)
    return dict(name=f"piecewise 512x512 grey, blocks 64->8, k=32, rms {tau}",
                channels=[img],
                params=[dict(tol=tau, tol_mode="rms", max_atoms=32, n_min=8, n_max=64)],
                jobs=[(0, 0)])


def _c2(size=2048, tau=0.02):
    rgb = np.stack([piecewise_image(size, size, seed=s, as_f32=False) for s in (2, 3, 4)], axis=-1)
    ycc = rgb_to_ycbcr(rgb).astype(np.float32).astype(np.float64)
    return dict(name=f"piecewise {size}x{size} RGB->YCbCr (3 jobs), blocks 64->8, k=32, rms {tau}",
                channels=[ycc[0], ycc[1], ycc[2]],
                params=[dict(tol=tau, tol_mode="rms", max_atoms=32, n_min=8, n_max=64)],
                jobs=[(0, 0), (1, 0), (2, 0)])


def _c4(n_images=16, n_trials=32):
    chans = []
    for i, (w, h) in enumerate(C4_SIZES[:n_images]):
        chans.append(piecewise_image(h, w, seed=100 + i))
    trials = sweep_trials(n_trials)
    jobs = [(i, t) for i in range(len(chans)) for t in range(len(trials))]
    return dict(name=f"sweep: {len(chans)} images x {len(trials)} trials",
                channels=chans, params=trials, jobs=jobs)


WORKLOADS = {"c0": _c0, "c1": _c1, "c2": _c2, "c3": _c2, "c4": _c4}


def workload(name: str, **kw) -> dict:
    """A workload: ``channels`` (list of float64 [H, W] arrays), ``params``
    (list of parameter dicts) and ``jobs`` (list of (channel, params) index
    pairs; one job is one channel encoded under one parameter set)."""
    return WORKLOADS[name](**kw)
