"""FP64 reference oracle for the AQMP encoder (test infrastructure only).

This module is a plain, slow, literal CPU implementation of what the GPU path
computes.  It exists to check that path: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  It shares no code,
tables or constants with the GPU library, which never imports it.

Everything is float64 NumPy, one quadtree node at a time.

Sources in the paper (AQMP, arXiv 2605.09190):

* Section 2.1: the 1D DCT-II matrix ``C[k, n] = alpha_k cos(pi/N (n + 1/2) k)``
  with ``alpha_0 = sqrt(1/N)``, ``alpha_k = sqrt(2/N)``; the 2D atoms are outer
  products of two 1D rows.
* Section 2.3 and Appendix A: the dictionary for block size N concatenates a
  DCT basis with a Haar basis; a block is flattened by concatenating its
  columns.
* Section 2.2, eq. (1)-(2) and the MP steps (a)-(d): residual initialised to
  the signal, arg-max of the absolute correlation, rank-1 residual update,
  stop when the residual norm falls below the tolerance or after k steps.
* Algorithms 1-2 (encoder) and 3 (decoder) of Section 2.3.
* Section 2.2 (the solver the authors' code ran) and the original OMP
  definition it cites: Orthogonal Matching Pursuit selects as MP does, then
  re-fits every selected coefficient by least squares; available as the
  solver "omp" of the encoder.

Readings taken where the paper is silent or inconsistent (each one is listed
with its reason in the design notes of the repository):

* plain MP (the rank-1 update of step (c)), not OMP;
* split when MP ends without meeting the accuracy target and N > N_min
  (rule "r1", the prose of Section 2.3); the pseudocode's literal
  ``||x||_0 >= k`` test is available as rule "r2";
* k counts MP iterations; re-selecting an atom gives a new record;
* the stop test is checked before every iteration, including the first,
  on squared norms with a strict ``<``;
* tolerance mode "rms": eps_N = tol * N (residual RMS over the block);
  mode "abs": the same eps at every level, as Algorithm 2 passes it down;
* M_N = 2 N^2: one orthonormal DCT basis and one orthonormal separable
  (Kronecker) Haar basis; atom index ``a = f N^2 + q N + p`` for the atom
  ``A[i, j] = T_f[p, i] T_f[q, j]``;
* both constant (DC) atoms are set to exactly 1/N, so the duplicate pair
  ties exactly; arg-max ties go to the lowest atom index;
* stop when the largest absolute correlation is exactly zero;
* children encode the original pixels of their quadrant (Algorithm 2
  recurses on the block ``b``) in the order TL, TR, BL, BR;
* a plane whose width or height is not a multiple of N_max is padded up to
  the next multiple by repeating its last row and column; the padding's
  blocks are coded like any other and the decoder keeps the image's own
  pixels.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

DCT = 1
HAAR = 2


# ---------------------------------------------------------------------------
# Dictionaries (Section 2.1; Section 2.3 "DCT basis with wavelets (e.g. Haar)";
# Appendix A)
# ---------------------------------------------------------------------------

def dct_matrix(n: int) -> np.ndarray:
    """1D DCT-II matrix of Section 2.1: ``C[k, m] = alpha_k cos(pi/n (m + 1/2) k)``."""
    k = np.arange(n, dtype=np.float64)[:, None]
    m = np.arange(n, dtype=np.float64)[None, :]
    alpha = np.where(k == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
    return alpha * np.cos(np.pi / n * (m + 0.5) * k)


def haar_matrix(n: int) -> np.ndarray:
    """Orthonormal 1D Haar matrix, built by the two-scale recursion.

    ``H_1 = [1]`` and ``H_2m = (1/sqrt 2) [H_m (x) (1, 1); I_m (x) (1, -1)]``.
    Row 0 is the constant; the remaining rows are the wavelets from coarse
    to fine.  The paper names Haar wavelets without a construction; this is
    the standard orthonormal one.
    """
    if n < 1 or n & (n - 1):
        raise ValueError("n must be a power of two")
    h = np.ones((1, 1))
    while h.shape[0] < n:
        m = h.shape[0]
        top = np.kron(h, np.array([[1.0, 1.0]]))
        bot = np.kron(np.eye(m), np.array([[1.0, -1.0]]))
        h = np.vstack([top, bot]) / np.sqrt(2.0)
    return h


def unravel(block: np.ndarray) -> np.ndarray:
    """Flatten an N x N block by concatenating its columns (Appendix A)."""
    return np.asarray(block, dtype=np.float64).reshape(-1, order="F")


def unravel_inv(vec: np.ndarray, n: int) -> np.ndarray:
    """Inverse of :func:`unravel`."""
    return np.asarray(vec, dtype=np.float64).reshape((n, n), order="F")


def dictionary(n: int, families: int = DCT | HAAR) -> np.ndarray:
    """Dictionary D_N as an ``N^2 x M`` matrix whose columns are unit atoms.

    For each family T (DCT first, then Haar) and each pair (p, q) the 2D atom
    is the outer product ``A[i, j] = T[p, i] T[q, j]`` (Section 2.1), flattened
    column-major; its index is ``f N^2 + q N + p``.  The constant atom of every
    family is set to exactly 1/N.
    """
    mats = []
    if families & DCT:
        mats.append(dct_matrix(n))
    if families & HAAR:
        mats.append(haar_matrix(n))
    if not mats:
        raise ValueError("empty dictionary")
    cols = []
    for t in mats:
        d = np.empty((n * n, n * n))
        for q in range(n):
            for p in range(n):
                a = np.outer(t[p], t[q])          # A[i, j] = T[p, i] T[q, j]
                d[:, q * n + p] = unravel(a)
        d[:, 0] = 1.0 / n                          # constant atom, exact
        cols.append(d)
    return np.hstack(cols)


def duplicate_groups(d: np.ndarray) -> np.ndarray:
    """``rep[a]`` = lowest index of an atom whose column equals atom ``a`` bit for bit."""
    m = d.shape[1]
    rep = np.arange(m)
    seen: dict[bytes, int] = {}
    for a in range(m):
        key = d[:, a].tobytes()
        if key in seen:
            rep[a] = seen[key]
        else:
            seen[key] = a
    return rep


class Dict:
    """One block size's dictionary with the transposed copy used for correlations."""

    def __init__(self, n: int, families: int = DCT | HAAR):
        self.n = n
        self.families = families
        self.D = dictionary(n, families)                  # [N^2, M]
        self.Dt = np.ascontiguousarray(self.D.T)          # [M, N^2]
        self.m = self.D.shape[1]
        self.rep = duplicate_groups(self.D)


_DICT_CACHE: dict[tuple[int, int], Dict] = {}


def get_dict(n: int, families: int = DCT | HAAR) -> Dict:
    key = (n, families)
    if key not in _DICT_CACHE:
        _DICT_CACHE[key] = Dict(n, families)
    return _DICT_CACHE[key]


# ---------------------------------------------------------------------------
# Matching Pursuit (Section 2.2, eq. (1)-(2), steps (a)-(d))
# ---------------------------------------------------------------------------

@dataclass
class MPResult:
    idx: list = field(default_factory=list)      # selected atom per iteration
    coef: list = field(default_factory=list)     # <r, phi_i> per iteration
    gap: list = field(default_factory=list)      # relative top-2 gap over distinct atoms
    e: list = field(default_factory=list)        # ||r||^2 before each iteration, then final
    stop: str = ""                               # "accuracy" | "sparsity" | "zero"

    @property
    def t(self) -> int:
        return len(self.idx)

    @property
    def e_final(self) -> float:
        return self.e[-1]


def top2_gap(c_abs: np.ndarray, rep: np.ndarray, i: int) -> float:
    """Relative gap between the best atom ``i`` and the best atom that is not a
    bit-identical copy of it: ``(|c|_(1) - |c|_(2)) / |c|_(1)``."""
    other = c_abs.copy()
    other[rep == rep[i]] = -1.0
    second = other.max() if other.size else -1.0
    if c_abs[i] == 0.0:
        return 0.0
    return float((c_abs[i] - max(second, 0.0)) / c_abs[i])


def omp(dic: Dict, y: np.ndarray, eps2: float, k: int) -> MPResult:
    """Orthogonal Matching Pursuit on one signal (Section 2.2; the OMP of the
    cited Pati et al. paper).

    ``r = y``, ``S = []``; before every iteration stop if ``||r||^2 < eps2``
    (eq. (2), accuracy) or if ``|S| = k`` (eq. (2), sparsity); otherwise
    ``c = D^T r``, ``i = argmax |c|`` (lowest index among equal values; a zero
    maximum stops), ``S <- S + [i]``, ``x_S = argmin_x ||y - D_S x||_2`` (least
    squares over the selected atoms), ``r = y - D_S x_S``.  ``coef`` holds the
    final least-squares coefficients in selection order.
    """
    y = np.array(y, dtype=np.float64, copy=True)
    r = y.copy()
    out = MPResult()
    sel: list[int] = []
    x = np.zeros(0)
    e = float(r @ r)
    out.e.append(e)
    while True:
        if e < eps2:
            out.stop = "accuracy"
            break
        if len(sel) >= k:
            out.stop = "sparsity"
            break
        c = dic.Dt @ r
        c_abs = np.abs(c)
        i = int(np.argmax(c_abs))          # first maximal index
        if c_abs[i] == 0.0:
            out.stop = "zero"
            break
        out.gap.append(top2_gap(c_abs, dic.rep, i))
        sel.append(i)
        a = dic.D[:, sel]
        x = np.linalg.lstsq(a, y, rcond=None)[0]
        r = y - a @ x
        e = float(r @ r)
        out.e.append(e)
    out.idx = list(sel)
    out.coef = [float(v) for v in x[:len(sel)]]
    return out


def mp(dic: Dict, y: np.ndarray, eps2: float, k: int) -> MPResult:
    """Plain Matching Pursuit on one signal.

    ``r = y``; before every iteration stop if ``||r||^2 < eps2`` (eq. (2),
    accuracy) or if ``k`` iterations have been made (eq. (2), sparsity);
    otherwise ``c = D^T r``, ``i = argmax |c|`` (lowest index among equal
    values), ``r <- r - c_i phi_i``.  A zero maximum correlation stops too.
    """
    r = np.array(y, dtype=np.float64, copy=True)
    out = MPResult()
    e = float(r @ r)
    out.e.append(e)
    while True:
        if e < eps2:
            out.stop = "accuracy"
            break
        if out.t >= k:
            out.stop = "sparsity"
            break
        c = dic.Dt @ r
        c_abs = np.abs(c)
        i = int(np.argmax(c_abs))          # first maximal index
        if c_abs[i] == 0.0:
            out.stop = "zero"
            break
        ci = float(c[i])
        out.gap.append(top2_gap(c_abs, dic.rep, i))
        r = r - ci * dic.D[:, i]
        e = float(r @ r)
        out.idx.append(i)
        out.coef.append(ci)
        out.e.append(e)
    return out


# ---------------------------------------------------------------------------
# Encoder (Algorithms 1-2) and decoder (Algorithm 3)
# ---------------------------------------------------------------------------

@dataclass
class Params:
    tol: float
    tol_mode: str = "rms"          # "rms": eps_N = tol*N ; "abs": eps_N = tol
    max_atoms: int = 32
    n_min: int = 8
    n_max: int = 64
    split_rule: str = "r1"         # "r1" accuracy not met ; "r2" ||x||_0 >= k literal
    k_per_level: dict | None = None
    families: int = DCT | HAAR
    solver: str = "mp"             # "mp": Section 2.2 steps (a)-(d) ; "omp": least-squares refit

    def eps2(self, n: int) -> float:
        eps = self.tol * n if self.tol_mode == "rms" else self.tol
        return float(eps) * float(eps)

    def k(self, n: int) -> int:
        if self.k_per_level is not None and n in self.k_per_level:
            return int(self.k_per_level[n])
        return int(self.max_atoms)

    @staticmethod
    def from_dict(d: dict) -> "Params":
        keys = {"tol", "tol_mode", "max_atoms", "n_min", "n_max", "split_rule",
                "k_per_level", "families", "solver"}
        return Params(**{k: v for k, v in d.items() if k in keys})


@dataclass
class Node:
    x0: int
    y0: int
    n: int
    mp: MPResult
    split: bool
    eps2: float
    norm2: float            # ||y||^2 of the node's original pixels


def split_decision(p: Params, n: int, res: MPResult) -> bool:
    """Whether a node of size ``n`` is refined into its four quadrants."""
    if n <= p.n_min:
        return False
    if p.split_rule == "r1":
        return res.e_final >= p.eps2(n)
    return res.t >= p.k(n)


def encode_block(img: np.ndarray, p: Params, x0: int, y0: int, n: int,
                 nodes: list[Node] | None = None) -> list[Node]:
    """Algorithm 2 on one block: MP, then either emit it or recurse into its
    quadrants (TL, TR, BL, BR) of the original pixels.  Returns the visited
    nodes in depth-first order; the leaves are those with ``split=False``."""
    if nodes is None:
        nodes = []
    block = img[y0:y0 + n, x0:x0 + n]
    y = unravel(block)
    dic = get_dict(n, p.families)
    res = (omp if p.solver == "omp" else mp)(dic, y, p.eps2(n), p.k(n))
    sp = split_decision(p, n, res)
    nodes.append(Node(x0, y0, n, res, sp, p.eps2(n), float(y @ y)))
    if sp:
        h = n // 2
        for dy, dx in ((0, 0), (0, h), (h, 0), (h, h)):
            encode_block(img, p, x0 + dx, y0 + dy, h, nodes)
    return nodes


def pad_edge(img: np.ndarray, n: int) -> np.ndarray:
    """The plane padded up to a multiple of ``n`` in both directions by
    repeating its last row and column."""
    h, w = img.shape
    return np.pad(img, ((0, -h % n), (0, -w % n)), mode="edge")


def top_blocks(h: int, w: int, n_max: int) -> list[tuple[int, int]]:
    """Top-level blocks of size n_max in raster order, as (x0, y0), over the
    plane padded up to a multiple of n_max."""
    return [(x, y) for y in range(0, h, n_max) for x in range(0, w, n_max)]


def encode_channel(img: np.ndarray, p: Params, blocks=None) -> list[Node]:
    """Algorithm 2 started at N_max on every top-level block (or on the given
    subset of top-level blocks)."""
    img = pad_edge(np.asarray(img, dtype=np.float64), p.n_max)
    if blocks is None:
        blocks = top_blocks(img.shape[0], img.shape[1], p.n_max)
    nodes: list[Node] = []
    for (x0, y0) in blocks:
        encode_block(img, p, x0, y0, p.n_max, nodes)
    return nodes


def encode(channels: Sequence[np.ndarray], p: Params) -> list[list[Node]]:
    """Algorithm 1: each channel is encoded independently."""
    return [encode_channel(c, p) for c in channels]


def leaves(nodes: list[Node]) -> list[Node]:
    return [nd for nd in nodes if not nd.split]


def decode(nodes: list[Node], h: int, w: int, families: int = DCT | HAAR) -> np.ndarray:
    """Algorithm 3: every leaf's block is ``unravel^-1(D_N x)`` placed at its
    position.  Pixels not covered by a leaf stay zero."""
    lv = leaves(nodes)
    hp = max([h] + [nd.y0 + nd.n for nd in lv])
    wp = max([w] + [nd.x0 + nd.n for nd in lv])
    out = np.zeros((hp, wp))
    for nd in lv:
        dic = get_dict(nd.n, families)
        x = np.zeros(dic.m)
        for i, c in zip(nd.mp.idx, nd.mp.coef):
            x[i] += c
        out[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n] = unravel_inv(dic.D @ x, nd.n)
    return out[:h, :w]


# ---------------------------------------------------------------------------
# Bitstream and compression rate (Section 2.3 encoder step (iii), decoder
# step (i); Section 3, the CR definition).  The paper names DEFLATE over the
# sparse vectors but no byte layout; this is the layout the encoder library
# writes (version 1, little-endian, described in its public header).
# ---------------------------------------------------------------------------

def quantize(coef, step: float) -> np.ndarray:
    """Uniform scalar quantiser of the coefficients (the lossy part of encoder
    step (ii), Section 2.3; the paper names no quantiser, this one is stated
    by the stream format): q = round-half-to-even(c / d), with d the step
    rounded to binary32 (the value the stream stores), computed in FP64.  The
    decoder reconstructs q * d."""
    d = float(np.float32(step))
    if not d > 0.0:
        raise ValueError("the quantiser step must be positive")
    return np.rint(np.asarray(coef, dtype=np.float64) / d).astype(np.int64)


def dequantize(q, step: float) -> np.ndarray:
    return np.asarray(q, dtype=np.float64) * float(np.float32(step))


def pack_stream(channels: Sequence[list], w: int, h: int, n_min: int, n_max: int,
                families: int = DCT | HAAR, step: float | None = None) -> bytes:
    """The uncompressed bitstream of one image: a header, then per channel
    (each a node list in depth-first order as ``encode_channel`` returns it)
    the split flags of the nodes with N > N_min, the leaves' atom counts,
    their atom indices (u16) and coefficients: binary32 (coefficient format
    0), or with ``step`` (format 1) the quantised values q of ``quantize`` as
    signed little-endian integers of the header's width (2 bytes when every
    |q| <= 32767, else 4), the binary32 step following the 20-byte header."""
    import struct
    counts = [nd.mp.t for nodes in channels for nd in nodes if not nd.split]
    cb = 2 if counts and max(counts) > 255 else 1
    qs = None
    qb = 0
    if step is not None:
        qs = [quantize([c for nd in nodes if not nd.split for c in nd.mp.coef], step) for nodes in channels]
        big = max([int(np.max(np.abs(q))) for q in qs if q.size] + [0])
        qb = 2 if big <= 32767 else 4
    out = bytearray(b"AQMP")
    out += struct.pack("<BBBBIIBBBB", 1, families, 0 if step is None else 1, len(channels), w, h,
                       n_min.bit_length() - 1, n_max.bit_length() - 1, cb, qb)
    if step is not None:
        out += struct.pack("<f", float(np.float32(step)))
    for ci, nodes in enumerate(channels):
        lv = [nd for nd in nodes if not nd.split]
        out += struct.pack("<III", len(nodes), len(lv), sum(nd.mp.t for nd in lv))
        bits = np.array([1 if nd.split else 0 for nd in nodes if nd.n > n_min], dtype=np.uint8)
        out += np.packbits(bits, bitorder="little").tobytes()
        out += np.array([nd.mp.t for nd in lv], dtype="<u1" if cb == 1 else "<u2").tobytes()
        out += np.array([i for nd in lv for i in nd.mp.idx], dtype="<u2").tobytes()
        if step is None:
            out += np.array([c for nd in lv for c in nd.mp.coef], dtype="<f4").tobytes()
        else:
            out += qs[ci].astype("<i2" if qb == 2 else "<i4").tobytes()
    return bytes(out)


def unpack_stream(data: bytes) -> dict:
    """Inverse of ``pack_stream``: the header fields and, per channel, the
    leaves ``(x0, y0, n, idx, coef)`` in depth-first order, recovered by
    walking the quadtree with the split flags."""
    import struct
    assert data[:4] == b"AQMP"
    ver, fam, fmt, nch, w, h, lmin, lmax, cb, qb = struct.unpack_from("<BBBBIIBBBB", data, 4)
    assert ver == 1 and fmt in (0, 1)
    n_min, n_max = 1 << lmin, 1 << lmax
    pos = 20
    step = None
    if fmt == 1:
        assert qb in (2, 4)
        step = float(struct.unpack_from("<f", data, pos)[0])
        pos += 4
    chans = []
    for _ in range(nch):
        n_nodes, n_leaves, n_atoms = struct.unpack_from("<III", data, pos)
        pos += 12
        shape = []                      # (x0, y0, n) of every leaf, depth-first
        nbits = 0
        bitbuf = np.frombuffer(data, dtype=np.uint8, offset=pos)
        bit_at = lambda i: (int(bitbuf[i >> 3]) >> (i & 7)) & 1

        def walk(x0, y0, n):
            nonlocal nbits
            split = 0
            if n > n_min:
                split = bit_at(nbits)
                nbits += 1
            if split:
                hh = n // 2
                for dy, dx in ((0, 0), (0, hh), (hh, 0), (hh, hh)):
                    walk(x0 + dx, y0 + dy, hh)
            else:
                shape.append((x0, y0, n))

        for (x0, y0) in top_blocks(h, w, n_max):
            walk(x0, y0, n_max)
        pos += (nbits + 7) // 8
        assert len(shape) == n_leaves
        cnt = np.frombuffer(data, dtype="<u1" if cb == 1 else "<u2", count=n_leaves, offset=pos).astype(int)
        pos += cb * n_leaves
        idx = np.frombuffer(data, dtype="<u2", count=n_atoms, offset=pos).astype(int)
        pos += 2 * n_atoms
        if fmt == 0:
            coef = np.frombuffer(data, dtype="<f4", count=n_atoms, offset=pos).astype(np.float64)
            pos += 4 * n_atoms
        else:
            q = np.frombuffer(data, dtype="<i2" if qb == 2 else "<i4", count=n_atoms, offset=pos)
            coef = q.astype(np.float64) * step
            pos += qb * n_atoms
        off = np.concatenate([[0], np.cumsum(cnt)])
        chans.append([(x0, y0, n, idx[off[i]:off[i + 1]].tolist(), coef[off[i]:off[i + 1]].tolist())
                      for i, (x0, y0, n) in enumerate(shape)])
    assert pos == len(data)
    return dict(families=fam, w=w, h=h, n_min=n_min, n_max=n_max, channels=chans, step=step)


def compress_stream(raw: bytes, level: int = 9) -> bytes:
    """Encoder step (iii): DEFLATE (zlib container) over the bitstream."""
    import zlib
    return zlib.compress(raw, level)


def compression_rate(compressed_size: int, w: int, h: int, channels: int) -> float:
    """CR = size_original / size_compressed (Section 3), the original being
    8-bit samples: w * h * channels bytes."""
    return float(w * h * channels) / float(compressed_size)


# ---------------------------------------------------------------------------
# SSIM (Section 3's quality measure)
# ---------------------------------------------------------------------------

SSIM_K1, SSIM_K2 = 0.01, 0.03


def ssim(x: np.ndarray, y: np.ndarray, mode: str = "window7", data_range: float = 1.0) -> float:
    """SSIM(x, y) = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
    with C1 = (K1 L)^2, C2 = (K2 L)^2, K1 = 0.01, K2 = 0.03, L = data_range.

    ``mode="global"``: the equation as written, with the means, variances and
    covariance of the whole planes (population moments).
    ``mode="window7"``: the equation on every 7 x 7 window lying inside the
    plane (uniform weights, sample variances and covariance with the 49/48
    factor), averaged over the windows (one per interior pixel)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    c1, c2 = (SSIM_K1 * data_range) ** 2, (SSIM_K2 * data_range) ** 2

    def s(mx, my, vx, vy, cxy):
        return ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))

    if mode == "global":
        mx, my = x.mean(), y.mean()
        return float(s(mx, my, ((x - mx) ** 2).mean(), ((y - my) ** 2).mean(), ((x - mx) * (y - my)).mean()))
    assert mode == "window7"
    win = 7
    from numpy.lib.stride_tricks import sliding_window_view as swv
    wx, wy = swv(x, (win, win)), swv(y, (win, win))        # [H-6, W-6, 7, 7]
    n = win * win
    mx, my = wx.mean(axis=(2, 3)), wy.mean(axis=(2, 3))
    dx, dy = wx - mx[..., None, None], wy - my[..., None, None]
    vx = (dx * dx).sum(axis=(2, 3)) / (n - 1)
    vy = (dy * dy).sum(axis=(2, 3)) / (n - 1)
    cxy = (dx * dy).sum(axis=(2, 3)) / (n - 1)
    return float(s(mx, my, vx, vy, cxy).mean())


def psnr(ref: np.ndarray, rec: np.ndarray, peak: float = 1.0) -> float:
    """PSNR in dB with the given peak; the MSE is taken in float64 over all
    samples, without clipping the reconstruction."""
    d = np.asarray(ref, dtype=np.float64) - np.asarray(rec, dtype=np.float64)
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(peak * peak / mse)
