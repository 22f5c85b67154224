"""Pins of the oracle's dictionaries against facts fixed outside the oracle.

Section 2.1 defines the DCT-II matrix and builds 2D atoms as outer products;
Section 2.3 / Appendix A concatenate a DCT basis with a Haar basis and flatten
blocks column by column.
"""
import os

import numpy as np
import pytest
import scipy.fft

from oracle import aqmp_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_gold(name, symbols=None):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or not line.strip():
            continue
        vals = []
        for tok in line.split():
            neg = tok.startswith("-")
            key = tok.lstrip("-")
            v = symbols[key] if symbols and key in symbols else float(key)
            vals.append(-v if neg else v)
        rows.append(vals)
    return np.array(rows)


def test_dct4_matches_hand_values():
    gold = _read_gold("dct4.txt")
    assert np.allclose(O.dct_matrix(4), gold, atol=1e-15, rtol=0)


def test_haar4_matches_hand_values():
    gold = _read_gold("haar4.txt", {"s": 0.5, "t": 1 / np.sqrt(2.0)})
    assert np.allclose(O.haar_matrix(4), gold, atol=1e-15, rtol=0)


def test_haar2_closed_form():
    assert np.allclose(O.haar_matrix(2), np.array([[1, 1], [1, -1]]) / np.sqrt(2), atol=1e-16)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64])
def test_1d_bases_orthonormal(n):
    for t in (O.dct_matrix(n), O.haar_matrix(n)):
        assert np.abs(t @ t.T - np.eye(n)).max() < 1e-13


@pytest.mark.parametrize("n", [4, 8, 16])
def test_dct_matrix_equals_scipy(n):
    # scipy's orthonormal DCT-II applied to the identity gives C^T.
    c = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)
    assert np.abs(O.dct_matrix(n) - c).max() < 1e-14


@pytest.mark.parametrize("n", [4, 8, 16])
def test_dct_half_is_2d_dct_column_major(n):
    """D^T unravel(Y), DCT half, at index q*N + p equals dctn(Y)[p, q]: this
    fixes the column-major flattening and the atom index order."""
    rng = np.random.default_rng(n)
    y = rng.normal(size=(n, n))
    d = O.dictionary(n)
    c = d.T @ O.unravel(y)
    ref = scipy.fft.dctn(y, type=2, norm="ortho")
    got = c[: n * n].reshape(n, n).T          # got[p, q] = c[q*N + p]
    assert np.abs(got - ref).max() < 1e-12
    # A transposed flattening would fail here on a non-symmetric block.
    c_wrong = d.T @ y.reshape(-1)             # row-major
    assert np.abs(c_wrong[: n * n].reshape(n, n).T - ref).max() > 1e-3


def _haar2d_pyramid_free(y):
    """Separable 2D Haar transform computed by the fast averaging/differencing
    recursion along each axis (independent of the matrix construction)."""
    def haar1d(v):
        v = np.array(v, dtype=float)
        n = v.shape[0]
        out = v.copy()
        coeffs = []
        cur = v
        while cur.shape[0] > 1:
            a = (cur[0::2] + cur[1::2]) / np.sqrt(2)
            d = (cur[0::2] - cur[1::2]) / np.sqrt(2)
            coeffs.insert(0, d)
            cur = a
        out = np.concatenate([cur] + coeffs)
        assert out.shape[0] == n
        return out
    t = np.apply_along_axis(haar1d, 0, y)
    return np.apply_along_axis(haar1d, 1, t)


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_haar_half_is_separable_haar_transform(n):
    rng = np.random.default_rng(100 + n)
    y = rng.normal(size=(n, n))
    d = O.dictionary(n)
    c = d.T @ O.unravel(y)
    got = c[n * n:].reshape(n, n).T
    ref = _haar2d_pyramid_free(y)
    assert np.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_atoms_unit_norm_dc_exact_one_duplicate(n):
    d = O.dictionary(n)
    assert d.shape == (n * n, 2 * n * n)
    assert np.abs(np.linalg.norm(d, axis=0) - 1).max() < 1e-14
    assert np.all(d[:, 0] == 1.0 / n) and np.all(d[:, n * n] == 1.0 / n)
    rep = O.duplicate_groups(d)
    dup = np.nonzero(rep != np.arange(d.shape[1]))[0]
    assert list(dup) == [n * n] and rep[n * n] == 0


@pytest.mark.parametrize("fam", [O.DCT, O.HAAR])
def test_single_family_is_orthonormal_basis(fam):
    d = O.dictionary(8, fam)
    assert d.shape == (64, 64)
    assert np.abs(d.T @ d - np.eye(64)).max() < 1e-13


def test_duplicate_dc_correlations_bit_identical():
    for n in (4, 8, 16, 32):
        dic = O.get_dict(n)
        rng = np.random.default_rng(n)
        for _ in range(10):
            c = dic.Dt @ rng.normal(size=n * n)
            assert c[0] == c[n * n]


def test_unravel_roundtrip_and_order():
    a = np.arange(9.0).reshape(3, 3)
    v = O.unravel(a)
    assert list(v) == [0, 3, 6, 1, 4, 7, 2, 5, 8]   # columns concatenated
    assert np.array_equal(O.unravel_inv(v, 3), a)
