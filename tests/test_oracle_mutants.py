"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case patches one plausible error into the oracle and checks that the
corresponding pin, evaluated on the patched oracle, fails.
"""
import numpy as np
import pytest
import scipy.fft

from oracle import aqmp_oracle as O


@pytest.fixture(autouse=True)
def _clear_cache():
    O._DICT_CACHE.clear()
    yield
    O._DICT_CACHE.clear()


def pin_orthonormal_dct(n=8):
    c = O.dct_matrix(n)
    return np.abs(c @ c.T - np.eye(n)).max() < 1e-13


def pin_dctn(n=8):
    rng = np.random.default_rng(0)
    y = rng.normal(size=(n, n))
    c = O.dictionary(n).T @ O.unravel(y)
    return np.abs(c[: n * n].reshape(n, n).T - scipy.fft.dctn(y, norm="ortho")).max() < 1e-12


def pin_energy(n=8):
    rng = np.random.default_rng(1)
    res = O.mp(O.get_dict(n), rng.normal(size=n * n), 0.0, 10)
    return all(abs(res.e[t + 1] - (res.e[t] - res.coef[t] ** 2)) < 1e-12 * res.e[0]
               for t in range(res.t))


def pin_constant_block(n=8):
    res = O.mp(O.get_dict(n), np.full(n * n, 0.4), 1e-12, 4)
    return res.idx == [0] and abs(res.coef[0] - 0.4 * n) < 1e-12


def pin_split_invariant():
    rng = np.random.default_rng(2)
    img = rng.uniform(size=(32, 32))
    p = O.Params(tol=0.02, max_atoms=4, n_min=8, n_max=32)
    for nd in O.encode_channel(img, p):
        if nd.split and not (nd.n > p.n_min and nd.mp.e_final >= p.eps2(nd.n)):
            return False
        if not nd.split and not (nd.mp.e_final < p.eps2(nd.n) or nd.n == p.n_min):
            return False
    return True


def test_pins_hold_on_unpatched_oracle():
    assert pin_orthonormal_dct() and pin_dctn() and pin_energy()
    assert pin_constant_block() and pin_split_invariant()


def test_wrong_dct_normalisation_caught(monkeypatch):
    orig = O.dct_matrix
    # planted: alpha_0 = sqrt(2/N) instead of sqrt(1/N)
    monkeypatch.setattr(O, "dct_matrix", lambda n: np.vstack([orig(n)[:1] * np.sqrt(2.0), orig(n)[1:]]))
    assert not pin_orthonormal_dct()


def test_transposed_atom_caught(monkeypatch):
    orig_outer = np.outer
    # planted: atoms built as A[i, j] = T[q, i] T[p, j] (operands swapped)
    monkeypatch.setattr(O.np, "outer", lambda a, b: orig_outer(b, a))
    try:
        assert not pin_dctn()
    finally:
        monkeypatch.setattr(O.np, "outer", orig_outer)


def test_update_sign_caught(monkeypatch):
    def bad_mp(dic, y, eps2, k):
        r = np.array(y, dtype=float)
        out = O.MPResult()
        out.e.append(float(r @ r))
        while out.t < k:
            c = dic.Dt @ r
            i = int(np.argmax(np.abs(c)))
            out.gap.append(0.0)
            r = r + c[i] * dic.D[:, i]          # planted: wrong sign
            out.idx.append(i); out.coef.append(float(c[i])); out.e.append(float(r @ r))
        return out
    monkeypatch.setattr(O, "mp", bad_mp)
    assert not pin_energy()


def test_highest_index_tie_break_caught(monkeypatch):
    def bad_mp(dic, y, eps2, k):
        r = np.array(y, dtype=float)
        out = O.MPResult()
        out.e.append(float(r @ r))
        while out.t < k and out.e[-1] >= eps2:
            c = np.abs(dic.Dt @ r)
            i = int(len(c) - 1 - np.argmax(c[::-1]))   # planted: last maximal index
            ci = float((dic.Dt @ r)[i])
            r = r - ci * dic.D[:, i]
            out.idx.append(i); out.coef.append(ci); out.e.append(float(r @ r))
        return out
    monkeypatch.setattr(O, "mp", bad_mp)
    assert not pin_constant_block()


def test_inverted_split_rule_caught(monkeypatch):
    def bad_split(p, n, res):
        return n > p.n_min and res.e_final < p.eps2(n)   # planted: inverted test
    monkeypatch.setattr(O, "split_decision", bad_split)
    assert not pin_split_invariant()


def pin_omp_sklearn(n=8):
    from sklearn.linear_model import orthogonal_mp
    rng = np.random.default_rng(4)
    y = rng.normal(size=n * n)
    d = O.get_dict(n)
    res = O.omp(d, y, 0.0, 10)
    x = np.zeros(d.m)
    x[res.idx] = res.coef
    return np.abs(orthogonal_mp(d.D, y, n_nonzero_coefs=10) - x).max() < 1e-10


def test_omp_pin_holds_on_unpatched_oracle():
    assert pin_omp_sklearn()


def test_omp_without_refit_caught(monkeypatch):
    """Planted: OMP that keeps MP's coefficients (no least-squares refit)."""
    monkeypatch.setattr(O, "omp", lambda dic, y, eps2, k: O.mp(dic, y, eps2, k))
    assert not pin_omp_sklearn()


def test_omp_refit_on_last_atom_only_caught(monkeypatch):
    """Planted: the refit solves only for the newest atom against the residual."""
    def bad_omp(dic, y, eps2, k):
        r = np.array(y, dtype=float)
        out = O.MPResult()
        out.e.append(float(r @ r))
        while out.t < k:
            c = dic.Dt @ r
            i = int(np.argmax(np.abs(c)))
            out.gap.append(0.0)
            ci = float(dic.D[:, i] @ r)
            r = r - ci * dic.D[:, i]
            out.idx.append(i); out.coef.append(ci); out.e.append(float(r @ r))
        return out
    monkeypatch.setattr(O, "omp", bad_omp)
    assert not pin_omp_sklearn()
