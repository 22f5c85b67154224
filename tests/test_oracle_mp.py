"""Pins of the oracle's Matching Pursuit (Section 2.2, eq. (1)-(2), steps (a)-(d))."""
import itertools

import numpy as np
import pytest

from oracle import aqmp_oracle as O


def _brute_step(d, r):
    """Scalar-loop scan of every atom: the best |<r, phi_a>|, lowest index first."""
    best, best_a = -1.0, -1
    for a in range(d.shape[1]):
        s = 0.0
        for j in range(d.shape[0]):
            s += r[j] * d[j, a]
        if abs(s) > best + 1e-12:
            best, best_a = abs(s), a
    return best_a


@pytest.mark.parametrize("seed", range(6))
def test_energy_identity(seed):
    """||r_{t+1}||^2 = ||r_t||^2 - c_t^2 for unit atoms (rank-1 update of step (c))."""
    rng = np.random.default_rng(seed)
    n = [4, 8, 16][seed % 3]
    y = rng.normal(size=n * n)
    res = O.mp(O.get_dict(n), y, 0.0, 40)
    assert res.t == 40 and res.stop == "sparsity"
    for t in range(res.t):
        lhs, rhs = res.e[t + 1], res.e[t] - res.coef[t] ** 2
        assert abs(lhs - rhs) <= 1e-12 * res.e[0]
        assert res.e[t + 1] <= res.e[t] + 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_4x4(seed):
    """Every step's choice equals an explicit scan of all 32 atoms of D_4."""
    rng = np.random.default_rng(10 + seed)
    d = O.dictionary(4)
    y = rng.uniform(0, 1, size=16)
    res = O.mp(O.get_dict(4), y, 0.0, 12)
    r = y.copy()
    for i, c in zip(res.idx, res.coef):
        a = _brute_step(d, r)
        assert a == i
        assert abs(c - float(r @ d[:, a])) < 1e-13
        r = r - c * d[:, a]


@pytest.mark.parametrize("seed", range(4))
def test_one_step_is_best_single_term(seed):
    """For k = 1 MP's atom minimises ||y - c phi_a|| over all atoms and all c
    (argmax |c| <=> argmin residual for unit atoms), found here exhaustively."""
    rng = np.random.default_rng(20 + seed)
    n = 4
    d = O.dictionary(n)
    y = rng.normal(size=n * n)
    res = O.mp(O.get_dict(n), y, 0.0, 1)
    errs = []
    for a in range(d.shape[1]):
        phi = d[:, a]
        c = np.linalg.lstsq(phi[:, None], y, rcond=None)[0][0]
        errs.append(float(np.sum((y - c * phi) ** 2)))
    errs = np.array(errs)
    best = np.min(errs)
    winners = np.nonzero(errs <= best + 1e-12)[0]
    assert res.idx[0] == winners.min()


@pytest.mark.parametrize("fam,n", list(itertools.product([O.DCT, O.HAAR], [4, 8])))
def test_parseval_and_exact_recovery_orthonormal(fam, n):
    """On an orthonormal-only dictionary MP with k = N^2 and eps = 0 recovers the
    signal exactly, takes each atom once, and its coefficients are the
    transform coefficients in decreasing magnitude (Parseval)."""
    rng = np.random.default_rng(n + fam)
    y = rng.normal(size=n * n)
    dic = O.get_dict(n, fam)
    res = O.mp(dic, y, 0.0, n * n)
    assert res.t == n * n
    assert res.e_final <= 1e-24 * max(1.0, res.e[0]) or res.e_final < 1e-20
    assert sorted(res.idx) == list(range(n * n))
    coefs = np.array(res.coef)
    assert abs(np.sum(coefs ** 2) - y @ y) < 1e-12 * (y @ y)
    tc = dic.D.T @ y
    assert np.allclose(coefs, tc[np.array(res.idx)], atol=1e-12)
    mags = np.abs(coefs)
    assert np.all(mags[:-1] >= mags[1:] - 1e-12)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_single_atom_signal(n):
    dic = O.get_dict(n)
    for a in [1, n + 3, n * n + 5, 2 * n * n - 1]:
        y = 0.7 * dic.D[:, a]
        res = O.mp(dic, y, 1e-20, 10)
        assert res.idx == [a] and abs(res.coef[0] - 0.7) < 1e-14
        assert res.e_final < 1e-20


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_constant_block(n):
    """A constant block needs one atom: the lowest-index DC atom with c = N v."""
    v = 0.37
    y = np.full(n * n, v)
    res = O.mp(O.get_dict(n), y, 1e-12, 8)
    assert res.idx == [0]
    assert abs(res.coef[0] - n * v) < 1e-13
    assert res.stop == "accuracy"


def test_initial_stop_and_zero_signal():
    dic = O.get_dict(8)
    y = np.full(64, 0.01)
    res = O.mp(dic, y, 1.0, 5)            # ||y||^2 = 0.0064 < 1: no iteration
    assert res.t == 0 and res.stop == "accuracy"
    res = O.mp(dic, np.zeros(64), 0.0, 5)
    assert res.t == 0 and res.stop == "zero"


def test_reselection_gives_new_record():
    """MP may select the same atom again (k counts iterations)."""
    dic = O.get_dict(4)
    rng = np.random.default_rng(5)
    found = False
    for _ in range(50):
        res = O.mp(dic, rng.normal(size=16), 0.0, 40)
        if len(set(res.idx)) < len(res.idx):
            found = True
            assert res.t == 40
            break
    assert found


def test_gap_is_over_distinct_atoms():
    """The DC duplicate pair ties exactly; the reported gap skips the copy."""
    n = 8
    dic = O.get_dict(n)
    y = np.full(n * n, 0.5)
    y[0] += 1e-3
    res = O.mp(dic, y, 0.0, 1)
    assert res.idx == [0]
    c = np.abs(dic.Dt @ y)
    assert c[0] == c[n * n]
    assert res.gap[0] > 0.5
