"""Pins of the oracle's Orthogonal Matching Pursuit (Section 2.2: the solver
the authors' code ran, scikit-learn's OrthogonalMatchingPursuit).

The library routine ``sklearn.linear_model.orthogonal_mp`` (Cholesky-updated
OMP, first maximal index on ties) fixes both stopping forms: a number of
atoms, and a squared-residual tolerance.  The remaining pins are properties
of least squares that hold for any correct OMP.
"""
import numpy as np
import pytest
from sklearn.linear_model import orthogonal_mp

from oracle import aqmp_oracle as O
from workloads import piecewise_image


def _signals(n, count, seed):
    rng = np.random.default_rng(seed)
    out = [rng.normal(size=n * n) for _ in range(count)]
    img = piecewise_image(4 * n, 4 * n, seed=seed)
    out += [O.unravel(img[y:y + n, x:x + n]) for (x, y) in ((0, 0), (n, 2 * n), (3 * n, n))]
    return out


def _full(res, m):
    x = np.zeros(m)
    x[res.idx] = res.coef
    return x


def _merge(d, x):
    """Coefficients with every group of bit-identical atoms (the two constant
    atoms) summed onto its representative: scikit-learn swaps selected columns
    to the front of its working matrix, so on an exact tie between identical
    atoms its first maximum is taken in a permuted order."""
    out = np.zeros_like(x)
    np.add.at(out, d.rep, x)
    return out


def _order_from_path(path):
    """Selection order from scikit-learn's coefficient path (column t holds the
    coefficients after t + 1 selections)."""
    order = []
    for t in range(path.shape[1]):
        new = [i for i in np.nonzero(path[:, t])[0] if i not in order]
        assert len(new) == 1
        order += new
    return order


@pytest.mark.parametrize("n", [4, 8, 16])
def test_omp_matches_sklearn_fixed_sparsity(n):
    d = O.get_dict(n)
    for y in _signals(n, 3, seed=n):
        k = min(12, n * n // 2)
        res = O.omp(d, y, 0.0, k)
        assert res.stop == "sparsity" and res.t == k
        path = orthogonal_mp(d.D, y, n_nonzero_coefs=k, return_path=True)
        assert [int(d.rep[i]) for i in _order_from_path(path)] == [int(d.rep[i]) for i in res.idx]
        assert np.abs(_merge(d, path[:, -1]) - _merge(d, _full(res, d.m))).max() < 1e-10 * max(1.0, np.abs(path).max())


@pytest.mark.parametrize("n", [4, 8])
def test_omp_matches_sklearn_tolerance(n):
    d = O.get_dict(n)
    for y in _signals(n, 2, seed=10 + n):
        eps2 = 0.05 * float(y @ y)
        res = O.omp(d, y, eps2, 10 ** 6)
        assert res.stop == "accuracy"
        ref = _merge(d, orthogonal_mp(d.D, y, tol=eps2))
        mine = _merge(d, _full(res, d.m))
        assert sorted(np.nonzero(ref)[0]) == sorted(np.nonzero(mine)[0])
        assert np.abs(ref - mine).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_omp_residual_orthogonal_and_monotone():
    d = O.get_dict(8)
    for y in _signals(8, 2, seed=3):
        res = O.omp(d, y, 0.0, 20)
        r = y - d.D[:, res.idx] @ np.array(res.coef)
        assert np.abs(d.D[:, res.idx].T @ r).max() < 1e-12 * np.linalg.norm(y)
        assert abs(float(r @ r) - res.e_final) < 1e-12 * float(y @ y)
        assert all(res.e[t + 1] <= res.e[t] * (1 + 1e-12) for t in range(res.t))
        assert len(set(res.idx)) == res.t


@pytest.mark.parametrize("fam", [O.DCT, O.HAAR])
def test_omp_equals_mp_on_an_orthonormal_basis(fam):
    """With one family the atoms are orthonormal: the least-squares refit
    leaves every earlier coefficient unchanged, so OMP and MP coincide."""
    d = O.get_dict(8, fam)
    for y in _signals(8, 2, seed=5):
        a = O.omp(d, y, 1e-3, 24)
        b = O.mp(d, y, 1e-3, 24)
        assert a.idx == b.idx
        assert np.abs(np.array(a.coef) - np.array(b.coef)).max() < 1e-12 * np.linalg.norm(y)


def test_omp_never_worse_than_mp_after_the_same_atoms():
    """For MP's own support, the least-squares fit is at least as good."""
    d = O.get_dict(8)
    for y in _signals(8, 2, seed=6):
        b = O.mp(d, y, 0.0, 12)
        s = sorted(set(b.idx))
        x = np.linalg.lstsq(d.D[:, s], y, rcond=None)[0]
        assert float(np.sum((y - d.D[:, s] @ x) ** 2)) <= b.e_final * (1 + 1e-12)


def test_omp_encoder_tree():
    img = piecewise_image(64, 64, seed=8)
    p = O.Params(tol=0.02, max_atoms=12, n_min=8, n_max=32, solver="omp")
    nodes = O.encode_channel(img, p)
    cover = np.zeros((64, 64), dtype=int)
    for nd in nodes:
        if nd.split:
            assert nd.mp.e_final >= p.eps2(nd.n) and nd.n > p.n_min
        else:
            assert nd.mp.e_final < p.eps2(nd.n) or nd.n == p.n_min
            cover[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n] += 1
    assert (cover == 1).all()
    rec = O.decode(nodes, 64, 64)
    for nd in O.leaves(nodes):
        blk = img[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n] - rec[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n]
        assert abs(float(np.sum(blk ** 2)) - nd.mp.e_final) < 1e-10 * max(1.0, nd.norm2)
