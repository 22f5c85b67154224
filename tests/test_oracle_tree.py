"""Pins of the oracle's quadtree encoder/decoder (Algorithms 1-3, Section 2.3)."""
import numpy as np
import pytest

from oracle import aqmp_oracle as O
from workloads import gradient_edges_image, piecewise_image


def _img(seed=0, n=64):
    return gradient_edges_image(n, n, seed=seed)


def _covers(nodes, h, w):
    cov = np.zeros((h, w), dtype=int)
    for nd in O.leaves(nodes):
        cov[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n] += 1
    return cov


@pytest.mark.parametrize("tol", [0.005, 0.02, 0.05])
def test_leaves_tile_image_and_split_invariant(tol):
    img = _img(1)
    p = O.Params(tol=tol, max_atoms=12, n_min=8, n_max=32)
    nodes = O.encode_channel(img, p)
    assert np.all(_covers(nodes, 64, 64) == 1)
    for nd in nodes:
        e = nd.mp.e_final
        if nd.split:
            assert nd.n > p.n_min and e >= p.eps2(nd.n)
            assert nd.mp.t == p.k(nd.n)          # R1 splits only after k steps
        else:
            assert e < p.eps2(nd.n) or nd.n == p.n_min
        assert nd.mp.t <= p.k(nd.n)


def test_children_are_original_quadrants():
    """Algorithm 2 recurses on the block b itself: a child's MP equals MP run
    directly on the child's pixels."""
    img = _img(2)
    p = O.Params(tol=0.002, max_atoms=6, n_min=8, n_max=32)
    nodes = O.encode_channel(img, p)
    assert any(nd.split for nd in nodes)
    for nd in nodes:
        y = O.unravel(img[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n])
        ref = O.mp(O.get_dict(nd.n), y, p.eps2(nd.n), p.k(nd.n))
        assert ref.idx == nd.mp.idx


def test_depth_first_child_order():
    img = _img(3)
    p = O.Params(tol=0.0, max_atoms=2, n_min=8, n_max=32)
    nodes = O.encode_channel(img, p)
    # every node splits down to 8: the first four 8x8 leaves are TL,TR,BL,BR of the first 16x16
    lv = O.leaves(nodes)
    assert [(l.x0, l.y0) for l in lv[:4]] == [(0, 0), (8, 0), (0, 8), (8, 8)]
    assert len(lv) == 64


def test_refinement_monotone_in_tolerance_and_k():
    img = piecewise_image(128, 128, seed=3)
    def leafset(tol, k):
        p = O.Params(tol=tol, max_atoms=k, n_min=8, n_max=64)
        return O.leaves(O.encode_channel(img, p))
    def refines(fine, coarse):
        for a in fine:
            if not any(b.x0 <= a.x0 and a.x0 + a.n <= b.x0 + b.n and
                       b.y0 <= a.y0 and a.y0 + a.n <= b.y0 + b.n for b in coarse):
                return False
        return True
    t1, t2 = leafset(0.01, 16), leafset(0.03, 16)
    assert refines(t1, t2) and len(t1) >= len(t2)
    k1, k2 = leafset(0.02, 8), leafset(0.02, 24)
    assert refines(k1, k2) and len(k1) >= len(k2)


def test_fixed_block_special_case():
    """N_min = N_max reduces AQMP to fixed-block MP."""
    img = _img(4)
    p = O.Params(tol=0.01, max_atoms=10, n_min=16, n_max=16)
    nodes = O.encode_channel(img, p)
    assert len(nodes) == 16 and not any(nd.split for nd in nodes)
    for nd, (x0, y0) in zip(nodes, O.top_blocks(64, 64, 16)):
        y = O.unravel(img[y0:y0 + 16, x0:x0 + 16])
        ref = O.mp(O.get_dict(16), y, (0.01 * 16) ** 2, 10)
        assert (nd.x0, nd.y0) == (x0, y0) and ref.idx == nd.mp.idx


def test_huge_tolerance_gives_no_atoms_no_splits():
    img = _img(5)
    p = O.Params(tol=1e6, max_atoms=10, n_min=8, n_max=32)
    nodes = O.encode_channel(img, p)
    assert len(nodes) == 4 and all(nd.mp.t == 0 and not nd.split for nd in nodes)
    assert np.all(O.decode(nodes, 64, 64) == 0)


def test_abs_mode_same_eps_every_level():
    p = O.Params(tol=0.3, tol_mode="abs", n_min=8, n_max=32)
    assert p.eps2(32) == p.eps2(8) == pytest.approx(0.09)
    q = O.Params(tol=0.02, tol_mode="rms")
    assert q.eps2(16) == pytest.approx((0.32) ** 2)


def test_split_rules_differ_only_when_last_atom_meets_target():
    img = piecewise_image(128, 128, seed=7)
    base = dict(tol=0.02, max_atoms=8, n_min=8, n_max=32)
    n1 = O.encode_channel(img, O.Params(split_rule="r1", **base))
    n2 = O.encode_channel(img, O.Params(split_rule="r2", **base))
    k = base["max_atoms"]
    for nodes, rule in ((n1, "r1"), (n2, "r2")):
        for nd in nodes:
            if nd.n > base["n_min"]:
                want = (nd.mp.e_final >= nd.eps2) if rule == "r1" else (nd.mp.t >= k)
                assert nd.split == want
    # where the k-th step met the target, R2 splits and R1 does not
    for nd in n2:
        if nd.split and nd.mp.e_final < nd.eps2:
            assert nd.mp.t == k


def test_decode_exact_with_full_basis():
    """With eps = 0 in ABS mode and k = N^2 on an orthonormal basis every leaf
    is recovered exactly; the decoder places blocks at their positions."""
    img = _img(6, 32)
    p = O.Params(tol=0.0, tol_mode="abs", max_atoms=64, n_min=8, n_max=8, families=O.DCT)
    nodes = O.encode_channel(img, p)
    rec = O.decode(nodes, 32, 32, families=O.DCT)
    assert np.abs(rec - img).max() < 1e-12
    # a transposed block placement would not reproduce a non-symmetric image
    assert np.abs(rec.T - img).max() > 1e-3


def test_decode_matches_residual_energy():
    """Per leaf, ||block - decoded block||^2 equals the MP residual energy."""
    img = _img(7)
    p = O.Params(tol=0.02, max_atoms=16, n_min=8, n_max=32)
    nodes = O.encode_channel(img, p)
    rec = O.decode(nodes, 64, 64)
    for nd in O.leaves(nodes):
        d = img[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n] - rec[nd.y0:nd.y0 + nd.n, nd.x0:nd.x0 + nd.n]
        assert abs(float(np.sum(d * d)) - nd.mp.e_final) < 1e-12 * max(1.0, nd.norm2)
    mse = np.mean((img - rec) ** 2)
    assert O.psnr(img, rec) == pytest.approx(10 * np.log10(1 / mse))


def test_non_multiple_plane_is_edge_padded():
    """A plane that is not a multiple of N_max is coded as its edge-padded
    version (last row and column repeated), and the decode keeps the plane's
    own pixels."""
    rng = np.random.default_rng(9)
    img = rng.uniform(size=(40, 52))
    p = O.Params(tol=0.03, max_atoms=6, n_min=8, n_max=16)
    padded = np.vstack([img, np.repeat(img[-1:], 8, axis=0)])
    padded = np.hstack([padded, np.repeat(padded[:, -1:], 12, axis=1)])
    assert padded.shape == (48, 64)
    assert np.array_equal(O.pad_edge(img, 16), padded)
    a = O.encode_channel(img, p)
    b = O.encode_channel(padded, p)
    assert [(n.x0, n.y0, n.n, n.mp.idx, n.split) for n in a] == [(n.x0, n.y0, n.n, n.mp.idx, n.split) for n in b]
    ra, rb = O.decode(a, 40, 52), O.decode(b, 48, 64)
    assert ra.shape == (40, 52)
    assert np.array_equal(ra, rb[:40, :52])
    assert len(O.top_blocks(40, 52, 16)) == 3 * 4


def test_multiple_plane_unchanged_by_padding():
    img = np.random.default_rng(10).uniform(size=(32, 48))
    assert O.pad_edge(img, 16) is not img and np.array_equal(O.pad_edge(img, 16), img)
