"""Self-test of the node-by-node parity checker on the CPU: an exact copy of
the oracle's tree passes; planted differences are reported."""
import copy

import numpy as np

from oracle import aqmp_oracle as O
from tests import parity_util as PU
from workloads import gradient_edges_image


class _Exp:
    def __init__(self, nodes, job=0):
        rows, idx, coef = [], [], []
        for nd in nodes:
            rows.append((job, nd.x0, nd.y0, nd.n, nd.mp.t, 1 if nd.split else 0, len(idx), nd.mp.e_final))
            idx += nd.mp.idx
            coef += nd.mp.coef
        from paper_2605_09190_amd.aqmp import LEAF_DTYPE
        self.leaves = np.array(rows, dtype=LEAF_DTYPE)
        self.atom_idx = np.array(idx, dtype=np.int32)
        self.coef = np.array(coef)


def _tree():
    img = gradient_edges_image(64, 64, seed=2)
    p = O.Params(tol=0.02, max_atoms=10, n_min=8, n_max=32)
    return img, p, O.encode_channel(img, p)


def test_identical_tree_passes():
    img, p, nodes = _tree()
    rep = PU.compare_job(img, nodes, PU.gpu_nodes_by_key(_Exp(nodes), 0), 1e-5, p.n_max)
    assert rep.ok() and rep.nodes == len(nodes) and rep.max_coef_err == 0


def test_wrong_atom_reported():
    img, p, nodes = _tree()
    bad = copy.deepcopy(nodes)
    nd = next(n for n in bad if n.mp.t > 3 and min(n.mp.gap[:4]) > 1e-3)
    nd.mp.idx[2] = (nd.mp.idx[2] + 1) % 128
    rep = PU.compare_job(img, nodes, PU.gpu_nodes_by_key(_Exp(bad), 0), 1e-5, p.n_max)
    assert not rep.ok() and rep.failures[0][0] == "atom mismatch"


def test_coefficient_error_reported():
    img, p, nodes = _tree()
    bad = copy.deepcopy(nodes)
    bad[0].mp.coef[0] *= 1 + 1e-3
    rep = PU.compare_job(img, nodes, PU.gpu_nodes_by_key(_Exp(bad), 0), 1e-5, p.n_max)
    assert not rep.ok() and rep.failures[0][0] == "coef"
    rep = PU.compare_job(img, nodes, PU.gpu_nodes_by_key(_Exp(bad), 0), 2e-3, p.n_max)
    assert rep.ok()


def test_missing_subtree_reported():
    img, p, nodes = _tree()
    split = next(n for n in nodes if n.split)
    bad = [n for n in copy.deepcopy(nodes)
           if not (n.n < split.n and split.x0 <= n.x0 < split.x0 + split.n and split.y0 <= n.y0 < split.y0 + split.n)]
    for n in bad:
        if (n.x0, n.y0, n.n) == (split.x0, split.y0, split.n):
            n.split = False
    rep = PU.compare_job(img, nodes, PU.gpu_nodes_by_key(_Exp(bad), 0), 1e-5, p.n_max)
    assert not rep.ok()
    kinds = {f[0] for f in rep.failures}
    assert "split" in kinds and "missing node on GPU" in kinds


def test_duplicate_dc_choice_is_reported():
    """A constant block ties the two DC atoms exactly; the lowest index must win,
    so a choice of the Haar copy is a tie-break error, not a near-tie."""
    img = np.full((8, 8), 0.5)
    p = O.Params(tol=1e-9, tol_mode="abs", max_atoms=1, n_min=8, n_max=8)
    nodes = O.encode_channel(img, p)
    assert nodes[0].mp.idx == [0] and nodes[0].mp.gap[0] > 0.5
    # the gap is over distinct atoms, so choosing atom 64 (the Haar copy) is
    # not a near-tie in the oracle's terms: it must be reported
    bad = copy.deepcopy(nodes)
    bad[0].mp.idx[0] = 64
    rep = PU.compare_job(img, nodes, PU.gpu_nodes_by_key(_Exp(bad), 0), 1e-5, 8)
    assert not rep.ok()
