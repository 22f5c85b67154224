"""Result export of the encoder library (the read calls of the boundary).

The library gathers a code's visited nodes on the device and sorts them into
the canonical order: job, then top-level block in raster order over the
padded plane, then depth-first with children TL, TR, BL, BR (Alg. 2), i.e.
Morton order of the node's corner inside its top-level block with the larger
node first.  Checked here against that order computed independently on the
host, for all three schedules and mixed jobs; the leaf export must be the
visited-node export restricted to leaves, atom for atom; and the tree must
match the oracle's (Alg. 2) node for node, in the oracle's own depth-first
order.
"""
import sys

import numpy as np
import pytest

from oracle import aqmp_oracle as O
from workloads import piecewise_image, gradient_edges_image

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09190_amd import aqmp
    return aqmp


@pytest.fixture(scope="module")
def dic(A):
    d = A.Dictionary(4, 64)
    yield d
    d.free()


def _dev(img):
    import torch
    return torch.from_numpy(np.ascontiguousarray(img)).to(torch.float32).cuda()


def _interleave(x, y):
    m = 0
    for b in range(8):
        m |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1)
    return m


def _order_key(rec, shapes, nmax):
    job, x0, y0, n = int(rec["job"]), int(rec["x0"]), int(rec["y0"]), int(rec["n"])
    h, w = shapes[job]
    nm = nmax[job]
    cols = -(-w // nm)
    top = (y0 // nm) * cols + x0 // nm
    return (job, top, _interleave(x0 % nm, y0 % nm), -n)


CHANS = [((70, 100), 31), ((128, 192), 32), ((64, 64), 33)]
PARAMS = [dict(tol=0.02, max_atoms=12, n_min=4, n_max=32), dict(tol=0.015, max_atoms=20, n_min=8, n_max=64),
          dict(tol=0.03, max_atoms=6, n_min=4, n_max=16)]
JOBS = [(0, 0), (1, 1), (2, 2), (1, 0), (0, 2)]


def _images():
    out = []
    for (h, w), seed in CHANS:
        out.append(piecewise_image(h, w, seed=seed) if seed % 2 else gradient_edges_image(h, w, seed=seed))
    return out


@pytest.mark.parametrize("schedule", [0, 1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_export_canonical_order_and_consistency(A, dic, schedule, prec):
    chans = _images()
    code = A.Code(dic, [_dev(c) for c in chans], PARAMS, JOBS, precision=prec, schedule=schedule)
    shapes = [chans[ci].shape for ci, _ in JOBS]
    nmax = [PARAMS[pi]["n_max"] for _, pi in JOBS]
    nodes = code.export_nodes()
    leaves = code.export()
    _say("schedule", schedule, "prec", prec, "nodes", len(nodes.leaves), "leaves", len(leaves.leaves))
    for e in (nodes, leaves):
        keys = [_order_key(r, shapes, nmax) for r in e.leaves]
        assert all(a < b for a, b in zip(keys, keys[1:])), "not in canonical order"
        off = np.concatenate([[0], np.cumsum(e.leaves["n_atoms"])[:-1]])
        assert np.array_equal(e.leaves["atom_off"], off)
        assert int(e.leaves["n_atoms"].sum()) == len(e.atom_idx) == len(e.coef)
    # the leaf export is the node export without the split nodes
    keep = (nodes.leaves["flags"] & 1) == 0
    assert keep.sum() == len(leaves.leaves)
    for f in ("job", "x0", "y0", "n", "n_atoms", "flags", "resid_sq"):
        assert np.array_equal(nodes.leaves[f][keep], leaves.leaves[f]), f
    sel = np.concatenate([np.arange(o, o + k) for o, k, s in zip(nodes.leaves["atom_off"], nodes.leaves["n_atoms"],
                                                                   keep) if s] or [np.zeros(0, int)])
    assert np.array_equal(nodes.atom_idx[sel], leaves.atom_idx)
    assert np.array_equal(nodes.coef[sel], leaves.coef)
    # sizes and statistics agree with the export
    nl, na = code.sizes()
    assert (nl, na) == (len(leaves.leaves), len(leaves.atom_idx))
    st = code.stats()
    assert int(sum(st["nodes"])) == len(nodes.leaves)
    assert int(st["iters_executed"]) == len(nodes.atom_idx)
    # every top-level block of every job is tiled exactly once by its leaves
    for j, (h, w) in enumerate(shapes):
        nm = nmax[j]
        ph, pw = -(-h // nm) * nm, -(-w // nm) * nm
        cover = np.zeros((ph, pw), dtype=np.int32)
        for r in leaves.leaves[leaves.leaves["job"] == j]:
            cover[r["y0"]:r["y0"] + r["n"], r["x0"]:r["x0"] + r["n"]] += 1
        assert (cover == 1).all(), f"job {j}"
    code.free()


def test_export_order_equals_oracle_depth_first(A, dic):
    """The Gram solver (FP64) on one padded plane: the node export equals the
    oracle's visited nodes (N, corner, split flag) in the oracle's own
    depth-first order."""
    img = piecewise_image(70, 100, seed=31)
    p = dict(tol=0.02, max_atoms=12, n_min=4, n_max=32)
    code = A.Code(dic, [_dev(img)], [p], [(0, 0)], schedule=1, solver=A.SOLVER_GRAM)
    e = code.export_nodes()
    code.free()
    onodes = O.encode_channel(img, O.Params.from_dict(p))
    want = [(nd.n, nd.x0, nd.y0, bool(nd.split)) for nd in onodes]
    got = [(int(r["n"]), int(r["x0"]), int(r["y0"]), bool(r["flags"] & 1)) for r in e.leaves]
    assert got == want


def test_export_empty_and_repeat(A, dic):
    """Reads before and after a re-encode: the cache is rebuilt, the device
    buffers are reused, the results are identical."""
    img = _dev(piecewise_image(64, 64, seed=5))
    p = dict(tol=0.02, max_atoms=8, n_min=8, n_max=32)
    code = A.Code(dic, [img], [p], [(0, 0)], precision=1, schedule=1)
    e1 = code.export_nodes()
    code.reencode([img])
    e2 = code.export_nodes()
    assert e1.leaves.tobytes() == e2.leaves.tobytes()
    assert e1.atom_idx.tobytes() == e2.atom_idx.tobytes()
    assert e1.coef.tobytes() == e2.coef.tobytes()
    code.free()
    # a tolerance every block meets at once: zero-atom leaves, no atoms at all
    code = A.Code(dic, [img], [dict(tol=10.0, max_atoms=8, n_min=8, n_max=32)], [(0, 0)], schedule=1)
    e = code.export()
    assert len(e.leaves) == 4 and len(e.atom_idx) == 0
    assert (e.leaves["n_atoms"] == 0).all() and (e.leaves["n"] == 32).all()
    code.free()


def test_export_capacity_error_writes_nothing(A, dic):
    """Buffers one record or one atom too small: AQMP_E_CAPACITY, nothing
    written, and the same call with the right sizes still succeeds."""
    import ctypes as C
    img = _dev(piecewise_image(64, 128, seed=6))
    code = A.Code(dic, [img], [dict(tol=0.02, max_atoms=8, n_min=8, n_max=32)], [(0, 0)], precision=1, schedule=1)
    nl, na = code.sizes()
    assert nl > 0 and na > 0
    for cl, ca in ((nl - 1, na), (nl, na - 1)):
        leaves = np.zeros(nl, dtype=A.LEAF_DTYPE)
        leaves["job"] = -7
        idx = np.full(na, -7, dtype=np.int32)
        coef = np.full(na, -7.0)
        rc = A.lib.aqmp_code_export(code.h, leaves.ctypes.data_as(C.c_void_p), idx.ctypes.data_as(C.c_void_p),
                                    coef.ctypes.data_as(C.c_void_p), C.c_int64(cl), C.c_int64(ca))
        assert rc == A.E_CAPACITY
        assert (leaves["job"] == -7).all() and (idx == -7).all() and (coef == -7.0).all()
    e = code.export()
    assert len(e.leaves) == nl and len(e.atom_idx) == na
    code.free()
