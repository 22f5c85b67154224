"""Gram solver (exact reformulation of MP through the dictionary's Gram
matrix, FP64 throughout) vs the FP64 oracle, node by node, through the C ABI.

Same comparison rules as the dense forms (identical trees and atom sequences
except counted near-ties); coefficients within 1e-9 relative (floored at
1e-3 ||y||): the only differences from the oracle are FP64 rounding order,
accumulated over at most k Gram updates of O(N) rounding each.
"""
import sys

import numpy as np
import pytest

from oracle import aqmp_oracle as O
from tests import parity_util as PU
from workloads import workload, gradient_edges_image, piecewise_image

pytestmark = pytest.mark.gpu

GRAM_TOL = 1e-9


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


def _dev(img, dtype="f32"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(img))
    t = t.to(torch.float32 if dtype == "f32" else torch.float64)
    return t.cuda()


def _run(A, dic, chans, params, jobs, sched, dtype="f32", blocks_per_job=None, families=O.DCT | O.HAAR):
    imgs = [_dev(c, dtype) for c in chans]
    code = A.Code(dic, imgs, params, jobs, schedule=sched, solver=A.SOLVER_GRAM)
    exp = code.export_nodes()
    rep = PU.Report()
    for j, (ci, pi) in enumerate(jobs):
        p = O.Params.from_dict(dict(params[pi], families=families))
        blocks = None if blocks_per_job is None else blocks_per_job[j]
        onodes = O.encode_channel(chans[ci], p, blocks=blocks)
        PU.compare_job(chans[ci], onodes, PU.gpu_nodes_by_key(exp, j), GRAM_TOL, p.n_max, families=families, rep=rep)
    code.free()
    return rep


@pytest.mark.parametrize("sched", [0, 1, 2])
def test_gram_c0_full_parity(A, dic, sched):
    w = workload("c0")
    _say("gram c0", sched)
    rep = _run(A, dic, w["channels"], w["params"], w["jobs"], sched)
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.nodes > 10


def test_gram_c1_sampled_parity(A, dic):
    """512 x 512, blocks 64 -> 8: every Gram level (16, 32, 64) runs."""
    w = workload("c1")
    rng = np.random.default_rng(11)
    tops = O.top_blocks(512, 512, 64)
    sample = [tops[i] for i in sorted(rng.choice(len(tops), size=8, replace=False))]
    _say("gram c1 sample", sample)
    rep = _run(A, dic, w["channels"], w["params"], [(0, 0)], 1, blocks_per_job=[sample])
    _say(rep.summary())
    assert rep.ok(), rep.summary()


def test_gram_mixed_jobs_small_sizes(A, dic):
    """Several jobs with different block ranges (4..32), k, tolerances, both
    split rules and an FP64 input plane; k = 70 makes nodes cross the
    64-record flush boundary of the pursuit kernel."""
    chans = [gradient_edges_image(64, 64, seed=3), piecewise_image(64, 128, seed=4)]
    params = [dict(tol=0.03, max_atoms=8, n_min=4, n_max=16),
              dict(tol=0.01, max_atoms=20, n_min=8, n_max=32, split_rule="r2"),
              dict(tol=0.5, tol_mode="abs", max_atoms=40, n_min=4, n_max=32),
              dict(tol=1e-4, max_atoms=70, n_min=16, n_max=32)]
    jobs = [(0, 0), (1, 1), (0, 2), (1, 0), (1, 3)]
    _say("gram mixed")
    rep = _run(A, dic, chans, params, jobs, 1, dtype="f64")
    _say(rep.summary())
    assert rep.ok(), rep.summary()


@pytest.mark.parametrize("fam", ["dct", "haar"])
def test_gram_single_family_dictionary(A, fam):
    """With one family the Gram column is a pure Kronecker delta."""
    F = O.DCT if fam == "dct" else O.HAAR
    d = A.Dictionary(8, 64, families=(A.DCT if fam == "dct" else A.HAAR))
    img = piecewise_image(128, 128, seed=21)
    p = dict(tol=0.02, max_atoms=16, n_min=8, n_max=64)
    _say("gram single family", fam)
    rep = _run(A, d, [img], [p], [(0, 0)], 1, families=F)
    d.free()
    _say(rep.summary())
    assert rep.ok(), rep.summary()


def test_gram_degenerate_blocks(A, dic):
    """A constant image (one DC atom per top block, then exact zero residual),
    an all-zero image (first stop test) and k = 0 (sparsity stop before any
    step)."""
    const = np.full((128, 128), 0.37)
    zero = np.zeros((64, 64))
    rng = np.random.default_rng(5)
    noise = rng.standard_normal((64, 64)) * 0.1
    params = [dict(tol=1e-6, tol_mode="abs", max_atoms=8, n_min=16, n_max=64),
              dict(tol=0.01, max_atoms=0, n_min=16, n_max=64)]
    rep = _run(A, dic, [const, zero, noise], params, [(0, 0), (1, 0), (2, 1), (2, 0)], 1, dtype="f64")
    _say(rep.summary())
    assert rep.ok(), rep.summary()


def test_gram_full_size_sampled_parity(A, dic):
    """The benchmark workload at its full size through the Gram solver, on a
    seeded sample of top-level blocks per job."""
    w = workload("c3")
    rng = np.random.default_rng(77)
    tops = O.top_blocks(2048, 2048, 64)
    samples = [[tops[i] for i in sorted(rng.choice(len(tops), size=3, replace=False))] for _ in w["jobs"]]
    _say("gram full size", samples)
    rep = _run(A, dic, w["channels"], w["params"], w["jobs"], 1, blocks_per_job=samples)
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.nodes >= 9


def test_gram_matches_dense_psnr_and_replays(A, dic):
    """Gram and dense FP32 solvers give the same reconstruction quality on the
    512 x 512 workload, and graph replays of the Gram encode are bit-identical."""
    import torch
    w = workload("c1")
    img = w["channels"][0]
    imgs = [_dev(img)]
    out = {}
    for solver in (A.SOLVER_DENSE, A.SOLVER_GRAM):
        code = A.Code(dic, imgs, w["params"], [(0, 0)], precision=0, schedule=1, solver=solver)
        rec = torch.zeros(512, 512, dtype=torch.float64, device="cuda")
        code.decode(0, rec)
        torch.cuda.synchronize()
        out[solver] = O.psnr(img, rec.cpu().numpy())
        if solver == A.SOLVER_GRAM:
            e1 = code.export_nodes()
            for _ in range(2):
                code.reencode(imgs)
                e2 = code.export_nodes()
                assert e1.leaves.tobytes() == e2.leaves.tobytes()
                assert e1.atom_idx.tobytes() == e2.atom_idx.tobytes()
                assert e1.coef.tobytes() == e2.coef.tobytes()
        code.free()
    _say("psnr dense/gram", out)
    assert abs(out[A.SOLVER_DENSE] - out[A.SOLVER_GRAM]) < 0.01
