"""OMP solver (Orthogonal Matching Pursuit with least-squares refits, FP64)
vs the oracle's OMP, node by node, through the C ABI.

Same comparison rules as the other solvers (identical trees and atom
sequences except counted near-ties, replayed with OMP).  Coefficients are the
final least-squares values; they are compared within 1e-8 relative (floored
at 1e-3 ||y||): both sides solve the same small least-squares problems in
FP64 by different factorisations (Householder on the CPU, an updated inverse
Cholesky factor on the GPU), so their differences scale with the condition
of the selected atoms' Gram matrix.
"""
import sys

import numpy as np
import pytest

from oracle import aqmp_oracle as O
from tests import parity_util as PU
from workloads import workload, gradient_edges_image, piecewise_image

pytestmark = pytest.mark.gpu

OMP_TOL = 1e-8


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
    code = A.Code(dic, imgs, params, jobs, schedule=sched, solver=A.SOLVER_OMP)
    exp = code.export_nodes()
    rep = PU.Report()
    for j, (ci, pi) in enumerate(jobs):
        p = O.Params.from_dict(dict(params[pi], families=families, solver="omp"))
        blocks = None if blocks_per_job is None else blocks_per_job[j]
        onodes = O.encode_channel(chans[ci], p, blocks=blocks)
        PU.compare_job(chans[ci], onodes, PU.gpu_nodes_by_key(exp, j), OMP_TOL, p.n_max, families=families,
                       rep=rep, solver="omp")
    code.free()
    return rep


@pytest.mark.parametrize("sched", [0, 1, 2])
def test_omp_c0_full_parity(A, dic, sched):
    w = workload("c0")
    _say("omp c0", sched)
    rep = _run(A, dic, w["channels"], w["params"], w["jobs"], sched)
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.nodes > 10


def test_omp_c1_sampled_parity(A, dic):
    """512 x 512, blocks 64 -> 8, k = 32."""
    w = workload("c1")
    rng = np.random.default_rng(12)
    tops = O.top_blocks(512, 512, 64)
    sample = [tops[i] for i in sorted(rng.choice(len(tops), size=6, replace=False))]
    _say("omp c1 sample", sample)
    rep = _run(A, dic, w["channels"], w["params"], [(0, 0)], 1, blocks_per_job=[sample])
    _say(rep.summary())
    assert rep.ok(), rep.summary()


def test_omp_mixed_jobs_small_sizes(A, dic):
    """Block ranges 4..32, both split rules, ABS tolerance, an FP64 plane, and
    k = 64 (the largest the OMP solver takes) at N = 16..32."""
    chans = [gradient_edges_image(64, 64, seed=3), piecewise_image(64, 128, seed=4)]
    params = [dict(tol=0.03, max_atoms=8, n_min=4, n_max=16),
              dict(tol=0.01, max_atoms=20, n_min=8, n_max=32, split_rule="r2"),
              dict(tol=0.5, tol_mode="abs", max_atoms=40, n_min=4, n_max=32),
              dict(tol=1e-3, max_atoms=64, n_min=16, n_max=32)]
    jobs = [(0, 0), (1, 1), (0, 2), (1, 0), (1, 3)]
    _say("omp mixed")
    rep = _run(A, dic, chans, params, jobs, 1, dtype="f64")
    _say(rep.summary())
    assert rep.ok(), rep.summary()


@pytest.mark.parametrize("fam", ["dct", "haar"])
def test_omp_single_family_dictionary(A, fam):
    """With one orthonormal family OMP reduces to MP: no cross terms."""
    F = O.DCT if fam == "dct" else O.HAAR
    d = A.Dictionary(8, 64, families=(A.DCT if fam == "dct" else A.HAAR))
    img = piecewise_image(128, 128, seed=21)
    p = dict(tol=0.02, max_atoms=16, n_min=8, n_max=64)
    _say("omp single family", fam)
    rep = _run(A, d, [img], [p], [(0, 0)], 1, families=F)
    d.free()
    _say(rep.summary())
    assert rep.ok(), rep.summary()


def test_omp_degenerate_blocks(A, dic):
    """Constant image (one constant atom, exact zero residual), all-zero image,
    and k = 0."""
    const = np.full((128, 128), 0.37)
    zero = np.zeros((64, 64))
    rng = np.random.default_rng(5)
    noise = rng.standard_normal((64, 64)) * 0.1
    params = [dict(tol=1e-6, tol_mode="abs", max_atoms=8, n_min=16, n_max=64),
              dict(tol=0.01, max_atoms=0, n_min=16, n_max=64)]
    rep = _run(A, dic, [const, zero, noise], params, [(0, 0), (1, 0), (2, 1), (2, 0)], 1, dtype="f64")
    _say(rep.summary())
    assert rep.ok(), rep.summary()


def test_omp_full_size_sampled_parity(A, dic):
    """The benchmark workload at its full size through the OMP solver, on a
    seeded sample of top-level blocks per job."""
    w = workload("c3")
    rng = np.random.default_rng(78)
    tops = O.top_blocks(2048, 2048, 64)
    samples = [[tops[i] for i in sorted(rng.choice(len(tops), size=3, replace=False))] for _ in w["jobs"]]
    _say("omp full size", samples)
    rep = _run(A, dic, w["channels"], w["params"], w["jobs"], 1, blocks_per_job=samples)
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.nodes >= 9


def test_omp_rejects_k_above_limit(A, dic):
    img = _dev(piecewise_image(64, 64, seed=1))
    with pytest.raises(Exception, match="OMP supports at most"):
        A.Code(dic, [img], [dict(tol=0.01, max_atoms=65, n_min=16, n_max=64)], [(0, 0)], schedule=1,
               solver=A.SOLVER_OMP)


def test_omp_decode_and_replays(A, dic):
    """Decoded image of the OMP encode matches the oracle's PSNR; graph
    replays are bit-identical."""
    import torch
    w = workload("c1")
    img = w["channels"][0]
    imgs = [_dev(img)]
    code = A.Code(dic, imgs, w["params"], [(0, 0)], schedule=1, solver=A.SOLVER_OMP)
    rec = torch.zeros(512, 512, dtype=torch.float64, device="cuda")
    code.decode(0, rec)
    torch.cuda.synchronize()
    ps_g = O.psnr(img, rec.cpu().numpy())
    e1 = code.export_nodes()
    for _ in range(2):
        code.reencode(imgs)
        e2 = code.export_nodes()
        assert e1.leaves.tobytes() == e2.leaves.tobytes()
        assert e1.atom_idx.tobytes() == e2.atom_idx.tobytes()
        assert e1.coef.tobytes() == e2.coef.tobytes()
    code.free()
    p = O.Params.from_dict(dict(w["params"][0], solver="omp"))
    onodes = O.encode_channel(img, p)
    ps_o = O.psnr(img, O.decode(onodes, 512, 512))
    _say("omp psnr", ps_g, ps_o)
    assert abs(ps_g - ps_o) < 0.01
