"""The batched hyperparameter sweep: 16 seeded images of mixed sizes (256x256
to 4096x3072) x 32 random-search trials (RMS tolerance, k, N_min, N_max) =
512 jobs encoded together in one captured graph, checked against the oracle
on a seeded sample of jobs and top-level blocks (top-level quadtrees are
independent, so a sampled block is compared exactly): 128 jobs in the BF16
form, 48 each for the Gram and OMP solvers, the oracle on a process pool.

Forms: the BF16 batched form over all 512 jobs; the plain FP32 form over a
subset of jobs; the Gram and OMP solvers over all 512 jobs.
"""
import sys

import numpy as np
import pytest

from oracle import aqmp_oracle as O
from tests import parity_util as PU
from workloads import workload

pytestmark = pytest.mark.gpu

TOL = {"bf16": 2e-3, "fp32": 1e-5, "gram": 1e-9, "omp": 1e-8}


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
def sweep():
    _say("generating the sweep workload")
    return workload("c4")


@pytest.fixture(scope="module")
def dic(A):
    d = A.Dictionary(4, 64)
    yield d
    d.free()


def _sample(w, n_jobs, seed):
    rng = np.random.default_rng(seed)
    js = sorted(int(j) for j in rng.choice(len(w["jobs"]), size=n_jobs, replace=False))
    out = []
    for j in js:
        ci, pi = w["jobs"][j]
        img, p = w["channels"][ci], w["params"][pi]
        tops = O.top_blocks(img.shape[0], img.shape[1], p["n_max"])
        out.append((j, tops[int(rng.integers(len(tops)))]))
    return out


def _check(w, exp, picks, tol, solver="mp", job_map=None):
    """Each picked (job, top-level block) node by node against the oracle,
    which runs on a process pool (one task per block)."""
    rep = PU.Report()
    tasks = []
    for j, blk in picks:
        ci, pi = w["jobs"][j]
        tasks.append((w["channels"][ci], dict(w["params"][pi], solver=solver), [blk]))
    _say("  oracle on", len(tasks), "blocks,", PU.pool_size(), "processes")
    onodes_all = PU.oracle_jobs_parallel(tasks)
    for (j, blk), onodes in zip(picks, onodes_all):
        ci, pi = w["jobs"][j]
        img = w["channels"][ci]
        gj = j if job_map is None else job_map[j]
        PU.compare_job(img, onodes, PU.gpu_nodes_by_key(exp, gj), tol, w["params"][pi]["n_max"], rep=rep,
                       solver=solver)
    _say("  compared", len(picks), "blocks,", rep.nodes, "nodes, failures", len(rep.failures))
    return rep


def _encode(A, dic, w, jobs, **kw):
    import torch
    imgs = [torch.from_numpy(np.ascontiguousarray(c)).to(torch.float32).cuda() for c in w["channels"]]
    code = A.Code(dic, imgs, w["params"], jobs, **kw)
    torch.cuda.synchronize()
    return code, imgs


@pytest.mark.timeout(900)
def test_sweep_bf16_batched_sampled_parity(A, dic, sweep):
    _say("sweep bf16 batched: encode", len(sweep["jobs"]), "jobs")
    code, imgs = _encode(A, dic, sweep, sweep["jobs"], precision=A.PREC_BF16, schedule=A.SCHED_BATCHED)
    st = code.stats()
    _say("stats", st["nodes"], st["iters_executed"])
    exp = code.export_nodes()
    code.free()
    picks = _sample(sweep, 128, seed=41)
    _say("picks", picks[:8], "...")
    rep = _check(sweep, exp, picks, TOL["bf16"])
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.nodes >= 128


@pytest.mark.timeout(900)
def test_sweep_fp32_plain_subset_parity(A, dic, sweep):
    """The plain FP32 form (jobs one after another), on 6 sampled jobs."""
    picks = _sample(sweep, 6, seed=42)
    jobs = [sweep["jobs"][j] for j, _ in picks]
    _say("sweep fp32 plain:", jobs)
    code, imgs = _encode(A, dic, sweep, jobs, precision=A.PREC_FP32, schedule=A.SCHED_PLAIN)
    exp = code.export_nodes()
    code.free()
    rep = _check(sweep, exp, picks, TOL["fp32"], job_map={j: i for i, (j, _) in enumerate(picks)})
    _say(rep.summary())
    assert rep.ok(), rep.summary()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("solver", ["gram", "omp"])
def test_sweep_solvers_sampled_parity(A, dic, sweep, solver):
    _say("sweep", solver, "batched: encode", len(sweep["jobs"]), "jobs")
    sv = A.SOLVER_GRAM if solver == "gram" else A.SOLVER_OMP
    code, imgs = _encode(A, dic, sweep, sweep["jobs"], schedule=A.SCHED_BATCHED, solver=sv)
    exp = code.export_nodes()
    code.free()
    picks = _sample(sweep, 48, seed=43 if solver == "gram" else 44)
    rep = _check(sweep, exp, picks, TOL[solver], solver="omp" if solver == "omp" else "mp")
    _say(rep.summary())
    assert rep.ok(), rep.summary()
