"""GPU path vs the FP64 oracle, node by node (all calls go through the C ABI).

Tolerances: identical quadtree and atom sequences except counted atom/stop
ties; coefficients within 1e-5 (FP32 correlation) or 2e-3 (BF16
correlation) relative, floored at 1e-3 ||y||; PSNR within 0.01 dB.
"""
import sys

import numpy as np
import pytest

from oracle import aqmp_oracle as O
from tests import parity_util as PU
from workloads import workload, gradient_edges_image, piecewise_image

pytestmark = pytest.mark.gpu

COEF_TOL = {0: 1e-5, 1: 2e-3}


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


def _encode(A, dic, chans, params, jobs, prec, sched, dtype="f32", stepwise=False, solver=0):
    imgs = [_dev(c, dtype) for c in chans]
    code = A.Code(dic, imgs, params, jobs, precision=prec, schedule=sched, stepwise=stepwise, solver=solver)
    return code, imgs


def _check(A, code, chans, params, jobs, prec, blocks_per_job=None, tol=None):
    exp = code.export_nodes()
    rep = PU.Report()
    for j, (ci, pi) in enumerate(jobs):
        img = chans[ci]
        p = O.Params.from_dict(params[pi])
        blocks = None if blocks_per_job is None else blocks_per_job[j]
        onodes = O.encode_channel(img, p, blocks=blocks)
        gpu = PU.gpu_nodes_by_key(exp, j)
        PU.compare_job(img, onodes, gpu, COEF_TOL[prec] if tol is None else tol, p.n_max, rep=rep)
    return rep


@pytest.mark.parametrize("prec,sched,stepwise", [(0, 0, False), (1, 1, False), (0, 1, False), (1, 0, False),
                                                  (1, 2, False), (1, 1, True)])
def test_c0_full_parity(A, dic, prec, sched, stepwise):
    """The BF16 form runs its N = 16 level as one whole-level pursuit unless
    stepwise is set; both must match the oracle."""
    w = workload("c0")
    _say("c0", prec, sched, stepwise)
    code, imgs = _encode(A, dic, w["channels"], w["params"], w["jobs"], prec, sched, stepwise=stepwise)
    rep = _check(A, code, w["channels"], w["params"], w["jobs"], prec)
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.nodes > 10


def test_c0_dictionary_matches_oracle(A, dic):
    for n in (4, 8, 16, 32, 64):
        g = dic.copy(n)
        o = O.get_dict(n).D
        assert g.shape == o.shape
        assert np.all(g[:, 0] == 1.0 / n) and np.all(g[:, n * n] == 1.0 / n)
        assert np.abs(g - o).max() < 4e-16


def test_decode_psnr_matches_oracle(A, dic):
    import torch
    w = workload("c0")
    img = w["channels"][0]
    p = O.Params.from_dict(w["params"][0])
    onodes = O.encode_channel(img, p)
    ps_o = O.psnr(img, O.decode(onodes, 64, 64))
    for prec in (0, 1):
        code, imgs = _encode(A, dic, w["channels"], w["params"], w["jobs"], prec, 1)
        out = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
        code.decode(0, out)
        torch.cuda.synchronize()
        ps_g = O.psnr(img, out.cpu().numpy())
        _say("psnr", prec, ps_o, ps_g)
        assert abs(ps_g - ps_o) < 0.01


_ORACLE_CACHE: dict = {}


def _oracle_cached(key, jobs):
    """Oracle nodes of (plane, params, blocks) jobs, computed once per key in
    a process pool and shared by the precision cases."""
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = PU.oracle_jobs_parallel(jobs)
    return _ORACLE_CACHE[key]


def _gpu_decode(A, code, job, img):
    """A job's GPU decode of the whole plane (on the device, into FP64),
    copied to the host."""
    import torch
    out = torch.zeros(img.shape, dtype=torch.float64, device="cuda")
    code.decode(job, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec,tau", [(0, 0.02), (1, 0.02), (0, 0.01), (1, 0.01), (0, 0.04), (1, 0.04)])
def test_c1_full_parity(A, dic, prec, tau):
    """The 512 x 512 image at the three RMS tolerances of its configuration:
    every one of the 64 top-level blocks node by node, and the PSNR of the
    whole plane within 0.01 dB of the oracle's."""
    w = workload("c1", tau=tau)
    img = w["channels"][0]
    p = w["params"][0]
    _say("c1 full", prec, tau)
    onodes = _oracle_cached(("c1", tau), [(img, p, None)])[0]
    code, imgs = _encode(A, dic, [img], [p], [(0, 0)], prec, 1)
    exp = code.export_nodes()
    rep = PU.compare_job(img, onodes, PU.gpu_nodes_by_key(exp, 0), COEF_TOL[prec], p["n_max"])
    ps_g = O.psnr(img, _gpu_decode(A, code, 0, img))
    ps_o = O.psnr(img, O.decode(onodes, 512, 512))
    code.free()
    _say(rep.summary(), "psnr gpu", ps_g, "oracle", ps_o)
    assert rep.ok(), rep.summary()
    assert len({(nd.x0, nd.y0) for nd in onodes if nd.n == 64}) == 64
    assert abs(ps_g - ps_o) < 0.01, (ps_g, ps_o)


@pytest.mark.parametrize("prec,sched", [(0, 1), (1, 1), (1, 2)])
def test_mixed_jobs_small_sizes(A, dic, prec, sched):
    """Several jobs with different block ranges (4..32), k, tolerances and both
    split rules in one batched pass, plus an FP64 input plane."""
    chans = [gradient_edges_image(64, 64, seed=3), piecewise_image(64, 128, seed=4)]
    params = [dict(tol=0.03, max_atoms=8, n_min=4, n_max=16),
              dict(tol=0.01, max_atoms=20, n_min=8, n_max=32, split_rule="r2"),
              dict(tol=0.5, tol_mode="abs", max_atoms=40, n_min=4, n_max=32)]
    jobs = [(0, 0), (1, 1), (0, 2), (1, 0)]
    _say("mixed", prec, sched)
    code, imgs = _encode(A, dic, chans, params, jobs, prec, sched, dtype="f64")
    rep = _check(A, code, chans, params, jobs, prec)
    _say(rep.summary())
    assert rep.ok(), rep.summary()


FULL_SIZE_BLOCKS = 128


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [1, 0])
def test_full_size_sampled_parity(A, dic, prec):
    """The benchmark workload at its full size (2048x2048 RGB -> YCbCr, three
    jobs, blocks 64 -> 8, k = 32) in the launch configuration the benchmark
    times (one batched graph), checked node by node on a seeded sample of 128
    of the 1024 top-level blocks per job, and the PSNR over the union of the
    sampled blocks within 0.01 dB of the oracle's, per job."""
    w = workload("c3")
    rng = np.random.default_rng(2024)
    tops = O.top_blocks(2048, 2048, 64)
    samples = [[tops[i] for i in sorted(rng.choice(len(tops), size=FULL_SIZE_BLOCKS, replace=False))]
               for _ in w["jobs"]]
    _say("full size", prec, [s[:4] for s in samples])
    jobs = [(w["channels"][ci], w["params"][pi], samples[j]) for j, (ci, pi) in enumerate(w["jobs"])]
    onodes = _oracle_cached(("c3", FULL_SIZE_BLOCKS), jobs)
    _say("oracle done", [len(o) for o in onodes])
    code, imgs = _encode(A, dic, w["channels"], w["params"], w["jobs"], prec, 1)
    exp = code.export_nodes()
    rep = PU.Report()
    dps = []
    for j, (ci, pi) in enumerate(w["jobs"]):
        img = w["channels"][ci]
        PU.compare_job(img, onodes[j], PU.gpu_nodes_by_key(exp, j), COEF_TOL[prec], 64, rep=rep)
        rec_g = _gpu_decode(A, code, j, img)
        rec_o = PU.decode_region(img.shape, onodes[j])
        ps_g = PU.psnr_region(img, rec_g, samples[j], 64)
        ps_o = PU.psnr_region(img, rec_o, samples[j], 64)
        dps.append(ps_g - ps_o)
        _say("job", j, "psnr (sampled blocks) gpu", ps_g, "oracle", ps_o)
    code.free()
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.nodes >= 3 * FULL_SIZE_BLOCKS
    assert max(abs(d) for d in dps) < 0.01, dps


@pytest.mark.parametrize("fam", ["dct", "haar"])
def test_single_family_dictionary_bf16(A, fam):
    """One-family dictionaries (M = N^2) through the BF16 form: generated-atom
    correlation at N = 32, 64 and the whole-level pursuit at N = 16 must see
    only the atoms that exist."""
    F = O.DCT if fam == "dct" else O.HAAR
    d = A.Dictionary(8, 64, families=(A.DCT if fam == "dct" else A.HAAR))
    img = piecewise_image(128, 128, seed=21)
    p = dict(tol=0.02, max_atoms=16, n_min=8, n_max=64)
    _say("single family", fam)
    imgs = [_dev(img)]
    code = A.Code(d, imgs, [p], [(0, 0)], precision=1, schedule=1)
    exp = code.export_nodes()
    onodes = O.encode_channel(img, O.Params.from_dict(dict(p, families=F)))
    rep = PU.compare_job(img, onodes, PU.gpu_nodes_by_key(exp, 0), COEF_TOL[1], 64, families=F)
    _say(rep.summary())
    code.free()
    d.free()
    assert rep.ok(), rep.summary()


def test_corr_variants_bit_identical(A, dic):
    """Every BF16 correlation kernel variant (direct-to-LDS, register-staged,
    generated atoms) sums the same products in the same k order: the
    exported trees, atoms and coefficients are bit-identical (stepwise, so
    that every level of 16 and up runs the variant kernels).  The removed
    variant numbers are rejected."""
    w = workload("c1")
    img = w["channels"][0]
    ref = None
    for v in (2, 3, 6):
        _say("variant", v)
        imgs = [_dev(img)]
        code = A.Code(dic, imgs, w["params"], [(0, 0)], precision=1, schedule=1, corr_variant=v, stepwise=True)
        e = code.export_nodes()
        cur = (e.leaves.tobytes(), e.atom_idx.tobytes(), e.coef.tobytes())
        if ref is None:
            ref = cur
        assert cur == ref, f"variant {v} differs"
        code.free()
    for v in (1, 4, 5, 7):
        with pytest.raises(A.AqmpError, match="corr_variant"):
            A.Code(dic, [_dev(img)], w["params"], [(0, 0)], precision=1, schedule=1, corr_variant=v)


def test_reencode_deterministic(A, dic):
    """Re-encoding (graph replay) reproduces the first encode bit for bit."""
    w = workload("c1")
    imgs = [_dev(w["channels"][0])]
    code = A.Code(dic, imgs, w["params"], [(0, 0)], precision=1, schedule=1)
    e1 = code.export_nodes()
    for _ in range(3):
        code.reencode(imgs)
        e2 = code.export_nodes()
        assert e1.leaves.tobytes() == e2.leaves.tobytes()
        assert e1.atom_idx.tobytes() == e2.atom_idx.tobytes()
        assert e1.coef.tobytes() == e2.coef.tobytes()


def test_reencode_other_images(A, dic):
    """Re-encoding with other images of the same shape (new device buffers,
    so the job table on the device changes) gives exactly what a fresh code
    of those images gives, and going back to the first images gives the
    first result again."""
    w = workload("c1")
    img_a = w["channels"][0]
    img_b = piecewise_image(img_a.shape[0], img_a.shape[1], seed=77)
    da, db = [_dev(img_a)], [_dev(img_b)]
    _say("reencode with other images")
    code = A.Code(dic, da, w["params"], [(0, 0)], precision=1, schedule=1)
    ea = code.export_nodes()
    ref_a = (ea.leaves.tobytes(), ea.atom_idx.tobytes(), ea.coef.tobytes())
    fresh = A.Code(dic, db, w["params"], [(0, 0)], precision=1, schedule=1)
    eb = fresh.export_nodes()
    ref_b = (eb.leaves.tobytes(), eb.atom_idx.tobytes(), eb.coef.tobytes())
    fresh.free()
    assert ref_a != ref_b
    for imgs, ref in ((db, ref_b), (db, ref_b), (da, ref_a)):
        code.reencode(imgs)
        e = code.export_nodes()
        assert (e.leaves.tobytes(), e.atom_idx.tobytes(), e.coef.tobytes()) == ref
    code.free()


def test_reencode_deterministic_full_size(A, dic):
    """The 2048 x 2048 three-channel encode: the active lists are rebuilt by
    atomic appends in a different order on every replay, and the exported
    trees, atoms and coefficients stay bit-identical."""
    w = workload("c3")
    imgs = [_dev(c) for c in w["channels"]]
    code = A.Code(dic, imgs, w["params"], w["jobs"], precision=1, schedule=1)
    e1 = code.export_nodes()
    ref = (e1.leaves.tobytes(), e1.atom_idx.tobytes(), e1.coef.tobytes())
    for i in range(3):
        code.reencode(imgs)
        e2 = code.export_nodes()
        assert (e2.leaves.tobytes(), e2.atom_idx.tobytes(), e2.coef.tobytes()) == ref, f"replay {i}"
    code.free()


@pytest.mark.parametrize("form", ["fp32", "bf16", "gram", "omp"])
def test_non_multiple_plane_edge_padded(A, dic, form):
    """A 100 x 70 plane with N_max = 32 (tiled as 128 x 96, last row and
    column repeated) and a 72 x 72 FP64 plane with N_max = 64: same nodes and
    atoms as the oracle on the padded plane; the decode writes the plane's own
    pixels only (a guard band around it stays untouched)."""
    import torch
    chans = [piecewise_image(70, 100, seed=31), gradient_edges_image(72, 72, seed=32)]
    params = [dict(tol=0.02, max_atoms=12, n_min=4, n_max=32), dict(tol=0.02, max_atoms=16, n_min=8, n_max=64)]
    jobs = [(0, 0), (1, 1)]
    solver = {"gram": A.SOLVER_GRAM, "omp": A.SOLVER_OMP}.get(form, A.SOLVER_DENSE)
    prec = 1 if form == "bf16" else 0
    imgs = [_dev(chans[0]), _dev(chans[1], "f64")]
    code = A.Code(dic, imgs, params, jobs, precision=prec, schedule=1, solver=solver)
    exp = code.export_nodes()
    rep = PU.Report()
    osolver = "omp" if form == "omp" else "mp"
    tol = {"fp32": 1e-5, "bf16": 2e-3, "gram": 1e-9, "omp": 1e-8}[form]
    onodes = []
    for j, (ci, pi) in enumerate(jobs):
        p = O.Params.from_dict(dict(params[pi], solver=osolver))
        on = O.encode_channel(chans[ci], p)
        onodes.append(on)
        PU.compare_job(chans[ci], on, PU.gpu_nodes_by_key(exp, j), tol, p.n_max, rep=rep, solver=osolver)
    _say("non-multiple", form, rep.summary())
    assert rep.ok(), rep.summary()
    # decode into the middle of a larger buffer: the guard band must stay NaN
    for j, (ci, pi) in enumerate(jobs):
        h, w = chans[ci].shape
        buf = torch.full((h + 8, w + 16), float("nan"), dtype=torch.float64, device="cuda")
        view = buf[4:4 + h, 8:8 + w]
        code.decode(j, view)
        torch.cuda.synchronize()
        b = buf.cpu().numpy()
        assert np.isnan(b[:4]).all() and np.isnan(b[4 + h:]).all()
        assert np.isnan(b[:, :8]).all() and np.isnan(b[:, 8 + w:]).all()
        rec = b[4:4 + h, 8:8 + w]
        assert np.isfinite(rec).all()
        ps_g = O.psnr(chans[ci], rec)
        ps_o = O.psnr(chans[ci], O.decode(onodes[j], h, w))
        assert abs(ps_g - ps_o) < 0.01, (ps_g, ps_o)
    code.free()


@pytest.mark.parametrize("prec", [0, 1])
def test_degenerate_blocks_dense(A, dic, prec):
    """Dense forms on a constant plane (one constant atom per top block, then
    an exact-zero residual), an all-zero plane (first stop test) and k = 0
    (sparsity stop before any step)."""
    const = np.full((128, 128), 0.37)
    zero = np.zeros((64, 64))
    rng = np.random.default_rng(5)
    noise = rng.standard_normal((64, 64)) * 0.1
    params = [dict(tol=1e-6, tol_mode="abs", max_atoms=8, n_min=8, n_max=64),
              dict(tol=0.01, max_atoms=0, n_min=8, n_max=64)]
    jobs = [(0, 0), (1, 0), (2, 1), (2, 0)]
    _say("degenerate dense", prec)
    code, imgs = _encode(A, dic, [const, zero, noise], params, jobs, prec, 1, dtype="f64")
    rep = _check(A, code, [const, zero, noise], params, jobs, prec)
    _say(rep.summary())
    assert rep.ok(), rep.summary()
    code.free()


@pytest.mark.parametrize("form", ["fp32", "bf16", "gram"])
def test_maximum_sparsity(A, dic, form):
    """k = 256 (AQMP_MAX_ATOMS) with a tolerance no block meets, on a
    noise-dominated plane: every node runs all 256 steps (MP may pick an atom
    again) and crosses every record window.  The dense forms keep the residual
    in FP32, whose drift against the FP64 oracle grows as the residual
    shrinks, so they run N = 32 only (the residual keeps >= 1.6% of its
    energy and no top-2 gap falls below 1e-5); the Gram solver (FP64) also
    runs N = 16 (down to 1e-4 of the block's energy).  Deeper still (N = 8
    here reaches 1e-15) two FP64 computations in different orders differ by
    about the tie window, so that case is not a parity case.  The plane is
    rounded to FP32 values: the library reads it as FP32."""
    rng = np.random.default_rng(78)
    img = np.clip(piecewise_image(64, 64, seed=77) + rng.normal(0, 0.2, size=(64, 64)), 0, 1)
    img = img.astype(np.float32).astype(np.float64)
    params = [dict(tol=1e-9, max_atoms=256, n_min=32, n_max=32), dict(tol=1e-9, max_atoms=256, n_min=16, n_max=16)]
    jobs = [(0, 0), (0, 1)] if form == "gram" else [(0, 0)]
    solver = A.SOLVER_GRAM if form == "gram" else A.SOLVER_DENSE
    prec = 1 if form == "bf16" else 0
    code = A.Code(dic, [_dev(img)], params, jobs, precision=prec, schedule=1, solver=solver)
    exp = code.export_nodes()
    tol = {"fp32": 1e-5, "bf16": 2e-3, "gram": 1e-9}[form]
    rep = PU.Report()
    for j, (ci, pi) in enumerate(jobs):
        p = O.Params.from_dict(params[pi])
        PU.compare_job(img, O.encode_channel(img, p), PU.gpu_nodes_by_key(exp, j), tol, p.n_max, rep=rep)
    _say("max k", form, rep.summary())
    assert rep.ok(), rep.summary()
    assert rep.iters >= 256 * 4
    code.free()
