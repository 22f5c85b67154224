"""The autotuner and the per-level kernel choice, on the GPU.

Every BF16 correlation kernel family computes the same keys, so forcing a
family per block size must leave the code bit-identical; the tuner's choice
on a workload must run and match the oracle like the default does.
"""
import sys

import numpy as np
import pytest

from oracle import aqmp_oracle as O
from tests import parity_util as PU
from workloads import workload, piecewise_image

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
    d = A.Dictionary(8, 64)
    yield d
    d.free()


def _dev(img):
    import torch
    return torch.from_numpy(np.ascontiguousarray(img)).to(torch.float32).cuda()


def _bytes(code):
    e = code.export_nodes()
    return e.leaves.tobytes(), e.atom_idx.tobytes(), e.coef.tobytes()


@pytest.mark.parametrize("levels", [{64: 2, 32: 3}, {64: 3, 32: 2}, {64: 2, 32: 6, 16: 3}])
def test_per_level_variants_are_bit_identical(A, dic, levels):
    w = workload("c1")
    imgs = [_dev(w["channels"][0])]
    ref = A.Code(dic, imgs, w["params"], [(0, 0)], precision=1, schedule=1, stepwise=True)
    want = _bytes(ref)
    ref.free()
    code = A.Code(dic, imgs, w["params"], [(0, 0)], precision=1, schedule=1, stepwise=True,
                  corr_variant_levels=levels)
    assert _bytes(code) == want, levels
    code.free()


def test_bad_level_word_is_rejected(A, dic, monkeypatch):
    imgs = [_dev(piecewise_image(64, 64, seed=2))]
    p = dict(tol=0.02, max_atoms=8, n_min=8, n_max=32)
    for word in (7 << 24, 1 << 24, 5 << 20, 4 << 16, 2 << 4, 2 << 28):
        monkeypatch.setattr(A, "pack_variant_levels", lambda _d, word=word: word)
        with pytest.raises(Exception, match="corr_variant_levels"):
            A.Code(dic, imgs, [p], [(0, 0)], precision=1, schedule=1, corr_variant_levels={64: 2})


def test_tuned_options_run_and_match_the_oracle(A, dic):
    from paper_2605_09190_amd import autotune
    w = workload("c1")
    img = w["channels"][0]
    p = w["params"][0]
    imgs = [_dev(img)]
    tuned = autotune.tune(A, dic, imgs, w["params"], [(0, 0)], reps=2, steps=3)
    _say("tuned", tuned)
    opt = tuned["options"]
    assert opt["schedule"] == A.SCHED_BATCHED            # one job: nothing to split
    for n, v in opt["corr_variant_levels"].items():
        assert n in (16, 32, 64) and v in autotune.CANDIDATES[n]
    assert set(tuned["measured"]["corr_ms"]) <= {"32", "64"}
    code = A.Code(dic, imgs, w["params"], [(0, 0)], precision=1, **opt)
    exp = code.export_nodes()
    code.free()
    rng = np.random.default_rng(12)
    tops = O.top_blocks(512, 512, 64)
    sample = [tops[i] for i in sorted(rng.choice(len(tops), size=4, replace=False))]
    onodes = O.encode_channel(img, O.Params.from_dict(p), blocks=sample)
    rep = PU.Report()
    PU.compare_job(img, onodes, PU.gpu_nodes_by_key(exp, 0), 2e-3, p["n_max"], rep=rep)
    _say(rep.summary())
    assert rep.ok(), rep.summary()


@pytest.mark.parametrize("tiles", [{64: (1, 1), 32: (7, 7)}, {64: (7, 7), 32: (1, 2)}, {64: (2, 4)}])
def test_node_tile_ranges_are_bit_identical(A, dic, tiles):
    """Every node-tile width of the generated-atom kernel gives the same keys
    per node, so forced ranges leave the code bit-identical (full size: the
    widths then really differ between steps)."""
    w = workload("c3")
    imgs = [_dev(c) for c in w["channels"]]
    ref = A.Code(dic, imgs, w["params"], w["jobs"], precision=1, schedule=1)
    want = _bytes(ref)
    ref.free()
    code = A.Code(dic, imgs, w["params"], w["jobs"], precision=1, schedule=1, corr_tile_levels=tiles)
    _say("tiles", tiles)
    assert _bytes(code) == want, tiles
    code.free()


def test_bad_tile_word_is_rejected(A, dic, monkeypatch):
    imgs = [_dev(piecewise_image(64, 64, seed=2))]
    p = dict(tol=0.02, max_atoms=8, n_min=8, n_max=32)
    for word in (1 << 16, 0x12, 0x81, 0x10):       # outside N = 32, 64; lo > hi; hi = 8; lo = 0
        monkeypatch.setattr(A, "pack_tile_levels", lambda _d, word=word: word)
        with pytest.raises(Exception, match="corr_tile_levels"):
            A.Code(dic, imgs, [p], [(0, 0)], precision=1, schedule=1, corr_tile_levels={32: (1, 2)})


def test_tuner_cache_round_trip(A, dic, tmp_path):
    """The tuned options are stored under the workload's key and returned
    from the cache the second time, without timing anything."""
    import time
    from paper_2605_09190_amd import autotune
    w = workload("c1")
    imgs = [_dev(w["channels"][0])]
    path = str(tmp_path / "tune.json")
    t0 = time.perf_counter()
    first = autotune.tune(A, dic, imgs, w["params"], [(0, 0)], reps=1, steps=2, cache=path)
    t1 = time.perf_counter()
    second = autotune.tune(A, dic, imgs, w["params"], [(0, 0)], reps=1, steps=2, cache=path)
    t2 = time.perf_counter()
    _say("tune", first["options"], "measured", first["measured"].get("tile_ms"), t1 - t0, t2 - t1)
    assert not first["cached"] and second["cached"]
    assert second["options"] == first["options"]
    assert t2 - t1 < (t1 - t0) / 4
    for n, rng in first["options"]["corr_tile_levels"].items():
        assert rng in autotune.TILE_CANDIDATES[n]
    # another workload (other shape) misses the cache
    imgs2 = [_dev(piecewise_image(256, 256, seed=9))]
    third = autotune.tune(A, dic, imgs2, w["params"], [(0, 0)], reps=1, steps=2, cache=path)
    assert not third["cached"]
