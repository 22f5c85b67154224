"""Host logic of the autotuner and of the per-level kernel word (no GPU)."""
import pytest

from paper_2605_09190_amd import autotune as T


def test_choose_keeps_the_default_within_the_margin():
    assert T.choose({6: 10.0, 5: 9.8, 1: 12.0}, 6, 0.03) == 6          # 2% faster: noise
    assert T.choose({6: 10.0, 5: 9.6, 1: 12.0}, 6, 0.03) == 5          # 4% faster: taken
    assert T.choose({6: 10.0, 5: 9.6, 1: 9.0}, 6, 0.03) == 1
    assert T.choose({5: 9.6, 1: 9.6}, 6, 0.03) == 5                    # default not timed: the first best
    assert T.choose({}, 6, 0.03) == 6
    assert T.choose({("whole", 0): 1.0, ("step", 2): 0.9}, ("whole", 0), 0.03) == ("step", 2)


def test_candidates_include_the_defaults():
    for n, v in T.DEFAULT.items():
        assert v in T.CANDIDATES[n]
    assert 6 not in T.CANDIDATES[16]          # the generated-atom kernel exists for N >= 32 only


def test_pack_variant_levels():
    import importlib
    try:
        A = importlib.import_module("paper_2605_09190_amd.aqmp")
    except ImportError:
        pytest.skip("library not built")
    assert A.pack_variant_levels({}) == 0
    assert A.pack_variant_levels({64: 6, 32: 3, 16: 2}) == (6 << 24) | (3 << 20) | (2 << 16)
    for bad in ({48: 2}, {128: 2}, {2: 2}, {64: 7}, {64: -1}, {64: 1}, {32: 4}, {16: 5}):
        with pytest.raises(ValueError):
            A.pack_variant_levels(bad)


def test_tile_candidates_include_the_defaults():
    for n, rng in T.DEFAULT_TILE.items():
        assert rng in T.TILE_CANDIDATES[n]
        for lo, hi in T.TILE_CANDIDATES[n]:
            assert 1 <= lo <= hi <= 7


def test_cache_key_and_round_trip(tmp_path):
    class Img:
        def __init__(self, h, w, dt):
            self.shape, self.dtype = (h, w), dt
    prm = [dict(tol=0.02, max_atoms=32, n_min=8, n_max=64, k_per_level={16: 4})]
    k1 = T.cache_key([Img(64, 48, "float32")], prm, [(0, 0)], "gpu", "abc")
    assert k1 == T.cache_key([Img(64, 48, "float32")], [dict(reversed(list(prm[0].items())))], [(0, 0)], "gpu", "abc")
    assert k1 != T.cache_key([Img(64, 49, "float32")], prm, [(0, 0)], "gpu", "abc")
    assert k1 != T.cache_key([Img(64, 48, "float32")], prm, [(0, 0)], "gpu", "abd")
    assert k1 != T.cache_key([Img(64, 48, "float32")], prm, [(0, 0)], "other", "abc")
    path = str(tmp_path / "c.json")
    assert T.cache_load(path, k1) is None
    opt = dict(corr_variant_levels={64: 2}, corr_tile_levels={32: (2, 5)}, stepwise=False, schedule=1)
    T.cache_store(path, k1, dict(options=T._options_to_json(opt), measured={}))
    T.cache_store(path, "other", dict(options=T._options_to_json(opt), measured={}))
    got = T.cache_load(path, k1)
    assert T._options_from_json(got["options"]) == opt


def test_source_hash_is_stable():
    assert T.source_hash() == T.source_hash() and len(T.source_hash()) == 64


def test_pack_tile_levels():
    import importlib
    try:
        A = importlib.import_module("paper_2605_09190_amd.aqmp")
    except ImportError:
        pytest.skip("library not built")
    assert A.pack_tile_levels({}) == 0
    assert A.pack_tile_levels({32: (2, 5), 64: (3, 7)}) == (2 | 5 << 4) | (3 | 7 << 4) << 8
    for bad in ({16: (1, 2)}, {64: (0, 3)}, {64: (4, 3)}, {32: (1, 8)}):
        with pytest.raises(ValueError):
            A.pack_tile_levels(bad)
