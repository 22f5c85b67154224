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
    assert A.pack_variant_levels({64: 5, 32: 1, 16: 4}) == (5 << 24) | (1 << 20) | (4 << 16)
    for bad in ({48: 1}, {128: 1}, {2: 1}, {64: 7}, {64: -1}):
        with pytest.raises(ValueError):
            A.pack_variant_levels(bad)
