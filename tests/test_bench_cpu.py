"""Host-side arithmetic of bench.py (no GPU): the algorithmic work per unit
that the roofline figures divide by, the gating of counter-measured traffic
on the source it was measured on, and the per-level report."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_select_bytes_per_node_iteration(bench):
    # FP32 residual read + written (8K), BF16 copy written (2K), keys of
    # every 256-atom tile (8 x 8 B each), record (12 B); K = N^2, M = 2K.
    assert bench.select_bytes(64, 1) == 8 * 4096 + 2 * 4096 + 32 * 64 + 12 == 43020
    assert bench.select_bytes(32, 1) == 8 * 1024 + 2 * 1024 + 8 * 64 + 12 == 10764
    assert bench.select_bytes(32, 0) == 8 * 1024 + 8 * 64 + 12
    assert bench.select_bytes(16, 1) == 8 * 256 + 2 * 256 + 2 * 64 + 12


def test_traffic_is_tied_to_the_measured_source(bench, monkeypatch):
    assert bench.measured_traffic("k_corr_bf16_gen<64>", "c1") is None        # other workload
    assert bench.measured_traffic("no such kernel", "c3") is None
    for name, t in bench.TRAFFIC.items():
        assert abs(t["fetch"] + t["write"] - t["bytes_per_launch"]) < 0.02e6, name
    # a source that differs from the measured one gives no figure
    t = dict(bench.TRAFFIC["k_select<64>"], sha256="0" * 64)
    monkeypatch.setitem(bench.TRAFFIC, "k_select<64>", t)
    assert bench.measured_traffic("k_select<64>", "c3") is None


def test_roofline_per_level_report(bench):
    iters = [0, 0, 0, 1000, 2000, 3000, 4000]
    stats = dict(iters_level=iters)
    timing = dict(corr_ms=[0, 0, 0, 0, 0, 0.5, 2.0], select_ms=[0, 0, 0, 0, 0, 0.4, 0.6],
                  level_ms=[0, 0, 0, 0.1, 0.3, 1.0, 3.0], steps=[0, 0, 0, 0, 0, 32, 32])
    r = bench.roofline(stats, timing, 1, lambda n: f"k<{n}>", workload="none")
    assert r["kernel"] == "k<64>" and r["units"] == 4000 and r["flops_per_unit"] == 4 * 64 ** 4
    assert r["achieved"] == pytest.approx(4 * 64 ** 4 * 4000 / 2e-3 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.PEAK_BF16_TFLOPS, abs=1e-4)
    assert r["traffic"] is None
    lv = r["per_level"]
    assert set(lv) == {"8", "16", "32", "64"}
    assert lv["64"]["select_gbs"] == pytest.approx(43020 * 4000 / 0.6e-3 / 1e9, rel=1e-3)
    assert lv["16"]["peak"] == "bf16 mfma" and lv["8"]["peak"] == "bf16 mfma"
    assert lv["8"]["frac"] == pytest.approx(4 * 8 ** 4 * 1000 / 0.1e-3 / 1e12 / bench.PEAK_BF16_TFLOPS, abs=1e-4)
    r32 = bench.roofline(stats, timing, 0, lambda n: f"k<{n}>", workload="none")
    assert r32["per_level"]["8"]["peak"] == "fp64"
    assert r32["per_level"]["8"]["frac"] == pytest.approx(4 * 8 ** 4 * 1000 / 0.1e-3 / 1e12 / bench.PEAK_FP64_TFLOPS,
                                                          abs=1e-4)


def test_more_than_one_gpu_is_refused(bench, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
