"""The library's host-only code (paper_2605_09190_amd/csrc/host_core.cpp: the
1D DCT and Haar tables of Section 2.1 and the bitstream writer of encoder
step (ii), Section 2.3) built on its own with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer, driven through tests/host_core_driver.cpp, and
checked against the oracle: the tables against ``dct_matrix`` and
``haar_matrix``, the stream bytes against ``pack_stream`` on random quadtrees
(both coefficient formats, one-byte and two-byte atom counts, two-byte and
four-byte quantised values, several channels, raw and DEFLATE), plus the
argument errors.  Any sanitizer report aborts the driver and fails the test.
"""
import os
import shutil
import subprocess
import zlib

import numpy as np
import pytest

from oracle import aqmp_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_09190_amd", "csrc")

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("san") / "host_core_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-Wall", "-Wextra", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
           f"-I{CSRC}", os.path.join(ROOT, "tests", "host_core_driver.cpp"), os.path.join(CSRC, "host_core.cpp"),
           "-o", exe, "-lz"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, text):
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, **SAN_ENV))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout.splitlines()


def test_tables_match_the_oracle(driver):
    sizes = [1, 2, 4, 8, 16, 32, 64]
    lines = _run(driver, "".join(f"T {n}\n" for n in sizes))
    pos = 0
    for n in sizes:
        assert lines[pos] == f"T {n}"
        vals = np.array([float.fromhex(v) for v in lines[pos + 1:pos + 1 + 2 * n * n]])
        pos += 1 + 2 * n * n
        c, h = vals[:n * n].reshape(n, n), vals[n * n:].reshape(n, n)
        # same formula, libm and NumPy cosines may differ in the last place
        np.testing.assert_allclose(c, O.dct_matrix(n), rtol=0, atol=2e-16)
        # the Haar recursion is the same sequence of roundings on both sides
        assert np.array_equal(h, O.haar_matrix(n))
        assert np.allclose(c @ c.T, np.eye(n), atol=1e-14) and np.allclose(h @ h.T, np.eye(n), atol=1e-14)
    assert pos == len(lines)


def _random_channel(rng, w, h, n_min, n_max, k_max, scale, p_split=0.45, wide_leaf=False):
    nodes = []

    def rec(x0, y0, n):
        split = n > n_min and rng.random() < p_split
        t = int(rng.integers(0, k_max + 1))
        if wide_leaf and not split and not any(not nd.split and nd.mp.t > 255 for nd in nodes):
            t = 300
        idx = rng.integers(0, min(65536, 2 * n * n), size=t).tolist()
        coef = (rng.standard_normal(t) * scale).tolist()
        nodes.append(O.Node(x0, y0, n, O.MPResult(idx=idx, coef=coef), split, 0.0, 0.0))
        if split:
            s = n // 2
            for dy, dx in ((0, 0), (0, s), (s, 0), (s, s)):
                rec(x0 + dx, y0 + dy, s)

    for by in range(0, h, n_max):
        for bx in range(0, w, n_max):
            rec(bx, by, n_max)
    return nodes


def _cmd(channels, w, h, n_min, n_max, step, level, families=3):
    out = [f"P {families} {w} {h} {n_min} {n_max} {float(step).hex()} {level} {len(channels)}"]
    for nodes in channels:
        out.append(str(len(nodes)))
        for nd in nodes:
            out.append(" ".join([str(nd.n), str(int(nd.split)), str(nd.mp.t)] + [str(i) for i in nd.mp.idx]
                                + [float(c).hex() for c in nd.mp.coef]))
    return "\n".join(out) + "\n"


CASES = [
    # (seed, w, h, n_min, n_max, channels, k_max, scale, step, level, wide_leaf)
    (1, 64, 64, 8, 32, 1, 6, 1.0, 0.0, -1, False),
    (2, 128, 64, 4, 64, 3, 12, 3.0, 0.0, 6, False),
    (3, 64, 64, 8, 64, 2, 8, 1.0, 0.0, -1, True),        # a leaf of 300 atoms: two-byte counts
    (4, 96, 32, 8, 32, 3, 8, 0.5, 0.05, -1, False),      # format 1, int16 values
    (5, 64, 64, 4, 16, 1, 8, 50.0, 1e-3, 9, False),      # format 1, int32 values
    (6, 32, 32, 32, 32, 1, 4, 1.0, 0.25, 0, False),      # N_min = N_max: no split flags
    (7, 64, 64, 8, 64, 1, 0, 1.0, 0.1, -1, False),       # every leaf empty
    (8, 128, 128, 1, 128, 2, 3, 1.0, 0.0, 1, False),     # deepest tree, 1x1 leaves
]


@pytest.mark.parametrize("case", CASES, ids=[f"seed{c[0]}" for c in CASES])
def test_stream_bytes_match_the_oracle(driver, case):
    seed, w, h, n_min, n_max, n_ch, k_max, scale, step, level, wide = case
    rng = np.random.default_rng(seed)
    chans = [_random_channel(rng, w, h, n_min, n_max, k_max, scale, wide_leaf=wide) for _ in range(n_ch)]
    want = O.pack_stream(chans, w, h, n_min, n_max, step=step if step > 0 else None)
    (line,) = _run(driver, _cmd(chans, w, h, n_min, n_max, step, level))
    tag, size, hexbytes = line.split(" ")
    assert tag == "OK"
    got = bytes.fromhex(hexbytes)
    assert len(got) == int(size)
    if level >= 0:
        got = zlib.decompress(got)
    assert got == want
    if wide:
        assert got[18] == 2
    if step > 0:
        assert got[6] == 1 and got[19] == (4 if scale / step > 32767 else 2)


ERRORS = [
    ("step too small for 32-bit", _cmd([[O.Node(0, 0, 8, O.MPResult(idx=[1], coef=[1e3]), False, 0, 0)]],
                                       8, 8, 8, 8, 1e-9, -1)),
    ("finite", _cmd([[]], 8, 8, 8, 8, float("nan"), -1)),
    ("rounds to zero", _cmd([[]], 8, 8, 8, 8, 1e-50, -1)),
    ("channels", _cmd([], 8, 8, 8, 8, 0.0, -1)),
    ("atom index", _cmd([[O.Node(0, 0, 8, O.MPResult(idx=[70000], coef=[1.0]), False, 0, 0)]], 8, 8, 8, 8, 0.0,
                        -1)),
    ("powers of two", _cmd([[]], 8, 8, 12, 24, 0.0, -1)),
    ("coefficient not finite", _cmd([[O.Node(0, 0, 8, O.MPResult(idx=[1], coef=[float("inf")]), False, 0, 0)]],
                                    8, 8, 8, 8, 0.0, -1)),
]


@pytest.mark.parametrize("msg,cmd", ERRORS, ids=[e[0].split()[0] for e in ERRORS])
def test_stream_argument_errors(driver, msg, cmd):
    (line,) = _run(driver, cmd)
    assert line.startswith("ERR -1 ") and msg in line
