"""The integer worklist steps on their own, through the C ABI, bit for bit
against NumPy: the active-list compaction (stable: the running nodes in
increasing order) and the split test with child emission (Algorithm 2's
refinement into the four quadrants).

Sizes run up to 10^6 items, i.e. 977 scan tiles of 1024 items: the
look-back then crosses more than 64 predecessor tiles, which exercises its
multi-probe path.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 1023, 1024, 1025, 65 * 1024 + 7, 1_000_000]


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


def _status(rng, n, p_run):
    st = rng.choice(np.array([1, 2, 3, 0x10], dtype=np.uint8), size=n)
    st[rng.random(n) < p_run] = 0
    return st


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p_run", [0.0, 0.01, 0.5, 1.0])
def test_compact_matches_numpy(A, n, p_run):
    import torch
    rng = np.random.default_rng(1000 + n + int(p_run * 100))
    st = _status(rng, n, p_run)
    _say("compact", n, p_run)
    d_st = torch.from_numpy(st).cuda()
    sentinel = -7
    out = torch.full((max(n, 1),), sentinel, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    A.worklist_compact(d_st, out, cnt)
    want = np.nonzero(st == 0)[0].astype(np.int32)
    c = int(cnt.item())
    got = out.cpu().numpy()
    assert c == len(want)
    assert np.array_equal(got[:c], want)
    assert np.all(got[c:] == sentinel)


def _params():
    return [dict(tol=0.02, tol_mode="rms", max_atoms=32, n_min=8, n_max=64),
            dict(tol=0.01, tol_mode="rms", max_atoms=12, n_min=4, n_max=32, split_rule="r2"),
            dict(tol=0.3, tol_mode="abs", max_atoms=20, n_min=16, n_max=64, k_per_level={32: 5}),
            dict(tol=0.05, tol_mode="rms", max_atoms=8, n_min=32, n_max=32)]


def _reference(params, n, prm_idx, x0, y0, e, t, st, child_base):
    """Split flags, children and count as Algorithm 2 defines them, with the
    same FP64 thresholds (eps_N = tol N in RMS mode, tol in ABS mode)."""
    nn = len(prm_idx)
    split = np.zeros(nn, dtype=bool)
    for pi, p in enumerate(params):
        m = prm_idx == pi
        if not n > p["n_min"]:
            continue
        if p.get("split_rule", "r1") == "r1":
            eps = p["tol"] * n if p.get("tol_mode", "rms") == "rms" else p["tol"]
            split[m] = e[m] >= eps * eps
        else:
            k = (p.get("k_per_level") or {}).get(n, p["max_atoms"])
            split[m] = t[m] >= k
    st2 = st.copy()
    st2[split] |= 0x10
    h = n // 2
    sp = np.nonzero(split)[0]
    cp = np.repeat(prm_idx[sp], 4)
    cx = np.repeat(x0[sp], 4) + np.tile([0, h, 0, h], len(sp))
    cy = np.repeat(y0[sp], 4) + np.tile([0, 0, h, h], len(sp))
    return st2, cp.astype(np.int32), cx.astype(np.int32), cy.astype(np.int32), child_base + 4 * len(sp)


@pytest.mark.parametrize("n_nodes", SIZES)
@pytest.mark.parametrize("n", [8, 32, 64])
def test_split_emit_matches_numpy(A, n_nodes, n):
    import torch
    rng = np.random.default_rng(2000 + n_nodes + n)
    params = _params()
    prm_idx = rng.integers(0, len(params), size=n_nodes).astype(np.int32)
    x0 = (rng.integers(0, 512, size=n_nodes) * n).astype(np.int32)
    y0 = (rng.integers(0, 512, size=n_nodes) * n).astype(np.int32)
    # residual norms around every threshold, with exact equality for some
    eps2 = np.array([(p["tol"] * n if p.get("tol_mode", "rms") == "rms" else p["tol"]) ** 2 for p in params])
    e = eps2[prm_idx] * rng.choice([0.5, 0.999999, 1.0, 1.000001, 3.0], size=n_nodes)
    t = rng.integers(0, 40, size=n_nodes).astype(np.int32)
    st = rng.choice(np.array([0, 1, 2, 3], dtype=np.uint8), size=n_nodes)
    child_base = 37
    _say("split", n, n_nodes)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d_st = dev(st)
    cap = child_base + 4 * n_nodes
    cp = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    cx = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    cy = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    A.worklist_split(params, n, dev(prm_idx), dev(x0), dev(y0), dev(e), dev(t), d_st, cp, cx, cy, cnt,
                     child_base=child_base)
    st2, wp, wx, wy, wc = _reference(params, n, prm_idx, x0, y0, e, t, st, child_base)
    c = int(cnt.item())
    assert c == wc
    assert np.array_equal(d_st.cpu().numpy(), st2)
    got_p, got_x, got_y = cp.cpu().numpy(), cx.cpu().numpy(), cy.cpu().numpy()
    assert np.array_equal(got_p[child_base:c], wp)
    assert np.array_equal(got_x[child_base:c], wx)
    assert np.array_equal(got_y[child_base:c], wy)
    for a in (got_p, got_x, got_y):
        assert np.all(a[:child_base] == -1) and np.all(a[c:] == -1)


def test_split_rejects_a_node_outside_the_parameter_table(A):
    """The kernel's own bounds check: a node naming parameter set 9 of a
    4-entry table is not split, and the call reports the error."""
    import torch
    params = _params()
    n_nodes = 3000
    prm_idx = np.zeros(n_nodes, dtype=np.int32)
    prm_idx[1234] = 9
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    z32 = np.zeros(n_nodes, dtype=np.int32)
    e = np.full(n_nodes, 10.0)
    d_st = torch.zeros(n_nodes, dtype=torch.uint8, device="cuda")
    out = [torch.zeros(4 * n_nodes, dtype=torch.int32, device="cuda") for _ in range(3)]
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(A.AqmpError, match="outside the table"):
        A.worklist_split(params, 64, dev(prm_idx), dev(z32), dev(z32), dev(e), dev(z32), d_st, *out, cnt)
    st = d_st.cpu().numpy()
    assert st[1234] == 0 and np.all(np.delete(st, 1234) == 0x10)
