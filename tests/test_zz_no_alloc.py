"""aqmp_worklist_compact_noalloc (no device allocation: the scan state is a
static device array of the library) against aqmp_worklist_compact, through
the C ABI: identical outputs bit for bit, on two calls in a row, the second
with a smaller input (the array keeps the first call's contents, which the
second must clear), plus the size limit."""
import ctypes as C
import sys

import numpy as np
import pytest

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


def _run(A, fn, st_dev, n):
    import torch
    out = torch.full((max(n, 1),), -5, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = fn(C.c_void_p(st_dev.data_ptr()), C.c_int64(n), C.c_void_p(out.data_ptr()), C.c_void_p(cnt.data_ptr()),
            C.c_void_p(stream))
    assert rc == A.OK, A.lib.aqmp_last_error().decode()
    return out.cpu().numpy(), int(cnt.item())


@pytest.mark.parametrize("sizes", [(1_000_000, 70_001), (3 * 1024 + 5, 1)])
def test_noalloc_matches_the_allocating_call(A, sizes):
    import torch
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(77 + n)
        st = rng.choice(np.array([0, 1, 2, 0x10], dtype=np.uint8), size=n, p=[0.6, 0.2, 0.1, 0.1])
        d_st = torch.from_numpy(st).cuda()
        _say("noalloc call", i, "n", n)
        got, c = _run(A, A.lib.aqmp_worklist_compact_noalloc, d_st, n)
        ref, c_ref = _run(A, A.lib.aqmp_worklist_compact, d_st, n)
        assert c == c_ref == int(np.sum(st == 0))
        assert np.array_equal(got, ref)
        assert np.array_equal(got[:c], np.nonzero(st == 0)[0].astype(np.int32))


def test_noalloc_rejects_sizes_beyond_its_static_state(A):
    import torch
    n = A.NOALLOC_MAX_ITEMS + 1
    # nothing is launched: the size is checked on the host first
    rc = A.lib.aqmp_worklist_compact_noalloc(C.c_void_p(1), C.c_int64(n), C.c_void_p(1), C.c_void_p(1),
                                             C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == A.E_INVALID
    assert b"exceeds the static scan state" in A.lib.aqmp_last_error()
