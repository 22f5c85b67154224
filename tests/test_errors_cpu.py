"""Error paths of the C ABI and of the binding that need no GPU.

* AQMP_E_NOMEM through the AQMP_MAX_DEVICE_BYTES cap: the cap is checked
  before any device allocation, so a dictionary build under a 1-byte cap
  fails with that code and message on any machine (run in a child process:
  the library reads the variable once).
* AQMP_E_INVALID for bad arguments, checked on the host before any HIP call.
* Code.decode rejects an output tensor of the wrong dtype, shape or device
  before it calls the library.
"""
import ctypes as C
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import ctypes as C, sys
sys.path.insert(0, sys.argv[1])
from paper_2605_09190_amd import aqmp as A
h = C.c_void_p()
rc = A.lib.aqmp_dictionary_build(4, 16, A.DCT | A.HAAR, None, C.byref(h))
print(rc, A.lib.aqmp_last_error().decode(), h.value is None)
'''


def test_nomem_from_the_device_byte_cap():
    env = dict(os.environ, AQMP_MAX_DEVICE_BYTES="1")
    out = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    rc, rest = out.stdout.strip().split(" ", 1)
    assert int(rc) == -4                                    # AQMP_E_NOMEM
    assert "AQMP_MAX_DEVICE_BYTES" in rest
    assert rest.endswith("True")                            # no handle created


def test_invalid_arguments_rejected_on_the_host():
    from paper_2605_09190_amd import aqmp as A
    h = C.c_void_p()
    assert A.lib.aqmp_dictionary_build(4, 128, A.DCT, None, C.byref(h)) == A.E_INVALID
    assert A.lib.aqmp_dictionary_build(8, 4, A.DCT, None, C.byref(h)) == A.E_INVALID
    assert A.lib.aqmp_dictionary_build(4, 8, 0, None, C.byref(h)) == A.E_INVALID
    assert A.lib.aqmp_dictionary_build(4, 8, A.DCT, None, None) == A.E_INVALID
    assert h.value is None
    assert A.lib.aqmp_encode(None, None, 0, None, 0, None, 0, None, None, C.byref(h)) == A.E_INVALID
    assert b"dictionary is null" in A.lib.aqmp_last_error()
    m = C.c_int()
    assert A.lib.aqmp_dictionary_atoms(None, 8, C.byref(m)) == A.E_INVALID
    assert A.lib.aqmp_decode(None, None, 0, None, 0, 0, None) == A.E_INVALID


class _FakeTensor:
    """Just the attributes Code.decode inspects; never reaches the library."""

    def __init__(self, shape, dtype, device="cuda:0", is_cuda=True):
        import torch
        self.shape = shape
        self.dtype = dtype
        self.is_cuda = is_cuda
        self.device = torch.device(device) if isinstance(device, str) else device

    def dim(self):
        return len(self.shape)

    def stride(self, i):
        return 1 if i == len(self.shape) - 1 else self.shape[-1]

    def data_ptr(self):
        raise AssertionError("decode must reject the tensor before using it")


def _code_stub(A):
    c = A.Code.__new__(A.Code)
    c.h = C.c_void_p()
    c.n_jobs = 2
    c._job_shape = [(64, 48), (32, 32)]
    c._keep = [_FakeTensor((64, 48), None)]
    return c


@pytest.mark.parametrize("shape,dtype,msg", [
    ((64, 48), "float16", "float32 or float64"),
    ((64, 48), "bfloat16", "float32 or float64"),
    ((64, 48), "int32", "float32 or float64"),
    ((63, 48), "float32", "plane is 64 x 48"),
    ((64, 47), "float64", "plane is 64 x 48"),
])
def test_decode_rejects_bad_outputs(shape, dtype, msg):
    import torch
    from paper_2605_09190_amd import aqmp as A
    c = _code_stub(A)
    with pytest.raises(ValueError, match=msg):
        c.decode(0, _FakeTensor(shape, getattr(torch, dtype)))
    c.h = C.c_void_p()


def test_decode_rejects_bad_job_and_device():
    import torch
    from paper_2605_09190_amd import aqmp as A
    c = _code_stub(A)
    with pytest.raises(ValueError, match="out of range"):
        c.decode(2, _FakeTensor((64, 48), torch.float32))
    with pytest.raises(ValueError, match="code is on"):
        c.decode(0, _FakeTensor((64, 48), torch.float32, device="cuda:1"))
