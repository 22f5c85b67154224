"""Error paths that need a device: AQMP_E_NODICT (a job uses a block size the
dictionary was not built for) and AQMP_E_NOMEM from the AQMP_MAX_DEVICE_BYTES
cap at encode time (in a child process, since the library reads the cap once
per process).  On failure no handle is created and nothing is left allocated
that a later encode would trip over."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_09190_amd import aqmp
    return aqmp


def test_nodict_when_a_block_size_is_missing(A):
    import torch
    d = A.Dictionary(8, 32)
    img = torch.rand(128, 128, dtype=torch.float32, device="cuda")
    with pytest.raises(A.AqmpError) as ei:
        A.Code(d, [img], [dict(tol=0.02, max_atoms=8, n_min=8, n_max=64)], [(0, 0)], precision=A.PREC_BF16,
               schedule=A.SCHED_BATCHED)
    assert ei.value.code == A.E_NODICT and "block size 64" in str(ei.value)
    with pytest.raises(A.AqmpError) as ei:
        d.atoms(64)
    assert ei.value.code == A.E_NODICT
    # the dictionary still works for the sizes it has
    code = A.Code(d, [img], [dict(tol=0.02, max_atoms=8, n_min=8, n_max=32)], [(0, 0)], precision=A.PREC_BF16,
                  schedule=A.SCHED_BATCHED)
    assert code.sizes()[0] > 0
    code.free()
    d.free()


CHILD = r'''
import sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_2605_09190_amd import aqmp as A
d = A.Dictionary(8, 32)
img = torch.rand(2048, 2048, dtype=torch.float32, device="cuda")
prm = [dict(tol=0.02, max_atoms=8, n_min=8, n_max=32)]
try:
    A.Code(d, [img], prm, [(0, 0)], precision=A.PREC_BF16, schedule=A.SCHED_BATCHED)
    print("no error")
except A.AqmpError as e:
    print("code", e.code, str(e))
small = torch.rand(64, 64, dtype=torch.float32, device="cuda")
c = A.Code(d, [small], prm, [(0, 0)], precision=A.PREC_BF16, schedule=A.SCHED_BATCHED)
print("small ok", c.sizes()[0] > 0)
'''


def test_nomem_from_the_cap_at_encode_time(A):
    # the dictionary (8..32) takes about 14 MB; a 2048^2 encode needs more than
    # 30 MB of work buffers, a 64^2 one well under 1 MB
    env = dict(os.environ, AQMP_MAX_DEVICE_BYTES=str(24 << 20))
    out = subprocess.run([sys.executable, "-u", "-c", CHILD, ROOT], env=env, capture_output=True, text=True,
                         timeout=240)
    print(out.stdout, out.stderr[-2000:], flush=True)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = out.stdout.strip().splitlines()
    assert lines[0].startswith("code -4") and "AQMP_MAX_DEVICE_BYTES" in lines[0]
    assert lines[1] == "small ok True"
