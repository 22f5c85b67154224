"""The C-ABI library loads on the CPU, exports every entry point declared in
include/aqmp.h, and its ctypes mirrors match the C struct layouts."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aqmp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aqmp_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_calls():
    names = _declared()
    for want in ("aqmp_dictionary_build", "aqmp_encode", "aqmp_decode"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2605_09190_amd import aqmp as A
    names = _declared()
    for n in names:
        assert hasattr(A.lib, n), n
    assert sorted(A.EXPORTS) == names


def test_library_symbols_are_exported_extern_c():
    lib = os.path.join(ROOT, "paper_2605_09190_amd", "libaqmp.so")
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in _declared():
        assert n in syms, n


def _c_layout(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "aqmp.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("aqmp_image %zu\n", sizeof(aqmp_image)); P(aqmp_image, dtype); P(aqmp_image, row_stride);
  printf("aqmp_params %zu\n", sizeof(aqmp_params)); P(aqmp_params, tol_mode); P(aqmp_params, k_per_level);
  printf("aqmp_job %zu\n", sizeof(aqmp_job));
  printf("aqmp_options %zu\n", sizeof(aqmp_options)); P(aqmp_options, solver); P(aqmp_options, corr_variant_levels);
  printf("aqmp_leaf %zu\n", sizeof(aqmp_leaf)); P(aqmp_leaf, atom_off); P(aqmp_leaf, resid_sq);
  printf("aqmp_stats %zu\n", sizeof(aqmp_stats)); P(aqmp_stats, iters_executed);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.join(ROOT, 'include')}", str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return dict(l.rsplit(" ", 1) for l in out.strip().splitlines())


def test_struct_layouts_match_ctypes(tmp_path):
    from paper_2605_09190_amd import aqmp as A
    c = {k: int(v) for k, v in _c_layout(tmp_path).items()}
    assert c["aqmp_image"] == C.sizeof(A.Image)
    assert c["aqmp_image.row_stride"] == A.Image.row_stride.offset
    assert c["aqmp_params"] == C.sizeof(A.Params)
    assert c["aqmp_params.k_per_level"] == A.Params.k_per_level.offset
    assert c["aqmp_job"] == C.sizeof(A.Job)
    assert c["aqmp_options"] == C.sizeof(A.Options)
    assert c["aqmp_options.solver"] == A.Options.solver.offset
    assert c["aqmp_options.corr_variant_levels"] == A.Options.corr_variant_levels.offset
    assert c["aqmp_leaf"] == C.sizeof(A.Leaf) == A.LEAF_DTYPE.itemsize
    assert c["aqmp_leaf.atom_off"] == A.Leaf.atom_off.offset
    assert c["aqmp_stats"] == C.sizeof(A.Stats)
    assert c["aqmp_stats.iters_executed"] == A.Stats.iters_executed.offset


def test_invalid_arguments_fail_without_a_device():
    """Argument errors are reported before any device call."""
    from paper_2605_09190_amd import aqmp as A
    h = C.c_void_p()
    assert A.lib.aqmp_dictionary_build(3, 64, 3, None, C.byref(h)) == A.E_INVALID
    assert A.lib.aqmp_dictionary_build(8, 4, 3, None, C.byref(h)) == A.E_INVALID
    assert A.lib.aqmp_dictionary_build(8, 128, 3, None, C.byref(h)) == A.E_INVALID
    assert A.lib.aqmp_dictionary_build(8, 16, 4, None, C.byref(h)) == A.E_INVALID
    assert b"power" in A.lib.aqmp_last_error() or b"famil" in A.lib.aqmp_last_error()
    assert A.lib.aqmp_encode(None, None, 0, None, 0, None, 0, None, None, C.byref(h)) == A.E_INVALID
    m = C.c_int()
    assert A.lib.aqmp_dictionary_atoms(None, 8, C.byref(m)) == A.E_INVALID
    A.lib.aqmp_dictionary_free(None)
    A.lib.aqmp_code_free(None)


def test_corr_kernel_names():
    """The kernel-name query is host-only and reflects the per-size defaults."""
    from paper_2605_09190_amd import aqmp as A
    assert A.corr_kernel(64, A.PREC_BF16) == "k_corr_bf16_gen<64>"
    assert A.corr_kernel(32, A.PREC_BF16) == "k_corr_bf16_gen<32>"
    assert A.corr_kernel(32, A.PREC_BF16, 2) == "k_corr_bf16_dma<32,32,2>"
    assert A.corr_kernel(32, A.PREC_BF16, 3) == "k_corr_bf16<32>"
    assert A.corr_kernel(16, A.PREC_BF16) == "k_corr_bf16_dma<16,32,2>"
    assert A.corr_kernel(16, A.PREC_BF16, 6) == "k_corr_bf16<16>"       # generated atoms: N >= 32 only
    for removed in (1, 4, 5):                                             # removed forms are rejected
        assert A.corr_kernel(64, A.PREC_BF16, removed) == ""
    assert A.corr_kernel(64, A.PREC_FP32) == "k_corr_f32<64>"
    assert A.corr_kernel(8, A.PREC_BF16) == "k_pursuit_bf16<8>"
    assert A.corr_kernel(8, A.PREC_FP32) == "k_mp_fused<8>"
    assert A.corr_kernel(4, A.PREC_BF16) == "k_mp_fused<4>"
    assert A.corr_kernel(4, A.PREC_FP32) == "k_mp_fused<4>"
    assert A.corr_kernel(48, A.PREC_BF16) == ""
    assert A.corr_kernel(128, A.PREC_BF16) == ""
    assert A.corr_kernel(64, 7) == ""
    assert A.corr_kernel(64, A.PREC_BF16, 9) == ""


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library the binding raises; it has no fallback."""
    from paper_2605_09190_amd import aqmp as A
    monkeypatch.setattr(A, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libaqmp.so"))
    with pytest.raises(ImportError):
        A._load()


def test_product_never_uses_the_oracle():
    """The package (binding, search loop, build) does not import, call or
    read anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_2605_09190_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f), encoding="utf-8").read()
                assert not re.search(r"\boracle\b", src), f
