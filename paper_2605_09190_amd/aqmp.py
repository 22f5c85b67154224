"""Thin ctypes binding of libaqmp.so (the C ABI in include/aqmp.h).

Argument marshalling only: every step of the encoder and decoder runs in the
library's HIP kernels.  PyTorch tensors supply device memory and the HIP
stream.  Importing this module loads the library and fails loudly when it
has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
# torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading it first
# makes libaqmp.so bind to that same runtime instead of a second copy from
# /opt/rocm, which would not see the device once torch has initialised it.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaqmp.so")

# enums of aqmp.h
OK, E_INVALID, E_SHAPE, E_NODICT, E_NOMEM, E_HIP, E_CAPACITY = 0, -1, -2, -3, -4, -5, -6
DCT, HAAR = 1, 2
F32, F64 = 0, 1
TOL_RMS, TOL_ABS = 0, 1
SPLIT_R1, SPLIT_R2 = 0, 1
PREC_FP32, PREC_BF16 = 0, 1
SCHED_PLAIN, SCHED_BATCHED, SCHED_CONCURRENT = 0, 1, 2
OPT_TIMING = 1
OPT_STEPWISE = 2
SOLVER_DENSE, SOLVER_GRAM, SOLVER_OMP = 0, 1, 2
MAX_ATOMS = 256
CANDIDATES = 8

# Every entry point declared in include/aqmp.h.
EXPORTS = [
    "aqmp_dictionary_build", "aqmp_dictionary_free", "aqmp_dictionary_atoms", "aqmp_dictionary_copy",
    "aqmp_encode", "aqmp_reencode", "aqmp_code_sizes", "aqmp_code_export", "aqmp_code_export_nodes",
    "aqmp_code_stats", "aqmp_code_timing", "aqmp_code_free", "aqmp_decode", "aqmp_last_error",
    "aqmp_corr_kernel", "aqmp_code_pack", "aqmp_ssim", "aqmp_worklist_compact", "aqmp_worklist_split",
    "aqmp_worklist_compact_noalloc", "aqmp_code_pack_quantized", "aqmp_decode_quantized",
]


class Image(C.Structure):
    _fields_ = [("dev_ptr", C.c_void_p), ("dtype", C.c_int32), ("w", C.c_int32), ("h", C.c_int32),
                ("row_stride", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_mode", C.c_int32), ("max_atoms", C.c_int32),
                ("n_min", C.c_int32), ("n_max", C.c_int32), ("split_rule", C.c_int32),
                ("k_per_level", C.c_int32 * 7)]


class Job(C.Structure):
    _fields_ = [("image", C.c_int32), ("params", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("schedule", C.c_int32), ("flags", C.c_int32),
                ("corr_variant", C.c_int32), ("solver", C.c_int32),
                ("corr_variant_levels", C.c_uint32), ("corr_tile_levels", C.c_uint32), ("reserved", C.c_int32)]


class Leaf(C.Structure):
    _fields_ = [("job", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32), ("n", C.c_int32),
                ("n_atoms", C.c_int32), ("flags", C.c_int32), ("atom_off", C.c_int64),
                ("resid_sq", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("nodes", C.c_int64 * 7), ("leaves", C.c_int64 * 7), ("iters_level", C.c_int64 * 7),
                ("iters_executed", C.c_int64), ("iters_emitted", C.c_int64), ("steps_launched", C.c_int64)]


class Timing(C.Structure):
    _fields_ = [("corr_ms", C.c_double * 7), ("select_ms", C.c_double * 7), ("level_ms", C.c_double * 7),
                ("steps", C.c_int64 * 7)]


LEAF_DTYPE = np.dtype([("job", "<i4"), ("x0", "<i4"), ("y0", "<i4"), ("n", "<i4"), ("n_atoms", "<i4"),
                       ("flags", "<i4"), ("atom_off", "<i8"), ("resid_sq", "<f8")])


class AqmpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"aqmp error {code}: {msg}")
        self.code = code


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2605_09190_amd.build.build() first")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int, C.c_int64
    lib.aqmp_dictionary_build.argtypes = [i32, i32, C.c_uint32, vp, C.POINTER(vp)]
    lib.aqmp_dictionary_free.argtypes = [vp]
    lib.aqmp_dictionary_free.restype = None
    lib.aqmp_dictionary_atoms.argtypes = [vp, i32, C.POINTER(C.c_int)]
    lib.aqmp_dictionary_copy.argtypes = [vp, i32, C.POINTER(C.c_double)]
    lib.aqmp_encode.argtypes = [vp, C.POINTER(Image), i32, C.POINTER(Params), i32, C.POINTER(Job), i32,
                                C.POINTER(Options), vp, C.POINTER(vp)]
    lib.aqmp_reencode.argtypes = [vp, C.POINTER(Image), i32, vp]
    lib.aqmp_code_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
    lib.aqmp_code_export.argtypes = [vp, vp, vp, vp, i64, i64]
    lib.aqmp_code_export_nodes.argtypes = [vp, vp, vp, vp, i64, i64]
    lib.aqmp_code_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.aqmp_code_timing.argtypes = [vp, C.POINTER(Timing)]
    lib.aqmp_code_free.argtypes = [vp]
    lib.aqmp_code_free.restype = None
    lib.aqmp_decode.argtypes = [vp, vp, i32, vp, i32, i64, vp]
    lib.aqmp_last_error.argtypes = []
    lib.aqmp_last_error.restype = C.c_char_p
    lib.aqmp_corr_kernel.argtypes = [i32, i32, i32]
    lib.aqmp_corr_kernel.restype = C.c_char_p
    lib.aqmp_ssim.argtypes = [C.POINTER(Image), C.POINTER(Image), i32, C.c_double, C.POINTER(C.c_double), vp]
    lib.aqmp_code_pack.argtypes = [vp, C.POINTER(C.c_int32), i32, i32, vp, i64, C.POINTER(C.c_int64)]
    lib.aqmp_code_pack_quantized.argtypes = [vp, C.POINTER(C.c_int32), i32, i32, C.c_double, vp, i64,
                                             C.POINTER(C.c_int64)]
    lib.aqmp_decode_quantized.argtypes = [vp, vp, i32, C.c_double, vp, i32, i64, vp]
    lib.aqmp_worklist_compact.argtypes = [vp, i64, vp, vp, vp]
    lib.aqmp_worklist_compact_noalloc.argtypes = [vp, i64, vp, vp, vp]
    lib.aqmp_worklist_split.argtypes = [C.POINTER(Params), i32, i32, vp, vp, vp, vp, vp, i64, C.c_int32, vp, vp, vp,
                                        vp, vp, vp]
    for name in EXPORTS:
        if not hasattr(lib, name):
            raise ImportError(f"{LIB_PATH} lacks {name}")
    return lib


lib = _load()


def _check(rc: int) -> None:
    if rc != OK:
        raise AqmpError(rc, lib.aqmp_last_error().decode())


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# The BF16 correlation variants of the library (0 = its default per block size).
CORR_VARIANTS = (0, 2, 3, 6)


def pack_variant_levels(per_n) -> int:
    """{N: variant} -> the aqmp_options.corr_variant_levels word (one nibble
    per block size, at bits 4 log2(N))."""
    word = 0
    for n, v in dict(per_n).items():
        lg = int(n).bit_length() - 1
        if 1 << lg != int(n) or not 2 <= lg <= 6 or int(v) not in CORR_VARIANTS:
            raise ValueError(f"bad per-level variant {n}: {v}")
        word |= int(v) << (4 * lg)
    return word


def pack_tile_levels(per_n) -> int:
    """{N: (lo, hi)} -> the aqmp_options.corr_tile_levels word (byte 8 (log2 N - 5)
    = lo | hi << 4, for N = 32, 64)."""
    word = 0
    for n, (lo, hi) in dict(per_n).items():
        if int(n) not in (32, 64) or not 1 <= int(lo) <= int(hi) <= 7:
            raise ValueError(f"bad node-tile range {n}: {(lo, hi)}")
        word |= (int(lo) | int(hi) << 4) << (8 * (int(n).bit_length() - 1 - 5))
    return word


def corr_kernel(n: int, precision: int, corr_variant: int = 0) -> str:
    """Name of the correlation kernel an encode runs at block size n ("" if invalid)."""
    return lib.aqmp_corr_kernel(int(n), int(precision), int(corr_variant)).decode()


def make_params(tol: float, tol_mode: str = "rms", max_atoms: int = 32, n_min: int = 8, n_max: int = 64,
                split_rule: str = "r1", k_per_level: dict | None = None, **_ignored) -> Params:
    p = Params()
    p.tol = float(tol)
    p.tol_mode = {"rms": TOL_RMS, "abs": TOL_ABS}[tol_mode] if isinstance(tol_mode, str) else int(tol_mode)
    p.max_atoms = int(max_atoms)
    p.n_min, p.n_max = int(n_min), int(n_max)
    p.split_rule = {"r1": SPLIT_R1, "r2": SPLIT_R2}[split_rule] if isinstance(split_rule, str) else int(split_rule)
    for i in range(7):
        p.k_per_level[i] = -1
    if k_per_level:
        for n, k in k_per_level.items():
            p.k_per_level[int(n).bit_length() - 1] = int(k)
    return p


def make_image(t) -> Image:
    """Describes a 2D CUDA tensor (float32 or float64, unit column stride)."""
    import torch
    if t.dim() != 2 or not t.is_cuda or t.stride(1) != 1:
        raise ValueError("images must be 2D CUDA tensors with unit column stride")
    if t.dtype not in (torch.float32, torch.float64):
        raise ValueError("images must be float32 or float64")
    im = Image()
    im.dev_ptr = t.data_ptr()
    im.dtype = F32 if t.dtype == torch.float32 else F64
    im.h, im.w = int(t.shape[0]), int(t.shape[1])
    im.row_stride = int(t.stride(0))
    return im


SSIM_GLOBAL, SSIM_WINDOW7 = 0, 1


def ssim(x, y, mode: int = SSIM_WINDOW7, data_range: float = 1.0, stream=None) -> float:
    """SSIM of two 2D CUDA tensors of one shape and dtype (Section 3)."""
    a, b = make_image(x), make_image(y)
    out = C.c_double()
    _check(lib.aqmp_ssim(C.byref(a), C.byref(b), int(mode), float(data_range), C.byref(out), _stream_handle(stream)))
    return out.value


def _dev_tensor(t, dtype, name):
    import torch
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor")
    return t.data_ptr()


NOALLOC_MAX_ITEMS = 1 << 24


def worklist_compact(status, out, count, stream=None, noalloc: bool = False) -> None:
    """Active-list compaction: out[:count] = indices of the zero bytes of
    status, in order (aqmp_worklist_compact, or aqmp_worklist_compact_noalloc
    with noalloc=True).  status uint8, out int32 with room for len(status),
    count one int32; all CUDA tensors."""
    import torch
    n = int(status.numel())
    if out.numel() < n or count.numel() < 1:
        raise ValueError("out needs room for every item and count one element")
    fn = lib.aqmp_worklist_compact_noalloc if noalloc else lib.aqmp_worklist_compact
    _check(fn(_dev_tensor(status, torch.uint8, "status"), n,
                                     _dev_tensor(out, torch.int32, "out"), _dev_tensor(count, torch.int32, "count"),
                                     _stream_handle(stream)))


def worklist_split(params, n: int, node_prm, x0, y0, e, t, status, child_prm, child_x0, child_y0, child_count,
                   child_base: int = 0, stream=None) -> None:
    """Split test and child emission of one level (aqmp_worklist_split)."""
    import torch
    nn = int(node_prm.numel())
    for name, a in (("x0", x0), ("y0", y0), ("e", e), ("t", t), ("status", status)):
        if a.numel() != nn:
            raise ValueError(f"{name} must have one entry per node")
    for name, a in (("child_prm", child_prm), ("child_x0", child_x0), ("child_y0", child_y0)):
        if a.numel() < child_base + 4 * nn:
            raise ValueError(f"{name} needs child_base + 4 entries per node")
    prms = (Params * len(params))(*[p if isinstance(p, Params) else make_params(**p) for p in params])
    i32 = torch.int32
    _check(lib.aqmp_worklist_split(prms, len(params), int(n), _dev_tensor(node_prm, i32, "node_prm"),
                                   _dev_tensor(x0, i32, "x0"), _dev_tensor(y0, i32, "y0"),
                                   _dev_tensor(e, torch.float64, "e"), _dev_tensor(t, i32, "t"), nn, int(child_base),
                                   _dev_tensor(status, torch.uint8, "status"),
                                   _dev_tensor(child_prm, i32, "child_prm"), _dev_tensor(child_x0, i32, "child_x0"),
                                   _dev_tensor(child_y0, i32, "child_y0"),
                                   _dev_tensor(child_count, i32, "child_count"), _stream_handle(stream)))


class Dictionary:
    """D_N for N = n_min .. n_max (powers of two), DCT and/or Haar families."""

    def __init__(self, n_min: int = 4, n_max: int = 64, families: int = DCT | HAAR, stream=None):
        h = C.c_void_p()
        _check(lib.aqmp_dictionary_build(n_min, n_max, families, _stream_handle(stream), C.byref(h)))
        self.h = h
        self.n_min, self.n_max, self.families = n_min, n_max, families

    def atoms(self, n: int) -> int:
        m = C.c_int()
        _check(lib.aqmp_dictionary_atoms(self.h, n, C.byref(m)))
        return m.value

    def copy(self, n: int) -> np.ndarray:
        """D_N in FP64 as an (N*N, M) array; columns are column-major flattened atoms."""
        m = self.atoms(n)
        buf = np.empty(n * n * m, dtype=np.float64)
        _check(lib.aqmp_dictionary_copy(self.h, n, buf.ctypes.data_as(C.POINTER(C.c_double))))
        return buf.reshape(m, n * n).T

    def free(self) -> None:
        if self.h:
            lib.aqmp_dictionary_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclass
class Export:
    leaves: np.ndarray      # structured LEAF_DTYPE
    atom_idx: np.ndarray    # int32
    coef: np.ndarray        # float64


class Code:
    """An encode: the quadtree leaves and their atoms, kept on the device."""

    def __init__(self, dic: Dictionary, images, params, jobs, precision: int = PREC_FP32,
                 schedule: int = SCHED_PLAIN, stream=None, timing: bool = False, corr_variant: int = 0,
                 stepwise: bool = False, solver: int = 0, corr_variant_levels=None, corr_tile_levels=None):
        self.dic = dic
        self._keep = list(images)
        imgs = (Image * len(images))(*[make_image(t) for t in images])
        prms = (Params * len(params))(*[p if isinstance(p, Params) else make_params(**p) for p in params])
        jbs = (Job * len(jobs))(*[Job(int(a), int(b)) for a, b in jobs])
        opt = Options()
        opt.precision, opt.schedule = int(precision), int(schedule)
        opt.flags = (OPT_TIMING if timing else 0) | (OPT_STEPWISE if stepwise else 0)
        opt.corr_variant = int(corr_variant)
        opt.corr_variant_levels = pack_variant_levels(corr_variant_levels or {})
        opt.corr_tile_levels = pack_tile_levels(corr_tile_levels or {})
        opt.solver = int(solver)
        h = C.c_void_p()
        _check(lib.aqmp_encode(dic.h, imgs, len(images), prms, len(params), jbs, len(jobs), C.byref(opt),
                               _stream_handle(stream), C.byref(h)))
        self.h = h
        self.n_jobs = len(jobs)
        # (rows, columns) of each job's plane: the decode writes that many samples
        self._job_shape = [(int(images[int(a)].shape[0]), int(images[int(a)].shape[1])) for a, _ in jobs]

    def reencode(self, images, stream=None) -> None:
        self._keep = list(images)
        imgs = (Image * len(images))(*[make_image(t) for t in images])
        _check(lib.aqmp_reencode(self.h, imgs, len(images), _stream_handle(stream)))

    def sizes(self) -> tuple[int, int]:
        a, b = C.c_int64(), C.c_int64()
        _check(lib.aqmp_code_sizes(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def stats(self) -> dict:
        s = Stats()
        _check(lib.aqmp_code_stats(self.h, C.byref(s)))
        return dict(nodes=list(s.nodes), leaves=list(s.leaves), iters_level=list(s.iters_level),
                    iters_executed=s.iters_executed, iters_emitted=s.iters_emitted,
                    steps_launched=s.steps_launched)

    def timing(self) -> dict:
        t = Timing()
        _check(lib.aqmp_code_timing(self.h, C.byref(t)))
        return dict(corr_ms=list(t.corr_ms), select_ms=list(t.select_ms), level_ms=list(t.level_ms),
                    steps=list(t.steps))

    def _export(self, fn, n_rec: int, n_atoms: int) -> Export:
        leaves = np.zeros(max(n_rec, 1), dtype=LEAF_DTYPE)
        idx = np.zeros(max(n_atoms, 1), dtype=np.int32)
        coef = np.zeros(max(n_atoms, 1), dtype=np.float64)
        _check(fn(self.h, leaves.ctypes.data, idx.ctypes.data, coef.ctypes.data, n_rec, n_atoms))
        return Export(leaves[:n_rec], idx[:n_atoms], coef[:n_atoms])

    def export(self) -> Export:
        n_leaves, n_atoms = self.sizes()
        return self._export(lib.aqmp_code_export, n_leaves, n_atoms)

    def pack(self, jobs, level: int = 9, step: float = 0.0) -> bytes:
        """The AQMP bitstream of the given jobs (the channels of one image),
        DEFLATE-compressed at `level` (0..9) or raw (-1); step > 0 quantises
        the coefficients (coefficient format 1)."""
        arr = (C.c_int32 * len(jobs))(*[int(j) for j in jobs])
        size = C.c_int64()
        st = C.c_double(float(step))
        _check(lib.aqmp_code_pack_quantized(self.h, arr, len(jobs), int(level), st, None, 0, C.byref(size)))
        buf = (C.c_uint8 * max(1, size.value))()
        _check(lib.aqmp_code_pack_quantized(self.h, arr, len(jobs), int(level), st, buf, size.value, C.byref(size)))
        return bytes(buf[:size.value])

    def export_nodes(self) -> Export:
        s = self.stats()
        return self._export(lib.aqmp_code_export_nodes, int(sum(s["nodes"])), int(s["iters_executed"]))

    def decode(self, job: int, out, stream=None, step: float = 0.0) -> None:
        """Writes job's reconstruction into out (a 2D float32 or float64 CUDA
        tensor on the code's device, at least as large as the job's plane);
        step > 0 decodes the quantised coefficients of a format 1 stream."""
        import torch
        if not 0 <= int(job) < self.n_jobs:
            raise ValueError(f"job {job} out of range (0..{self.n_jobs - 1})")
        if out.dim() != 2 or not out.is_cuda or out.stride(1) != 1:
            raise ValueError("out must be a 2D CUDA tensor with unit column stride")
        if out.dtype not in (torch.float32, torch.float64):
            raise ValueError("out must be float32 or float64")
        h, w = self._job_shape[int(job)]
        if out.shape[0] < h or out.shape[1] < w:
            raise ValueError(f"out is {tuple(out.shape)}; the job's plane is {h} x {w}")
        if out.device != self._keep[0].device:
            raise ValueError(f"out is on {out.device}; the code is on {self._keep[0].device}")
        dt = F32 if out.dtype == torch.float32 else F64
        _check(lib.aqmp_decode_quantized(self.dic.h, self.h, job, float(step), out.data_ptr(), dt,
                                         int(out.stride(0)), _stream_handle(stream)))

    def free(self) -> None:
        if self.h:
            lib.aqmp_code_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
