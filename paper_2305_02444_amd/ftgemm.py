"""ctypes binding of libftgemm (include/ftgemm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libftgemm.so.  Matrices are torch tensors on a ROCm device,
holding column-major (BLAS) data: a tensor X of shape (rows, cols) with
X.stride(0) == 1 and X.stride(1) == ld >= rows (``colmajor_empty`` and
``to_device`` make such tensors).  If the library has not been built the
import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftgemm.so")
HEADER = os.path.join(HERE, "..", "include", "ftgemm.h")

OP_N, OP_T = 0, 1
F64, BF16, FP8_E4M3 = 0, 1, 2
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NO_MEMORY = 0, 1, 2, 3, 4
KIND_CORRECTED, KIND_CHECKSUM_ONLY, KIND_RECOMPUTED, KIND_UNCORRECTABLE = 1, 2, 3, 4
INJ_ADD, INJ_BITFLIP = 0, 1
TGT_ACC, TGT_ROW_CHECKSUM, TGT_COL_CHECKSUM, TGT_WEIGHTED_CHECKSUM = 0, 1, 2, 3


class FaultRecord(C.Structure):
    _fields_ = [("problem", C.c_int32), ("kind", C.c_int32), ("tile_m", C.c_int32),
                ("tile_n", C.c_int32), ("row", C.c_int64), ("col", C.c_int64),
                ("nbad_rows", C.c_int32), ("nbad_cols", C.c_int32), ("d_row", C.c_double),
                ("d_col", C.c_double), ("tau_row", C.c_double), ("tau_col", C.c_double),
                ("before", C.c_double), ("after", C.c_double)]


class InjectionEcho(C.Structure):
    _fields_ = [("problem", C.c_int32), ("applied", C.c_int32), ("row", C.c_int64),
                ("col", C.c_int64), ("k_index", C.c_int64), ("before", C.c_double),
                ("after", C.c_double)]


class Report(C.Structure):
    _fields_ = [("tiles_verified", C.c_uint64), ("detected", C.c_uint64),
                ("corrected", C.c_uint64), ("checksum_only", C.c_uint64),
                ("recomputed", C.c_uint64), ("uncorrectable", C.c_uint64),
                ("max_ratio", C.c_double), ("record_count", C.c_uint32),
                ("echo_count", C.c_uint32), ("record_capacity", C.c_uint32),
                ("echo_capacity", C.c_uint32), ("records", C.POINTER(FaultRecord)),
                ("echoes", C.POINTER(InjectionEcho))]


class Injection(C.Structure):
    _fields_ = [("problem", C.c_int32), ("mode", C.c_int32), ("target", C.c_int32),
                ("bit", C.c_int32), ("row", C.c_int64), ("col", C.c_int64),
                ("k_index", C.c_int64), ("delta", C.c_double)]


class GemmDesc(C.Structure):
    _fields_ = [("dtype", C.c_int), ("transA", C.c_int), ("transB", C.c_int),
                ("abft", C.c_int32), ("m", C.c_int64), ("n", C.c_int64), ("k", C.c_int64),
                ("lda", C.c_int64), ("ldb", C.c_int64), ("ldc", C.c_int64),
                ("alpha", C.c_double), ("beta", C.c_double), ("scaleA", C.c_double),
                ("scaleB", C.c_double), ("A", C.c_void_p), ("B", C.c_void_p),
                ("C", C.c_void_p)]


def exported_functions_in_header(path: str = HEADER):
    """Names of the functions include/ftgemm.h declares."""
    text = open(path).read()
    return sorted(set(re.findall(r"^[A-Za-z_][A-Za-z0-9_ *]*?\b(ftgemm_[a-z_]+)\s*\(",
                                 text, re.M)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes libftgemm bind to that one copy instead of a second one.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libftgemm.so is not built (python -m paper_2305_02444_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i64, dbl = C.c_void_p, C.c_int64, C.c_double
        L.ftgemm_gemm.restype = C.c_int
        L.ftgemm_gemm.argtypes = [C.c_int, C.c_int, i64, i64, i64, dbl, vp, i64, vp, i64, dbl,
                                  vp, i64, C.POINTER(Report), vp]
        L.ftgemm_gemm_ex.restype = C.c_int
        L.ftgemm_gemm_ex.argtypes = [C.POINTER(GemmDesc), C.POINTER(Report), vp]
        L.ftgemm_batch_tiling.restype = C.c_int
        L.ftgemm_batch_tiling.argtypes = [C.c_int32, C.POINTER(GemmDesc), C.POINTER(C.c_int32)]
        L.ftgemm_load_tune_table.restype = C.c_int
        L.ftgemm_load_tune_table.argtypes = [C.c_char_p]
        L.ftgemm_gemm_ex_noalloc.restype = C.c_int
        L.ftgemm_gemm_ex_noalloc.argtypes = [C.POINTER(GemmDesc), C.POINTER(Report), vp]
        for name in ("ftgemm_gemm_batched", "ftgemm_gemm_batched_loop"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = [C.c_int32, C.POINTER(GemmDesc), C.POINTER(Report), vp]
        L.ftgemm_set_fault_plan.restype = C.c_int
        L.ftgemm_set_fault_plan.argtypes = [C.POINTER(Injection), C.c_int32]
        L.ftgemm_query_tiling.restype = C.c_int
        L.ftgemm_query_tiling.argtypes = [C.c_int, i64, i64, i64] + [C.POINTER(C.c_int32)] * 4
        L.ftgemm_query_tiling_ex.restype = C.c_int
        L.ftgemm_query_tiling_ex.argtypes = [C.POINTER(GemmDesc)] + [C.POINTER(C.c_int32)] * 4
        L.ftgemm_last_invalid_arg.restype = C.c_int32
        L.ftgemm_last_invalid_arg.argtypes = []
        L.ftgemm_status_string.restype = C.c_char_p
        L.ftgemm_status_string.argtypes = [C.c_int]
        L.ftgemm_finalize.restype = None
        L.ftgemm_finalize.argtypes = []
        _lib = L
    return _lib


class FTGemmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.position = lib().ftgemm_last_invalid_arg() if status == ERR_INVALID_ARG else 0
        msg = lib().ftgemm_status_string(status).decode()
        if self.position:
            msg += " (argument %d)" % self.position
        super().__init__("%s: %s" % (where, msg))


def _check(status, where):
    if status != OK:
        raise FTGemmError(status, where)


# -- tensors ------------------------------------------------------------------

def colmajor_empty(rows, cols, dtype, device="cuda", ld=None):
    """Device tensor (rows, cols) with column-major strides (1, ld)."""
    import torch
    ld = max(1, rows) if ld is None else ld
    base = torch.empty((max(cols, 1), ld), dtype=dtype, device=device)
    return base[:cols, :rows].t() if cols > 0 else base[:0, :rows].t()


def to_device(x, dtype=None, device="cuda", ld=None):
    """Copy a column-major numpy array (or torch tensor) to a device tensor
    with column-major strides."""
    import numpy as np
    import torch
    if isinstance(x, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(x.T)).t()
    else:
        t = x
    dtype = t.dtype if dtype is None else dtype
    out = colmajor_empty(t.shape[0], t.shape[1], dtype, device, ld)
    out.copy_(t.to(dtype) if t.dtype != dtype else t)
    return out


def _ld(t):
    if t.dim() != 2:
        raise ValueError("matrices must be 2-D")
    if t.shape[0] > 1 and t.stride(0) != 1:
        raise ValueError("matrices must be column-major (stride(0) == 1)")
    return max(t.stride(1), max(t.shape[0], 1)) if t.shape[1] > 1 else max(t.shape[0], 1)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# -- reports ------------------------------------------------------------------

@dataclass
class ReportView:
    tiles_verified: int
    detected: int
    corrected: int
    checksum_only: int
    recomputed: int
    uncorrectable: int
    max_ratio: float
    record_count: int
    echo_count: int
    records: list = field(default_factory=list)
    echoes: list = field(default_factory=list)


class ReportBuffer:
    def __init__(self, record_capacity=4096, echo_capacity=4096):
        self.recs = (FaultRecord * max(record_capacity, 1))()
        self.echo = (InjectionEcho * max(echo_capacity, 1))()
        self.rep = Report()
        self.rep.record_capacity = record_capacity
        self.rep.echo_capacity = echo_capacity
        self.rep.records = C.cast(self.recs, C.POINTER(FaultRecord))
        self.rep.echoes = C.cast(self.echo, C.POINTER(InjectionEcho))

    def view(self) -> ReportView:
        r = self.rep
        recs = []
        for x in self.recs[:min(r.record_count, r.record_capacity)]:
            recs.append(dict(problem=x.problem, kind=x.kind, tile_m=x.tile_m, tile_n=x.tile_n,
                             row=x.row, col=x.col, nbad_rows=x.nbad_rows,
                             nbad_cols=x.nbad_cols, d_row=x.d_row, d_col=x.d_col,
                             tau_row=x.tau_row, tau_col=x.tau_col, before=x.before,
                             after=x.after))
        recs.sort(key=lambda d: (d["problem"], d["tile_n"], d["tile_m"]))
        ech = [dict(problem=e.problem, applied=bool(e.applied), row=e.row, col=e.col,
                    k_index=e.k_index, before=e.before, after=e.after)
               for e in self.echo[:min(r.echo_count, r.echo_capacity)]]
        return ReportView(r.tiles_verified, r.detected, r.corrected, r.checksum_only,
                          r.recomputed, r.uncorrectable, r.max_ratio, r.record_count,
                          r.echo_count, recs, ech)


# -- entry points ---------------------------------------------------------------

_DTYPE_CODE = {}


def _dtype_code(t):
    import torch
    if not _DTYPE_CODE:
        _DTYPE_CODE.update({torch.float64: F64, torch.bfloat16: BF16,
                            torch.float8_e4m3fn: FP8_E4M3, torch.uint8: FP8_E4M3})
    return _DTYPE_CODE[t.dtype]


def make_desc(A, B, Cm, alpha=1.0, beta=0.0, transA=False, transB=False, abft=True,
              scaleA=1.0, scaleB=1.0, dtype=None):
    m, n = Cm.shape
    k = A.shape[0] if transA else A.shape[1]
    d = GemmDesc()
    d.dtype = _dtype_code(A) if dtype is None else dtype
    d.transA = OP_T if transA else OP_N
    d.transB = OP_T if transB else OP_N
    # abft: False / True, or the mode number (0, 1, 2 = one-sided, 3 = unfused,
    # 4 = weighted)
    d.abft = int(abft) if not isinstance(abft, bool) else (1 if abft else 0)
    d.m, d.n, d.k = m, n, k
    d.lda, d.ldb, d.ldc = _ld(A), _ld(B), _ld(Cm)
    d.alpha, d.beta = float(alpha), float(beta)
    d.scaleA, d.scaleB = float(scaleA), float(scaleB)
    d.A, d.B, d.C = A.data_ptr(), B.data_ptr(), Cm.data_ptr()
    return d


def gemm(A, B, Cm, alpha=1.0, beta=0.0, transA=False, transB=False, report=None,
         stream=None):
    """FP64 fault-tolerant GEMM: Cm <- alpha op(A) op(B) + beta Cm.
    report: a ReportBuffer to fill (the call then waits for the stream)."""
    m, n = Cm.shape
    k = A.shape[0] if transA else A.shape[1]
    rp = C.byref(report.rep) if report is not None else None
    st = lib().ftgemm_gemm(OP_T if transA else OP_N, OP_T if transB else OP_N, m, n, k,
                           float(alpha), A.data_ptr(), _ld(A), B.data_ptr(), _ld(B),
                           float(beta), Cm.data_ptr(), _ld(Cm), rp, _stream(stream))
    _check(st, "ftgemm_gemm")


def gemm_ex(desc: GemmDesc, report=None, stream=None):
    rp = C.byref(report.rep) if report is not None else None
    _check(lib().ftgemm_gemm_ex(C.byref(desc), rp, _stream(stream)), "ftgemm_gemm_ex")


def batch_tiling(descs):
    """Rows of the tiles each problem takes in gemm_batched now."""
    arr = (GemmDesc * len(descs))(*descs)
    rows = (C.c_int32 * max(len(descs), 1))()
    _check(lib().ftgemm_batch_tiling(len(descs), arr, rows), "ftgemm_batch_tiling")
    return [int(r) for r in rows[:len(descs)]]


def load_tune_table(path=None):
    """Replace the tuning table with the file at path (None: empty)."""
    _check(lib().ftgemm_load_tune_table(path.encode() if path else None),
           "ftgemm_load_tune_table")


def gemm_ex_noalloc(desc: GemmDesc, report=None, stream=None):
    rp = C.byref(report.rep) if report is not None else None
    _check(lib().ftgemm_gemm_ex_noalloc(C.byref(desc), rp, _stream(stream)),
           "ftgemm_gemm_ex_noalloc")


def gemm_batched(descs, reports=None, stream=None, loop=False):
    arr = (GemmDesc * len(descs))(*descs)
    if reports is not None:
        reps = (Report * len(descs))(*[r.rep for r in reports])
    else:
        reps = None
    f = lib().ftgemm_gemm_batched_loop if loop else lib().ftgemm_gemm_batched
    _check(f(len(descs), arr, reps, _stream(stream)), "ftgemm_gemm_batched")
    if reports is not None:
        for r, src in zip(reports, reps):
            r.rep = src


def set_fault_plan(faults):
    """faults: iterable of objects with row, col, k_index, mode, delta, bit,
    target and (optionally) problem attributes.  Empty clears the plan."""
    faults = list(faults)
    arr = (Injection * max(len(faults), 1))()
    for q, f in enumerate(faults):
        arr[q] = Injection(int(getattr(f, "problem", 0)), int(f.mode), int(f.target),
                           int(f.bit), int(f.row), int(f.col), int(f.k_index), float(f.delta))
    _check(lib().ftgemm_set_fault_plan(arr, len(faults)), "ftgemm_set_fault_plan")


def clear_fault_plan():
    _check(lib().ftgemm_set_fault_plan(None, 0), "ftgemm_set_fault_plan")


def query_tiling(dtype, m, n, k):
    v = [C.c_int32() for _ in range(4)]
    _check(lib().ftgemm_query_tiling(dtype, m, n, k, *[C.byref(x) for x in v]),
           "ftgemm_query_tiling")
    return tuple(x.value for x in v)


def query_tiling_ex(dtype, m, n, k, abft=1):
    """Tiling of the call with this dtype, shape and abft mode."""
    d = GemmDesc()
    d.dtype, d.abft, d.m, d.n, d.k = dtype, int(abft), m, n, k
    v = [C.c_int32() for _ in range(4)]
    _check(lib().ftgemm_query_tiling_ex(C.byref(d), *[C.byref(x) for x in v]),
           "ftgemm_query_tiling_ex")
    return tuple(x.value for x in v)
