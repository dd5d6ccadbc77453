"""Python face of the CPU oracle (test infrastructure only).

The oracle is the plain, slow statement of the fault-tolerant GEMM written
from the paper (FT-GEMM, HPDC'23: Section 2.1 for the GEMM, Sections 2.2 and
2.3 for the checksum encoding, verification and the per-part split).  It is
loaded only by the test suite, the smoke check and the CPU-baseline leg of
the benchmark.  It shares no code with the GPU library.

All matrices are float64 numpy arrays in column-major (Fortran) order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ftgemm_oracle.c")
LIB = os.path.join(HERE, "libftgemm_oracle.so")

# Fault modes / targets / record kinds, as defined in ftgemm_oracle.c.
ADD, BITFLIP = 0, 1
TGT_ACC, TGT_ROW_CHECKSUM, TGT_COL_CHECKSUM, TGT_WEIGHTED_CHECKSUM = 0, 1, 2, 3
CORRECTED, CHECKSUM_ONLY, RECOMPUTED, UNCORRECTABLE = 1, 2, 3, 4

DEFAULT_LAMBDA = 8.0


LIB_NATIVE = os.path.join(HERE, "libftgemm_oracle_native.so")


def compile_source(src: str, out: str, native: bool = False) -> str:
    """gcc -O3 with OpenMP: portable x86-64 code, or (native) code for the
    host it is built on (-march=native), as the CPU baseline is timed."""
    tmp = out + ".tmp%d" % os.getpid()
    arch = ["-march=native"] if native else []
    subprocess.check_call(["gcc", "-O3"] + arch + ["-std=c11", "-fPIC", "-shared", "-fopenmp",
                           "-Wall", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_source(SRC, LIB)
    return LIB


def native() -> "Oracle":
    """The same source built for the host it runs on (compiled on first use,
    there: the build container's CPU may differ from the one timed)."""
    compile_source(SRC, LIB_NATIVE, native=True)
    return Oracle(LIB_NATIVE)


class _Inj(C.Structure):
    _fields_ = [("row", C.c_int64), ("col", C.c_int64), ("k_index", C.c_int64),
                ("mode", C.c_int32), ("target", C.c_int32), ("delta", C.c_double),
                ("bit", C.c_int32), ("pad", C.c_int32)]


class _Rec(C.Structure):
    _fields_ = [("tile_m", C.c_int64), ("tile_n", C.c_int64), ("row", C.c_int64),
                ("col", C.c_int64), ("kind", C.c_int32), ("nbad_rows", C.c_int32),
                ("nbad_cols", C.c_int32), ("pad", C.c_int32), ("d_row", C.c_double),
                ("d_col", C.c_double), ("tau_row", C.c_double), ("tau_col", C.c_double),
                ("before", C.c_double), ("after", C.c_double)]


class _Echo(C.Structure):
    _fields_ = [("row", C.c_int64), ("col", C.c_int64), ("k_index", C.c_int64),
                ("applied", C.c_int32), ("pad", C.c_int32), ("before", C.c_double),
                ("after", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("ta", C.c_int32), ("tb", C.c_int32), ("m", C.c_int64), ("n", C.c_int64),
                ("k", C.c_int64), ("lda", C.c_int64), ("ldb", C.c_int64), ("ldc", C.c_int64),
                ("alpha", C.c_double), ("beta", C.c_double), ("tm", C.c_int64),
                ("tn", C.c_int64), ("bk", C.c_int64), ("acc_bits", C.c_int32),
                ("correct", C.c_int32), ("lam", C.c_double), ("mma_grid", C.c_double),
                ("mma_group", C.c_int32), ("one_sided", C.c_int32), ("weighted", C.c_int32),
                ("slice_k", C.c_int64)]


@dataclass
class Injection:
    row: int
    col: int
    k_index: int
    mode: int = ADD
    delta: float = 0.0
    bit: int = 0
    target: int = TGT_ACC


@dataclass
class FTResult:
    C: np.ndarray            # corrected output (only processed tiles are written)
    raw: np.ndarray          # output before correction
    records: list            # one dict per tile with a detection
    echo: list               # per injection: applied, before, after
    max_ratio: float         # max |d| / tau over checksums that passed


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _dims(A, B, ta, tb):
    m = A.shape[1] if ta else A.shape[0]
    k = A.shape[0] if ta else A.shape[1]
    kb = B.shape[1] if tb else B.shape[0]
    n = B.shape[0] if tb else B.shape[1]
    if kb != k:
        raise ValueError("inner dimensions of op(A) and op(B) differ")
    return m, n, k


class Oracle:
    """ctypes wrapper around one build of ftgemm_oracle.c."""

    def __init__(self, path: str):
        L = C.CDLL(path)
        dp, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.oracle_bf16_value.restype = C.c_double
        L.oracle_bf16_value.argtypes = [C.c_uint16]
        L.oracle_e4m3_value.restype = C.c_double
        L.oracle_e4m3_value.argtypes = [C.c_uint8]
        L.oracle_decode_bf16.argtypes = [C.c_void_p, dp, C.c_int64]
        L.oracle_decode_e4m3.argtypes = [C.c_void_p, dp, C.c_int64]
        L.oracle_gemm.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_int64,
                                  C.c_double, dp, C.c_int64, dp, C.c_int64, C.c_double,
                                  dp, C.c_int64, dp, C.c_int64]
        L.oracle_gemm_entries.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_double, dp,
                                          C.c_int64, dp, C.c_int64, C.c_double, dp,
                                          C.c_int64, i64p, i64p, C.c_int64, dp]
        L.oracle_ftgemm.restype = C.c_int64
        L.oracle_ftgemm.argtypes = [C.POINTER(_Params), dp, dp, dp, dp, C.c_int64, dp,
                                    C.POINTER(_Inj), C.c_int64, i64p, C.c_int64,
                                    C.POINTER(_Rec), C.c_int64, C.POINTER(_Echo), dp]
        L.oracle_tile_thresholds.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_int64,
                                             C.c_int64, dp, dp]
        L.oracle_tile_checksums.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_int64,
                                            C.c_int64, dp, dp, dp, dp]
        L.oracle_set_threads.restype = C.c_int32
        L.oracle_set_threads.argtypes = [C.c_int32]
        L.oracle_tile_weighted.argtypes = [C.POINTER(_Params), dp, dp, dp, C.c_int64,
                                           C.c_int64, dp, dp, dp]
        L.oracle_sizeof.restype = C.c_int64
        L.oracle_sizeof.argtypes = [C.c_int]
        for idx, cls in enumerate((_Inj, _Rec, _Echo, _Params)):
            assert L.oracle_sizeof(idx) == C.sizeof(cls), cls
        self.L = L

    def set_threads(self, n: int) -> int:
        """OpenMP threads of the following calls; returns the previous count."""
        return int(self.L.oracle_set_threads(int(n)))

    # -- number formats ---------------------------------------------------
    def decode_bf16(self, bits):
        bits = np.ascontiguousarray(bits, dtype=np.uint16)
        out = np.empty(bits.shape, dtype=np.float64)
        self.L.oracle_decode_bf16(bits.ctypes.data, _dptr(out), bits.size)
        return out

    def decode_e4m3(self, bits):
        bits = np.ascontiguousarray(bits, dtype=np.uint8)
        out = np.empty(bits.shape, dtype=np.float64)
        self.L.oracle_decode_e4m3(bits.ctypes.data, _dptr(out), bits.size)
        return out

    # -- plain GEMM -------------------------------------------------------
    def gemm(self, A, B, Cin=None, alpha=1.0, beta=0.0, ta=False, tb=False):
        """C = alpha op(A) op(B) + beta Cin, FP64 triple loop (Section 2.1)."""
        A, B = _f64(A), _f64(B)
        m, n, k = _dims(A, B, ta, tb)
        Cin = np.zeros((max(m, 1), max(n, 1)), order="F") if Cin is None else _f64(Cin)
        out = np.empty((m, n), order="F")
        self.L.oracle_gemm(int(ta), int(tb), m, n, k, alpha, _dptr(A), max(1, A.shape[0]),
                           _dptr(B), max(1, B.shape[0]), beta, _dptr(Cin),
                           max(1, Cin.shape[0]), _dptr(out), max(1, m))
        return out

    def gemm_entries(self, A, B, rows, cols, Cin=None, alpha=1.0, beta=0.0, ta=False,
                     tb=False, k=None):
        """C[rows[t], cols[t]] of the plain GEMM, one dot product each.  With k
        given, only the first k terms of each inner product are summed."""
        A, B = _f64(A), _f64(B)
        m, n, kk = _dims(A, B, ta, tb)
        k = kk if k is None else k
        Cin = np.zeros((1, 1), order="F") if Cin is None else _f64(Cin)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(rows.shape, dtype=np.float64)
        i64p = C.POINTER(C.c_int64)
        self.L.oracle_gemm_entries(int(ta), int(tb), k, alpha, _dptr(A), max(1, A.shape[0]),
                                   _dptr(B), max(1, B.shape[0]), beta, _dptr(Cin),
                                   max(1, Cin.shape[0]), rows.ctypes.data_as(i64p),
                                   cols.ctypes.data_as(i64p), rows.size, _dptr(out))
        return out

    # -- fault-tolerant GEMM ----------------------------------------------
    def _params(self, A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, acc_bits, correct, lam,
                mma=(0.0, 1), one_sided=False, slice_k=0, weighted=False):
        m, n, k = _dims(A, B, ta, tb)
        return _Params(int(ta), int(tb), m, n, k, max(1, A.shape[0]), max(1, B.shape[0]),
                       max(1, Cin.shape[0]), alpha, beta, tm, tn, bk, acc_bits,
                       int(correct), lam, float(mma[0]), int(mma[1]), int(bool(one_sided)),
                       int(bool(weighted)), int(slice_k))

    def ftgemm(self, A, B, Cin=None, alpha=1.0, beta=0.0, ta=False, tb=False, tm=128,
               tn=128, bk=16, acc_bits=64, injections=(), tiles=None, correct=True,
               lam=DEFAULT_LAMBDA, mma=(0.0, 1), one_sided=False, slice_k=0, weighted=False):
        """Fault-tolerant GEMM, tile by tile (Sections 2.2 and 2.3).  mma:
        (grid, group) of a multiplier that truncates its in-instruction
        sums, which widens the thresholds; (0, 1) for exact sums.
        one_sided: only the column checksum (one entry per row) is kept, and
        a tile with any disagreeing row is computed again.
        slice_k: 0, or the length of the slices of a split inner dimension;
        each slice is verified as a tile of its own and the reduction of the
        slices is verified against their summed checksums (records: one per
        slice that found something, then one for the reduction).
        weighted: each tile also keeps a weighted row checksum per column
        (weights i + 1 over its rows), which locates and confirms
        corrections of several errors."""
        A, B = _f64(A), _f64(B)
        m, n, k = _dims(A, B, ta, tb)
        Cin = np.zeros((max(m, 1), max(n, 1)), order="F") if Cin is None else _f64(Cin)
        P = self._params(A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, acc_bits, correct, lam,
                         mma, one_sided, slice_k, weighted)
        out = np.full((m, n), np.nan, order="F")
        raw = np.full((m, n), np.nan, order="F")
        inj = list(injections)
        inj_arr = (_Inj * max(len(inj), 1))()
        for q, f in enumerate(inj):
            inj_arr[q] = _Inj(f.row, f.col, f.k_index, f.mode, f.target, f.delta, f.bit, 0)
        echo = (_Echo * max(len(inj), 1))()
        if tiles is None:
            tl, nt = None, 0
            tl_arr = None
        else:
            tl_arr = np.ascontiguousarray(tiles, dtype=np.int64)
            tl, nt = tl_arr.ctypes.data_as(C.POINTER(C.c_int64)), tl_arr.size
        ntiles = (-(-m // tm)) * (-(-n // tn)) if m > 0 and n > 0 else 0
        per_tile = (-(-k // slice_k) + 1) if 0 < slice_k < k else 1
        cap = max(ntiles if tiles is None else nt, 1) * per_tile
        recs = (_Rec * cap)()
        mr = C.c_double(0.0)
        nrec = self.L.oracle_ftgemm(C.byref(P), _dptr(A), _dptr(B), _dptr(Cin), _dptr(out),
                                    max(1, m), _dptr(raw), inj_arr, len(inj), tl, nt, recs,
                                    cap, echo, C.byref(mr))
        records = [dict(tile_m=r.tile_m, tile_n=r.tile_n, row=r.row, col=r.col, kind=r.kind,
                        nbad_rows=r.nbad_rows, nbad_cols=r.nbad_cols, d_row=r.d_row,
                        d_col=r.d_col, tau_row=r.tau_row, tau_col=r.tau_col,
                        before=r.before, after=r.after) for r in recs[:min(nrec, cap)]]
        records.sort(key=lambda d: (d["tile_n"], d["tile_m"]))
        ech = [dict(row=e.row, col=e.col, k_index=e.k_index, applied=bool(e.applied),
                    before=e.before, after=e.after) for e in echo[:len(inj)]]
        return FTResult(out, raw, records, ech, mr.value)

    def tile_thresholds(self, A, B, tile_m, tile_n, Cin=None, alpha=1.0, beta=0.0,
                        ta=False, tb=False, tm=128, tn=128, bk=16, acc_bits=64,
                        lam=DEFAULT_LAMBDA, mma=(0.0, 1)):
        """(tau_row[w], tau_col[h]) of one tile."""
        A, B = _f64(A), _f64(B)
        m, n, k = _dims(A, B, ta, tb)
        Cin = np.zeros((max(m, 1), max(n, 1)), order="F") if Cin is None else _f64(Cin)
        P = self._params(A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, acc_bits, True, lam, mma)
        h = min(tm, m - tile_m * tm)
        w = min(tn, n - tile_n * tn)
        tr, tc = np.empty(w), np.empty(h)
        self.L.oracle_tile_thresholds(C.byref(P), _dptr(A), _dptr(B), _dptr(Cin), tile_m,
                                      tile_n, _dptr(tr), _dptr(tc))
        return tr, tc

    def tile_checksums(self, A, B, tile_m, tile_n, Cin=None, alpha=1.0, beta=0.0,
                       ta=False, tb=False, tm=128, tn=128, bk=16):
        """Encoded (Pr, Pc) and reference (Rr, Rc) checksums of one fault-free tile."""
        A, B = _f64(A), _f64(B)
        m, n, k = _dims(A, B, ta, tb)
        Cin = np.zeros((max(m, 1), max(n, 1)), order="F") if Cin is None else _f64(Cin)
        P = self._params(A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, 64, True,
                         DEFAULT_LAMBDA)
        h = min(tm, m - tile_m * tm)
        w = min(tn, n - tile_n * tn)
        Pr, Pc, Rr, Rc = np.empty(w), np.empty(h), np.empty(w), np.empty(h)
        self.L.oracle_tile_checksums(C.byref(P), _dptr(A), _dptr(B), _dptr(Cin), tile_m,
                                     tile_n, _dptr(Pr), _dptr(Pc), _dptr(Rr), _dptr(Rc))
        return Pr, Pc, Rr, Rc


    def tile_weighted(self, A, B, tile_m, tile_n, Cin=None, alpha=1.0, beta=0.0, ta=False,
                      tb=False, tm=128, tn=128, bk=16, acc_bits=64, lam=DEFAULT_LAMBDA):
        """Weighted encoded checksums, thresholds and reference sums (Pw, tw,
        Rw) of one fault-free tile."""
        A, B = _f64(A), _f64(B)
        m, n, k = _dims(A, B, ta, tb)
        Cin = np.zeros((max(m, 1), max(n, 1)), order="F") if Cin is None else _f64(Cin)
        P = self._params(A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, acc_bits, True, lam,
                         weighted=True)
        w = min(tn, n - tile_n * tn)
        Pw, tw, Rw = np.empty(w), np.empty(w), np.empty(w)
        self.L.oracle_tile_weighted(C.byref(P), _dptr(A), _dptr(B), _dptr(Cin), tile_m, tile_n,
                                    _dptr(Pw), _dptr(tw), _dptr(Rw))
        return Pw, tw, Rw


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def __getattr__(name):
    # oracle.gemm(...), oracle.ftgemm(...) ... delegate to the default build.
    if name in ("gemm", "gemm_entries", "ftgemm", "tile_thresholds", "tile_checksums",
                "decode_bf16", "decode_e4m3"):
        return getattr(default(), name)
    raise AttributeError(name)
