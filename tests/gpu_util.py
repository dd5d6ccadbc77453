"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs, and compare."""
import sys

import numpy as np

from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_oracle(plan):
    return [O.Injection(f.row, f.col, f.k_index, f.mode, f.delta, f.bit, f.target)
            for f in plan]


def gpu_f64(A, B, Cin, alpha, beta, ta=False, tb=False, plan=(), abft=True, ldc_pad=0):
    import torch
    dA, dB = F.to_device(A), F.to_device(B)
    m, n = Cin.shape
    dC = F.to_device(Cin, ld=m + ldc_pad if ldc_pad else None)
    F.set_fault_plan(plan)
    rb = F.ReportBuffer()
    if abft:
        F.gemm(dA, dB, dC, alpha, beta, ta, tb, report=rb)
    else:
        F.gemm_ex(F.make_desc(dA, dB, dC, alpha, beta, ta, tb, abft=False))
    torch.cuda.synchronize()
    F.clear_fault_plan()
    out = np.asfortranarray(dC.cpu().numpy())
    return out, rb.view()


def normwise(got, ref):
    den = np.max(np.abs(ref)) if ref.size else 1.0
    return float(np.max(np.abs(got - ref)) / (den if den > 0 else 1.0)) if ref.size else 0.0


def flagged(records):
    return sorted((r["row"], r["col"], r["kind"]) for r in records)


def f64_tiling(m, n, k):
    tm, tn, bk, sk = F.query_tiling(F.F64, m, n, k)
    return tm, tn, bk
