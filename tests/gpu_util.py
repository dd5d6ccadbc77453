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


# -- low precision (BF16, FP8 E4M3) ---------------------------------------------

def lp_inputs(A, B, dtype):
    """Quantise float64 operands to the input format: (codes_A, codes_B,
    scale_A, scale_B, decoded_A, decoded_B).  The decoded values come from
    the oracle's own decoders, so the oracle sees exactly the GPU's inputs."""
    orc = O.default()
    if dtype == F.BF16:
        ca, cb = synth.to_bf16_bits(A), synth.to_bf16_bits(B)
        return ca, cb, 1.0, 1.0, _fortran(orc.decode_bf16(ca), A), _fortran(orc.decode_bf16(cb), B)
    sa, sb = synth.e4m3_scale(A), synth.e4m3_scale(B)
    ca, cb = synth.to_e4m3_bits(A, sa), synth.to_e4m3_bits(B, sb)
    return ca, cb, sa, sb, _fortran(orc.decode_e4m3(ca), A), _fortran(orc.decode_e4m3(cb), B)


def _fortran(dec, like):
    assert dec.shape == like.shape
    return np.asfortranarray(dec)


def codes_to_device(codes, dtype):
    import torch
    if dtype == F.BF16:
        t = F.to_device(codes.view(np.int16))
        return t.view(torch.bfloat16)
    return F.to_device(codes.view(np.uint8))


def gpu_lp(codes_a, codes_b, Cin, alpha, beta, dtype, ta=False, tb=False, plan=(), abft=True,
           scale_a=1.0, scale_b=1.0, ldc_pad=0):
    """Run the BF16 / FP8 fault-tolerant GEMM; Cin is float32-representable."""
    import torch
    dA, dB = codes_to_device(codes_a, dtype), codes_to_device(codes_b, dtype)
    m, n = Cin.shape
    dC = F.to_device(np.asfortranarray(Cin, dtype=np.float32),
                     ld=m + ldc_pad if ldc_pad else None)
    F.set_fault_plan(plan)
    rb = F.ReportBuffer()
    d = F.make_desc(dA, dB, dC, alpha, beta, ta, tb, abft=abft, scaleA=scale_a, scaleB=scale_b,
                    dtype=dtype)
    F.gemm_ex(d, report=rb)
    torch.cuda.synchronize()
    F.clear_fault_plan()
    out = np.asfortranarray(dC.cpu().numpy().astype(np.float64))
    return out, rb.view()


# The FP8 matrix instructions cut each product to 2^-14 of its group's
# largest product binade, in groups of 8 inner indices; the oracle's
# thresholds take that as (grid, group).  BF16 products are added exactly.
FP8_MMA = (2.0 ** -14, 8)


def lp_mma(dtype):
    return FP8_MMA if dtype == F.FP8_E4M3 else (0.0, 1)


def lp_tiling(dtype, m, n, k):
    tm, tn, bk, sk = F.query_tiling(dtype, m, n, k)
    return tm, tn, bk


# -- rounding bound of a rebuilt element -------------------------------------

U32 = 2.0 ** -24
LAMBDA = 8.0


def _enc_error(chk, vec, parts):
    """lambda-sigma model of the FP32 rounding of one encoded checksum
    sum_p chk_p vec_p accumulated in order of p: the partial sums' roundings
    (u sqrt(sum_k S_k^2)), the products' roundings, and the roundings inside
    each chk_p, an FP32 sum whose partial sums are parts[:, p]."""
    prod = chk * vec
    S = np.cumsum(prod)
    e_acc = np.sqrt(np.sum(S * S))
    e_prod = np.sqrt(np.sum(prod * prod))
    X = np.sqrt(np.sum(parts * parts, axis=0))
    e_chk = np.sqrt(np.sum((X * vec) ** 2))
    return LAMBDA * U32 * (e_acc + e_prod + e_chk)


def rebuild_bound(dA, dB, ta, tb, alpha, tm, tn, got, exact, i, j):
    """How far an element rebuilt from its tile's FP32 checksums may lie from
    the exact product.  Rebuilt from column j's checksum it is
    P_j - sum_{i' != i} out(i', j): its error is the encoded checksum's own
    rounding error plus the other outputs' errors in the column, which the
    test measures exactly (got - exact); from row i's checksum likewise.
    The checksum's rounding is modelled from the actual partial sums (a
    lambda = 8 standard-deviation bound, about sqrt(k) tighter than the
    detection threshold's norm bound), and the rebuilt value's own FP32
    rounding is added.  The larger of the two sides is returned."""
    oA = dA.T if ta else dA
    oB = dB.T if tb else dB
    i0, j0 = (i // tm) * tm, (j // tn) * tn
    I = slice(i0, min(i0 + tm, oA.shape[0]))
    J = slice(j0, min(j0 + tn, oB.shape[1]))
    # from the column: x = e^T A_I, encoded sum_p x_p B(p, j)
    part_x = np.cumsum(oA[I, :], axis=0)
    e_col = abs(alpha) * _enc_error(part_x[-1], oB[:, j], part_x)
    other_c = np.sum(got[I, j] - exact[I, j]) - (got[i, j] - exact[i, j])
    # from the row: y = B_J e, encoded sum_p A(i, p) y_p
    part_y = np.cumsum(oB[:, J], axis=1).T
    e_row = abs(alpha) * _enc_error(part_y[-1], oA[i, :], part_y)
    other_r = np.sum(got[i, J] - exact[i, J]) - (got[i, j] - exact[i, j])
    own = 2.0 * U32 * abs(exact[i, j])
    return max(abs(other_c) + e_col, abs(other_r) + e_row) + own
