"""The entry point that allocates nothing (ftgemm_gemm_ex_noalloc), through
the C ABI, against ftgemm_gemm_ex on the same inputs: two calls in a row,
the second on a smaller problem, for FP64 and BF16 / FP8, with faults
planned.  The output must match ftgemm_gemm_ex's (FP64: bit for bit; low
precision: bit for bit outside rebuilt elements, and within the format's
normwise tolerance everywhere), and the flagged (row, col, kind) records and
the fault echoes must be the same.  The library keeps the last call's
report area in its fixed array, so the second call's counters show that it
was cleared.  (Fault-tolerant FP8 tiles have 128 rows in the entry point
that allocates nothing, so its count of verified tiles differs there.)"""
import ctypes

import numpy as np
import pytest

from gpu_util import codes_to_device, flagged, lp_inputs, normwise, say
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = {F.F64: 1e-12, F.BF16: 1e-5, F.FP8_E4M3: 1e-4}


def _run_both(dtype, m, n, k, plan, seed, ta=False, tb=False):
    import torch
    A, B, Cin = synth.operands(80, seed, m, n, k, "normal", ta, tb)
    if dtype == F.F64:
        dA, dB, sa, sb = F.to_device(A), F.to_device(B), 1.0, 1.0
        C0 = F.to_device(Cin)
    else:
        ca, cb, sa, sb, _, _ = lp_inputs(A, B, dtype)
        dA, dB = codes_to_device(ca, dtype), codes_to_device(cb, dtype)
        C0 = F.to_device(np.asfortranarray(Cin, dtype=np.float32))
    outs, reps = [], []
    for noalloc in (False, True):
        dC = C0.clone()
        d = F.make_desc(dA, dB, dC, 1.25, -0.5, ta, tb, scaleA=sa, scaleB=sb, dtype=dtype)
        F.set_fault_plan(plan)
        rb = F.ReportBuffer()
        say("case dtype=%d m=%d n=%d k=%d faults=%d noalloc=%d" % (dtype, m, n, k, len(plan),
                                                                    noalloc))
        (F.gemm_ex_noalloc if noalloc else F.gemm_ex)(d, report=rb)
        torch.cuda.synchronize()
        F.clear_fault_plan()
        outs.append(np.asfortranarray(dC.cpu().numpy().astype(np.float64)))
        reps.append(rb.view())
    return outs, reps


def _tiles(m, n, rows):
    return -(-m // rows) * -(-n // 128)


def _check(dtype, outs, reps, nfaults):
    got, want = outs[1], outs[0]
    m, n = got.shape
    rn, re = reps[1], reps[0]
    assert flagged(rn.records) == flagged(re.records)
    assert (rn.detected, rn.corrected, rn.recomputed, rn.checksum_only) == \
        (re.detected, re.corrected, re.recomputed, re.checksum_only)
    rows = F.query_tiling(dtype, m, n, 1)[0]
    assert re.tiles_verified == _tiles(m, n, rows)
    assert rn.tiles_verified == _tiles(m, n, 128 if dtype == F.FP8_E4M3 else rows)
    assert [(e["row"], e["col"], e["applied"], e["before"], e["after"]) for e in rn.echoes] == \
        [(e["row"], e["col"], e["applied"], e["before"], e["after"]) for e in re.echoes]
    assert rn.detected == nfaults and re.corrected == nfaults
    if dtype == F.F64:
        assert np.array_equal(got, want)
        return
    rebuilt = np.zeros(got.shape, dtype=bool)
    for r in re.records:
        if r["kind"] == F.KIND_CORRECTED:
            rebuilt[r["row"], r["col"]] = True
    assert np.array_equal(got[~rebuilt], want[~rebuilt])
    assert normwise(got, want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [pytest.param(F.F64, id="f64"), pytest.param(F.BF16, id="bf16"),
                                   pytest.param(F.FP8_E4M3, id="fp8")])
def test_noalloc_matches_gemm_ex_twice(dtype):
    Fa = synth.Fault
    # first call: large enough that ftgemm_gemm_ex takes its low-precision
    # norms pass (256 tiles of 256 x 128), A transposed; faults far above
    # the thresholds, one per tile
    m, n, k = (1024, 768, 512) if dtype == F.F64 else (4096, 2048, 256)
    big = 1e4 if dtype == F.F64 else 1e5
    plan = [Fa(5, 7, 3, synth.ADD, big), Fa(700, 600, k - 1, synth.ADD, -big),
            Fa(m - 1, n - 1, k // 2, synth.ADD, big)]
    if dtype == F.FP8_E4M3:
        plan = [Fa(f.row, f.col, f.k_index, f.mode, f.delta * 64.0 * 64.0) for f in plan]
    outs, reps = _run_both(dtype, m, n, k, plan, 1, ta=True)
    _check(dtype, outs, reps, len(plan))
    # second call: smaller, other faults; the fixed report area is cleared
    m2, n2, k2 = 300, 200, 100
    plan2 = [Fa(150, 10, 50, synth.ADD, big if dtype != F.FP8_E4M3 else big * 4096.0)]
    outs, reps = _run_both(dtype, m2, n2, k2, plan2, 2, tb=True)
    _check(dtype, outs, reps, len(plan2))


def test_noalloc_limits():
    """A fault plan beyond the 256 slots, and the modes whose workspace grows
    with the problem, are refused before anything runs."""
    import torch
    A = F.to_device(np.ones((64, 64), order="F"))
    B = F.to_device(np.ones((64, 64), order="F"))
    Cm = F.to_device(np.zeros((64, 64), order="F"))
    d = F.make_desc(A, B, Cm, 1.0, 0.0)
    F.set_fault_plan([synth.Fault(i % 64, i // 64, 0, synth.ADD, 1.0) for i in range(257)])
    assert F.lib().ftgemm_gemm_ex_noalloc(ctypes.byref(d), None, None) == F.ERR_UNSUPPORTED
    F.clear_fault_plan()
    assert F.lib().ftgemm_gemm_ex_noalloc(None, None, None) == F.ERR_INVALID_ARG
    F.gemm_ex_noalloc(d)
    torch.cuda.synchronize()
    assert np.array_equal(Cm.cpu().numpy(), np.full((64, 64), 64.0))
