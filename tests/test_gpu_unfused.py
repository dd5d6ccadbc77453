"""The unfused FP64 mode (abft = 3) on the GPU against the CPU oracle in its
detection-only mode (correct = False).

The unfused mode forms the same per-tile checksums and thresholds as the fused
kernel, in separate passes around the checksum-free GEMM, and only detects:
every inconsistent tile gets one record (kind UNCORRECTABLE, the output left
as computed).  Flagged (row, col, nbad_rows, nbad_cols) per tile must agree
exactly with the oracle's; the output must equal the oracle's output before
correction within 1e-12 normwise (FP64); the records' thresholds within 1e-6
relative of the oracle's (exact FP64 norms).  Accumulator faults of the
unfused mode are additions to the finished output (alpha * delta), which the
oracle's additions at step k_index equal up to rounding."""
import numpy as np
import pytest

from gpu_util import gpu_f64, normwise, say, to_oracle
from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12
T = 128
Fa = synth.Fault


def gpu_unfused(A, B, Cin, alpha, beta, ta=False, tb=False, plan=(), ldc_pad=0):
    import torch
    m = Cin.shape[0]
    dA, dB = F.to_device(A), F.to_device(B)
    dC = F.to_device(Cin, ld=m + ldc_pad if ldc_pad else None)
    F.set_fault_plan(plan)
    rb = F.ReportBuffer()
    F.gemm_ex(F.make_desc(dA, dB, dC, alpha, beta, ta, tb, abft=3), report=rb)
    torch.cuda.synchronize()
    F.clear_fault_plan()
    return np.asfortranarray(dC.cpu().numpy()), rb.view()


def _key(r):
    return (r["tile_m"], r["tile_n"], r["row"], r["col"], r["nbad_rows"], r["nbad_cols"])


def _compare(A, B, Cin, alpha, beta, ta, tb, plan, tiles=None):
    m, n = Cin.shape
    k = A.shape[0] if ta else A.shape[1]
    say("unfused case m=%d n=%d k=%d ta=%d tb=%d faults=%d" % (m, n, k, ta, tb, len(plan)))
    got, rep = gpu_unfused(A, B, Cin, alpha, beta, ta, tb, plan)
    ref = O.default().ftgemm(A, B, Cin, alpha, beta, ta, tb, T, T, 32, 64, to_oracle(plan),
                             tiles=tiles, correct=False)
    mask = ~np.isnan(ref.raw)
    assert normwise(got[mask], ref.raw[mask]) <= TOL
    recs = rep.records
    if tiles is not None:
        keep = set(int(t) for t in tiles)
        tiles_m = -(-m // T)
        recs = [r for r in recs if r["tile_m"] + r["tile_n"] * tiles_m in keep]
    assert sorted(_key(r) for r in recs) == sorted(_key(r) for r in ref.records)
    by_tile = {(r["tile_m"], r["tile_n"]): r for r in ref.records}
    for r in recs:
        o = by_tile[(r["tile_m"], r["tile_n"])]
        assert r["kind"] == F.KIND_UNCORRECTABLE
        for t, dv in (("tau_row", "d_row"), ("tau_col", "d_col")):
            assert abs(r[t] - o[t]) <= 1e-6 * o[t], (t, r, o)
            assert abs(r[dv] - o[dv]) <= 1e-6 * abs(o[dv]) + o[t] / 8, (dv, r, o)
    return got, rep, ref


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
def test_unfused_ragged(ta, tb):
    """333 x 222 x 111 (ragged in every dimension), beta != 0: a fault in the
    corner tile, two on one row of tile (1, 0), one on each encoded checksum
    of tile (0, 1)."""
    m, n, k = 333, 222, 111
    A, B, Cin = synth.operands(70, 0, m, n, k, "normal", ta, tb)
    plan = [Fa(m - 1, n - 1, k - 1, synth.ADD, 5e2),
            Fa(T + 7, 2, 0, synth.ADD, 1e3),
            Fa(T + 7, 40, k // 2, synth.ADD, -3e3),
            Fa(3, T + 4, 10, synth.ADD, 1e2, target=synth.TGT_COL_CHECKSUM),
            Fa(5, T + 6, 10, synth.ADD, -1e2, target=synth.TGT_ROW_CHECKSUM)]
    got, rep, ref = _compare(A, B, Cin, -0.7, 1.3, ta, tb, plan)
    assert rep.detected == rep.uncorrectable == 3 and rep.corrected == 0
    assert rep.tiles_verified == 3 * 2
    assert all(e["applied"] for e in rep.echoes)
    assert 0 < rep.max_ratio < 1


def test_unfused_fault_free_bits():
    """Without faults and with beta = 0 the unfused call writes the bits of
    the call without checksums, and nothing is flagged."""
    m, n, k = 1000, 700, 900
    A, B, Cin = synth.operands(71, 0, m, n, k, "uniform")
    got, rep = gpu_unfused(A, B, Cin, 2.0, 0.0)
    plain, _ = gpu_f64(A, B, Cin, 2.0, 0.0, abft=False)
    assert np.array_equal(got, plain)
    assert not rep.records and rep.tiles_verified == 8 * 6
    assert 0 < rep.max_ratio < 1


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 3, 5), (129, 127, 17), (64, 200, 1)])
def test_unfused_small_shapes(m, n, k):
    """Shapes below and just above one tile, beta != 0, with C's leading
    dimension padded: no tile flagged, the output that of the call without
    checksums, and one fault in the last tile detected."""
    A, B, Cin = synth.operands(73, m + n + k, m, n, k, "uniform")
    got, rep = gpu_unfused(A, B, Cin, 0.75, -1.5, ldc_pad=5)
    plain, _ = gpu_f64(A, B, Cin, 0.75, -1.5, abft=False, ldc_pad=5)
    assert np.array_equal(got, plain)
    assert not rep.records and rep.tiles_verified == (-(-m // T)) * (-(-n // T))
    plan = [Fa(m - 1, n - 1, k - 1, synth.ADD, 1e3)]
    got, rep, ref = _compare(A, B, Cin, 0.75, -1.5, False, False, plan)
    assert rep.detected == 1 and rep.records[0]["row"] == m - 1 and rep.records[0]["col"] == n - 1


def test_unfused_beta_zero_ignores_c():
    """beta = 0 never reads C: NaN in C does not reach the output or the
    checksums."""
    m, n, k = 300, 260, 140
    A, B, _ = synth.operands(74, 0, m, n, k, "normal", False, True)
    Cnan = np.asfortranarray(np.full((m, n), np.nan))
    got, rep, ref = _compare(A, B, Cnan, 1.25, 0.0, False, True, [])
    assert np.all(np.isfinite(got)) and not rep.records


def test_unfused_rejects_low_precision():
    import torch
    a = torch.zeros((64, 64), dtype=torch.bfloat16, device="cuda").t()
    c = torch.zeros((64, 64), dtype=torch.float32, device="cuda").t()
    with pytest.raises(F.FTGemmError):
        F.gemm_ex(F.make_desc(a, a, c, abft=3))


def test_unfused_8192_sampled_tiles():
    """m = n = k = 8192, as the benchmark times it: nothing flagged without
    faults; one +1e3 fault in each of 12 tiles, every one flagged and no
    other tile; the oracle checks the faulty tiles and sampled clean and
    corner tiles."""
    size = 8192
    A, B, Cin = synth.operands(72, size, size, size, size, "normal")
    tiles_m = size // T
    ntiles = tiles_m * tiles_m
    extra = [0, ntiles - 1, tiles_m - 1, ntiles - tiles_m] + [
        int(t) for t in synth.rng(72, 1, 9).choice(ntiles, 3, replace=False)]
    got, rep, _ = _compare(A, B, Cin, 1.0, 1.0, False, False, [], tiles=extra)
    assert rep.detected == 0 and rep.tiles_verified == ntiles
    g = synth.rng(72, size, synth.STREAM_PLAN)
    plan = synth.additive_plan(g, size, size, size, T, T, 12, lambda _g: 1e3)
    faulty = sorted({(f.row // T) + (f.col // T) * tiles_m for f in plan})
    got, rep, _ = _compare(A, B, Cin, 1.0, 1.0, False, False, plan,
                           tiles=sorted(set(faulty) | set(extra)))
    assert rep.detected == len(faulty) == len(plan)
    assert sorted(r["tile_m"] + r["tile_n"] * tiles_m for r in rep.records) == faulty
