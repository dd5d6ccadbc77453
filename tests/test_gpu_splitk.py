"""FP64 fault-tolerant GEMM with a split inner dimension, against the CPU
oracle: the small-output shapes (few output tiles, long inner dimension)
where each slice verifies its own partial product and a verified reduction
forms C = alpha * sum_s W_s + beta * C_in.

Tolerance as for the unsplit FP64 path: normwise 1e-12.  The oracle is run
with the same slices (each ceil(steps / S) steps of bk long, the last one
shorter), so the flagged (row, col, kind) records -- one per slice that
found something, one for a reduction that did not verify -- agree exactly
with the oracle's.  The number of verifications is S per tile for the
slices plus one per tile for the reduction."""
import numpy as np
import pytest

from gpu_util import flagged, gpu_f64, normwise, say, to_oracle
from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _tiling(m, n, k):
    return F.query_tiling(F.F64, m, n, k)


def _slice_k(k, bk, s):
    """Inner length of each slice when the call is split s ways."""
    if s <= 1:
        return 0
    steps = -(-k // bk)
    return -(-steps // s) * bk


def _run(A, B, Cin, alpha, beta, plan, ta=False, tb=False, tiles=None, abft=True):
    m, n = Cin.shape
    k = A.shape[0] if ta else A.shape[1]
    tm, tn, bk, s = _tiling(m, n, k)
    say("case m=%d n=%d k=%d slices=%d faults=%d" % (m, n, k, s, len(plan)))
    got, rep = gpu_f64(A, B, Cin, alpha, beta, ta, tb, plan, abft=abft)
    ref = O.default().ftgemm(A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, 64, to_oracle(plan),
                             tiles=tiles, slice_k=_slice_k(k, bk, s))
    mask = ~np.isnan(ref.C)
    err = normwise(got[mask], ref.C[mask])
    assert err <= TOL, err
    recs = rep.records
    if tiles is not None:
        tiles_m = -(-m // tm)
        keep = set(int(t) for t in tiles)
        recs = [r for r in recs if r["tile_m"] + r["tile_n"] * tiles_m in keep]
    return got, rep, ref, recs, s


def _plan(g, m, n, k, count, sigma):
    return synth.additive_plan(g, m, n, k, 128, 128, count, synth.log_magnitude(sigma))


def test_split_choice_for_small_outputs():
    assert _tiling(16384, 16384, 256)[3] == 1
    assert _tiling(1024, 1024, 32768)[3] == 8
    assert _tiling(16384, 64, 16384)[3] == 4
    assert _tiling(4096, 4096, 4096)[3] == 1
    assert _tiling(64, 64, 64)[3] == 1          # too short to split


@pytest.mark.parametrize("m,n,k", [(1024, 1024, 32768), (16384, 64, 16384)])
def test_c3_split_shapes(m, n, k):
    """Normal inputs, alpha = beta = 1, one fault per 32 tiles (at least one)
    of size 10^U(0,6) * sqrt(k + 1); every fault rebuilt; full compare."""
    A, B, Cin = synth.operands(50, k, m, n, k, "normal")
    tiles = (-(-m // 128)) * (-(-n // 128))
    g = synth.rng(50, k, synth.STREAM_PLAN)
    plan = _plan(g, m, n, k, max(1, tiles // 32), np.sqrt(k + 1.0))
    got, rep, ref, recs, s = _run(A, B, Cin, 1.0, 1.0, plan)
    assert s > 1
    assert flagged(recs) == flagged(ref.records)
    assert rep.corrected == len(plan) == rep.detected
    assert rep.tiles_verified == tiles * (s + 1)
    # error-free: nothing flagged by the slices or the reduction
    got, rep, ref, recs, s = _run(A, B, Cin, 1.0, 1.0, [])
    assert not rep.records and 0 < rep.max_ratio < 1


def test_c3_long_short_shape_sampled():
    """(16384, 16384, 256): enough tiles, no split; sampled tiles."""
    m = n = 16384
    k = 256
    A, B, Cin = synth.operands(50, k, m, n, k, "normal")
    tiles_m = m // 128
    g = synth.rng(50, k, synth.STREAM_PLAN)
    plan = _plan(g, m, n, k, tiles_m * tiles_m // 32, np.sqrt(k + 1.0))
    faulty = sorted({(f.row // 128) + (f.col // 128) * tiles_m for f in plan})
    tiles = sorted(set(faulty[:24]) | {0, tiles_m * tiles_m - 1})
    got, rep, ref, recs, s = _run(A, B, Cin, 1.0, 1.0, plan, tiles=tiles)
    assert s == 1
    assert flagged(recs) == flagged(ref.records)
    assert rep.corrected == len(plan) == rep.detected


@pytest.mark.parametrize("ta,tb", [(False, False), (True, True)])
def test_split_ragged_and_checksum_faults(ta, tb):
    """Ragged edges and a short last slice; accumulator faults in several
    slices, a fault on an encoded checksum, and one on a checksum whose
    inner index lies past the end (taken by the last slice)."""
    m, n, k = 300, 200, 5000
    A, B, Cin = synth.operands(51, 0, m, n, k, "normal", ta, tb)
    tm, tn, bk, s = _tiling(m, n, k)
    assert s > 1
    Fa = synth.Fault
    plan = [Fa(5, 7, 10, synth.ADD, 300.0),            # tile (0,0), first slice
            Fa(130, 20, 4990, synth.ADD, -250.0),      # tile (1,0), last slice
            Fa(260, 150, 2500, synth.ADD, 1e4),        # tile (2,1), a middle slice
            Fa(20, 140, 1234, synth.ADD, 50.0, target=synth.TGT_ROW_CHECKSUM),   # tile (0,1)
            Fa(140, 190, 99999, synth.ADD, 70.0, target=synth.TGT_COL_CHECKSUM)]  # tile (1,1)
    got, rep, ref, recs, s = _run(A, B, Cin, 0.75, -1.25, plan, ta, tb)
    assert flagged(recs) == flagged(ref.records)
    assert sorted(r["kind"] for r in recs) == sorted([F.KIND_CORRECTED] * 3 +
                                                     [F.KIND_CHECKSUM_ONLY] * 2)
    for e in rep.echoes:
        assert e["applied"]


def test_split_two_faults_one_tile():
    """Two faults of one tile in the same slice: that slice pairs them by
    their residuals and corrects both (two equal faults cannot be paired:
    it recomputes); in different slices: each slice rebuilds its own, one
    record per slice, as the oracle run with the same slices does."""
    m, n, k = 256, 128, 8192
    A, B, Cin = synth.operands(52, 0, m, n, k, "uniform")
    tm, tn, bk, s = _tiling(m, n, k)
    assert s > 1
    Fa = synth.Fault
    same = [Fa(3, 4, 10, synth.ADD, 100.0), Fa(50, 60, 20, synth.ADD, 200.0)]
    got, rep, ref, recs, _ = _run(A, B, Cin, 1.0, 1.0, same)
    assert [(r["row"], r["col"], r["kind"], r["nbad_rows"]) for r in recs] == \
        [(3, 4, F.KIND_CORRECTED, 2)]
    assert flagged(recs) == flagged(ref.records)
    equal = [Fa(3, 4, 10, synth.ADD, 100.0), Fa(50, 60, 20, synth.ADD, 100.0)]
    got, rep, ref, recs, _ = _run(A, B, Cin, 1.0, 1.0, equal)
    assert [r["kind"] for r in recs] == [F.KIND_RECOMPUTED]
    assert flagged(recs) == flagged(ref.records)
    apart = [Fa(3, 4, 10, synth.ADD, 100.0), Fa(50, 60, k - 5, synth.ADD, 200.0)]
    got, rep, ref, recs, _ = _run(A, B, Cin, 1.0, 1.0, apart)
    assert sorted((r["row"], r["col"], r["kind"]) for r in recs) == \
        [(3, 4, F.KIND_CORRECTED), (50, 60, F.KIND_CORRECTED)]
    assert flagged(recs) == flagged(ref.records)
    assert [r["nbad_rows"] for r in ref.records] == [1, 1]


def test_split_plain_kernel():
    A, B, Cin = synth.operands(53, 0, 200, 300, 7000, "normal")
    got, rep = gpu_f64(A, B, Cin, 1.5, 0.5, abft=False)
    assert _tiling(200, 300, 7000)[3] > 1
    assert normwise(got, O.default().gemm(A, B, Cin, 1.5, 0.5)) <= TOL
