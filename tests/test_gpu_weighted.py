"""FP64 weighted mode (abft 4) on the GPU against the oracle's weighted mode.

Each tile also keeps a weighted row checksum per column (weights i + 1 over
its local rows).  Tolerance: normwise max|C - C_oracle| / max|C_oracle| <=
1e-12 (FP64); flagged (row, col, kind) sets must agree exactly with the
oracle's."""
import numpy as np
import pytest

from gpu_util import flagged, normwise, say, to_oracle
from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12
F_ = synth.Fault
W = synth.TGT_WEIGHTED_CHECKSUM


def _gpu(A, B, Cin, alpha, beta, ta=False, tb=False, plan=(), abft=4):
    import torch
    dA, dB, dC = F.to_device(A), F.to_device(B), F.to_device(Cin)
    F.set_fault_plan(plan)
    rb = F.ReportBuffer()
    F.gemm_ex(F.make_desc(dA, dB, dC, alpha, beta, ta, tb, abft=abft), report=rb)
    torch.cuda.synchronize()
    F.clear_fault_plan()
    return np.asfortranarray(dC.cpu().numpy()), rb.view()


def _compare(A, B, Cin, alpha, beta, ta, tb, plan, tiles=None):
    m, n = Cin.shape
    k = A.shape[0] if ta else A.shape[1]
    tm, tn, bk, sk = F.query_tiling_ex(F.F64, m, n, k, abft=4)
    assert sk == 1
    say("weighted case m=%d n=%d k=%d ta=%d tb=%d faults=%d" % (m, n, k, ta, tb, len(plan)))
    got, rep = _gpu(A, B, Cin, alpha, beta, ta, tb, plan)
    ref = O.default().ftgemm(A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, 64,
                             to_oracle(plan), tiles=tiles, weighted=True)
    mask = ~np.isnan(ref.C)
    assert normwise(got[mask], ref.C[mask]) <= TOL
    recs = rep.records
    if tiles is not None:
        tiles_m = -(-m // tm)
        keep = set(int(t) for t in tiles)
        recs = [r for r in recs if r["tile_m"] + r["tile_n"] * tiles_m in keep]
    assert flagged(recs) == flagged(ref.records)
    return got, rep, ref


def test_patterns_against_oracle():
    """One pattern per 128 x 128 tile of a 512 x 300 x 200 product (ragged
    last tile column): two equal errors in distinct rows and columns and
    four equal ones (located by the ratio of weighted to plain residual,
    corrected), the corners of a rectangle and a row whose two errors cancel
    beside a row with two (recomputed), three errors along a column and two
    along a row (corrected and confirmed), a fault on a weighted checksum
    alone (nothing flagged, echo applied), a data error plus a fault on its
    column's weighted checksum (recomputed), an infinite error (rebuilt), a
    single error, and a fault on a plain checksum (checksum-only)."""
    m, n, k = 512, 300, 200
    A, B, Cin = synth.operands(31, 0, m, n, k, "uniform")
    plan = [F_(17, 90, 10, synth.ADD, 30.0), F_(60, 3, 150, synth.ADD, 30.0),        # (0, 0)
            F_(140, 250, 5, synth.ADD, 25.0), F_(150, 130, 60, synth.ADD, 25.0),     # (1, 1)
            F_(200, 200, 199, synth.ADD, 25.0), F_(255, 155, 99, synth.ADD, 25.0),
            F_(260, 270, 3, synth.ADD, 25.0), F_(260, 290, 30, synth.ADD, 40.0),     # (2, 2)
            F_(300, 270, 50, synth.ADD, 40.0),
            F_(2, 130, 1, synth.ADD, 10.0), F_(5, 130, 1, synth.ADD, 6.0),          # (0, 1)
            F_(5, 140, 1, synth.ADD, -6.0), F_(2, 140, 4, synth.ADD, 7.0),
            F_(130, 9, 5, synth.ADD, 50.0), F_(137, 9, 9, synth.ADD, 60.0),        # (1, 0)
            F_(144, 9, 20, synth.ADD, -70.0),
            F_(270, 2, 3, synth.ADD, 100.0), F_(270, 11, 17, synth.ADD, -40.0),    # (2, 0)
            F_(4, 260, 0, synth.ADD, 500.0, target=W),                             # (0, 2)
            F_(140, 280, 3, synth.ADD, 30.0), F_(128, 280, 0, synth.ADD, 90.0, target=W),  # (1, 2)
            F_(400, 10, 4, synth.ADD, np.inf),                                     # (3, 0)
            F_(450, 200, 77, synth.ADD, 20.0),                                     # (3, 1)
            F_(390, 290, 0, synth.ADD, 9.0, target=synth.TGT_ROW_CHECKSUM)]        # (3, 2)
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, False, False, plan)
    kinds = {(r["tile_m"], r["tile_n"]): r["kind"] for r in rep.records}
    assert kinds == {(0, 0): F.KIND_CORRECTED, (1, 1): F.KIND_CORRECTED,
                     (2, 2): F.KIND_RECOMPUTED, (0, 1): F.KIND_RECOMPUTED,
                     (1, 0): F.KIND_CORRECTED, (2, 0): F.KIND_CORRECTED,
                     (1, 2): F.KIND_RECOMPUTED, (3, 0): F.KIND_CORRECTED,
                     (3, 1): F.KIND_CORRECTED, (3, 2): F.KIND_CHECKSUM_ONLY}
    named = {(r["tile_m"], r["tile_n"]): (r["row"], r["col"], r["nbad_rows"], r["nbad_cols"])
             for r in rep.records if r["kind"] == F.KIND_CORRECTED}
    assert named[(0, 0)] == (17, 90, 2, 2) and named[(1, 1)] == (140, 250, 4, 4)
    assert named[(1, 0)] == (130, 9, 3, 1) and named[(2, 0)] == (270, 2, 1, 2)
    by_tile = {(r["tile_m"], r["tile_n"]): r for r in ref.records}
    for r in rep.records:
        if r["kind"] == F.KIND_CORRECTED and np.isfinite(r["before"]):
            o = by_tile[(r["tile_m"], r["tile_n"])]
            assert abs(r["before"] - o["before"]) <= 1e-12 * abs(o["before"])
            assert abs(r["after"] - o["after"]) <= 1e-12 * max(1.0, abs(o["after"]))
    echo = {(e["row"], e["col"]): e for e in rep.echoes}
    assert echo[(4, 260)]["applied"]
    assert abs(echo[(4, 260)]["after"] - echo[(4, 260)]["before"] - 500.0) < 1e-9
    assert np.all(np.isfinite(got))
    # the plain mode cannot pair the equal errors of tile (0, 0)
    _, rep1 = _gpu(A, B, Cin, 1.0, 0.5, plan=plan[:2], abft=1)
    assert [r["kind"] for r in rep1.records] == [F.KIND_RECOMPUTED]


@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
def test_transposes(ta, tb):
    """Equal errors paired by the weighted checksums under every transpose
    (the weighted sums of A are formed from its staged values in either
    layout); ragged 300 x 257 x 77."""
    m, n, k = 300, 257, 77
    A, B, Cin = synth.operands(32, 0, m, n, k, "normal")
    if ta:
        A = np.asfortranarray(A.T)
    if tb:
        B = np.asfortranarray(B.T)
    plan = [F_(3, 5, 10, synth.ADD, 15.0), F_(100, 70, 60, synth.ADD, 15.0),
            F_(299, 256, 76, synth.ADD, -8.0), F_(260, 140, 0, synth.ADD, 12.0),
            F_(270, 150, 40, synth.ADD, 12.0), F_(290, 141, 20, synth.ADD, 12.0)]
    got, rep, ref = _compare(A, B, Cin, -0.7, 1.3, ta, tb, plan)
    assert rep.corrected == 3 and not rep.recomputed


def test_fault_free_output_equals_mode_1():
    """Without faults the weighted mode stores the same C as mode 1, bit for
    bit (the same products in the same order), and flags nothing."""
    A, B, Cin = synth.operands(33, 0, 1000, 777, 555, "normal")
    g4, r4 = _gpu(A, B, Cin, 1.25, -0.5)
    g1, r1 = _gpu(A, B, Cin, 1.25, -0.5, abft=1)
    assert np.array_equal(g4, g1) and not r4.records and not r1.records
    assert r4.tiles_verified == r1.tiles_verified == 8 * 7


def test_sampled_tiles_4096():
    """4096^3, uniform operands: pairs of equal errors of size 10^U(0,2)
    times the typical |C| in sampled tiles, each corrected; the oracle checks
    those tiles plus corners.  (Much larger pairs round their own reference
    sums by more than the fault-free threshold, and the tile is computed
    again on either side.)"""
    size = 4096
    A, B, Cin = synth.operands(20, size, size, size, size, "uniform")
    sigma = np.sqrt(size / 9.0 + 1.0 / 3.0)
    tiles_m = size // 128
    g = synth.rng(34, size, synth.STREAM_PLAN)
    picks = g.choice(tiles_m * tiles_m, 12, replace=False)
    plan = []
    for t in picks:
        ti, tj = int(t) % tiles_m, int(t) // tiles_m
        r = g.choice(128, 2, replace=False)
        c = g.choice(128, 2, replace=False)
        d = sigma * 10.0 ** g.uniform(0.0, 2.0)
        for q in range(2):
            plan.append(F_(ti * 128 + int(r[q]), tj * 128 + int(c[q]),
                           int(g.integers(0, size)), synth.ADD, d))
    tiles = sorted(set(int(t) for t in picks) | {0, tiles_m * tiles_m - 1})
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, False, False, plan, tiles=tiles)
    assert rep.corrected == 12 == rep.detected
    assert rep.tiles_verified == tiles_m * tiles_m


def test_refused_where_unsupported():
    """Batches and the entry point that allocates nothing refuse the
    weighted mode, leaving C as it was."""
    import torch
    A, B, Cin = synth.operands(35, 0, 64, 64, 64, "normal")
    dA, dB, dC = F.to_device(A), F.to_device(B), F.to_device(Cin)
    d = F.make_desc(dA, dB, dC, 1.0, 0.0, abft=4)
    L = F.lib()
    import ctypes as C
    assert L.ftgemm_gemm_ex_noalloc(C.byref(d), None, None) == F.ERR_UNSUPPORTED
    assert L.ftgemm_gemm_batched(1, C.byref(d), None, None) == F.ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), Cin)
