"""FP64 fault-tolerant GEMM on the GPU against the CPU oracle.

Tolerance: normwise max|C - C_oracle| / max|C_oracle| <= 1e-12 (FP64).
Flagged (row, col, kind) sets must agree exactly with the oracle's and with
the accepted fault plan."""
import numpy as np
import pytest

from gpu_util import f64_tiling, flagged, gpu_f64, normwise, say, to_oracle
from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _plan_acc(g, m, n, k, tm, tn, count, delta):
    return synth.additive_plan(g, m, n, k, tm, tn, count,
                               delta if callable(delta) else (lambda _g: delta))


def _compare(A, B, Cin, alpha, beta, ta, tb, plan, tiles=None):
    m, n = Cin.shape
    k = A.shape[0] if ta else A.shape[1]
    tm, tn, bk = f64_tiling(m, n, k)
    say("case m=%d n=%d k=%d ta=%d tb=%d faults=%d" % (m, n, k, ta, tb, len(plan)))
    got, rep = gpu_f64(A, B, Cin, alpha, beta, ta, tb, plan)
    ref = O.default().ftgemm(A, B, Cin, alpha, beta, ta, tb, tm, tn, bk, 64,
                             to_oracle(plan), tiles=tiles)
    if tiles is None:
        err = normwise(got, ref.C)
    else:
        mask = ~np.isnan(ref.C)
        err = normwise(got[mask], ref.C[mask])
    assert err <= TOL, err
    recs = rep.records
    if tiles is not None:
        tiles_m = -(-m // tm)
        keep = set(int(t) for t in tiles)
        recs = [r for r in recs if r["tile_m"] + r["tile_n"] * tiles_m in keep]
    assert flagged(recs) == flagged(ref.records)
    return got, rep, ref


def test_c1_256_four_additive_errors():
    """256^3, alpha 1, beta 0.5, U[-1,1] from seed 0; four +1e3 faults on
    accumulators in four distinct tiles, all located and corrected."""
    A, B, Cin = synth.operands(1, 0, 256, 256, 256, "uniform")
    g = synth.rng(1, 0, synth.STREAM_PLAN)
    plan = _plan_acc(g, 256, 256, 256, 128, 128, 4, 1e3)
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, False, False, plan)
    assert sorted((f.row, f.col) for f in plan) == sorted((r[0], r[1]) for r in flagged(rep.records))
    assert rep.corrected == 4 and rep.detected == 4 and rep.tiles_verified == 4
    assert all(r["kind"] == F.KIND_CORRECTED for r in rep.records)
    for e, f in zip(rep.echoes, plan):
        assert e["applied"] and (e["row"], e["col"]) == (f.row, f.col)
        assert abs((e["after"] - e["before"]) - 1e3) < 1e-9
    assert 0 < rep.max_ratio < 1


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
def test_ragged_transposes(ta, tb):
    m, n, k = 300, 260, 77
    A, B, Cin = synth.operands(2, 1, m, n, k, "normal", ta, tb)
    g = synth.rng(2, 1, synth.STREAM_PLAN)
    plan = _plan_acc(g, m, n, k, 128, 128, 5, synth.log_magnitude(3.0))
    got, rep, ref = _compare(A, B, Cin, -0.7, 1.3, ta, tb, plan)
    assert rep.corrected == 5


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 3, 5), (128, 128, 16), (129, 127, 17),
                                   (64, 200, 1), (200, 64, 300)])
def test_small_and_edge_shapes(m, n, k):
    A, B, Cin = synth.operands(3, m * 1000 + n, m, n, k, "uniform")
    _compare(A, B, Cin, 1.0, 1.0, False, False, [])


def test_special_cases():
    A, B, Cin = synth.operands(4, 0, 70, 50, 40, "uniform")
    # alpha == 0: C <- beta C
    got, rep = gpu_f64(A, B, Cin, 0.0, 0.5)
    assert np.array_equal(got, 0.5 * Cin)
    # beta == 0: C_in never read, NaNs do not propagate
    nanC = np.full_like(Cin, np.nan)
    got, rep = gpu_f64(A, B, nanC, 1.0, 0.0)
    ref = O.default().gemm(A, B, None, 1.0, 0.0)
    assert normwise(got, ref) <= TOL and not rep.records
    # k == 0: C <- beta C
    A0 = np.zeros((70, 0), order="F")
    B0 = np.zeros((0, 50), order="F")
    got, rep = gpu_f64(A0, B0, Cin, 1.0, 2.0)
    assert np.array_equal(got, 2.0 * Cin)
    # beta == 1 and alpha == 0: untouched
    got, rep = gpu_f64(A, B, Cin, 0.0, 1.0)
    assert np.array_equal(got, Cin)


def test_padded_leading_dimension_of_c():
    A, B, Cin = synth.operands(5, 0, 130, 140, 33, "uniform")
    got, rep = gpu_f64(A, B, Cin, 1.0, 1.0, ldc_pad=7)
    ref = O.default().gemm(A, B, Cin, 1.0, 1.0)
    assert normwise(got, ref) <= TOL


def test_line_corrections():
    """Errors confined to one row or one column of a tile: two and four in
    a row, three in a column -- each loses its crossing entry's residual
    and the line is confirmed by its own; C within 1e-12 of the oracle's.
    A line holding a non-finite value (an FP64 exponent flip) cannot be
    corrected by residuals: that tile is computed again."""
    m, n, k = 384, 300, 200
    A, B, Cin = synth.operands(7, 0, m, n, k, "uniform")
    bk = f64_tiling(m, n, k)[2]
    F_ = synth.Fault
    part = A[:, :bk] @ B[:bk, :]
    cand = [(int(i), int(j)) for i, j in np.argwhere((np.abs(part) >= 1) & (np.abs(part) < 2))
            if 256 <= i < 384 and j == 40 and i != 300]
    assert cand
    plan = [F_(17, 3, 10, synth.ADD, 30.0), F_(17, 90, 150, synth.ADD, -40.0),      # (0, 0)
            F_(140, 130, 5, synth.ADD, 2.0), F_(140, 150, 60, synth.ADD, 5.0),      # (1, 1)
            F_(140, 200, 199, synth.ADD, -3.0), F_(140, 255, 99, synth.ADD, 6.0),
            F_(260, 280, 0, synth.ADD, 20.0), F_(300, 280, 70, synth.ADD, 8.0),     # (2, 2)
            F_(383, 280, 199, synth.ADD, -5.0),
            F_(300, 40, 70, synth.ADD, 8.0),                                        # (2, 0)
            F_(cand[0][0], 40, 3, synth.BITFLIP, 0.0, 62)]
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, False, False, plan)
    kinds = {(r["tile_m"], r["tile_n"]): r["kind"] for r in rep.records}
    assert kinds == {(0, 0): F.KIND_CORRECTED, (1, 1): F.KIND_CORRECTED,
                     (2, 2): F.KIND_CORRECTED, (2, 0): F.KIND_RECOMPUTED}
    assert np.all(np.isfinite(got))


def test_crossing_pairs():
    """Errors in distinct rows and columns of a tile: two, four and three
    per tile, each flagged row paired with the column of equal residual and
    corrected; two equal errors, and three on the corners of a rectangle,
    cannot be paired -> recomputed.  C within 1e-12 of the oracle's; the
    record names the first flagged row and its paired column, with the
    oracle's values before and after."""
    m, n, k = 384, 300, 200
    A, B, Cin = synth.operands(8, 0, m, n, k, "uniform")
    F_ = synth.Fault
    plan = [F_(17, 90, 10, synth.ADD, 30.0), F_(60, 3, 150, synth.ADD, -40.0),      # (0, 0)
            F_(140, 250, 5, synth.ADD, 2.0), F_(150, 130, 60, synth.ADD, 5.0),      # (1, 1)
            F_(200, 200, 199, synth.ADD, -3.0), F_(255, 155, 99, synth.ADD, 6.0),
            F_(260, 280, 0, synth.ADD, 20.0), F_(300, 260, 70, synth.ADD, 8.0),     # (2, 2)
            F_(383, 299, 199, synth.ADD, -5.0),
            F_(10, 260, 3, synth.ADD, 7.0), F_(20, 270, 30, synth.ADD, 7.0),        # (0, 2)
            F_(270, 10, 3, synth.ADD, 4.0), F_(270, 20, 30, synth.ADD, 9.0),        # (2, 0)
            F_(280, 10, 50, synth.ADD, 11.0)]
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, False, False, plan)
    kinds = {(r["tile_m"], r["tile_n"]): r["kind"] for r in rep.records}
    assert kinds == {(0, 0): F.KIND_CORRECTED, (1, 1): F.KIND_CORRECTED,
                     (2, 2): F.KIND_CORRECTED, (0, 2): F.KIND_RECOMPUTED,
                     (2, 0): F.KIND_RECOMPUTED}
    named = sorted((r["row"], r["col"], r["nbad_rows"]) for r in rep.records
                   if r["kind"] == F.KIND_CORRECTED)
    assert named == [(17, 90, 2), (140, 250, 4), (260, 280, 3)]
    by_row = {r["row"]: r for r in ref.records}
    for r in rep.records:
        if r["kind"] == F.KIND_CORRECTED:
            o = by_row[r["row"]]
            assert abs(r["before"] - o["before"]) <= 1e-12 * abs(o["before"])
            assert abs(r["after"] - o["after"]) <= 1e-12 * max(1.0, abs(o["after"]))


def test_fault_classes():
    """Two equal faults in one tile (rows and columns that cannot be paired)
    -> recomputed; a fault on an encoded checksum
    only -> checksum-only, data untouched; a data fault plus a fault on its
    column's encoded checksum -> recomputed; an FP64 exponent flip that
    yields Inf/NaN -> rebuilt; a perturbation far below the threshold ->
    not flagged."""
    m = n = k = 256
    A, B, Cin = synth.operands(6, 0, m, n, k, "uniform")
    F_ = synth.Fault
    bk = f64_tiling(m, n, k)[2]
    part = A[:, :bk] @ B[:bk, :]
    cand = np.argwhere((np.abs(part) >= 1) & (np.abs(part) < 2))
    ri, ci = map(int, cand[0])
    plan = [
        F_(3, 5, 10, synth.ADD, 50.0), F_(40, 90, 200, synth.ADD, 50.0),       # tile (0,0)
        F_(130, 7, 0, synth.ADD, 3.0, target=synth.TGT_ROW_CHECKSUM),           # tile (1,0)
        F_(10, 200, 5, synth.ADD, 40.0),
        F_(0, 200, 5, synth.ADD, 2.0, target=synth.TGT_ROW_CHECKSUM),           # tile (0,1)
    ]
    # a flip in the tile (1,1), on an accumulator whose first-step value is in [1,2)
    tile_of = lambda r, c: (r // 128, c // 128)
    used = {tile_of(f.row, f.col) for f in plan}
    for ri, ci in map(tuple, cand):
        if tile_of(ri, ci) not in used:
            break
    plan.append(F_(int(ri), int(ci), 3, synth.BITFLIP, 0.0, 62))
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, False, False, plan)
    kinds = sorted(r["kind"] for r in rep.records)
    assert kinds == sorted([F.KIND_RECOMPUTED, F.KIND_CHECKSUM_ONLY, F.KIND_RECOMPUTED,
                            F.KIND_CORRECTED])
    flip = [e for e in rep.echoes if e["row"] == ri and e["col"] == ci][0]
    assert flip["applied"] and not np.isfinite(flip["after"])
    # tiny fault: not flagged
    tr, tc = O.default().tile_thresholds(A, B, 0, 0, Cin, 1.0, 1.0, tm=128, tn=128, bk=bk)
    tiny = [F_(7, 9, 30, synth.ADD, 1e-3 * min(tr.min(), tc.min()))]
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, False, False, tiny)
    assert not rep.records


def test_single_errors_on_every_column_class():
    """One error per tile at local columns 0, 16, ..., 112 and rows in both
    wave rows: each is rebuilt as the oracle rebuilds it."""
    m, n, k = 1024, 1024, 96
    A, B, Cin = synth.operands(36, 0, m, n, k, "uniform")
    F_ = synth.Fault
    plan = []
    for t in range(16):
        ti, tj = t % 8, (t // 8) * 4 + t % 4
        plan.append(F_(ti * 128 + (53 * t + 64) % 128, tj * 128 + 16 * (t % 8),
                       (7 * t) % k, synth.ADD, 40.0 + t))
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, False, False, plan)
    assert rep.corrected == 16 == rep.detected


def test_plain_kernel_matches_oracle():
    A, B, Cin = synth.operands(7, 0, 333, 222, 111, "normal")
    got, rep = gpu_f64(A, B, Cin, 1.5, -0.5, abft=False)
    assert normwise(got, O.default().gemm(A, B, Cin, 1.5, -0.5)) <= TOL


def test_bitwise_reproducible():
    A, B, Cin = synth.operands(8, 0, 384, 256, 200, "uniform")
    plan = [synth.Fault(100, 100, 50, synth.ADD, 7.0)]
    g1, r1 = gpu_f64(A, B, Cin, 1.0, 1.0, plan=plan)
    g2, r2 = gpu_f64(A, B, Cin, 1.0, 1.0, plan=plan)
    assert np.array_equal(g1, g2) and flagged(r1.records) == flagged(r2.records)


@pytest.mark.parametrize("size", [2048])
def test_c2_square_full_compare(size):
    """m = n = k = 2048, alpha = beta = 1, U[-1,1]: error-free, then one
    fault per 64 tiles of size 10^U(0,6) times the typical |C|."""
    A, B, Cin = synth.operands(20, size, size, size, size, "uniform")
    _, rep, _ = _compare(A, B, Cin, 1.0, 1.0, False, False, [])
    assert not rep.records and rep.max_ratio < 1
    sigma = np.sqrt(size / 9.0 + 1.0 / 3.0)
    ntiles = (size // 128) ** 2
    g = synth.rng(20, size, synth.STREAM_PLAN)
    plan = _plan_acc(g, size, size, size, 128, 128, -(-ntiles // 64), synth.log_magnitude(sigma))
    _, rep, _ = _compare(A, B, Cin, 1.0, 1.0, False, False, plan)
    assert rep.corrected == len(plan) == rep.detected


@pytest.mark.parametrize("size", [4096, 8192])
def test_c2_sampled_tiles(size):
    """4096^3 and the full 8192^3 timed by the benchmark; error-free, then
    one fault per 64 tiles: the oracle checks every tile that holds a fault
    (up to 24) plus sampled clean and corner tiles."""
    A, B, Cin = synth.operands(20, size, size, size, size, "uniform")
    sigma = np.sqrt(size / 9.0 + 1.0 / 3.0)
    tiles_m = size // 128
    g = synth.rng(20, size, synth.STREAM_PLAN)
    plan = _plan_acc(g, size, size, size, 128, 128, tiles_m * tiles_m // 64,
                     synth.log_magnitude(sigma))
    faulty = sorted({(f.row // 128) + (f.col // 128) * tiles_m for f in plan})
    extra = [0, tiles_m * tiles_m - 1, tiles_m - 1] + list(synth.rng(20, 1, 9).choice(
        tiles_m * tiles_m, 8, replace=False))
    tiles = sorted(set(faulty[:24]) | set(int(t) for t in extra))
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, False, False, [], tiles=tiles)
    assert not rep.records and 0 < rep.max_ratio < 1
    assert rep.tiles_verified == tiles_m * tiles_m
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, False, False, plan, tiles=tiles)
    assert rep.corrected == len(plan) == rep.detected
    assert rep.tiles_verified == tiles_m * tiles_m
