"""BF16 and FP8 (E4M3, per-tensor scale) fault-tolerant GEMM on the GPU
against the CPU oracle.

The oracle runs in FP64 on the same quantised inputs (decoded by its own
decoders), with alpha' = alpha * sA * sB, FP32 accumulators for bit flips
and u = 2^-24 in its thresholds; for FP8 its thresholds also carry the
term of the matrix instructions' truncated group sums (grid 2^-14 of the
group's largest product, groups of 8 inner indices).

Tolerance on C, normwise max|C - C_oracle| / max|C_oracle|: 1e-5 for BF16
and 1e-4 for FP8.  BF16 products are exact in FP32 and added as in FP32, so
the only errors are the FP32 accumulation (a random walk of unit roundoffs
of the partial sums, below 1e-6 normwise for k <= 8192 with these inputs)
and the FP32 rounding of the output (2^-24 relative); 1e-5 leaves a margin
of ten.  The FP8 instructions cut every product to a multiple of 2^-14 times
its group's largest product: a group of 8 errs by at most 8 * 2^-14 M_g
(M_g about 3 sigma_a sigma_b for normal inputs), and the k / 8 groups of an
element add like a random walk, against max|C| of about 4.5 sqrt(k)
sigma_a sigma_b -- about 2^-11 * 3 / (4.5 sqrt(8)) = 1.2e-4 normwise if
every group erred the same way; as a random walk the groups' errors give
about 1.2e-4 / sqrt(k / 8) at most (1e-5 .. 3e-5 measured), so 1e-4.  An
element rebuilt by the correction carries the rounding error of the FP32
encoded checksum it is rebuilt from and the other outputs' errors along
its line: rebuilt elements are held instead to that error, the other
outputs' part measured exactly and the checksum's part bounded from the
actual partial sums (gpu_util.rebuild_bound).

Flagged (row, col, kind) sets must agree exactly with the oracle's; planned
bit flips are kept only when their effect is at least 8 times the larger
threshold of their row and column (or not finite), so that both sides'
decisions are far from the threshold."""
import numpy as np
import pytest

from gpu_util import (flagged, gpu_lp, lp_inputs, lp_mma, lp_tiling, normwise,
                      rebuild_bound, say, to_oracle)
from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = {F.BF16: 1e-5, F.FP8_E4M3: 1e-4}
DTYPES = [pytest.param(F.BF16, id="bf16"), pytest.param(F.FP8_E4M3, id="fp8")]


def _c32(Cin):
    return np.asfortranarray(Cin.astype(np.float32).astype(np.float64))


def _flip32(v, bit):
    b = np.array([v], dtype=np.float32).view(np.uint32)
    b ^= np.uint32(1 << bit)
    return float(b.view(np.float32)[0])


def _compare(A, B, Cin, alpha, beta, dtype, ta=False, tb=False, plan=(), tiles=None, q=None):
    """Quantise, run both sides, compare C and the flagged sets."""
    m, n = Cin.shape
    k = A.shape[0] if ta else A.shape[1]
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    ca, cb, sa, sb, dA, dB = lp_inputs(A, B, dtype) if q is None else q
    Cin = _c32(Cin)
    say("case dtype=%d m=%d n=%d k=%d ta=%d tb=%d faults=%d" % (dtype, m, n, k, ta, tb,
                                                               len(plan)))
    got, rep = gpu_lp(ca, cb, Cin, alpha, beta, dtype, ta, tb, plan, scale_a=sa, scale_b=sb)
    ref = O.default().ftgemm(dA, dB, Cin, alpha * sa * sb, beta, ta, tb, tm, tn, bk, 32,
                             to_oracle(plan), tiles=tiles, mma=lp_mma(dtype))
    recs = rep.records
    tiles_m = -(-m // tm)
    if tiles is not None:
        keep = set(int(t) for t in tiles)
        recs = [r for r in recs if r["tile_m"] + r["tile_n"] * tiles_m in keep]
    assert flagged(recs) == flagged(ref.records)
    mask = ~np.isnan(ref.C)
    # elements the correction rebuilt (every one the oracle changed in a
    # corrected tile) are held to the rounding bound of a rebuild
    corrected = {(r["tile_m"], r["tile_n"]) for r in recs if r["kind"] == F.KIND_CORRECTED}
    for i, j in np.argwhere(mask & ~(ref.raw == ref.C)):
        if (i // tm, j // tn) not in corrected:
            continue
        bound = rebuild_bound(dA, dB, ta, tb, alpha * sa * sb, tm, tn, got, ref.C, i, j)
        tau = max(r["tau_row"] for r in recs if (r["tile_m"], r["tile_n"]) == (i // tm, j // tn))
        assert abs(got[i, j] - ref.C[i, j]) <= bound, (i, j, got[i, j], ref.C[i, j], bound, tau)
        mask[i, j] = False
    err = normwise(got[mask], ref.C[mask])
    assert err <= TOL[dtype], err
    return got, rep, ref


def _guarded_flips(A, B, dA, dB, sa, sb, alpha, beta, Cin, dtype, count, g, ta=False, tb=False):
    """Bit flips on FP32 accumulators (exponent and high fraction bits) in
    distinct tiles, kept when their effect is far above the thresholds."""
    m, n = Cin.shape
    k = A.shape[0] if ta else A.shape[1]
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    orc = O.default()
    cand = synth.bitflip_plan(g, m, n, k, tm, tn, min(4 * count, (-(-m // tm)) * (-(-n // tn))))
    kept = []
    for f in cand:
        kend = min(k, (f.k_index // bk + 1) * bk)
        before = float(orc.gemm_entries(dA, dB, [f.row], [f.col], ta=ta, tb=tb, k=kend)[0])
        before = float(np.float32(before))
        after = _flip32(before, f.bit)
        tr, tc = orc.tile_thresholds(dA, dB, f.row // tm, f.col // tn, _c32(Cin),
                                     alpha * sa * sb, beta, ta, tb, tm, tn, bk, 32,
                                     mma=lp_mma(dtype))
        tau = max(tr[f.col % tn], tc[f.row % tm])
        if not np.isfinite(after) or abs(alpha * sa * sb * (after - before)) >= 8 * tau:
            kept.append(f)
        if len(kept) == count:
            break
    return kept


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
def test_lp_ragged_transposes(dtype, ta, tb):
    """Ragged in every dimension (m, n not multiples of 8; k not a multiple
    of the 16-byte load), beta != 0, additive faults on accumulators."""
    m, n, k = 203, 141, 301
    A, B, Cin = synth.operands(30, 1, m, n, k, "normal", ta, tb)
    q = lp_inputs(A, B, dtype)
    g = synth.rng(30, 1, synth.STREAM_PLAN)
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    # accumulator deltas of 1e3 .. 1e5 in output units (accumulators carry
    # the FP8 scales out)
    plan = synth.additive_plan(g, m, n, k, tm, tn, 4,
                               synth.log_magnitude(1e3 / (q[2] * q[3]), 0.0, 2.0))
    got, rep, ref = _compare(A, B, Cin, -0.7, 1.3, dtype, ta, tb, plan, q=q)
    assert rep.corrected == 4 == rep.detected


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 3, 5), (128, 128, 64), (129, 127, 65),
                                   (64, 300, 129), (300, 17, 1000), (8, 9, 16)])
def test_lp_small_and_edge_shapes(dtype, m, n, k):
    A, B, Cin = synth.operands(31, m * 1000 + n, m, n, k, "uniform")
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, dtype)
    assert not rep.records and rep.tiles_verified == (-(-m // 128)) * (-(-n // 128))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,n,k", [(333, 222, 111), (3999, 2001, 301)])
def test_lp_plain_kernel_bitwise_equals_ft(dtype, m, n, k):
    """With no faults the checksum-free kernel writes the same bits (128-row
    tiles at 333 x 222, 256-row ones at 3999 x 2001)."""
    A, B, Cin = synth.operands(32, 0, m, n, k, "normal")
    ca, cb, sa, sb, dA, dB = lp_inputs(A, B, dtype)
    C32 = _c32(Cin)
    ft, rep = gpu_lp(ca, cb, C32, 1.5, -0.5, dtype, scale_a=sa, scale_b=sb)
    plain, _ = gpu_lp(ca, cb, C32, 1.5, -0.5, dtype, abft=False, scale_a=sa, scale_b=sb)
    assert np.array_equal(ft, plain) and not rep.records
    ref = O.default().gemm(dA, dB, C32, 1.5 * sa * sb, -0.5)
    assert normwise(plain, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_lp_special_cases(dtype):
    A, B, Cin = synth.operands(33, 0, 70, 50, 40, "uniform")
    ca, cb, sa, sb, dA, dB = lp_inputs(A, B, dtype)
    C32 = _c32(Cin)
    got, rep = gpu_lp(ca, cb, C32, 0.0, 0.5, dtype, scale_a=sa, scale_b=sb)
    assert np.array_equal(got, _c32(0.5 * C32))
    nanC = np.full_like(C32, np.nan)
    got, rep = gpu_lp(ca, cb, nanC, 1.0, 0.0, dtype, scale_a=sa, scale_b=sb)
    ref = O.default().gemm(dA, dB, None, sa * sb, 0.0)
    assert normwise(got, ref) <= TOL[dtype] and not rep.records
    got, rep = gpu_lp(ca, cb, C32, 0.0, 1.0, dtype, scale_a=sa, scale_b=sb)
    assert np.array_equal(got, C32)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("pad", [5, 2])
@pytest.mark.parametrize("abft", [1, 0])
def test_lp_padded_leading_dimension_of_c(dtype, pad, abft):
    """ldc = 135 (columns off 16-byte boundaries: one store per element) and
    132 (16-byte stores of four rows, the last tile row's partial group of
    130 rows element by element), with and without checksums."""
    A, B, Cin = synth.operands(34, 0, 130, 140, 33, "uniform")
    ca, cb, sa, sb, dA, dB = lp_inputs(A, B, dtype)
    C32 = _c32(Cin)
    got, rep = gpu_lp(ca, cb, C32, 1.0, 1.0, dtype, scale_a=sa, scale_b=sb, ldc_pad=pad,
                      abft=abft)
    assert normwise(got, O.default().gemm(dA, dB, C32, sa * sb, 1.0)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_lp_bitflips_and_fault_classes(dtype):
    """FP32 accumulator bit flips (exponent / high fraction bits) located
    and rebuilt; a checksum-only fault; two equal faults in one tile (rows
    and columns that cannot be paired) recomputed."""
    m = n = 512
    k = 1024
    A, B, Cin = synth.operands(35, 0, m, n, k, "normal")
    q = lp_inputs(A, B, dtype)
    ca, cb, sa, sb, dA, dB = q
    g = synth.rng(35, 0, synth.STREAM_PLAN)
    flips = _guarded_flips(A, B, dA, dB, sa, sb, 1.0, 1.0, Cin, dtype, 8, g)
    assert len(flips) >= 6
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, dtype, plan=flips, q=q)
    assert rep.corrected == len(flips) == rep.detected
    for e, f in zip(rep.echoes, flips):
        assert e["applied"] and (e["row"], e["col"]) == (f.row, f.col)
        assert np.float32(e["after"]).view(np.uint32) == \
            np.float32(e["before"]).view(np.uint32) ^ np.uint32(1 << f.bit)
    # fault classes in tiles the flips left alone
    used = {(f.row // 128, f.col // 128) for f in flips}
    free = [(a, b) for b in range(4) for a in range(4) if (a, b) not in used]
    (a0, b0), (a1, b1) = free[0], free[1]
    Fa = synth.Fault
    unit = 1.0 / (sa * sb)  # accumulator units per output unit
    plan = [Fa(128 * a0 + 3, 128 * b0 + 5, 10, synth.ADD, 5e4 * unit),
            Fa(128 * a0 + 40, 128 * b0 + 90, 900, synth.ADD, 5e4 * unit),
            Fa(128 * a1 + 7, 128 * b1 + 1, 0, synth.ADD, 1e5, target=synth.TGT_ROW_CHECKSUM)]
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, dtype, plan=plan, q=q)
    assert sorted(r["kind"] for r in rep.records) == sorted([F.KIND_RECOMPUTED,
                                                            F.KIND_CHECKSUM_ONLY])


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
def test_lp_256_row_tiles(ta, tb):
    """The 256 x 128 BF16 tile (chosen from 256 tiles on): ragged in every
    dimension, beta != 0, additive faults on accumulators in the last row
    and column tiles and the interior, checked against the oracle on the
    whole output."""
    dtype = F.BF16
    m, n, k = 3999, 2001, 301
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    assert (tm, tn) == (256, 128)
    A, B, Cin = synth.operands(31, 1, m, n, k, "normal", ta, tb)
    q = lp_inputs(A, B, dtype)
    unit = 1.0 / (q[2] * q[3])  # accumulator units per output unit
    Fa = synth.Fault
    plan = [Fa(m - 1, n - 1, k - 1, synth.ADD, 2e3 * unit),      # corner tile, last step
            Fa(3840 + 100, 70, 64, synth.ADD, -5e3 * unit),      # last row tile
            Fa(255, 1920 + 7, 0, synth.ADD, 1e4 * unit),         # last column tile, first step
            Fa(1000, 1000, 150, synth.ADD, 3e3 * unit)]          # interior
    got, rep, ref = _compare(A, B, Cin, 0.9, -1.1, dtype, ta, tb, plan, q=q)
    assert rep.corrected == 4 == rep.detected
    assert rep.tiles_verified == 16 * 16


def test_lp_256_row_single_errors_on_every_column_class():
    """One error per tile of the 256 x 128 BF16 tile (taken from 256 tiles
    on), at local columns 0, 16, ..., 112 and rows in every wave: each is
    rebuilt, as the oracle rebuilds it."""
    dtype = F.BF16
    m, n, k = 4096, 2048, 256
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    assert (tm, tn) == (256, 128)
    A, B, Cin = synth.operands(35, 1, m, n, k, "normal")
    q = lp_inputs(A, B, dtype)
    unit = 1.0 / (q[2] * q[3])
    Fa = synth.Fault
    plan, tiles = [], []
    for t in range(16):
        ti, tj = t, (5 * t) % (n // tn)
        row = ti * tm + (37 * t + 192) % tm
        col = tj * tn + 16 * (t % 8)
        plan.append(Fa(row, col, (29 * t) % k, synth.ADD, (1.5e3 + 100 * t) * unit))
        tiles.append(ti + tj * (m // tm))
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, dtype, plan=plan, tiles=tiles, q=q)
    assert rep.corrected == 16 == rep.detected


def test_lp_8192_flips_rebuilt_in_wave_3():
    """Two FP32 exponent flips at 8192^3 BF16 (256 x 128 tiles), each on
    lane 0 of wave 3 of its tile (local rows 192 and 193, column 32): both
    are rebuilt, as the oracle rebuilds them.  A build that kept the
    report's running maximum in thread 0 alone across the beta pass lost
    thread 0's share of the rebuild's column sum there, so these tiles were
    computed again instead."""
    size = 8192
    A, B, Cin = synth.operands(41, size, size, size, size, "normal")
    q = lp_inputs(A, B, F.BF16)
    Fa = synth.Fault
    plan = [Fa(5568, 2720, 2858, synth.BITFLIP, 0.0, 24), Fa(4545, 7584, 1555, synth.BITFLIP, 0.0, 26)]
    tiles = sorted((f.row // 256) + (f.col // 128) * (size // 256) for f in plan)
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, F.BF16, plan=plan, tiles=tiles, q=q)
    assert rep.corrected == 2 == rep.detected


@pytest.mark.parametrize("rows", [256, 128])
@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
def test_lp_fp8_two_sided_from_the_norms_pass(ta, tb, rows, tmp_path):
    """Two-sided FP8 with at least 256 tiles, so the threshold norms and
    both operand checksums come from the pass over A and B before the
    product: on the default 256 x 128 tiles and on 128 x 128 ones (set by
    the tuning table); ragged in every dimension (k not a multiple of the
    step), every transpose (each operand's checksums then come from the
    other of the pass's two kernels), faults in the last row and column
    tiles and the interior, checked against the oracle on the whole
    output."""
    dtype = F.FP8_E4M3
    m, n, k = 3999, 2001, 301
    if rows == 128:
        table = tmp_path / "fp8_128.tune"
        table.write_text("tile %d 1 128\n" % dtype)
        F.load_tune_table(str(table))
    try:
        _fp8_two_sided_from_the_norms_pass(ta, tb, rows, dtype, m, n, k)
    finally:
        F.load_tune_table(None)


def _fp8_two_sided_from_the_norms_pass(ta, tb, rows, dtype, m, n, k):
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    assert (tm, tn) == (rows, 128)
    A, B, Cin = synth.operands(32, 1, m, n, k, "normal", ta, tb)
    q = lp_inputs(A, B, dtype)
    unit = 1.0 / (q[2] * q[3])  # accumulator units per output unit
    Fa = synth.Fault
    plan = [Fa(m - 1, n - 1, k - 1, synth.ADD, 2e3 * unit),      # corner tile, last step
            Fa(3968 + 20, 70, 200, synth.ADD, -5e3 * unit),      # last row tile
            Fa(127, 1920 + 7, 0, synth.ADD, 1e4 * unit),         # last column tile, first step
            Fa(1000, 1000, 150, synth.ADD, 3e3 * unit)]          # interior
    got, rep, ref = _compare(A, B, Cin, 0.9, -1.1, dtype, ta, tb, plan, q=q)
    assert rep.corrected == 4 == rep.detected
    assert rep.tiles_verified == -(-m // rows) * 16


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, True)])
def test_lp_line_corrections(dtype, ta, tb):
    """Errors confined to one row or one column of a tile are rebuilt from
    the other side's checksums and confirmed by the line's own: two and
    four in a row, three in a column; a data error with a checksum fault on
    another column of its row is computed again."""
    m, n, k = 384, 300, 200
    A, B, Cin = synth.operands(36, 1, m, n, k, "normal", ta, tb)
    q = lp_inputs(A, B, dtype)
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    assert (tm, tn) == (128, 128)
    u = 1.0 / (q[2] * q[3])  # accumulator units per output unit
    Fa = synth.Fault
    plan = [Fa(17, 3, 10, synth.ADD, 3e3 * u), Fa(17, 90, 150, synth.ADD, -4e3 * u),   # (0, 0)
            Fa(140, 130, 5, synth.ADD, 2e3 * u), Fa(140, 150, 60, synth.ADD, 5e3 * u),  # (1, 1)
            Fa(140, 200, 199, synth.ADD, -3e3 * u), Fa(140, 255, 99, synth.ADD, 6e3 * u),
            Fa(260, 40, 0, synth.ADD, 2e3 * u), Fa(300, 40, 70, synth.ADD, 8e3 * u),     # (2, 0)
            Fa(383, 40, 199, synth.ADD, -5e3 * u),
            Fa(5, 270, 30, synth.ADD, 4e3 * u),                                          # (0, 2)
            Fa(0, 290, 30, synth.ADD, 3e3, target=synth.TGT_ROW_CHECKSUM)]
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, dtype, ta, tb, plan, q=q)
    kinds = {(r["tile_m"], r["tile_n"]): r["kind"] for r in rep.records}
    assert kinds == {(0, 0): F.KIND_CORRECTED, (1, 1): F.KIND_CORRECTED,
                     (2, 0): F.KIND_CORRECTED, (0, 2): F.KIND_RECOMPUTED}


@pytest.mark.parametrize("dtype", DTYPES)
def test_lp_crossing_pairs(dtype):
    """Errors in distinct rows and columns of a tile (two, four, three per
    tile) paired by their residuals and corrected; two equal errors ->
    recomputed.  Rebuilt elements are held to their thresholds, the rest
    to the format's tolerance, flagged sets exactly."""
    m, n, k = 384, 300, 200
    A, B, Cin = synth.operands(37, 1, m, n, k, "normal")
    q = lp_inputs(A, B, dtype)
    tm, tn, bk = lp_tiling(dtype, m, n, k)
    assert (tm, tn) == (128, 128)
    u = 1.0 / (q[2] * q[3])  # accumulator units per output unit
    Fa = synth.Fault
    plan = [Fa(17, 90, 10, synth.ADD, 3e3 * u), Fa(60, 3, 150, synth.ADD, -4e3 * u),   # (0, 0)
            Fa(140, 250, 5, synth.ADD, 2e3 * u), Fa(150, 130, 60, synth.ADD, 5e3 * u),  # (1, 1)
            Fa(200, 200, 199, synth.ADD, -3e3 * u), Fa(255, 155, 99, synth.ADD, 6e3 * u),
            Fa(260, 280, 0, synth.ADD, 2e3 * u), Fa(300, 260, 70, synth.ADD, 8e3 * u),  # (2, 2)
            Fa(383, 299, 199, synth.ADD, -5e3 * u),
            Fa(10, 260, 3, synth.ADD, 7e3 * u), Fa(20, 270, 30, synth.ADD, 7e3 * u)]    # (0, 2)
    got, rep, ref = _compare(A, B, Cin, 1.0, 0.5, dtype, False, False, plan, q=q)
    kinds = {(r["tile_m"], r["tile_n"]): r["kind"] for r in rep.records}
    assert kinds == {(0, 0): F.KIND_CORRECTED, (1, 1): F.KIND_CORRECTED,
                     (2, 2): F.KIND_CORRECTED, (0, 2): F.KIND_RECOMPUTED}
    named = sorted((r["row"], r["col"], r["nbad_rows"]) for r in rep.records
                   if r["kind"] == F.KIND_CORRECTED)
    assert named == [(17, 90, 2), (140, 250, 4), (260, 280, 3)]


@pytest.mark.parametrize("dtype", DTYPES)
def test_lp_8192_sampled_tiles(dtype):
    """m = n = k = 8192, normal inputs, as timed by the benchmark (256 x 128
    tiles).  Error-free: no tile flagged.  With
    one guarded FP32
    bit flip per 64 tiles: every one located and rebuilt; the oracle checks
    the tiles holding a fault plus sampled clean and corner tiles."""
    size = 8192
    A, B, Cin = synth.operands(40, size, size, size, size, "normal")
    q = lp_inputs(A, B, dtype)
    ca, cb, sa, sb, dA, dB = q
    tm, tn, bk = lp_tiling(dtype, size, size, size)
    assert (tm, tn) == (256, 128)
    tiles_m, tiles_n = size // tm, size // tn
    ntiles = tiles_m * tiles_n
    extra = [0, ntiles - 1, tiles_m - 1, ntiles - tiles_m] + [
        int(t) for t in synth.rng(40, 1, 9).choice(ntiles, 5, replace=False)]
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, dtype, tiles=sorted(set(extra)), q=q)
    assert rep.detected == 0 and rep.tiles_verified == ntiles
    assert 0 < rep.max_ratio < 1
    g = synth.rng(40, size, synth.STREAM_PLAN)
    flips = _guarded_flips(A, B, dA, dB, sa, sb, 1.0, 1.0, Cin, dtype, ntiles // 64, g)
    assert len(flips) == ntiles // 64
    faulty = sorted({(f.row // tm) + (f.col // tn) * tiles_m for f in flips})
    tiles = sorted(set(faulty[:12]) | set(extra))
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, dtype, plan=flips, tiles=tiles, q=q)
    assert rep.corrected == len(flips) == rep.detected


@pytest.mark.parametrize("dtype", DTYPES)
def test_group_sums_of_the_matrix_instructions(dtype):
    """The arithmetic the thresholds assume, observed through the library:
    448 * 448 + 7 * 1 within one group of 8 inner indices comes out as
    448^2 in FP8 (7 is below 2^-14 of the product's binade 2^17 and is cut),
    but exactly when the two products sit in different groups, and always
    exactly in BF16.  The fault-tolerant call flags nothing."""
    k = 16
    for pos, exact_expected in ((1, dtype != F.FP8_E4M3), (8, True)):
        A = np.zeros((1, k), order="F")
        B = np.zeros((k, 1), order="F")
        A[0, 0], B[0, 0] = 448.0, 448.0
        A[0, pos], B[pos, 0] = 7.0, 1.0
        if dtype == F.BF16:
            ca, cb = synth.to_bf16_bits(A), synth.to_bf16_bits(B)
        else:
            ca, cb = synth.to_e4m3_bits(A, 1.0), synth.to_e4m3_bits(B, 1.0)
        C0 = np.zeros((1, 1), order="F")
        for abft in (False, True):
            got, rep = gpu_lp(ca, cb, C0, 1.0, 0.0, dtype, abft=abft)
            want = 200711.0 if exact_expected else 200704.0
            assert got[0, 0] == want, (dtype, pos, abft, got[0, 0])
            assert not rep.records
