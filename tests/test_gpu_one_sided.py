"""The one-sided low-precision mode (abft = 2) on the GPU against the CPU
oracle in its one-sided mode.

Only the column checksum C e of each tile is kept (one entry per row); a
tile with any disagreeing row is computed again.  The thresholds are built
from the row norms of op(A) and column norms of op(B), which the library
takes in a pass over A and B before the product; the records' thresholds are
held to the oracle's (exact FP64 norms) within 1e-4 relative, which pins that
pass.  Flagged (row, kind) sets must agree exactly; C within the format's
tolerance (BF16 1e-5, FP8 5e-4 normwise, as for the two-sided mode): a
recomputed tile is computed exactly like a fault-free one, so no element is
exempt."""
import numpy as np
import pytest

from gpu_util import flagged, gpu_lp, lp_inputs, lp_mma, normwise, say
from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = {F.BF16: 1e-5, F.FP8_E4M3: 5e-4}
DTYPES = [pytest.param(F.BF16, id="bf16"), pytest.param(F.FP8_E4M3, id="fp8")]
Fa = synth.Fault


def _c32(Cin):
    return np.asfortranarray(Cin.astype(np.float32).astype(np.float64))


def _tiling(dtype, m, n, k):
    tm, tn, bk, _ = F.query_tiling_ex(dtype, m, n, k, abft=2)
    return tm, tn, bk


def _flip32(v, bit):
    b = np.array([v], dtype=np.float32).view(np.uint32)
    b ^= np.uint32(1 << bit)
    return float(b.view(np.float32)[0])


def _guarded_flips(A, dA, dB, sa, sb, Cin, dtype, count, g, tm, tn, bk):
    """FP32 accumulator exponent flips in distinct tiles whose change of the
    output is at least 8 times the threshold of its row (or not finite)."""
    m, n = Cin.shape
    k = A.shape[1]
    orc = O.default()
    cand = synth.bitflip_plan(g, m, n, k, tm, tn, 4 * count, bits=[27, 28, 29, 30])
    kept = []
    for f in cand:
        kend = min(k, (f.k_index // bk + 1) * bk)
        before = float(np.float32(orc.gemm_entries(dA, dB, [f.row], [f.col], k=kend)[0]))
        after = _flip32(before, f.bit)
        _, tc = orc.tile_thresholds(dA, dB, f.row // tm, f.col // tn, _c32(Cin), sa * sb, 1.0,
                                    False, False, tm, tn, bk, 32, mma=lp_mma(dtype))
        if not np.isfinite(after) or abs(sa * sb * (after - before)) >= 8 * tc[f.row % tm]:
            kept.append(f)
        if len(kept) == count:
            break
    return kept


def _compare(A, B, Cin, alpha, beta, dtype, ta=False, tb=False, plan=(), tiles=None, q=None):
    m, n = Cin.shape
    k = A.shape[0] if ta else A.shape[1]
    tm, tn, bk = _tiling(dtype, m, n, k)
    ca, cb, sa, sb, dA, dB = lp_inputs(A, B, dtype) if q is None else q
    Cin = _c32(Cin)
    say("one-sided case dtype=%d m=%d n=%d k=%d ta=%d tb=%d tile=%dx%d faults=%d" % (
        dtype, m, n, k, ta, tb, tm, tn, len(plan)))
    got, rep = gpu_lp(ca, cb, Cin, alpha, beta, dtype, ta, tb, plan, abft=2,
                      scale_a=sa, scale_b=sb)
    ref = O.default().ftgemm(dA, dB, Cin, alpha * sa * sb, beta, ta, tb, tm, tn, bk, 32,
                             [O.Injection(f.row, f.col, f.k_index, f.mode, f.delta, f.bit,
                                          f.target) for f in plan],
                             tiles=tiles, mma=lp_mma(dtype), one_sided=True)
    recs = rep.records
    tiles_m = -(-m // tm)
    if tiles is not None:
        keep = set(int(t) for t in tiles)
        recs = [r for r in recs if r["tile_m"] + r["tile_n"] * tiles_m in keep]
    assert flagged(recs) == flagged(ref.records)
    by_row = {r["row"]: r for r in ref.records}
    for r in recs:
        o = by_row[r["row"]]
        assert r["col"] == -1 and r["kind"] == F.KIND_RECOMPUTED
        assert r["nbad_cols"] == 0 and r["nbad_rows"] == o["nbad_rows"]
        assert abs(r["tau_col"] - o["tau_col"]) <= 1e-4 * o["tau_col"], (r, o)
    mask = ~np.isnan(ref.C)
    err = normwise(got[mask], ref.C[mask])
    assert err <= TOL[dtype], err
    return got, rep, ref


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,n,k", [(203, 141, 301), (3999, 2001, 301)])
@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
def test_one_sided_ragged(dtype, m, n, k, ta, tb):
    """Ragged in every dimension, beta != 0; accumulator faults in the
    corner, last-row and interior tiles, two in one tile (different rows),
    one on a column-checksum entry and one on a row-checksum entry (which
    the one-sided mode does not have: not applied).  3999 x 2001 runs the
    256 x 128 tiles."""
    A, B, Cin = synth.operands(60, m, m, n, k, "normal", ta, tb)
    q = lp_inputs(A, B, dtype)
    tm, tn, bk = _tiling(dtype, m, n, k)
    assert tm == (256 if m > 1000 else 128)
    unit = 1.0 / (q[2] * q[3])  # accumulator units per output unit
    plan = [Fa(m - 1, n - 1, k - 1, synth.ADD, 2e3 * unit),            # corner, last step
            Fa(m - 3, 5, bk, synth.ADD, -5e3 * unit),                  # last row tile
            Fa(tm + 7, 2, 0, synth.ADD, 1e4 * unit),                   # tile (1, 0)
            Fa(tm + 40, 9, k // 2, synth.ADD, 3e3 * unit),             # same tile, other row
            Fa(3, tn + 4, 10, synth.ADD, 1e5, target=synth.TGT_COL_CHECKSUM),
            Fa(5, tn + 6, 10, synth.ADD, 1e5, target=synth.TGT_ROW_CHECKSUM)]
    got, rep, ref = _compare(A, B, Cin, -0.7, 1.3, dtype, ta, tb, plan, q=q)
    assert rep.recomputed == rep.detected == len(ref.records) >= 3 and rep.corrected == 0
    applied = [e["applied"] for e in rep.echoes]
    assert applied == [True] * 5 + [False]
    assert applied == [e["applied"] for e in ref.echo]


@pytest.mark.parametrize("dtype", DTYPES)
def test_one_sided_fault_free_bits(dtype):
    """Without faults the one-sided call writes the bits of the kernel
    without checksums and of the two-sided one (here all three take the
    same 256-row tiles)."""
    m, n, k = 3999, 2001, 301
    A, B, Cin = synth.operands(61, 0, m, n, k, "normal")
    ca, cb, sa, sb, dA, dB = lp_inputs(A, B, dtype)
    C32 = _c32(Cin)
    one, rep = gpu_lp(ca, cb, C32, 1.5, -0.5, dtype, abft=2, scale_a=sa, scale_b=sb)
    plain, _ = gpu_lp(ca, cb, C32, 1.5, -0.5, dtype, abft=False, scale_a=sa, scale_b=sb)
    two, _ = gpu_lp(ca, cb, C32, 1.5, -0.5, dtype, abft=True, scale_a=sa, scale_b=sb)
    assert np.array_equal(one, plain) and np.array_equal(one, two)
    assert not rep.records and rep.tiles_verified == 16 * 16
    assert 0 < rep.max_ratio < 1


@pytest.mark.parametrize("dtype", DTYPES)
def test_one_sided_8192_sampled_tiles(dtype):
    """m = n = k = 8192 (256 x 128 tiles), as the benchmark times it.
    Error-free: nothing flagged.  One FP32 exponent flip (bits 27..30) per
    64 tiles, kept when its change is at least 8 times its row's threshold:
    every one detected and its tile recomputed; the oracle checks the
    faulty tiles (up to 10) and sampled clean and corner tiles."""
    size = 8192
    A, B, Cin = synth.operands(62, size, size, size, size, "normal")
    q = lp_inputs(A, B, dtype)
    tm, tn, bk = _tiling(dtype, size, size, size)
    assert (tm, tn) == (256, 128)
    tiles_m, tiles_n = size // tm, size // tn
    ntiles = tiles_m * tiles_n
    extra = [0, ntiles - 1, tiles_m - 1, ntiles - tiles_m] + [
        int(t) for t in synth.rng(62, 1, 9).choice(ntiles, 4, replace=False)]
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, dtype, tiles=sorted(set(extra)), q=q)
    assert rep.detected == 0 and rep.tiles_verified == ntiles
    gp = synth.rng(62, size, synth.STREAM_PLAN)
    flips = _guarded_flips(A, q[4], q[5], q[2], q[3], Cin, dtype, ntiles // 64, gp, tm, tn, bk)
    assert len(flips) == ntiles // 64
    faulty = sorted({(f.row // tm) + (f.col // tn) * tiles_m for f in flips})
    got, rep, ref = _compare(A, B, Cin, 1.0, 1.0, dtype, plan=flips,
                             tiles=sorted(set(faulty[:10]) | set(extra)), q=q)
    assert rep.detected == rep.recomputed == len(flips)
