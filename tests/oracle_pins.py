"""Pins of the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own formulas.  Each function takes an
``Oracle`` instance (the real build, or a deliberately broken copy in
test_oracle_mutants.py) and raises AssertionError when the pin fails.
"""
import numpy as np

from golden_io import read_threshold_example
from oracle import oracle as O
from paper_2305_02444_amd import synth


def _ops(A, B, ta, tb):
    return (A.T if ta else A), (B.T if tb else B)


def pin_gemm_vs_numpy(orc):
    """Plain GEMM equals numpy's matmul (a library routine) for every
    transpose combination, odd shapes and padded leading dimensions."""
    g = np.random.default_rng(11)
    for ta in (False, True):
        for tb in (False, True):
            m, n, k = 37, 29, 41
            sa = (k, m) if ta else (m, k)
            sb = (n, k) if tb else (k, n)
            # leading dimension larger than the row count: take a slice of a
            # taller Fortran array
            Abig = np.asfortranarray(g.uniform(-1, 1, (sa[0] + 5, sa[1])))
            Bbig = np.asfortranarray(g.uniform(-1, 1, (sb[0] + 3, sb[1])))
            A, B = Abig[:sa[0]], Bbig[:sb[0]]
            Cin = np.asfortranarray(g.uniform(-1, 1, (m, n)))
            alpha, beta = -0.75, 1.5
            got = orc.gemm(A, B, Cin, alpha, beta, ta, tb)
            oa, ob = _ops(A, B, ta, tb)
            ref = alpha * (oa @ ob) + beta * Cin
            err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
            assert err < 1e-14, (ta, tb, err)


def pin_gemm_integer_exact(orc):
    """On small integers every partial sum is exact: bit equality with numpy."""
    g = np.random.default_rng(12)
    A = np.asfortranarray(g.integers(-8, 9, (19, 23)).astype(float))
    B = np.asfortranarray(g.integers(-8, 9, (23, 17)).astype(float))
    Cin = np.asfortranarray(g.integers(-8, 9, (19, 17)).astype(float))
    got = orc.gemm(A, B, Cin, 2.0, -3.0)
    assert np.array_equal(got, 2.0 * (A @ B) - 3.0 * Cin)


def pin_blas_special_cases(orc):
    g = np.random.default_rng(13)
    A = np.asfortranarray(g.uniform(-1, 1, (9, 7)))
    B = np.asfortranarray(g.uniform(-1, 1, (7, 5)))
    Cin = np.asfortranarray(g.uniform(-1, 1, (9, 5)))
    # alpha == 0: beta * C
    assert np.array_equal(orc.gemm(A, B, Cin, 0.0, 0.5), 0.5 * Cin)
    # beta == 0: C_in is never read, NaNs in it do not propagate
    nanC = np.full((9, 5), np.nan, order="F")
    got = orc.gemm(A, B, nanC, 1.0, 0.0)
    assert np.all(np.isfinite(got))
    # k == 0: beta * C
    A0 = np.zeros((9, 0), order="F")
    B0 = np.zeros((0, 5), order="F")
    assert np.array_equal(orc.gemm(A0, B0, Cin, 1.0, 2.0), 2.0 * Cin)
    # the fault-tolerant path follows the same conventions
    r = orc.ftgemm(A, B, nanC, 1.0, 0.0, tm=4, tn=4, bk=2)
    assert np.all(np.isfinite(r.C)) and not r.records
    r = orc.ftgemm(A0, B0, Cin, 1.0, 2.0, tm=4, tn=4, bk=2)
    assert np.array_equal(r.C, 2.0 * Cin) and not r.records


def pin_checksum_identities(orc):
    """e^T(AB) = (e^T A)B and (AB)e = A(Be) hold exactly on small integers:
    the encoded checksums (built from the operands and C_in) must equal the
    reference checksums (sums of the computed C) bit for bit, in every tile,
    including ragged edge tiles and transposed operands."""
    for ta in (False, True):
        for tb in (False, True):
            g = synth.rng(90, int(ta) * 2 + int(tb), 0)
            m, n, k = 21, 18, 40
            A = np.asfortranarray(g.integers(-8, 9, (k, m) if ta else (m, k)).astype(float))
            B = np.asfortranarray(g.integers(-8, 9, (n, k) if tb else (k, n)).astype(float))
            Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
            for ti in range(-(-m // 8)):
                for tj in range(-(-n // 8)):
                    Pr, Pc, Rr, Rc = orc.tile_checksums(A, B, ti, tj, Cin, 2.0, -1.0, ta,
                                                        tb, tm=8, tn=8, bk=5)
                    assert np.array_equal(Pr, Rr), (ta, tb, ti, tj)
                    assert np.array_equal(Pc, Rc), (ta, tb, ti, tj)
                    # and the reference side really is the sum of the product
                    oa, ob = _ops(A, B, ta, tb)
                    Cf = 2.0 * (oa @ ob) - 1.0 * Cin
                    blk = Cf[ti * 8:ti * 8 + 8, tj * 8:tj * 8 + 8]
                    assert np.array_equal(Rr, blk.sum(axis=0))
                    assert np.array_equal(Rc, blk.sum(axis=1))


def pin_brute_force_location(orc):
    """A single injected error is located exactly where the faulty output
    differs from the fault-free product (found by brute force)."""
    g = np.random.default_rng(14)
    m, n, k = 50, 45, 64
    A = np.asfortranarray(g.uniform(-1, 1, (m, k)))
    B = np.asfortranarray(g.uniform(-1, 1, (k, n)))
    Cin = np.asfortranarray(g.uniform(-1, 1, (m, n)))
    Cff = A @ B * 1.25 + 0.5 * Cin
    for trial in range(12):
        row, col, kidx = int(g.integers(m)), int(g.integers(n)), int(g.integers(k))
        delta = float(g.choice([-1, 1]) * 10 ** g.uniform(-3, 3))
        r = orc.ftgemm(A, B, Cin, 1.25, 0.5, tm=16, tn=16, bk=8,
                       injections=[O.Injection(row, col, kidx, O.ADD, delta)])
        diff = np.abs(r.raw - Cff)
        bad = np.argwhere(diff > 1e-9)
        assert bad.tolist() == [[row, col]], (trial, bad)
        assert len(r.records) == 1
        rec = r.records[0]
        assert (rec["row"], rec["col"], rec["kind"]) == (row, col, O.CORRECTED)
        assert (rec["tile_m"], rec["tile_n"]) == (row // 16, col // 16)
        assert np.max(np.abs(r.C - Cff)) < 1e-12


def pin_exact_recovery(orc):
    """Integer data and an integer perturbation: the corrected output equals
    the fault-free product bit for bit."""
    g = synth.rng(91, 0, 0)
    m, n, k = 33, 30, 24
    A = np.asfortranarray(g.integers(-8, 9, (m, k)).astype(float))
    B = np.asfortranarray(g.integers(-8, 9, (k, n)).astype(float))
    Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
    Cff = 3.0 * (A @ B) + 2.0 * Cin
    plan = [O.Injection(3, 4, 5, O.ADD, 1000.0), O.Injection(20, 17, 23, O.ADD, -77.0),
            O.Injection(32, 29, 0, O.ADD, 5.0)]
    r = orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=4, injections=plan)
    assert np.array_equal(r.C, Cff)
    assert sorted((d["row"], d["col"]) for d in r.records) == [(3, 4), (20, 17), (32, 29)]
    assert all(d["kind"] == O.CORRECTED for d in r.records)
    # the perturbed value is what the record calls "before"
    for d in r.records:
        assert d["before"] == Cff[d["row"], d["col"]] + 3.0 * {3: 1000.0, 20: -77.0, 32: 5.0}[d["row"]]
        assert d["after"] == Cff[d["row"], d["col"]]


def pin_nonfinite_recovery(orc):
    """Exponent bit flips of FP32 accumulators that produce Inf or NaN are
    repaired by rebuilding the element from its column."""
    g = np.random.default_rng(15)
    m, n, k = 40, 40, 32
    A = np.asfortranarray(g.uniform(-1, 1, (m, k)))
    B = np.asfortranarray(g.uniform(-1, 1, (k, n)))
    Cff = A @ B
    # find an accumulator whose partial sum after the first step (bk = 8)
    # lies in [1, 2): flipping bit 30 makes its exponent all ones (Inf/NaN)
    part = A[:, :8] @ B[:8, :]
    cand = np.argwhere((np.abs(part) >= 1) & (np.abs(part) < 2))
    assert len(cand)
    row, col = map(int, cand[0])
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=8, acc_bits=32,
                   injections=[O.Injection(row, col, 3, O.BITFLIP, bit=30)])
    assert not np.isfinite(r.raw[row, col])
    assert r.echo[0]["applied"] and not np.isfinite(r.echo[0]["after"])
    assert len(r.records) == 1 and r.records[0]["kind"] == O.CORRECTED
    assert np.max(np.abs(r.C - Cff)) < 1e-12


def pin_classification(orc):
    """Two equal errors in one tile (their rows and columns cannot be
    paired) -> recomputed; a fault in an encoded checksum only ->
    checksum-only with C untouched; a perturbation far below the rounding
    threshold -> not flagged."""
    g = np.random.default_rng(16)
    m, n, k = 32, 32, 48
    A = np.asfortranarray(g.uniform(-1, 1, (m, k)))
    B = np.asfortranarray(g.uniform(-1, 1, (k, n)))
    Cff = A @ B
    two = [O.Injection(1, 2, 3, O.ADD, 50.0), O.Injection(5, 9, 40, O.ADD, 50.0)]
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=16, injections=two)
    assert [d["kind"] for d in r.records] == [O.RECOMPUTED]
    assert r.records[0]["nbad_rows"] == 2 and r.records[0]["nbad_cols"] == 2
    assert np.max(np.abs(r.C - Cff)) < 1e-13
    ck = [O.Injection(20, 21, 10, O.ADD, 3.0, target=O.TGT_ROW_CHECKSUM)]
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=16, injections=ck)
    assert [d["kind"] for d in r.records] == [O.CHECKSUM_ONLY]
    assert r.records[0]["col"] == 21 and r.records[0]["row"] == -1
    assert np.max(np.abs(r.C - Cff)) < 1e-13
    ck = [O.Injection(20, 21, 10, O.ADD, 3.0, target=O.TGT_COL_CHECKSUM)]
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=16, injections=ck)
    assert [d["kind"] for d in r.records] == [O.CHECKSUM_ONLY]
    assert r.records[0]["row"] == 20 and r.records[0]["col"] == -1
    # two errors in one row: one row and two columns disagree -> both
    # rebuilt from their columns and confirmed by the row
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=16, injections=[
        O.Injection(3, 1, 3, O.ADD, 5.0), O.Injection(3, 7, 30, O.ADD, 8.0)])
    assert [(d["kind"], d["row"], d["col"]) for d in r.records] == [(O.CORRECTED, 3, 1)]
    assert np.max(np.abs(r.C - Cff)) < 1e-13
    # two errors cancelling in their column: two rows and no column disagree;
    # that is not a single checksum fault -> recomputed, not left alone
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=16, injections=[
        O.Injection(2, 4, 3, O.ADD, 6.0), O.Injection(9, 4, 3, O.ADD, -6.0)])
    assert [d["kind"] for d in r.records] == [O.RECOMPUTED]
    assert r.records[0]["nbad_rows"] == 2 and r.records[0]["nbad_cols"] == 0
    assert np.max(np.abs(r.C - Cff)) < 1e-12
    # a data error plus a fault in the encoded checksum of its own column:
    # the rebuilt value does not confirm against the row side -> recomputed
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=16, injections=[
        O.Injection(6, 5, 3, O.ADD, 40.0),
        O.Injection(0, 5, 3, O.ADD, 2.0, target=O.TGT_ROW_CHECKSUM)])
    assert [d["kind"] for d in r.records] == [O.RECOMPUTED]
    assert np.max(np.abs(r.C - Cff)) < 1e-13
    tr, tc = orc.tile_thresholds(A, B, 1, 1, tm=16, tn=16, bk=16)
    tiny = 0.01 * min(tr.min(), tc.min())
    r = orc.ftgemm(A, B, tm=16, tn=16, bk=16,
                   injections=[O.Injection(20, 21, 10, O.ADD, tiny)])
    assert not r.records


def pin_line_correction(orc):
    """Errors confined to one row (or one column) of a tile, on integer
    data: each element where the flagged line crosses a flagged entry loses
    that entry's residual, the line is confirmed by its own residual, and
    the output equals the fault-free product bit for bit.  More than four
    elements on the line, a checksum fault that joins the line, or a value
    that is not finite (its residual cannot be subtracted) -> recomputed."""
    g = synth.rng(93, 0, 0)
    m, n, k = 32, 32, 24
    A = np.asfortranarray(g.integers(-8, 9, (m, k)).astype(float))
    B = np.asfortranarray(g.integers(-8, 9, (k, n)).astype(float))
    Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
    Cff = 3.0 * (A @ B) + 2.0 * Cin
    run = lambda plan: orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, injections=plan)
    Inj = O.Injection
    # two in row 20 (tile (1, 0)), four in row 5 (tile (0, 1)), three in
    # column 9 (tile (1, 0) is taken: column 9 of tile (0, 0))
    plan = [Inj(20, 2, 3, O.ADD, 100.0), Inj(20, 11, 17, O.ADD, -40.0),
            Inj(5, 16, 0, O.ADD, 7.0), Inj(5, 18, 8, O.ADD, 9.0), Inj(5, 25, 8, O.ADD, -3.0),
            Inj(5, 31, 23, O.ADD, 1.0e6),
            Inj(1, 9, 5, O.ADD, 50.0), Inj(7, 9, 9, O.ADD, 60.0), Inj(14, 9, 20, O.ADD, -70.0)]
    r = run(plan)
    assert np.array_equal(r.C, Cff)
    got = sorted((d["kind"], d["row"], d["col"], d["nbad_rows"], d["nbad_cols"])
                 for d in r.records)
    assert got == [(O.CORRECTED, 1, 9, 3, 1), (O.CORRECTED, 5, 16, 1, 4),
                   (O.CORRECTED, 20, 2, 1, 2)]
    # the record's before / after are those of the first rebuilt element
    d = [d for d in r.records if d["row"] == 20][0]
    assert d["before"] == Cff[20, 2] + 300.0 and d["after"] == Cff[20, 2]
    # a non-finite value among several on a line: computed again (alone on
    # its row and column it is rebuilt, see pin_nonfinite_recovery)
    r = orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, injections=[
        Inj(3, 4, 7, O.ADD, np.inf), Inj(3, 12, 7, O.ADD, 5.0)])
    assert np.array_equal(r.C, Cff) and [d["kind"] for d in r.records] == [O.RECOMPUTED]
    # five on one line: more than a line rebuild takes
    five = [Inj(6, j, 2, O.ADD, 10.0 + j) for j in (0, 3, 6, 9, 12)]
    r = run(five)
    assert [(d["kind"], d["nbad_cols"]) for d in r.records] == [(O.RECOMPUTED, 5)]
    assert np.array_equal(r.C, Cff)
    # a data error and a checksum fault on another column of its row: the
    # rebuilt checksum column does not confirm against the row
    r = run([Inj(6, 3, 2, O.ADD, 10.0), Inj(0, 12, 2, O.ADD, 30.0, target=O.TGT_ROW_CHECKSUM)])
    assert [(d["kind"], d["nbad_rows"], d["nbad_cols"]) for d in r.records] == \
        [(O.RECOMPUTED, 1, 2)]
    assert np.array_equal(r.C, Cff)


def pin_crossing_pairs(orc):
    """Errors in distinct rows and columns of a tile, on integer data: the
    flagged rows and columns are exactly those where the faulty output
    differs from the fault-free product (brute force); each row is paired
    with the column of equal residual, each crossing loses that residual,
    and the output equals the fault-free product bit for bit.  Errors that
    cannot be paired one to one -> recomputed: two equal errors, three
    errors of distinct sizes on the corners of a rectangle, a data error
    beside a fault on each checksum, five errors.  Three on a rectangle's
    corners with the two off the shared corner equal cannot be told from a
    pair, and are corrected as one (the stated limit)."""
    g = synth.rng(94, 0, 0)
    m, n, k = 32, 32, 24
    A = np.asfortranarray(g.integers(-8, 9, (m, k)).astype(float))
    B = np.asfortranarray(g.integers(-8, 9, (k, n)).astype(float))
    Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
    Cff = 3.0 * (A @ B) + 2.0 * Cin
    Inj = O.Injection
    run = lambda plan: orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, injections=plan)
    # two in tile (0, 0), four in tile (1, 1), three in tile (1, 0)
    plan = [Inj(9, 2, 3, O.ADD, 100.0), Inj(4, 11, 17, O.ADD, -40.0),
            Inj(16, 16, 0, O.ADD, 7.0), Inj(20, 30, 8, O.ADD, 9.0), Inj(25, 18, 8, O.ADD, -3.0),
            Inj(31, 25, 23, O.ADD, 1.0e6),
            Inj(17, 1, 5, O.ADD, 50.0), Inj(23, 9, 9, O.ADD, 60.0), Inj(30, 14, 20, O.ADD, -70.0)]
    r = run(plan)
    assert np.array_equal(r.C, Cff)
    for d in r.records:
        i0, j0 = 16 * d["tile_m"], 16 * d["tile_n"]
        bad = np.argwhere(r.raw[i0:i0 + 16, j0:j0 + 16] != Cff[i0:i0 + 16, j0:j0 + 16])
        assert d["nbad_rows"] == len(set(bad[:, 0])) == d["nbad_cols"] == len(set(bad[:, 1]))
    got = sorted((d["kind"], d["row"], d["col"], d["nbad_rows"]) for d in r.records)
    # the record names the first flagged row and the column it was paired with
    assert got == [(O.CORRECTED, 4, 11, 2), (O.CORRECTED, 16, 16, 4), (O.CORRECTED, 17, 1, 3)]
    d = [d for d in r.records if d["row"] == 4][0]
    assert d["before"] == Cff[4, 11] - 120.0 and d["after"] == Cff[4, 11]
    assert d["d_row"] == d["d_col"] == -120.0
    # The limit of one row and one column checksum per tile: three errors
    # on the corners of a rectangle, the two off the shared corner equal,
    # leave the same residuals as two errors in distinct rows and columns
    # (rows 2 and 7: 65 and 40; columns 3 and 12: 65 and 40).  The reading
    # with fewer errors is taken: the pair is corrected, which leaves four
    # wrong elements whose row and column sums all agree.  The record's
    # counts (two rows, two columns) tell a paired correction from a single
    # one.
    r = run([Inj(2, 3, 1, O.ADD, 25.0), Inj(2, 12, 9, O.ADD, 40.0), Inj(7, 3, 9, O.ADD, 40.0)])
    assert [(d["kind"], d["row"], d["col"], d["nbad_rows"], d["nbad_cols"])
            for d in r.records] == [(O.CORRECTED, 2, 3, 2, 2)]
    diff = r.C - Cff
    assert sorted(map(tuple, np.argwhere(diff != 0).tolist())) == [(2, 3), (2, 12), (7, 3), (7, 12)]
    assert not diff.sum(axis=0).any() and not diff.sum(axis=1).any()
    for plan in ([Inj(2, 3, 1, O.ADD, 25.0), Inj(7, 12, 9, O.ADD, 25.0)],
                 [Inj(2, 3, 1, O.ADD, 25.0), Inj(2, 12, 9, O.ADD, 40.0),
                  Inj(7, 3, 9, O.ADD, 55.0)],
                 [Inj(2, 3, 1, O.ADD, 25.0), Inj(7, 12, 9, O.ADD, 40.0, target=O.TGT_ROW_CHECKSUM),
                  Inj(9, 14, 9, O.ADD, 55.0, target=O.TGT_COL_CHECKSUM)],
                 [Inj(i, i + 1, 2, O.ADD, 10.0 * (i + 1)) for i in range(0, 15, 3)]):
        r = run(plan)
        assert [d["kind"] for d in r.records] == [O.RECOMPUTED], plan
        assert np.array_equal(r.C, Cff)


def pin_single_flag_rule(orc):
    """A lone disagreeing checksum entry is taken for a checksum fault only
    when a data error could not have hidden on the other side.  On integer
    data (fault-free residuals exactly zero) with FP32 thresholds, whose two
    sides differ by the operands' norms: a data error larger than its
    column's threshold but within its row's flags one side only; brute
    force shows the output really changed, and the tile is computed again
    (the output equals the fault-free product bit for bit).  A checksum
    fault beyond the entry's threshold plus twice the other side's largest
    is classified checksum-only with the output untouched; a smaller one,
    indistinguishable from a hidden data error, is computed again."""
    g = synth.rng(95, 0, 0)
    m = n = 16
    k = 64
    # rows of A and columns of B with norms spread over two orders of size
    A = g.integers(-8, 9, (m, k)).astype(float) * np.repeat([1.0, 4.0, 16.0, 64.0], 4)[:, None]
    B = g.integers(-8, 9, (k, n)).astype(float) * np.repeat([1.0, 4.0, 16.0, 64.0], 4)[None, :]
    A, B = np.asfortranarray(A), np.asfortranarray(B)
    Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
    Cff = A @ B + Cin
    kw = dict(Cin=Cin, alpha=1.0, beta=1.0, tm=16, tn=16, bk=16, acc_bits=32)
    tr, tc = orc.tile_thresholds(A, B, 0, 0, **kw)
    Inj = O.Injection
    # column 0 has the smallest row-checksum threshold, row 15 the largest
    # column-checksum threshold
    j, i = int(np.argmin(tr)), int(np.argmax(tc))
    assert tc[i] > 4.0 * tr[j]
    delta = 0.5 * (tr[j] + tc[i])          # above tr[j], below tc[i]
    r = orc.ftgemm(A, B, injections=[Inj(i, j, 5, O.ADD, delta)], **kw)
    assert np.argwhere(r.raw != Cff).tolist() == [[i, j]]
    assert [(d["kind"], d["nbad_rows"], d["nbad_cols"], d["col"]) for d in r.records] == \
        [(O.RECOMPUTED, 0, 1, j)]
    assert np.array_equal(r.C, Cff)
    bound_c = tr[j] + 2.0 * tc.max()
    bound_r = tc[i] + 2.0 * tr.max()
    for target, size, bound, kind in (
            (O.TGT_ROW_CHECKSUM, 1.5 * bound_c, bound_c, O.CHECKSUM_ONLY),
            (O.TGT_ROW_CHECKSUM, 0.5 * (tr[j] + bound_c), bound_c, O.RECOMPUTED),
            (O.TGT_COL_CHECKSUM, 1.5 * bound_r, bound_r, O.CHECKSUM_ONLY),
            (O.TGT_COL_CHECKSUM, 0.5 * (tc[i] + bound_r), bound_r, O.RECOMPUTED)):
        r = orc.ftgemm(A, B, injections=[Inj(i, j, 5, O.ADD, size, target=target)], **kw)
        assert [d["kind"] for d in r.records] == [kind], (target, size, bound)
        assert np.array_equal(r.raw, Cff) and np.array_equal(r.C, Cff)


def pin_split_inner_dimension(orc):
    """A split inner dimension: slices of slice_k indices, each verified as a
    tile of its own, then the verified reduction.  On integer data every
    partial sum is exact, so: the split result equals the fault-free
    product bit for bit with no record; two faults of one tile in different
    slices are each located by brute force on the slice partials (the raw
    output differs from the product exactly there) and rebuilt by their
    slice (two CORRECTED records, output exact); a checksum fault in a slice
    is classified checksum-only there and its entry replaced by the
    verified sum, so the reduction agrees (no reduction record); faults
    planned past the end of the inner dimension: an accumulator fault is
    not applied, a checksum fault goes to the last slice."""
    g = synth.rng(96, 0, 0)
    m, n, k = 40, 36, 70
    A = np.asfortranarray(g.integers(-8, 9, (k, m)).astype(float))   # op(A) = A^T
    B = np.asfortranarray(g.integers(-8, 9, (k, n)).astype(float))
    Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
    Cff = 2.0 * (A.T @ B) - 1.0 * Cin
    Inj = O.Injection
    kw = dict(ta=True, tm=16, tn=16, bk=8, slice_k=24)    # slices of 24, 24, 22
    r = orc.ftgemm(A, B, Cin, 2.0, -1.0, **kw)
    assert np.array_equal(r.C, Cff) and not r.records
    # unsplit on random data: the same product within rounding
    Ar, Br, Cr = synth.operands(96, 1, 50, 45, 100, "normal")
    a = orc.ftgemm(Ar, Br, Cr, 1.0, 1.0, tm=16, tn=16, bk=8, slice_k=32)
    b = orc.ftgemm(Ar, Br, Cr, 1.0, 1.0, tm=16, tn=16, bk=8)
    assert np.max(np.abs(a.C - b.C)) < 1e-12 * np.max(np.abs(b.C)) and not a.records
    # two faults in tile (0, 0): k 5 (slice 0) and 50 (slice 2)
    r = orc.ftgemm(A, B, Cin, 2.0, -1.0, injections=[
        Inj(3, 4, 5, O.ADD, 100.0), Inj(9, 12, 50, O.ADD, -30.0)], **kw)
    assert np.argwhere(r.raw != Cff).tolist() == [[3, 4], [9, 12]]
    assert [(d["kind"], d["row"], d["col"], d["tile_m"], d["tile_n"]) for d in r.records] == \
        [(O.CORRECTED, 3, 4, 0, 0), (O.CORRECTED, 9, 12, 0, 0)]
    assert np.array_equal(r.C, Cff)
    assert [d["before"] - d["after"] for d in r.records] == [100.0, -30.0]  # slice partials
    # a row-checksum fault in slice 1 of tile (1, 1), and faults past the end
    r = orc.ftgemm(A, B, Cin, 2.0, -1.0, injections=[
        Inj(20, 21, 30, O.ADD, 500.0, target=O.TGT_ROW_CHECKSUM),
        Inj(33, 2, k + 5, O.ADD, 77.0),
        Inj(35, 30, k + 5, O.ADD, 900.0, target=O.TGT_COL_CHECKSUM)], **kw)
    assert np.array_equal(r.C, Cff)
    assert [(d["kind"], d["row"], d["col"]) for d in r.records] == \
        [(O.CHECKSUM_ONLY, -1, 21), (O.CHECKSUM_ONLY, 35, -1)]
    assert [e["applied"] for e in r.echo] == [True, False, True]


def pin_weighted_checksums(orc):
    """The weighted row checksums of the hand-worked tile
    (tests/golden/threshold_example.txt): encoded values and thresholds from
    norms worked out by hand; and on integer data the weighted identity
    e_w^T (A B) = (e_w^T A) B holds bit for bit in every tile, ragged and
    transposed ones included, its reference side being the weighted column
    sums of the product (numpy)."""
    d = read_threshold_example()
    kw = dict(Cin=d["Cin"], alpha=d["alpha"], beta=d["beta"], tm=4, tn=4, bk=2,
              lam=d["lambda"])
    Pw, tw, Rw = orc.tile_weighted(d["A"], d["B"], 0, 0, **kw)
    assert np.array_equal(Pw, d["weighted_checksums"]) and np.array_equal(Rw, Pw)
    nb = np.array([1.0, 5.0, 7.0, 5.0])
    for acc_bits, u in ((64, 2.0 ** -53), (32, 2.0 ** -24)):
        Pw, tw, Rw = orc.tile_weighted(d["A"], d["B"], 0, 0, acc_bits=acc_bits, **kw)
        want = 8.0 * u * (2.0 * nb * (5.0 * np.sqrt(d["weighted_frob2"]) +
                                      2.0 * np.sqrt(d["weighted_x2"])) +
                          np.sqrt(d["weighted_cin2"]))
        assert np.allclose(tw, want, rtol=1e-14, atol=0), (acc_bits, tw / u, want / u)
    for ta in (False, True):
        for tb in (False, True):
            g = synth.rng(98, int(ta) * 2 + int(tb), 0)
            m, n, k = 21, 18, 40
            A = np.asfortranarray(g.integers(-8, 9, (k, m) if ta else (m, k)).astype(float))
            B = np.asfortranarray(g.integers(-8, 9, (n, k) if tb else (k, n)).astype(float))
            Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
            oa, ob = _ops(A, B, ta, tb)
            Cf = 2.0 * (oa @ ob) - 1.0 * Cin
            for ti in range(-(-m // 8)):
                for tj in range(-(-n // 8)):
                    Pw, tw, Rw = orc.tile_weighted(A, B, ti, tj, Cin, 2.0, -1.0, ta, tb, tm=8,
                                                   tn=8, bk=5)
                    blk = Cf[ti * 8:ti * 8 + 8, tj * 8:tj * 8 + 8]
                    wts = np.arange(1, blk.shape[0] + 1, dtype=float)
                    assert np.array_equal(Rw, wts @ blk), (ta, tb, ti, tj)
                    assert np.array_equal(Pw, Rw), (ta, tb, ti, tj)


def pin_weighted_location(orc):
    """The weighted mode on integer data (residuals exact): every error
    pattern below is set against brute force (where the faulty output
    differs from the fault-free product).  Two equal errors in distinct rows
    and columns, which residual pairing cannot tell apart, are located by the
    ratio of weighted to plain residual and corrected; three errors on the
    corners of a rectangle with the two off-corner ones equal, which pairing
    misreads, and a row whose two errors cancel beside a row with two
    errors, which a line correction misreads, are computed again; errors
    along a column and along a row are corrected and confirmed; a fault on
    the weighted checksum alone changes nothing; a data error plus a fault on
    its column's weighted checksum is computed again; a lone non-finite
    error is still rebuilt."""
    g = synth.rng(99, 0, 0)
    m, n, k = 32, 32, 24
    A = np.asfortranarray(g.integers(-8, 9, (m, k)).astype(float))
    B = np.asfortranarray(g.integers(-8, 9, (k, n)).astype(float))
    Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
    Cff = 3.0 * (A @ B) + 2.0 * Cin
    Inj = O.Injection
    run = lambda plan, wt=True: orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8,
                                           injections=plan, weighted=wt)
    # equal errors: pairing recomputes, the weighted mode corrects
    two = [Inj(2, 3, 1, O.ADD, 25.0), Inj(7, 12, 9, O.ADD, 25.0)]
    r = run(two, False)
    assert [d["kind"] for d in r.records] == [O.RECOMPUTED]
    r = run(two)
    assert np.argwhere(r.raw != Cff).tolist() == [[2, 3], [7, 12]]
    assert [(d["kind"], d["row"], d["col"], d["nbad_rows"]) for d in r.records] == \
        [(O.CORRECTED, 2, 3, 2)]
    assert np.array_equal(r.C, Cff)
    # four equal errors in distinct rows and columns of tile (1, 1)
    four = [Inj(16 + 3 * q, 16 + 5 * q, 2 * q, O.ADD, 40.0) for q in range(4)]
    r = run(four)
    assert [(d["kind"], d["nbad_rows"], d["nbad_cols"]) for d in r.records] == \
        [(O.CORRECTED, 4, 4)]
    assert np.array_equal(r.C, Cff)
    # the rectangle: pairing corrects it wrongly, the weighted mode recomputes
    rect = [Inj(2, 3, 1, O.ADD, 25.0), Inj(2, 12, 9, O.ADD, 40.0), Inj(7, 3, 9, O.ADD, 40.0)]
    assert not np.array_equal(run(rect, False).C, Cff)
    r = run(rect)
    assert [d["kind"] for d in r.records] == [O.RECOMPUTED] and np.array_equal(r.C, Cff)
    # a row with two errors and a row whose two errors cancel: rows 2 and 5
    # of tile (0, 0); only row 2 and columns 3, 9 disagree on the plain sums
    canc = [Inj(2, 3, 1, O.ADD, 10.0), Inj(5, 3, 1, O.ADD, 6.0), Inj(5, 9, 1, O.ADD, -6.0),
            Inj(2, 9, 4, O.ADD, 7.0)]
    r = run(canc, False)
    assert [d["kind"] for d in r.records] == [O.CORRECTED] and not np.array_equal(r.C, Cff)
    r = run(canc)
    assert [d["kind"] for d in r.records] == [O.RECOMPUTED] and np.array_equal(r.C, Cff)
    # lines: three errors in column 9 (tile (0, 0)), two in row 20 (tile (1, 0))
    lines = [Inj(1, 9, 5, O.ADD, 50.0), Inj(7, 9, 9, O.ADD, 60.0), Inj(14, 9, 20, O.ADD, -70.0),
             Inj(20, 2, 3, O.ADD, 100.0), Inj(20, 11, 17, O.ADD, -40.0)]
    r = run(lines)
    assert sorted((d["kind"], d["row"], d["col"]) for d in r.records) == \
        [(O.CORRECTED, 1, 9), (O.CORRECTED, 20, 2)]
    assert np.array_equal(r.C, Cff)
    # checksum faults on the weighted entries
    r = run([Inj(4, 6, 0, O.ADD, 500.0, target=O.TGT_WEIGHTED_CHECKSUM)])
    assert not r.records and r.echo[0]["applied"] and np.array_equal(r.C, Cff)
    r = run([Inj(4, 6, 3, O.ADD, 30.0), Inj(0, 6, 0, O.ADD, 90.0, target=O.TGT_WEIGHTED_CHECKSUM)])
    assert [d["kind"] for d in r.records] == [O.RECOMPUTED] and np.array_equal(r.C, Cff)
    # a lone infinite error is rebuilt as in the plain mode
    r = run([Inj(9, 10, 4, O.ADD, np.inf)])
    assert [d["kind"] for d in r.records] == [O.CORRECTED] and np.array_equal(r.C, Cff)


def pin_one_sided(orc):
    """One-sided mode (only the column checksum, one entry per row;
    recompute on any disagreement).  On integer data: each accumulator fault
    flags exactly the row where the faulty output differs from the
    fault-free product (brute force), with residual alpha * delta; the tile
    is computed again and the output equals the fault-free product bit for
    bit.  A fault on the column checksum of a row flags that row; one on
    the row checksum has no entry to land on.  Fault-free: nothing flagged."""
    g = synth.rng(92, 0, 0)
    m, n, k = 37, 34, 40
    A = np.asfortranarray(g.integers(-8, 9, (m, k)).astype(float))
    B = np.asfortranarray(g.integers(-8, 9, (k, n)).astype(float))
    Cin = np.asfortranarray(g.integers(-8, 9, (m, n)).astype(float))
    Cff = 3.0 * (A @ B) + 2.0 * Cin
    r = orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, one_sided=True)
    assert np.array_equal(r.C, Cff) and not r.records
    plan = [O.Injection(3, 4, 5, O.ADD, 1000.0),      # tile (0, 0)
            O.Injection(20, 17, 39, O.ADD, -77.0),    # tile (1, 1), last step
            O.Injection(36, 33, 0, O.ADD, 5.0)]       # corner tile (2, 2)
    r = orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, injections=plan, one_sided=True)
    assert np.array_equal(r.C, Cff)
    rows = np.unique(np.argwhere(r.raw != Cff)[:, 0]).tolist()
    assert rows == [3, 20, 36]
    assert sorted(d["row"] for d in r.records) == rows
    for d in r.records:
        assert d["kind"] == O.RECOMPUTED and d["col"] == -1
        assert d["nbad_rows"] == 1 and d["nbad_cols"] == 0
        assert d["d_row"] == 0.0 and d["tau_row"] == 0.0
        assert d["d_col"] == 3.0 * {3: 1000.0, 20: -77.0, 36: 5.0}[d["row"]]
    # two faults in different rows of one tile: both rows flagged, one record
    r = orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, one_sided=True, injections=[
        O.Injection(17, 1, 3, O.ADD, 9.0), O.Injection(30, 12, 30, O.ADD, 4.0)])
    assert [(d["kind"], d["row"], d["nbad_rows"]) for d in r.records] == [(O.RECOMPUTED, 17, 2)]
    assert np.array_equal(r.C, Cff)
    # checksum targets: the column checksum of row 20 is an entry, the row
    # checksum of column 21 is not
    r = orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, one_sided=True, injections=[
        O.Injection(20, 21, 10, O.ADD, 50.0, target=O.TGT_COL_CHECKSUM),
        O.Injection(5, 6, 10, O.ADD, 50.0, target=O.TGT_ROW_CHECKSUM)])
    assert [(d["kind"], d["row"], d["d_col"]) for d in r.records] == [(O.RECOMPUTED, 20, -50.0)]
    assert r.echo[0]["applied"] and not r.echo[1]["applied"]
    assert np.array_equal(r.C, Cff)
    # the two-sided mode on the same faults corrects instead
    r = orc.ftgemm(A, B, Cin, 3.0, 2.0, tm=16, tn=16, bk=8, injections=plan)
    assert all(d["kind"] == O.CORRECTED for d in r.records) and np.array_equal(r.C, Cff)


def pin_no_false_positives(orc):
    """Fault-free runs flag nothing, for both accumulator precisions, and the
    largest residual stays well inside its threshold."""
    for dist, seed in (("uniform", 0), ("normal", 1)):
        A, B, Cin = synth.operands(92, seed, 70, 66, 300, dist)
        for acc in (64, 32):
            r = orc.ftgemm(A, B, Cin, 1.0, 1.0, tm=32, tn=32, bk=16, acc_bits=acc)
            assert not r.records
            assert r.max_ratio < 0.1, r.max_ratio


def pin_ragged_and_subset(orc):
    """Ragged edge tiles, k not a multiple of the step, a subset of tiles."""
    A, B, Cin = synth.operands(93, 0, 45, 39, 29, "uniform")
    Cff = 0.5 * (A @ B) - 2.0 * Cin
    plan = [O.Injection(44, 38, 28, O.ADD, 9.0)]
    r = orc.ftgemm(A, B, Cin, 0.5, -2.0, tm=16, tn=16, bk=8, injections=plan)
    assert np.max(np.abs(r.C - Cff)) < 1e-13
    assert [(d["row"], d["col"], d["kind"]) for d in r.records] == [(44, 38, O.CORRECTED)]
    tiles_m = 3
    sub = [2 + 2 * tiles_m]  # tile (2, 2): the bottom-right ragged tile
    r = orc.ftgemm(A, B, Cin, 0.5, -2.0, tm=16, tn=16, bk=8, injections=plan, tiles=sub)
    assert np.max(np.abs(r.C[32:, 32:] - Cff[32:, 32:])) < 1e-13
    assert np.all(np.isnan(r.C[:32, :]))
    assert len(r.records) == 1


def pin_threshold_worked_example(orc):
    """The threshold of every checksum entry of a 4 x 4 tile equals the
    value worked out by hand in tests/golden/threshold_example.txt, for FP64
    and FP32 accumulation and for a multiplier that truncates its products
    (each term of the bound has its own factor there, so dropping or
    mis-scaling any one of them changes the values)."""
    d = read_threshold_example()
    kw = dict(Cin=d["Cin"], alpha=d["alpha"], beta=d["beta"], tm=4, tn=4, bk=2,
              lam=d["lambda"])
    for acc_bits, u in ((64, 2.0 ** -53), (32, 2.0 ** -24)):
        tr, tc = orc.tile_thresholds(d["A"], d["B"], 0, 0, acc_bits=acc_bits, **kw)
        assert np.allclose(tr, d["tau_row_u"] * u, rtol=1e-15, atol=0), (acc_bits, tr / u)
        assert np.allclose(tc, d["tau_col_u"] * u, rtol=1e-15, atol=0), (acc_bits, tc / u)
    g = 2.0 ** d["mma_grid_log2"]
    tr, tc = orc.tile_thresholds(d["A"], d["B"], 0, 0, acc_bits=32,
                                 mma=(g, int(d["mma_group"])), **kw)
    u = 2.0 ** -24
    assert np.allclose(tr, d["tau_row_u"] * u + d["tau_row_mma_64ths"] / 64.0, rtol=1e-15,
                       atol=0)
    assert np.allclose(tc, d["tau_col_u"] * u + d["tau_col_mma_64ths"] / 64.0, rtol=1e-15,
                       atol=0)


def _bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64:
    products of two such values are exact in FP32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _fp32_tile_residuals(A, B, Cin, alpha, beta):
    """Residuals R - P of one tile computed the way an FP32-accumulating
    kernel forms them, written out here independently of the oracle: the
    product accumulated step by step in FP32, the operand checksums x and y
    summed in FP32, the encoded products x.B and A.y accumulated in FP32,
    the beta part and the reference sums in FP64."""
    h, k = A.shape
    w = B.shape[1]
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    acc = np.zeros((h, w), np.float32)
    for p in range(k):
        acc = (acc + np.outer(A32[:, p], B32[p, :])).astype(np.float32)
    out = (np.float32(alpha) * acc + np.float32(beta) * Cin.astype(np.float32))
    out = out.astype(np.float32).astype(np.float64)
    x = np.zeros(k, np.float32)
    y = np.zeros(k, np.float32)
    for i in range(h):
        x = (x + A32[i, :]).astype(np.float32)
    for j in range(w):
        y = (y + B32[:, j]).astype(np.float32)
    Pr = np.zeros(w, np.float32)
    Pc = np.zeros(h, np.float32)
    for p in range(k):
        Pr = (Pr + x[p] * B32[p, :]).astype(np.float32)
        Pc = (Pc + A32[:, p] * y[p]).astype(np.float32)
    dr = out.sum(axis=0) - (alpha * Pr.astype(np.float64) + beta * Cin.sum(axis=0))
    dc = out.sum(axis=1) - (alpha * Pc.astype(np.float64) + beta * Cin.sum(axis=1))
    return dr, dc


def pin_threshold_sound_and_tight(orc):
    """The threshold bounds real rounding and is not absurdly loose.  The
    test forms each tile's residuals with its own FP32 accumulation (and the
    FP64 ones with numpy's matmul, a different summation order from the
    oracle's); over several seeds and inner dimensions the largest |d|/tau
    must lie in [1e-4, 1).  Same-sign data (partial sums that only grow)
    push the FP32 residual to about 5% of tau at every k, so a threshold
    missing its sqrt(k) growth or using the FP64 unit roundoff for FP32
    accumulation fails; mean-zero data keep it near 1e-3, so a threshold
    a hundred times too large fails too."""
    h = w = 32
    for dist in ("normal", "positive"):
        for k in (256, 4096):
            worst = 0.0
            for seed in range(3):
                g = np.random.default_rng([97, seed, k])
                if dist == "normal":
                    A = _bf16(g.standard_normal((h, k)))
                    B = _bf16(g.standard_normal((k, w)))
                else:
                    A = _bf16(g.uniform(0.0, 1.0, (h, k)))
                    B = _bf16(g.uniform(0.0, 1.0, (k, w)))
                Cin = _bf16(g.standard_normal((h, w)))
                A, B, Cin = (np.asfortranarray(v) for v in (A, B, Cin))
                dr, dc = _fp32_tile_residuals(A, B, Cin, 1.0, 1.0)
                tr, tc = orc.tile_thresholds(A, B, 0, 0, Cin, 1.0, 1.0, tm=h, tn=w, bk=16,
                                             acc_bits=32)
                worst = max(worst, np.max(np.abs(dr) / tr), np.max(np.abs(dc) / tc))
            assert 1e-4 <= worst < 1.0, ("fp32", dist, k, worst)
    # FP64 accumulation: numpy's matmul (blocked, FMA) against the oracle's
    # thresholds; the residuals are pure rounding and stay far inside tau
    for seed in range(3):
        A, B, Cin = synth.operands(97, seed, 48, 40, 2048, "uniform")
        C = A @ B + Cin
        x, y = A.sum(axis=0), B.sum(axis=1)
        dr = C.sum(axis=0) - (x @ B + Cin.sum(axis=0))
        dc = C.sum(axis=1) - (A @ y + Cin.sum(axis=1))
        tr, tc = orc.tile_thresholds(A, B, 0, 0, Cin, 1.0, 1.0, tm=48, tn=40, bk=16)
        worst = max(np.max(np.abs(dr) / tr), np.max(np.abs(dc) / tc))
        assert 1e-5 <= worst < 1.0, ("fp64", seed, worst)


def pin_gemm_entries_vs_numpy(orc):
    """Single entries of the plain GEMM (used to check large runs on
    sampled outputs) equal numpy's matmul, for every transpose, with padded
    leading dimensions, beta = 0 with NaN in C_in, and a prefix of k."""
    g = np.random.default_rng(17)
    m, n, k = 41, 35, 57
    for ta in (False, True):
        for tb in (False, True):
            sa = (k, m) if ta else (m, k)
            sb = (n, k) if tb else (k, n)
            A = np.asfortranarray(g.uniform(-1, 1, (sa[0] + 3, sa[1])))[:sa[0]]
            B = np.asfortranarray(g.uniform(-1, 1, (sb[0] + 2, sb[1])))[:sb[0]]
            Cin = np.asfortranarray(g.uniform(-1, 1, (m + 4, n)))[:m]
            rows = g.integers(0, m, 50)
            cols = g.integers(0, n, 50)
            oa, ob = _ops(A, B, ta, tb)
            got = orc.gemm_entries(A, B, rows, cols, Cin, -1.5, 0.25, ta, tb)
            ref = (-1.5 * (oa @ ob) + 0.25 * Cin)[rows, cols]
            assert np.max(np.abs(got - ref)) < 1e-13, (ta, tb)
            nanC = np.full((m, n), np.nan, order="F")
            got = orc.gemm_entries(A, B, rows, cols, nanC, 2.0, 0.0, ta, tb)
            assert np.max(np.abs(got - 2.0 * (oa @ ob)[rows, cols])) < 1e-13
            got = orc.gemm_entries(A, B, rows, cols, None, 1.0, 0.0, ta, tb, k=20)
            ref = (oa[:, :20] @ ob[:20, :])[rows, cols]
            assert np.max(np.abs(got - ref)) < 1e-13


ALL_PINS = [pin_gemm_vs_numpy, pin_gemm_integer_exact, pin_blas_special_cases,
            pin_checksum_identities, pin_brute_force_location, pin_exact_recovery,
            pin_nonfinite_recovery, pin_classification, pin_line_correction,
            pin_crossing_pairs, pin_one_sided,
            pin_no_false_positives, pin_ragged_and_subset, pin_threshold_sound_and_tight,
            pin_threshold_worked_example, pin_gemm_entries_vs_numpy,
            pin_single_flag_rule, pin_split_inner_dimension, pin_weighted_checksums,
            pin_weighted_location]
