"""Batched fault-tolerant GEMM (one persistent launch replayed from a HIP
graph, work order and low-precision tile rows picked by the library's
autotuner) against the CPU oracle, problem by problem, and against the loop
of per-problem launches.

Each problem has its own checksums, report and faults (the plan's `problem`
field is the index in the batch).  Tolerances as for single calls: 1e-12
normwise for FP64, 1e-5 for BF16.  The batched and the per-problem paths run
the same tile code, so their outputs must be bitwise equal.  The oracle
takes each problem's tile rows from ftgemm_batch_tiling; tests that compare
with single launches (whose tiles follow the single-call rule) keep every
problem on 128-row tiles through the tuning table."""
import contextlib
import os
import tempfile

import numpy as np
import pytest

from gpu_util import flagged, lp_mma, normwise, rebuild_bound, say, to_oracle
from oracle import oracle as O
from paper_2305_02444_amd import ftgemm as F
from paper_2305_02444_amd import synth

pytestmark = pytest.mark.gpu
TOL = {F.F64: 1e-12, F.BF16: 1e-5}


def _problem(wid, p, m, n, k, dtype, dist="uniform"):
    A, B, Cin = synth.operands(wid, p, m, n, k, dist)
    if dtype == F.F64:
        return A, B, Cin, A, B
    orc = O.default()
    ca, cb = synth.to_bf16_bits(A), synth.to_bf16_bits(B)
    return ca, cb, np.asfortranarray(Cin.astype(np.float32).astype(np.float64)), \
        np.asfortranarray(orc.decode_bf16(ca)), np.asfortranarray(orc.decode_bf16(cb))


def _device(x, dtype):
    import torch
    if dtype == F.F64:
        return F.to_device(x)
    return F.to_device(x.view(np.int16)).view(torch.bfloat16)


def _batch(shapes, dtype, wid, alpha=1.0, beta=0.0):
    """Host problems, device tensors and descriptors of a batch."""
    import torch
    host, dev, descs = [], [], []
    for p, (m, n, k) in enumerate(shapes):
        A, B, Cin, dA, dB = _problem(wid, p, m, n, k, dtype)
        tA, tB = _device(A, dtype), _device(B, dtype)
        tC = F.to_device(Cin, dtype=torch.float64 if dtype == F.F64 else torch.float32)
        host.append((dA, dB, Cin))
        dev.append((tA, tB, tC))
        descs.append(F.make_desc(tA, tB, tC, alpha, beta, dtype=dtype))
    return host, dev, descs


@contextlib.contextmanager
def _table(text):
    """A tuning table with these lines for the duration (then an empty one)."""
    fd, path = tempfile.mkstemp(suffix=".tune")
    with os.fdopen(fd, "w") as fh:
        fh.write(text)
    try:
        F.load_tune_table(path)
        yield path
    finally:
        F.load_tune_table(None)
        os.unlink(path)


NO_BIG_TILES = "batch_mstar 1000000000\n"


def _plan(shapes, wid, dtype, lo_exp, rows=None):
    """Truncated Poisson(1) faults per problem (at most 3, one per tile of
    rows[p] x 128), additive, 10^U(lo, 6) times the typical |C|."""
    g = synth.rng(wid, 0, synth.STREAM_PLAN)
    plan = []
    for p, (m, n, k) in enumerate(shapes):
        tm = rows[p] if rows else 128
        tiles = (-(-m // tm)) * (-(-n // 128))
        cnt = min(synth.truncated_poisson(g, 1.0, 3), tiles if k > 0 else 0)
        sigma = np.sqrt(k / 9.0)
        for f in synth.additive_plan(g, m, n, k, tm, 128, cnt,
                                     synth.log_magnitude(sigma, lo_exp, 6.0)):
            f.problem = p
            plan.append(f)
    return plan


def _outputs(dev, dtype):
    import torch
    torch.cuda.synchronize()
    return [np.asfortranarray(t[2].cpu().numpy().astype(np.float64)) for t in dev]


def _check_problem(p, got, host, shapes, plan, rep, dtype, alpha, beta, tiles=None, tm=128):
    dA, dB, Cin = host[p]
    m, n, k = shapes[p]
    pp = [f for f in plan if f.problem == p]
    ref = O.default().ftgemm(dA, dB, Cin, alpha, beta, tm=tm, tn=128,
                             bk=F.query_tiling(dtype, m, n, k)[2],
                             acc_bits=64 if dtype == F.F64 else 32, injections=to_oracle(pp),
                             tiles=tiles, mma=lp_mma(dtype))
    mask = ~np.isnan(ref.C)
    if dtype != F.F64:
        # rebuilt elements: held to the rounding bound of a rebuild
        corrected = {(r["tile_m"], r["tile_n"]) for r in rep.records
                     if r["kind"] == F.KIND_CORRECTED}
        for i, j in np.argwhere(mask & (ref.raw != ref.C)):
            if (i // tm, j // 128) in corrected:
                assert abs(got[i, j] - ref.C[i, j]) <= \
                    rebuild_bound(dA, dB, False, False, alpha, tm, 128, got, ref.C, i, j)
                mask[i, j] = False
    assert normwise(got[mask], ref.C[mask]) <= TOL[dtype], p
    recs = rep.records
    if tiles is not None:
        tm_ = -(-m // tm)
        keep = set(int(t) for t in tiles)
        recs = [r for r in recs if r["tile_m"] + r["tile_n"] * tm_ in keep]
    assert flagged(recs) == flagged(ref.records), p


@pytest.mark.parametrize("dtype", [pytest.param(F.F64, id="f64"), pytest.param(F.BF16, id="bf16")])
def test_small_batch_matches_oracle_and_loop(dtype):
    g = synth.rng(60, dtype, 7)
    shapes = [(int(g.integers(1, 300)), int(g.integers(1, 300)), int(g.integers(1, 400)))
              for _ in range(40)]
    shapes[3] = (0, 50, 10)        # empty
    shapes[7] = (60, 70, 0)        # k == 0: C <- beta C (beta 0 here: zeros)
    plan = _plan(shapes, 60, dtype, 1.0)
    say("batch of %d, %d faults" % (len(shapes), len(plan)))
    host, dev, descs = _batch(shapes, dtype, 60)
    F.set_fault_plan(plan)
    reps = [F.ReportBuffer() for _ in shapes]
    with _table(NO_BIG_TILES):
        assert F.batch_tiling(descs) == [128] * len(shapes)
        F.gemm_batched(descs, reps)
    got = _outputs(dev, dtype)
    views = [r.view() for r in reps]
    for p in range(len(shapes)):
        if shapes[p][0] and shapes[p][1]:
            _check_problem(p, got[p], host, shapes, plan, views[p], dtype, 1.0, 0.0)
    assert sum(v.corrected for v in views) == len(plan)
    # the same problems, one launch each
    host2, dev2, descs2 = _batch(shapes, dtype, 60)
    reps2 = [F.ReportBuffer() for _ in shapes]
    F.gemm_batched(descs2, reps2, loop=True)
    got2 = _outputs(dev2, dtype)
    F.clear_fault_plan()
    for p in range(len(shapes)):
        assert np.array_equal(got[p], got2[p]), p
        assert flagged(reps2[p].view().records) == flagged(views[p].records)


@pytest.mark.parametrize("dtype", [pytest.param(F.F64, id="f64"), pytest.param(F.BF16, id="bf16")])
def test_batch_several_errors_per_tile(dtype):
    """The persistent kernel's tiles correct what single calls correct:
    errors in distinct rows and columns paired by residual, errors along
    one row, and send two equal errors to a recompute; flagged sets as the
    oracle's, outputs bitwise equal to the loop of single launches.
    Rebuilt low-precision elements are held to their tile's thresholds."""
    shapes = [(200, 300, 150), (128, 128, 64), (300, 200, 257)]
    Fa = synth.Fault
    plan = [Fa(5, 7, 3, synth.ADD, 30.0), Fa(40, 90, 100, synth.ADD, -70.0),        # (0,0) pair
            Fa(150, 130, 7, synth.ADD, 20.0), Fa(150, 200, 140, synth.ADD, 45.0),    # (1,1) line
            Fa(3, 9, 0, synth.ADD, 11.0), Fa(60, 20, 30, synth.ADD, -17.0),          # three pairs
            Fa(100, 127, 63, synth.ADD, 23.0),
            Fa(130, 140, 5, synth.ADD, 50.0), Fa(170, 190, 200, synth.ADD, 50.0)]    # equal
    for f, p in zip(plan, [0, 0, 0, 0, 1, 1, 1, 2, 2]):
        f.problem = p
    say("batch of %d, %d faults (pairs, line, equal)" % (len(shapes), len(plan)))
    host, dev, descs = _batch(shapes, dtype, 65, alpha=1.0, beta=0.0)
    F.set_fault_plan(plan)
    reps = [F.ReportBuffer() for _ in shapes]
    with _table(NO_BIG_TILES):
        F.gemm_batched(descs, reps)
    got = _outputs(dev, dtype)
    host2, dev2, descs2 = _batch(shapes, dtype, 65, alpha=1.0, beta=0.0)
    F.gemm_batched(descs2, [F.ReportBuffer() for _ in shapes], loop=True)
    got2 = _outputs(dev2, dtype)
    F.clear_fault_plan()
    kinds = []
    for p, (m, n, k) in enumerate(shapes):
        assert np.array_equal(got[p], got2[p]), p
        dA, dB, Cin = host[p]
        ref = O.default().ftgemm(dA, dB, Cin, 1.0, 0.0, tm=128, tn=128,
                                 bk=F.query_tiling(dtype, m, n, k)[2],
                                 acc_bits=64 if dtype == F.F64 else 32,
                                 injections=to_oracle([f for f in plan if f.problem == p]),
                                 mma=lp_mma(dtype))
        recs = reps[p].view().records
        assert flagged(recs) == flagged(ref.records), p
        kinds += sorted((p, r["kind"], r["nbad_rows"], r["nbad_cols"]) for r in recs)
        mask = np.ones(got[p].shape, dtype=bool)
        if dtype != F.F64:
            corrected = {(r["tile_m"], r["tile_n"]) for r in recs
                         if r["kind"] == F.KIND_CORRECTED}
            for i, j in np.argwhere(ref.raw != ref.C):
                if (i // 128, j // 128) in corrected:
                    assert abs(got[p][i, j] - ref.C[i, j]) <= \
                        rebuild_bound(dA, dB, False, False, 1.0, 128, 128, got[p], ref.C, i, j)
                    mask[i, j] = False
        assert normwise(got[p][mask], ref.C[mask]) <= TOL[dtype], p
    assert kinds == [(0, F.KIND_CORRECTED, 1, 2), (0, F.KIND_CORRECTED, 2, 2),
                     (1, F.KIND_CORRECTED, 3, 3), (2, F.KIND_RECOMPUTED, 2, 2)]


def test_graph_replay_new_data_and_beta():
    """Same shapes twice (the captured graph and the tuned schedule are
    reused) with different data; then beta != 0 (no tuning: C is read)."""
    shapes = [(130, 250, 64), (64, 64, 300), (257, 129, 33), (128, 128, 128)] * 3
    for wid in (61, 62):
        host, dev, descs = _batch(shapes, F.F64, wid)
        reps = [F.ReportBuffer() for _ in shapes]
        F.gemm_batched(descs, reps)
        got = _outputs(dev, F.F64)
        for p in range(len(shapes)):
            _check_problem(p, got[p], host, shapes, [], reps[p].view(), F.F64, 1.0, 0.0)
    host, dev, descs = _batch(shapes, F.F64, 63, alpha=-0.5, beta=2.0)
    reps = [F.ReportBuffer() for _ in shapes]
    F.gemm_batched(descs, reps)
    got = _outputs(dev, F.F64)
    for p in range(len(shapes)):
        _check_problem(p, got[p], host, shapes, [], reps[p].view(), F.F64, -0.5, 2.0)


def test_batch_argument_errors():
    import torch
    host, dev, descs = _batch([(10, 10, 10), (20, 20, 20)], F.F64, 64)
    bad = F.make_desc(dev[0][0], dev[0][1], dev[0][2], 1.0, 0.0)
    bad.lda = 1
    with pytest.raises(F.FTGemmError) as e:
        F.gemm_batched([descs[0], bad])
    assert F.lib().ftgemm_last_invalid_arg() == 8
    x = F.colmajor_empty(10, 10, torch.bfloat16).zero_()
    y = F.colmajor_empty(10, 10, torch.float32).zero_()
    other = F.make_desc(x, x, y, 1.0, 0.0, dtype=F.BF16)
    with pytest.raises(F.FTGemmError):
        F.gemm_batched([descs[0], other])


@pytest.mark.parametrize("dtype", [pytest.param(F.F64, id="f64"), pytest.param(F.BF16, id="bf16")])
def test_c5_512_problems(dtype):
    """512 problems, m, n, k log-uniform in [64, 2048], U[-1,1], alpha = 1,
    beta = 0, truncated Poisson(1) faults per problem.  Every fault located
    and rebuilt in its own problem; the oracle checks every faulty tile and
    a sample of whole problems."""
    shapes = synth.batched_shapes(70, dtype, 512)
    host, dev, descs = _batch(shapes, dtype, 70)
    # the first call tunes the work order and (BF16) the tile rows; the
    # faults are then placed one per tile of each problem's chosen tiles
    F.clear_fault_plan()
    F.gemm_batched(descs)
    rows = F.batch_tiling(descs)
    assert set(rows) <= {128, 256} and (dtype != F.F64 or set(rows) == {128})
    say("tile rows chosen: %d of 512 problems on 256-row tiles" % rows.count(256))
    plan = _plan(shapes, 70 + dtype, dtype, 1.0, rows)
    F.set_fault_plan(plan)
    reps = [F.ReportBuffer() for _ in shapes]
    F.gemm_batched(descs, reps)
    got = _outputs(dev, dtype)
    F.clear_fault_plan()
    views = [r.view() for r in reps]
    for p, v in enumerate(views):
        want = sorted((f.row, f.col) for f in plan if f.problem == p)
        assert sorted((r["row"], r["col"]) for r in v.records) == want, p
        assert v.corrected == len(want) and v.detected == len(want), p
    small = sorted(range(512), key=lambda p: shapes[p][0] * shapes[p][1] * shapes[p][2])[:6]
    for p in small:
        _check_problem(p, got[p], host, shapes, plan, views[p], dtype, 1.0, 0.0, tm=rows[p])
    faulty = sorted({f.problem for f in plan})
    # every faulty problem on 256-row tiles (up to 6), then others, up to 12
    faulty = ([p for p in faulty if rows[p] == 256][:6] +
              [p for p in faulty if rows[p] == 128])[:12]
    for p in faulty:
        m, n, k = shapes[p]
        tm_ = -(-m // rows[p])
        tiles = sorted({(f.row // rows[p]) + (f.col // 128) * tm_ for f in plan
                        if f.problem == p})
        _check_problem(p, got[p], host, shapes, plan, views[p], dtype, 1.0, 0.0, tiles=tiles,
                       tm=rows[p])


def test_batch_tile_rows_per_problem():
    """BF16 problems of at least 256 rows on 256-row tiles and the others on
    128-row tiles, in one persistent launch (the table fixes the threshold):
    ragged shapes, faults one per tile of each problem's tiles, every
    problem checked against the oracle on its own tiles; the checksum-free
    batch writes the same bits."""
    dtype = F.BF16
    shapes = [(300, 200, 150), (255, 130, 64), (256, 128, 64), (600, 300, 333), (100, 500, 70),
              (513, 129, 257)]
    host, dev, descs = _batch(shapes, dtype, 66)
    with _table("batch_mstar 256\n"):
        rows = F.batch_tiling(descs)
        assert rows == [256, 128, 256, 256, 128, 256]
        plan = _plan(shapes, 66, dtype, 1.0, rows)
        F.set_fault_plan(plan)
        reps = [F.ReportBuffer() for _ in shapes]
        F.gemm_batched(descs, reps)
        got = _outputs(dev, dtype)
        F.clear_fault_plan()
        views = [r.view() for r in reps]
        for p in range(len(shapes)):
            _check_problem(p, got[p], host, shapes, plan, views[p], dtype, 1.0, 0.0, tm=rows[p])
        assert sum(v.corrected for v in views) == len(plan) > 0
        plain = [F.make_desc(t[0], t[1], t[2], 1.0, 0.0, abft=False, dtype=dtype) for t in dev]
        F.gemm_batched(plain)
        got2 = _outputs(dev, dtype)
    for p in range(len(shapes)):
        clean = np.ones(got[p].shape, dtype=bool)
        for r in views[p].records:
            clean[r["row"], r["col"]] = False
        assert np.array_equal(got[p][clean], got2[p][clean]), p
