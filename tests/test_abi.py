"""The C ABI without a GPU: the library loads, exports every function the
header declares, and rejects bad arguments on the host (before any HIP
call) with the BLAS position of the culprit."""
import ctypes as C

import pytest

from paper_2305_02444_amd import ftgemm as F


def test_exports_every_declared_function():
    names = F.exported_functions_in_header()
    assert "ftgemm_gemm" in names and "ftgemm_gemm_batched" in names
    L = F.lib()
    for name in names:
        assert hasattr(L, name), name


def _gemm(**kw):
    a = dict(ta=0, tb=0, m=4, n=4, k=4, alpha=1.0, A=1, lda=4, B=1, ldb=4, beta=0.0, Cp=1,
             ldc=4)
    a.update(kw)
    L = F.lib()
    st = L.ftgemm_gemm(a["ta"], a["tb"], a["m"], a["n"], a["k"], a["alpha"], a["A"], a["lda"],
                       a["B"], a["ldb"], a["beta"], a["Cp"], a["ldc"], None, None)
    return st, L.ftgemm_last_invalid_arg()


@pytest.mark.parametrize("kw,pos", [
    (dict(ta=2), 1), (dict(tb=-1), 2), (dict(m=-1), 3), (dict(n=-5), 4), (dict(k=-1), 5),
    (dict(alpha=float("nan")), 6), (dict(A=None), 7), (dict(lda=3), 8),
    (dict(ta=1, lda=3), 8), (dict(B=None), 9), (dict(ldb=3), 10), (dict(tb=1, ldb=3), 10),
    (dict(beta=float("inf")), 11), (dict(Cp=None), 12), (dict(ldc=3), 13),
])
def test_invalid_argument_positions(kw, pos):
    st, p = _gemm(**kw)
    assert st == F.ERR_INVALID_ARG and p == pos


def test_quick_returns_touch_nothing():
    # m == 0 / n == 0: nothing to do, null pointers are fine
    assert _gemm(m=0, A=None, B=None, Cp=None, lda=4, ldc=1) == (F.OK, 0)
    assert _gemm(n=0, A=None, B=None, Cp=None) == (F.OK, 0)
    # alpha == 0 and beta == 1, or k == 0 and beta == 1: C unchanged
    assert _gemm(alpha=0.0, beta=1.0, A=None, B=None) == (F.OK, 0)
    assert _gemm(k=0, beta=1.0, A=None, B=None) == (F.OK, 0)


def test_gemm_ex_descriptor_checks():
    L = F.lib()
    assert L.ftgemm_gemm_ex(None, None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 14
    d = F.GemmDesc()
    d.dtype, d.m, d.n, d.k, d.lda, d.ldb, d.ldc = 7, 4, 4, 4, 4, 4, 4
    d.alpha, d.A, d.B, d.C = 1.0, 1, 1, 1
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 14
    d.dtype, d.scaleA, d.scaleB = F.FP8_E4M3, 0.0, 1.0
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG


def test_abft_modes_checked_on_the_host():
    """abft outside 0..4 is an argument error; the one-sided mode (2) is
    refused for FP64, the unfused (3) and weighted (4) modes for BF16 and
    FP8, and all three in batches, before anything runs."""
    L = F.lib()
    d = F.GemmDesc()
    d.dtype, d.m, d.n, d.k, d.lda, d.ldb, d.ldc = F.BF16, 4, 4, 4, 4, 4, 4
    d.alpha, d.scaleA, d.scaleB, d.A, d.B, d.C = 1.0, 1.0, 1.0, 1, 1, 1
    for bad in (-1, 5, 7):
        d.abft = bad
        assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
        assert L.ftgemm_last_invalid_arg() == 14
    d.dtype, d.abft = F.F64, 2
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_UNSUPPORTED
    d.dtype = F.BF16
    assert L.ftgemm_gemm_batched(1, C.byref(d), None, None) == F.ERR_UNSUPPORTED
    d.abft = 3
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_UNSUPPORTED
    d.dtype = F.F64
    assert L.ftgemm_gemm_batched(1, C.byref(d), None, None) == F.ERR_UNSUPPORTED
    d.abft = 4
    assert L.ftgemm_gemm_batched(1, C.byref(d), None, None) == F.ERR_UNSUPPORTED
    d.dtype = F.BF16
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_UNSUPPORTED
    d.dtype = F.FP8_E4M3
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_UNSUPPORTED


def test_query_tiling_ex():
    """The tiling of the call a descriptor describes: the one-sided mode
    also gives FP8 256-row tiles; modes 0 and 1 agree with
    ftgemm_query_tiling where it speaks for them."""
    for dt in (F.F64, F.BF16, F.FP8_E4M3):
        for shape in ((8192, 8192, 8192), (1000, 1000, 300), (1024, 1024, 32768)):
            assert F.query_tiling_ex(dt, *shape, abft=1) == F.query_tiling(dt, *shape)
    assert F.query_tiling_ex(F.FP8_E4M3, 8192, 8192, 8192, abft=2) == (256, 128, 128, 1)
    assert F.query_tiling_ex(F.FP8_E4M3, 8192, 8192, 8192, abft=0) == (256, 128, 128, 1)
    assert F.query_tiling_ex(F.BF16, 8192, 8192, 8192, abft=2) == (256, 128, 64, 1)
    assert F.query_tiling_ex(F.FP8_E4M3, 1000, 1000, 300, abft=2) == (128, 128, 128, 1)
    L = F.lib()
    v = [C.c_int32() for _ in range(4)]
    assert L.ftgemm_query_tiling_ex(None, *[C.byref(x) for x in v]) == F.ERR_INVALID_ARG
    d = F.GemmDesc()
    d.dtype, d.abft, d.m, d.n, d.k = F.F64, 2, 64, 64, 64
    assert L.ftgemm_query_tiling_ex(C.byref(d), *[C.byref(x) for x in v]) == F.ERR_UNSUPPORTED
    d.dtype, d.abft = F.BF16, 3
    assert L.ftgemm_query_tiling_ex(C.byref(d), *[C.byref(x) for x in v]) == F.ERR_UNSUPPORTED
    d.dtype, d.abft = F.F64, 3
    assert L.ftgemm_query_tiling_ex(C.byref(d), *[C.byref(x) for x in v]) == F.OK
    assert [x.value for x in v] == list(F.query_tiling(F.F64, 64, 64, 64))
    # the weighted mode never splits the inner dimension
    assert F.query_tiling(F.F64, 1024, 1024, 32768)[3] > 1
    assert F.query_tiling_ex(F.F64, 1024, 1024, 32768, abft=4) == (128, 128, 32, 1)
    d.dtype, d.abft = F.BF16, 4
    assert L.ftgemm_query_tiling_ex(C.byref(d), *[C.byref(x) for x in v]) == F.ERR_UNSUPPORTED
    d.dtype, d.abft = F.F64, 5
    assert L.ftgemm_query_tiling_ex(C.byref(d), *[C.byref(x) for x in v]) == F.ERR_INVALID_ARG
    d.abft = 1
    assert L.ftgemm_query_tiling_ex(C.byref(d), None, None, None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 2


def test_fault_plan_validation():
    L = F.lib()
    bad = F.Injection(0, 5, 0, 0, 1, 1, 1, 1.0)  # unknown mode
    assert L.ftgemm_set_fault_plan(C.byref(bad), 1) == F.ERR_INVALID_ARG
    bad = F.Injection(0, F.INJ_BITFLIP, F.TGT_ROW_CHECKSUM, 3, 1, 1, 1, 0.0)
    assert L.ftgemm_set_fault_plan(C.byref(bad), 1) == F.ERR_INVALID_ARG
    bad = F.Injection(0, F.INJ_BITFLIP, F.TGT_WEIGHTED_CHECKSUM, 3, 1, 1, 1, 0.0)
    assert L.ftgemm_set_fault_plan(C.byref(bad), 1) == F.ERR_INVALID_ARG
    bad = F.Injection(0, F.INJ_ADD, 4, 0, 1, 1, 1, 1.0)
    assert L.ftgemm_set_fault_plan(C.byref(bad), 1) == F.ERR_INVALID_ARG
    ok = F.Injection(0, F.INJ_ADD, F.TGT_WEIGHTED_CHECKSUM, 0, 1, 1, 1, 2.0)
    assert L.ftgemm_set_fault_plan(C.byref(ok), 1) == F.OK
    bad = F.Injection(0, F.INJ_BITFLIP, F.TGT_ACC, 64, 1, 1, 1, 0.0)
    assert L.ftgemm_set_fault_plan(C.byref(bad), 1) == F.ERR_INVALID_ARG
    assert L.ftgemm_set_fault_plan(None, -1) == F.ERR_INVALID_ARG
    ok = F.Injection(0, F.INJ_ADD, F.TGT_ACC, 0, 1, 1, 1, 2.0)
    assert L.ftgemm_set_fault_plan(C.byref(ok), 1) == F.OK
    assert L.ftgemm_set_fault_plan(None, 0) == F.OK


def test_query_tiling():
    tm, tn, bk, sk = F.query_tiling(F.F64, 256, 256, 256)
    assert (tm, tn, sk) == (128, 128, 1) and bk in (16, 32)
    assert F.lib().ftgemm_query_tiling(9, 1, 1, 1, None, None, None, None) == F.ERR_INVALID_ARG
    # low precision: 128 bytes of the inner dimension per row per step, no
    # split; 256-row tiles once there are at least 256 of them
    assert F.query_tiling(F.BF16, 8192, 8192, 8192) == (256, 128, 64, 1)
    assert F.query_tiling(F.FP8_E4M3, 8192, 8192, 8192) == (256, 128, 128, 1)
    assert F.query_tiling(F.FP8_E4M3, 4096, 1920, 64) == (128, 128, 128, 1)   # 16 x 15
    assert F.query_tiling(F.BF16, 4096, 2048, 64) == (256, 128, 64, 1)      # 16 x 16 tiles
    assert F.query_tiling(F.BF16, 3841, 2048, 64) == (256, 128, 64, 1)      # 16 x 16
    assert F.query_tiling(F.BF16, 4096, 1920, 64) == (128, 128, 64, 1)      # 16 x 15
    assert F.query_tiling(F.BF16, 1024, 1024, 32768) == (128, 128, 64, 1)


def test_split_choice():
    """FP64 splits the inner dimension only when the output has fewer tiles
    than compute units and the inner dimension is long: slices of at least
    8 steps, at most 16, aimed at 512 workgroups."""
    bk = F.query_tiling(F.F64, 64, 64, 64)[2]
    cases = {(8192, 8192, 8192): 1,           # 4096 tiles
             (16384, 16384, 256): 1,          # 16384 tiles
             (1024, 1024, 32768): 8,          # 64 tiles -> 512 workgroups
             (16384, 64, 16384): 4,           # 128 tiles
             (256, 256, 256): 1,              # inner dimension too short
             (128, 128, 32 * bk): 4,          # 1 tile, 32 steps -> 4 slices of 8
             (128, 128, 1 << 20): 16}         # 1 tile, capped at 16 slices
    for (m, n, k), want in cases.items():
        assert F.query_tiling(F.F64, m, n, k)[3] == want, (m, n, k)



def test_status_strings():
    L = F.lib()
    for s in range(5):
        assert L.ftgemm_status_string(s).startswith(b"FTGEMM")


def test_operand_windows_wider_than_the_loaders_reach_are_refused():
    """A step of an operand (and, for FP64, a tile of C_in) is read through
    one buffer window of at most 2^31 - 1 bytes with 32-bit offsets.  A leading dimension that makes the
    window wider would read zeros or wrapped addresses with no sign (the
    checksums are summed from the same staged values), so it is refused on
    the host with the operand's position; the largest leading dimension
    that fits is accepted (checked up to the argument checks: the call then
    stops at the quick return alpha = 0, beta = 1)."""
    L = F.lib()
    lim = 2 ** 31 - 1

    def desc(dtype, ta, tb, m, n, k, lda, ldb):
        d = F.GemmDesc()
        d.dtype, d.transA, d.transB = dtype, ta, tb
        d.m, d.n, d.k, d.lda, d.ldb, d.ldc = m, n, k, lda, ldb, m
        d.alpha, d.beta, d.scaleA, d.scaleB, d.A, d.B, d.C = 1.0, 0.0, 1.0, 1.0, 1, 1, 1
        return d

    # FP64, A not transposed: its rows run along the stored rows, so a step
    # spans 32 stored columns: 31 ld + 128 elements of 8 bytes
    ok = (lim // 8 - 128) // 31
    d = desc(F.F64, 0, 0, 512, 512, 512, ok + 1, 512)
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 8
    # A transposed: a step spans the tile's 128 rows of op(A), as stored columns
    ok_t = (lim // 8 - 32) // 127
    d = desc(F.F64, 1, 0, 512, 512, 512, ok_t + 1, 512)
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 8
    # B not transposed (inner index along the stored rows): 128 stored columns
    d = desc(F.F64, 0, 0, 512, 512, 512, 512, ok_t + 1)
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 10
    # BF16 and FP8 tiles reach 256 outer indices
    ok_bf = (lim // 2 - 64) // 255
    d = desc(F.BF16, 1, 0, 512, 512, 512, ok_bf + 1, 512)
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 8
    d = desc(F.FP8_E4M3, 0, 1, 512, 512, 512, 512, (lim - 256) // 127 + 1)
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 10
    # the same in a batch
    d = desc(F.F64, 1, 0, 512, 512, 512, ok_t + 1, 512)
    assert L.ftgemm_gemm_batched(1, C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 8
    # one stored column longer than the window: the dimension's position
    d = desc(F.F64, 1, 0, 64, 64, lim // 8 + 1, lim // 8 + 1, lim // 8 + 1)
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 5
    # the beta pass reads each tile of C_in through one window: 127 ldc + 128
    # FP64 elements, or 127 ldc + 256 FP32 ones
    ok_c = (lim // 8 - 128) // 127
    d = desc(F.F64, 0, 0, 512, 512, 512, 512, 512)
    d.ldc = ok_c + 1
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 13
    d = desc(F.BF16, 0, 0, 512, 512, 512, 512, 512)
    d.ldc = (lim // 4 - 256) // 127 + 1
    assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.ERR_INVALID_ARG
    assert L.ftgemm_last_invalid_arg() == 13
    wide_c = desc(F.F64, 0, 0, 512, 512, 512, 512, 512)
    wide_c.ldc = ok_c
    # the largest leading dimensions that fit pass the checks
    for d in (desc(F.F64, 0, 0, 512, 512, 512, ok, 512),
              desc(F.F64, 1, 1, 512, 512, 512, ok_t, ok),
              desc(F.BF16, 1, 0, 512, 512, 512, ok_bf, 512), wide_c):
        d.alpha, d.beta = 0.0, 1.0
        assert L.ftgemm_gemm_ex(C.byref(d), None, None) == F.OK


def test_tuning_table(tmp_path):
    """The tuning table on the host: a file with a malformed line is refused
    (position 1) and leaves the table as it was; 'tile' lines force the
    tiles of single low-precision calls; 'batch_mstar' fixes which batched
    low-precision problems take 256-row tiles; FP64 keeps 128 x 128; an
    empty table restores the defaults."""
    bad = tmp_path / "bad.tune"
    bad.write_text("tile 1 1 200\n")
    with pytest.raises(F.FTGemmError):
        F.load_tune_table(str(bad))
    assert F.lib().ftgemm_last_invalid_arg() == 1
    with pytest.raises(F.FTGemmError):
        F.load_tune_table(str(tmp_path / "missing.tune"))
    assert F.query_tiling_ex(F.BF16, 8192, 8192, 8192)[:2] == (256, 128)
    good = tmp_path / "good.tune"
    good.write_text("# comment\ntile 1 1 128\ntile 2 0 128   # plain FP8 on 128 rows\n"
                    "batch_mstar 512\n")
    F.load_tune_table(str(good))
    try:
        assert F.query_tiling_ex(F.BF16, 8192, 8192, 8192)[:2] == (128, 128)
        assert F.query_tiling(F.BF16, 8192, 8192, 8192)[:2] == (128, 128)
        assert F.query_tiling_ex(F.FP8_E4M3, 8192, 8192, 8192, abft=0)[:2] == (128, 128)
        assert F.query_tiling_ex(F.BF16, 8192, 8192, 8192, abft=2)[:2] == (256, 128)
        descs = []
        for m in (100, 511, 512, 2000):
            d = F.GemmDesc()
            d.dtype, d.m, d.n, d.k = F.BF16, m, 64, 64
            descs.append(d)
        assert F.batch_tiling(descs) == [128, 128, 256, 256]
        for d in descs:
            d.dtype = F.F64
        assert F.batch_tiling(descs) == [128] * 4
    finally:
        F.load_tune_table(None)
    assert F.query_tiling_ex(F.BF16, 8192, 8192, 8192)[:2] == (256, 128)
    assert F.query_tiling_ex(F.FP8_E4M3, 8192, 8192, 8192, abft=0)[:2] == (256, 128)
