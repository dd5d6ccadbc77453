"""The pins have teeth: plausible mistakes planted in copies of the oracle
(on the CPU, never in the GPU path) must each fail at least one pin."""
import os

import pytest

import oracle_pins
from oracle import oracle as O

MUTANTS = {
    "dropped_beta_term_in_row_checksum": (
        "Pr[jj] = alpha * s + beta * c;", "Pr[jj] = alpha * s;"),
    "wrong_operand_checksum_in_row_checksum": (
        "s += x[p] * opB(B, P->ldb, P->tb, p, j0 + jj);",
        "s += y[p] * opB(B, P->ldb, P->tb, p, j0 + jj);"),
    "wrong_sign_in_correction": (
        "double fixed = Pr[jbad] - sr;", "double fixed = sr - Pr[jbad];"),
    "line_residual_added_not_subtracted": (
        "out[ii + jj * h] -= d;", "out[ii + jj * h] += d;"),
    "line_confirmed_without_its_own_residual": (
        "if (wok && fabs(dl - sumd) <= (by_row ? tc[line] : tr[line])) {",
        "if (fabs(sumd) <= (by_row ? tc[line] : tr[line]) || 1) {"),
    "pair_residual_added_not_subtracted": (
        "out[rows[a] + jj * h] -= Rr[jj] - Pr[jj];", "out[rows[a] + jj * h] += Rr[jj] - Pr[jj];"),
    "pairing_not_one_to_one": (
        "if (found != 1 || (taken >> mate[a]) & 1u) paired = 0;",
        "if (found < 1) paired = 0;"),
    "transposed_operand_A": (
        "return ta ? A[p + i * lda] : A[i + p * lda];",
        "return ta ? A[i + p * lda] : A[p + i * lda];"),
    "wrong_row_index_in_column_sum": (
        "s += out[ii + jj * h];\n            Rc[ii] = s;",
        "s += out[jj + ii * h];\n            Rc[ii] = s;"),
    "threshold_drops_sqrt_k": (
        "double sk = sqrt((double)k);", "double sk = 1.0;"),
    "threshold_drops_sqrt_h": (
        "double sh = sqrt((double)h);", "double sh = 1.0;"),
    "threshold_unit_roundoffs_swapped": (
        "return (P->acc_bits == 32) ? ldexp(1.0, -24) : ldexp(1.0, -53);",
        "return (P->acc_bits == 32) ? ldexp(1.0, -53) : ldexp(1.0, -24);"),
    "threshold_drops_beta_term": (
        " + 2.0 * u * fabs(beta) * nrm_cin);", ");"),
    "threshold_lambda_a_tenth": (
        "return lambda * (fabs(alpha)", "return 0.1 * lambda * (fabs(alpha)"),
    "threshold_drops_truncation_term": (
        "P->lambda * fabs(alpha) * trunc * sqrt((double)h) * ma * nb[jj];", "0.0;"),
    "entries_read_cin_transposed": (
        "out[t] = (beta == 0.0) ? alpha * s : alpha * s + beta * Cin[i + j * ldc];",
        "out[t] = (beta == 0.0) ? alpha * s : alpha * s + beta * Cin[j + i * ldc];"),
    "single_flag_always_checksum_only": (
        "const double bound = (by_col ? tr[jbad] : tc[ibad]) + 2.0 * other;",
        "const double bound = -1.0;"),
    "single_flag_bound_ignores_other_side": (
        "const double bound = (by_col ? tr[jbad] : tc[ibad]) + 2.0 * other;",
        "const double bound = (by_col ? tr[jbad] : tc[ibad]);"),
    "split_checksum_fault_entry_not_replaced": (
        "if (by_col) Pr[jbad] = Rr[jbad]; else Pc[ibad] = Rc[ibad];", ""),
    "split_fault_lands_in_the_next_slice": (
        "const int in = f->k_index >= kb &&", "const int in = f->k_index >= kb + 8 &&"),
    "split_reduction_drops_beta": (
        "if (beta != 0.0) { v = v + beta * c; vr = vr + beta * c; }", ""),
    "weighted_encode_weights_off_by_one": (
        "s += (double)(ii + 1) * opA(A, P->lda, P->ta, i0 + ii, p);",
        "s += (double)(ii) * opA(A, P->lda, P->ta, i0 + ii, p);"),
    "weighted_line_confirm_skipped": (
        "if (!(fabs(dw[x] - (double)(line + 1) * d) <=", "if (0 && !(fabs(dw[x] - (double)(line + 1) * d) <="),
    "weighted_single_confirm_skipped": (
        "const int wok = !wt || !isfinite(dcol)", "const int wok = 1 || !isfinite(dcol)"),
    "weighted_location_off_by_one": (
        "const int64_t r = (int64_t)llround(ratio) - 1;", "const int64_t r = (int64_t)llround(ratio);"),
    "threshold_zero": (
        "return lambda * (fabs(alpha)", "return 0.0 * (fabs(alpha)"),
    "fault_one_step_late": (
        "if (f->target != TGT_ACC || f->k_index / P->bk != s)",
        "if (f->target != TGT_ACC || f->k_index / P->bk + 1 != s)"),
    "ragged_tile_loses_a_row": (
        "const int64_t h = (P->m - i0 < P->tm) ? P->m - i0 : P->tm;\n    const int64_t w = (P->n - j0 < P->tn) ? P->n - j0 : P->tn;\n    const double alpha",
        "const int64_t h = (P->m - i0 < P->tm) ? P->m - i0 - 1 : P->tm;\n    const int64_t w = (P->n - j0 < P->tn) ? P->n - j0 : P->tn;\n    const double alpha"),
    "correction_not_confirmed": (
        "if (wok && fabs(sc + fixed - Pc[ibad]) <= tc[ibad]) {", "if (1) {"),
    "bf16_exponent_bias_off_by_one": (
        "v = ldexp((double)(128 + f), e - 127 - 7);", "v = ldexp((double)(128 + f), e - 126 - 7);"),
    "e4m3_nan_code_wrong": (
        "if (e == 0xf && f == 0x7)", "if (e == 0xf && f == 0x6)"),
    "beta_zero_reads_cin": (
        "col[i] = (beta == 0.0) ? alpha * col[i]\n                                   : alpha * col[i] + beta * Cin[i + j * ldc];",
        "col[i] = alpha * col[i] + beta * Cin[i + j * ldc];"),
}


def _format_pins(orc):
    import numpy as np
    import torch
    codes = np.arange(1 << 16, dtype=np.uint16)
    mine = orc.decode_bf16(codes)
    ref = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).double().numpy()
    assert np.array_equal(np.isnan(mine), np.isnan(ref))
    assert np.array_equal(mine[~np.isnan(mine)], ref[~np.isnan(ref)])
    c8 = np.arange(256, dtype=np.uint8)
    mine = orc.decode_e4m3(c8)
    ref = torch.from_numpy(c8).view(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(np.isnan(mine), np.isnan(ref))
    assert np.array_equal(mine[~np.isnan(mine)], ref[~np.isnan(ref)])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(O.SRC).read()
    assert src.count(old) == 1, "mutation site not found: " + name
    path = os.path.join(tmp_path, "mutant.c")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    mutant = O.Oracle(O.compile_source(path, os.path.join(tmp_path, "libmutant.so")))
    failures = []
    for pin in oracle_pins.ALL_PINS + [_format_pins]:
        try:
            pin(mutant)
        except AssertionError:
            failures.append(pin.__name__)
    assert failures, "no pin caught the mutant " + name
