"""Pins of the oracle's threshold term for multipliers that truncate their
in-instruction sums (the FP8 matrix instructions).

The arithmetic, stated as a rule: products are summed in groups of 8
consecutive inner indices; each product is cut toward zero to a multiple of
2^-14 * 2^E, 2^E the binade of the largest product magnitude in its group.
A brute-force model of that rule (written here, independently of the
oracle) produces the output of a tile; its checksum residuals against the
exact encoded checksums must stay below the oracle's thresholds with the
term (no false positives) on four input families, and must exceed the
thresholds without it on sparse non-negative data (the term is needed)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2305_02444_amd import synth

GRID, GROUP = 2.0 ** -14, 8


def truncating_product(A, B):
    P = A[:, None, :] * B.T[None, :, :]              # (h, w, k)
    h, w, k = P.shape
    kk = -(-k // GROUP) * GROUP
    Pp = np.zeros((h, w, kk))
    Pp[..., :k] = P
    G = Pp.reshape(h, w, kk // GROUP, GROUP)
    M = np.abs(G).max(-1)
    q = GRID * 2.0 ** np.floor(np.log2(np.where(M > 0, M, 1.0)))
    return (np.trunc(G / q[..., None]) * q[..., None]).sum(-1).sum(-1)


def _quant(x, orc):
    s = synth.e4m3_scale(x)
    return np.asfortranarray(orc.decode_e4m3(synth.to_e4m3_bits(x, s)))


def _family(kind, g, h, k, w):
    if kind == "normal":
        return g.standard_normal((h, k)), g.standard_normal((k, w))
    if kind == "positive":
        return g.uniform(0, 1, (h, k)), g.uniform(0, 1, (k, w))
    if kind == "outliers":
        return (g.standard_normal((h, k)) * np.where(g.random((h, k)) < 0.01, 50, 1),
                g.standard_normal((k, w)) * np.where(g.random((k, w)) < 0.01, 50, 1))
    return (np.abs(g.standard_normal((h, k))) * np.where(g.random((h, k)) < 0.1, 30, 1),
            np.abs(g.standard_normal((k, w))) * np.where(g.random((k, w)) < 0.1, 30, 1))


def test_model_rule_on_hand_cases():
    # 448^2 = 200704 has binade 2^17, so the grid is 8
    A = np.array([[448.0, 7.0, 9.0, -12.0]])
    for col, want in ((1, 200704.0), (2, 200712.0), (3, 200696.0)):
        B = np.zeros((4, 1))
        B[0, 0], B[col, 0] = 448.0, 1.0
        assert truncating_product(A, B)[0, 0] == want
    A = np.zeros((1, 16))
    A[0, 0], A[0, 8] = 448.0, 7.0
    B = np.zeros((16, 1))
    B[0, 0], B[8, 0] = 448.0, 1.0
    assert truncating_product(A, B)[0, 0] == 200711.0  # different groups


@pytest.mark.parametrize("kind", ["normal", "positive", "outliers", "sparse"])
@pytest.mark.parametrize("k", [128, 1024])
def test_threshold_covers_truncated_sums(kind, k):
    orc = O.default()
    g = np.random.default_rng([7, k, len(kind)])
    A0, B0 = _family(kind, g, 128, k, 128)
    A, B = _quant(np.asfortranarray(A0), orc), _quant(np.asfortranarray(B0), orc)
    C = truncating_product(A, B)
    Pr, Pc, _, _ = orc.tile_checksums(A, B, 0, 0, None, 1.0, 0.0, tm=128, tn=128, bk=128)
    dr, dc = C.sum(0) - Pr, C.sum(1) - Pc
    tr, tc = orc.tile_thresholds(A, B, 0, 0, None, 1.0, 0.0, tm=128, tn=128, bk=128,
                                 acc_bits=32, mma=(GRID, GROUP))
    assert np.all(np.abs(dr) <= tr) and np.all(np.abs(dc) <= tc)
    if kind == "sparse" and k == 128:
        tr0, tc0 = orc.tile_thresholds(A, B, 0, 0, None, 1.0, 0.0, tm=128, tn=128, bk=128,
                                       acc_bits=32)
        assert np.any(np.abs(dr) > tr0) or np.any(np.abs(dc) > tc0)


def test_term_scales_as_stated():
    """Doubling every entry of A doubles max|A_I| and the column-checksum
    term; the difference of the thresholds with and without the term is
    lambda * |alpha| * grid * sqrt(group) * sqrt(h) * max|A_I| * ||b_j||."""
    orc = O.default()
    g = np.random.default_rng(3)
    A = np.asfortranarray(g.standard_normal((50, 40)))
    B = np.asfortranarray(g.standard_normal((40, 30)))
    tr1, tc1 = orc.tile_thresholds(A, B, 0, 0, None, 2.0, 0.0, acc_bits=32, bk=8,
                                   mma=(GRID, GROUP))
    tr0, tc0 = orc.tile_thresholds(A, B, 0, 0, None, 2.0, 0.0, acc_bits=32, bk=8)
    lam = 8.0
    want_r = lam * 2.0 * GRID * np.sqrt(GROUP) * np.sqrt(50) * np.abs(A).max() * \
        np.linalg.norm(B, axis=0)
    want_c = lam * 2.0 * GRID * np.sqrt(GROUP) * np.sqrt(30) * np.abs(B).max() * \
        np.linalg.norm(A, axis=1)
    assert np.allclose(tr1 - tr0, want_r, rtol=1e-12)
    assert np.allclose(tc1 - tc0, want_c, rtol=1e-12)
