"""The oracle on the hand-worked example in tests/golden/worked_example.txt
(checksum encoding, reference sums, and the three fault classes)."""
import numpy as np

from golden_io import read_worked_example
from oracle import oracle as O

TARGETS = {"acc": O.TGT_ACC, "rowck": O.TGT_ROW_CHECKSUM, "colck": O.TGT_COL_CHECKSUM}
KINDS = {"corrected": O.CORRECTED, "checksum_only": O.CHECKSUM_ONLY,
         "recomputed": O.RECOMPUTED}


def test_worked_example(orc):
    d = read_worked_example()
    kw = dict(alpha=d["alpha"], beta=d["beta"], tm=d["tm"], tn=d["tn"], bk=d["bk"])
    # the plain product
    assert np.array_equal(orc.gemm(d["A"], d["B"], d["Cin"], d["alpha"], d["beta"]), d["C"])
    # encoded checksums, tile by tile, equal the hand-worked values
    for ti, tj, _, r0, r1, _, c0, c1 in d["checksums"]:
        Pr, Pc, Rr, Rc = orc.tile_checksums(d["A"], d["B"], int(ti), int(tj), d["Cin"], **kw)
        assert Pr.tolist() == [float(r0), float(r1)]
        assert Pc.tolist() == [float(c0), float(c1)]
        assert Rr.tolist() == Pr.tolist() and Rc.tolist() == Pc.tolist()
    # faults
    plan = [O.Injection(int(r), int(c), int(kk), O.ADD, float(dv), target=TARGETS[t])
            for r, c, kk, t, dv in d["fault"]]
    res = orc.ftgemm(d["A"], d["B"], d["Cin"], injections=plan, **kw)
    assert np.array_equal(res.C, d["C"])
    got = {(r["tile_m"], r["tile_n"]): r for r in res.records}
    assert len(got) == len(d["expect"])
    for e in d["expect"]:
        r = got[(int(e[0]), int(e[1]))]
        assert r["kind"] == KINDS[e[2]]
        if e[2] == "corrected":
            assert (r["row"], r["col"], r["before"], r["after"]) == \
                (int(e[3]), int(e[4]), float(e[5]), float(e[6]))
