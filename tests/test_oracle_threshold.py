"""The oracle's detection threshold is linear in its multiplier lambda (the
hand-worked values of every term, and the soundness-and-tightness check,
are pins in oracle_pins.py and run with the others)."""
import numpy as np

from golden_io import read_threshold_example


def test_threshold_scales_with_lambda(orc):
    d = read_threshold_example()
    kw = dict(Cin=d["Cin"], alpha=d["alpha"], beta=d["beta"], tm=4, tn=4, bk=2)
    tr8, tc8 = orc.tile_thresholds(d["A"], d["B"], 0, 0, lam=8.0, **kw)
    tr1, tc1 = orc.tile_thresholds(d["A"], d["B"], 0, 0, lam=1.0, **kw)
    assert np.array_equal(tr8, 8.0 * tr1) and np.array_equal(tc8, 8.0 * tc1)
