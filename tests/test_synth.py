"""The seeded input and fault-plan generators (shared by the GPU tests, the
benchmark and the oracle's checks; they hold none of the method's
arithmetic): deterministic per seed, and the plans place faults where they
say."""
import numpy as np

from paper_2305_02444_amd import synth


def test_operands_are_seeded():
    a = synth.operands(3, 7, 40, 30, 20, "normal")
    b = synth.operands(3, 7, 40, 30, 20, "normal")
    c = synth.operands(3, 8, 40, 30, 20, "normal")
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], c[0])
    A, B, C = a
    assert A.shape == (40, 20) and B.shape == (20, 30) and C.shape == (40, 30)


def test_additive_plan_one_fault_per_tile():
    g = synth.rng(1, 0, synth.STREAM_PLAN)
    plan = synth.additive_plan(g, 1000, 700, 300, 128, 128, 20, lambda _g: 5.0)
    tiles = [(f.row // 128, f.col // 128) for f in plan]
    assert len(plan) == 20 and len(set(tiles)) == 20
    assert all(0 <= f.row < 1000 and 0 <= f.col < 700 and 0 <= f.k_index < 300 for f in plan)


def test_crossing_pairs_plan():
    """Two faults per tile, in different rows and columns of the tile,
    with deltas that differ; ragged edge tiles stay in bounds."""
    g = synth.rng(2, 0, synth.STREAM_PLAN)
    m, n, k = 300, 260, 50
    plan = synth.crossing_pairs_plan(g, m, n, k, 128, 128, 6, synth.log_magnitude(1.0))
    assert len(plan) == 12
    for a, b in zip(plan[0::2], plan[1::2]):
        assert (a.row // 128, a.col // 128) == (b.row // 128, b.col // 128)
        assert a.row != b.row and a.col != b.col
        assert abs(a.delta - b.delta) > 1e-3 * max(abs(a.delta), abs(b.delta))
    assert all(0 <= f.row < m and 0 <= f.col < n and 0 <= f.k_index < k for f in plan)
    assert len({(f.row // 128, f.col // 128) for f in plan}) == 6
