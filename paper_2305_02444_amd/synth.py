"""Seeded synthetic workloads for the fault-tolerant GEMM.

This module only draws random numbers: matrices with the distributions the
workloads call for, their quantisation to the low-precision input formats,
random fault plans (positions, inner-dimension steps, magnitudes, bits) and
random problem shapes for batched runs.  It holds none of the method's
arithmetic -- no checksum, no threshold, no GEMM -- so the GPU path and the
CPU oracle can both be fed from it without sharing any of the computation.

The paper (Section 3) states only matrix sizes; the value distributions
(uniform on [-1, 1], standard normal) and the fault plans are this
project's synthetic stand-ins.

Every stream is numpy PCG64 seeded by SeedSequence([workload_id, seed,
stream_id]), so each operand and the fault plan are independent and
reproducible.  Matrices are float64 column-major (Fortran order) arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Stream identifiers inside one workload.
STREAM_A, STREAM_B, STREAM_C, STREAM_PLAN, STREAM_SHAPES = 0, 1, 2, 3, 4

# Fault modes / targets (the library and the oracle each define the same
# numbering for their own structures).
ADD, BITFLIP = 0, 1
TGT_ACC, TGT_ROW_CHECKSUM, TGT_COL_CHECKSUM, TGT_WEIGHTED_CHECKSUM = 0, 1, 2, 3

E4M3_MAX = 448.0


def rng(workload_id: int, seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload_id, seed, stream])))


def matrix(rows: int, cols: int, dist: str, g: np.random.Generator) -> np.ndarray:
    """A rows x cols float64 column-major matrix with i.i.d. entries."""
    if dist == "uniform":
        v = g.uniform(-1.0, 1.0, size=(cols, rows))
    elif dist == "normal":
        v = g.standard_normal(size=(cols, rows))
    elif dist.startswith("int"):
        lim = int(dist[3:] or 8)
        v = g.integers(-lim, lim + 1, size=(cols, rows)).astype(np.float64)
    else:
        raise ValueError(dist)
    return v.T  # column-major view of a C-ordered (cols, rows) block


def operands(workload_id: int, seed: int, m: int, n: int, k: int, dist: str,
             ta: bool = False, tb: bool = False, with_c: bool = True):
    """(A, B, C) as stored: A is m x k (or k x m when ta), B is k x n (or n x k)."""
    A = matrix(k, m, dist, rng(workload_id, seed, STREAM_A)) if ta else \
        matrix(m, k, dist, rng(workload_id, seed, STREAM_A))
    B = matrix(n, k, dist, rng(workload_id, seed, STREAM_B)) if tb else \
        matrix(k, n, dist, rng(workload_id, seed, STREAM_B))
    Cm = matrix(m, n, dist, rng(workload_id, seed, STREAM_C)) if with_c else None
    return A, B, Cm


# -- quantisation of inputs to the low-precision formats -------------------

def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even bfloat16 codes (uint16), same shape and order."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x.T if x.flags.f_contiguous and x.ndim == 2 else x))
    bits = t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    return bits.T if x.flags.f_contiguous and x.ndim == 2 else bits


def e4m3_scale(x: np.ndarray) -> float:
    """Per-tensor scale so that x / scale spans the E4M3 range (amax / 448)."""
    amax = float(np.max(np.abs(x))) if x.size else 0.0
    return amax / E4M3_MAX if amax > 0 else 1.0


def to_e4m3_bits(x: np.ndarray, scale: float) -> np.ndarray:
    """OCP E4M3 (finite) codes (uint8) of x / scale, round-to-nearest-even."""
    import torch
    xc = x.T if x.flags.f_contiguous and x.ndim == 2 else x
    t = torch.from_numpy(np.ascontiguousarray(xc / scale))
    t = torch.clamp(t, -E4M3_MAX, E4M3_MAX)
    bits = t.to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    return bits.T if x.flags.f_contiguous and x.ndim == 2 else bits


# -- fault plans ------------------------------------------------------------

@dataclass
class Fault:
    row: int
    col: int
    k_index: int
    mode: int = ADD
    delta: float = 0.0
    bit: int = 0
    target: int = TGT_ACC
    problem: int = 0


def tiles_without_replacement(g, tiles_m: int, tiles_n: int, count: int):
    count = min(count, tiles_m * tiles_n)
    ids = g.choice(tiles_m * tiles_n, size=count, replace=False)
    return [(int(t % tiles_m), int(t // tiles_m)) for t in ids]


def position_in_tile(g, tile, m, n, k, tm, tn):
    ti, tj = tile
    r0, c0 = ti * tm, tj * tn
    row = r0 + int(g.integers(0, min(tm, m - r0)))
    col = c0 + int(g.integers(0, min(tn, n - c0)))
    kidx = int(g.integers(0, max(k, 1)))
    return row, col, kidx


def additive_plan(g, m, n, k, tm, tn, count, magnitude):
    """count faults in distinct tiles; magnitude(g) draws each delta."""
    tm_ = -(-m // tm)
    tn_ = -(-n // tn)
    plan = []
    for tile in tiles_without_replacement(g, tm_, tn_, count):
        row, col, kidx = position_in_tile(g, tile, m, n, k, tm, tn)
        plan.append(Fault(row, col, kidx, ADD, float(magnitude(g))))
    return plan


def crossing_pairs_plan(g, m, n, k, tm, tn, count, magnitude, equal=False):
    """Two faults in each of count distinct tiles, in different rows and
    different columns of the tile (tiles with a single row or column are
    skipped); magnitude(g) draws each delta, redrawn until the two differ
    by more than 1 in 1000 -- or, with equal, one delta for both."""
    tm_ = -(-m // tm)
    tn_ = -(-n // tn)
    plan = []
    for (ti, tj) in tiles_without_replacement(g, tm_, tn_, count):
        h, w = min(tm, m - ti * tm), min(tn, n - tj * tn)
        if h < 2 or w < 2:
            continue
        rows = g.choice(h, size=2, replace=False)
        cols = g.choice(w, size=2, replace=False)
        d1 = float(magnitude(g))
        d2 = d1 if equal else float(magnitude(g))
        while not equal and abs(d1 - d2) <= 1e-3 * max(abs(d1), abs(d2)):
            d2 = float(magnitude(g))
        for r, c, d in ((rows[0], cols[0], d1), (rows[1], cols[1], d2)):
            plan.append(Fault(ti * tm + int(r), tj * tn + int(c), int(g.integers(0, max(k, 1))),
                              ADD, d))
    return plan


def log_magnitude(sigma: float, lo_exp: float = 0.0, hi_exp: float = 6.0):
    """Random-sign delta of size 10^U(lo, hi) * sigma."""
    def draw(g):
        return (1.0 if g.random() < 0.5 else -1.0) * 10.0 ** g.uniform(lo_exp, hi_exp) * sigma
    return draw


# Exponent bits and the high fraction bits of an IEEE binary32 value (the
# sign bit is excluded).
FP32_FLIP_BITS = list(range(23, 31)) + list(range(19, 23))


def bitflip_plan(g, m, n, k, tm, tn, count, bits=FP32_FLIP_BITS):
    tm_ = -(-m // tm)
    tn_ = -(-n // tn)
    plan = []
    for tile in tiles_without_replacement(g, tm_, tn_, count):
        row, col, kidx = position_in_tile(g, tile, m, n, k, tm, tn)
        plan.append(Fault(row, col, kidx, BITFLIP, 0.0, int(g.choice(bits))))
    return plan


def truncated_poisson(g, mean: float, cap: int) -> int:
    while True:
        v = int(g.poisson(mean))
        if v <= cap:
            return v


def log_uniform_int(g, lo: int, hi: int) -> int:
    return int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))


def batched_shapes(workload_id: int, seed: int, count: int, lo: int = 64, hi: int = 2048):
    g = rng(workload_id, seed, STREAM_SHAPES)
    return [(log_uniform_int(g, lo, hi), log_uniform_int(g, lo, hi), log_uniform_int(g, lo, hi))
            for _ in range(count)]
