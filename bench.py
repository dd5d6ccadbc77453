#!/usr/bin/env python3
"""Benchmark of libftgemm on one MI355X.

Metric: fault-tolerant GEMM TFLOP/s and the ABFT overhead against the same
kernel with every checksum operation compiled out, at 8192^3 in FP64 (the
headline) and BF16 / FP8 (extra legs), with and without injected faults.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --profile KIND   (a short workload for rocprofv3 passes; see profile_run)

A step is one full fault-tolerant GEMM call C = alpha*A*B + beta*C
(alpha = beta = 1, inputs uniform on [-1, 1], column-major N/N) on inputs
already resident in HBM: operand checksums, encoded checksums, reference
sums, verification (and correction when faults are injected) included.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "bf16": 2516.6, "fp8": 5033.2}  # dense MFMA TFLOP/s, MI355X
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2305_02444_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(name, files):
    """HBM bytes per launch from a committed counter summary, or None when the
    kernel source changed since the counters were taken."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            key, val = line.split(":", 1)
            vals[key.strip()] = val.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash(files):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def with_table(F, text, fn):
    """Run fn() with a tuning table holding these lines, then an empty one."""
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".tune")
    with os.fdopen(fd, "w") as fh:
        fh.write(text)
    try:
        F.load_tune_table(path)
        return fn()
    finally:
        F.load_tune_table(None)
        os.unlink(path)


# warm-up time of the legs beside the headline (see timed)
SETTLE_MS = 50.0


def timed(torch, fn, steps, warmup, reset=None, settle_ms=0.0):
    """Average per-call time (ms) over `steps` calls, from HIP events on the
    launch stream around each call.  reset (optional) runs before every
    call, outside the events: it restores C from a pristine copy, since
    with beta != 0 C is read and written.  The warm-up is `warmup` calls,
    continued until it has taken settle_ms of device time: a short kernel
    launched right after a different heavy one has measured up to 10%
    slower for some tens of milliseconds, which a few warm-up calls of a
    2 ms kernel do not cover.  Returns (ms_per_call, ms_total / steps), the
    second including the resets."""
    stream = torch.cuda.current_stream()
    w0 = torch.cuda.Event(enable_timing=True)
    w1 = torch.cuda.Event(enable_timing=True)
    w0.record(stream)
    done = 0
    while done < warmup or settle_ms > 0.0:
        if reset:
            reset()
        fn()
        done += 1
        if done >= warmup and settle_ms > 0.0:
            w1.record(stream)
            torch.cuda.synchronize()
            if w0.elapsed_time(w1) >= settle_ms or done >= warmup + 500:
                break
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for s in range(steps):
        if reset:
            reset()
        ev[s][0].record(stream)
        fn()
        ev[s][1].record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    total = start.elapsed_time(end) / steps
    per = sum(a.elapsed_time(b) for a, b in ev) / steps
    return per, total


def cpu_baseline(A, B, Cin, m, n, k, budget_s=(8.0, 6.0)):
    """The oracle (untuned) on the host cores, built there with -O3
    -march=native -fopenmp, on a bounded sample of tiles of the same
    problem, with all cores and with one; rate in useful TFLOP/s
    (2 * tile flops / time)."""
    import numpy as np
    from oracle import oracle as O
    orc = O.native()
    tiles_m = -(-m // 128)
    ntiles = tiles_m * (-(-n // 128))
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    g = np.random.default_rng(1234)

    def rate(threads, budget):
        orc.set_threads(threads)
        cal = min(ntiles, max(threads, 2))
        t0 = time.perf_counter()
        orc.ftgemm(A, B, Cin, 1.0, 1.0, tiles=g.choice(ntiles, cal, replace=False))
        per_tile = (time.perf_counter() - t0) / cal
        count = int(min(ntiles, max(cal, budget / max(per_tile, 1e-6))))
        tiles = g.choice(ntiles, count, replace=False)
        t0 = time.perf_counter()
        orc.ftgemm(A, B, Cin, 1.0, 1.0, tiles=tiles)
        dt = time.perf_counter() - t0
        return 2.0 * 128 * 128 * k * count / dt / 1e12, count, dt

    v_all, c_all, dt_all = rate(cores, budget_s[0])
    v_one, c_one, dt_one = rate(1, budget_s[1])
    orc.set_threads(cores)
    return {"value": v_all, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "value_1_thread": v_one,
            "build": "gcc -O3 -march=native -fopenmp on the host timed",
            "sample": "%d (all cores, %.1f s) and %d (1 thread, %.1f s) of %d 128x128 output "
                      "tiles of the %dx%dx%d FP64 fault-tolerant GEMM (encode, multiply, verify "
                      "per tile)" % (c_all, dt_all, c_one, dt_one, ntiles, m, n, k)}


def lp_leg(torch, F, synth, np, dtype, size, steps, warmup, settle_ms=SETTLE_MS):
    """One low-precision leg at size^3: normal(0,1) inputs quantised to the
    format (FP8: per-tensor scales amax / 448), FP32 C, alpha = beta = 1."""
    m = n = k = size
    flops = 2.0 * m * n * k
    wid = 41 if dtype == F.BF16 else 42
    A, B, Cin = synth.operands(wid, size, m, n, k, "normal")
    if dtype == F.BF16:
        ca, cb, sa, sb = synth.to_bf16_bits(A), synth.to_bf16_bits(B), 1.0, 1.0
        dA = F.to_device(ca.view(np.int16)).view(torch.bfloat16)
        dB = F.to_device(cb.view(np.int16)).view(torch.bfloat16)
        deq = lambda t, s_: t.to(torch.float64)
    else:
        sa, sb = synth.e4m3_scale(A), synth.e4m3_scale(B)
        ca, cb = synth.to_e4m3_bits(A, sa), synth.to_e4m3_bits(B, sb)
        dA, dB = F.to_device(ca.view(np.uint8)), F.to_device(cb.view(np.uint8))
        deq = lambda t, s_: t.view(torch.float8_e4m3fn).to(torch.float64) * s_
    dC0 = F.to_device(np.asfortranarray(Cin, dtype=np.float32))
    dC = dC0.clone()
    del A, B

    def call(abft):
        d = F.make_desc(dA, dB, dC, 1.0, 1.0, abft=abft, scaleA=sa, scaleB=sb, dtype=dtype)
        return lambda: F.gemm_ex(d)

    F.clear_fault_plan()
    rb = F.ReportBuffer()
    dC.copy_(dC0)
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, scaleA=sa, scaleB=sb, dtype=dtype), report=rb)
    clean = rb.view()
    # accuracy on sampled 256 x 256 blocks against an FP64 product of the
    # decoded inputs (the quantisation itself is not counted)
    g = synth.rng(wid, size, 9)
    errs = []
    for _ in range(4):
        i0 = int(g.integers(0, m - 256)) if m > 256 else 0
        j0 = int(g.integers(0, n - 256)) if n > 256 else 0
        ref = deq(dA[i0:i0 + 256, :], sa).contiguous() @ deq(dB[:, j0:j0 + 256], sb).contiguous() + \
            dC0[i0:i0 + 256, j0:j0 + 256].to(torch.float64)
        got = dC[i0:i0 + 256, j0:j0 + 256].to(torch.float64)
        errs.append(float((got - ref).abs().max() / ref.abs().max()))
    reset = lambda: dC.copy_(dC0)
    t_ft, _ = timed(torch, call(True), steps, warmup, reset, SETTLE_MS)
    t_plain, _ = timed(torch, call(False), steps, warmup, reset, SETTLE_MS)
    tm, tn, bk, _ = F.query_tiling(dtype, m, n, k)
    tm0 = F.query_tiling_ex(dtype, m, n, k, abft=0)[0]
    # the same kernel with checksums compiled out on the fault-tolerant
    # call's own tile (the plain call's default tile may differ)
    if tm0 != tm:
        t_plain_same, _ = with_table(F, "tile %d 0 %d\n" % (dtype, tm),
                                     lambda: timed(torch, call(False), steps, warmup, reset,
                                                   SETTLE_MS))
    else:
        t_plain_same = t_plain
    # the operand checksums and norms formed in the tiles from the staged
    # operands (the entry point that allocates nothing takes no pass before
    # the product; fault-tolerant FP8 tiles have 128 rows there), against
    # the kernel without checksums on the same tile
    dn = F.make_desc(dA, dB, dC, 1.0, 1.0, scaleA=sa, scaleB=sb, dtype=dtype)
    t_in_tile, _ = timed(torch, lambda: F.gemm_ex_noalloc(dn), steps, warmup, reset, SETTLE_MS)
    tm_in = 128 if dtype == F.FP8_E4M3 else tm
    if tm_in == tm:
        t_plain_in = t_plain_same
    elif tm_in == tm0:
        t_plain_in = t_plain
    else:
        t_plain_in, _ = with_table(F, "tile %d 0 %d\n" % (dtype, tm_in),
                                   lambda: timed(torch, call(False), steps, warmup, reset,
                                                 SETTLE_MS))
    tiles = (-(-m // tm)) * (-(-n // tn))
    gp = synth.rng(wid, size, synth.STREAM_PLAN)
    # exponent flips (bits 27..30) of FP32 accumulators: always far above
    # the rounding threshold unless the accumulator is exactly zero
    plan = synth.bitflip_plan(gp, m, n, k, tm, tn, -(-tiles // 64), bits=[27, 28, 29, 30])
    F.set_fault_plan(plan)
    t_inj, _ = timed(torch, call(True), steps, warmup, reset, SETTLE_MS)
    rb = F.ReportBuffer()
    dC.copy_(dC0)
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, scaleA=sa, scaleB=sb, dtype=dtype), report=rb)
    inj = rb.view()
    F.clear_fault_plan()
    name = "bf16" if dtype == F.BF16 else "fp8"
    # flips the verification did not see, and flips seen on one side only
    # (a change between the row and the column threshold: classified as a
    # checksum fault): the change they made to the output, against the
    # thresholds of the flagged tiles
    kinds = {(r["tile_m"], r["tile_n"]): r["kind"] for r in inj.records}
    taus = sorted(max(r["tau_row"], r["tau_col"]) for r in inj.records)
    alpha_p = sa * sb
    missed, one_side = [], []
    for e in inj.echoes:
        kind = kinds.get((e["row"] // tm, e["col"] // tn))
        change = abs(alpha_p * (e["after"] - e["before"]))
        if kind is None:
            missed.append(change)
        elif kind == F.KIND_CHECKSUM_ONLY:
            one_side.append(change)
    # Guard-banded flips (the acceptance test of the fault-tolerance claim):
    # candidate flips of exponent and high fraction bits in distinct tiles;
    # their output change comes from the echoes of one run, the thresholds
    # of their entry's row and column from a probe run that plants unequal
    # faults on both checksum entries (the tile then recomputes, and its
    # record carries both thresholds); a flip is kept when its change is at
    # least 4 times the larger threshold, or not finite.
    need = -(-tiles // 64)
    cand = synth.bitflip_plan(synth.rng(wid, size, synth.STREAM_PLAN + 7), m, n, k, tm, tn,
                              min(4 * need, tiles))
    F.set_fault_plan(cand)
    rbc = F.ReportBuffer(record_capacity=len(cand) + 8, echo_capacity=len(cand))
    dC.copy_(dC0)
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, scaleA=sa, scaleB=sb, dtype=dtype), report=rbc)
    echoes = rbc.view().echoes
    probe = []
    for f in cand:
        probe.append(synth.Fault(f.row, f.col, 0, synth.ADD, 1.0e6,
                                 target=synth.TGT_ROW_CHECKSUM))
        probe.append(synth.Fault(f.row, f.col, 0, synth.ADD, 3.0e6,
                                 target=synth.TGT_COL_CHECKSUM))
    F.set_fault_plan(probe)
    rbp = F.ReportBuffer(record_capacity=len(cand) + 8, echo_capacity=len(probe))
    dC.copy_(dC0)
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, scaleA=sa, scaleB=sb, dtype=dtype), report=rbp)
    tau_of = {(r["tile_m"], r["tile_n"]): max(r["tau_row"], r["tau_col"])
              for r in rbp.view().records}
    accepted, band = [], 0
    for f, e in zip(cand, echoes):
        tau = tau_of.get((f.row // tm, f.col // tn))
        change = abs(alpha_p * (e["after"] - e["before"]))
        if tau is None or not e["applied"]:
            continue
        if not np.isfinite(e["after"]) or change >= 4.0 * tau:
            if len(accepted) < need:
                accepted.append(f)
        else:
            band += 1
    F.set_fault_plan(accepted)
    t_gb, _ = timed(torch, call(True), steps, warmup, reset, SETTLE_MS)
    rbg = F.ReportBuffer()
    dC.copy_(dC0)
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, scaleA=sa, scaleB=sb, dtype=dtype), report=rbg)
    gb = rbg.view()
    F.clear_fault_plan()
    guarded = {"faults_per_call": len(accepted), "candidates": len(cand),
               "rejected_by_guard_band": band,
               "kind": "FP32 bit flip (bits 19..30), guard-banded",
               "tflops": round(flops / (t_gb * 1e-3) / 1e12, 3),
               "overhead_pct": round(100.0 * (t_gb / t_plain - 1.0), 2),
               "detected": int(gb.detected), "corrected": int(gb.corrected),
               "recomputed": int(gb.recomputed), "checksum_only": int(gb.checksum_only)}
    # one-sided mode (column checksum only, tile recomputed on detection,
    # threshold norms from one pass over A and B)
    dC.copy_(dC0)
    rb1 = F.ReportBuffer()
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, abft=2, scaleA=sa, scaleB=sb, dtype=dtype),
              report=rb1)
    clean1 = rb1.view()
    t_one, _ = timed(torch, call(2), steps, warmup, reset, SETTLE_MS)
    tm1, tn1, bk1, _ = F.query_tiling_ex(dtype, m, n, k, abft=2)
    tiles1 = (-(-m // tm1)) * (-(-n // tn1))
    plan1 = synth.bitflip_plan(synth.rng(wid, size, synth.STREAM_PLAN), m, n, k, tm1, tn1,
                               -(-tiles1 // 64), bits=[27, 28, 29, 30])
    F.set_fault_plan(plan1)
    t_one_inj, _ = timed(torch, call(2), steps, warmup, reset, SETTLE_MS)
    rb1 = F.ReportBuffer()
    dC.copy_(dC0)
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, abft=2, scaleA=sa, scaleB=sb, dtype=dtype),
              report=rb1)
    inj1 = rb1.view()
    F.clear_fault_plan()
    one_sided = {
        "tflops": round(flops / (t_one * 1e-3) / 1e12, 3),
        "ms_per_call": round(t_one, 4),
        "abft_overhead_pct": round(100.0 * (t_one / t_plain - 1.0), 2),
        "tile": [tm1, tn1, bk1],
        "error_free_check": {"detected": int(clean1.detected), "max_ratio": clean1.max_ratio,
                             "tiles_verified": int(clean1.tiles_verified)},
        "injected": {"faults_per_call": len(plan1), "kind": "FP32 exponent bit flip",
                     "tflops": round(flops / (t_one_inj * 1e-3) / 1e12, 3),
                     "overhead_pct": round(100.0 * (t_one_inj / t_plain - 1.0), 2),
                     "detected": int(inj1.detected), "recomputed": int(inj1.recomputed)},
    }
    achieved = flops / (t_ft * 1e-3) / 1e12
    return {
        "tflops": round(flops / (t_ft * 1e-3) / 1e12, 3),
        "ms_per_call": round(t_ft, 4),
        "plain_tflops": round(flops / (t_plain * 1e-3) / 1e12, 3),
        "plain_tile": [tm0, tn, bk],
        "abft_overhead_pct": round(100.0 * (t_ft / t_plain - 1.0), 2),
        "plain_same_tile_tflops": round(flops / (t_plain_same * 1e-3) / 1e12, 3),
        "abft_overhead_same_tile_pct": round(100.0 * (t_ft / t_plain_same - 1.0), 2),
        "checksums_in_tiles": {"tflops": round(flops / (t_in_tile * 1e-3) / 1e12, 3),
                               "tile": [tm_in, tn, bk],
                               "abft_overhead_same_tile_pct":
                                   round(100.0 * (t_in_tile / t_plain_in - 1.0), 2)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[name],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK[name], 4),
                     "traffic": read_traffic("ftgemm_%s_8192_counters.txt" % name,
                                             ["ftgemm_lp.hip", "ftgemm_lp_ilp.hip",
                                              "ftgemm_norms.hip", "ftgemm_device.h"])
                     if size == 8192 else None},
        "injected": {"faults_per_call": len(plan), "kind": "FP32 exponent bit flip",
                     "tflops": round(flops / (t_inj * 1e-3) / 1e12, 3),
                     "overhead_pct": round(100.0 * (t_inj / t_plain - 1.0), 2),
                     "corrected": int(inj.corrected), "detected": int(inj.detected),
                     "checksum_only": int(inj.checksum_only),
                     "undetected_output_change": [float("%.4g" % d) for d in missed],
                     "one_side_output_change": [float("%.4g" % d) for d in one_side],
                     "median_threshold": float("%.4g" % taus[len(taus) // 2]) if taus else None},
        "injected_guard_banded": guarded,
        "error_free_check": {"detected": int(clean.detected), "max_ratio": clean.max_ratio,
                             "tiles_verified": int(clean.tiles_verified)},
        "max_rel_err_vs_fp64": max(errs),
        "config": "m=n=k=%d, normal(0,1) inputs%s, FP32 C, alpha=beta=1, tile %dx%dx%d" % (
            size, " with per-tensor scales" if name == "fp8" else "", tm, tn, bk),
        "one_sided": one_sided,
    }


def split_leg(torch, F, synth, steps, warmup, settle_ms=SETTLE_MS):
    """Small-output FP64 shapes (normal inputs, alpha = beta = 1): the split
    inner dimension and its verified reduction, one fault per 32 tiles."""
    out = []
    for (m, n, k) in ((16384, 16384, 256), (16384, 64, 16384), (1024, 1024, 32768)):
        g = torch.Generator(device="cuda").manual_seed(m + n + k)
        A = F.colmajor_empty(m, k, torch.float64).normal_(generator=g)
        B = F.colmajor_empty(k, n, torch.float64).normal_(generator=g)
        C0 = F.colmajor_empty(m, n, torch.float64).normal_(generator=g)
        C = C0.clone()
        reset = lambda: C.copy_(C0)
        flops = 2.0 * m * n * k
        slices = F.query_tiling(F.F64, m, n, k)[3]
        F.clear_fault_plan()
        t_ft, _ = timed(torch, lambda: F.gemm_ex(F.make_desc(A, B, C, 1.0, 1.0)), steps, warmup,
                        reset, SETTLE_MS)
        t_pl, _ = timed(torch, lambda: F.gemm_ex(F.make_desc(A, B, C, 1.0, 1.0, abft=False)),
                        steps, warmup, reset, SETTLE_MS)
        tiles = (-(-m // 128)) * (-(-n // 128))
        plan = synth.additive_plan(synth.rng(50, k, synth.STREAM_PLAN), m, n, k, 128, 128,
                                   max(1, tiles // 32), synth.log_magnitude((k + 1.0) ** 0.5))
        F.set_fault_plan(plan)
        t_inj, _ = timed(torch, lambda: F.gemm_ex(F.make_desc(A, B, C, 1.0, 1.0)), steps, warmup,
                         reset, SETTLE_MS)
        rb = F.ReportBuffer()
        reset()
        F.gemm_ex(F.make_desc(A, B, C, 1.0, 1.0), report=rb)
        v = rb.view()
        F.clear_fault_plan()
        out.append({"shape": [m, n, k], "slices": slices,
                    "tflops": round(flops / (t_ft * 1e-3) / 1e12, 3),
                    "plain_tflops": round(flops / (t_pl * 1e-3) / 1e12, 3),
                    "abft_overhead_pct": round(100.0 * (t_ft / t_pl - 1.0), 2),
                    "injected": {"faults_per_call": len(plan),
                                 "overhead_pct": round(100.0 * (t_inj / t_pl - 1.0), 2),
                                 "corrected": int(v.corrected), "detected": int(v.detected)}})
        del A, B, C, C0
        torch.cuda.empty_cache()
    return out


def batched_leg(torch, F, synth, np, dtype, steps, warmup, settle_ms=SETTLE_MS):
    """512 problems, m, n, k log-uniform in [64, 2048], U[-1,1], alpha = 1,
    beta = 0: one persistent launch replayed from a graph against the loop
    of per-problem launches; truncated Poisson(1) faults per problem."""
    shapes = synth.batched_shapes(70, dtype, 512)
    g = torch.Generator(device="cuda").manual_seed(70 + dtype)
    tdt = torch.float64 if dtype == F.F64 else torch.bfloat16
    cdt = torch.float64 if dtype == F.F64 else torch.float32
    tens, descs, descs_plain = [], [], []
    flops = 0.0
    for (m, n, k) in shapes:
        A = F.colmajor_empty(m, k, cdt).uniform_(-1, 1, generator=g).to(tdt)
        B = F.colmajor_empty(k, n, cdt).uniform_(-1, 1, generator=g).to(tdt)
        C = F.colmajor_empty(m, n, cdt).zero_()
        tens.append((A, B, C))
        descs.append(F.make_desc(A, B, C, 1.0, 0.0, dtype=dtype))
        descs_plain.append(F.make_desc(A, B, C, 1.0, 0.0, abft=False, dtype=dtype))
        flops += 2.0 * m * n * k
    F.clear_fault_plan()
    F.gemm_batched(descs)  # tunes the tiles and the schedule, captures the graph
    rows = F.batch_tiling(descs)
    t_b, _ = timed(torch, lambda: F.gemm_batched(descs), steps, warmup, settle_ms=SETTLE_MS)
    F.gemm_batched(descs_plain)
    rows_plain = F.batch_tiling(descs_plain)
    t_bp, _ = timed(torch, lambda: F.gemm_batched(descs_plain), steps, warmup, settle_ms=SETTLE_MS)
    per_choice = {}
    if dtype != F.F64:
        # each tile choice fixed by the table, fault-tolerant against plain
        for label, mstar in (("all_128", 10 ** 9), ("256_from_512", 512),
                             ("256_from_256", 256)):
            def both():
                F.gemm_batched(descs)
                a, _ = timed(torch, lambda: F.gemm_batched(descs), steps, warmup,
                             settle_ms=SETTLE_MS)
                F.gemm_batched(descs_plain)
                b, _ = timed(torch, lambda: F.gemm_batched(descs_plain), steps, warmup,
                             settle_ms=SETTLE_MS)
                return a, b
            a, b = with_table(F, "batch_mstar %d\n" % mstar, both)
            per_choice[label] = {"tflops": round(flops / (a * 1e-3) / 1e12, 3),
                                 "plain_tflops": round(flops / (b * 1e-3) / 1e12, 3),
                                 "abft_overhead_pct": round(100.0 * (a / b - 1.0), 2)}
    t_l, _ = timed(torch, lambda: F.gemm_batched(descs, loop=True), max(2, steps // 4), 1)
    gp = synth.rng(70, dtype, synth.STREAM_PLAN)
    plan = []
    for p, (m, n, k) in enumerate(shapes):
        tiles = (-(-m // rows[p])) * (-(-n // 128))
        cnt = min(synth.truncated_poisson(gp, 1.0, 3), tiles)
        for f in synth.additive_plan(gp, m, n, k, rows[p], 128, cnt,
                                     synth.log_magnitude((k / 9.0) ** 0.5, 1.0, 6.0)):
            f.problem = p
            plan.append(f)
    F.set_fault_plan(plan)
    t_bi, _ = timed(torch, lambda: F.gemm_batched(descs), steps, warmup, settle_ms=SETTLE_MS)
    reps = [F.ReportBuffer(record_capacity=8, echo_capacity=8) for _ in shapes]
    F.gemm_batched(descs, reps)
    views = [r.view() for r in reps]
    F.clear_fault_plan()
    out = {"problems": len(shapes), "gflop_per_call": round(flops / 1e9, 1),
            "tile_rows_256": rows.count(256), "tile_rows_256_plain": rows_plain.count(256),
            "tflops": round(flops / (t_b * 1e-3) / 1e12, 3),
            "ms_per_call": round(t_b, 4),
            "plain_tflops": round(flops / (t_bp * 1e-3) / 1e12, 3),
            "abft_overhead_pct": round(100.0 * (t_b / t_bp - 1.0), 2),
            "loop_tflops": round(flops / (t_l * 1e-3) / 1e12, 3),
            "speedup_vs_loop": round(t_l / t_b, 2),
            "injected": {"faults_per_call": len(plan),
                         "overhead_pct": round(100.0 * (t_bi / t_bp - 1.0), 2),
                         "corrected": sum(int(v.corrected) for v in views),
                         "detected": sum(int(v.detected) for v in views)}}
    if per_choice:
        out["per_tile_choice"] = per_choice
    return out


PROFILE_KINDS = ["f64", "f64-plain", "f64-unfused", "f64-weighted", "bf16", "bf16-plain",
                 "bf16-fused", "fp8", "fp8-plain", "fp8-plain-128", "fp8-fused", "copy"]


def profile_run(kind, size, calls=3):
    """A short fixed workload for counter passes: `calls` GEMMs of one format
    at size^3 (alpha = beta = 1, no report), or, for `copy`, device copies of
    a 512 MiB buffer (the scale of the traffic counters).  Kinds: the
    fault-tolerant call (f64, bf16, fp8), the same kernel with checksums
    compiled out on its default tile (-plain) and, for FP8, on the 128-row
    tile of the call that forms its checksums in the tiles (fp8-plain-128),
    the unfused and
    weighted FP64 modes, and the low-precision fault tolerance with every operand checksum
    formed in the tiles from the staged operands (-fused: the entry point
    that allocates nothing, which takes no pass before the product)."""
    import torch
    from paper_2305_02444_amd import ftgemm as F
    torch.cuda.set_device(0)
    if kind == "copy":
        src = torch.empty(64 << 20, dtype=torch.float64, device="cuda").uniform_()
        dst = torch.empty_like(src)
        for _ in range(calls):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copy of %d bytes x %d" % (src.numel() * 8, calls), flush=True)
        return
    m = n = k = size
    g = torch.Generator(device="cuda").manual_seed(5)
    base = kind.split("-")[0]
    abft = ({"plain": 0, "unfused": 3, "weighted": 4}.get(kind.split("-")[1], 1)
            if "-" in kind else 1)
    call = F.gemm_ex_noalloc if kind.endswith("-fused") else F.gemm_ex
    if base == "f64":
        A = F.colmajor_empty(m, k, torch.float64)
        B = F.colmajor_empty(k, n, torch.float64)
        A.uniform_(-1, 1, generator=g)
        B.uniform_(-1, 1, generator=g)
        Cm = F.colmajor_empty(m, n, torch.float64).uniform_(-1, 1, generator=g)
        d = F.make_desc(A, B, Cm, 1.0, 1.0, abft=abft)
    else:
        dt = torch.bfloat16 if base == "bf16" else torch.float8_e4m3fn
        A = F.colmajor_empty(m, k, torch.float32).normal_(generator=g)
        B = F.colmajor_empty(k, n, torch.float32).normal_(generator=g)
        scale = 1.0 if kind == "bf16" else 1.0 / 64.0
        A8, B8 = (A / scale).to(dt), (B / scale).to(dt)
        del A, B
        Cm = F.colmajor_empty(m, n, torch.float32).normal_(generator=g)
        code = F.BF16 if base == "bf16" else F.FP8_E4M3
        if base == "fp8":
            A8, B8 = A8.view(torch.uint8), B8.view(torch.uint8)
        d = F.make_desc(A8, B8, Cm, 1.0, 1.0, abft=abft, scaleA=scale, scaleB=scale, dtype=code)
    F.clear_fault_plan()

    def run():
        for _ in range(calls):
            call(d)
        torch.cuda.synchronize()
    if kind == "fp8-plain-128":
        with_table(F, "tile %d 0 128\n" % F.FP8_E4M3, run)
    else:
        run()
    print("%s GEMM %d^3 x %d" % (kind, size, calls), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-low-precision", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--profile", choices=PROFILE_KINDS)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the fault-tolerant GEMM shards by output tile with "
              "no cross-GPU exchange, and this build runs on a single MI355X; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        profile_run(args.profile, args.size)
        return

    import numpy as np
    import torch

    from paper_2305_02444_amd import ftgemm as F
    from paper_2305_02444_amd import synth

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    F.lib()  # fails loudly when the library is missing

    m = n = k = args.size
    flops = 2.0 * m * n * k
    A, B, Cin = synth.operands(20, m, m, n, k, "uniform")
    dA, dB = F.to_device(A), F.to_device(B)
    dC0 = F.to_device(Cin)
    dC = dC0.clone()

    def call(abft):
        d = F.make_desc(dA, dB, dC, 1.0, 1.0, abft=abft)
        return lambda: F.gemm_ex(d)

    # correctness of the timed configuration (report-bearing, not timed)
    F.clear_fault_plan()
    rb = F.ReportBuffer()
    dC.copy_(dC0)
    F.gemm(dA, dB, dC, 1.0, 1.0, report=rb)
    clean = rb.view()

    F.clear_fault_plan()
    reset = lambda: dC.copy_(dC0)
    t_ft, t_ft_wall = timed(torch, call(True), args.steps, args.warmup, reset)
    t_plain, _ = timed(torch, call(False), args.steps, args.warmup, reset)

    tiles = (m // 128) * (n // 128)
    g = synth.rng(20, m, synth.STREAM_PLAN)
    sigma = float(np.sqrt(k / 9.0 + 1.0 / 3.0))
    plan = synth.additive_plan(g, m, n, k, 128, 128, -(-tiles // 64), synth.log_magnitude(sigma))
    F.set_fault_plan(plan)
    t_inj, _ = timed(torch, call(True), args.steps, args.warmup, reset)
    rb = F.ReportBuffer()
    reset()
    F.gemm(dA, dB, dC, 1.0, 1.0, report=rb)
    inj = rb.view()
    # two faults in each of 64 other tiles, in different rows and columns
    # (corrected by pairing the flagged rows and columns)
    plan2 = synth.crossing_pairs_plan(synth.rng(20, m + 1, synth.STREAM_PLAN), m, n, k, 128, 128,
                                      -(-tiles // 64), synth.log_magnitude(sigma))
    F.set_fault_plan(plan2)
    t_pairs, _ = timed(torch, call(True), args.steps, args.warmup, reset)
    rb = F.ReportBuffer()
    reset()
    F.gemm(dA, dB, dC, 1.0, 1.0, report=rb)
    inj2 = rb.view()
    F.set_fault_plan(plan)
    # the unfused ablation (separate checksum passes around the plain
    # GEMM, detection only) under the same faults, then error-free
    rb = F.ReportBuffer()
    reset()
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, abft=3), report=rb)
    inj_uf = rb.view()
    t_uf_inj, _ = timed(torch, call(3), args.steps, args.warmup, reset)
    F.clear_fault_plan()
    dC.copy_(dC0)
    rb = F.ReportBuffer()
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, abft=3), report=rb)
    clean_uf = rb.view()
    t_uf, _ = timed(torch, call(3), args.steps, args.warmup, reset)
    # the weighted mode (also a weighted row checksum per column): error-free,
    # then two equal faults in each of 64 other tiles, in different rows and
    # columns (paired by the weighted checksums; the plain mode recomputes)
    dC.copy_(dC0)
    rb = F.ReportBuffer()
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, abft=4), report=rb)
    clean_w = rb.view()
    t_w, _ = timed(torch, call(4), args.steps, args.warmup, reset)
    plan3 = synth.crossing_pairs_plan(synth.rng(20, m + 2, synth.STREAM_PLAN), m, n, k, 128, 128,
                                      -(-tiles // 64), synth.log_magnitude(sigma, 0.0, 2.0),
                                      equal=True)
    F.set_fault_plan(plan3)
    t_w_inj, _ = timed(torch, call(4), args.steps, args.warmup, reset)
    rb = F.ReportBuffer()
    reset()
    F.gemm_ex(F.make_desc(dA, dB, dC, 1.0, 1.0, abft=4), report=rb)
    inj_w = rb.view()
    rb = F.ReportBuffer()
    reset()
    F.gemm(dA, dB, dC, 1.0, 1.0, report=rb)
    inj_w1 = rb.view()
    F.clear_fault_plan()

    value = flops / (t_ft * 1e-3) / 1e12
    achieved = value
    traffic = read_traffic("ftgemm_f64_8192_counters.txt",
                           ["ftgemm_f64.hip", "ftgemm_device.h"]) if m == 8192 else None
    out = {
        "metric": "FT-GEMM TFLOP/s and ABFT overhead vs plain GEMM at 8192^3 FP64/BF16",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_ft, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fault-tolerant DGEMM, FP64, m=n=k=%d, column-major N/N, "
                               "alpha=beta=1, inputs uniform[-1,1], error-free" % m,
                   "m": m, "n": n, "k": k, "tile": list(F.query_tiling(F.F64, m, n, k)[:3])},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK["f64"], 4),
                     "traffic": traffic},
        "plain_tflops": round(flops / (t_plain * 1e-3) / 1e12, 3),
        "abft_overhead_pct": round(100.0 * (t_ft / t_plain - 1.0), 2),
        "injected": {"faults_per_call": len(plan),
                     "tflops": round(flops / (t_inj * 1e-3) / 1e12, 3),
                     "overhead_pct": round(100.0 * (t_inj / t_plain - 1.0), 2),
                     "corrected": int(inj.corrected), "detected": int(inj.detected)},
        "injected_two_per_tile": {"faults_per_call": len(plan2),
                                  "tiles": len(plan2) // 2,
                                  "tflops": round(flops / (t_pairs * 1e-3) / 1e12, 3),
                                  "overhead_pct": round(100.0 * (t_pairs / t_plain - 1.0), 2),
                                  "corrected": int(inj2.corrected),
                                  "recomputed": int(inj2.recomputed),
                                  "detected": int(inj2.detected)},
        "error_free_check": {"detected": int(clean.detected), "max_ratio": clean.max_ratio,
                             "tiles_verified": int(clean.tiles_verified)},
        "unfused": {"tflops": round(flops / (t_uf * 1e-3) / 1e12, 3),
                    "ms_per_call": round(t_uf, 4),
                    "abft_overhead_pct": round(100.0 * (t_uf / t_plain - 1.0), 2),
                    "error_free_check": {"detected": int(clean_uf.detected),
                                         "max_ratio": clean_uf.max_ratio,
                                         "tiles_verified": int(clean_uf.tiles_verified)},
                    "injected": {"faults_per_call": len(plan),
                                 "overhead_pct": round(100.0 * (t_uf_inj / t_plain - 1.0), 2),
                                 "detected": int(inj_uf.detected)}},
        "weighted": {"tflops": round(flops / (t_w * 1e-3) / 1e12, 3),
                     "abft_overhead_pct": round(100.0 * (t_w / t_plain - 1.0), 2),
                     "error_free_check": {"detected": int(clean_w.detected),
                                          "max_ratio": clean_w.max_ratio},
                     "injected_equal_pairs": {
                         "faults_per_call": len(plan3),
                         "tflops": round(flops / (t_w_inj * 1e-3) / 1e12, 3),
                         "overhead_pct": round(100.0 * (t_w_inj / t_plain - 1.0), 2),
                         "corrected": int(inj_w.corrected),
                         "recomputed": int(inj_w.recomputed),
                         "mode_1_corrected": int(inj_w1.corrected),
                         "mode_1_recomputed": int(inj_w1.recomputed)}},
    }
    if not args.no_low_precision:
        del dA, dB, dC, dC0
        torch.cuda.empty_cache()
        lp = {}
        for dt in (F.BF16, F.FP8_E4M3):
            lp["bf16" if dt == F.BF16 else "fp8"] = lp_leg(torch, F, synth, np, dt, m,
                                                          args.steps, args.warmup)
            print("# leg done: %s" % ("bf16" if dt == F.BF16 else "fp8"), file=sys.stderr,
                  flush=True)
        lp["bf16"]["speedup_vs_fp64"] = round(lp["bf16"]["tflops"] / value, 2)
        lp["fp8"]["speedup_vs_fp64"] = round(lp["fp8"]["tflops"] / value, 2)
        out["low_precision"] = lp
    if not args.no_split:
        out["split_k"] = split_leg(torch, F, synth, args.steps, args.warmup)
        print("# leg done: split", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = {}
        for dt in (F.F64, F.BF16):
            out["batched"]["f64" if dt == F.F64 else "bf16"] = batched_leg(
                torch, F, synth, np, dt, args.steps, args.warmup)
            print("# leg done: batched", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, Cin, m, n, k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
