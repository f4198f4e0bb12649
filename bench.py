"""Benchmark: Vegas events/s on one MI355X, FP32-eval at matched sigma against
FP64, with per-iteration latency percentiles, the iteration kernel's ALU
roofline, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload gauss8d]
                    [--no-cpu] [--no-serving]

One step is one whole integration of the workload: grid reset to uniform,
n_iter iterations (draw, map, integrand, moments, histogram) with a grid
refinement after each but the last, and the inverse-variance combination.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes, one VALU
# instruction per lane per clock at 2.4 GHz (a wave64 instruction occupies its
# SIMD for 4 clocks) = 3.93e13 lane-instructions/s. Measured on gfx950: the
# 32x32->64 multiply-add and binary64 fma issue at about this rate.
PEAK_VALU_SLOTS = 256 * 64 * 2.4e9
PEAK_FP32_FLOPS = 157.3e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_valu_per_event(dim: int, prec: int, fid: int = 2):
    """VALU lane-instructions of one event: the minimal gfx950 instruction
    sequence of the method, counted operation by operation, one issue slot
    per instruction (issued instructions are measured separately with
    SQ_INSTS_VALU; the difference is loop and compiler overhead). Counted
    for the Gaussian and the LO toy in both precisions and for RAMBO 2->4 in
    FP32-eval (its configured precision); None otherwise. Binary64 square
    roots and divisions count as the compiler's correctly rounded sequences
    for gfx950: square root 18 (reciprocal square root 1; the scaling of
    small arguments: compare, two selects, two ldexp = 5; Newton steps: 7
    fmas and 2 products = 9; the special-case class test and two selects =
    3), division 11 (two scale steps, reciprocal, 5 fmas, a product, the
    fused correction and the fix-up).

    Common to every integrand:
      Philox4x32-10 per 4 dimensions: 10 rounds x (2 v_mad_u64_u32 + 2
        three-input xor v_bitop3) = 40, less round 1's product of the
        workgroup-uniform counter word t (scalar unit) = 39 for the first
        block; later blocks of the same event share round 1's product of the
        event index and the part of round 2 that does not depend on the
        block number: 35 each
      event index and loop: 64-bit add (1) + compare (1) = 2
      map per dimension: 32x32->64 product giving bin and remainder (1), LDS
        histogram address (1; the grid record is read with the bin as a
        buffer index) = 2, then
        FP64: remainder converted (1), x = fma (1), Jacobian factor nb Delta
          and product (2), the product of the first dimension folded = 4 per
          dimension - 1
        FP32: the factor 1 + remainder 2^-23 from the remainder's bits
          (alignbit, 1), x = fma (1) = 2 per dimension; log2 J per pair of
          dimensions: the product of their widths (1), its scaling by nb^2
          (1), log2 (1) and the sum (1) = 4 per pair, the first sum folded;
          an unpaired last dimension: scaling by nb, log2 and sum (3)
      non-finite check (class, two selects, count select + add) = 5;
      moments (w^2, two adds) = 3
      FP32 weight: w = f 2^(log2 J + log2 f) with a binary64 exponent:
        floor, subtract, exp2, two converts, ldexp = 6, plus the binary64
        product by f and its conversion (2) where f is not a constant 1
    Gaussian: per dimension subtract + fma = 2; FP32 log2 f = fma (1) and
      its add to log2 J (1); FP64 exp of the sum (lower clamp, Cody-Waite
      reduction: product, rounding and two fmas; degree-13 Taylor polynomial
      by Horner's rule: 13 fmas; convert and ldexp = 19) + the fma forming
      its argument (1) and the product by J (1) = 21
    LO toy (FP32): c = fma (1); s^ = x1 x2 S (2); 1 - x1, 1 - x2 (2); their
      product and its cube (3); rsqrt of x1 x2 and its product (2);
      s^ - m^2 (1); (dm^2 + (m G)^2) s^ (2); 1 + c^2 (1), reciprocal (1) and
      three products (3); cut compare and select (2) = 20
    LO toy (FP64): phi is unused, so its point is never formed (the map's
      conversion and fma of that dimension, -2); c = fma (1); x1 x2 and s^
      (2); the cut sqrt(s^) > 20: square root (18), compare (1) and the
      final two-word select (2); (1 - x1)(1 - x2) (3); s^ - m^2 (1); the
      numerator y^3 (1 + c^2) norm: square, cube, fma, two products (5); the
      denominator sqrt(x1 x2) (dm^2 + (m G)^2) s^: square root (18), fma and
      two products (3); the division (11); the product by J (1)
      = 19 + 2 x 18 + 11 = 66
    RAMBO 2->4 (FP32), per particle: cos theta = min(fma, 1) (2); sin theta
      = sqrt(max(fma, 0)) (3); sin, cos (2); energy -ln(u u') = max(-log2 x
      ln 2, 0) with the product (4); three momentum components (3); then
      the four sums of the four particles (12); mass^2 (4), rsqrt (1), boost
      vector (3), gamma (1), 1/(1 + gamma) (2), the cut on the unscaled
      invariants, c M^2 / 2s (1); per particle the boost of the unscaled
      momenta: b.q (3), q0 + a b.q (1), E (1), three components (3); the
      four cyclic invariants of the unscaled momenta (dot product 4, cut
      compare 1 each; three products); the weight (W / 16 s^4) M^8 / prod
      (M^4, M^8, constant, reciprocal, product, select: 6) = 145
    """
    blocks = (dim + 3) // 4
    common = 39 + 35 * (blocks - 1) + 2 + 2 * dim + 5 + 3
    if prec == 1:
        common += 2 * dim + 4 * (dim // 2) - 1 + 3 * (dim % 2)
    else:
        common += 4 * dim - 1
    if fid == 2:
        return common + 2 * dim + (2 + 6 if prec == 1 else 21)
    if prec != 1 and not (fid == 3 and dim == 4):
        return None
    if fid == 3 and dim == 4 and prec != 1:
        return common - 2 + 19 + 2 * 18 + 11
    if fid == 3 and dim == 4:
        return common + 20 + 6 + 2
    if fid == 4 and dim == 16:
        return common + 145 + 6 + 2
    return None


def fp32_flops_per_event(dim: int) -> float:
    """Binary32 floating-point operations of the FP32-eval Gaussian per event
    (fma = 2): map fma (2), width multiply (1), subtract and fma (3) per
    dimension, and the weight's fma, subtract, exp2 (4)."""
    return dim * 6 + 4


# The configured throughput workloads measured by a default run.
CONFIG_WORKLOADS = ("gauss8d", "lo_toy", "rambo24")

KERNEL_SOURCES = ("vegas_math.hpp", "vegas_device.hpp", "vegas_iterate.hpp", "vegas_types.hpp", "iter_gauss.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_iterate_gauss8d_fp32eval.md")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_09341_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch of the iteration kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None if the kernel sources changed since those counters were taken."""
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel source sha256\[:16\]: ([0-9a-f]{16})", text)
    m_b = re.search(r"HBM traffic per launch \(bytes\): ([0-9.e+]+)", text)
    if not m_hash or not m_b or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_b.group(1))


def optional(name, fn, *args):
    """A section of the report beside the headline: an exception in it is
    recorded in the report (and logged) instead of ending the run."""
    try:
        return fn(*args)
    except Exception as e:  # noqa: BLE001 - recorded, not swallowed
        log(f"{name} failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def measure(vg, W, wl, steps, warmup, latency_reps):
    """Both precisions of one workload: whole runs replayed from the captured
    iteration graph (throughput), the same runs launched one by one with HIP
    events around every iteration kernel on the handle's stream (kernel
    time), and synchronous single iterations (latency)."""
    import torch

    def make(prec):
        h = vg.vegas_create(wl.dim, wl.nb)
        vg.vegas_set_params(h, wl.fid, wl.params)
        vg.vegas_set_precision(h, prec)
        return h

    def step(h):
        vg.vegas_reset(h)
        I_t, s_t = vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
        return I_t, s_t, vg.vegas_result(h)

    results = {}
    for prec in (W.FP32_EVAL, W.FP64):
        log(f"{wl.name} prec={prec}: {warmup} warmup + {steps} timed steps")
        h = make(prec)
        for _ in range(warmup):
            step(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            I_t, s_t, comb = step(h)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        vg.vegas_timing(h, True, True)
        per_step = []  # average iteration-kernel time of each step
        k_ms = k_n = 0
        t1 = time.perf_counter()
        for _ in range(steps):
            step(h)
            ms, n = vg.vegas_timing(h, True, True)
            per_step.append(ms / max(n, 1))
            k_ms += ms
            k_n += n
        torch.cuda.synchronize()
        dt_eager = time.perf_counter() - t1
        vg.vegas_timing(h, False)
        # per-iteration latency: one synchronous vegas_iterate (launch, kernels,
        # result in mapped host memory, synchronisation) on the adapted grid
        lat = []
        for _ in range(latency_reps):
            a = time.perf_counter()
            vg.vegas_iterate(h, wl.fid, wl.n_events, wl.seed)
            lat.append(time.perf_counter() - a)
        log(f"{wl.name} prec={prec}: {dt / steps * 1e3:.3f} ms/step (eager "
            f"{dt_eager / steps * 1e3:.3f}), kernel {k_ms / max(k_n, 1) * 1e3:.1f} us, "
            f"latency p50 {pct(lat, 50) * 1e3:.3f} ms")
        results[prec] = dict(dt=dt, dt_eager=dt_eager, I_t=I_t, s_t=s_t, comb=comb, k_ms=k_ms,
                             k_n=k_n, lat=lat, per_step=per_step)
        del h
    return results


def workload_summary(W, wl, res, steps):
    """events/s of both precisions, matched sigma, and the iteration
    kernel's roofline fraction (algorithmic VALU count x events per launch /
    average launch time / VALU issue peak)."""
    r32, r64 = res[W.FP32_EVAL], res[W.FP64]
    ev = wl.n_events * wl.n_iter * steps
    I32, s32, _ = r32["comb"]
    I64, s64, _ = r64["comb"]
    out = {"events_per_iteration": wl.n_events, "iterations": wl.n_iter, "dim": wl.dim,
           "n_bins": wl.nb}
    for prec, key in ((W.FP32_EVAL, "fp32_eval"), (W.FP64, "fp64")):
        r = res[prec]
        k_s = r["k_ms"] / max(r["k_n"], 1) * 1e-3
        slots = alg_valu_per_event(wl.dim, prec, wl.fid)
        out[key] = {"events_per_s": ev / r["dt"], "ms_per_step": r["dt"] / steps * 1e3,
                    "kernel_us": k_s * 1e6,
                    "kernel_us_p10_p50_p90": [pct(r["per_step"], q) * 1e3 for q in (10, 50, 90)],
                    "valu_per_event_algorithmic": slots,
                    "frac": slots * wl.n_events / k_s / PEAK_VALU_SLOTS if slots else None,
                    "latency_ms_p50_p99": [pct(r["lat"], 50) * 1e3, pct(r["lat"], 99) * 1e3],
                    "I": r["comb"][0], "sigma": r["comb"][1]}
        if not slots:
            out[key]["frac_note"] = ("no algorithmic count for this binary64 loop (the workload's "
                                     "configured precision is FP32-eval; its compiled loop carries "
                                     "register-pressure overhead, SGPR spills restored with "
                                     "v_readlane and 64-bit moves, that an operation count would "
                                     "not hold); reported by time")
    out["sigma_ratio"] = s32 / s64
    out["matched"] = abs(s32 / s64 - 1.0) < 1e-2
    out["fp32_minus_fp64_over_sigma"] = (I32 - I64) / s64
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="gauss8d")
    ap.add_argument("--latency-reps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads, the events_limit sweep, the run-time "
                         "integrand and the small-workload latency (so a kernel trace sees only "
                         "the timed launches of one workload)")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy three times, so that a "
                         "counter run can scale FETCH_SIZE/WRITE_SIZE by a known size")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    from paper_2010_09341_amd import workloads as W
    wl = W.WORKLOADS[args.workload]
    others = [] if args.no_extras else [n for n in CONFIG_WORKLOADS if n != wl.name]
    # The oracle on every host core runs first, in processes forked before
    # this process imports torch or makes any HIP call (the HIP runtime is not
    # fork-safe).
    cpu_all = None
    if not args.no_cpu:
        cpu_all = {name: optional(f"{name} oracle on all cores", cpu_baseline_all_cores,
                                  W.WORKLOADS[name])
                   for name in [wl.name] + others}

    from paper_2010_09341_amd import vegas as vg
    if not os.path.exists(vg.LIB_PATH):  # built already unless nothing is
        from paper_2010_09341_amd import build as _build
        _build.build()

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    events_per_step = wl.n_events * wl.n_iter

    # The other workloads first: by the time the headline workload's warmup
    # steps start, the GPU has left its idle clocks (measured: right after a
    # cold start the first 20 timed 8-D steps take 0.64 ms each, every later
    # 20 take 0.58 ms).
    per_other = {}
    t_gpu0 = time.perf_counter()
    def other_workload(o):
        res_o = measure(vg, W, o, args.steps, min(args.warmup, 5), min(args.latency_reps, 100))
        summary = workload_summary(W, o, res_o, args.steps)
        summary["fp64_I_t"] = [float(v) for v in res_o[W.FP64]["I_t"]]
        return summary

    for name in others:
        per_other[name] = optional(name, other_workload, W.WORKLOADS[name])
    gpu_busy_before_s = time.perf_counter() - t_gpu0

    results = measure(vg, W, wl, args.steps, args.warmup, args.latency_reps)
    r32, r64 = results[W.FP32_EVAL], results[W.FP64]
    value = events_per_step * args.steps / r32["dt"]
    value64 = events_per_step * args.steps / r64["dt"]
    I32, s32, _ = r32["comb"]
    I64, s64, _ = r64["comb"]
    matched = abs(s32 / s64 - 1.0) < 1e-2

    # roofline of the iteration kernel (FP32-eval), from HIP events around
    # every launch of it inside the timed steps
    k_avg_s = r32["k_ms"] / max(r32["k_n"], 1) * 1e-3
    slots = alg_valu_per_event(wl.dim, W.FP32_EVAL, wl.fid)
    achieved = slots * wl.n_events / k_avg_s if slots else None
    k64_avg_s = r64["k_ms"] / max(r64["k_n"], 1) * 1e-3
    slots64 = alg_valu_per_event(wl.dim, W.FP64, wl.fid)

    per_workload = {wl.name: workload_summary(W, wl, results, args.steps), **per_other}

    out = {
        "metric": "Vegas events/sec at matched sigma (FP32-eval vs FP64) on 1 GPU; "
                  "p50/p99 latency",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "gpu_busy_before_warmup_s": round(gpu_busy_before_s, 3),
        "ms_per_step": r32["dt"] / args.steps * 1e3,
        "ms_per_step_eager_launches": r32["dt_eager"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-eval/f64-accumulate",
        "data": "synthetic",
        "config": {
            "workload": f"{wl.name}: {wl.note}; Philox seed {wl.seed}, refinement alpha "
                        f"{wl.alpha}",
            "dim": wl.dim, "n_bins": wl.nb, "events_per_iteration": wl.n_events,
            "iterations": wl.n_iter, "events_per_step": events_per_step,
            "parallelism": "single GPU",
        },
        "matched_sigma": {"fp32_eval": {"I": I32, "sigma": s32},
                          "fp64": {"I": I64, "sigma": s64, "events_per_s": value64,
                                   "ms_per_step": r64["dt"] / args.steps * 1e3},
                          "sigma_ratio": s32 / s64, "matched": matched,
                          "fp32_minus_fp64_over_sigma": (I32 - I64) / s64,
                          "figure_of_merit_fp32": 1.0 / (s32 ** 2 * r32["dt"] / args.steps),
                          "figure_of_merit_fp64": 1.0 / (s64 ** 2 * r64["dt"] / args.steps)},
        "latency_ms": {
            "what": "one synchronous vegas_iterate of the workload's events/iteration",
            "fp32_eval": {"p50": pct(r32["lat"], 50) * 1e3, "p99": pct(r32["lat"], 99) * 1e3},
            "fp64": {"p50": pct(r64["lat"], 50) * 1e3, "p99": pct(r64["lat"], 99) * 1e3},
        },
        "roofline": {
            "bound": "alu",
            "kernel": f"k_iterate<{wl.dim},{wl.name},fp32-eval>",
            "achieved": achieved / 1e12 if achieved else None,
            "peak": PEAK_VALU_SLOTS / 1e12,
            "unit": "T VALU lane-instructions/s",
            "frac": achieved / PEAK_VALU_SLOTS if achieved else None,
            "traffic": traffic_from_profile() if wl.name == "gauss8d" else None,
            "valu_per_event_algorithmic": slots,
            "avg_launch_us": k_avg_s * 1e6,
            "launch_us_p10_p50_p90": [pct(r32["per_step"], q) * 1e3 for q in (10, 50, 90)],
            "launches": r32["k_n"],
            "fp32_flop_frac_of_157TF": (fp32_flops_per_event(wl.dim) * wl.n_events / k_avg_s
                                        / PEAK_FP32_FLOPS) if wl.fid == W.F_GAUSS else None,
            "fp64_kernel": {"avg_launch_us": k64_avg_s * 1e6,
                            "launch_us_p10_p50_p90": [pct(r64["per_step"], q) * 1e3
                                                      for q in (10, 50, 90)],
                            "frac": (slots64 * wl.n_events / k64_avg_s / PEAK_VALU_SLOTS)
                            if slots64 else None},
            # every configured throughput workload (8-D Gaussian, LO toy, RAMBO
            # 2->4), both precisions, with the iteration kernel's fraction of
            # the VALU issue peak
            "workloads": per_workload,
        },
    }
    if not args.no_extras:
        out["latency_ms"]["gauss4d_fp64"] = optional("gauss4d latency", small_latency, vg, W,
                                                     args.latency_reps)
        if wl.name == "gauss8d":
            out["one_gpu_share_of_8"] = optional("one GPU share", gpu_share, vg, W, wl,
                                                 max(20, args.steps // 4))
            # the same share of the other configured workloads (N/8 events
            # per iteration each)
            if isinstance(out["one_gpu_share_of_8"], dict) and others:
                out["one_gpu_share_of_8"]["workloads"] = {
                    name: optional(f"{name} one GPU share", gpu_share, vg, W, W.WORKLOADS[name],
                                   max(5, args.steps // 4))
                    for name in others}
        out["events_limit_sweep"] = optional("events_limit sweep", events_limit_sweep, vg, W, wl,
                                             max(3, args.steps // 4))
    if wl.fid == W.F_GAUSS and not args.no_extras:
        out["user_integrand"] = optional(
            "run-time integrand", user_integrand_section, vg, W, wl, max(3, args.steps // 4),
            {W.FP32_EVAL: value, W.FP64: value64})
    closed = W.gauss_closed_form(wl.dim, wl.params[0]) if wl.fid == W.F_GAUSS else None
    if closed is not None:
        out["closed_form"] = {"I": closed, "fp32_pull": (I32 - closed) / s32,
                              "fp64_pull": (I64 - closed) / s64}

    if not args.no_cpu:
        log("cpu baseline (oracle)")

        def cpu_section():
            cb = cpu_baseline(wl, r64["I_t"], r64["s_t"])
            cb["all_cores"] = cpu_all[wl.name]
            # bounded one-core samples and all-core rates of the other workloads
            cb["workloads"] = {
                name: {"one_core": optional(f"{name} cpu sample", cpu_sample, W.WORKLOADS[name]),
                       "all_cores": cpu_all[name]}
                for name in others}
            # the GPU's FP64 iterations of the other workloads against the
            # oracle's whole run of the same workload (stored by
            # tests/golden/make_golden.py)
            for name in others:
                ref = golden_I_t(name)
                got = per_workload[name].get("fp64_I_t")
                if ref is not None and got is not None:
                    cb["workloads"][name]["fp64_gpu_vs_oracle_max_rel_err_I_t"] = \
                        float(np.max(np.abs(np.asarray(got) - ref) / np.abs(ref)))
            return cb

        out["cpu_baseline"] = optional("cpu baseline", cpu_section)
    if not args.no_serving:
        out["serving"] = optional("serving", serving_section, vg, W, args.serving_requests)
    # the paper's own timings (Table 1), context only: another machine, an
    # integral and event count it does not state
    out["paper_context"] = {
        "what": "seconds per iteration on SLURM CPU nodes of 4 cores (Table 1); integrand, events "
                "and precision not stated; not a target",
        "nodes_1_2_3_s": [59.7, 33.3, 22.3]}
    print(json.dumps(out))


def events_limit_sweep(vg, W, wl, steps):
    """The paper's batch-size experiment (Fig. 2) on MI355X: a whole FP32-eval
    run with at most a fraction of the events per kernel launch. Random
    numbers are drawn on the device, so small batches cost launches, not
    host-to-device transfers."""
    rows = []
    for frac in (0.02, 0.05, 0.1, 0.25, 0.5, 1.0):
        h = vg.vegas_create(wl.dim, wl.nb)
        vg.vegas_set_params(h, wl.fid, wl.params)
        vg.vegas_set_precision(h, W.FP32_EVAL)
        vg.vegas_set_events_limit(h, int(round(frac * wl.n_events)))
        vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
        t0 = time.perf_counter()
        for _ in range(steps):
            vg.vegas_reset(h)
            vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
        dt = (time.perf_counter() - t0) / steps
        rows.append({"events_limit_fraction": frac, "launches_per_iteration": int(round(1 / frac)),
                     "ms_per_run": dt * 1e3, "events_per_s": wl.n_events * wl.n_iter / dt})
    return rows


USER_GAUSS = r"""
// exp(-sum_d ((x_d - 1/2)/a)^2) / (a sqrt(pi))^dim, with p = {1/a^2, (a sqrt(pi))^-dim}
__device__ double vegas_user_f64(const double* x, int dim, const double* p) {
  double s = 0.0;
  for (int d = 0; d < dim; ++d) {
    const double u = x[d] - 0.5;
    s = fma(u, u, s);
  }
  return exp(-p[0] * s) * p[1];
}
__device__ float vegas_user_f32(const float* x, int dim, const float* p) {
  float s = 0.0f;
  for (int d = 0; d < dim; ++d) {
    const float u = x[d] - 0.5f;
    s = fmaf(u, u, s);
  }
  return __expf(-p[0] * s) * p[1];
}
"""


def user_integrand_section(vg, W, wl, steps, builtin):
    """The workload's Gaussian written as user source in the same
    exp-of-a-sum form as the built-in one and compiled at run time (for
    exactly wl.dim dimensions): whole runs per second against the built-in
    Gaussian kernel."""
    t0 = time.perf_counter()
    fid = vg.vegas_integrand_compile(USER_GAUSS, wl.dim)
    compile_s = time.perf_counter() - t0
    out = {"what": "the Gaussian as user HIP source, compiled with hiprtc",
           "compile_s": compile_s}
    for prec, key in ((W.FP32_EVAL, "fp32_eval"), (W.FP64, "fp64")):
        h = vg.vegas_create(wl.dim, wl.nb)
        a = wl.params[0]
        vg.vegas_set_params(h, fid, [1.0 / (a * a), (a * math.sqrt(math.pi)) ** -wl.dim])
        vg.vegas_set_precision(h, prec)
        vg.vegas_run(h, fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
        t0 = time.perf_counter()
        for _ in range(steps):
            vg.vegas_reset(h)
            I_t, s_t = vg.vegas_run(h, fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
        dt = (time.perf_counter() - t0) / steps
        I, s, _ = vg.vegas_result(h)
        v = wl.n_events * wl.n_iter / dt
        out[key] = {"events_per_s": v, "vs_builtin": v / builtin[prec], "I": I, "sigma": s}
    return out


def small_latency(vg, W, reps):
    """Per-iteration latency of the 4-D Gaussian parity workload (1e5 events,
    FP64): synchronous vegas_iterate, launch to result on the host."""
    wl = W.WORKLOADS["gauss4d"]
    h = vg.vegas_create(wl.dim, wl.nb)
    vg.vegas_set_params(h, wl.fid, wl.params)
    vg.vegas_run(h, wl.fid, wl.n_events, wl.seed, wl.n_iter, wl.alpha)
    lat = []
    for _ in range(reps):
        a = time.perf_counter()
        vg.vegas_iterate(h, wl.fid, wl.n_events, wl.seed)
        lat.append(time.perf_counter() - a)
    return {"what": f"one synchronous vegas_iterate of {wl.note}", "repeats": reps,
            "p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3}


def replay(vg, W, trace, rate, max_slots, budget=4 << 30, graph=False, chain=None,
           chunk_events=0, lanes=None):
    """Submit the trace at `rate` requests/s (inf: all at once) to a server
    with `max_slots` slots; returns latency percentiles and throughput."""
    import threading
    srv = vg.vegas_server_create(budget, max_slots, chunk_events)
    vg.vegas_server_set_graph(srv, graph)
    if chain is not None:
        vg.vegas_server_set_chain(srv, chain)
    if lanes is not None:
        vg.vegas_server_set_lanes(srv, lanes)
    # warm the server's kernels outside the measurement
    warm = vg.vegas_server_submit(srv, 3, 20, W.F_GAUSS, [0.2], 10_000, 2, 1.5, 0)
    vg.vegas_server_wait(srv, warm)
    base = trace[0].arrival_s
    scale = 0.0 if math.isinf(rate) else 200.0 / rate
    tickets = [None] * len(trace)
    t0 = time.perf_counter()

    def submit():
        for i, r in enumerate(trace):
            due = t0 + (r.arrival_s - base) * scale
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                time.sleep(min(due - now, 0.001) if due - now > 0.002 else 0)
            tickets[i] = vg.vegas_server_submit(srv, r.dim, r.nb, r.fid, r.params, r.n_events,
                                                r.n_iter, r.alpha, r.seed, r.prec)

    th = threading.Thread(target=submit)
    th.start()
    lat = []
    for i in range(len(trace)):
        while tickets[i] is None:
            time.sleep(0.0002)
        _, _, _, l = vg.vegas_server_wait(srv, tickets[i])
        lat.append(l)
    t_end = time.perf_counter()
    th.join()
    done, events, items, peak = vg.vegas_server_stats(srv)
    ticks, graph_ticks = vg.vegas_server_ticks(srv)
    chains = vg.vegas_server_chains(srv)
    vg.vegas_server_destroy(srv)
    ev = sum(r.n_events * r.n_iter for r in trace)
    return {"rate_per_s": rate if not math.isinf(rate) else "closed-loop",
            "p50_ms": pct(lat, 50) * 1e3, "p99_ms": pct(lat, 99) * 1e3,
            "mean_ms": float(np.mean(lat)) * 1e3, "events_per_s": ev / (t_end - t0),
            "makespan_s": t_end - t0, "peak_concurrent": peak, "ticks": ticks,
            "chains": chains, "graph_replayed_ticks": graph_ticks}


def replay_median(vg, W, trace, rate, max_slots, repeats, **kw):
    """replay() `repeats` times; each figure is the median over the replays
    (the peak concurrency the largest). A host-side stall of a few
    milliseconds, seen about once in twenty replays, holds up every integral
    in flight, so one replay's p99 at a high rate can jump by ~10 ms; the
    median of three is not moved by one such replay. Each replay's p99 is
    kept in p99_ms_replays."""
    runs = [replay(vg, W, trace, rate, max_slots, **kw) for _ in range(repeats)]
    out = dict(runs[0])
    for k in ("p50_ms", "p99_ms", "mean_ms", "events_per_s", "makespan_s"):
        out[k] = float(np.median([r[k] for r in runs]))
    out["peak_concurrent"] = max(r["peak_concurrent"] for r in runs)
    out["p99_ms_replays"] = [r["p99_ms"] for r in runs]
    return out


def best_at(rows, slo_ms):
    ok = [r for r in rows if r["p99_ms"] <= slo_ms]
    return max((r["events_per_s"] for r in ok), default=0.0)


def serving_section(vg, W, n_requests):
    """The serving stream (1000 Poisson arrivals at 200/s, mixed integrals),
    batched (up to 256 integrals at once) and one integral at a time, then a
    rate sweep (each rate replayed three times, medians); the sustained
    throughput of each mode compared under a p99 objective equal to the
    one-at-a-time p99 at 200/s, and at fixed objectives. Both modes chain the
    ticks up to the next completion and run chains on four streams (lanes);
    the batched server with one lane, with and without chains, is measured
    beside them, and the chunk size is swept at 1000 requests/s (the paper's
    events_limit, Fig. 2, for the serving loop)."""
    trace = W.serving_trace(n_requests, rate_per_s=200.0, seed=0)
    res = {"trace": f"{n_requests} requests, Poisson arrivals at 200/s, dims U{{2..12}}, bins "
                    "U{20..100}, events/iteration log-U[1e4, 1e7], 5-10 iterations, Gaussian or "
                    "Breit-Wigner x flat, FP32-eval; trace seed 0",
           "total_events": int(sum(r.n_events * r.n_iter for r in trace))}
    modes = {"batched": 256, "one_at_a_time": 1}
    rates = [200.0, 500.0, 1000.0, 1500.0, 2000.0, 3000.0, 4000.0, 6000.0, 8000.0, 10000.0,
             float("inf")]
    for mode, slots in modes.items():
        rows = []
        for rate in rates:
            log(f"serving {mode} at {rate}/s")
            rows.append(replay_median(vg, W, trace, rate, slots, 1 if math.isinf(rate) else 3))
        res[mode] = rows
    # the same batched server with one stream and one tick per host
    # synchronisation (the design without lanes and chains), and with one
    # stream and chains
    for key, kw in (("batched_one_lane_one_tick_per_sync", dict(chain=1, lanes=1)),
                    ("batched_one_lane", dict(lanes=1))):
        rows = []
        for rate in (200.0, 1000.0, 4000.0):
            log(f"serving {key} at {rate}/s")
            rows.append(replay_median(vg, W, trace, rate, 256, 3, **kw))
        res[key] = rows
    # SLO: the one-at-a-time p99 at the trace's own rate (200/s)
    slo = res["one_at_a_time"][0]["p99_ms"]
    res["p99_slo_ms"] = slo
    res["p99_slo_definition"] = "one-at-a-time p99 at 200 requests/s"
    best = {mode: best_at(res[mode], slo) for mode in modes}
    res["throughput_at_slo_events_per_s"] = best
    res["batched_over_one_at_a_time_at_slo"] = (best["batched"] / best["one_at_a_time"]
                                                if best["one_at_a_time"] > 0 else None)
    # the same comparison at fixed p99 objectives
    table = []
    for target in (0.7, 1.0, 1.5, 2.0, 5.0, 10.0):
        row = {"p99_ms": target}
        for mode in modes:
            row[mode] = best_at(res[mode], target)
        row["ratio"] = row["batched"] / row["one_at_a_time"] if row["one_at_a_time"] else None
        table.append(row)
    res["throughput_at_p99_objectives"] = table
    # the same server with repeated ticks replayed from captured hipGraphs
    log("serving batched at 1000/s with graph replays")
    res["batched_graph_replays_1000_per_s"] = replay(vg, W, trace, 1000.0, 256, graph=True)
    # chunk size of the work items (default: a function of the integral's
    # event count; fixed sizes below, each integral cut into ceil(N/chunk)
    # work items of one 256-thread workgroup)
    sweep = []
    for chunk in (10_000, 100_000, 1_000_000, 10_000_000, 100_000_000):
        log(f"serving batched at 1000/s, chunk {chunk}")
        row = replay(vg, W, trace, 1000.0, 256, chunk_events=chunk)
        row["chunk_events"] = chunk
        sweep.append(row)
    res["chunk_sweep_1000_per_s"] = sweep
    return res


def _oracle_iterations(args):
    """Whole oracle iterations (draw, map, integrand, moments, histogram) of
    n events on the uniform grid, iteration counters t0, t0 + 1, ..., until
    `seconds` have passed; returns (events, seconds)."""
    import oracle
    dim, nb, fid, params, n, seed, t0, seconds, start = args
    e = oracle.uniform_grid(dim, nb)
    while time.time() < start:  # every process starts together
        time.sleep(0.001)
    t = time.perf_counter()
    done = 0
    while True:
        oracle.iterate(e, fid, params, n, seed, t0 + done // n)
        done += n
        if time.perf_counter() - t >= seconds:
            return done, time.perf_counter() - t


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it, with its family/model/stepping."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping") and k not in info:
                    info[k] = v
            if not line.strip() and info:
                break
    except OSError:
        pass
    return (f"{info.get('model name', '?')} (family {info.get('cpu family', '?')}, model "
            f"{info.get('model', '?')}, stepping {info.get('stepping', '?')})")


def cpu_baseline_all_cores(wl, seconds=4.0):
    """The oracle as written on every host core available to the process (at
    most 16): one forked process per core, each running whole iterations of
    the workload's events split over the cores (distinct iteration counters,
    so distinct random streams) for about `seconds`. Must run before this
    process initialises the GPU."""
    import multiprocessing as mp
    import oracle
    oracle.lib()  # build before forking
    cores = min(16, len(os.sched_getaffinity(0)))
    n = max(wl.n_events // cores, 1 << 16)
    with mp.get_context("fork").Pool(cores) as pool:
        start = time.time() + 0.5
        jobs = [(wl.dim, wl.nb, wl.fid, wl.params, n, wl.seed, 1000 * i, seconds, start)
                for i in range(cores)]
        res = pool.map(_oracle_iterations, jobs, chunksize=1)
    events = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return {"value": events / wall, "unit": "events/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"whole oracle iterations (draw, map, integrand, moments, histogram) of "
                      f"{n} events of {wl.name} on the uniform grid, one forked process per "
                      f"core, {events} events in {wall:.1f} s"}


def golden_I_t(name):
    """The oracle's per-iteration estimates of a whole run of the workload, as
    stored under tests/golden/, or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_fp64_seed0.json")
    try:
        with open(path) as f:
            return np.array([float(v) for v in json.load(f)["I_t"]])
    except (OSError, KeyError, ValueError):
        return None


def cpu_sample(wl, max_events=2_000_000):
    """The oracle on one core: one whole iteration of at most `max_events`
    events of the workload on the uniform grid (a few seconds)."""
    import oracle
    n = min(wl.n_events, max_events)
    e = oracle.uniform_grid(wl.dim, wl.nb)
    t0 = time.perf_counter()
    oracle.iterate(e, wl.fid, wl.params, n, wl.seed, 0)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"one iteration of {n} events of {wl.name} (FP64, seed {wl.seed}, "
                      f"uniform grid), {dt:.1f} s"}


def gpu_share(vg, W, wl, steps):
    """One GPU's share of the workload on 8 GPUs (events split by index, one
    exchange of 2 + D*nb values per iteration not included): N/8 events per
    iteration, whole FP32-eval runs."""
    n = wl.n_events // 8
    h = vg.vegas_create(wl.dim, wl.nb)
    vg.vegas_set_params(h, wl.fid, wl.params)
    vg.vegas_set_precision(h, W.FP32_EVAL)
    for _ in range(5):
        vg.vegas_reset(h)
        vg.vegas_run(h, wl.fid, n, wl.seed, wl.n_iter, wl.alpha)
    t0 = time.perf_counter()
    for _ in range(steps):
        vg.vegas_reset(h)
        vg.vegas_run(h, wl.fid, n, wl.seed, wl.n_iter, wl.alpha)
    dt = (time.perf_counter() - t0) / steps
    return {"events_per_iteration": n, "ms_per_run": dt * 1e3, "events_per_s": n * wl.n_iter / dt}


def cpu_baseline(wl, gpu_I_t, gpu_s_t):
    """The FP64 oracle, single-threaded as written, on the same workload
    (same seed; the whole run of the 8-D Gaussian, about 7 s of CPU work on
    an EPYC core; the first iterations of the larger workloads)."""
    import oracle
    n_ev = min(wl.n_events, 10_000_000)
    n_iter = wl.n_iter if wl.n_events <= 10_000_000 else 5
    t0 = time.perf_counter()
    I_t, s_t, _, _ = oracle.run(wl.dim, wl.nb, wl.fid, wl.params, n_ev, wl.seed, n_iter,
                                wl.alpha)
    dt = time.perf_counter() - t0
    res = {"value": n_ev * n_iter / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
           "cpu": cpu_model(),
           "sample": f"first {n_iter} of {wl.n_iter} iterations of {wl.name} at "
                     f"{n_ev:.0e} events each (FP64, seed {wl.seed}), {dt:.1f} s"}
    if n_ev == wl.n_events:
        rel = np.max(np.abs(np.asarray(gpu_I_t[:n_iter]) - I_t) / np.abs(I_t))
        res["fp64_gpu_vs_oracle_max_rel_err_I_t"] = float(rel)
    return res


if __name__ == "__main__":
    main()
