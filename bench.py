#!/usr/bin/env python3
"""Benchmark of randomized HALS (rnmf) on one MI355X.

Workload: the tall synthetic matrix of the paper's performance study
(Sec. 4.4), 100,000 x 5,000 FP32, a rank-50 product of uniform [0, 1)
factors plus N(0, 0.05^2) noise clipped at 0; k = 50, p = 20, q = 2
(the BF16 form adds one subspace iteration), 200 sweeps.  Inputs are
synthetic and seeded (synth.WORKLOADS["tall_100000x5000"]).

A step is one rnmf_factorize call: (BF16 cast,) sketch, compression,
W~ = Q^T W0, 200 compressed-HALS sweeps and the final relative error.
`value` is sweeps per second of whole steps in the BF16 form, with X already
resident in HBM.  The JSON line also carries the FP32 form, the time to reach
1.01 x the FP32 form's final error for both forms, the HBM bandwidth of the
passes over X, the roofline of the dominant kernel (the persistent sweep
kernel, timed with HIP events on its stream inside rnmf_factorize) and the
FP64 oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import numpy as np
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rHALS iters/s + s to rel-err≤1.01×FP32 (100k×5k,k=50): BF16 vs FP32; HBM GB/s"
WORKLOAD = "tall_100000x5000"
PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X published dense FP32 matrix peak
PEAK_BF16_TFLOPS = 2500.0         # MI355X published dense BF16 matrix peak
PEAK_HBM_GBPS = 8000.0            # MI355X published HBM3E bandwidth
SWEEP_SRC = os.path.join(ROOT, "paper_1711_02037_amd", "csrc", "sweep.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_flops(m, n, l, k):
    """Algorithmic flops of one compressed-HALS sweep (fused multiply-add = 2):
    R = B^T W~ (2nlk), S = W^T W (2mk^2), H rows (2nk^2), T = B H^T (2nlk),
    V = H H^T (2nk^2), W~ updates (2lk^2), lift and map-back (4mlk)."""
    return 4 * m * l * k + 4 * n * l * k + 4 * n * k * k + 2 * m * k * k + 2 * l * k * k


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel_hash):
    """HBM bytes per sweep-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "sweep_kernel_tall_100000x5000_counters.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256_16") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the host oracle baseline")
    ap.add_argument("--no-target", action="store_true", help="skip the time-to-target protocol")
    ap.add_argument("--no-hals", action="store_true", help="skip the deterministic HALS comparison")
    ap.add_argument("--no-svd-init", action="store_true", help="skip the SVD-based initialization comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload (512 uneven problems)")
    ap.add_argument("--no-backward", action="store_true", help="skip the reverse pass through unrolled sweeps")
    ap.add_argument("--no-stack", action="store_true", help="skip the 32,256 x 2,410 image-stack workload")
    ap.add_argument("--no-orders", action="store_true", help="skip the update-order timings")
    ap.add_argument("--no-speedup", action="store_true", help="skip the HALS/rHALS speedup study over k")
    ap.add_argument("--timeline", default="",
                    help="write the traced sweep's per-column timeline (markdown table) to this file")
    ap.add_argument("--no-kernel-profile", action="store_true",
                    help="skip the per-kernel X-pass timing (torch.profiler; off under rocprofv3)")
    ap.add_argument("--speedup-ks", default="", help="comma-separated ranks for a per-sweep HALS/rHALS "
                    "speedup series (Sec. 4.4 figure), e.g. 10,20,50")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method's multi-GPU sharding is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1711_02037_amd as rn

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if not rn.available():
        print("librnmf.so is not built (python -m paper_1711_02037_amd.build)", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    w = synth.workload(WORKLOAD)
    m, n, k, p, q, sweeps = w["m"], w["n"], w["k"], w["p"], w["q"], w["sweeps"]
    l = synth.sketch_cols(k, p, m, n)

    t0 = time.time()
    Xh, Omh, W0h, H0h, _ = synth.make(WORKLOAD, threads=min(16, os.cpu_count() or 1))
    log(f"generated {m}x{n} in {time.time() - t0:.1f}s")
    X = torch.from_numpy(Xh).to(dev)
    Om = torch.from_numpy(Omh).to(dev)
    W0 = torch.from_numpy(W0h).to(dev)
    H0 = torch.from_numpy(H0h).to(dev)
    nb = max(rn.workspace_bytes(rn.OP_FACTORIZE, m, n, rn.make_opts(k, p, q, precision=pr))
             for pr in ("fp32", "bf16"))
    ws = rn._workspace(nb, dev)

    # Plain elementwise copy of known size (X.numel() * 4 bytes read and
    # written): the reference point that scales the HBM byte counters.
    torch.cuda.synchronize()
    Xc = X * 1.0
    torch.cuda.synchronize()
    del Xc
    log(f"copy calibration: {X.numel() * 4 / 1e9:.3f} GB read + {X.numel() * 4 / 1e9:.3f} GB written")

    def step(prec, iters=sweeps):
        return rn.factorize(X, k, p, q, max_iter=iters, precision=prec, omega=Om, W0=W0, H0=H0, ws=ws)

    last = {}

    def timed_steps(prec, nsteps, nwarm):
        for _ in range(nwarm):
            step(prec)
        torch.cuda.synchronize()
        reps = []
        t = time.perf_counter()
        for _ in range(nsteps):
            Wd, Hd, info = step(prec)
            reps.append(info)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        last[prec] = (Wd.cpu().numpy(), Hd.cpu().numpy())
        return el, reps

    # ---- headline: whole steps, BF16 form, then FP32 form --------------------
    el_b, reps_b = timed_steps("bf16", args.steps, args.warmup)
    log(f"bf16: {el_b / args.steps * 1e3:.2f} ms/step, rel_err {reps_b[-1]['rel_err']:.6f}")
    el_f, reps_f = timed_steps("fp32", args.steps, args.warmup)
    log(f"fp32: {el_f / args.steps * 1e3:.2f} ms/step, rel_err {reps_f[-1]['rel_err']:.6f}")
    value = sweeps * args.steps / el_b

    # ---- dominant kernel: the persistent sweep kernel ------------------------
    ms_sw = statistics.mean(r["ms_sweeps"] for r in reps_b + reps_f)
    flops = sweep_flops(m, n, l, k) * sweeps
    achieved = flops / (ms_sw * 1e-3) / 1e12
    khash = source_hash(SWEEP_SRC)
    roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP32_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 5),
                "traffic": traffic_for(khash), "kernel": "sweep_kernel<float>",
                "ms_per_launch": round(ms_sw, 4), "sweeps_per_launch": sweeps,
                "flop_per_sweep": sweep_flops(m, n, l, k), "kernel_src_sha256_16": khash}

    # ---- passes over X: compression = one X pass ------------------------------
    Q32 = rn.sketch(X, k, p, q, omega=Om)
    split = sweep_split(rn, torch, X, Q32, W0, H0, k, timeline=args.timeline)
    roofline["limited_by"] = ("latency of the k-long chain of device-wide exchanges (one per W column); "
                              "the FLOP fraction is reported against the FP32 vector peak")
    roofline["per_sweep_us"] = split
    log(f"sweep split: {split}")
    Xb = rn.cast_bf16(X)
    Qb = rn.sketch(Xb, k, p, q, omega=Om, precision="bf16")
    cws = rn._workspace(max(rn.workspace_bytes(rn.OP_COMPRESS, m, n, rn.make_opts(k, p, q, precision=pr))
                            for pr in ("fp32", "bf16")), dev)

    def pass_gbps(Xin, Qin, prec, reps=10):
        rn.compress(Xin, Qin, prec, ws=cws)
        st = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            rn.compress(Xin, Qin, prec, ws=cws)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        return Xin.numel() * Xin.element_size() / (ms * 1e-3) / 1e9, ms

    gb32, ms32 = pass_gbps(X, Q32, "fp32")
    gb16, ms16 = pass_gbps(Xb, Qb, "bf16")
    xpass = {"fp32_compress_GBps": round(gb32, 1), "fp32_compress_ms": round(ms32, 4),
             "bf16_compress_GBps": round(gb16, 1), "bf16_compress_ms": round(ms16, 4),
             "frac_of_8TBps": {"fp32": round(gb32 / PEAK_HBM_GBPS, 4), "bf16": round(gb16 / PEAK_HBM_GBPS, 4)},
             "note": "one rnmf_compress call = pack Q + one pass over X + split reduce, timed with events"}
    if not args.no_kernel_profile:
        xpass["per_kernel"] = xpass_kernels(rn, torch, step, m, n, l)
    log(f"X pass: fp32 {gb32:.0f} GB/s, bf16 {gb16:.0f} GB/s; per kernel {xpass.get('per_kernel')}")

    # ---- time to 1.01 x FP32 final error --------------------------------------
    ttt = None
    if not args.no_target:
        ttt = time_to_target(rn, torch, X, Om, W0, H0, k, p, q, sweeps, ws, step, reps_f[-1]["rel_err"])

    # ---- deterministic HALS on the same X (Sec. 3.1 vs Sec. 3.2) -------------
    hals = None
    if not args.no_hals:
        hals = hals_compare(rn, torch, X, W0, H0, sweeps, reps_f, ws_dev=dev)
        log(f"HALS: {hals['ms_per_sweep']:.3f} ms/sweep, rHALS {hals['rhals_ms_per_sweep']:.3f} ms/sweep, "
            f"speedup {hals['speedup_per_sweep']:.2f}x per sweep, {hals['speedup_200_sweeps']:.2f}x per run")
    # ---- speedup of rHALS over HALS for several k, both shapes of Sec. 4.4 --
    study = None
    if not args.no_speedup:
        ks = [int(v) for v in args.speedup_ks.split(",") if v] or [10, 20, 30, 40, 50, 64]
        study = speedup_study(rn, torch, synth, X, p, q, ks, dev)

    # ---- SVD-based initialization against the seeded uniform one -------------
    svd = None
    if not args.no_svd_init:
        svd = svd_init_compare(rn, torch, X, Om, Q32, k, p, q, sweeps, reps_f, dev)
        log(f"SVD init: {svd['ms']:.3f} ms; error after {sweeps} sweeps {svd['rel_err']:.6f} "
            f"(uniform init {svd['rel_err_uniform_init']:.6f})")

    # ---- batched workload: 512 uneven problems in one persistent launch ------
    batch = None
    if not args.no_batch:
        batch = batch_bench(rn, torch, synth, dev)
        log(f"batch: {batch['problems']} problems in {batch['ms_per_run']:.2f} ms per run "
            f"({batch['problems_per_s']:.0f} problems/s, {batch['x_GBps']:.0f} GB/s of X); one at a time "
            f"~{batch['one_at_a_time_ms_estimate']:.0f} ms ({batch['speedup_vs_one_at_a_time']:.1f}x); "
            f"bf16 {batch['bf16']['ms_per_run']:.2f} ms per run, error ratio to fp32 up to "
            f"{batch['bf16']['max_ratio_to_fp32']:.4f}")

    # ---- reverse pass through 20 unrolled FP32 sweeps (two workloads) ---------
    back = None
    if not args.no_backward:
        back = backward_section(rn, torch, synth, X, Q32, W0, H0, dev)
        for nm in ("diff_8192x2048", "tall_100000x5000"):
            b = back[nm]
            log(f"backward {nm}: {b['ms_backward']:.2f} ms for {b['T']} sweeps from recorded states (recording "
                f"forward {b['ms_forward_recorded']:.2f} ms, one-launch forward {b['ms_forward']:.2f} ms, "
                f"checkpointed backward (every {b['ckpt_every']}) {b['ms_backward_checkpointed']:.2f} ms)")

    # ---- the image-stack workload: iters/s of both forms -------------------------
    c2 = None
    if not args.no_stack:
        c2 = c2_bench(rn, torch, synth, dev)
        log(f"stack_32256x2410: bf16 {c2['bf16']['iters_per_s']:.0f} iters/s "
            f"({c2['bf16']['sweep_loop_iters_per_s']:.0f} in the sweep loop), fp32 {c2['fp32']['iters_per_s']:.0f} "
            f"iters/s ({c2['fp32']['sweep_loop_iters_per_s']:.0f})")

    # ---- update orders: interleaved and shuffled sweeps (ordered path) --------
    orders = None
    if not args.no_orders:
        orders = orders_bench(rn, torch, X, Q32, W0, H0, dev)
        log(f"orders: interleaved {orders['interleaved_ms_per_sweep']:.2f} ms/sweep, shuffled "
            f"{orders['shuffled_ms_per_sweep']:.2f} ms/sweep, blocked list {orders['blocked_list_ms_per_sweep']:.2f} "
            f"ms/sweep (sweep kernel {orders['sweep_kernel_ms_per_sweep']:.3f})")

    # ---- FP64 oracle on the host ---------------------------------------------
    cpu = parity = None
    if not args.no_cpu:
        del X, Xb
        torch.cuda.empty_cache()
        cpu, parity = cpu_baseline(Xh, Omh, W0h, H0h, k, q, sweeps, last, synth, w)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(el_b / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded rank-50 uniform product + N(0,0.05^2) noise, clipped)",
        "config": {"workload": WORKLOAD, "m": m, "n": n, "k": k, "p": p, "q": q + 1, "l": l,
                   "sweeps": sweeps, "step": "cast+sketch+compress+init+200 sweeps+rel_err",
                   "x_pass_arithmetic": "bf16 MFMA (X bf16; Q split hi+lo in the compression Q^T X, operand bf16 in the subspace-iteration passes), fp32 accumulate",
                   "sweep_arithmetic": "fp32 (H phase fp64)"},
        "rel_err": {"bf16": reps_b[-1]["rel_err"], "fp32": reps_f[-1]["rel_err"]},
        "oracle_parity": parity,
        "fp32": {"value": round(sweeps * args.steps / el_f, 2), "unit": "iters/s",
                 "ms_per_step": round(el_f / args.steps * 1e3, 3), "q": q},
        "stage_ms": {"bf16": {kk: round(statistics.mean(r[kk] for r in reps_b), 4)
                              for kk in ("ms_qb", "ms_sweeps", "ms_error")},
                     "fp32": {kk: round(statistics.mean(r[kk] for r in reps_f), 4)
                              for kk in ("ms_qb", "ms_sweeps", "ms_error")}},
        "sweeps_per_s_kernel": round(sweeps / (ms_sw * 1e-3), 1),
        "time_to_target": ttt,
        "hals_vs_rhals": hals,
        "speedup_study": study,
        "svd_init": svd,
        "batched": batch,
        "backward": back,
        "orders": orders,
        "stack_32256x2410": c2,
        "xpass": xpass,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def c2_bench(rn, torch, synth, dev, steps=2):
    """iters/s on the image-stack workload (32,256 x 2,410, k = 16, 500
    sweeps), BF16 and FP32 forms: whole factorize steps and the sweep loop
    alone (its launch timed with events inside rnmf_factorize)."""
    w = synth.workload("stack_32256x2410")
    Xh, Omh, W0h, H0h, _ = synth.make("stack_32256x2410", threads=16)
    X, Om = torch.from_numpy(Xh).to(dev), torch.from_numpy(Omh).to(dev)
    W0, H0 = torch.from_numpy(W0h).to(dev), torch.from_numpy(H0h).to(dev)
    k, p, q, sw = w["k"], w["p"], w["q"], w["sweeps"]
    out = {"m": w["m"], "n": w["n"], "k": k, "sweeps": sw}
    for prec in ("bf16", "fp32"):
        rn.factorize(X, k, p, q, max_iter=sw, precision=prec, omega=Om, W0=W0, H0=H0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = [rn.factorize(X, k, p, q, max_iter=sw, precision=prec, omega=Om, W0=W0, H0=H0)[2]
                for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ms_sw = statistics.mean(r["ms_sweeps"] for r in reps)
        out[prec] = {"iters_per_s": round(sw * steps / el, 1), "ms_per_step": round(el / steps * 1e3, 3),
                     "sweep_loop_iters_per_s": round(sw / (ms_sw * 1e-3), 1), "ms_qb": round(reps[-1]["ms_qb"], 4),
                     "rel_err": reps[-1]["rel_err"]}
    return out


def time_to_target(rn, torch, X, Om, W0, H0, k, p, q, sweeps, ws, step, e32_final, cap=400, rounds=7):
    """Calibration with an error probe after every sweep (untimed) finds, for
    each form, the first sweep s_f that reaches tau = 1.01 x the FP32 form's
    error after `sweeps` sweeps.  Then end-to-end runs of exactly s_f sweeps
    are timed in alternation (FP32, BF16, FP32, ...; `rounds` each, after a
    warm-up of each), so that a drift of the GPU clock over the run weighs on
    both forms alike; the median of each form is reported."""
    tau = 1.01 * e32_final
    res = {"target_rel_err": tau, "fp32_final_rel_err_200": e32_final}
    m, n = X.shape
    forms = (("fp32", q), ("bf16", q + 1))
    sfs = {}
    for prec, qq in forms:
        Q = rn.sketch(X, k, p, q, omega=Om, precision=prec)
        B = rn.compress(X, Q, prec)
        W = W0.clone()
        H = H0.clone()
        Wt = rn.compress(W, Q, "fp32")
        hws = rn._workspace(rn.workspace_bytes(rn.OP_HALS_STEP, m, n, rn.make_opts(k, p, 0)), X.device)
        sf = None
        for s_ in range(1, cap + 1):
            rn.hals_step(Q, B, W, Wt, H, nsweeps=1, ws=hws)
            e = rn.rel_error(X, W, H)
            if e <= tau:
                sf = s_
                break
        if sf is None:
            res[prec] = {"sweeps": None, "seconds": None, "note": f"not reached within {cap} sweeps"}
        else:
            sfs[prec] = sf
    times = {prec: [] for prec in sfs}
    errs = {prec: None for prec in sfs}
    for prec in sfs:
        step(prec, sfs[prec])
    for _ in range(rounds):
        for prec in sfs:
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, info = step(prec, sfs[prec])
            torch.cuda.synchronize()
            times[prec].append(time.perf_counter() - t)
            errs[prec] = info["rel_err"]
    for prec, qq in forms:
        if prec not in sfs:
            continue
        med = statistics.median(times[prec])
        res[prec] = {"sweeps": sfs[prec], "seconds": round(med, 6), "rel_err": errs[prec],
                     "reached": errs[prec] <= tau, "q": qq, "runs": rounds}
        log(f"time to target {prec}: {sfs[prec]} sweeps, {med * 1e3:.2f} ms")
    if res.get("fp32", {}).get("seconds") and res.get("bf16", {}).get("seconds"):
        res["bf16_speedup"] = round(res["fp32"]["seconds"] / res["bf16"]["seconds"], 4)
    return res


def hals_compare(rn, torch, X, W0, H0, sweeps, reps_f, ws_dev):
    """Deterministic HALS (two passes over X per sweep) against randomized HALS
    on the same X, W0, H0 and sweep count, FP32: time per sweep (events on the
    current stream), the error after `sweeps` sweeps, and the speedups."""
    m, n = X.shape
    k = H0.shape[0]
    W, H = W0.clone(), H0.clone()
    hws = rn._workspace(rn.workspace_bytes(rn.OP_HALS, m, n, rn.make_opts(k, 0, 0)), ws_dev)
    rn.hals(X, W, H, nsweeps=1, ws=hws)  # warm-up sweep
    W, H = W0.clone(), H0.clone()
    st = torch.cuda.current_stream(ws_dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    rn.hals(X, W, H, nsweeps=sweeps, ws=hws)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    err = rn.rel_error(X, W, H)
    r_ms_sweep = statistics.mean(r["ms_sweeps"] for r in reps_f) / sweeps
    r_ms_run = statistics.mean(r["ms_qb"] + r["ms_sweeps"] + r["ms_error"] for r in reps_f)
    return {"precision": "fp32", "sweeps": sweeps, "ms_per_sweep": round(ms / sweeps, 4),
            "seconds": round(ms / 1e3, 5), "rel_err": err,
            "rhals_ms_per_sweep": round(r_ms_sweep, 4), "rhals_seconds": round(r_ms_run / 1e3, 5),
            "rhals_rel_err": reps_f[-1]["rel_err"],
            "speedup_per_sweep": round(ms / sweeps / r_ms_sweep, 3),
            "speedup_200_sweeps": round(ms / r_ms_run, 3),
            "note": "HALS streams X twice per sweep; rHALS streams it (2q+2) times once, then sweeps on B"}


def sweep_split(rn, torch, X, Q, W0, H0, k, timeline=None):
    """Where a sweep's time goes: one traced two-sweep launch (phase timestamps
    of workgroup 0 in the first sweep, from the device's 100 MHz counter) on
    this workload's Q and B = Q^T X.  Per W column: the device-wide exchange
    (from the column's partial store to its totals) and the local work between
    exchanges (update vector, lift, clip, map-back)."""
    B = rn.compress(X, Q)
    Wt0 = rn.compress(W0, Q)
    W, Wt, H = W0.clone(), Wt0.clone(), H0.clone()
    ts = rn.hals_step(Q, B, W, Wt, H, nsweeps=2, trace=True)[3]
    pre = [ts[5 + 2 * j] for j in range(k)]
    post = [ts[6 + 2 * j] for j in range(k)]
    if any(v is None for v in pre + post + [ts[2], ts[3], ts[4], ts[5 + 2 * k], ts[7 + 2 * k], ts[8 + 2 * k]]):
        return None
    ex = [b - a for a, b in zip(pre, post)]
    loc = [pre[j] - post[j - 1] for j in range(1, k)]
    if timeline:
        # per-column timeline of the traced sweep (microseconds from the
        # sweep's start), for the record under profiles/
        t0 = ts[2]
        rows = ["| column | start of exchange | totals arrived | exchange | local work before it |",
                "|---:|---:|---:|---:|---:|"]
        for j in range(k):
            lw = pre[j] - (post[j - 1] if j > 0 else ts[4])
            rows.append(f"| {j} | {pre[j] - t0:.2f} | {post[j] - t0:.2f} | {ex[j]:.2f} | {lw:.2f} |")
        phases = [("H phase", ts[2], ts[3]), ("T/V products and exchange", ts[3], ts[4]),
                  ("W phase (all columns)", ts[4], ts[5 + 2 * k]),
                  ("S products and exchange", ts[5 + 2 * k], ts[7 + 2 * k]), ("whole sweep", ts[2], ts[8 + 2 * k])]
        head = ["| phase | us |", "|---|---:|"] + [f"| {nm} | {b_ - a_:.2f} |" for nm, a_, b_ in phases]
        with open(timeline, "w") as f:
            f.write("\n".join(head) + "\n\n" + "\n".join(rows) + "\n")
    return {"sweep": round(ts[8 + 2 * k] - ts[2], 2), "h_phase": round(ts[3] - ts[2], 2),
            "tv_products_and_exchange": round(ts[4] - ts[3], 2), "w_phase": round(ts[5 + 2 * k] - ts[4], 2),
            "s_products_and_exchange": round(ts[7 + 2 * k] - ts[5 + 2 * k], 2),
            "per_column_exchange": round(sum(ex) / len(ex), 3), "per_column_local": round(sum(loc) / len(loc), 3),
            "columns": k, "source": "first sweep of a traced launch, workgroup 0"}


def svd_init_compare(rn, torch, X, Om, Q, k, p, q, sweeps, reps_f, ws_dev, reps=5):
    """rnmf_svd_init on the FP32 Q and B of this workload (events on the current
    stream, mean of `reps` calls after one warm-up), and the FP32 form's error
    after `sweeps` sweeps when it starts from that initialization instead of
    the seeded uniform W0, H0."""
    m, n = X.shape
    B = rn.compress(X, Q)
    sws = rn._workspace(rn.workspace_bytes(rn.OP_SVD_INIT, m, n, rn.make_opts(k, p, 0)), ws_dev)
    rn.svd_init(Q, B, k, ws=sws)
    st = torch.cuda.current_stream(ws_dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        rn.svd_init(Q, B, k, ws=sws)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    _, _, info = rn.factorize(X, k, p, q, max_iter=sweeps, precision="fp32", omega=Om, init="svd")
    return {"ms": round(ms, 4), "rel_err": info["rel_err"], "rel_err_uniform_init": reps_f[-1]["rel_err"],
            "sweeps": sweeps, "precision": "fp32",
            "note": "nonnegative double SVD of the randomized SVD Q B (FP64 Jacobi on B B^T)"}


def backward_bench(rn, torch, X, Q, W0, H0, dev, T=20, ckpt=20, reps=3):
    """Reverse pass through T FP32 sweeps: rnmf_unroll with every state
    recorded (T one-sweep launches) and rnmf_backward reading that record,
    rnmf_backward recomputing the forward from checkpoints every `ckpt`
    sweeps, and one launch of the same T forward sweeps.  Events on the
    current stream, mean of `reps` calls after one warm-up."""
    m, n = X.shape
    k, l = H0.shape[0], Q.shape[1]
    B = rn.compress(X, Q)
    Wt0 = rn.compress(W0.contiguous(), Q)
    g = torch.Generator(device=dev)
    g.manual_seed(1711)
    gW = torch.randn((m, k), dtype=torch.float64, device=dev, generator=g)
    gH = torch.randn((k, n), dtype=torch.float64, device=dev, generator=g)
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    uws = rn._workspace(rn.workspace_bytes(rn.OP_HALS_STEP, m, n, rn.make_opts(k, l - k, 0)), dev)
    W, Wt, H = W0.clone(), Wt0.clone(), H0.clone()
    states = rn.unroll(Q, B, W, Wt, H, T, ws=uws)

    def fwd_rec():
        W.copy_(W0); Wt.copy_(Wt0); H.copy_(H0)
        rn.unroll(Q, B, W, Wt, H, T, ws=uws)

    ms_fr = timed(fwd_rec)
    bws = rn._workspace(rn.backward_workspace_bytes(m, n, l, k, T, 0, "fp32"), dev)
    ms_b = timed(lambda: rn.backward(Q, B, W0, Wt0, H0, T, gW, gH, states=states, ws=bws))
    cws = rn._workspace(rn.backward_workspace_bytes(m, n, l, k, T, ckpt, "fp32"), dev)
    ms_bc = timed(lambda: rn.backward(Q, B, W0, Wt0, H0, T, gW, gH, ckpt_every=ckpt, ws=cws))

    def fwd_one():
        W.copy_(W0); Wt.copy_(Wt0); H.copy_(H0)
        rn.hals_step(Q, B, W, Wt, H, nsweeps=T)

    ms_f = timed(fwd_one)
    return {"m": m, "n": n, "k": k, "l": l, "T": T, "ckpt_every": ckpt,
            "precision": "fp32 states, fp64 adjoints", "ms_backward": round(ms_b, 3),
            "ms_forward_recorded": round(ms_fr, 3), "ms_backward_checkpointed": round(ms_bc, 3),
            "ms_forward": round(ms_f, 3), "ratio_to_forward": round((ms_fr + ms_b) / ms_f, 2)}


def backward_section(rn, torch, synth, X, Q, W0, H0, dev):
    """The reverse pass on the differentiation workload (8,192 x 2,048, k = 32,
    T = 20, checkpoints every 5 sweeps) and on this benchmark's workload
    (T = 20, all states kept)."""
    w = synth.workload("diff_8192x2048")
    Xh, Omh, W0h, H0h, _ = synth.make("diff_8192x2048")
    Xd = torch.from_numpy(Xh).to(dev)
    Qd = rn.sketch(Xd, w["k"], w["p"], w["q"], omega=torch.from_numpy(Omh).to(dev))
    c5 = backward_bench(rn, torch, Xd, Qd, torch.from_numpy(W0h).to(dev), torch.from_numpy(H0h).to(dev), dev,
                        T=w["sweeps"], ckpt=w["ckpt_every"])
    c3 = backward_bench(rn, torch, X, Q, W0, H0, dev, T=20, ckpt=20)
    return {"diff_8192x2048": c5, "tall_100000x5000": c3,
            "note": "gradients of (W_T, H_T) with respect to B, W0, H0 with Q fixed. ms_backward reads the states "
                    "that rnmf_unroll recorded (ms_forward_recorded: T one-sweep launches plus the copies); "
                    "ms_backward_checkpointed recomputes them from checkpoints every ckpt_every sweeps; "
                    "ms_forward is one launch of T sweeps; ratio_to_forward = (recorded forward + backward) / "
                    "ms_forward"}


def orders_bench(rn, torch, X, Q, W0, H0, dev, nsw=3):
    """Milliseconds per sweep of rnmf_hals_ordered on this workload (FP32) for
    the interleaved order, a shuffled order (one seeded permutation per sweep)
    and the blocked list, beside the persistent sweep kernel's blocked sweep;
    events on the current stream."""
    import numpy as np
    m, n = X.shape
    k = H0.shape[0]
    B = rn.compress(X, Q)
    Wt0 = rn.compress(W0.contiguous(), Q)
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g = np.random.default_rng(1711)
    lists = {"interleaved": [rn.order_interleaved(k)] * nsw,
             "shuffled": [rn.order_interleaved(k, g.permutation(k)) for _ in range(nsw)],
             "blocked_list": [rn.order_blocked(k)] * nsw}
    out = {}
    for name, od in lists.items():
        W, Wt, H = W0.clone(), Wt0.clone(), H0.clone()
        rn.hals_ordered(Q, B, W, Wt, H, od[:1])
        e0.record(st)
        rn.hals_ordered(Q, B, W, Wt, H, od)
        e1.record(st)
        e1.synchronize()
        out[name + "_ms_per_sweep"] = round(e0.elapsed_time(e1) / nsw, 3)
    W, Wt, H = W0.clone(), Wt0.clone(), H0.clone()
    rn.hals_step(Q, B, W, Wt, H, nsweeps=1)
    e0.record(st)
    rn.hals_step(Q, B, W, Wt, H, nsweeps=20)
    e1.record(st)
    e1.synchronize()
    out["sweep_kernel_ms_per_sweep"] = round(e0.elapsed_time(e1) / 20, 4)
    out["note"] = ("rnmf_hals_ordered runs any order of block updates with a few launches per block; the blocked "
                   "orders run in the persistent sweep kernel (rnmf_hals_step)")
    return out


def batch_bench(rn, torch, synth, dev, reps=3):
    """The batched workload: 512 independent problems, m ~ U[256, 4096],
    n ~ U[128, 2048], k ~ U{4..32}, p = 10, q = 2, 100 sweeps each, run as one
    persistent launch captured in a HIP graph (after autotuning the X-pass
    tiling); wall time of `reps` replays by events on the replay stream."""
    from concurrent.futures import ThreadPoolExecutor
    w = synth.BATCH
    shapes = synth.batch_shapes()
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        host = list(ex.map(lambda i: synth.batch_problem(i, *shapes[i]), range(len(shapes))))
    log(f"batch: generated {len(host)} problems in {time.time() - t0:.1f}s")
    probs = [tuple(torch.from_numpy(a).to(dev) for a in p) for p in host]
    del host
    b = rn.Batch(probs, autotune=True, q=w["q"])
    g = b.capture(w["q"], w["sweeps"])
    st = torch.cuda.current_stream(dev)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        g.replay()
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rel, status = b.results()
    del g
    # the BF16 form (C4: FP32 storage, X passes on bfloat16 matrix cores, one
    # more subspace iteration), the same problems and sweeps
    bb = rn.Batch(probs, q=w["q"], precision="bf16")
    gb = bb.capture(w["q"], w["sweeps"])
    gb.replay()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        gb.replay()
    e1.record(st)
    e1.synchronize()
    ms_bf = e0.elapsed_time(e1) / reps
    rel_bf, status_bf = bb.results()
    del gb, bb
    # the same problems one at a time through the single-problem path
    # (rnmf_factorize per problem), on a seeded sample, scaled to the batch
    pick = synth.stream(w["seed"], 98).choice(len(shapes), size=24, replace=False)
    for i in pick[:2]:
        X, Om, W0, H0 = probs[i]
        rn.factorize(X, W0.shape[1], w["p"], w["q"], max_iter=w["sweeps"], omega=Om, W0=W0, H0=H0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in pick:
        X, Om, W0, H0 = probs[i]
        rn.factorize(X, W0.shape[1], w["p"], w["q"], max_iter=w["sweeps"], omega=Om, W0=W0, H0=H0)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t1) * 1e3 / len(pick) * len(shapes)
    xbytes = sum(m * n * 4 for m, n, k in shapes)
    passes = 2 * w["q"] + 2 + 1  # range finder and compression, plus the error pass
    out = {"problems": len(shapes), "sweeps": w["sweeps"], "q": w["q"], "p": w["p"],
           "ms_per_run": round(ms, 3), "problems_per_s": round(len(shapes) / (ms * 1e-3), 1),
           "sweeps_per_s": round(len(shapes) * w["sweeps"] / (ms * 1e-3), 1),
           "x_bytes": xbytes, "x_passes": passes,
           "x_GBps": round(passes * xbytes / (ms * 1e-3) / 1e9, 1),
           "frac_of_8TBps": round(passes * xbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
           "tiling": b.tiling, "all_ok": all(x == 0 for x in status),
           "one_at_a_time_ms_estimate": round(loop_ms, 1),
           "speedup_vs_one_at_a_time": round(loop_ms / ms, 2),
           "rel_err_mean": float(np.mean(rel)), "rel_err_max": float(np.max(rel)),
           "arithmetic": "fp32 (FP64 Grams, Cholesky and error sums)",
           "bf16": {"ms_per_run": round(ms_bf, 3), "problems_per_s": round(len(shapes) / (ms_bf * 1e-3), 1),
                    "q": w["q"] + 1, "all_ok": all(x == 0 for x in status_bf),
                    "rel_err_mean": float(np.mean(rel_bf)), "rel_err_max": float(np.max(rel_bf)),
                    "max_ratio_to_fp32": float(np.max(np.asarray(rel_bf) / np.asarray(rel))),
                    "arithmetic": "X passes bf16 MFMA (X rounded, operand split hi+lo), fp32 accumulate"},
           "note": "one persistent launch per run, captured in a HIP graph; per-problem range finder, "
                   "compression, sweeps and error run inside one workgroup"}
    del b, probs
    torch.cuda.empty_cache()
    return out


def xpass_kernels(rn, torch, step, m, n, l):
    """Device time of each X-pass kernel in one factorize step of each form,
    from torch.profiler (the HIP runtime's kernel records): GB/s of X moved
    per pass, fraction of 8 TB/s, and the matrix cores' utilisation against
    the dense peak of the arithmetic they run (executed products: the BF16
    compression's split operand doubles them)."""
    import re
    from torch.profiler import profile, ProfilerActivity
    lp = ((l + 15) // 16) * 16
    kinds = {
        "nn_bf16": (r"nn2_kernel<unsigned short", 2, 2 * m * n * lp, PEAK_BF16_TFLOPS),
        "tn_bf16_one_plane": (r"tn2_kernel<unsigned short, \d+, 1>", 2, 2 * m * n * lp, PEAK_BF16_TFLOPS),
        "tn_bf16_hi_lo": (r"tn2_kernel<unsigned short, \d+, 2>", 2, 2 * 2 * m * n * lp, PEAK_BF16_TFLOPS),
        "nn_fp32": (r"nn2_kernel<float", 4, 2 * m * n * lp, PEAK_FP32_MFMA_TFLOPS),
        "tn_fp32": (r"tn2_kernel<float", 4, 2 * m * n * lp, PEAK_FP32_MFMA_TFLOPS),
        "cast_bf16": (r"cast_bf16_kernel", 6, 0, None),
    }
    times = {key: [] for key in kinds}
    try:
        for prec in ("bf16", "fp32"):
            torch.cuda.synchronize()
            with profile(activities=[ProfilerActivity.CUDA]) as prof:
                step(prec, 1)
                torch.cuda.synchronize()
            for e in prof.events():
                dt = getattr(e, "device_time", 0.0) or 0.0
                if dt <= 0.0:
                    continue
                for key, (pat, _, _, _) in kinds.items():
                    if re.search(pat, e.name):
                        times[key].append(dt)
    except Exception as ex:  # the profiler is optional context for the line
        return {"error": str(ex)[:200]}
    out = {}
    for key, (pat, es, flops, peak) in kinds.items():
        if not times[key]:
            continue
        us = statistics.mean(times[key])
        gbps = m * n * es / (us * 1e-6) / 1e9
        d = {"calls": len(times[key]), "us": round(us, 1), "x_GBps": round(gbps, 1),
             "frac_of_8TBps": round(gbps / PEAK_HBM_GBPS, 4)}
        if peak:
            d["mfma_TFLOPs"] = round(flops / (us * 1e-6) / 1e12, 2)
            d["frac_of_mfma_peak"] = round(flops / (us * 1e-6) / 1e12 / peak, 4)
        out[key] = d
    out["note"] = ("bytes: X once per pass (cast: 4 B read + 2 B written per element); MFMA flops as executed "
                   f"(l = {l} padded to {lp} columns; the BF16 compression B = Q^T X reads hi + lo operand planes, "
                   "the passes of the subspace iteration one plane)")
    return out


def speedup_series(rn, torch, X, ks, p, q, nsw=20, sweeps=200):
    """HALS against randomized HALS for several ranks k on one X (FP32,
    seeded uniform starts; Sec. 4.4, the figure on varying k): per-sweep time
    of each (events over an nsw-sweep launch) and the end-to-end time of
    `sweeps` sweeps (HALS: sweeps x its per-sweep time; rHALS: one
    rnmf_factorize run of `sweeps` sweeps, range finder, compression and
    final error included)."""
    out = []
    m, n = X.shape
    dev = X.device
    st = torch.cuda.current_stream(dev)
    for k in ks:
        g = torch.Generator(device="cpu").manual_seed(1000 + k)
        W0 = torch.rand((m, k), generator=g).to(dev)
        H0 = torch.rand((k, n), generator=g).to(dev)
        W, H = W0.clone(), H0.clone()
        hws = rn._workspace(rn.workspace_bytes(rn.OP_HALS, m, n, rn.make_opts(k, 0, 0)), dev)
        rn.hals(X, W, H, nsweeps=1, ws=hws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        rn.hals(X, W, H, nsweeps=nsw, ws=hws)
        e1.record(st)
        e1.synchronize()
        h_ms = e0.elapsed_time(e1) / nsw
        del hws
        rn.factorize(X, k, p, q, max_iter=nsw, precision="fp32", W0=W0, H0=H0)  # warm-up
        _, _, info = rn.factorize(X, k, p, q, max_iter=sweeps, precision="fp32", W0=W0, H0=H0)
        r_ms = info["ms_sweeps"] / sweeps
        r_run = info["ms_qb"] + info["ms_sweeps"] + info["ms_error"]
        out.append({"k": k, "l": info["l"], "hals_ms_per_sweep": round(h_ms, 4), "rhals_ms_per_sweep": round(r_ms, 4),
                    "rhals_ms_qb": round(info["ms_qb"], 3), "speedup_per_sweep": round(h_ms / r_ms, 3),
                    "hals_ms_run": round(h_ms * sweeps, 2), "rhals_ms_run": round(r_run, 2),
                    "speedup_run": round(h_ms * sweeps / r_run, 3), "rhals_rel_err": info["rel_err"]})
        log(f"{m}x{n} k={k}: HALS {h_ms:.3f} ms/sweep, rHALS {r_ms:.3f} ms/sweep ({h_ms / r_ms:.2f}x), "
            f"{sweeps}-sweep runs {h_ms * sweeps:.1f} vs {r_run:.1f} ms ({h_ms * sweeps / r_run:.2f}x)")
        torch.cuda.empty_cache()
    return out


def speedup_study(rn, torch, synth, X, p, q, ks, dev):
    """The speedup study of Sec. 4.4 on both of its matrix shapes: the
    benchmark's 100,000 x 5,000 X and a 25,000 x 25,000 rank-50 product."""
    out = {"ks": ks, "sweeps": 200, "precision": "fp32",
           "tall_100000x5000": speedup_series(rn, torch, X, ks, p, q)}
    Xs, _, _, _, _ = synth.make("square_25000x25000", threads=min(16, os.cpu_count() or 1))
    Xd = torch.from_numpy(Xs).to(dev)
    del Xs
    out["square_25000x25000"] = speedup_series(rn, torch, Xd, ks, p, q)
    del Xd
    torch.cuda.empty_cache()
    out["note"] = ("per sweep: HALS streams X twice, rHALS sweeps on B; run: HALS sweeps x its per-sweep time "
                   "against one rnmf_factorize of the same sweeps (range finder and error included)")
    return out


def _sub_err(X, W, H, rows):
    import numpy as np
    Xs = X[rows].astype(np.float64)
    return float(np.linalg.norm(Xs - W[rows].astype(np.float64) @ H.astype(np.float64)) / np.linalg.norm(Xs))


def cpu_baseline(Xh, Omh, W0h, H0h, k, q, sweeps, gpu_factors, synth, w):
    """The FP64 oracle on the host's cores, on the same workload: the full QB
    stage and all `sweeps` sweeps (about 20 s on 16 cores), timed as the
    baseline (sweeps per second of the whole factorisation).  Its final
    relative error, on the whole matrix and on the 10,000-row subsample of
    row chunks, is put beside each GPU form's; a second oracle run with q + 1
    subspace iterations is the reference for the BF16 form (q + 1)."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max((d.get("num_threads", 0) for d in threadpool_info()), default=os.cpu_count())
    except Exception:
        cores = os.cpu_count()
    m = Xh.shape[0]
    rows = np.concatenate([np.arange(c * synth.CHUNK_ROWS, min(m, (c + 1) * synth.CHUNK_ROWS))
                           for c in synth.subsample_chunks(m, 10, w["seed"])])
    X = Xh.astype(np.float64)
    res = {}
    for qq in (q, q + 1):
        t = time.perf_counter()
        Q, B = oracle.qb(X, Omh.astype(np.float64), qq)
        t_qb = time.perf_counter() - t
        W, H = W0h.astype(np.float64), H0h.astype(np.float64)
        Wt = Q.T @ W
        t = time.perf_counter()
        for _ in range(sweeps):
            W, Wt, H = oracle.rhals_sweep(Q, B, W, Wt, H)
        t_sw = time.perf_counter() - t
        res[qq] = dict(t_qb=t_qb, t_sw=t_sw, rel_err=oracle.rel_error(X, W, H), sub=_sub_err(Xh, W, H, rows))
        log(f"oracle q={qq}: QB {t_qb:.2f}s, {sweeps} sweeps {t_sw:.1f}s on {cores} threads, "
            f"rel_err {res[qq]['rel_err']:.8f}")
    base = res[q]
    cpu = {"value": round(sweeps / (base["t_qb"] + base["t_sw"]), 4), "unit": "iters/s", "cores": cores,
           "kind": "oracle",
           "sample": f"the whole workload in FP64 (100000x5000, q={q}): QB stage ({base['t_qb']:.2f} s) + "
                     f"{sweeps} sweeps ({base['t_sw']:.1f} s); the final error is not timed"}
    parity = {"subsample_rows": int(rows.size)}
    for prec, qq in (("fp32", q), ("bf16", q + 1)):
        Wg, Hg = gpu_factors[prec]
        eg = oracle.rel_error(X, Wg, Hg)
        sg = _sub_err(Xh, Wg, Hg, rows)
        o = res[qq]
        parity[prec] = {"q": qq, "gpu_rel_err": eg, "oracle_rel_err": o["rel_err"],
                        "abs_diff": abs(eg - o["rel_err"]), "ratio": eg / o["rel_err"],
                        "gpu_rel_err_subsample": sg, "oracle_rel_err_subsample": o["sub"],
                        "abs_diff_subsample": abs(sg - o["sub"])}
    parity["bf16"]["ratio_to_oracle_q"] = parity["bf16"]["gpu_rel_err"] / res[q]["rel_err"]
    parity["bars"] = "fp32: abs_diff <= 1e-4; bf16: ratio <= 1.01 (both oracle runs)"
    return cpu, parity


if __name__ == "__main__":
    main()
