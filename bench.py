#!/usr/bin/env python3
"""Benchmark: restored MPix/s to the oracle-converged PSNR, VE vs plain FP, on one MI355X; batched
throughput; serving throughput with p50/p99 latency.

Headline workload (the 256x256 deblurring configuration): a seeded 256x256 piecewise-smooth
image, uniform 9x9 blur, noise sigma sqrt(2), lambda 0.02, 15 CG iterations per FP call, seeded
TNRD-style denoiser (5 stages x 24 filters 5x5, 63-RBF influence functions), RRE with L = 5.

Protocol (headline)
  1. target PSNR* = PSNR of the FP64 oracle's plain FP run to a relative change < 1e-6
     (tests/golden/bench_target_deblur256.json, written by a script that calls only the oracle);
  2. instrumented, untimed: solves with max_fp_calls = n = 1, 2, ... find n*, the FP-call
     count from which every returned vector stays within 0.05 dB of PSNR*;
  3. timed: `steps` solves with max_fp_calls = n* (after `warmup` untimed ones). A step is one
     whole solve y -> x through the C ABI, inputs resident in HBM. value = pixels * steps /
     time; p50/p99 are per-solve latencies.
Forms: plain FP (FP32), VE (RRE) with FP32 filter banks, VE (RRE) with BF16 filter banks on
MFMA. `value` is the VE + BF16 form. The roofline object covers the dominant kernel (the fused
denoiser stage of that form), timed with HIP events on the library's stream; the same kernel
on a 2048 x 2048 image (16384 tiles, every CU busy) is reported beside it.

Batched (64 images, sides log-uniform 128..1024, uniform 9x9 or Gaussian 7x7 blur, sigma sqrt(2)
or 5): one redve_solve_batch to a relative change < 1e-5 per image; each image's PSNR is
checked against its own plain-FP fixed point (GPU FP32, relative change < 1e-6).
Serving (Poisson arrivals, sides log-uniform 128..2048, deblurring 9x9 or 3x super-resolution):
saturation throughput with every request queued at once, then a Poisson trace at 0.7 x that
request rate; latency = completion - submission.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BAND_DB = 0.05


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nmax", type=int, default=40, help="longest instrumented solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="least host time the oracle baseline is sampled for")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-images", type=int, default=64)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sd", action="store_true")
    ap.add_argument("--no-torch-profiler", action="store_true",
                    help="skip the per-kernel splits taken with torch's profiler (for runs under "
                         "rocprofv3, which records the kernels itself)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="timed requests of the serving trace (after --serve-warmup more)")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-distinct", type=int, default=200,
                    help="distinct seeded problems the trace's requests cycle through")
    ap.add_argument("--no-sr", action="store_true",
                    help="skip the 512x512 3x super-resolution workload")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-max-active", type=int, default=64)
    ap.add_argument("--cost-protocol", action="store_true",
                    help="run only the cost-based comparison (FP calls VE needs to reach the cost "
                         "of 200 FP calls, m in {0,5,10}, kappa in {3,5,10}) and print it")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run only a calibration copy and the dominant kernels (for rocprofv3 "
                         "--pmc FETCH_SIZE / WRITE_SIZE runs), print nothing")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


NO_TORCH_PROFILER = False


def main():
    global NO_TORCH_PROFILER
    args = parse()
    NO_TORCH_PROFILER = args.no_torch_profiler
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the restoration of one image runs on one device and "
              "the library has no multi-GPU path (--gpus 1 only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workload as W
    from paper_1805_02158_amd import Restorer

    set_denoiser_shape(W.make_denoiser())
    target = json.load(open(os.path.join(ROOT, "tests", "golden", "bench_target_deblur256.json")))
    psnr_star = target["psnr_star_db"]

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = W.problem("deblur256")
    H, Wd = prob.hr_shape
    npx = H * Wd
    x_true = torch.tensor(prob.x_true, dtype=torch.float32, device=dev)
    noise = torch.tensor(prob.noise, dtype=torch.float32, device=dev)

    R = Restorer(0)
    R.configure(prob, method="rre", L=prob.L, m=0, tol=0.0)
    y = R.apply_H(x_true) + float(prob.sigma) * noise  # observation, eq. (1)
    torch.cuda.synchronize()
    if args.pmc_probe:
        pmc_probe(torch, R, prob, y)
        return
    if args.cost_protocol:
        print(json.dumps(cost_protocol(torch, W, Restorer)), flush=True)
        return

    def psnr(x, ref=x_true):
        mse = torch.mean((x.double() - ref.double()) ** 2).item()
        return 10.0 * math.log10(255.0 ** 2 / mse)

    out = torch.empty((H, Wd), dtype=torch.float32, device=dev)

    state = {"prec": "fp32", "lin": "cg"}  # configure() above loaded the FP32 banks

    def solve(method, prec, calls, lin="cg"):
        if state["prec"] != prec:
            R.set_denoiser(prob.denoiser, prec)
            state["prec"] = prec
        if state["lin"] != lin:
            R.set_linear_solver(lin)
            state["lin"] = lin
        R.set_extrapolation(method, prob.L, 0)
        R.set_solver(prob.cg_iters, calls, 0.0, 0)
        _, st = R.solve(y, H, Wd, out=out)
        return st

    def n_star(method, prec, lin="cg"):
        trace = []
        for n in range(1, args.nmax + 1):
            solve(method, prec, n, lin)
            trace.append((n, psnr(out)))
        ns = None
        for n, p in trace:
            if abs(p - psnr_star) <= BAND_DB:
                ns = n if ns is None else ns
            else:
                ns = None
        return ns, trace

    def timed(method, prec, calls, lin="cg"):
        for _ in range(args.warmup):
            solve(method, prec, calls, lin)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            st = solve(method, prec, calls, lin)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        return {"mpix_s": npx * args.steps / total / 1e6, "ms_per_step": total / args.steps * 1e3,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "fp_calls_to_target": calls, "cycles": st["cycles"], "psnr_db": psnr(out)}

    # the three forms of the configuration (15 CG iterations per FP call), then, beside them,
    # RRE + BF16 with the exact Fourier linear step (F4) in place of CG
    forms = {"plain_fp32": ("none", "fp32", "cg"), "ve_fp32": ("rre", "fp32", "cg"),
             "ve_bf16": ("rre", "bf16", "cg"), "ve_bf16_fft": ("rre", "bf16", "fft")}
    res_forms = {}
    for name, (method, prec, lin) in forms.items():
        ns, tr = n_star(method, prec, lin)
        if ns is None:
            print(json.dumps({"error": f"target PSNR not reached by {name}", "trace": tr}))
            sys.exit(1)
        res_forms[name] = timed(method, prec, ns, lin)
        res_forms[name]["linear_step"] = lin
        res_forms[name]["roofline_whole_solve"] = whole_solve_roofline(
            npx * ns / (res_forms[name]["ms_per_step"] * 1e-3), prec, prob.cg_iters, lin)
        log(name, res_forms[name])
    solve("rre", "bf16", 1, "cg")  # back to the CG linear step
    ve = res_forms["ve_bf16"]
    fp = res_forms["plain_fp32"]

    # ---- rooflines of the two kernels of an FP call, timed with HIP events on the library's
    # stream (torch's current stream): the fused denoiser stage of the headline form (BF16
    # banks) and the CG kernel; `roofline` is the one with the larger share of an FP call
    # (5 stages, 15 CG iterations) at the headline size. The library runs two CG iterations
    # per launch (k_cg_block) for a separable square 7x7 or 9x9 PSF without decimation on
    # images of fewer than 512 16x16 tiles (256x256 here), one (k_cg_iter) otherwise.
    R.set_denoiser(prob.denoiser, "bf16")
    stage_us = time_stage(torch, R, y, prob.denoiser.stages)
    blk_us = 2 * time_cg_iter(torch, R, y)  # 30 iterations = 15 launches of two
    roof_stage = roofline_stage(npx, stage_us, "k_tnrd_stage_bf16", "bf16")
    roof_cg = roofline_cg(npx, blk_us, "k_cg_block<4>", 2)
    share = {"k_tnrd_stage_bf16": prob.denoiser.stages * stage_us,
             "k_cg_block<4>": (prob.cg_iters // 2) * blk_us}
    roof = roof_cg if share["k_cg_block<4>"] >= share["k_tnrd_stage_bf16"] else roof_stage
    roof["share_of_fp_call_us"] = share
    big = torch.tensor(W.make_image(2048, 2048, 77), dtype=torch.float32, device=dev)
    stage_big_us = time_stage(torch, R, big, prob.denoiser.stages)
    roof_big = roofline_stage(big.numel(), stage_big_us, "k_tnrd_stage_bf16", "bf16")
    cg_big_us = time_cg_iter(torch, R, big)
    # the one-iteration kernel the rules pick there: 32x32 tiles keeping r, p, d only
    cg_big_kernel = "k_cg_iter32<4>" if R.get_tuning(2048, 2048)[0]["cg_tile"] == 32 else "k_cg_iter<4>"
    roof_cg_big = roofline_cg(big.numel(), cg_big_us, cg_big_kernel, 1)
    R.set_denoiser(prob.denoiser, "fp32")
    stage32_big_us = time_stage(torch, R, big, prob.denoiser.stages)
    roof32_big = roofline_stage(big.numel(), stage32_big_us, "k_tnrd_stage_f32", "fp32")
    del big

    res = {
        "metric": "restored MPix/s to oracle-converged PSNR (VE vs plain FP); p50/p99 solve latency",
        "value": ve["mpix_s"],
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ve["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded piecewise-smooth image, seeded TNRD-style denoiser)",
        "config": {"workload": "deblur 256x256, uniform 9x9 blur, sigma sqrt(2), lambda 0.02, "
                               "15 CG/FP call, TNRD-style D 5x24x(5x5), RRE L=5 m=0",
                   "method": "FP + RRE (L=5)",
                   "precision": "BF16 filter-bank operands on MFMA with FP32 accumulation; "
                                "RBF influence, update and CG in FP32; VE Gram/solve in FP64",
                   "forms": {"value (ve_bf16)": "the mixed-precision form (BF16 banks) of this "
                                                "workload, RRE L=5",
                             "ve_fp32": "the FP32 form of this workload, RRE L=5",
                             "plain_fp32": "plain FP, FP32",
                             "ve_bf16_fft": "RRE L=5, BF16 banks, exact Fourier linear step "
                                            "instead of 15 CG iterations"},
                   "fp_calls_to_target": ve["fp_calls_to_target"],
                   "psnr_target_db": psnr_star, "band_db": BAND_DB},
        "p50_ms": ve["p50_ms"],
        "p99_ms": ve["p99_ms"],
        "psnr_db": ve["psnr_db"],
        "forms": res_forms,
        "ve_bf16_speedup_vs_plain_fp32": fp["ms_per_step"] / ve["ms_per_step"],
        "roofline": roof,
        "roofline_kernels": {"k_tnrd_stage_bf16": roof_stage, "k_cg_block<4>": roof_cg},
        "roofline_2048x2048": {"k_tnrd_stage_bf16": roof_big, "k_tnrd_stage_f32": roof32_big,
                               cg_big_kernel: roof_cg_big},
    }
    if not args.no_sd:
        res["steepest_descent"] = bench_sd(args, torch, np, R, prob, y, out, psnr, psnr_star)
    res["ve_kernels_2048x2048"] = bench_ve_kernels(torch, W, Restorer, prob)
    res["fft_kernels_2048x2048"] = bench_fft_kernels(torch, W, Restorer, prob)
    if not args.no_sr:
        res["sr512"] = bench_sr(args, torch, np, W, Restorer)
    if not args.no_batch:
        res["batched"] = bench_batch(args, torch, np, W, Restorer, psnr)
    if not args.no_serve:
        res["serving"] = bench_serve(args, torch, np, W, Restorer)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(prob, ve["fp_calls_to_target"], args.cpu_seconds)
    print(json.dumps(res), flush=True)


def time_stage(torch, R, x, stages, reps=20):
    """Average duration of one denoiser stage launch: HIP events around `reps` denoiser calls
    (each `stages` launches back to back) on the library's stream."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    R.denoise(x)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        R.denoise(x)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / (reps * stages)


def time_cg_iter(torch, R, x, reps=10):
    """Average time of one CG iteration: HIP events around `reps` CG runs of 45 and of 15
    iterations (the same set-up launches); the difference over 30 * reps iterations."""
    stream = torch.cuda.current_stream()

    def run(iters):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            R.cg(x, x, iters)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    run(15)
    return (run(45) - run(15)) * 1e3 / (30 * reps)


# Algorithmic HBM traffic of one CG iteration per pixel (x, r, p each read and written once,
# A p never stored), and the published MI355X HBM3E bandwidth.
CG_BYTES_PER_PX = 24
HBM_PEAK_GBS = 8000.0


def roofline_cg(npx, launch_us, kernel, iters_per_launch):
    """CG is bound by HBM bandwidth (its stencil work is under 100 FLOP per pixel and
    iteration). achieved = algorithmic bytes per launch (24 B per pixel and iteration, times
    the iterations one launch takes) / average launch time. traffic: the bytes the FETCH_SIZE
    and WRITE_SIZE counters saw per launch at this size (profiles/traffic.json), null if the
    kernel's source changed since."""
    work = npx * CG_BYTES_PER_PX * iters_per_launch
    achieved = work / (launch_us * 1e-6) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_of(kernel, npx),
            "avg_launch_us": launch_us, "bytes_per_launch": work, "bytes_per_px": CG_BYTES_PER_PX,
            "iterations_per_launch": iters_per_launch, "pixels_per_launch": npx}


def traffic_of(kernel, npx):
    """HBM bytes per launch measured by the counters for this kernel at this size, if the
    source it was measured on is the current one."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    for e in json.load(open(path)):
        if e["kernel"] != kernel or e["pixels_per_launch"] != npx:
            continue
        src = os.path.join(ROOT, e["source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != e["source_sha256"]:
            return None
        return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
    return None


def pmc_probe(torch, R, prob, y):
    """Launches for the counter runs: 5 plain copies of 256 MiB (calibration: each moves
    exactly 256 MiB in and 256 MiB out), then at the headline size 5 CG runs of 15 iterations
    (FP32), 5 denoiser calls with BF16 banks and 5 FP calls with them (their last stage forms
    the CG start), then a CG run and a denoiser call on a 2048x2048 image and one denoiser
    call there with FP32 banks; CG runs with the one-iteration kernel forced to 32x32 tiles at
    2048x2048 and to either tile at 4096x4096; an FP call with the Fourier linear step and an
    RRE solve of 7 FP calls (one extrapolation) at 2048x2048; 3 rounds of the batched engine on
    the 64-image workload."""
    src = torch.rand(64 << 20, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    for _ in range(5):
        R.cg(y, y, prob.cg_iters)
    R.set_denoiser(prob.denoiser, "bf16")
    for _ in range(5):
        R.denoise(y)
    for _ in range(5):
        R.fp_step(y, y)
    # the same kernels with every CU busy (2048x2048: 16384 tiles)
    import workload as W
    big = torch.tensor(W.make_image(2048, 2048, 77), dtype=torch.float32, device="cuda")
    R.cg(big, big, prob.cg_iters)
    R.denoise(big)
    R.set_denoiser(prob.denoiser, "fp32")
    R.denoise(big)
    R.set_tuning({"cg_per_launch": 1, "cg_tile": 32})
    R.cg(big, big, prob.cg_iters)
    huge = torch.tensor(W.make_image(4096, 4096, 78), dtype=torch.float32, device="cuda")
    R.cg(huge, huge, prob.cg_iters)
    R.set_tuning({"cg_per_launch": 1, "cg_tile": 16})
    R.cg(huge, huge, prob.cg_iters)
    R.set_tuning(None)
    del huge
    R.set_denoiser(prob.denoiser, "bf16").set_linear_solver("fft")
    R.fp_step(big, big)
    R.set_linear_solver("cg")
    out = torch.empty_like(big)
    R.set_extrapolation("rre", prob.L, 0).set_solver(prob.cg_iters, prob.L + 2, 0.0, 0)
    R.solve(big, 2048, 2048, out=out)
    torch.cuda.synchronize()
    probs = W.batch_items(64)
    items = [dict(y=torch.tensor(p.x_true, dtype=torch.float32, device="cuda"), hx=p.hr_shape[0],
                  wx=p.hr_shape[1], psf=p.psf, decim=p.decim, sigma=p.sigma, lam=p.lam)
             for p in probs]
    R.set_solver(prob.cg_iters, 3, 0.0, 0)
    R.solve_batch(items)
    torch.cuda.synchronize()


# Algorithmic work of one denoiser stage per output pixel, and the roofline that bounds each
# part (the stage runs them in one kernel, so its time is bounded by the slowest of the three):
#  * filter banks: forward and adjoint, F filters of 25 taps: 2 x F x 25 multiply-adds = 2400
#    FLOP for F = 24, on MFMA (BF16 operands: 2.5 PFLOP/s dense; FP32 operands: 157.3 TFLOP/s).
#    The MFMA tiles issue more than that (positions of the tile + halo, taps and filters padded):
#    per 16x16 tile 25 groups of 16 positions x (forward 32 taps x 32 filters + adjoint 32 x 32)
#    in BF16 = 6400 FLOP per pixel; in FP32 the K-steps stop at the last real tap or filter
#    (7 x 4 taps, 6 x 4 filters): 5200 FLOP per pixel.
#  * influence functions: F evaluations of the Gaussian RBF sum over the 2K + 1 centres nearest
#    z (K = 5 in the BF16 form, 7 in the FP32 form; the terms beyond add less than 1e-6 / 1e-12
#    of a weight, so this is the defined sum to the form's precision; all 63 centres would be
#    4.2x to 5.7x more), each term 8 vector-ALU slots (difference, square, scale; exp at a
#    quarter rate: 4; multiply-add), i.e. 16 FLOP-equivalents at the unpacked FP32 vector peak
#    (256 CUs x 64 lanes x 2.4 GHz x 2 = 78.6 TFLOP/s; the library is compiled with packed FP32
#    off, so the published 157.3 is not reachable).
#  * state: read u and f, write u: 12 B at 8 TB/s.
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}
VALU_PEAK_TFLOPS = 78.6
TERM_FLOP_EQ = 16
STAGE_STATE_BYTES = 12


# The denoiser whose stages are rated (set from the workload in main): filters F, their side k,
# RBF centres J and their spacing / width, stages T.
DENOISER = {"nfilt": 24, "ksize": 5, "nrbf": 63, "gamma_over_dmu": 1.0, "stages": 5}


def set_denoiser_shape(d):
    DENOISER.update(nfilt=int(d.nfilt), ksize=int(d.ksize), nrbf=int(d.nrbf),
                    gamma_over_dmu=float(d.gamma) / float(d.dmu), stages=int(d.stages))


def stage_work(prec):
    """Work of one stage per output pixel for the denoiser in DENOISER. The window half-width K
    follows the library's rule, (K + 1/2) dmu >= reach gamma with reach 5.2565 (BF16: terms
    below 1e-6 of a weight) or 7.4338 (FP32: 1e-12); the issued bank FLOP count the MFMA tile's
    padding (taps to 32, filters to 32, 400 positions per 256 outputs; FP32 K-steps stop at the
    last real tap or filter)."""
    F, k, J = DENOISER["nfilt"], DENOISER["ksize"], DENOISER["nrbf"]
    reach = 5.2565 if prec == "bf16" else 7.4338
    K = max(1, math.ceil(reach * DENOISER["gamma_over_dmu"] - 0.5))
    terms = F * min(2 * K + 1, J)
    taps = k * k
    if prec == "bf16":
        issued = 2 * 32 * 32 * 2 * 400 / 256
    else:
        issued = (math.ceil(taps / 4) * 4 * 32 + math.ceil(F / 4) * 4 * 32) * 2 * 400 / 256
    return {"bank_flop_px": 2 * F * taps * 2, "bank_issued_flop_px": issued,
            "phi_terms_px": terms, "phi_flop_eq_px": terms * TERM_FLOP_EQ,
            "state_bytes_px": STAGE_STATE_BYTES, "window_K": K, "filters": F, "centres": J}


def stage_bound_ps(prec):
    """Roofline time of one stage per pixel (ps): the slowest of banks, phi and state."""
    w = stage_work(prec)
    return max(w["bank_flop_px"] / MFMA_PEAK_TFLOPS[prec], w["phi_flop_eq_px"] / VALU_PEAK_TFLOPS,
               w["state_bytes_px"] / HBM_PEAK_GBS * 1e3)


def roofline_stage(npx, stage_us, kernel, prec):
    """The fused denoiser stage: bound by the influence functions on the vector ALUs (their
    roofline time is 30-50x the banks' on MFMA and 35-50x the state traffic's). achieved = the
    influence functions' FLOP-equivalents per launch / average launch time, against the unpacked
    vector peak; the banks' MFMA utilisation (algorithmic and issued FLOP against the MFMA peak
    of their operand type) and the state traffic are reported beside it."""
    w = stage_work(prec)
    t = stage_us * 1e-6
    achieved = npx * w["phi_flop_eq_px"] / t / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS,
            "traffic": traffic_of(kernel, npx), "avg_launch_us": stage_us,
            "flop_per_launch": npx * w["phi_flop_eq_px"], "pixels_per_launch": npx,
            "work_per_px": w,
            "banks_mfma": {"bound": "mfma", "peak": MFMA_PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                           "achieved_algorithmic": npx * w["bank_flop_px"] / t / 1e12,
                           "frac_algorithmic": npx * w["bank_flop_px"] / t / 1e12
                           / MFMA_PEAK_TFLOPS[prec],
                           "achieved_issued": npx * w["bank_issued_flop_px"] / t / 1e12,
                           "frac_issued": npx * w["bank_issued_flop_px"] / t / 1e12
                           / MFMA_PEAK_TFLOPS[prec]},
            "state_hbm": {"achieved_gbs": npx * STAGE_STATE_BYTES / t / 1e9,
                          "frac": npx * STAGE_STATE_BYTES / t / 1e9 / HBM_PEAK_GBS}}


def bench_sd(args, torch, np, R, prob, y, out, psnr, psnr_star, nmax=2000, nmax_ve=300):
    """Steepest descent as the base iteration (x - mu g(x), default mu; Sec. IV), plain and
    with MPE (kappa = 8, L = 9) at the headline workload, BF16 banks: FP-call count n* to the
    same target band, and the timed solve of n* calls."""
    H, Wd = prob.hr_shape
    npx = H * Wd
    R.set_denoiser(prob.denoiser, "bf16")
    R.set_base("sd", 0.0)
    res = {"workload": "deblur 256x256 as the headline, steepest descent with the default step "
                       "1 / (||H||^2/sigma^2 + 2 lambda), BF16 banks"}

    def band_start(trace):
        ns = None
        for n, p in trace:
            if abs(p - psnr_star) <= BAND_DB:
                ns = n if ns is None else ns
            else:
                ns = None
        return ns

    # plain SD: one step at a time (every iterate is a returned vector)
    x = y.clone()
    trace = []
    for n in range(1, nmax + 1):
        x = R.fp_step(y, x)
        trace.append((n, psnr(x)))
    ns_sd = band_start(trace)
    # SD-MPE: solves of n calls
    trace = []
    for n in range(1, nmax_ve + 1):
        R.set_extrapolation("mpe", 9, 0)
        R.set_solver(prob.cg_iters, n, 0.0, 0)
        R.solve(y, H, Wd, out=out)
        trace.append((n, psnr(out)))
    ns_ve = band_start(trace)

    def timed(method, L, calls, steps=10):
        R.set_extrapolation(method, L, 0)
        R.set_solver(prob.cg_iters, calls, 0.0, 0)
        R.solve(y, H, Wd, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            R.solve(y, H, Wd, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        return {"fp_calls_to_target": calls, "mpix_s": npx / dt / 1e6, "ms_per_solve": dt * 1e3,
                "psnr_db": psnr(out)}

    res["plain_sd"] = timed("none", 5, ns_sd) if ns_sd else {"fp_calls_to_target": None,
                                                              "searched_up_to": nmax}
    res["sd_mpe_L9"] = timed("mpe", 9, ns_ve) if ns_ve else {"fp_calls_to_target": None,
                                                              "searched_up_to": nmax_ve}
    R.set_base("fp", 0.0)
    log("steepest descent", res)
    return res


def cost_protocol(torch, W, Restorer, fp_calls=200):
    """The cost-based comparison of Sec. IV (Tables I-II): E* = E(x after fp_calls plain FP
    calls), E of eq. (4); for MPE and RRE with m in {0, 5, 10} and kappa in {3, 5, 10}
    (L = kappa + 1 difference columns), the smallest FP-call count at the end of a cycle whose
    vector has E <= E* (None: not within fp_calls). Synthetic stand-ins for the paper's images:
    the 256x256 deblurring and the 512x512 3x super-resolution workloads, FP32 banks."""
    out = {"metric": "FP calls for extrapolation to reach the objective of 200 plain FP calls",
           "fp_calls": fp_calls, "workloads": {}}
    for name in ("deblur256", "sr512"):
        prob = W.problem(name)
        R = Restorer(0)
        R.configure(prob, method="none", tol=0.0, max_fp_calls=fp_calls)
        xt = torch.tensor(prob.x_true, dtype=torch.float32, device="cuda")
        nz = torch.tensor(prob.noise, dtype=torch.float32, device="cuda")
        y = R.apply_H(xt) + float(prob.sigma) * nz
        H, Wd = prob.hr_shape
        t0 = time.perf_counter()
        x, _ = R.solve(y, H, Wd)
        e_star = R.objective(y, x)
        res = {"E_fp": e_star}
        for method in ("mpe", "rre"):
            table = {}
            for m in (0, 5, 10):
                for kappa in (3, 5, 10):
                    L, cyc, hit = kappa + 1, m + kappa + 1, None
                    R.set_extrapolation(method, L, m)
                    for c in range(1, fp_calls // cyc + 1):
                        R.set_solver(prob.cg_iters, c * cyc, 0.0, 0)
                        xn, _ = R.solve(y, H, Wd)
                        if R.objective(y, xn) <= e_star:
                            hit = c * cyc
                            break
                    table[f"m{m}_k{kappa}"] = hit
            res[method] = table
        res["seconds"] = time.perf_counter() - t0
        out["workloads"][name] = res
        log("cost protocol", name, res)
        R.close()
    return out


def observe(torch, R, probs):
    """y = H x_true + sigma n on the GPU (each problem's own operator)."""
    ys = []
    for p in probs:
        R.set_operator(p.psf, p.decim)
        xt = torch.tensor(p.x_true, dtype=torch.float32, device="cuda")
        n = torch.tensor(p.noise, dtype=torch.float32, device="cuda")
        ys.append(R.apply_H(xt) + float(p.sigma) * n)
    torch.cuda.synchronize()
    return ys


# Whole-solve roofline: the declared work of one FP call per pixel, by kernel class, each at its
# own roofline, summed (the classes run one after another): the denoiser's 5 stages (each the
# slowest of its banks on MFMA, its influence functions on the vector ALUs and its 12 B of
# state, see stage_bound_ps), the linear step (CG: n_cg x 24 B, x, r, p read and written once
# per iteration; the exact Fourier step: 30 B, r0 read and the half spectrum written by the row
# pass (4 + 4), the half spectrum and its scale factors read and the spectrum written by the
# column pass (4 + 2 + 4), the spectrum, x_in read and x_out written by the inverse row pass
# (4 + 4 + 4)) and the extrapolation's difference and combination passes (16.8 B per FP call
# for L = 5: u written, the Gram reads and the combination spread over a cycle of 5 calls).
FFT_BYTES_PER_PX = 30


def roofline_ps_per_px_call(prec="bf16", n_cg=15, linear="cg"):
    stages = DENOISER["stages"] * stage_bound_ps(prec)
    lin = (n_cg * CG_BYTES_PER_PX if linear == "cg" else FFT_BYTES_PER_PX) / HBM_PEAK_GBS * 1e3
    ve = 16.8 / HBM_PEAK_GBS * 1e3
    return {"stages_ps": stages, "linear_ps": lin, "ve_ps": ve, "total_ps": stages + lin + ve,
            "precision": prec, "linear_step": linear}


def whole_solve_roofline(px_calls_per_s, prec="bf16", n_cg=15, linear="cg"):
    """Fraction of the whole-solve roofline: declared time per pixel per FP call over the measured
    one (pixel-FP-calls per second)."""
    r = roofline_ps_per_px_call(prec, n_cg, linear)
    measured = 1e12 / px_calls_per_s
    return {"declared_ps_per_px_fp_call": r, "measured_ps_per_px_fp_call": measured,
            "frac": r["total_ps"] / measured}


def batch_kernels(torch, run, prec, px_calls, n_cg=15):
    """Per kernel class of one batched solve (profiler device times): launches, total time,
    share, and for the dominant classes the achieved rate over the whole solve: the stage
    (5 per FP call; influence-function FLOP-equivalents against the unpacked vector peak) and
    the CG iterations (24 B per pixel and iteration against HBM; the 32x32 form takes 14 of the
    15 per FP call, every image of this workload being on it)."""
    kt = kernel_times(torch, run)
    by = {}
    for name, (c, us) in kt.items():
        base = name.split("<")[0]
        bc, bu = by.get(base, (0, 0.0))
        by[base] = (bc + c, bu + us)
    total = sum(us for _, us in by.values())
    out = {k: {"launches": c, "total_ms": us / 1e3, "share": us / total}
           for k, (c, us) in sorted(by.items(), key=lambda kv: -kv[1][1])}
    w = stage_work(prec)
    for k in out:
        t = out[k]["total_ms"] * 1e-3
        if k.startswith("k_tnrd_stage"):
            a = DENOISER["stages"] * px_calls * w["phi_flop_eq_px"] / t / 1e12
            out[k].update({"bound": "alu", "achieved_tflops": a, "peak": VALU_PEAK_TFLOPS,
                           "frac": a / VALU_PEAK_TFLOPS})
        elif k in ("k_cg_iter_batch", "k_cg_iter32_batch"):
            # the 32x32 form takes every iteration but the last (pointwise, on the 16x16 list)
            # of the images on it; where it runs, the 16x16 form takes only those last ones
            iters = n_cg - 1 if k == "k_cg_iter32_batch" else (1 if "k_cg_iter32_batch" in out else n_cg)
            a = iters * px_calls * CG_BYTES_PER_PX / t / 1e9
            out[k].update({"bound": "hbm", "achieved_gbs": a, "peak": HBM_PEAK_GBS,
                           "frac": a / HBM_PEAK_GBS, "iterations_per_fp_call": iters})
    return out


def bench_batch(args, torch, np, W, Restorer, psnr):
    probs = W.batch_items(args.batch_images)
    R = Restorer(0)
    ys = observe(torch, R, probs)
    xts = [torch.tensor(p.x_true, dtype=torch.float32, device="cuda") for p in probs]
    items = [dict(y=y, hx=p.hr_shape[0], wx=p.hr_shape[1], psf=p.psf, decim=p.decim,
                  sigma=p.sigma, lam=p.lam) for p, y in zip(probs, ys)]
    mpix = sum(p.x_true.size for p in probs) / 1e6
    d = W.make_denoiser()

    def run(method, prec, tol, max_calls, switch=0.0):
        R.set_denoiser(d, prec).set_extrapolation(method, 5, 0).set_solver(15, max_calls, tol, 0)
        R.set_precision_switch(switch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs, st = R.solve_batch(items)
        return time.perf_counter() - t0, outs, st

    # each image's own converged PSNR: plain FP (FP32) to a relative change < 1e-6
    _, ref, ref_st = run("none", "fp32", 1e-6, 2000)
    ref_psnr = [psnr(o, xt) for o, xt in zip(ref, xts)]
    log("batched reference: calls", max(s["fp_calls"] for s in ref_st))
    out = {"workload": f"{len(probs)} images, sides log-uniform 128..1024, {mpix:.2f} MPix, "
                       "uniform 9x9 or Gaussian 7x7 blur, sigma sqrt(2) or 5, lambda 0.02, 15 CG",
           "stop": "per image: relative change < 1e-5",
           "reference": "per image: plain FP (FP32) to relative change < 1e-6",
           "mpix": mpix}
    # ve_bf16_switch: the BF16 form whose images move to FP32 banks once their relative change
    # falls below 1e-4 (the last cycles, where BF16 rounding slows the approach to 1e-5)
    for name, method, prec, reps, sw in (("ve_bf16", "rre", "bf16", 3, 0.0),
                                         ("ve_bf16_switch", "rre", "bf16", 3, 1e-4),
                                         ("ve_fp32", "rre", "fp32", 1, 0.0),
                                         ("plain_fp32", "none", "fp32", 1, 0.0)):
        run(method, prec, 1e-5, 500, sw)  # warm-up: workspace and graphs
        times = []
        for _ in range(reps):
            dt, outs, st = run(method, prec, 1e-5, 500, sw)
            times.append(dt)
        dt = float(np.median(times))
        dps = [psnr(o, xt) - rp for o, xt, rp in zip(outs, xts, ref_psnr)]
        calls = [s["fp_calls"] for s in st]
        out[name] = {"mpix_s": mpix / dt, "s_per_batch": dt,
                     "fp_calls_mean": float(np.mean(calls)), "fp_calls_max": int(max(calls)),
                     "mpix_fp_calls_per_s": sum(c * p.x_true.size for c, p in zip(calls, probs))
                     / dt / 1e6,
                     "images_within_band": int(sum(abs(v) <= BAND_DB for v in dps)),
                     "worst_dpsnr_db": float(min(dps))}
        out[name]["roofline_whole_solve"] = whole_solve_roofline(
            out[name]["mpix_fp_calls_per_s"] * 1e6, prec)
        out[name]["kernels"] = batch_kernels(
            torch, lambda: run(method, prec, 1e-5, 500, sw), prec,
            sum(c * p.x_true.size for c, p in zip(calls, probs)))
        if sw:
            out[name]["switch_rel_change"] = sw
            out[name]["note"] = ("stage work counted at the BF16 window (K=5) for every call, "
                                 "also those on FP32 banks (K=7): a lower bound of the rate")
        log("batched", name, out[name])
    out["ve_bf16_speedup_vs_plain_fp32"] = out["plain_fp32"]["s_per_batch"] / out["ve_bf16"]["s_per_batch"]
    out["ve_bf16_switch_speedup_vs_plain_fp32"] = (out["plain_fp32"]["s_per_batch"]
                                                   / out["ve_bf16_switch"]["s_per_batch"])
    R.set_precision_switch(0.0)
    R.close()
    return out


def bench_serve(args, torch, np, W, Restorer):
    """Continuous-batching server on the serving trace: requests with sides log-uniform in
    128..2048, deblurring (9x9 uniform) or 3x SR (Gaussian 7x7), sigma sqrt(2) or 5. The
    requests cycle through `serve_distinct` seeded problems of that distribution (their
    observations made once on the GPU); arrivals are a Poisson process. Saturation: every
    request queued at once (throughput). Then the same requests at 0.7 x that rate (latency
    p50 / p99 from submission to completion), `serve_warmup` requests first, untimed."""
    from paper_1805_02158_amd import Server
    trace = W.serve_trace(args.serve_distinct, 1.0)
    probs = [p for _, p in trace]
    R = Restorer(0)
    ys = observe(torch, R, probs)
    base = [dict(y=y, hx=p.hr_shape[0], wx=p.hr_shape[1], psf=p.psf, decim=p.decim,
                 sigma=p.sigma, lam=p.lam) for p, y in zip(probs, ys)]
    nw, nt = args.serve_warmup, args.serve_requests
    reqs = [base[i % len(base)] for i in range(nw + nt)]
    px = [base[i % len(base)]["hx"] * base[i % len(base)]["wx"] for i in range(nw + nt)]
    gaps = np.random.default_rng(4001).exponential(1.0, nw + nt)  # Poisson arrivals at rate 1
    R.set_denoiser(W.make_denoiser(), "bf16").set_extrapolation("rre", 5, 0).set_solver(15, 500, 1e-5, 0)
    budget = int(args.serve_budget_gb * (1 << 30))

    srv = Server(R, budget, args.serve_max_active)

    def serve(arrivals, rq):
        rounds0 = srv.counts()["rounds"]
        t0 = time.perf_counter()
        tickets = []
        for a, d in zip(arrivals, rq):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            tickets.append(srv.submit(**d)[0])
        st = [srv.wait(t) for t in tickets]
        makespan = time.perf_counter() - t0
        lat = np.array([s["ms"] for s in st])
        bad = sum(s["status"] != 0 for s in st)
        return makespan, lat, srv.counts()["rounds"] - rounds0, bad

    serve([0.0] * nw, reqs[:nw])  # warm-up: the graphs of the tile-list lengths
    mk, lat_sat, rounds_sat, bad = serve([0.0] * nt, reqs[nw:])
    mpix = sum(px[nw:]) / 1e6
    rate_sat = nt / mk
    log("serving saturation", f"{rate_sat:.1f} req/s, {mpix / mk:.1f} MPix/s")
    rate = 0.7 * rate_sat
    arr = np.cumsum(gaps) / rate
    serve(arr[:nw] - arr[0], reqs[:nw])  # warm-up at the trace's rate
    mk2, lat, rounds2, bad2 = serve(arr[nw:] - arr[nw], reqs[nw:])
    occ = srv.occupancy()
    srv.close()
    res = {"workload": f"{nt} requests after {nw} warm-up, cycling through {len(base)} seeded "
                       f"problems with sides log-uniform 128..2048 ({mpix:.1f} MPix timed), "
                       "deblur 9x9 uniform or 3x SR Gaussian 7x7, sigma sqrt(2) or 5, RRE L=5, "
                       "BF16 banks, stop at relative change < 1e-5",
           "hbm_budget_gb": args.serve_budget_gb, "max_active": args.serve_max_active,
           "occupancy": occ,
           "saturation": {"req_s": rate_sat, "mpix_s": mpix / mk, "rounds": rounds_sat,
                          "p50_ms": float(np.percentile(lat_sat, 50)),
                          "p99_ms": float(np.percentile(lat_sat, 99)), "failed": bad},
           "poisson": {"rate_req_s": rate, "mpix_s": mpix / mk2, "rounds": rounds2,
                       "p50_ms": float(np.percentile(lat, 50)),
                       "p99_ms": float(np.percentile(lat, 99)), "failed": bad2}}
    log("serving", res)
    R.close()
    return res


def bench_sr(args, torch, np, W, Restorer, steps=10):
    """The 512x512 3x super-resolution workload (Gaussian 7x7, sigma 5, lambda 0.02, 15 CG,
    RRE with L = 8): restored MPix/s to its oracle-converged PSNR (tests/golden/
    bench_target_sr512.json, written by a script that calls only the oracle), by the protocol
    of the headline workload: n* from untimed solves of n = 1, 2, ... FP calls (plain FP: from
    the FP iterates themselves), then `steps` timed solves of n* calls."""
    path = os.path.join(ROOT, "tests", "golden", "bench_target_sr512.json")
    if not os.path.exists(path):
        return {"skipped": "no oracle target for the 512x512 SR workload"}
    psnr_star = json.load(open(path))["psnr_star_db"]
    prob = W.problem("sr512")
    H, Wd = prob.hr_shape
    npx = H * Wd
    R = Restorer(0)
    R.configure(prob, method="rre", L=prob.L, m=0, tol=0.0)
    xt = torch.tensor(prob.x_true, dtype=torch.float32, device="cuda")
    y = R.apply_H(xt) + float(prob.sigma) * torch.tensor(prob.noise, dtype=torch.float32,
                                                            device="cuda")
    out = torch.empty((H, Wd), dtype=torch.float32, device="cuda")

    def psnr(x):
        mse = torch.mean((x.double() - xt.double()) ** 2).item()
        return 10.0 * math.log10(255.0 ** 2 / mse)

    def band_start(trace):
        ns = None
        for n, p in trace:
            if abs(p - psnr_star) <= BAND_DB:
                ns = n if ns is None else ns
            else:
                ns = None
        return ns

    res = {"workload": "512x512 3x super-resolution (171x171 observation), Gaussian 7x7 std 1.6, "
                       "sigma 5, lambda 0.02, 15 CG/FP call, TNRD-style D 5x24x(5x5), RRE L=8",
           "psnr_target_db": psnr_star}
    for name, method, prec, nmax in (("ve_bf16", "rre", "bf16", 80), ("ve_fp32", "rre", "fp32", 80),
                                     ("plain_fp32", "none", "fp32", 400)):
        R.set_denoiser(prob.denoiser, prec).set_extrapolation(method, prob.L, 0)
        trace = []
        if method == "none":
            R.set_solver(prob.cg_iters, 0, 0.0, 0)
            x = R.solve(y, H, Wd)[0]  # the initial vector (no FP call)
            for n in range(1, nmax + 1):
                x = R.fp_step(y, x)
                trace.append((n, psnr(x)))
        else:
            for n in range(1, nmax + 1):
                R.set_solver(prob.cg_iters, n, 0.0, 0)
                R.solve(y, H, Wd, out=out)
                trace.append((n, psnr(out)))
        ns = band_start(trace)
        if ns is None:
            res[name] = {"fp_calls_to_target": None, "searched_up_to": nmax}
            continue
        R.set_solver(prob.cg_iters, ns, 0.0, 0)
        R.solve(y, H, Wd, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            R.solve(y, H, Wd, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"fp_calls_to_target": ns, "mpix_s": npx / dt / 1e6, "ms_per_solve": dt * 1e3,
                     "psnr_db": psnr(out),
                     "roofline_whole_solve": whole_solve_roofline(npx * ns / dt, prec,
                                                                  prob.cg_iters)}
        log("sr512", name, res[name])
    R.close()
    return res


def kernel_times(torch, fn):
    """Device time of each kernel `fn` launches, from torch's profiler (it records the HIP
    kernels of every library in the process): {name: (launches, total microseconds)}."""
    if NO_TORCH_PROFILER:
        fn()
        torch.cuda.synchronize()
        return {}
    from torch.profiler import ProfilerActivity, profile
    torch.cuda.synchronize()
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        fn()
        torch.cuda.synchronize()
    import re
    out = {}
    for e in prof.key_averages():
        us = getattr(e, "device_time_total", None)
        if us is None:
            us = getattr(e, "cuda_time_total", 0.0)
        m = re.search(r"(k_[A-Za-z0-9_]+(<[^>(]*>)?)\(", e.key)
        if "redve::" not in e.key or us <= 0 or not m:
            continue
        name = m.group(1)
        c, t = out.get(name, (0, 0.0))
        out[name] = (c + e.count, t + us)
    return out


# Algorithmic HBM bytes per pixel of the extrapolation passes (window column j, L = 5):
# the difference pass reads x_new and x_old and the j earlier columns and writes u (12 + 4 j);
# the last CG iteration fused with it reads r, p, d and x_in (x_new is formed there, x_old is
# x_in) and the j columns and writes x_out and u (24 + 4 j, what the counters see); the
# combination reads x_m and the L - 1 columns of U_(kappa-1) and writes the result (4 (L + 1)).
def ve_bytes_per_px(kernel, L=5):
    if kernel.startswith("k_diff_gram<"):
        return 12 + 4 * int(kernel[len("k_diff_gram<"):-1])
    if kernel.startswith("k_cg_last_diff<"):
        return 24 + 4 * int(kernel[len("k_cg_last_diff<"):-1])
    if kernel == "k_ve_combine":
        return 4 * (L - 1 + 2)
    return None


def bench_ve_kernels(torch, W, Restorer, prob):
    """The extrapolation's streaming passes on a 2048 x 2048 image (4.19 M pixels, every CU
    busy), device times from the profiler: five extrapolations of a six-iterate window (L = 5)
    and one RRE cycle of five FP calls; achieved GB/s = algorithmic bytes / average duration."""
    npx = 2048 * 2048
    R = Restorer(0)
    R.configure(prob, precision="bf16", method="rre", L=5, m=0, tol=0.0, max_fp_calls=5)
    big = torch.tensor(W.make_image(2048, 2048, 77), dtype=torch.float32, device="cuda")
    xs = torch.stack([big + 0.01 * k * k for k in range(6)]).contiguous()
    R.extrapolate(xs)
    R.solve(big, 2048, 2048)

    def run():
        for _ in range(5):
            R.extrapolate(xs)
        R.solve(big, 2048, 2048)

    times = kernel_times(torch, run)
    out = {}
    for name, (count, us) in sorted(times.items()):
        b = ve_bytes_per_px(name)
        if b is None and name != "k_ve_solve":
            continue
        avg = us / count
        e = {"launches": count, "avg_us": avg}
        if b is not None:
            gbs = npx * b / (avg * 1e-6) / 1e9
            e.update({"bytes_per_px": b, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS})
        out[name] = e
    R.close()
    log("ve kernels 2048x2048", out)
    return {"pixels": npx, "peak_gbs": HBM_PEAK_GBS, "kernels": out}


# Algorithmic HBM bytes per pixel of the Fourier linear step's kernels (FFT_BYTES_PER_PX).
FFT_KERNEL_BYTES = {"k_fft_rows_fwd": 8, "k_fft_cols": 10, "k_fft_rows_inv": 12}


def bench_fft_kernels(torch, W, Restorer, prob):
    """The exact Fourier linear step's three kernels on a 2048 x 2048 image (device times from
    the profiler over five FP calls with BF16 banks): achieved GB/s = algorithmic bytes /
    average duration."""
    npx = 2048 * 2048
    R = Restorer(0)
    R.configure(prob, precision="bf16", method="none", tol=0.0)
    R.set_linear_solver("fft")
    big = torch.tensor(W.make_image(2048, 2048, 77), dtype=torch.float32, device="cuda")
    R.fp_step(big, big)

    def run():
        for _ in range(5):
            R.fp_step(big, big)

    times = kernel_times(torch, run)
    out = {}
    for name, (count, us) in sorted(times.items()):
        b = FFT_KERNEL_BYTES.get(name.split("<")[0])  # the row kernels are templates
        if b is None:
            continue
        avg = us / count
        gbs = npx * b / (avg * 1e-6) / 1e9
        out[name] = {"launches": count, "avg_us": avg, "bytes_per_px": b, "achieved_gbs": gbs,
                     "frac": gbs / HBM_PEAK_GBS}
    R.close()
    log("fft kernels 2048x2048", out)
    return {"pixels": npx, "peak_gbs": HBM_PEAK_GBS, "kernels": out}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, calls, min_seconds):
    """The FP64 oracle (plain C, OpenMP over rows/filters) on the host: whole RRE solves
    (L = 5, the GPU's FP-call count to the target) of the same image, repeated until at least
    `min_seconds` have passed (at most 50 solves), on all the threads OpenMP takes; then one
    FP call of the same solve on one thread (a bounded sample, scaled to a whole solve)."""
    import oracle
    op = oracle.OracleProblem(prob)
    threads = oracle.num_threads()
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.solve(op, "rre", L=prob.L, m=0, tol=0.0, max_calls=calls)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or n >= 50:
            break
    npx = prob.x_true.size
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    op.fp(op.x0())
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(threads)
    return {"value": npx * n / dt / 1e6, "unit": "MPix/s", "cores": threads,
            "kind": "oracle",
            # pixels x FP calls per second, the batched workload's unit of work (the oracle's
            # cost per pixel and FP call does not depend on the image's size)
            "mpix_fp_calls_per_s": npx * n * calls / dt / 1e6,
            "sample": f"{n} whole RRE solves ({calls} FP calls each, FP64) of the same 256x256 "
                      f"image, {dt:.1f} s",
            "one_core": {"value": npx / (dt1 * calls) / 1e6, "unit": "MPix/s", "cores": 1,
                         "sample": f"one FP call on one thread, {dt1:.1f} s, scaled to a "
                                   f"{calls}-call solve"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


if __name__ == "__main__":
    main()
