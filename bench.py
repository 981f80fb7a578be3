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
    ap.add_argument("--serve-requests", type=int, default=160)
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


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the restoration of one image runs on one device and "
              "this build has no multi-GPU path (--gpus 1 only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workload as W
    from paper_1805_02158_amd import Restorer

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

    state = {"prec": "fp32"}  # configure() above loaded the FP32 banks

    def solve(method, prec, calls):
        if state["prec"] != prec:
            R.set_denoiser(prob.denoiser, prec)
            state["prec"] = prec
        R.set_extrapolation(method, prob.L, 0)
        R.set_solver(prob.cg_iters, calls, 0.0, 0)
        _, st = R.solve(y, H, Wd, out=out)
        return st

    def n_star(method, prec):
        trace = []
        for n in range(1, args.nmax + 1):
            solve(method, prec, n)
            trace.append((n, psnr(out)))
        ns = None
        for n, p in trace:
            if abs(p - psnr_star) <= BAND_DB:
                ns = n if ns is None else ns
            else:
                ns = None
        return ns, trace

    def timed(method, prec, calls):
        for _ in range(args.warmup):
            solve(method, prec, calls)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            st = solve(method, prec, calls)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        return {"mpix_s": npx * args.steps / total / 1e6, "ms_per_step": total / args.steps * 1e3,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "fp_calls_to_target": calls, "cycles": st["cycles"], "psnr_db": psnr(out)}

    forms = {"plain_fp32": ("none", "fp32"), "ve_fp32": ("rre", "fp32"), "ve_bf16": ("rre", "bf16")}
    res_forms = {}
    for name, (method, prec) in forms.items():
        ns, tr = n_star(method, prec)
        if ns is None:
            print(json.dumps({"error": f"target PSNR not reached by {name}", "trace": tr}))
            sys.exit(1)
        res_forms[name] = timed(method, prec, ns)
        res_forms[name]["roofline_whole_solve"] = whole_solve_roofline(
            npx * ns / (res_forms[name]["ms_per_step"] * 1e-3), prob.cg_iters)
        log(name, res_forms[name])
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
    roof_stage = roofline_stage(npx, stage_us, "k_tnrd_stage_bf16")
    roof_cg = roofline_cg(npx, blk_us, "k_cg_block<4>", 2)
    share = {"k_tnrd_stage_bf16": prob.denoiser.stages * stage_us,
             "k_cg_block<4>": (prob.cg_iters // 2) * blk_us}
    roof = roof_cg if share["k_cg_block<4>"] >= share["k_tnrd_stage_bf16"] else roof_stage
    roof["share_of_fp_call_us"] = share
    big = torch.tensor(W.make_image(2048, 2048, 77), dtype=torch.float32, device=dev)
    stage_big_us = time_stage(torch, R, big, prob.denoiser.stages)
    roof_big = roofline_stage(big.numel(), stage_big_us, "k_tnrd_stage_bf16")
    cg_big_us = time_cg_iter(torch, R, big)
    roof_cg_big = roofline_cg(big.numel(), cg_big_us, "k_cg_iter<4>", 1)
    R.set_denoiser(prob.denoiser, "fp32")
    stage32_big_us = time_stage(torch, R, big, prob.denoiser.stages)
    roof32_big = roofline_stage(big.numel(), stage32_big_us, "k_tnrd_stage_f32")
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
                               "k_cg_iter<4>": roof_cg_big},
    }
    if not args.no_sd:
        res["steepest_descent"] = bench_sd(args, torch, np, R, prob, y, out, psnr, psnr_star)
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
    call there with FP32 banks."""
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
    torch.cuda.synchronize()


# Algorithmic work of one denoiser stage per output pixel: two 24-filter 5x5 banks (forward
# and adjoint, 2 x 24 x 25 multiply-adds = 2400 FLOP) and 24 influence functions, each the
# Gaussian RBF sum over the 15 centres within 7.5 gamma of z (the terms beyond add less than
# 1e-12 of a weight, so this is the sum as defined to FP32 precision; all 63 would be 4.2x
# more), each term counted as 6 FLOP (difference, square, scale, exp, multiply-add) = 2160 FLOP.
# The BF16 stage on small images reads phi from a table instead, which does less than this.
STAGE_FLOP_PER_PX = 2 * 24 * 25 * 2 + 24 * 15 * 6
# Published MI355X FP32 vector peak (256 CUs, 2.4 GHz).
FP32_PEAK_TFLOPS = 157.3


def roofline_stage(npx, stage_us, kernel):
    """The fused denoiser stage is bound by plain ALU arithmetic: its data stays in LDS and
    registers (HBM traffic about 12 B per pixel) and the influence functions and the banks'
    operand staging run on the vector ALUs in either precision. achieved = algorithmic FLOP
    per launch / average launch time, against the FP32 vector peak."""
    work = npx * STAGE_FLOP_PER_PX
    achieved = work / (stage_us * 1e-6) / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic_of(kernel, npx), "avg_launch_us": stage_us,
            "flop_per_launch": work,
            "flop_per_px": STAGE_FLOP_PER_PX, "pixels_per_launch": npx}


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
# own roofline, summed (the classes run one after another): the denoiser's 5 stages (state
# traffic 5 x 12 B; 5 x STAGE_FLOP_PER_PX at the FP32 vector peak, which bounds them), the CG
# step (n_cg x 24 B: x, r, p read and written once per iteration) and the extrapolation's
# difference and combination passes (16.8 B per FP call for L = 5: u written, the Gram reads
# and the combination spread over a cycle of 5 calls).
def roofline_ps_per_px_call(n_cg=15):
    stages = max(5 * 12 / HBM_PEAK_GBS * 1e3, 5 * STAGE_FLOP_PER_PX / FP32_PEAK_TFLOPS)
    cg = n_cg * CG_BYTES_PER_PX / HBM_PEAK_GBS * 1e3
    ve = 16.8 / HBM_PEAK_GBS * 1e3
    return {"stages_ps": stages, "cg_ps": cg, "ve_ps": ve, "total_ps": stages + cg + ve}


def whole_solve_roofline(px_calls_per_s, n_cg=15):
    """Fraction of the whole-solve roofline: declared time per pixel per FP call over the measured
    one (pixel-FP-calls per second)."""
    r = roofline_ps_per_px_call(n_cg)
    measured = 1e12 / px_calls_per_s
    return {"declared_ps_per_px_fp_call": r, "measured_ps_per_px_fp_call": measured,
            "frac": r["total_ps"] / measured}


def bench_batch(args, torch, np, W, Restorer, psnr):
    probs = W.batch_items(args.batch_images)
    R = Restorer(0)
    ys = observe(torch, R, probs)
    xts = [torch.tensor(p.x_true, dtype=torch.float32, device="cuda") for p in probs]
    items = [dict(y=y, hx=p.hr_shape[0], wx=p.hr_shape[1], psf=p.psf, decim=p.decim,
                  sigma=p.sigma, lam=p.lam) for p, y in zip(probs, ys)]
    mpix = sum(p.x_true.size for p in probs) / 1e6
    d = W.make_denoiser()

    def run(method, prec, tol, max_calls):
        R.set_denoiser(d, prec).set_extrapolation(method, 5, 0).set_solver(15, max_calls, tol, 0)
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
    for name, method, prec, reps in (("ve_bf16", "rre", "bf16", 3), ("ve_fp32", "rre", "fp32", 1),
                                     ("plain_fp32", "none", "fp32", 1)):
        run(method, prec, 1e-5, 500)  # warm-up: workspace and graphs
        times = []
        for _ in range(reps):
            dt, outs, st = run(method, prec, 1e-5, 500)
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
            out[name]["mpix_fp_calls_per_s"] * 1e6)
        log("batched", name, out[name])
    out["ve_bf16_speedup_vs_plain_fp32"] = out["plain_fp32"]["s_per_batch"] / out["ve_bf16"]["s_per_batch"]
    R.close()
    return out


def bench_serve(args, torch, np, W, Restorer):
    from paper_1805_02158_amd import Server
    trace = W.serve_trace(args.serve_requests, 1.0)
    probs = [p for _, p in trace]
    R = Restorer(0)
    ys = observe(torch, R, probs)
    reqs = [dict(y=y, hx=p.hr_shape[0], wx=p.hr_shape[1], psf=p.psf, decim=p.decim,
                 sigma=p.sigma, lam=p.lam) for p, y in zip(probs, ys)]
    mpix = sum(p.x_true.size for p in probs) / 1e6
    R.set_denoiser(W.make_denoiser(), "bf16").set_extrapolation("rre", 5, 0).set_solver(15, 500, 1e-5, 0)
    budget = int(args.serve_budget_gb * (1 << 30))

    srv = Server(R, budget, args.serve_max_active)

    def serve(arrivals):
        rounds0 = srv.counts()["rounds"]
        t0 = time.perf_counter()
        tickets = []
        for a, d in zip(arrivals, reqs):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            tickets.append(srv.submit(**d)[0])
        st = [srv.wait(t) for t in tickets]
        makespan = time.perf_counter() - t0
        lat = np.array([s["ms"] for s in st])
        bad = sum(s["status"] != 0 for s in st)
        return makespan, lat, srv.counts()["rounds"] - rounds0, bad

    serve([0.0] * 16)  # warm-up: the graphs of the first tile-list lengths
    mk, lat_sat, rounds_sat, bad = serve([0.0] * len(reqs))
    rate_sat = len(reqs) / mk
    rate = 0.7 * rate_sat
    arrivals = [a / rate for a, _ in trace]  # the trace's arrivals (drawn at rate 1) at `rate`
    mk2, lat, rounds2, bad2 = serve(arrivals)
    srv.close()
    res = {"workload": f"{len(reqs)} requests, sides log-uniform 128..2048 ({mpix:.1f} MPix), "
                       "deblur 9x9 uniform or 3x SR Gaussian 7x7, sigma sqrt(2) or 5, RRE L=5, "
                       "BF16 banks, stop at relative change < 1e-5",
           "hbm_budget_gb": args.serve_budget_gb, "max_active": args.serve_max_active,
           "saturation": {"req_s": rate_sat, "mpix_s": mpix / mk, "rounds": rounds_sat,
                          "p50_ms": float(np.percentile(lat_sat, 50)),
                          "p99_ms": float(np.percentile(lat_sat, 99)), "failed": bad},
           "poisson": {"rate_req_s": rate, "mpix_s": mpix / mk2, "rounds": rounds2,
                       "p50_ms": float(np.percentile(lat, 50)),
                       "p99_ms": float(np.percentile(lat, 99)), "failed": bad2}}
    log("serving", res)
    R.close()
    return res


def cpu_baseline(prob, calls, min_seconds):
    """The FP64 oracle (plain C, OpenMP over rows/filters) on the host: whole RRE solves
    (L = 5, the GPU's FP-call count to the target) of the same image, repeated until at least
    `min_seconds` have passed (at most 50 solves)."""
    import oracle
    op = oracle.OracleProblem(prob)
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.solve(op, "rre", L=prob.L, m=0, tol=0.0, max_calls=calls)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or n >= 50:
            break
    npx = prob.x_true.size
    return {"value": npx * n / dt / 1e6, "unit": "MPix/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} whole RRE solves ({calls} FP calls each, FP64) of the same 256x256 "
                      f"image, {dt:.1f} s"}


if __name__ == "__main__":
    main()
