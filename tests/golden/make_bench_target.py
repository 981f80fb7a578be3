"""Writes bench_target_<workload>.json: the oracle-converged PSNR of a benchmark workload
(deblur256: the 256x256 deblurring; sr512: the 512x512 3x super-resolution).

Calls only the FP64 oracle and the seeded workload generator. The target is the PSNR of plain
FP (eq. (7)) run until the relative change of consecutive iterates is below 1e-6 (cap 1000 FP
calls). For context it also records, for the oracle itself, the FP-call count after which
every returned vector stays within 0.05 dB of that PSNR (plain FP, RRE and MPE with the
workload's window).

Run: python tests/golden/make_bench_target.py [deblur256|sr512]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload as W  # noqa: E402

BAND_DB = 0.05


def stable_from(trace, target, band=BAND_DB):
    """Smallest FP-call count from which every returnable vector is within `band` dB."""
    n_star = None
    for calls, p in trace:
        if abs(p - target) <= band:
            if n_star is None:
                n_star = calls
        else:
            n_star = None
    return n_star


DESCRIPTIONS = {
    "deblur256": "deblur256: 256x256 synthetic image, uniform 9x9 blur, sigma sqrt(2), lambda 0.02, "
                 "15 CG iterations, seeded TNRD-style denoiser (5 stages x 24 filters)",
    "sr512": "sr512: 512x512 synthetic image, Gaussian 7x7 blur (std 1.6) and 3x decimation, "
             "sigma 5, lambda 0.02, 15 CG iterations, seeded TNRD-style denoiser (5 stages x 24 "
             "filters)",
}


def main(name="deblur256"):
    prob = W.problem(name)
    op = oracle.OracleProblem(prob)
    t0 = time.time()
    ref = oracle.solve(op, "none", tol=1e-6, max_calls=1000)
    psnr_star = oracle.psnr(ref.x, prob.x_true)
    out = {
        "workload": DESCRIPTIONS[name],
        "psnr_star_db": psnr_star,
        "psnr_input_db": oracle.psnr(op.x0(), prob.x_true),
        "oracle_fp_calls_to_1e-6": ref.calls,
        "band_db": BAND_DB,
        "oracle_threads": oracle.num_threads(),
    }
    for method in ("none", "rre", "mpe"):
        tr = []
        oracle.solve(op, method, L=prob.L, m=0, tol=1e-6, max_calls=300,
                     on_vector=lambda c, v: tr.append((c, oracle.psnr(v, prob.x_true))))
        out[f"oracle_n_star_{method}"] = stable_from(tr, psnr_star)
    out["seconds"] = round(time.time() - t0, 1)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"bench_target_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "deblur256")
