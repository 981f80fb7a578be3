"""Batched and serving forms through the C ABI (redve_solve_batch, redve_server_*).

* each image of a batch matches the single-image solve (same FP-call schedule, different
  grouping of the FP64 partial sums) and the FP64 oracle, within max(1e-4, 3x the movement of
  the oracle's result under FP32 rounding of its state);
* an image's batched result is bitwise independent of the other images of the batch;
* the server returns, for every request, bitwise the result of serving it alone, whatever
  arrives meanwhile; admission respects the device-memory budget.
"""
import math
import time

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def say(*a):
    print(*a, flush=True)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host(t):
    return t.detach().cpu().double().numpy()


def restorer(method="rre", L=5, tol=0.0, calls=10, precision="fp32"):
    from paper_1805_02158_amd import Restorer
    r = Restorer(0)
    r.set_denoiser(W.make_denoiser(), precision)
    r.set_extrapolation(method, L, 0)
    r.set_solver(15, calls, tol, 0)
    return r


def mixed_problems(orc, n=6, seed=0):
    """Uneven sizes, both blurs, deblurring and 3x SR, two noise levels (seeded per image)."""
    sizes = [(64, 96), (37, 53), (128, 128), (45, 160), (96, 33), (80, 80), (130, 97), (50, 50)]
    out = []
    for i in range(n):
        h, w = sizes[i % len(sizes)]
        sr = i % 3 == 2
        psf = W.psf_gaussian(7, 1.6) if (sr or i % 2) else W.psf_uniform(9)
        decim = 3 if sr else 1
        sigma = 5.0 if sr else (math.sqrt(2) if i % 2 == 0 else 5.0)
        x = W.make_image(h, w, 500 + 37 * seed + i)
        prob = W.Problem(f"m{i}", x, psf, decim, sigma, 0.02,
                         W.make_noise(W.lr_shape(h, w, decim), 600 + 37 * seed + i), 15, W.make_denoiser())
        y32 = f32(orc.OracleProblem(prob).y)
        out.append((prob, y32))
    return out


class _RoundedState:
    """The oracle's FP map with its state rounded to FP32 (what a FP32 solver keeps)."""

    def __init__(self, op):
        self.op, self.shape = op, op.shape

    def x0(self):
        return f32(self.op.x0())

    def fp(self, x):
        return f32(self.op.fp(x))


def _bound(orc, op, ref, method, L, calls):
    """max(1e-4, 3 x the movement of the oracle's fixed-schedule result when only its state is
    rounded to FP32): the part of a FP32 solve's error that no summation order avoids."""
    if method == "none":
        return 1e-4
    moved = orc.solve(_RoundedState(op), method, L=L, m=0, tol=0.0, max_calls=calls)
    return max(1e-4, 3.0 * rel(moved.x, ref.x))


def as_dicts(torch, probs):
    return [dict(y=dev(torch, y), hx=p.hr_shape[0], wx=p.hr_shape[1], psf=p.psf, decim=p.decim,
                 sigma=p.sigma, lam=p.lam) for p, y in probs]


def single(torch, r, prob, y32):
    r.set_operator(prob.psf, prob.decim).set_noise(prob.sigma).set_lambda(prob.lam)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    return host(x), st


@pytest.mark.parametrize("method", ["rre", "mpe", "none"])
def test_batch_matches_single_and_oracle(torch, orc, method):
    say("batch vs single", method)
    probs = mixed_problems(orc, 6)
    r = restorer(method, 5, 0.0, 10)
    outs, stats = r.solve_batch(as_dicts(torch, probs))
    for (prob, y32), xo, st in zip(probs, outs, stats):
        xs, sst = single(torch, r, prob, y32)
        xb = host(xo)
        assert st["fp_calls"] == sst["fp_calls"] == 10 and st["cycles"] == sst["cycles"]
        e1 = rel(xb, xs)
        op = orc.OracleProblem(prob, y=y32)
        ref = orc.solve(op, method, L=5, m=0, tol=0.0, max_calls=10)
        e2 = rel(xb, ref.x)
        bound = _bound(orc, op, ref, method, 5, 10)
        say(f"  {prob.name} {prob.hr_shape} decim {prob.decim}: vs single {e1:.2e}, "
            f"vs oracle {e2:.2e} (bound {bound:.1e})")
        # the single-image and batched solves differ only in how FP64 partial sums are grouped
        assert e1 <= bound / 3
        assert e2 <= bound


def test_batch_result_independent_of_the_batch(torch, orc):
    say("batch independence")
    probs = mixed_problems(orc, 6)
    r = restorer("rre", 5, 0.0, 10)
    alone, _ = r.solve_batch(as_dicts(torch, probs[2:3]))
    mixed, _ = r.solve_batch(as_dicts(torch, probs))
    rev, _ = r.solve_batch(as_dicts(torch, probs[::-1]))
    assert torch.equal(alone[0], mixed[2])
    assert torch.equal(alone[0], rev[3])


def deblur_problems(orc, seed=0):
    """Deblurring only (every image on the 32x32 CG form): images smaller than one 32x32 tile
    and than its 12-pixel halo, ragged tiles, and images with interior tiles; both blurs."""
    sizes = [(2, 3), (8, 8), (37, 53), (96, 33), (130, 97), (300, 260)]
    out = []
    for i, (h, w) in enumerate(sizes):
        psf = W.psf_gaussian(7, 1.6) if i % 2 else W.psf_uniform(9)
        sigma = math.sqrt(2) if i % 2 == 0 else 5.0
        prob = W.Problem(f"d{i}", W.make_image(h, w, 700 + 31 * seed + i), psf, 1, sigma, 0.02,
                         W.make_noise((h, w), 800 + 31 * seed + i), 15, W.make_denoiser())
        out.append((prob, f32(orc.OracleProblem(prob).y)))
    return out


def test_batch_cg32_fp_call(torch, orc):
    """One batched FP call (FP32 banks) of deblurring images, whose CG iterations run on the
    32x32 tile list, against the oracle's FP map."""
    probs = deblur_problems(orc)
    r = restorer("none", 5, 0.0, 1)
    outs, stats = r.solve_batch(as_dicts(torch, probs))
    for (prob, y32), xo, st in zip(probs, outs, stats):
        op = orc.OracleProblem(prob, y=y32)
        x0 = f32(op.x0())
        xr = op.fp(x0)
        xb = host(xo)
        e, es = rel(xb, xr), rel(xb - x0, xr - x0)
        say(f"  {prob.name} {prob.hr_shape}: rel L2 {e:.2e}, relative to the step {es:.2e}")
        assert st["fp_calls"] == 1
        assert e <= 2e-6 and es <= 2e-5


def test_batch_cg32_solve_and_independence(torch, orc):
    """Fixed-schedule RRE solves of the deblurring batch against the oracle, and each image's
    result bitwise the same alone and beside images on the 16x16 form (3x SR)."""
    probs = deblur_problems(orc, seed=1)
    r = restorer("rre", 5, 0.0, 10)
    outs, stats = r.solve_batch(as_dicts(torch, probs))
    for (prob, y32), xo, st in zip(probs, outs, stats):
        op = orc.OracleProblem(prob, y=y32)
        ref = orc.solve(op, "rre", L=5, m=0, tol=0.0, max_calls=10)
        e, bound = rel(host(xo), ref.x), _bound(orc, op, ref, "rre", 5, 10)
        say(f"  {prob.name} {prob.hr_shape}: rel L2 vs oracle {e:.2e} (bound {bound:.1e})")
        assert st["fp_calls"] == ref.calls and st["cycles"] == ref.cycles
        assert e <= bound
    sr = [pq for pq in mixed_problems(orc, 6) if pq[0].decim > 1]
    mix = [probs[4]] + sr + [probs[5]]
    alone4, _ = r.solve_batch(as_dicts(torch, probs[4:5]))
    alone5, _ = r.solve_batch(as_dicts(torch, probs[5:6]))
    mixed, _ = r.solve_batch(as_dicts(torch, mix))
    assert torch.equal(alone4[0], outs[4]) and torch.equal(alone4[0], mixed[0])
    assert torch.equal(alone5[0], outs[5]) and torch.equal(alone5[0], mixed[-1])


def test_batch_engine_reuse(torch, orc):
    """The handle keeps the batched engine between calls: a repeated batch is bitwise the
    same; after a settings change (CG count, extrapolation method) the result is bitwise that
    of a fresh handle with the new settings; switching back restores the first result."""
    say("batch reuse")
    probs = mixed_problems(orc, 5, seed=4)
    r = restorer("rre", 5, 0.0, 10)
    a, _ = r.solve_batch(as_dicts(torch, probs))
    b, _ = r.solve_batch(as_dicts(torch, probs))
    r.set_solver(10, 10, 0.0, 0)
    c, _ = r.solve_batch(as_dicts(torch, probs))
    fc = restorer("rre", 5, 0.0, 10).set_solver(10, 10, 0.0, 0).solve_batch(as_dicts(torch, probs))[0]
    r.set_solver(15, 10, 0.0, 0).set_extrapolation("mpe", 5, 0)
    e, _ = r.solve_batch(as_dicts(torch, probs))
    fe = restorer("mpe", 5, 0.0, 10).solve_batch(as_dicts(torch, probs))[0]
    r.set_extrapolation("rre", 5, 0)
    d, _ = r.solve_batch(as_dicts(torch, probs))
    fresh, _ = restorer("rre", 5, 0.0, 10).solve_batch(as_dicts(torch, probs))
    for i in range(len(probs)):
        say(f"  image {i}: cg 10 vs 15 max|diff| {float((c[i] - a[i]).abs().max()):.3e}, "
            f"mpe vs rre {float((e[i] - a[i]).abs().max()):.3e}")
        assert torch.equal(a[i], b[i]) and torch.equal(a[i], d[i]) and torch.equal(a[i], fresh[i])
        assert torch.equal(c[i], fc[i]) and torch.equal(e[i], fe[i])
        assert not torch.equal(a[i], e[i])


def test_single_cg_count_matters(torch, orc):
    """Diagnostic companion of the reuse test: the single-image path with 10 and 15 CG
    iterations per FP call, fixed schedule of 10 calls (differences printed)."""
    prob, y32 = mixed_problems(orc, 1, seed=4)[0]
    out = []
    for cg in (10, 15):
        r = restorer("rre", 5, 0.0, 10).set_solver(cg, 10, 0.0, 0)
        xs, st = single(torch, r, prob, y32)
        out.append(xs)
    say(f"  single path: cg 10 vs 15 rel diff {rel(out[0], out[1]):.3e}")
    one = []
    for cg in (10, 15):
        r = restorer("none", 5, 0.0, 1).set_solver(cg, 1, 0.0, 0)
        xs, st = single(torch, r, prob, y32)
        one.append(xs)
    d1 = rel(one[0], one[1])
    say(f"  one FP call: cg 10 vs 15 rel diff {d1:.3e}")
    assert d1 > 0


def test_batch_converged_and_m(torch, orc):
    """Tolerance-driven RRE with m = 1: every image reaches the oracle's fixed point."""
    say("batch converged")
    probs = mixed_problems(orc, 4, seed=1)
    from paper_1805_02158_amd import Restorer
    r = Restorer(0)
    r.set_denoiser(W.make_denoiser())
    r.set_extrapolation("rre", 4, 1)
    r.set_solver(15, 300, 1e-5, 0)
    outs, stats = r.solve_batch(as_dicts(torch, probs))
    for (prob, y32), xo, st in zip(probs, outs, stats):
        ref = orc.solve(orc.OracleProblem(prob, y=y32), "rre", L=4, m=1, tol=1e-9, max_calls=400)
        e = rel(host(xo), ref.x)
        say(f"  {prob.name}: {st['fp_calls']} calls, rel vs fixed point {e:.2e}")
        assert st["status"] == 0 and st["final_delta"] < 1e-5
        assert e <= 1e-4


def test_batch_64_images(torch, orc):
    """The batched workload: 64 images with sides log-uniform in [128, 1024], uniform 9x9 or
    Gaussian 7x7 blur, sigma sqrt(2) or 5, RRE L = 5, BF16 filter banks, to tolerance 1e-5.
    Every image converges; a sample matches its single-image solve and, for the smallest
    images, the oracle's fixed point within the BF16 bar."""
    say("batch 64")
    items = W.batch_items(64)
    probs = [(p, f32(orc.OracleProblem(p).y)) for p in items]
    ys = [dev(torch, y) for _, y in probs]
    r = restorer("rre", 5, 1e-5, 300, precision="bf16")
    dicts = [dict(y=y, hx=p.hr_shape[0], wx=p.hr_shape[1], psf=p.psf, decim=p.decim,
                  sigma=p.sigma, lam=p.lam) for (p, _), y in zip(probs, ys)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, stats = r.solve_batch(dicts)
    dt = time.perf_counter() - t0
    mpix = sum(p.x_true.size for p, _ in probs) / 1e6
    say(f"  {mpix:.1f} MPix in {dt * 1e3:.0f} ms, calls {min(s['fp_calls'] for s in stats)}.."
        f"{max(s['fp_calls'] for s in stats)}")
    assert all(s["status"] == 0 and s["final_delta"] < 1e-5 for s in stats)
    for i in (0, 7, 31, 63):
        p = probs[i][0]
        r.set_operator(p.psf, p.decim).set_noise(p.sigma).set_lambda(p.lam)
        xs, _ = r.solve(ys[i], *p.hr_shape)
        e = rel(host(outs[i]), host(xs))
        say(f"  image {i} {p.hr_shape}: vs single {e:.2e}")
        assert e <= 1e-4
    small = sorted(range(64), key=lambda i: probs[i][0].x_true.size)[:2]
    for i in small:
        p, y32 = probs[i]
        ref = orc.solve(orc.OracleProblem(p, y=y32), "rre", L=5, m=0, tol=1e-9, max_calls=400)
        e = rel(host(outs[i]), ref.x)
        dp = orc.psnr(host(outs[i]), p.x_true) - orc.psnr(ref.x, p.x_true)
        say(f"  image {i} {p.hr_shape}: vs oracle fixed point {e:.2e}, dPSNR {dp:+.4f}")
        assert e <= 5e-3 and abs(dp) <= 0.05


# ------------------------------------------------------------------ serving


def _serve(torch, r, reqs, budget, max_active, stagger=0.0):
    from paper_1805_02158_amd import Server
    srv = Server(r, budget, max_active)
    tickets = []
    for d in reqs:
        tickets.append(srv.submit(**d))
        if stagger:
            time.sleep(stagger)
    stats = [srv.wait(t) for t, _ in tickets]
    counts = srv.counts()
    counts.update(srv.occupancy())
    srv.close()
    return [o for _, o in tickets], stats, counts


def test_server_same_alone_and_in_mix(torch, orc):
    """Continuous batching: requests arrive while others run (staggered submits); each result
    is bitwise the result of serving that request alone."""
    say("server mix")
    probs = mixed_problems(orc, 8, seed=2)
    r = restorer("rre", 5, 1e-5, 200)
    reqs = as_dicts(torch, probs)
    outs, stats, counts = _serve(torch, r, reqs, 256 << 20, 4, stagger=0.002)
    say(f"  counts {counts}")
    assert counts["finished"] == 8 and counts["queued"] == 0
    for i in (0, 3, 5):
        alone, st_alone, _ = _serve(torch, r, [as_dicts(torch, probs[i:i + 1])[0]], 256 << 20, 4)
        assert torch.equal(alone[0], outs[i]), i
        assert st_alone[0]["fp_calls"] == stats[i]["fp_calls"]
    for (prob, y32), xo, st in zip(probs, outs, stats):
        assert st["status"] == 0 and st["final_delta"] < 1e-5 and st["ms"] > 0
    # and the batched solver agrees
    outs_b, _ = r.solve_batch(reqs)
    for a, b in zip(outs, outs_b):
        assert torch.equal(a, b)


def test_server_admission_respects_budget(torch, orc):
    """A budget that holds about two of the images: requests queue and are admitted in order
    as memory frees up (rounds run with a request waiting), the pixels admitted at once never
    exceed what the budget buys, and all finish with the oracle's result."""
    say("server budget")
    probs = mixed_problems(orc, 6, seed=3)
    r = restorer("rre", 5, 1e-5, 200)
    per_px = 4 * (14 + 5)
    budget = per_px * (2 * 128 * 128 + 4096)
    outs, stats, counts = _serve(torch, r, as_dicts(torch, probs), budget, 8)
    say(f"  counts {counts}, sizes {[p.hr_shape for p, _ in probs]}")
    assert counts["finished"] == 6
    assert counts["capacity_px"] == budget // per_px
    assert 0 < counts["peak_px"] <= counts["capacity_px"]
    assert counts["waited_rounds"] >= 1
    assert counts["peak_px"] < sum(-(-p.hr_shape[0] * p.hr_shape[1] // 64) * 64 for p, _ in probs)
    for (prob, y32), xo in zip(probs, outs):
        ref = orc.solve(orc.OracleProblem(prob, y=y32), "rre", L=5, m=0, tol=1e-9, max_calls=400)
        assert rel(host(xo), ref.x) <= 1e-4
