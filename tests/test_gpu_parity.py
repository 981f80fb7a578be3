"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element by element.

Inputs are seeded and synthetic; the GPU receives the FP32 rounding of the oracle's inputs and
the oracle recomputes on those same FP32 values in FP64. Tolerances (relative L2):
  single operators (blur, adjoint, A)  2e-6   FP32 sums of <= 225 products
  CG, denoiser, one FP call            2e-5   FP32 recurrences over 15 iterations / 5 stages
  solves                               1e-4   the FP32 bar for results
Extrapolated vectors can be ill-conditioned functions of the iterates (sum |gamma| reaches 1e4
in early super-resolution cycles): rounding the FP64 oracle's own iterates to FP32 after every
FP call then moves its result by more than 1e-4. For a solve stopped at a fixed FP-call count
the bound is max(1e-4, 3 x that movement), which the test measures with the oracle; converged
results are held to 1e-4.
"""
import math

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


def dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host(t):
    return t.detach().cpu().double().numpy()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def restorer(prob=None, **kw):
    from paper_1805_02158_amd import Restorer
    r = Restorer(0)
    if prob is not None:
        r.configure(prob, **kw)
    return r


def say(*a):
    print(*a, flush=True)


PSFS = {"u9": W.psf_uniform(9), "g7": W.psf_gaussian(7, 1.6),
        "asym": np.random.default_rng(5).standard_normal((5, 3))}
SHAPES = [(64, 64), (37, 53), (5, 7), (2, 2), (16, 33), (256, 256), (300, 130)]


# ------------------------------------------------------------------ operators


def _within_fp32_sum(got, ref, absref, nterms):
    """Elementwise: |got - ref| <= (n + 2) 2^-24 |.|-weighted sum, the bound on a sum of n FP32
    products (and the final rounding) against the exact sum; absref is the same operator
    applied to |inputs|, so cancellation in ref does not shrink the bar."""
    bound = (nterms + 2) * 2.0 ** -24 * absref + 1e-30
    err = np.abs(got.astype(np.float64) - ref)
    return float((err / bound).max())


@pytest.mark.parametrize("psf", list(PSFS))
@pytest.mark.parametrize("decim", [1, 3])
@pytest.mark.parametrize("shape", SHAPES)
def test_operators(torch, orc, psf, decim, shape):
    """H, H^T and A against the oracle, elementwise within the FP32 rounding bound of their
    sums (the kernels sum in FP32, the oracle in FP64), and to 2e-6 relative L2 where the
    output has many elements. Inputs are seeded from the case's name."""
    import zlib
    say("operators", psf, decim, shape)
    k = PSFS[psf]
    r = restorer()
    r.set_operator(k, decim).set_noise(5.0 if decim > 1 else math.sqrt(2)).set_lambda(0.02)
    rng = np.random.default_rng(zlib.crc32(repr((psf, decim, shape)).encode()))
    x = f32(rng.uniform(0, 255, shape))
    ky = f32(k)
    ka = np.abs(ky)
    nt = ky.size
    sig = 5.0 if decim > 1 else math.sqrt(2)
    y = host(r.apply_H(dev(torch, x)))
    yo = orc.apply_H(x, ky, decim)
    assert _within_fp32_sum(y, yo, orc.apply_H(x, ka, decim), nt) <= 1.0
    z = f32(rng.standard_normal(orc.lr_shape(*shape, decim)) * 50)
    ht = host(r.apply_Ht(dev(torch, z), *shape))
    hto = orc.apply_Ht(z, shape, ky, decim)
    assert _within_fp32_sum(ht, hto, orc.apply_Ht(np.abs(z), shape, ka, decim), nt) <= 1.0
    a = host(r.apply_A(dev(torch, x)))
    ao = orc.apply_A(x, ky, decim, sig, 0.02)
    # A = H^T H / sigma^2 + lambda I: two nested sums of nt products each
    assert _within_fp32_sum(a, ao, orc.apply_A(x, ka, decim, sig, 0.02), 2 * nt + 2) <= 1.0
    if y.size >= 64:
        assert rel(y, yo) <= 2e-6 and rel(ht, hto) <= 2e-6 and rel(a, ao) <= 2e-6


@pytest.mark.parametrize("shape,psf,decim", [((64, 64), "u9", 1), ((37, 53), "g7", 3),
                                             ((256, 256), "u9", 1), ((8, 8), "g7", 1),
                                             ((37, 53), "g7", 1)])
def test_cg(torch, orc, shape, psf, decim):
    """CG on A x = rhs against the oracle's CG. Undecimated 7x7 and 9x9 cases run two
    iterations per kernel for all but the last (and an odd) iteration: the counts cover no
    block (1, 2), one block (3, 4), several with and without a single iteration left over."""
    say("cg", shape, psf, decim)
    k = PSFS[psf]
    sig = 5.0 if decim > 1 else math.sqrt(2)
    r = restorer()
    r.set_operator(k, decim).set_noise(sig).set_lambda(0.02)
    rng = np.random.default_rng(7)
    x0 = f32(rng.uniform(0, 255, shape))
    rhs = f32(orc.apply_A(rng.uniform(0, 255, shape), k, decim, sig, 0.02))
    for iters in (0, 1, 2, 3, 4, 10, 15):
        xg = host(r.cg(dev(torch, rhs), dev(torch, x0), iters))
        xo = orc.cg(rhs, x0, f32(k), decim, sig, 0.02, iters)
        assert rel(xg, xo) <= 2e-5, iters


# ------------------------------------------------------------------ denoiser


@pytest.mark.parametrize("shape", [(64, 64), (37, 53), (2, 2), (3, 5), (17, 16), (256, 256),
                                   (400, 330)])
def test_denoiser(torch, orc, shape):
    """The FP32 form (FP32 operands on MFMA): the denoiser output and its update against the
    oracle. Images of fewer and of more than 512 tiles take the 1024- and 512-thread tiles."""
    say("denoiser", shape)
    d = W.make_denoiser()
    r = restorer()
    r.set_denoiser(d)
    x = f32(W.make_image(*shape, 77) + 5 * W.make_noise(shape, 78))
    g = host(r.denoise(dev(torch, x)))
    o = orc.denoise(x, orc.Denoiser(d))
    say(f"  rel L2 {rel(g, o):.2e}, update rel L2 {rel(g - x, o - x):.2e}")
    assert rel(g, o) <= 2e-5
    assert rel(g - x, o - x) <= 2e-4
    assert np.abs(g - o).max() <= 2e-3


def test_denoiser_fp32_large_on_vector_alus(torch, orc):
    """A FP32 denoiser whose MFMA tile would not fit 64 KiB of LDS (32 filters of 127 centres)
    runs on the vector-ALU stage: the same bar."""
    d = W.make_denoiser(stages=2, nfilt=32, nrbf=127, mu0=-630.0)
    r = restorer()
    r.set_denoiser(d)
    for shape in ((37, 53), (64, 64)):
        x = f32(W.make_image(*shape, 79) + 5 * W.make_noise(shape, 80))
        g = host(r.denoise(dev(torch, x)))
        o = orc.denoise(x, orc.Denoiser(d))
        say(f"  {shape}: rel L2 {rel(g, o):.2e}")
        assert rel(g, o) <= 2e-5


def test_denoiser_constant_and_identity(torch, orc):
    say("denoiser constant")
    r = restorer()
    r.set_denoiser(W.make_denoiser())
    for c in (0.0, 37.5, 255.0):
        x = np.full((40, 24), c)
        assert np.abs(host(r.denoise(dev(torch, x))) - c).max() <= 1e-3 * max(c, 1)
    r.set_denoiser(W.identity_denoiser())
    x = np.random.default_rng(1).uniform(0, 255, (19, 23))
    assert np.array_equal(host(r.denoise(dev(torch, x))), f32(x))


# ------------------------------------------------------------------ one FP call


@pytest.mark.parametrize("name", ["tiny", "deblur64"])
def test_fp_step(torch, orc, name):
    say("fp_step", name)
    prob = W.problem(name)
    op = orc.OracleProblem(prob, y=f32(orc.OracleProblem(prob).y))
    r = restorer(prob)
    x = f32(op.y)
    for _ in range(3):
        xg = host(r.fp_step(dev(torch, op.y), dev(torch, x)))
        xo = op.fp(x)
        say(f"  rel L2 {rel(xg, xo):.2e}, relative to the step {rel(xg - x, xo - x):.2e}")
        assert rel(xg, xo) <= 2e-5
        assert rel(xg - x, xo - x) <= 1e-4
        x = f32(xo)


@pytest.mark.parametrize("shape", [(37, 53), (250, 490), (250, 510)])
def test_fp_step_uniform9_at_the_tile_boundary(torch, orc, shape):
    """One FP call of eq. (7) on a uniform 9x9 deblurring with 15 CG iterations (FP32 banks), on
    both sides of the 512-tile boundary: below it (37x53: 12 tiles, 250x490: 496) the last
    denoiser stage also forms the CG start and two CG iterations run per launch; at 250x510
    (512 tiles) the start has its own kernel and one iteration runs per launch. The bar of the
    FP32 form, two calls in a row."""
    say("fp_step u9", shape)
    prob = W.Problem(f"u9_{shape[0]}x{shape[1]}", W.make_image(*shape, 1003), W.psf_uniform(9), 1,
                     W.SQRT2, 0.02, W.make_noise(shape, 2003), 15, W.make_denoiser())
    op = orc.OracleProblem(prob, y=f32(orc.OracleProblem(prob).y))
    r = restorer(prob)
    x = f32(op.y)
    for _ in range(2):
        xg = host(r.fp_step(dev(torch, op.y), dev(torch, x)))
        xo = op.fp(x)
        say(f"  rel L2 {rel(xg, xo):.2e}, relative to the step {rel(xg - x, xo - x):.2e}")
        assert rel(xg, xo) <= 2e-5
        assert rel(xg - x, xo - x) <= 1e-4
        x = f32(xo)


# Denoisers beside the default one for the last stage forming the CG start: one stage (the last
# stage is also the first) and 32 filters (LDS row stride 33; with FP32 banks their MFMA tile
# exceeds 64 KiB, so that form runs the vector-ALU stage and the separate start kernel).
FUSED_DENOISERS = {"one stage": dict(stages=1), "32 filters": dict(stages=2, nfilt=32)}


def _fused_problem(psf, form, shape):
    return W.Problem(f"{psf}_{form}", W.make_image(*shape, 1004), PSFS[psf], 1, W.SQRT2, 0.02,
                     W.make_noise(shape, 2004), 15, W.make_denoiser(**FUSED_DENOISERS[form]),
                     "rre", 5, 0, 1e-5, 400)


@pytest.mark.parametrize("psf", ["u9", "g7"])
@pytest.mark.parametrize("form", list(FUSED_DENOISERS))
def test_fp_step_fused_start_forms(torch, orc, psf, form):
    """One FP call of eq. (7) with FP32 banks on a 37x53 deblurring, 9x9 and 7x7 PSFs (halo
    radius 4 and 3), against the oracle's, the FP32 bar, two calls in a row."""
    say("fp_step fused start", psf, form)
    prob = _fused_problem(psf, form, (37, 53))
    op = orc.OracleProblem(prob, y=f32(orc.OracleProblem(prob).y))
    r = restorer(prob)
    x = f32(op.y)
    for _ in range(2):
        xg = host(r.fp_step(dev(torch, op.y), dev(torch, x)))
        xo = op.fp(x)
        say(f"  rel L2 {rel(xg, xo):.2e}, relative to the step {rel(xg - x, xo - x):.2e}")
        assert rel(xg, xo) <= 2e-5
        assert rel(xg - x, xo - x) <= 1e-4
        x = f32(xo)


# ------------------------------------------------------------------ extrapolation


@pytest.mark.parametrize("method", ["mpe", "rre", "svd_mpe"])
@pytest.mark.parametrize("L", [2, 5, 8])
def test_extrapolate(torch, orc, method, L):
    say("extrapolate", method, L)
    prob = W.problem("tiny")
    op = orc.OracleProblem(prob)
    xs = [f32(op.y)]
    for _ in range(L):
        xs.append(f32(op.fp(xs[-1])))
    r = restorer(prob, method=method, L=L)
    xg, gam, bd = r.extrapolate(dev(torch, np.stack(xs)))
    xo, go, bo = orc.ve_step(xs, method)
    assert bd == bo
    assert rel(host(xg), xo.reshape(op.shape)) <= 2e-6
    if go is not None and len(go) == L:
        assert np.abs(gam - go).max() <= 1e-6 * max(1.0, np.abs(go).max())


def test_extrapolate_linear_exactness(torch, orc):
    """Sec. III-A through the GPU path: a linear iteration with 3 distinct eigenvalues is
    extrapolated to its fixed point from kappa + 2 = 5 iterates (L = 4)."""
    say("extrapolate linear")
    rng = np.random.default_rng(3)
    shape = (32, 32)
    N = shape[0] * shape[1]
    v = [rng.standard_normal(N) for _ in range(3)]
    lam = [0.8, -0.5, 0.3]
    xstar = rng.uniform(50, 200, N)
    coef = rng.standard_normal(3) * 5
    xs = [xstar + sum(coef[i] * lam[i] ** k * v[i] for i in range(3)) for k in range(5)]
    xs32 = [f32(x) for x in xs]
    for method in ("mpe", "rre", "svd_mpe"):
        r = restorer()
        r.set_extrapolation(method, 4, 0)
        xg, _, bd = r.extrapolate(dev(torch, np.stack([x.reshape(shape) for x in xs32])))
        assert not bd
        # L = 4 columns of differences span 3 modes: rank 3 -> exact up to FP32 input rounding
        assert rel(host(xg).ravel(), xstar) <= 1e-5, method


# ------------------------------------------------------------------ whole solves


def _oracle_solve(orc, prob, y32, method, L, m, tol, calls):
    op = orc.OracleProblem(prob, y=y32)
    return orc.solve(op, method, L=L, m=m, tol=tol, max_calls=calls), op


class _RoundedState:
    """The oracle's FP map with its output rounded to FP32 (the state a FP32 solver keeps)."""

    def __init__(self, op):
        self.op, self.shape = op, op.shape

    def x0(self):
        return f32(self.op.x0())

    def fp(self, x):
        return f32(self.op.fp(x))


def _bound(orc, op, ref, method, L, m, calls):
    """max(1e-4, 3 x the movement of the oracle's result under FP32 rounding of its state)."""
    if method == "none":
        return 1e-4
    moved = orc.solve(_RoundedState(op), method, L=L, m=m, tol=0.0, max_calls=calls)
    floor = rel(moved.x, ref.x)
    say(f"  FP32-state sensitivity of the oracle: {floor:.2e}")
    return max(1e-4, 3.0 * floor)


@pytest.mark.parametrize("name,method,L,calls", [("deblur64", "none", 5, 20), ("deblur64", "rre", 5, 20),
                                                 ("deblur64", "mpe", 5, 20), ("deblur64", "svd_mpe", 5, 20),
                                                 ("tiny", "rre", 3, 13), ("tiny", "mpe", 4, 7)])
def test_solve_fixed_schedule(torch, orc, name, method, L, calls):
    say("solve", name, method, L, calls)
    prob = W.problem(name)
    y32 = f32(orc.OracleProblem(prob).y)
    ref, op = _oracle_solve(orc, prob, y32, method, L, 0, 0.0, calls)
    r = restorer(prob, method=method, L=L, m=0, tol=0.0, max_fp_calls=calls)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    assert st["fp_calls"] == ref.calls and st["cycles"] == ref.cycles
    assert st["breakdowns"] == ref.breakdowns
    err = rel(host(x), ref.x)
    say(f"  rel L2 vs oracle: {err:.2e}")
    assert err <= _bound(orc, op, ref, method, L, 0, calls)


def test_solve_m_positive(torch, orc):
    say("solve m>0")
    prob = W.problem("tiny")
    y32 = f32(orc.OracleProblem(prob).y)
    ref, op = _oracle_solve(orc, prob, y32, "rre", 3, 2, 0.0, 16)
    r = restorer(prob, method="rre", L=3, m=2, tol=0.0, max_fp_calls=16)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    assert st["fp_calls"] == 16 and st["cycles"] == ref.cycles == 3
    err = rel(host(x), ref.x)
    say(f"  rel L2 vs oracle: {err:.2e}")
    assert err <= _bound(orc, op, ref, "rre", 3, 2, 16)


@pytest.mark.parametrize("method", ["rre", "mpe"])
def test_solve_deblur256_full_size(torch, orc, method):
    """The benchmark workload (256x256, uniform 9x9, L = 5) at its launch configuration, at a
    fixed schedule of two cycles."""
    say("solve deblur256", method)
    prob = W.problem("deblur256")
    y32 = f32(orc.OracleProblem(prob).y)
    ref, op = _oracle_solve(orc, prob, y32, method, 5, 0, 0.0, 10)
    r = restorer(prob, method=method, tol=0.0, max_fp_calls=10)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    assert st["cycles"] == 2
    err = rel(host(x), ref.x)
    say(f"  rel L2 vs oracle: {err:.2e}")
    assert err <= _bound(orc, op, ref, method, 5, 0, 10)


def test_solve_sr(torch, orc):
    """3x super-resolution (Gaussian 7x7 + decimation, sigma 5) with RRE, L = 8, on a 130x97
    image (LR 44x33), one cycle plus a partial one."""
    say("solve sr")
    x_true = W.make_image(130, 97, 1234)
    prob = W.Problem("sr", x_true, W.psf_gaussian(7, 1.6), 3, 5.0, 0.02,
                     W.make_noise(W.lr_shape(130, 97, 3), 4321), 15, W.make_denoiser(),
                     "rre", 8, 0, 0.0, 11)
    y32 = f32(orc.OracleProblem(prob).y)
    ref, op = _oracle_solve(orc, prob, y32, "rre", 8, 0, 0.0, 11)
    r = restorer(prob)
    x, st = r.solve(dev(torch, y32), 130, 97)
    assert st["fp_calls"] == 11 and st["cycles"] == 1
    err = rel(host(x), ref.x)
    say(f"  rel L2 vs oracle: {err:.2e}")
    assert err <= _bound(orc, op, ref, "rre", 8, 0, 11)


def test_solve_identity_denoiser(torch, orc):
    say("solve identity denoiser")
    prob = W.problem("tiny")
    prob.denoiser = W.identity_denoiser()
    y32 = f32(orc.OracleProblem(prob).y)
    ref, op = _oracle_solve(orc, prob, y32, "rre", 5, 0, 0.0, 10)
    r = restorer(prob, method="rre", L=5, tol=0.0, max_fp_calls=10)
    x, _ = r.solve(dev(torch, y32), *prob.hr_shape)
    err = rel(host(x), ref.x)
    say(f"  rel L2 vs oracle: {err:.2e}")
    assert err <= _bound(orc, op, ref, "rre", 5, 0, 10)


def test_solve_converges_to_fixed_point(torch, orc):
    """Tolerance-driven RRE solve of the benchmark workload: the FP64 RED gradient at the GPU
    result has fallen by 1e3 and the result matches the oracle's fixed point."""
    say("solve converged deblur256")
    prob = W.problem("deblur256")
    op = orc.OracleProblem(prob)
    y32 = f32(op.y)
    op = orc.OracleProblem(prob, y=y32)
    r = restorer(prob, method="rre", tol=1e-5, max_fp_calls=200)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    xg = host(x)
    say("  stats", st)
    g0 = np.linalg.norm(op.gradient(op.x0()))
    assert np.linalg.norm(op.gradient(xg)) <= 1e-3 * g0
    ref = orc.solve(op, "rre", L=5, m=0, tol=1e-8, max_calls=200)
    err = rel(xg, ref.x)
    say(f"  rel L2 vs oracle fixed point: {err:.2e}")
    assert err <= 1e-4
    assert abs(orc.psnr(xg, prob.x_true) - orc.psnr(ref.x, prob.x_true)) <= 0.01


def test_solve_sr_converges(torch, orc):
    """3x super-resolution solved to tolerance: the result matches the oracle's fixed point."""
    say("solve sr converged")
    x_true = W.make_image(130, 97, 1234)
    prob = W.Problem("sr", x_true, W.psf_gaussian(7, 1.6), 3, 5.0, 0.02,
                     W.make_noise(W.lr_shape(130, 97, 3), 4321), 15, W.make_denoiser(),
                     "rre", 8, 0, 1e-5, 400)
    y32 = f32(orc.OracleProblem(prob).y)
    op = orc.OracleProblem(prob, y=y32)
    r = restorer(prob)
    x, st = r.solve(dev(torch, y32), 130, 97)
    say("  stats", st)
    ref = orc.solve(op, "rre", L=8, m=0, tol=1e-9, max_calls=400)
    err = rel(host(x), ref.x)
    say(f"  rel L2 vs oracle fixed point: {err:.2e}")
    assert err <= 1e-4


def test_solve_deterministic(torch):
    say("determinism")
    prob = W.problem("deblur64")
    import oracle
    y32 = f32(oracle.OracleProblem(prob).y)
    r = restorer(prob, method="rre", tol=0.0, max_fp_calls=10)
    a, _ = r.solve(dev(torch, y32), 64, 64)
    b, _ = r.solve(dev(torch, y32), 64, 64)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ argument checking


def test_errors(torch):
    import paper_1805_02158_amd as P
    say("errors")
    r = restorer()
    y = torch.zeros((8, 8), device="cuda")
    with pytest.raises(P.RedveError) as e:
        r.solve(y, 8, 8)
    assert e.value.code == P.E_STATE
    with pytest.raises(P.RedveError) as e:
        r.set_operator(np.ones((4, 4)) / 16, 1)
    assert e.value.code == P.E_ARG
    with pytest.raises(P.RedveError) as e:
        r.set_extrapolation("rre", 1, 0)
    assert e.value.code == P.E_ARG
    with pytest.raises(P.RedveError) as e:
        r.set_noise(0.0)
    assert e.value.code == P.E_ARG
    d = W.make_denoiser()
    bad = W.DenoiserParams(d.stages, d.nfilt, d.ksize, d.nrbf, d.mu0, d.dmu, d.gamma,
                           d.filters + 0.1, d.rbf_w, d.react)
    with pytest.raises(P.RedveError) as e:
        r.set_denoiser(bad)
    assert e.value.code == P.E_ARG
    prob = W.problem("tiny")
    r.configure(prob)
    with pytest.raises(P.RedveError) as e:
        r.solve(torch.zeros((10, 10), device="cuda"), 32, 32)  # y shape mismatch
    assert e.value.code == P.E_ARG
    with pytest.raises(P.RedveError) as e:
        r.solve(torch.zeros((1, 1), device="cuda"), 1, 1)
    assert e.value.code == P.E_ARG
    # the BF16 stage's LDS: the weight rows (window evaluation) must fit a workgroup's LDS,
    # 160 KiB on gfx950, which every denoiser within the limits does (32 filters of 127 centres
    # take 75 KiB); the FP32 form takes the vector-ALU stage beyond 64 KiB
    big = W.make_denoiser(stages=1, nfilt=32, nrbf=127, mu0=-630.0)
    r.set_denoiser(big, "bf16")
    r.set_denoiser(big, "fp32")


# ------------------------------------------------------------------ mixed precision (BF16 banks)
# Bar for the BF16 form: 5e-3 relative L2 and 0.05 dB PSNR against the FP64 oracle.


@pytest.mark.parametrize("shape", [(64, 64), (37, 53), (3, 5), (256, 256)])
def test_denoiser_bf16(torch, orc, shape):
    """BF16 filter banks (per-window centred operands, FP32 accumulation): the denoiser update
    f(x) - x matches the oracle's to the BF16 bar, 5e-3 relative L2 (BF16 keeps 8 significant
    bits, 3.9e-3 of each operand; the centred operands keep the update's error near 5e-4)."""
    say("denoiser bf16", shape)
    d = W.make_denoiser()
    r = restorer()
    r.set_denoiser(d, "bf16")
    x = f32(W.make_image(*shape, 77) + 5 * W.make_noise(shape, 78))
    g = host(r.denoise(dev(torch, x)))
    o = orc.denoise(x, orc.Denoiser(d))
    err = rel(g - x, o - x)
    say(f"  update rel L2 {err:.2e}")
    assert err <= 5e-3
    c = np.full((24, 40), 88.0)
    assert np.abs(host(r.denoise(dev(torch, c))) - 88.0).max() <= 1e-3


# Denoisers of the BF16 form by how the stage evaluates phi on a small image: tables (row
# stride 25 or 33, 78 to 274 intervals per filter) or, where the tables exceed the LDS
# (gamma = dmu / 3: 394 intervals of 24 filters; 32 filters of 127 centres), the exact window,
# which every denoiser takes on images of 512 tiles or more.
BF16_FORMS = {
    "table 32x63": dict(stages=2, nfilt=32),
    "table 24x127": dict(stages=2, nrbf=127, mu0=-630.0),
    "table gamma 2.2 dmu": dict(stages=2, gamma=22.0),
    "window gamma dmu/3": dict(stages=2, gamma=10.0 / 3.0),
    "window 32x127": dict(stages=2, nfilt=32, nrbf=127, mu0=-630.0),
}


@pytest.mark.parametrize("form", list(BF16_FORMS))
def test_denoiser_bf16_forms(torch, orc, form):
    """Each evaluation of phi in the BF16 stage against the oracle's full sum: the update
    f(x) - x to 5e-3 relative L2, on a small ragged image (tables where they fit) and on one of
    525 tiles (window)."""
    d = W.make_denoiser(**BF16_FORMS[form])
    r = restorer()
    r.set_denoiser(d, "bf16")
    for shape in [(37, 53), (400, 330)]:
        say("denoiser bf16", form, shape)
        x = f32(W.make_image(*shape, 91) + 5 * W.make_noise(shape, 92))
        g = host(r.denoise(dev(torch, x)))
        o = orc.denoise(x, orc.Denoiser(d))
        err = rel(g - x, o - x)
        say(f"  update rel L2 {err:.2e}")
        assert err <= 5e-3


def _converged_bf16(torch, orc, prob, method, L, tol=1e-5, calls=400, precision="bf16"):
    y32 = f32(orc.OracleProblem(prob).y)
    op = orc.OracleProblem(prob, y=y32)
    r = restorer(prob, precision=precision, method=method, L=L, tol=tol, max_fp_calls=calls)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    xg = host(x)
    ref = orc.solve(op, method, L=L, m=0, tol=1e-8, max_calls=calls)
    err = rel(xg, ref.x)
    dp = orc.psnr(xg, prob.x_true) - orc.psnr(ref.x, prob.x_true)
    say(f"  stats {st}")
    say(f"  rel L2 vs oracle fixed point {err:.2e}, dPSNR {dp:+.4f} dB")
    return err, dp


def test_solve_bf16_deblur(torch, orc):
    say("solve bf16 deblur 256")
    err, dp = _converged_bf16(torch, orc, W.problem("deblur256"), "rre", 5)
    assert err <= 5e-3 and abs(dp) <= 0.05


@pytest.mark.parametrize("psf", ["u9", "g7"])
@pytest.mark.parametrize("form", list(FUSED_DENOISERS))
def test_solve_bf16_fused_start_forms(torch, orc, psf, form):
    """BF16 banks (tabulated phi) with the CG start formed by the last stage, for a 9x9 and a
    7x7 PSF, one stage and 32 filters: converged RRE solves of a 64x64 deblurring against the
    oracle's fixed point, the BF16 bar."""
    say("solve bf16 fused start", psf, form)
    err, dp = _converged_bf16(torch, orc, _fused_problem(psf, form, (64, 64)), "rre", 5)
    assert err <= 5e-3 and abs(dp) <= 0.05


def test_solve_bf16_sr_512(torch, orc):
    """The mixed-precision workload at full size: 512x512, Gaussian 7x7 + 3x decimation,
    sigma 5, RRE with L = 8, FP64 Gram and small solve."""
    say("solve bf16 sr 512")
    err, dp = _converged_bf16(torch, orc, W.problem("sr512"), "rre", 8, calls=300)
    assert err <= 5e-3 and abs(dp) <= 0.05


def test_solve_fp32_sr_512(torch, orc):
    """The same workload with FP32 banks, converged, against the oracle's fixed point: the FP32
    bar, 1e-4."""
    say("solve fp32 sr 512")
    err, dp = _converged_bf16(torch, orc, W.problem("sr512"), "rre", 8, calls=300,
                              precision="fp32")
    assert err <= 1e-4 and abs(dp) <= 0.05


@pytest.mark.parametrize("name,L,calls", [("deblur256", 5, 5), ("deblur256", 5, 10),
                                          ("sr512", 8, 16)])
def test_solve_bf16_fixed_schedule(torch, orc, name, L, calls):
    """BF16 banks at the same schedule as the FP64 oracle (the benchmark's 5 FP calls of RRE
    at 256x256, two cycles, and two cycles of the 3x SR workload): the BF16 bar, 5e-3 relative
    L2 and 0.05 dB."""
    say("solve bf16 fixed schedule", name, L, calls)
    prob = W.problem(name)
    y32 = f32(orc.OracleProblem(prob).y)
    ref = orc.solve(orc.OracleProblem(prob, y=y32), "rre", L=L, m=0, tol=0.0, max_calls=calls)
    r = restorer(prob, precision="bf16", method="rre", L=L, m=0, tol=0.0, max_fp_calls=calls)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    assert st["fp_calls"] == ref.calls and st["cycles"] == ref.cycles
    xg = host(x)
    err = rel(xg, ref.x)
    dp = orc.psnr(xg, prob.x_true) - orc.psnr(ref.x, prob.x_true)
    say(f"  rel L2 vs oracle {err:.2e}, dPSNR {dp:+.4f} dB")
    assert err <= 5e-3 and abs(dp) <= 0.05


@pytest.mark.parametrize("name,method,L,cycles", [("deblur64", "rre", 5, 3), ("deblur64", "mpe", 5, 3),
                                                  ("deblur64", "svd_mpe", 5, 2), ("tiny", "rre", 3, 4)])
def test_solve_stepwise_on_the_gpu_trajectory(torch, orc, name, method, L, cycles):
    """Each step of a fixed-schedule VE solve checked where it happens: every FP call against
    the oracle's FP map started from the GPU's own FP32 iterate (the FP32 bars: 2e-5 relative,
    and 1e-4 of the step, where the step is larger than the output's own FP32 rounding: the
    error may be 1e-4 ||step|| + 2^-22 ||x||), and every extrapolation against the oracle's
    (Algorithm 1 / eq. (19) / SVD-MPE) on the GPU's own FP32 window (2e-6; the breakdown flag
    equal). The solve's result is that trajectory's (the same kernels as the single steps)."""
    say("stepwise", name, method, L, cycles)
    prob = W.problem(name)
    y32 = f32(orc.OracleProblem(prob).y)
    op = orc.OracleProblem(prob, y=y32)
    r = restorer(prob, method=method, L=L, m=0, tol=0.0, max_fp_calls=cycles * L)
    y = dev(torch, y32)
    x = dev(torch, op.x0())
    worst_fp = worst_step = worst_ve = 0.0
    for c in range(cycles):
        win = [x]
        for _ in range(L):
            xin = win[-1]
            xg = r.fp_step(y, xin)
            xi, xo = host(xin), op.fp(host(xin))
            worst_fp = max(worst_fp, rel(host(xg), xo))
            bar = 1e-4 * np.linalg.norm(xo - xi) + 2.0 ** -22 * np.linalg.norm(xo)
            worst_step = max(worst_step, float(np.linalg.norm(host(xg) - xo)) / bar)
            win.append(xg)
        stack = torch.stack(win)
        xe, g, bd = r.extrapolate(stack)
        xo, go, bo = orc.ve_step([host(v).ravel() for v in win], method)
        assert bd == bo
        worst_ve = max(worst_ve, rel(host(xe).ravel(), xo))
        x = xe
    say(f"  worst FP call {worst_fp:.2e} (of its step bar {worst_step:.2f}), worst extrapolation "
        f"{worst_ve:.2e}")
    assert worst_fp <= 2e-5 and worst_step <= 1.0 and worst_ve <= 2e-6
    xs, st = r.solve(y, *prob.hr_shape)
    e = rel(host(xs), host(x))
    say(f"  solve vs the stepwise trajectory {e:.2e}")
    assert st["fp_calls"] == cycles * L and e <= 1e-6
