"""The exact Fourier linear step (redve_set_linear_solver(REDVE_LIN_FFT)) against the oracle's
ExactFPMap (the FP map of eq. (7) with A inverted in the DFT basis, numpy FFT in FP64): one FP
call on sizes that take every radix path of the library's FFT (powers of two, 3 and 5, and
prime lengths 37 and 53 that take the direct-sum stage), fixed-schedule solves with and without
extrapolation, a converged solve on the fixed point shared with the CG map, and the refusals
(super-resolution, sides above 4096, batched engine)."""
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


def ragged():
    """37x53, a non-symmetric 5x3 PSF (the DFT convention must match the blur's)."""
    psf = np.random.default_rng(21).uniform(0, 1, (5, 3))
    psf /= psf.sum()
    return W.Problem("ragged", W.make_image(37, 53, 1700), psf, 1, W.SQRT2, 0.02,
                     W.make_noise((37, 53), 1800), 15, W.make_denoiser())


def sized(h, w, seed):
    """Uniform 9x9 deblurring of an h x w image (sizes chosen for their factors)."""
    return W.Problem(f"u9_{h}x{w}", W.make_image(h, w, seed), W.psf_uniform(9), 1, W.SQRT2, 0.02,
                     W.make_noise((h, w), seed + 100), 15, W.make_denoiser())


PROBLEMS = {"tiny": lambda: W.problem("tiny"), "deblur64": lambda: W.problem("deblur64"),
            "ragged": ragged, "deblur256": lambda: W.problem("deblur256"),
            "45x60": lambda: sized(45, 60, 1901), "2x3": lambda: sized(2, 3, 1902),
            "384x500": lambda: sized(384, 500, 1903), "17x1024": lambda: sized(17, 1024, 1904),
            # every shape of the row and column workgroups: rows of 1536 (radix 3) and 2048
            # (512 threads, four elements each), of 3125 (radix 5) and 4096 (eight each); columns
            # of 2048 (two per workgroup) and 4096 (one)
            "7x1536": lambda: sized(7, 1536, 1905), "9x2048": lambda: sized(9, 2048, 1906),
            "3x3125": lambda: sized(3, 3125, 1907), "5x4096": lambda: sized(5, 4096, 1908),
            "2048x9": lambda: sized(2048, 9, 1909), "4096x6": lambda: sized(4096, 6, 1910)}


def restorer(prob, **kw):
    from paper_1805_02158_amd import Restorer
    return Restorer(0).configure(prob, **kw).set_linear_solver("fft")


class _Rounded:
    def __init__(self, base):
        self.base, self.shape = base, base.shape

    def x0(self):
        return f32(self.base.x0())

    def fp(self, x):
        return f32(self.base.fp(x))


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_fft_fp_step(torch, orc, name):
    say("fft fp step", name)
    prob = PROBLEMS[name]()
    op = orc.OracleProblem(prob, y=f32(orc.OracleProblem(prob).y))
    ex = orc.ExactFPMap(op)
    r = restorer(prob)
    x = f32(op.x0())
    for _ in range(3):
        xg = host(r.fp_step(dev(torch, op.y), dev(torch, x)))
        xo = ex.fp(x)
        say(f"  rel L2 {rel(xg, xo):.2e}, relative to the step {rel(xg - x, xo - x):.2e}")
        assert rel(xg, xo) <= 2e-5
        assert rel(xg - x, xo - x) <= 1e-4
        x = f32(xo)


@pytest.mark.parametrize("name,method,L,calls", [("deblur64", "none", 5, 20),
                                                 ("deblur64", "rre", 5, 20),
                                                 ("ragged", "mpe", 4, 16)])
def test_fft_solve_fixed_schedule(torch, orc, name, method, L, calls):
    prob = PROBLEMS[name]()
    y32 = f32(orc.OracleProblem(prob).y)
    ex = orc.ExactFPMap(orc.OracleProblem(prob, y=y32))
    ref = orc.solve(ex, method, L=L, m=0, tol=0.0, max_calls=calls)
    r = restorer(prob, method=method, L=L, m=0, tol=0.0, max_fp_calls=calls)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    assert st["fp_calls"] == ref.calls and st["cycles"] == ref.cycles
    err = rel(host(x), ref.x)
    bound = 1e-4
    if method != "none":
        moved = orc.solve(_Rounded(ex), method, L=L, m=0, tol=0.0, max_calls=calls)
        bound = max(1e-4, 3.0 * rel(moved.x, ref.x))
    say(f"  {name} {method}: rel L2 vs oracle {err:.2e} (bound {bound:.1e})")
    assert err <= bound


def test_fft_converges_to_the_shared_fixed_point(torch, orc):
    """RRE with the exact solve reaches the fixed point of the CG-based oracle iteration."""
    prob = W.problem("deblur256")
    y32 = f32(orc.OracleProblem(prob).y)
    ref = orc.solve(orc.OracleProblem(prob, y=y32), "rre", L=5, m=0, tol=1e-10, max_calls=300)
    r = restorer(prob, method="rre", L=5, m=0, tol=1e-6, max_fp_calls=200)
    x, st = r.solve(dev(torch, y32), *prob.hr_shape)
    e = rel(host(x), ref.x)
    say(f"  {st['fp_calls']} FP calls, rel L2 vs the fixed point {e:.2e}")
    assert st["status"] == 0 and e <= 1e-4


def test_fft_refusals(torch):
    from paper_1805_02158_amd import E_ARG, RedveError
    sr = W.problem("sr512")
    r = restorer(sr)
    y = torch.zeros(W.lr_shape(512, 512, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(RedveError):
        r.solve(y, 512, 512)
    wide = sized(2, 4100, 1905)
    rw = restorer(wide)
    yw = torch.zeros((2, 4100), dtype=torch.float32, device="cuda")
    with pytest.raises(RedveError) as ei:
        rw.solve(yw, 2, 4100)
    assert ei.value.code == E_ARG
    p = W.problem("tiny")
    r2 = restorer(p)
    with pytest.raises(RedveError):
        r2.solve_batch([dict(y=dev(torch, np.zeros(p.hr_shape)), hx=32, wx=32, psf=p.psf, decim=1,
                             sigma=p.sigma, lam=p.lam)])
