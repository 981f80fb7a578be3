"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks one part of the oracle against something other than itself: a library
routine (FFT, dense solve, QR, SVD, scipy filtering), a closed form, an invariant, or brute
force on a tiny input. Together they are chosen so that a dropped term, a wrong sign or index,
or a transposed operand anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

import workload as W

RNG = np.random.default_rng(12345)


def _psf_pad(psf, shape):
    """Embed a centred PSF in an H x W array at wrap-around offsets (for FFT convolution)."""
    kh, kw = psf.shape
    rh, rw = kh // 2, kw // 2
    K = np.zeros(shape)
    for a in range(-rh, rh + 1):
        for b in range(-rw, rw + 1):
            K[a % shape[0], b % shape[1]] += psf[a + rh, b + rw]
    return K


def _dense(op, shape_in):
    n = int(np.prod(shape_in))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(np.ravel(op(e.reshape(shape_in))))
    return np.stack(cols, axis=1)


# ------------------------------------------------------------------ degradation operator


@pytest.mark.parametrize("shape", [(16, 16), (13, 21), (5, 7), (40, 9)])
def test_blur_is_circular_convolution(orc, shape):
    """Eq. (1) with block-circulant H (footnote to eq. (7)): B x = x (*) h, computed by FFT.
    A non-symmetric PSF catches a flipped or transposed kernel."""
    psf = RNG.standard_normal((5, 3))
    x = RNG.standard_normal(shape)
    ref = np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(_psf_pad(psf, shape))))
    assert np.allclose(orc.blur(x, psf), ref, atol=1e-12 * np.abs(ref).max() + 1e-13)
    ref_adj = np.real(np.fft.ifft2(np.fft.fft2(x) * np.conj(np.fft.fft2(_psf_pad(psf, shape)))))
    assert np.allclose(orc.blur_adj(x, psf), ref_adj, atol=1e-12 * np.abs(ref_adj).max() + 1e-13)


@pytest.mark.parametrize("shape,s", [((12, 12), 3), ((13, 11), 3), ((10, 7), 2), ((9, 9), 1)])
def test_H_and_Ht_adjoint_and_decimation(orc, shape, s):
    """y = S B x keeps samples (s i, s j); H^T is its exact adjoint."""
    psf = RNG.standard_normal((7, 7))
    x = RNG.standard_normal(shape)
    bx = orc.blur(x, psf)
    y = orc.apply_H(x, psf, s)
    assert y.shape == (-(-shape[0] // s), -(-shape[1] // s))
    assert np.array_equal(y, bx[::s, ::s])
    z = RNG.standard_normal(y.shape)
    lhs = float(np.sum(y * z))
    rhs = float(np.sum(x * orc.apply_Ht(z, shape, psf, s)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0) * 10
    zf = orc.decimate_adj(z, shape, s)
    assert np.count_nonzero(zf) <= z.size and np.array_equal(zf[::s, ::s], z)


def test_A_matches_dense_operator_and_fft_eigenvalues(orc):
    """A = H^T H / sigma^2 + lambda I assembled densely is symmetric positive definite and, for
    periodic deblurring, has eigenvalues |h_hat|^2 / sigma^2 + lambda (footnote to eq. (7))."""
    shape, psf, sigma, lam = (8, 8), W.psf_gaussian(7, 1.6), math.sqrt(2), 0.02
    A = _dense(lambda p: orc.apply_A(p, psf, 1, sigma, lam), shape)
    assert np.allclose(A, A.T, atol=1e-14)
    ev = np.sort(np.linalg.eigvalsh(A))
    hh = np.abs(np.fft.fft2(_psf_pad(psf, shape))) ** 2 / sigma ** 2 + lam
    assert np.allclose(ev, np.sort(hh.ravel()), rtol=1e-10, atol=1e-12)
    # with decimation: H built from explicit dense blur and sampling matrices
    B = _dense(lambda p: orc.blur(p, psf), shape)
    S = np.zeros((9, 64))
    for r, (i, j) in enumerate([(i, j) for i in range(0, 8, 3) for j in range(0, 8, 3)]):
        S[r, i * 8 + j] = 1.0
    Hd = S @ B
    A3 = _dense(lambda p: orc.apply_A(p, psf, 3, 5.0, lam), shape)
    assert np.allclose(A3, Hd.T @ Hd / 25.0 + lam * np.eye(64), atol=1e-14)


@pytest.mark.parametrize("s,sigma", [(1, math.sqrt(2)), (3, 5.0)])
def test_cg_equals_dense_solve_8x8(orc, s, sigma):
    """64 CG iterations on an 8x8 image reproduce numpy.linalg.solve of the dense system."""
    shape, psf, lam = (8, 8), W.psf_gaussian(7, 1.6), 0.02
    A = _dense(lambda p: orc.apply_A(p, psf, s, sigma, lam), shape)
    rhs = RNG.standard_normal(shape) * 10
    x0 = RNG.standard_normal(shape)
    xs = np.linalg.solve(A, rhs.ravel()).reshape(shape)
    x = orc.cg(rhs, x0, psf, s, sigma, lam, 64)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_cg_matches_fourier_closed_form(orc):
    """Periodic deblurring: CG to convergence = IFFT(FFT(rhs) / (|h_hat|^2/sigma^2 + lambda)),
    the Fourier-domain inversion of the footnote to eq. (7)."""
    shape, psf, sigma, lam = (32, 24), W.psf_uniform(9), math.sqrt(2), 0.02
    rhs = RNG.standard_normal(shape) * 50
    den = np.abs(np.fft.fft2(_psf_pad(psf, shape))) ** 2 / sigma ** 2 + lam
    xs = np.real(np.fft.ifft2(np.fft.fft2(rhs) / den))
    x = orc.cg(rhs, np.zeros(shape), psf, 1, sigma, lam, 400)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_cg_warm_start_keeps_solution_and_zero_residual_stops(orc):
    shape, psf = (8, 8), W.psf_uniform(9)
    x = RNG.standard_normal(shape)
    rhs = orc.apply_A(x, psf, 1, 1.0, 0.5)
    out = orc.cg(rhs, x, psf, 1, 1.0, 0.5, 10)
    assert np.allclose(out, x, rtol=0, atol=1e-12)


# ------------------------------------------------------------------ denoiser


@pytest.mark.parametrize("shape", [(9, 9), (12, 7), (3, 5), (2, 2)])
def test_filter_fwd_is_reflect_correlation(orc, shape):
    """K u = correlation of the half-sample symmetric extension (scipy mode='reflect')."""
    k = RNG.standard_normal((5, 5))
    u = RNG.standard_normal(shape)
    ref = ndi.correlate(u, k, mode="reflect")
    assert np.allclose(orc.filter_fwd(u, k), ref, atol=1e-13)


@pytest.mark.parametrize("shape", [(7, 6), (4, 9), (2, 3)])
def test_filter_adj_is_dense_transpose(orc, shape):
    """K^T built column by column equals the transpose of K built column by column."""
    k = RNG.standard_normal((5, 5))
    K = _dense(lambda u: orc.filter_fwd(u, k), shape)
    Kt = _dense(lambda v: orc.filter_adj(v, k), shape)
    assert np.allclose(Kt, K.T, atol=1e-14)


def test_phi_closed_forms(orc):
    """phi(z) = sum_j w_j exp(-(z - mu_j)^2 / (2 gamma^2)): a unit weight on one centre gives
    1 at the centre and exp(-1/2) one width away; antisymmetric weights give an odd phi."""
    w = np.zeros(63)
    w[40] = 1.0
    mu = -310.0 + 10.0 * 40
    assert orc.phi(np.array([mu]), w)[0] == pytest.approx(1.0, abs=1e-15)
    assert orc.phi(np.array([mu + 10.0]), w)[0] == pytest.approx(math.exp(-0.5), rel=1e-14)
    assert orc.phi(np.array([mu - 20.0]), w)[0] == pytest.approx(math.exp(-2.0), rel=1e-14)
    d = W.make_denoiser()
    z = np.linspace(-400, 400, 161)
    for t, i in [(0, 0), (2, 13), (4, 23)]:
        wt = d.rbf_w[t, i]
        assert abs(orc.phi(np.array([0.0]), wt)[0]) <= 1e-12
        assert np.allclose(orc.phi(z, wt), -orc.phi(-z, wt), atol=1e-12)


def _stage_independent(d, t, u, f):
    """One stage u - sum_i K_i^T phi_i(K_i u) - theta_t (u - f) (Sec. IV's TNRD-style
    diffusion step), rebuilt from scipy reflect correlation, a dense transpose of it, and a
    direct sum of Gaussians."""
    shape = u.shape
    mu = d.mu0 + d.dmu * np.arange(d.nrbf)
    g = np.zeros(u.size)
    for i in range(d.nfilt):
        k = d.filters[t, i]
        K = _dense(lambda v: ndi.correlate(v, k, mode="reflect"), shape)
        z = K @ u.ravel()
        v = (d.rbf_w[t, i][None, :] * np.exp(-(z[:, None] - mu[None, :]) ** 2
                                              / (2 * d.gamma ** 2))).sum(1)
        g += K.T @ v
    return (u.ravel() - g - d.react[t] * (u.ravel() - f.ravel())).reshape(shape)


def test_stage_from_independent_pieces(orc):
    """One stage of the oracle equals the stage rebuilt from independent pieces."""
    d = W.make_denoiser()
    den = orc.Denoiser(d)
    shape = (6, 7)
    u = RNG.uniform(0, 255, shape)
    f = RNG.uniform(0, 255, shape)
    t = 2
    ref = _stage_independent(d, t, u, f)
    assert np.allclose(orc.tnrd_stage(u, f, den, t), ref, atol=1e-11)


def test_denoiser_composes_stages_in_order_with_fixed_reaction_input(orc):
    """D(x) = u_T with u_0 = x and u_t = stage_t(u_{t-1}; f = x): the stages run in the order
    t = 0 .. T-1 and the reaction term of every stage pulls towards the denoiser's input x,
    not towards the previous stage's output. Rebuilt from the independent stage above on a
    6x7 image with T = 5; the two plausible slips (reversed stage order, reaction towards
    u_{t-1}) are far from the result, so either would fail."""
    d = W.make_denoiser()
    den = orc.Denoiser(d)
    x = RNG.uniform(0, 255, (6, 7))
    u = x.copy()
    for t in range(d.stages):
        u = _stage_independent(d, t, u, x)
    got = orc.denoise(x, den)
    assert np.abs(got - u).max() <= 1e-11 * max(1.0, np.abs(u).max())
    rev = x.copy()
    for t in reversed(range(d.stages)):
        rev = _stage_independent(d, t, rev, x)
    prev = x.copy()
    for t in range(d.stages):
        prev = _stage_independent(d, t, prev, prev)
    assert np.abs(got - rev).max() > 1e-3
    assert np.abs(got - prev).max() > 1e-3


@pytest.mark.parametrize("c", [0.0, 37.5, 255.0])
def test_denoiser_keeps_constants(orc, c):
    """Zero-mean filters and odd influence functions: D maps a constant image to itself."""
    den = orc.Denoiser(W.make_denoiser())
    x = np.full((11, 13), c)
    assert np.abs(orc.denoise(x, den) - x).max() <= 1e-12


def test_denoiser_zero_stages_is_identity(orc):
    den = orc.Denoiser(W.identity_denoiser())
    x = RNG.uniform(0, 255, (8, 9))
    assert np.array_equal(orc.denoise(x, den), x)


def test_denoiser_denoises(orc):
    """The seeded D is a denoiser: it raises PSNR of an image with N(0, 5^2) noise."""
    den = orc.Denoiser(W.make_denoiser())
    x = W.make_image(64, 64, 1000)
    noisy = x + 5.0 * W.make_noise(x.shape, 7)
    assert orc.psnr(orc.denoise(noisy, den), x) > orc.psnr(noisy, x) + 0.5


def test_denoiser_passivity(orc):
    """Strong passivity (Sec. II-B): the spectral radius of the Jacobian of D is at most one,
    estimated by power iteration on finite-difference Jacobian-vector products."""
    den = orc.Denoiser(W.make_denoiser())
    x = W.make_image(24, 24, 1003)
    fx = orc.denoise(x, den)
    v = RNG.standard_normal(x.shape)
    h = 1e-4
    lam = 0.0
    for _ in range(40):
        v /= np.linalg.norm(v)
        jv = (orc.denoise(x + h * v, den) - orc.denoise(x - h * v, den)) / (2 * h)
        lam = np.linalg.norm(jv)
        v = jv
    assert lam <= 1.0 + 1e-6
    assert np.isfinite(fx).all()


def test_psnr_closed_form(orc):
    x = RNG.uniform(0, 255, (10, 10))
    assert orc.psnr(x + 1.0, x) == pytest.approx(20 * math.log10(255.0), rel=1e-12)


# ------------------------------------------------------------------ vector extrapolation


def _U(n=40, k1=5, seed=0):
    return np.random.default_rng(seed).standard_normal((n, k1))


def test_mgs_against_numpy_qr(orc):
    """Algorithm 2: Q R = U, Q^T Q = I, and R equals LAPACK's R up to the sign of each row."""
    U = _U()
    Q, R = orc.mgs(U)
    assert np.allclose(Q @ R, U, atol=1e-13)
    assert np.allclose(Q.T @ Q, np.eye(5), atol=1e-13)
    Rn = np.linalg.qr(U, mode="r")
    assert np.allclose(np.abs(R), np.abs(Rn), atol=1e-12)
    assert np.allclose(np.triu(R), R)
    assert (np.diag(R) > 0).all()


def test_cholesky_of_gram_equals_mgs_r(orc):
    """Full-rank U: chol(U^T U)^T = R of MGS (the Gram route reaches the same R)."""
    U = _U(200, 6, 3)
    _, R = orc.mgs(U)
    C = np.linalg.cholesky(U.T @ U).T
    assert np.allclose(C, R, rtol=1e-10, atol=1e-12)


def test_algorithm1_combination_identity(orc):
    """x_m + Q_{k-1} eta (Algorithm 1, step 4) equals sum_i gamma_i x_{m+i} (eq. (11))."""
    X = np.random.default_rng(5).standard_normal((30, 6))
    U = X[:, 1:] - X[:, :-1]
    Q, R = orc.mgs(U)
    for g in (orc.mpe_gamma(R), orc.rre_gamma(R), orc.svd_mpe_gamma(R)):
        assert abs(g.sum() - 1) < 1e-12
        direct = X[:, :len(g)] @ g
        assert np.allclose(orc.extrapolate(X[:, 0], Q, R, g), direct, atol=1e-10)


def test_mpe_solves_constrained_least_squares(orc):
    """MPE (eq. (18)): c minimises ||U c|| subject to c_kappa = 1 (normal equations of the
    first kappa columns against the last)."""
    U = _U(50, 5, 9)
    _, R = orc.mgs(U)
    g = orc.mpe_gamma(R)
    c = g / g[-1]
    cp, *_ = np.linalg.lstsq(U[:, :-1], -U[:, -1], rcond=None)
    assert np.allclose(c[:-1], cp, rtol=1e-10, atol=1e-12)


def test_rre_optimality_and_kkt(orc):
    """RRE (eq. (19)): gamma minimises ||U gamma|| subject to sum gamma = 1; matches the KKT
    solve and beats MPE's gamma and random feasible gammas."""
    U = _U(60, 5, 11)
    _, R = orc.mgs(U)
    g = orc.rre_gamma(R)
    G = U.T @ U
    kkt = np.block([[2 * G, np.ones((5, 1))], [np.ones((1, 5)), np.zeros((1, 1))]])
    sol = np.linalg.solve(kkt, np.concatenate([np.zeros(5), [1.0]]))
    assert np.allclose(g, sol[:5], rtol=1e-9, atol=1e-12)
    best = np.linalg.norm(U @ g)
    assert best <= np.linalg.norm(U @ orc.mpe_gamma(R)) + 1e-12
    rng = np.random.default_rng(1)
    for _ in range(50):
        r = rng.standard_normal(5)
        r /= r.sum()
        assert best <= np.linalg.norm(U @ r) + 1e-12


def test_svd_mpe_is_smallest_right_singular_vector_of_U(orc):
    """SVD-MPE: the right singular vectors of R are those of U (U = QR)."""
    U = _U(70, 5, 13)
    _, R = orc.mgs(U)
    g = orc.svd_mpe_gamma(R)
    v = np.linalg.svd(U)[2][-1]
    assert np.allclose(g, v / v.sum(), rtol=1e-9, atol=1e-12)


def test_mpe_rre_relation(orc):
    """Sec. III-B: mu_k RRE_k = mu_{k-1} RRE_{k-1} + v_k MPE_k with positive scalars, i.e.
    RRE_k is a convex combination of RRE_{k-1} and MPE_k."""
    rng = np.random.default_rng(21)
    A = np.diag(rng.uniform(-0.9, 0.9, 12))
    Qr, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    A = Qr @ A @ Qr.T
    b = rng.standard_normal(12)
    xs = [rng.standard_normal(12)]
    for _ in range(5):
        xs.append(A @ xs[-1] + b)
    X = np.stack(xs, axis=1)
    for k1 in (3, 4, 5):
        U = X[:, 1:k1 + 1] - X[:, :k1]
        Q, R = orc.mgs(U)
        rre_k = orc.extrapolate(X[:, 0], Q, R, orc.rre_gamma(R))
        mpe_k = orc.extrapolate(X[:, 0], Q, R, orc.mpe_gamma(R))
        Q1, R1 = orc.mgs(U[:, :-1])
        rre_k1 = orc.extrapolate(X[:, 0], Q1, R1, orc.rre_gamma(R1))
        M = np.stack([rre_k1 - mpe_k], axis=1)
        t, *_ = np.linalg.lstsq(M, rre_k - mpe_k, rcond=None)
        assert np.linalg.norm(M @ t - (rre_k - mpe_k)) <= 1e-9 * np.linalg.norm(rre_k)
        assert 0.0 < t[0] < 1.0


class _Linear:
    """x -> A x + b, the linear process of eq. (8), with the FP-call interface."""

    def __init__(self, A, b, x0):
        self.A, self.b, self._x0 = A, b, x0
        self.shape = x0.shape

    def x0(self):
        return self._x0.copy()

    def fp(self, x):
        return self.A @ x + self.b


@pytest.mark.parametrize("method", ["mpe", "rre", "svd_mpe"])
def test_linear_exactness_full_degree(orc, method):
    """Sec. III-A: with kappa equal to the degree of the minimal polynomial (here N = 6), one
    extrapolation from x_0 .. x_{kappa+1} lands on x* = (I - A)^{-1} b."""
    rng = np.random.default_rng(2)
    N = 6
    Qr, _ = np.linalg.qr(rng.standard_normal((N, N)))
    A = Qr @ np.diag(np.linspace(-0.9, 0.9, N)) @ Qr.T
    b = rng.standard_normal(N)
    xstar = np.linalg.solve(np.eye(N) - A, b)
    op = _Linear(A, b, rng.standard_normal(N))
    if method == "svd_mpe":
        # kappa = N makes U rank deficient: SVD-MPE takes the exact null vector
        pass
    r = orc.solve(op, method, L=N + 1, m=0, tol=0.0, max_calls=N + 1)
    assert r.cycles == 1
    assert np.linalg.norm(r.x - xstar) <= 1e-9 * np.linalg.norm(xstar)


@pytest.mark.parametrize("method", ["mpe", "rre"])
def test_linear_exactness_few_eigenvalues(orc, method):
    """A with d = 3 distinct eigenvalues in N = 10 dimensions: kappa = d suffices."""
    rng = np.random.default_rng(3)
    N, d = 10, 3
    Qr, _ = np.linalg.qr(rng.standard_normal((N, N)))
    ev = np.repeat([0.8, -0.5, 0.3], [4, 3, 3])
    A = Qr @ np.diag(ev) @ Qr.T
    b = rng.standard_normal(N)
    xstar = np.linalg.solve(np.eye(N) - A, b)
    op = _Linear(A, b, rng.standard_normal(N))
    r = orc.solve(op, method, L=d + 1, m=0, tol=0.0, max_calls=d + 1)
    assert np.linalg.norm(r.x - xstar) <= 1e-9 * np.linalg.norm(xstar)
    r2 = orc.solve(op, method, L=d, m=0, tol=0.0, max_calls=d)
    assert np.linalg.norm(r2.x - xstar) > 1e-6 * np.linalg.norm(xstar)


@pytest.mark.parametrize("method", ["mpe", "rre"])
def test_asymptotic_rate_eq20(orc, method):
    """Eq. (20): x_(m,kappa) - x* = O(lambda_{kappa+1}^m) for diagonalisable A."""
    N, kappa = 8, 2
    lam = np.array([0.95, 0.9, 0.6, 0.5, 0.4, 0.3, 0.2, 0.1])
    rng = np.random.default_rng(4)
    A = np.diag(lam)
    b = rng.standard_normal(N)
    xstar = b / (1 - lam)
    x0 = rng.standard_normal(N)
    ms = np.arange(20, 60, 5)
    errs = []
    for m in ms:
        op = _Linear(A, b, x0)
        r = orc.solve(op, method, L=kappa + 1, m=int(m), tol=0.0, max_calls=int(m) + kappa + 1)
        errs.append(np.linalg.norm(r.x - xstar))
    slope = np.polyfit(ms, np.log(errs), 1)[0]
    assert slope == pytest.approx(math.log(lam[kappa]), rel=0.05)


class _Sequence:
    """Replays a fixed list of iterates as FP calls."""

    def __init__(self, xs):
        self.xs = [np.asarray(v, float) for v in xs]
        self.shape = self.xs[0].shape
        self.k = 0

    def x0(self):
        return self.xs[0].copy()

    def fp(self, x):
        self.k += 1
        return self.xs[self.k].copy()


def test_mpe_breakdown_returns_last_iterate(orc):
    """MPE does not exist when sum c = 0 (Sec. III-B): with u_0 = (1, 0) and u_1 = (1, 5) the
    least-squares c_0 is -1. The solve then continues from the last FP iterate and counts a
    breakdown, while RRE still extrapolates."""
    xs = [np.zeros(2), np.array([1.0, 0.0]), np.array([2.0, 5.0])]
    xnew, g, broke = orc.ve_step(xs, "mpe")
    assert broke and g is None and np.array_equal(xnew, xs[-1])
    r = orc.solve(_Sequence(xs), "mpe", L=2, m=0, tol=0.0, max_calls=2)
    assert r.breakdowns == 1 and np.array_equal(r.x, xs[-1])
    xr, gr, broke_r = orc.ve_step(xs, "rre")
    assert not broke_r and abs(gr.sum() - 1) < 1e-14


def test_rre_when_mpe_does_not_exist(orc):
    """Sec. III-B: if MPE does not exist, RRE_kappa = RRE_{kappa-1}. A last column equal to the
    first makes c = (-1, 0, 0, 1) with sum c = 0."""
    U = _U(20, 3, 1)
    U = np.concatenate([U, U[:, :1]], axis=1)
    _, R = orc.mgs(U)
    assert orc.mpe_gamma(R) is None
    g = orc.rre_gamma(R)
    _, R3 = orc.mgs(U[:, :3])
    assert np.allclose(g, orc.rre_gamma(R3), rtol=1e-10)
    assert abs(g.sum() - 1) < 1e-12


@pytest.mark.parametrize("method", ["mpe", "rre", "svd_mpe"])
def test_stability_guard_closed_form(orc, method):
    """Sec. III-D, eq. (21), on one geometric mode x_k = x* + v lam^k with L = 2 (kappa = 1):
    U = [u, lam u] has rank one, every variant's coefficients are gamma = (-lam, 1) / (1 - lam)
    (MPE: c = (-lam, 1); RRE takes MPE's null vector; SVD-MPE the null singular vector), so
    sum |gamma| = (1 + lam) / (1 - lam) = 1999 at lam = 0.999 in closed form, and the exact
    extrapolation is x*. A cap above that sum keeps x*; below it the guard returns the last
    iterate, flagged as a breakdown, with the rejected coefficients. (The differences lose
    five digits to cancellation, which 1 / (1 - lam) magnifies: gamma agrees to 1e-7.)"""
    rng = np.random.default_rng(77)
    lam = 0.999
    xstar = rng.uniform(50, 200, 40)
    v = rng.standard_normal(40)
    xs = [xstar + v * lam ** k for k in range(3)]
    l1 = (1 + lam) / (1 - lam)
    x, g, broke = orc.ve_step(xs, method, gamma_cap=2500.0)
    assert not broke and abs(np.abs(g).sum() - l1) <= 1e-7 * l1
    assert np.allclose(g, np.array([-lam, 1.0]) / (1 - lam), rtol=1e-7)
    assert np.linalg.norm(x - xstar) <= 1e-9 * np.linalg.norm(xstar)
    x, g, broke = orc.ve_step(xs, method, gamma_cap=1500.0)
    assert broke and np.array_equal(x, xs[-1]) and abs(np.abs(g).sum() - l1) <= 1e-7 * l1
    x, g, broke = orc.ve_step(xs, method, gamma_cap=0)  # off
    assert not broke and np.linalg.norm(x - xstar) <= 1e-9 * np.linalg.norm(xstar)


def test_guard_rejecting_every_window_is_plain_fp(orc):
    """sum |gamma| >= |sum gamma| = 1, so a cap below 1 rejects every extrapolation: each cycle
    then continues from its last FP iterate and the solve is plain FP, call for call (the
    rejected cycles count as breakdowns)."""
    P = W.Problem("guard", W.make_image(16, 16, 1011), W.psf_gaussian(7, 1.6), 1, W.SQRT2, 0.02,
                  W.make_noise((16, 16), 2011), 10, W.make_denoiser())
    op = orc.OracleProblem(P)
    plain = orc.solve(op, "none", tol=0.0, max_calls=15)
    for method in ("mpe", "rre", "svd_mpe"):
        r = orc.solve(op, method, L=5, m=0, tol=0.0, max_calls=15, gamma_cap=0.5)
        assert r.cycles == 3 and r.breakdowns == 3 and r.rejected == 3
        assert np.array_equal(r.x, plain.x)
        free = orc.solve(op, method, L=5, m=0, tol=0.0, max_calls=15)
        assert free.rejected == 0 and not np.array_equal(free.x, plain.x)


# ------------------------------------------------------------------ the RED fixed point


@pytest.fixture(scope="module")
def small_solution(orc):
    P = W.Problem("pin", W.make_image(32, 32, 1010), W.psf_uniform(9), 1, W.SQRT2, 0.02,
                  W.make_noise((32, 32), 2010), 15, W.make_denoiser())
    op = orc.OracleProblem(P)
    res = {m: orc.solve(op, m, L=5, m=0, tol=1e-9, max_calls=400) for m in ("none", "rre", "mpe")}
    return op, res


def test_fixed_point_gradient_vanishes(orc, small_solution):
    """Eq. (5)-(6): the RED gradient H^T(Hx - y)/sigma^2 + lambda (x - f(x)) vanishes at the
    reported fixed point."""
    op, res = small_solution
    g0 = np.linalg.norm(op.gradient(op.x0()))
    for m, r in res.items():
        assert np.linalg.norm(op.gradient(r.x)) <= 1e-6 * g0, m


def test_fp_mpe_rre_agree_and_ve_needs_fewer_calls(orc, small_solution):
    """The fixed point is unique (contraction, Sec. II-B); VE changes the path, not the
    answer, and reaches it with fewer FP calls (Sec. IV)."""
    op, res = small_solution
    ref = res["none"].x
    for m in ("rre", "mpe"):
        assert np.linalg.norm(res[m].x - ref) <= 1e-6 * np.linalg.norm(ref)
        assert res[m].calls < res["none"].calls


def test_fp_contraction(orc, small_solution):
    """The FP map is a contraction at x*: rho([H^T H/sigma^2 + lambda I]^-1 lambda grad f) < 1,
    estimated by power iteration on finite-difference products of the FP map."""
    op, res = small_solution
    x = res["none"].x
    v = np.random.default_rng(8).standard_normal(x.shape)
    # CG with many iterations approximates the exact inverse
    op.n_cg = 200
    est = 0.0
    for _ in range(25):
        v /= np.linalg.norm(v)
        jv = (op.fp(x + 1e-3 * v) - op.fp(x - 1e-3 * v)) / 2e-3
        est = np.linalg.norm(jv)
        v = jv
    op.n_cg = 15
    assert est < 1.0


def test_identity_denoiser_gives_least_squares(orc):
    """With D = identity the FP iteration is linear with fixed point H^T H x = H^T y: the
    least-squares solution of a dense 8x8 deblurring problem. The 3x3 PSF has |h_hat| >= 0.2,
    so the iteration contracts by at most lambda / (0.04 / sigma^2 + lambda) = 1/3 per call."""
    psf = np.full((3, 3), 0.05)
    psf[1, 1] = 0.6
    P = W.Problem("ls", RNG.uniform(0, 255, (8, 8)), psf, 1, 1.0, 0.02,
                  RNG.standard_normal((8, 8)), 64, W.identity_denoiser())
    op = orc.OracleProblem(P)
    Hd = _dense(lambda p: orc.blur(p, op.psf), (8, 8))
    xs = np.linalg.solve(Hd.T @ Hd, Hd.T @ op.y.ravel()).reshape(8, 8)
    r = orc.solve(op, "none", tol=0.0, max_calls=80)
    assert np.linalg.norm(r.x - xs) <= 1e-10 * np.linalg.norm(xs)
    r2 = orc.solve(op, "rre", L=6, m=0, tol=0.0, max_calls=30)
    assert np.linalg.norm(r2.x - xs) <= 1e-9 * np.linalg.norm(xs)


# ------------------------------------------------------------------ steepest descent (Sec. IV)


def test_sd_map_fixes_the_fp_fixed_point(orc, small_solution):
    """The SD step x - mu g(x) with g of eq. (5) leaves the FP fixed point in place (g(x*) = 0,
    eq. (6)): FP and SD share x*."""
    op, res = small_solution
    x = res["rre"].x
    sd = orc.SDMap(op)
    assert np.linalg.norm(sd.fp(x) - x) <= 1e-6 * np.linalg.norm(x)


@pytest.mark.parametrize("method", ["mpe", "rre"])
def test_sd_ve_reaches_the_fp_fixed_point(orc, small_solution, method):
    """SD-MPE / SD-RRE (Algorithm 3 with the SD step as the base iteration, kappa = 8, i.e.
    L = 9 difference columns; Sec. IV) converge to the same x* as FP, in a few hundred calls
    (plain SD needs thousands on this problem)."""
    op, res = small_solution
    ref = res["none"].x
    r = orc.solve(orc.SDMap(op), method, L=9, m=0, tol=1e-10, max_calls=400)
    assert r.calls < 400
    assert np.linalg.norm(r.x - ref) <= 1e-7 * np.linalg.norm(ref)


def test_sd_identity_denoiser_gives_least_squares(orc):
    """With D = identity, SD with the default step 1/L, L = ||H||^2/sigma^2 + 2 lambda, is
    gradient descent on ||Hx - y||^2 / (2 sigma^2): it converges to the least-squares solution
    of a dense 8x8 problem (|h_hat| >= 0.2, rate 1 - mu 0.04 / sigma^2 = 0.96 per call). A step
    of the wrong sign, or beyond 2 / L, diverges instead."""
    psf = np.full((3, 3), 0.05)
    psf[1, 1] = 0.6
    P = W.Problem("ls", RNG.uniform(0, 255, (8, 8)), psf, 1, 1.0, 0.02,
                  RNG.standard_normal((8, 8)), 64, W.identity_denoiser())
    op = orc.OracleProblem(P)
    Hd = _dense(lambda p: orc.blur(p, op.psf), (8, 8))
    xs = np.linalg.solve(Hd.T @ Hd, Hd.T @ op.y.ravel()).reshape(8, 8)
    sd = orc.SDMap(op)
    assert abs(sd.mu - 1.0 / (1.0 + 0.04)) < 1e-15
    r = orc.solve(sd, "none", tol=0.0, max_calls=800)
    assert np.linalg.norm(r.x - xs) <= 1e-9 * np.linalg.norm(xs)


# ------------------------------------------------------------------ the objective (eq. (4))


def test_objective_identity_denoiser_is_least_squares(orc):
    """With D = identity the prior x^T (x - f(x)) vanishes and E(x) = ||Hx - y||^2 / (2 sigma^2),
    computed here with a dense H; a central finite difference of E along a random direction
    matches the gradient of eq. (5) (the data term's gradient H^T (Hx - y) / sigma^2)."""
    psf = W.psf_gaussian(5, 1.0)
    P = W.Problem("obj", RNG.uniform(0, 255, (8, 10)), psf, 1, 1.7, 0.02,
                  RNG.standard_normal((8, 10)), 15, W.identity_denoiser())
    op = orc.OracleProblem(P)
    Hd = _dense(lambda p: orc.blur(p, op.psf), (8, 10))
    x = RNG.uniform(0, 255, (8, 10))
    r = Hd @ x.ravel() - op.y.ravel()
    assert abs(op.objective(x) - r @ r / (2 * 1.7 ** 2)) <= 1e-12 * abs(op.objective(x))
    v = RNG.standard_normal((8, 10))
    fd = (op.objective(x + 1e-3 * v) - op.objective(x - 1e-3 * v)) / 2e-3
    assert abs(fd - (op.gradient(x).ravel() @ v.ravel())) <= 1e-7 * abs(fd)


def test_objective_prior_vanishes_on_constants(orc):
    """D(c 1) = c 1 (zero-mean filters, odd phi), so the RED prior of a constant image is 0 and
    E reduces to the data term; for a textured image the prior term is positive here."""
    P = W.problem("tiny")
    op = orc.OracleProblem(P)
    c = np.full(P.hr_shape, 87.5)
    r = orc.apply_H(c, op.psf, op.s) - op.y
    assert abs(op.objective(c) - r.ravel() @ r.ravel() / (2 * op.sigma ** 2)) <= 1e-9 * op.objective(c)
    x = op.x0()
    prior = 0.5 * op.lam * (x.ravel() @ (x - op.denoise(x)).ravel())
    assert prior > 0


@pytest.mark.parametrize("s", [1, 3])
def test_objective_closed_form_one_stage_denoiser(orc, s):
    """Eq. (4) with the data term of eq. (1): E(x) = ||Hx - y||^2 / (2 sigma^2) +
    (lambda / 2) x^T (x - f(x)). With one stage and f's reaction input equal to x,
    x - f(x) = sum_i K_i^T phi_i(K_i x), so the prior is (lambda / 2) sum_i <K_i x, phi_i(K_i x)>:
    built here from scipy reflect correlation and direct Gaussian sums, with H x from an FFT
    circular convolution (decimated for s = 3). A prior weight of lambda instead of lambda / 2
    (or a missing 1/2 on the data term) is off by far more than the tolerance."""
    full = W.make_denoiser()
    d1 = W.DenoiserParams(1, full.nfilt, full.ksize, full.nrbf, full.mu0, full.dmu, full.gamma,
                          full.filters[:1], full.rbf_w[:1], full.react[:1])
    shape = (12, 13)
    psf = W.psf_gaussian(7, 1.6)
    sigma, lam = 1.7, 0.05
    P = W.Problem("obj1", W.make_image(*shape, 1031), psf, s, sigma, lam,
                  W.make_noise(W.lr_shape(*shape, s), 2031), 15, d1)
    op = orc.OracleProblem(P)
    x = W.make_image(*shape, 1032)
    hx = np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(_psf_pad(psf, shape))))[::s, ::s]
    data = float(((hx - op.y) ** 2).sum()) / (2 * sigma ** 2)
    mu = d1.mu0 + d1.dmu * np.arange(d1.nrbf)
    zphi = 0.0
    for i in range(d1.nfilt):
        z = ndi.correlate(x, d1.filters[0, i], mode="reflect").ravel()
        phi = (d1.rbf_w[0, i][None, :] * np.exp(-(z[:, None] - mu[None, :]) ** 2
                                                 / (2 * d1.gamma ** 2))).sum(1)
        zphi += float(z @ phi)
    prior = 0.5 * lam * zphi
    assert prior > 1e-3 * data
    E = op.objective(x)
    assert abs(E - (data + prior)) <= 1e-10 * abs(data + prior)


# ------------------------------------------------------------------ exact linear step (footnote to eq. (7))


def test_exact_fp_map_is_cg_to_convergence(orc):
    """The Fourier-diagonal FP map equals the CG FP map with CG run to convergence (300
    iterations on a 24x20 problem), for a non-symmetric PSF (the DFT convention of `blur`)."""
    psf = np.random.default_rng(11).uniform(0, 1, (5, 3))
    psf /= psf.sum()
    P = W.Problem("ex", W.make_image(24, 20, 1020), psf, 1, W.SQRT2, 0.02,
                  W.make_noise((24, 20), 2020), 300, W.make_denoiser())
    op = orc.OracleProblem(P)
    ex = orc.ExactFPMap(op)
    x = op.x0()
    for _ in range(3):
        a, b = ex.fp(x), op.fp(x)
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
        x = a


def test_exact_fp_shares_the_fixed_point(orc, small_solution):
    """The exact-solve FP iteration (with RRE) converges to the same x* as truncated-CG FP."""
    op, res = small_solution
    r = orc.solve(orc.ExactFPMap(op), "rre", L=5, m=0, tol=1e-11, max_calls=200)
    assert np.linalg.norm(r.x - res["none"].x) <= 1e-7 * np.linalg.norm(res["none"].x)
