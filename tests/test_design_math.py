"""CPU checks of the algebra the GPU kernels rely on (no GPU needed).

These restate, in numpy, identities the HIP kernels use in place of the oracle's literal
steps, and check them against the oracle's plain definitions.
"""
import math

import numpy as np
import pytest

import workload as W


def _window_recurrence(z, w, mu0, dmu, gamma, K):
    """The denoiser kernel's influence-function evaluation, in float64: nearest centre j0, one
    exp, then term(k+1) = term(k) R_k, R_{k+1} = R_k B^2 on both sides, |k| <= K."""
    J = len(w)
    c = math.log2(math.e) / (2 * gamma * gamma)
    j0 = int(np.clip(np.rint((z - mu0) / dmu), 0, J - 1))
    d0 = z - (mu0 + dmu * j0)
    if abs(d0) > (K + 0.5) * dmu:
        return 0.0
    g0 = 2.0 ** (-c * d0 * d0)
    a, ai, b = 2.0 ** (2 * c * dmu * d0), 2.0 ** (-2 * c * dmu * d0), 2.0 ** (-c * dmu * dmu)
    wp = lambda j: w[j] if 0 <= j < J else 0.0  # noqa: E731
    acc = wp(j0) * g0
    gu, ru, gd, rd = g0, a * b, g0, ai * b
    for k in range(1, K + 1):
        gu *= ru
        ru *= b * b
        gd *= rd
        rd *= b * b
        acc += wp(j0 + k) * gu + wp(j0 - k) * gd
    return acc


def test_rbf_window_recurrence_matches_full_sum(orc):
    """Seven centres either side (gamma = dmu) reproduce the 63-term sum to 1e-12 of the
    largest weight, over and beyond the centre range."""
    d = W.make_denoiser()
    z = np.concatenate([np.linspace(-420, 420, 1201), [0.0, 5.0, -5.0, 305.0, 315.0]])
    K = max(1, math.ceil(7.4338 * d.gamma / d.dmu - 0.5))
    assert K == 7
    for t, i in [(0, 0), (1, 7), (3, 19), (4, 23)]:
        w = d.rbf_w[t, i]
        full = orc.phi(z, w, d.mu0, d.dmu, d.gamma)
        win = np.array([_window_recurrence(v, w, d.mu0, d.dmu, d.gamma, K) for v in z])
        assert np.abs(win - full).max() <= 1e-12 * np.abs(w).max()


def _window_horner(z, w, mu0, dmu, gamma, K):
    """The denoiser kernel's evaluation with a compile-time window, in float64, branch-free:
    j0 = the nearest centre clamped to -K .. J-1+K (the weight row is zero-padded by 2K), d0 =
    z - mu_j0 clamped to [-dmu, dmu], then phi = G0 A^-K sum_{m=0}^{2K} c_|m-K| w[j0+m-K] A^m
    by Horner in A, with A = exp2(2 c dmu d0), c_k = exp2(-c dmu^2 k^2) and the prefactor
    G0 A^-K one exp2."""
    J = len(w)
    c = math.log2(math.e) / (2 * gamma * gamma)
    t = (z - mu0) / dmu
    j0 = int(min(max(np.rint(t) if np.isfinite(t) else (np.inf if t > 0 else -np.inf), -K),
                 J - 1 + K))
    d0 = min(max(z - (mu0 + dmu * j0), -dmu), dmu)
    wp = lambda j: w[j] if 0 <= j < J else 0.0  # noqa: E731
    ck = [2.0 ** (-c * dmu * dmu * k * k) for k in range(K + 1)]
    a = 2.0 ** (2 * c * dmu * d0)
    pre = 2.0 ** (-c * d0 * d0 - K * 2 * c * dmu * d0)
    poly = ck[K] * wp(j0 + K)
    for m in range(2 * K - 1, -1, -1):
        poly = poly * a + ck[abs(m - K)] * wp(j0 + m - K)
    return pre * poly


@pytest.mark.parametrize("K,eps", [(7, 1e-12), (5, 1e-6)])
def test_rbf_window_horner_matches_full_sum(orc, K, eps):
    """The branch-free Horner arrangement of the window reproduces the 63-term sum to eps of
    the largest weight for every z: inside the centre range, past it (where the clamped j0 and
    the zero padding take the last weights), far beyond it (where the d0 clamp binds) and at
    infinity. K = 7 is the FP32 form's window (eps 1e-12), K = 5 the BF16 form's (1e-6)."""
    d = W.make_denoiser()
    far = [1e4, -1e4, 3e38, -3e38]
    z = np.concatenate([np.linspace(-420, 420, 1201), [0.0, 5.0, -5.0, 4.999, 305.0, 315.0],
                        d.mu0 + d.dmu * (np.arange(-12, 75) + 0.5)])
    for t, i in [(0, 0), (1, 7), (3, 19), (4, 23)]:
        w = d.rbf_w[t, i]
        full = orc.phi(z, w, d.mu0, d.dmu, d.gamma)
        hor = np.array([_window_horner(v, w, d.mu0, d.dmu, d.gamma, K) for v in z])
        assert np.abs(hor - full).max() <= eps * np.abs(w).max()
        tail = np.array([_window_horner(v, w, d.mu0, d.dmu, d.gamma, K) for v in far])
        assert np.all(np.isfinite(tail)) and np.abs(tail).max() <= eps * np.abs(w).max()
        inf = [_window_horner(v, w, d.mu0, d.dmu, d.gamma, K) for v in (np.inf, -np.inf)]
        assert all(np.isfinite(v) and abs(v) <= eps * np.abs(w).max() for v in inf)
    # a mistake in the coefficient order (c_k paired with the wrong weight) is caught
    w = d.rbf_w[2, 5]
    bad = 0.0
    for v in (3.0, 47.0, -118.0):
        j0 = int(np.rint((v - d.mu0) / d.dmu))
        d0 = v - (d.mu0 + d.dmu * j0)
        c = math.log2(math.e) / (2 * d.gamma ** 2)
        a = 2.0 ** (2 * c * d.dmu * d0)
        pre = 2.0 ** (-c * d0 * d0 - K * 2 * c * d.dmu * d0)
        poly = 0.0
        for m in range(2 * K, -1, -1):
            poly = poly * a + 2.0 ** (-c * d.dmu ** 2 * (m - K) ** 2) * w[j0 - (m - K)]
        bad = max(bad, abs(pre * poly - orc.phi(np.array([v]), w, d.mu0, d.dmu, d.gamma)[0]))
    assert bad > 1e-3 * np.abs(w).max()


def _hermite_table(w, mu0, dmu, gamma):
    """The BF16 stage's influence-function table, in numpy: knots z_k = lo + k h (h = gamma / 2,
    lo = mu0 - 5.2565 gamma, up to the last centre + 5.2565 gamma), phi and h phi' from the full
    sum, and per interval the cubic (a0, a1, a2, a3) in u of the Hermite interpolant, rounded to
    float32 as stored."""
    J = len(w)
    h = 0.5 * gamma
    lo = mu0 - 5.2565 * gamma
    n = math.ceil(((J - 1) * dmu + 2 * 5.2565 * gamma) / h)
    zk = lo + h * np.arange(n + 1)
    e = zk[:, None] - (mu0 + dmu * np.arange(J))[None, :]
    g = w[None, :] * np.exp(-e * e / (2 * gamma * gamma))
    v = g.sum(1)
    dv = (-(e / gamma ** 2) * g).sum(1) * h
    a0, a1 = v[:-1], dv[:-1]
    a2 = 3 * (v[1:] - v[:-1]) - 2 * dv[:-1] - dv[1:]
    a3 = 2 * (v[:-1] - v[1:]) + dv[:-1] + dv[1:]
    return np.stack([a0, a1, a2, a3], 1).astype(np.float32), lo, h, n


def _table_eval(z, tab, lo, h, n):
    """The kernel's lookup in float32: t = z / h - lo / h, k = clamp(floor t), u = t - floor t."""
    z = np.asarray(z, np.float32)
    t = z * np.float32(1.0 / h) + np.float32(-lo / h)
    tf = np.floor(t)
    k = np.clip(tf, 0, n - 1).astype(np.int64)
    u = (t - tf).astype(np.float64)
    c = tab[k].astype(np.float64)
    return ((c[:, 3] * u + c[:, 2]) * u + c[:, 1]) * u + c[:, 0]


@pytest.mark.parametrize("ratio", [1.0 / 3.0, 1.0, 2.2])
def test_rbf_table_within_hermite_bound(orc, ratio):
    """The tabulated influence function is within the cubic Hermite bound h^4 / 384 max |phi^(4)|
    of the 63-term sum (plus the tails beyond the table, below 1e-6 of the weights, and float32
    rounding), over and beyond the centre range, for gamma / dmu from 1/3 to 2.2; at
    gamma = dmu the error is below 1e-3 of the largest weight, under the BF16 operands'
    3.9e-3."""
    d = W.make_denoiser()
    gamma = ratio * d.dmu
    mu = d.mu0 + d.dmu * np.arange(d.nrbf)
    z = np.concatenate([np.linspace(mu[0] - 12 * gamma - 40, mu[-1] + 12 * gamma + 40, 4001),
                        mu, mu + 0.5 * d.dmu])
    for t, i in [(0, 0), (2, 11), (4, 23)]:
        w = d.rbf_w[t, i]
        tab, lo, h, n = _hermite_table(w, d.mu0, d.dmu, gamma)
        appx = _table_eval(z, tab, lo, h, n)
        full = orc.phi(z, w, d.mu0, d.dmu, gamma)
        e = z[:, None] - mu[None, :]
        g4 = ((e ** 4 / gamma ** 8 - 6 * e ** 2 / gamma ** 6 + 3 / gamma ** 4)
              * np.abs(w)[None, :] * np.exp(-e * e / (2 * gamma * gamma))).sum(1)
        bound = h ** 4 / 384 * g4.max() + 1e-6 * np.abs(w).sum() + 1e-6 * np.abs(full).max()
        err = np.abs(appx - full).max()
        assert err <= bound, (ratio, t, i, err, bound)
        if ratio == 1.0:
            assert err <= 1e-3 * np.abs(w).max()
    # a wrong cubic (a2 and a3 of each other's form) is caught
    w = d.rbf_w[1, 3]
    tab, lo, h, n = _hermite_table(w, d.mu0, d.dmu, d.dmu)
    tab[:, [2, 3]] = tab[:, [3, 2]]
    bad = np.abs(_table_eval(z, tab, lo, h, n) - orc.phi(z, w, d.mu0, d.dmu, d.dmu)).max()
    assert bad > 1e-2 * np.abs(w).max()


def test_correction_form_cg_equals_warm_start(orc):
    """CG on A d = rhs - A x0 from d = 0, then x0 + d, gives the warm-started CG iterate."""
    psf = W.psf_uniform(9)
    rng = np.random.default_rng(0)
    x0 = rng.uniform(0, 255, (16, 16))
    rhs = rng.uniform(0, 100, (16, 16))
    r0 = rhs - orc.apply_A(x0, psf, 1, math.sqrt(2), 0.02)
    for n in (1, 5, 15):
        d = orc.cg(r0, np.zeros_like(x0), psf, 1, math.sqrt(2), 0.02, n)
        x = orc.cg(rhs, x0, psf, 1, math.sqrt(2), 0.02, n)
        assert np.allclose(x0 + d, x, rtol=0, atol=1e-9 * np.abs(x).max())


def test_residual_form_of_fp_rhs(orc):
    """rhs - A x = H^T (y - H x) / sigma^2 + lambda (f(x) - x) for the right-hand side of eq. (7)."""
    prob = W.problem("tiny")
    op = orc.OracleProblem(prob)
    x = op.y + 3.0
    fx = op.denoise(x)
    lhs = (op.b0 + op.lam * fx) - orc.apply_A(x, op.psf, op.s, op.sigma, op.lam)
    rhs = (orc.apply_Ht(op.y - orc.apply_H(x, op.psf, op.s), op.shape, op.psf, op.s)
           / op.sigma ** 2 + op.lam * (fx - x))
    assert np.allclose(lhs, rhs, atol=1e-10 * np.abs(op.b0).max())


def test_gram_route_extrapolation_equals_mgs_route(orc):
    """x_m + U_{k-1} xi (the GPU's combine, with R from chol(U^T U)) equals Algorithm 1's
    x_m + Q_{k-1} R_{k-1} xi with Q, R from modified Gram-Schmidt."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((200, 6)).cumsum(axis=1)
    U = X[:, 1:] - X[:, :-1]
    Q, R = orc.mgs(U)
    Rc = np.linalg.cholesky(U.T @ U).T
    for gfun in (orc.mpe_gamma, orc.rre_gamma, orc.svd_mpe_gamma):
        g = gfun(Rc)
        k = len(g) - 1
        xi = 1.0 - np.cumsum(g)[:k]
        via_u = X[:, 0] + U[:, :k] @ xi
        assert np.allclose(via_u, orc.extrapolate(X[:, 0], Q, R, gfun(R)), atol=1e-9)
