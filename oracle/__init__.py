"""FP64 CPU oracle for RED + vector extrapolation (TEST INFRASTRUCTURE ONLY).

A plain, slow, obviously correct reference of the method of Hong, Romano and Elad,
"Acceleration of RED via Vector Extrapolation":

* operators, denoiser, CG and one FP call (Sec. II, eq. (7)) are plain C in red_oracle.c,
  called through ctypes;
* vector extrapolation is numpy, written step by step from Sec. III: MGS QR (Algorithm 2),
  MPE (Algorithm 1, eq. (18)), RRE (eq. (19)), SVD-MPE (Sec. III-B), and the full-cycling
  driver (Algorithm 3) with the termination of Sec. III-C.

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this package; the
GPU library never does, and the two share no code. Everything is float64.

Readings where the paper is silent (see the design notes for the list): initial vector
x0 = y for deblurring and s^2 H^T y for s-fold super-resolution; CG warm-started at x_k with a
fixed iteration count; termination on the relative change of consecutive FP iterates;
MPE/RRE breakdown thresholds below.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "red_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile red_oracle.c with gcc (-O2, OpenMP over independent outer loops)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        d = ctypes.c_double
        sig = {
            "orc_blur": [dp, i, i, dp, i, i, dp],
            "orc_blur_adj": [dp, i, i, dp, i, i, dp],
            "orc_decimate": [dp, i, i, i, dp],
            "orc_decimate_adj": [dp, i, i, i, dp],
            "orc_apply_H": [dp, i, i, dp, i, i, i, dp],
            "orc_apply_Ht": [dp, i, i, dp, i, i, i, dp],
            "orc_apply_A": [dp, i, i, dp, i, i, i, d, d, dp],
            "orc_cg": [dp, dp, i, i, dp, i, i, i, d, d, i],
            "orc_filter_fwd": [dp, i, i, dp, i, dp],
            "orc_filter_adj": [dp, i, i, dp, i, dp],
            "orc_phi": [d, dp, i, d, d, d],
            "orc_tnrd_stage": [dp, dp, i, i, ctypes.c_void_p, i, dp],
            "orc_denoise": [dp, i, i, ctypes.c_void_p, dp],
            "orc_fp_step": [dp, dp, i, i, dp, i, i, i, d, d, i, ctypes.c_void_p, dp],
            "orc_num_threads": [],
            "orc_set_num_threads": [i],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None
        L.orc_phi.restype = ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _Tnrd(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int), ("nfilt", ctypes.c_int), ("ksize", ctypes.c_int),
                ("nrbf", ctypes.c_int), ("mu0", ctypes.c_double), ("dmu", ctypes.c_double),
                ("gamma", ctypes.c_double), ("filters", ctypes.POINTER(ctypes.c_double)),
                ("rbf_w", ctypes.POINTER(ctypes.c_double)),
                ("react", ctypes.POINTER(ctypes.c_double))]


class Denoiser:
    """Holds the FP64 parameter arrays alive for the C struct."""

    def __init__(self, params):
        self.params = params
        self.filters = _f64(params.filters)
        self.rbf_w = _f64(params.rbf_w)
        self.react = _f64(params.react)
        if self.filters.size == 0:
            self.filters = np.zeros(1)
            self.rbf_w = np.zeros(1)
            self.react = np.zeros(1)
        self.struct = _Tnrd(params.stages, params.nfilt, params.ksize, params.nrbf,
                            params.mu0, params.dmu, params.gamma, _p(self.filters),
                            _p(self.rbf_w), _p(self.react))

    @property
    def ptr(self):
        return ctypes.cast(ctypes.pointer(self.struct), ctypes.c_void_p)


# ---------------------------------------------------------------------------------------
# Operator wrappers (Sec. II-A, eq. (1); Sec. II-B, eq. (7))
# ---------------------------------------------------------------------------------------


def blur(x, psf):
    x, psf = _f64(x), _f64(psf)
    out = np.empty_like(x)
    lib().orc_blur(_p(x), x.shape[0], x.shape[1], _p(psf), psf.shape[0], psf.shape[1], _p(out))
    return out


def blur_adj(z, psf):
    z, psf = _f64(z), _f64(psf)
    out = np.empty_like(z)
    lib().orc_blur_adj(_p(z), z.shape[0], z.shape[1], _p(psf), psf.shape[0], psf.shape[1],
                       _p(out))
    return out


def lr_shape(H, W, s):
    return ((H + s - 1) // s, (W + s - 1) // s)


def decimate(x, s):
    x = _f64(x)
    out = np.empty(lr_shape(*x.shape, s))
    lib().orc_decimate(_p(x), x.shape[0], x.shape[1], s, _p(out))
    return out


def decimate_adj(y, shape, s):
    y = _f64(y)
    assert y.shape == lr_shape(*shape, s)
    out = np.empty(shape)
    lib().orc_decimate_adj(_p(y), shape[0], shape[1], s, _p(out))
    return out


def apply_H(x, psf, s):
    x, psf = _f64(x), _f64(psf)
    out = np.empty(lr_shape(*x.shape, s))
    lib().orc_apply_H(_p(x), x.shape[0], x.shape[1], _p(psf), psf.shape[0], psf.shape[1], s,
                      _p(out))
    return out


def apply_Ht(y, shape, psf, s):
    y, psf = _f64(y), _f64(psf)
    assert y.shape == lr_shape(*shape, s)
    out = np.empty(shape)
    lib().orc_apply_Ht(_p(y), shape[0], shape[1], _p(psf), psf.shape[0], psf.shape[1], s,
                       _p(out))
    return out


def apply_A(p, psf, s, sigma, lam):
    p, psf = _f64(p), _f64(psf)
    out = np.empty_like(p)
    lib().orc_apply_A(_p(p), p.shape[0], p.shape[1], _p(psf), psf.shape[0], psf.shape[1], s,
                      float(sigma), float(lam), _p(out))
    return out


def cg(rhs, x0, psf, s, sigma, lam, n_iter):
    rhs, psf = _f64(rhs), _f64(psf)
    x = _f64(x0).copy()
    lib().orc_cg(_p(rhs), _p(x), x.shape[0], x.shape[1], _p(psf), psf.shape[0], psf.shape[1],
                 s, float(sigma), float(lam), int(n_iter))
    return x


def filter_fwd(u, k):
    u, k = _f64(u), _f64(k)
    out = np.empty_like(u)
    lib().orc_filter_fwd(_p(u), u.shape[0], u.shape[1], _p(k), k.shape[0], _p(out))
    return out


def filter_adj(v, k):
    v, k = _f64(v), _f64(k)
    out = np.empty_like(v)
    lib().orc_filter_adj(_p(v), v.shape[0], v.shape[1], _p(k), k.shape[0], _p(out))
    return out


def phi(z, w, mu0=-310.0, dmu=10.0, gamma=10.0):
    w = _f64(w)
    f = lib().orc_phi
    return np.array([f(float(v), _p(w), w.size, mu0, dmu, gamma) for v in np.ravel(z)]).reshape(
        np.shape(z))


def tnrd_stage(u, f, den: Denoiser, t):
    u, f = _f64(u), _f64(f)
    out = np.empty_like(u)
    lib().orc_tnrd_stage(_p(u), _p(f), u.shape[0], u.shape[1], den.ptr, int(t), _p(out))
    return out


def denoise(x, den: Denoiser):
    x = _f64(x)
    out = np.empty_like(x)
    lib().orc_denoise(_p(x), x.shape[0], x.shape[1], den.ptr, _p(out))
    return out


def psnr(x, x_true):
    """10 log10(255^2 / MSE) over all pixels, no clipping or border crop."""
    mse = np.mean((np.asarray(x, np.float64) - np.asarray(x_true, np.float64)) ** 2)
    return float(10.0 * np.log10(255.0 ** 2 / mse)) if mse > 0 else float("inf")


# ---------------------------------------------------------------------------------------
# Problem: y = H x_true + sigma n (eq. (1)) and the FP map of eq. (7)
# ---------------------------------------------------------------------------------------


class OracleProblem:
    """The FP map x -> CG_{n_cg}(A, b0 + lambda D(x); x) of eq. (7) for one observation."""

    def __init__(self, prob, y=None):
        self.prob = prob
        self.psf = _f64(prob.psf)
        self.s = int(prob.decim)
        self.sigma = float(prob.sigma)
        self.lam = float(prob.lam)
        self.n_cg = int(prob.cg_iters)
        self.den = Denoiser(prob.denoiser)
        self.x_true = _f64(prob.x_true)
        self.shape = self.x_true.shape
        if y is None:
            y = apply_H(self.x_true, self.psf, self.s) + self.sigma * _f64(prob.noise)
        self.y = _f64(y)
        self.b0 = apply_Ht(self.y, self.shape, self.psf, self.s) / (self.sigma ** 2)
        self.calls = 0

    def x0(self):
        """Initial vector (the paper leaves it open): y for deblurring, s^2 H^T y for SR."""
        if self.s == 1:
            return self.y.copy()
        return float(self.s * self.s) * apply_Ht(self.y, self.shape, self.psf, self.s)

    def fp(self, x):
        x = _f64(x)
        out = np.empty_like(x)
        H, W = x.shape
        lib().orc_fp_step(_p(x), _p(self.b0), H, W, _p(self.psf), self.psf.shape[0],
                          self.psf.shape[1], self.s, self.sigma, self.lam, self.n_cg,
                          self.den.ptr, _p(out))
        self.calls += 1
        return out

    def denoise(self, x):
        return denoise(x, self.den)

    def objective(self, x):
        """E(x) = ||Hx - y||^2 / (2 sigma^2) + (lambda/2) x^T (x - f(x)), eq. (4)."""
        r = apply_H(x, self.psf, self.s) - self.y
        return float(r.ravel() @ r.ravel() / (2 * self.sigma ** 2)
                     + 0.5 * self.lam * (x.ravel() @ (x - self.denoise(x)).ravel()))

    def gradient(self, x):
        """H^T (Hx - y) / sigma^2 + lambda (x - f(x)), eq. (5) with eq. (1)."""
        r = apply_H(x, self.psf, self.s) - self.y
        return apply_Ht(r, self.shape, self.psf, self.s) / self.sigma ** 2 + self.lam * (
            x - self.denoise(x))

    def sd_step_size(self):
        """Default fixed step of steepest descent (Sec. IV fixes it by hand): 1 / L with
        L = ||H||^2 / sigma^2 + 2 lambda, a Lipschitz constant of grad E when the denoiser is
        strongly passive (rho(grad f) <= 1, Sec. II-B); ||H|| <= sum |h|."""
        nh = float(np.abs(self.psf).sum())
        return 1.0 / (nh * nh / self.sigma ** 2 + 2.0 * self.lam)

    def sd(self, x, mu):
        """One steepest-descent step x - mu grad E(x) (the gradient of eq. (5)); one denoiser
        call."""
        self.calls += 1
        return _f64(x) - mu * self.gradient(_f64(x))


class ExactFPMap:
    """The FP map of eq. (7) with the inverse applied exactly, for periodic deblurring (s = 1):
    A = H^T H / sigma^2 + lambda I is diagonalised by the 2-D DFT (the footnote to eq. (7)), so
    x_{k+1} = F^-1[ F(b0 + lambda f(x_k)) / (|h_hat|^2 / sigma^2 + lambda) ]. h_hat is the DFT of
    the PSF placed with its centre at the origin (circular convolution, as `blur`)."""

    def __init__(self, op: OracleProblem):
        if op.s != 1:
            raise ValueError("the exact Fourier solve needs s = 1 (deblurring)")
        self.op, self.shape = op, op.shape
        H, W = op.shape
        kh, kw = op.psf.shape
        h = np.zeros((H, W))
        for a in range(kh):
            for b in range(kw):
                h[(a - kh // 2) % H, (b - kw // 2) % W] += op.psf[a, b]
        self.den = np.abs(np.fft.fft2(h)) ** 2 / op.sigma ** 2 + op.lam

    def x0(self):
        return self.op.x0()

    def fp(self, x):
        self.op.calls += 1
        rhs = self.op.b0 + self.op.lam * self.op.denoise(_f64(x))
        return np.real(np.fft.ifft2(np.fft.fft2(rhs) / self.den))


class SDMap:
    """Steepest descent with a fixed step as the base iteration of Algorithm 3 (SD, and
    SD-MPE / SD-RRE with extrapolation; Sec. IV): fp(x) = x - mu grad E(x). Its fixed point is
    the stationary point of E, the same x* as the FP map's."""

    def __init__(self, op: OracleProblem, mu=None):
        self.op = op
        self.mu = op.sd_step_size() if mu is None else float(mu)
        self.shape = op.shape

    def x0(self):
        return self.op.x0()

    def fp(self, x):
        return self.op.sd(x, self.mu)


# ---------------------------------------------------------------------------------------
# Vector extrapolation (Sec. III-B)
# ---------------------------------------------------------------------------------------

# Breakdown thresholds (the paper only says MPE and SVD-MPE may not exist, Sec. III-B).
RANK_EPS = 1e-13   # R_jj <= RANK_EPS * R_00 counts as a rank-deficient column
SUM_EPS = 1e-12    # |sum c| <= SUM_EPS * ||c||_1 counts as a vanishing normaliser
# Stability guard (reading of Sec. III-D, eq. (21)): coefficients with sum |gamma| above a cap,
# or not finite, are rejected and the cycle continues from its last FP iterate. The default cap
# is infinite, so only non-finite coefficients are rejected: the paper rejects none, and windows
# with sum |gamma| near 1e8 still accelerate steepest descent here. Callers may set a finite cap.
GAMMA_CAP = float("inf")


def mgs(U):
    """Algorithm 2: modified Gram-Schmidt QR of U (N x (kappa+1)). Returns Q, R with
    r_ji = q_j^T u_i^(j), u_i^(j+1) = u_i^(j) - r_ji q_j, r_ii = ||u_i^(i)||, q_i = u_i^(i)/r_ii.
    A zero column gives r_ii = 0 and q_i = 0."""
    U = np.array(U, dtype=np.float64)
    N, k1 = U.shape
    Q = np.zeros_like(U)
    R = np.zeros((k1, k1))
    for i in range(k1):
        ui = U[:, i].copy()
        for j in range(i):
            R[j, i] = Q[:, j] @ ui
            ui = ui - R[j, i] * Q[:, j]
        R[i, i] = np.sqrt(ui @ ui)
        Q[:, i] = ui / R[i, i] if R[i, i] > 0 else 0.0
    return Q, R


def _back_sub(R, b):
    """Solve the upper-triangular system R x = b by back substitution."""
    n = len(b)
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (b[i] - R[i, i + 1:n] @ x[i + 1:n]) / R[i, i]
    return x


def _fwd_sub_transposed(R, b):
    """Solve R^T x = b (R upper triangular) by forward substitution."""
    n = len(b)
    x = np.zeros(n)
    for i in range(n):
        x[i] = (b[i] - R[0:i, i] @ x[0:i]) / R[i, i]
    return x


def _full_rank(R, k):
    """First k diagonal entries of R are above the rank threshold."""
    if k == 0:
        return True
    d = np.abs(np.diag(R)[:k])
    return R[0, 0] > 0 and bool(np.all(d > RANK_EPS * R[0, 0]))


def mpe_gamma(R):
    """Algorithm 1, step 2: R_{kappa-1} c' = -r_{kappa+1}, c = (c', 1), gamma = c / sum c.
    Returns None when MPE does not exist (singular R_{kappa-1} or sum c ~ 0)."""
    k = R.shape[0] - 1
    if not _full_rank(R, k):
        return None
    cp = _back_sub(R[:k, :k], -R[:k, k]) if k > 0 else np.zeros(0)
    c = np.concatenate([cp, [1.0]])
    s = c.sum()
    if abs(s) <= SUM_EPS * np.abs(c).sum():
        return None
    return c / s


def rre_gamma(R):
    """RRE (eq. (19)): R^T R d = 1 by forward then backward substitution, gamma = d / sum d.
    If the last column is dependent on the others, ||U gamma|| = 0 is reached by MPE's null
    vector, so gamma_RRE = gamma_MPE; if that does not exist either, drop the last column
    (RRE with kappa-1; the relation of Sec. III-B between RRE_kappa and RRE_{kappa-1})."""
    k = R.shape[0] - 1
    if _full_rank(R, k + 1):
        d = _back_sub(R, _fwd_sub_transposed(R, np.ones(k + 1)))
        return d / d.sum()
    if k >= 1:
        g = mpe_gamma(R)
        if g is not None:
            return g
        return rre_gamma(R[:k, :k])
    return np.ones(1)


def svd_mpe_gamma(R):
    """SVD-MPE (Sec. III-B): R = U S V^T, gamma = v_last / sum(v_last), v_last the right
    singular vector of the smallest singular value. None if the sum vanishes."""
    _, _, Vt = np.linalg.svd(R)
    v = Vt[-1, :]
    s = v.sum()
    if abs(s) <= SUM_EPS * np.abs(v).sum():
        return None
    return v / s


def extrapolate(x_m, Q, R, gamma):
    """Algorithm 1, steps 3-4: xi_0 = 1 - gamma_0, xi_j = xi_{j-1} - gamma_j;
    eta = R_{k-1} xi; x_(m,k) = x_m + Q_{k-1} eta (k = len(gamma) - 1)."""
    k = len(gamma) - 1
    xi = np.zeros(k)
    acc = 1.0
    for j in range(k):
        acc = acc - gamma[j]
        xi[j] = acc
    eta = R[:k, :k] @ xi
    return x_m + (Q[:, :k] @ eta).reshape(x_m.shape)


@dataclass
class SolveResult:
    x: np.ndarray
    calls: int
    cycles: int
    breakdowns: int
    deltas: list
    gamma_l1: list
    trace: list  # (calls, vector) when record=True, else []
    rejected: int = 0  # extrapolations the stability guard rejected (also in breakdowns)


def _rel_change(new, old):
    n = np.linalg.norm(old)
    return float(np.linalg.norm(new - old) / n) if n > 0 else float("inf")


def ve_step(xs, method, gamma_cap=GAMMA_CAP):
    """Given x_m .. x_{m+kappa+1} (flattened rows), return (x_new, gamma, broke_down).

    When the coefficients exist but sum |gamma| exceeds gamma_cap (> 0), or is not finite,
    they are rejected by the stability guard: x_new is the last iterate, broke_down is True
    and gamma is returned for the statistics."""
    X = np.stack([np.ravel(v) for v in xs], axis=1)
    U = X[:, 1:] - X[:, :-1]                     # Algorithm 1, step 1
    Q, R = mgs(U)                                 # Algorithm 2
    if method == "mpe":
        g = mpe_gamma(R)
    elif method == "rre":
        g = rre_gamma(R)
    elif method == "svd_mpe":
        g = svd_mpe_gamma(R)
    else:
        raise ValueError(method)
    if g is None:
        return X[:, -1].copy(), None, True
    if gamma_cap is not None and gamma_cap > 0 and not (np.abs(g).sum() <= gamma_cap):
        return X[:, -1].copy(), g, True
    return extrapolate(X[:, 0], Q, R, g), g, False


def solve(op: OracleProblem, method="none", L=5, m=0, tol=1e-5, max_calls=500, extra_fp=0,
          x0=None, record=False, on_vector=None, gamma_cap=GAMMA_CAP):
    """Plain FP (method='none') or Algorithm 3 (full cycling) with MPE/RRE/SVD-MPE.

    Cycle: m FP calls to reach x_m, then L = kappa+1 more to x_{m+kappa+1}; extrapolate;
    restart from x_(m,kappa). Termination (Sec. III-C): the relative change of two
    consecutive FP iterates drops below tol, or the total FP-call budget is spent. If the
    budget ends inside a cycle, the last FP iterate is returned. `extra_fp` FP calls follow.
    `on_vector(calls, x)` sees every vector the solve could return (FP iterates and
    extrapolated vectors). gamma_cap is the stability guard of ve_step (<= 0 or None: off);
    a rejected extrapolation counts as a breakdown and in `rejected`."""
    shape = op.shape
    x = op.x0() if x0 is None else _f64(x0).copy()
    calls = cycles = breakdowns = rejected = 0
    deltas, gl1, trace = [], [], []

    def note(v):
        if record:
            trace.append((calls, v.copy()))
        if on_vector is not None:
            on_vector(calls, v)

    if method == "none":
        while calls < max_calls:
            xn = op.fp(x)
            calls += 1
            d = _rel_change(xn, x)
            deltas.append(d)
            x = xn
            note(x)
            if d < tol:
                break
    else:
        while calls < max_calls:
            xs = [x]
            done_early = False
            for _ in range(m + L):
                if calls >= max_calls:
                    done_early = True
                    break
                xn = op.fp(xs[-1])
                calls += 1
                deltas.append(_rel_change(xn, xs[-1]))
                xs.append(xn)
                note(xn)
            if done_early:
                x = xs[-1]
                break
            xw = xs[m:]
            xnew, g, broke = ve_step(xw, method, gamma_cap)
            cycles += 1
            if broke:
                breakdowns += 1
                rejected += g is not None
            else:
                gl1.append(float(np.abs(g).sum()))
            x = xnew.reshape(shape)
            note(x)
            if deltas[-1] < tol:
                break
    for _ in range(extra_fp):
        x = op.fp(x)
        calls += 1
        note(x)
    return SolveResult(x, calls, cycles, breakdowns, deltas, gl1, trace, rejected)
