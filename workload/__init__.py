"""Seeded synthetic workloads for RED restoration (deblurring and 3x super-resolution).

This module only draws random numbers and builds parameter arrays. It holds none of the
restoration method's arithmetic: it never applies a blur, a decimation, the denoiser or a
solver. An observation y = H x_true + sigma * n is formed by whoever consumes the workload
(the oracle in tests, the GPU library in the benchmark) from the pieces returned here:
the clean image x_true, the point-spread function, the decimation factor, sigma and the
standard-normal noise n.

Stand-ins (the paper's test images and its trained TNRD model are not available):
  * images: a linear-gradient background, axis-aligned rectangles of random level and
    i.i.d. Gaussian texture (std 8), clipped to [0, 255];
  * PSFs: the two kernels of the deblurring experiments (Sec. IV-A: 9x9 uniform, and a
    Gaussian of standard deviation 1.6) and the 7x7 Gaussian + 3x decimation of the
    super-resolution experiment (Sec. IV-B);
  * denoiser: a TNRD-style reaction-diffusion model (Sec. IV names TNRD as the denoising
    engine) with T=5 stages, 24 zero-mean 5x5 filters per stage and odd influence functions,
    each a sum of 63 Gaussian radial basis functions centred on [-310, 310].

All generators use numpy's PCG64 (`numpy.random.default_rng`) with fixed seeds, so every
array is bit-identical across machines.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------------------
# Images
# ----------------------------------------------------------------------------------------


def make_image(h: int, w: int, seed: int) -> np.ndarray:
    """Piecewise-smooth test image in [0, 255], float64, shape (h, w)."""
    rng = np.random.default_rng(seed)
    a0 = rng.uniform(40.0, 100.0)
    gy = rng.uniform(-60.0, 60.0)
    gx = rng.uniform(-60.0, 60.0)
    ii = np.arange(h, dtype=np.float64)[:, None] / max(h - 1, 1)
    jj = np.arange(w, dtype=np.float64)[None, :] / max(w - 1, 1)
    img = a0 + gy * ii + gx * jj
    img = np.broadcast_to(img, (h, w)).copy()
    n_rect = max(4, int(round(16.0 * math.sqrt(h * w) / 256.0)))
    for _ in range(n_rect):
        rh = max(2, int(round(rng.uniform(0.05, 0.4) * h)))
        rw = max(2, int(round(rng.uniform(0.05, 0.4) * w)))
        rh, rw = min(rh, h), min(rw, w)
        r0 = int(rng.integers(0, h - rh + 1))
        c0 = int(rng.integers(0, w - rw + 1))
        level = rng.uniform(-80.0, 80.0)
        img[r0:r0 + rh, c0:c0 + rw] += level
    img += rng.normal(0.0, 8.0, size=(h, w))
    return np.clip(img, 0.0, 255.0)


def make_noise(shape, seed: int) -> np.ndarray:
    """Standard-normal noise field n (the observation adds sigma * n)."""
    return np.random.default_rng(seed).standard_normal(shape)


# ----------------------------------------------------------------------------------------
# Point-spread functions
# ----------------------------------------------------------------------------------------


def psf_uniform(k: int = 9) -> np.ndarray:
    """k x k box PSF, each tap 1/k^2 (Sec. IV-A, 9x9 uniform blur)."""
    return np.full((k, k), 1.0 / (k * k))


def psf_gaussian(k: int = 7, std: float = 1.6) -> np.ndarray:
    """k x k Gaussian PSF of the given standard deviation, normalised to unit sum
    (Sec. IV-A deblurring, Sec. IV-B super-resolution: std 1.6)."""
    r = (k - 1) // 2
    a = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * std * std))
    return g / g.sum()


def lr_shape(h: int, w: int, decim: int) -> tuple[int, int]:
    """Shape of the decimated observation: samples (decim*i, decim*j) are kept."""
    return (-(-h // decim), -(-w // decim))


# ----------------------------------------------------------------------------------------
# TNRD-style denoiser parameters
# ----------------------------------------------------------------------------------------


@dataclass(frozen=True)
class DenoiserParams:
    stages: int
    nfilt: int
    ksize: int
    nrbf: int
    mu0: float
    dmu: float
    gamma: float
    filters: np.ndarray = field(repr=False)  # (T, F, k, k) correlation taps, zero mean
    rbf_w: np.ndarray = field(repr=False)    # (T, F, J) antisymmetric RBF weights
    react: np.ndarray = field(repr=False)    # (T,) reaction weights theta_t


def _rbf_slope_max(w: np.ndarray, mu: np.ndarray, gamma: float) -> np.ndarray:
    """max over a z-grid of d/dz sum_j w_j exp(-(z-mu_j)^2/(2 gamma^2)), per row of w.

    Used only to scale the seeded weights (a parameter choice); the restoration method never
    evaluates this derivative."""
    z = np.arange(-320.0, 320.0 + 1e-9, 0.05)
    d = z[:, None] - mu[None, :]                       # (Z, J)
    dg = -(d / (gamma * gamma)) * np.exp(-(d * d) / (2.0 * gamma * gamma))
    slopes = w.reshape(-1, w.shape[-1]) @ dg.T          # (rows, Z)
    return slopes.max(axis=1).reshape(w.shape[:-1])


@functools.lru_cache(maxsize=4)
def make_denoiser(seed: int = 1805, stages: int = 5, nfilt: int = 24, ksize: int = 5,
                  nrbf: int = 63, mu0: float = -310.0, dmu: float = 10.0,
                  gamma: float = 10.0, target: float = 0.1) -> DenoiserParams:
    """Seeded TNRD-style parameters.

    * filters: N(0,1) taps minus their mean, scaled to unit l1 norm (zero mean makes a
      constant image a fixed point of every stage);
    * influence weights: w_{t,i,j} = a_{t,i} sgn(mu_j) R_{t,i}(|j - c|), c the centre index,
      R(n) = sum_{l<=n} delta_l exp(-l/6), delta_l ~ U(0,1): odd, saturating functions;
    * a_{t,i} so that max_z phi'_{t,i}(z) * max_omega sum_i |k_hat_{t,i}(omega)|^2 = target,
      which bounds every stage's diffusion operator norm by `target` (passivity);
    * reaction weights theta_t ~ U(0.05, 0.15).
    """
    assert nrbf % 2 == 1
    rng = np.random.default_rng(seed)
    raw = rng.standard_normal((stages, nfilt, ksize, ksize))
    delta = rng.uniform(0.0, 1.0, size=(stages, nfilt, nrbf // 2))
    react = rng.uniform(0.05, 0.15, size=stages)

    filt = raw - raw.mean(axis=(2, 3), keepdims=True)
    filt = filt / np.abs(filt).sum(axis=(2, 3), keepdims=True)

    c = nrbf // 2
    mu = mu0 + dmu * np.arange(nrbf)
    l = np.arange(1, c + 1, dtype=np.float64)
    rcum = np.concatenate([np.zeros((stages, nfilt, 1)),
                           np.cumsum(delta * np.exp(-l / 6.0), axis=-1)], axis=-1)  # R(0..c)
    idx = np.abs(np.arange(nrbf) - c)
    sgn = np.sign(np.arange(nrbf) - c).astype(np.float64)
    w_unit = sgn[None, None, :] * rcum[:, :, idx]

    spec = np.fft.fft2(filt, s=(256, 256))
    s_t = (np.abs(spec) ** 2).sum(axis=1).max(axis=(1, 2))        # (T,)
    slope = _rbf_slope_max(w_unit, mu, gamma)                        # (T, F)
    a = target / (slope * s_t[:, None])
    rbf_w = a[:, :, None] * w_unit
    for arr in (filt, rbf_w, react):
        arr.setflags(write=False)
    return DenoiserParams(stages, nfilt, ksize, nrbf, mu0, dmu, gamma, filt, rbf_w, react)


def identity_denoiser(ksize: int = 5, nrbf: int = 63) -> DenoiserParams:
    """Zero-stage denoiser: D(x) = x (a special case that makes the FP iteration linear)."""
    z = np.zeros((0, 1, ksize, ksize))
    return DenoiserParams(0, 1, ksize, nrbf, -310.0, 10.0, 10.0, z,
                          np.zeros((0, 1, nrbf)), np.zeros((0,)))


# ----------------------------------------------------------------------------------------
# Problem configurations
# ----------------------------------------------------------------------------------------


@dataclass
class Problem:
    """One restoration problem: the pieces of y = H x_true + sigma * n and solver settings."""
    name: str
    x_true: np.ndarray
    psf: np.ndarray
    decim: int
    sigma: float
    lam: float
    noise: np.ndarray
    cg_iters: int
    denoiser: DenoiserParams
    method: str = "none"   # none | mpe | rre | svd_mpe
    L: int = 5
    m: int = 0
    tol: float = 1e-5
    max_fp_calls: int = 500

    @property
    def hr_shape(self):
        return self.x_true.shape

    @property
    def lr_shape(self):
        return lr_shape(*self.x_true.shape, self.decim)


SQRT2 = math.sqrt(2.0)


def problem(name: str) -> Problem:
    """Named workloads.

    tiny       32x32 deblur, Gaussian 7x7 (CPU-test size)
    deblur64   64x64, Gaussian 7x7 std 1.6, sigma sqrt(2), lambda 0.02, 10 CG, plain FP, 20 calls
    deblur256  256x256, uniform 9x9, sigma sqrt(2), lambda 0.02, 15 CG, MPE/RRE L=5, tol 1e-5
    sr512      512x512, Gaussian 7x7 + 3x decimation, sigma 5, lambda 0.02, 15 CG, RRE L=8
    """
    d = make_denoiser()
    if name == "tiny":
        return Problem("tiny", make_image(32, 32, 1099), psf_gaussian(7, 1.6), 1, SQRT2, 0.02,
                       make_noise((32, 32), 2099), 10, d, "none", 5, 0, 0.0, 20)
    if name == "deblur64":
        return Problem("deblur64", make_image(64, 64, 1000), psf_gaussian(7, 1.6), 1, SQRT2, 0.02,
                       make_noise((64, 64), 2000), 10, d, "none", 5, 0, 0.0, 20)
    if name == "deblur256":
        return Problem("deblur256", make_image(256, 256, 1001), psf_uniform(9), 1, SQRT2, 0.02,
                       make_noise((256, 256), 2001), 15, d, "rre", 5, 0, 1e-5, 500)
    if name == "sr512":
        x = make_image(512, 512, 1002)
        return Problem("sr512", x, psf_gaussian(7, 1.6), 3, 5.0, 0.02,
                       make_noise(lr_shape(512, 512, 3), 2002), 15, d, "rre", 8, 0, 1e-5, 500)
    raise KeyError(name)


def batch_items(n: int = 64, lo: int = 128, hi: int = 1024, seed: int = 3000):
    """Uneven batch: sides log-uniform in [lo, hi] (independent h, w), operator uniform 9x9 or
    Gaussian 7x7 (deblurring) with p=1/2, sigma in {sqrt(2), 5} with p=1/2."""
    d = make_denoiser()
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed + i)
        h = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        w = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        psf = psf_uniform(9) if rng.uniform() < 0.5 else psf_gaussian(7, 1.6)
        sigma = SQRT2 if rng.uniform() < 0.5 else 5.0
        out.append(Problem(f"b{i}", make_image(h, w, seed + 10000 + i), psf, 1, sigma, 0.02,
                           make_noise((h, w), seed + 20000 + i), 15, d, "rre", 5, 0, 1e-5, 500))
    return out


def serve_trace(n: int, rate_hz: float, lo: int = 128, hi: int = 2048, seed: int = 4000):
    """Poisson arrival trace of restoration requests: (arrival_s, Problem) pairs. Sides
    log-uniform in [lo, hi]; deblurring (uniform 9x9) or 3x super-resolution (Gaussian 7x7,
    std 1.6) with p=1/2; sigma in {sqrt(2), 5} with p=1/2."""
    d = make_denoiser()
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        h = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        w = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        sr = rng.uniform() < 0.5
        sigma = SQRT2 if rng.uniform() < 0.5 else 5.0
        psf = psf_gaussian(7, 1.6) if sr else psf_uniform(9)
        decim = 3 if sr else 1
        s_img, s_noise = int(rng.integers(1 << 30)), int(rng.integers(1 << 30))
        out.append((t, Problem(f"r{i}", make_image(h, w, s_img), psf, decim, sigma, 0.02,
                               make_noise(lr_shape(h, w, decim), s_noise), 15, d, "rre", 5, 0,
                               1e-5, 500)))
    return out
