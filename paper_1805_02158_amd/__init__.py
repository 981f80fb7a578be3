"""redve: RED restoration by fixed-point iteration with vector extrapolation, on MI355X.

Thin Python binding of the C ABI in include/redve.h (libredve.so, built for gfx950). It only
marshals arguments: torch tensors provide device memory and the HIP stream; every step of the
method runs in the library's HIP kernels. There is no CPU fallback: without the built library
or a GPU every call raises RedveError.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libredve.so")

OK, E_ARG, E_STATE, E_NOMEM, E_HIP, E_NONFINITE, E_DIVERGED = 0, -1, -2, -3, -4, -5, -6
VE_NONE, VE_MPE, VE_RRE, VE_SVD_MPE = 0, 1, 2, 3
PREC_FP32, PREC_BF16 = 0, 1
BASE_FP, BASE_SD = 0, 1
LIN_CG, LIN_FFT = 0, 1
METHODS = {"none": VE_NONE, "mpe": VE_MPE, "rre": VE_RRE, "svd_mpe": VE_SVD_MPE}
PRECISIONS = {"fp32": PREC_FP32, "bf16": PREC_BF16}
BASES = {"fp": BASE_FP, "sd": BASE_SD}
LINEAR = {"cg": LIN_CG, "fft": LIN_FFT}

# Every symbol include/redve.h declares.
EXPORTS = (
    "redve_create", "redve_destroy", "redve_set_stream", "redve_last_error",
    "redve_workspace_bytes", "redve_set_operator", "redve_set_noise", "redve_set_lambda",
    "redve_set_denoiser", "redve_set_extrapolation", "redve_set_solver", "redve_set_base",
    "redve_set_linear_solver", "redve_solve", "redve_apply_H", "redve_apply_Ht",
    "redve_apply_A", "redve_cg", "redve_denoise", "redve_fp_step", "redve_objective",
    "redve_extrapolate", "redve_solve_batch", "redve_server_create", "redve_server_submit",
    "redve_server_poll", "redve_server_wait", "redve_server_counts", "redve_server_destroy",
    "redve_extrapolate_noalloc", "redve_extrapolate_noalloc_max", "redve_set_guard",
    "redve_set_autotune", "redve_set_tuning", "redve_get_tuning", "redve_server_occupancy",
    "redve_set_precision_switch",
)


class RedveError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"redve error {code}: {msg}")
        self.code = code


class _Tnrd(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int), ("nfilt", ctypes.c_int), ("ksize", ctypes.c_int),
                ("nrbf", ctypes.c_int), ("mu0", ctypes.c_double), ("dmu", ctypes.c_double),
                ("gamma", ctypes.c_double), ("filters", ctypes.POINTER(ctypes.c_double)),
                ("rbf_w", ctypes.POINTER(ctypes.c_double)),
                ("react", ctypes.POINTER(ctypes.c_double)), ("precision", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("stage_threads", ctypes.c_int), ("phi_table", ctypes.c_int),
                ("cg_per_launch", ctypes.c_int), ("cg_threads", ctypes.c_int),
                ("fused_start", ctypes.c_int), ("cg_tile", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Item(ctypes.Structure):
    _fields_ = [("y", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("hx", ctypes.c_int), ("wx", ctypes.c_int),
                ("psf", ctypes.POINTER(ctypes.c_double)), ("kh", ctypes.c_int),
                ("kw", ctypes.c_int), ("decim", ctypes.c_int), ("sigma", ctypes.c_double),
                ("lam", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("fp_calls", ctypes.c_int), ("cycles", ctypes.c_int),
                ("breakdowns", ctypes.c_int), ("status", ctypes.c_int),
                ("final_delta", ctypes.c_double), ("max_gamma_l1", ctypes.c_double),
                ("ms", ctypes.c_double), ("rejected", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libredve.so and declare its signatures (no GPU needed to load it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RedveError(E_STATE, f"{path} is not built (run paper_1805_02158_amd/build.py)")
    L = ctypes.CDLL(path)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "redve_create": ([ctypes.POINTER(vp), i, vp], i),
        "redve_destroy": ([vp], i),
        "redve_set_stream": ([vp, vp], i),
        "redve_last_error": ([vp], ctypes.c_char_p),
        "redve_workspace_bytes": ([vp, i, i], sz),
        "redve_set_operator": ([vp, dp, i, i, i], i),
        "redve_set_noise": ([vp, d], i),
        "redve_set_lambda": ([vp, d], i),
        "redve_set_denoiser": ([vp, ctypes.POINTER(_Tnrd)], i),
        "redve_set_extrapolation": ([vp, i, i, i], i),
        "redve_set_solver": ([vp, i, i, d, i], i),
        "redve_set_base": ([vp, i, d], i),
        "redve_set_linear_solver": ([vp, i], i),
        "redve_solve": ([vp, vp, i, i, vp, vp, i, i, ctypes.POINTER(Stats)], i),
        "redve_apply_H": ([vp, vp, i, i, vp], i),
        "redve_apply_Ht": ([vp, vp, i, i, vp], i),
        "redve_apply_A": ([vp, vp, i, i, vp], i),
        "redve_cg": ([vp, vp, vp, i, i, i], i),
        "redve_denoise": ([vp, vp, i, i, vp], i),
        "redve_fp_step": ([vp, vp, vp, i, i, vp], i),
        "redve_objective": ([vp, vp, vp, i, i, dp], i),
        "redve_extrapolate": ([vp, vp, i, i, i, vp, dp, ctypes.POINTER(i)], i),
        "redve_solve_batch": ([vp, i, ctypes.POINTER(Item), ctypes.POINTER(Stats)], i),
        "redve_server_create": ([ctypes.POINTER(vp), vp, sz, i], i),
        "redve_server_submit": ([vp, ctypes.POINTER(Item), ctypes.POINTER(ctypes.c_ulonglong)], i),
        "redve_server_poll": ([vp, ctypes.c_ulonglong, ctypes.POINTER(i), ctypes.POINTER(Stats)], i),
        "redve_server_wait": ([vp, ctypes.c_ulonglong, ctypes.POINTER(Stats)], i),
        "redve_server_counts": ([vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                 ctypes.POINTER(ctypes.c_longlong)], i),
        "redve_server_destroy": ([vp], i),
        "redve_extrapolate_noalloc": ([vp, vp, i, i, i, vp, dp, ctypes.POINTER(i)], i),
        "redve_extrapolate_noalloc_max": ([i], sz),
        "redve_set_guard": ([vp, d], i),
        "redve_set_precision_switch": ([vp, d], i),
        "redve_set_autotune": ([vp, i, ctypes.c_char_p], i),
        "redve_server_occupancy": ([vp, ctypes.POINTER(sz), ctypes.POINTER(sz),
                                    ctypes.POINTER(ctypes.c_longlong)], i),
        "redve_set_tuning": ([vp, ctypes.POINTER(Tuning)], i),
        "redve_get_tuning": ([vp, i, i, ctypes.POINTER(Tuning), dp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RedveError(E_STATE, "no GPU visible: the redve library runs only on MI355X")
    return torch


def _f64p(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dev(t, shape=None):
    """Device pointer of a contiguous float32 CUDA tensor (validated)."""
    if t is None:
        return None
    if not (t.is_cuda and t.dtype.is_floating_point and t.dtype.itemsize == 4 and t.is_contiguous()):
        raise RedveError(E_ARG, "expected a contiguous float32 tensor on the GPU")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise RedveError(E_ARG, f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def lr_shape(h, w, s):
    return ((h + s - 1) // s, (w + s - 1) // s)


class Restorer:
    """One library handle (include/redve.h). Not thread-safe; one per host thread."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self._L = load_library()
        self.device = int(device)
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        h = ctypes.c_void_p()
        self._check(self._L.redve_create(ctypes.byref(h), self.device,
                                         ctypes.c_void_p(stream.cuda_stream)), None)
        self._h = h
        self.decim = 1
        self._keep = []

    # -- plumbing
    def _check(self, rc, h="self"):
        if rc != OK:
            msg = ""
            if h is not None and getattr(self, "_h", None) is not None:
                msg = self._L.redve_last_error(self._h).decode()
            raise RedveError(rc, msg)

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._L.redve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._stream = stream
        self._check(self._L.redve_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    # -- problem statement
    def set_operator(self, psf, decim: int = 1):
        a, p = _f64p(psf)
        self._check(self._L.redve_set_operator(self._h, p, a.shape[0], a.shape[1], int(decim)))
        self.decim = int(decim)
        return self

    def set_noise(self, sigma: float):
        self._check(self._L.redve_set_noise(self._h, float(sigma)))
        return self

    def set_lambda(self, lam: float):
        self._check(self._L.redve_set_lambda(self._h, float(lam)))
        return self

    def set_denoiser(self, params, precision: str = "fp32"):
        f, fp = _f64p(params.filters if params.stages else np.zeros(1))
        w, wp = _f64p(params.rbf_w if params.stages else np.zeros(1))
        r, rp = _f64p(params.react if params.stages else np.zeros(1))
        s = _Tnrd(params.stages, params.nfilt, params.ksize, params.nrbf, params.mu0,
                  params.dmu, params.gamma, fp, wp, rp, PRECISIONS[precision])
        self._check(self._L.redve_set_denoiser(self._h, ctypes.byref(s)))
        return self

    def set_extrapolation(self, method: str = "none", L: int = 5, m: int = 0):
        self._check(self._L.redve_set_extrapolation(self._h, METHODS[method], int(L), int(m)))
        return self

    def set_solver(self, cg_iters=15, max_fp_calls=500, tol=1e-5, extra_fp=0):
        self._check(self._L.redve_set_solver(self._h, int(cg_iters), int(max_fp_calls),
                                             float(tol), int(extra_fp)))
        return self

    def set_base(self, base: str = "fp", mu: float = 0.0):
        """Base iteration: "fp" (eq. (7)) or "sd" (steepest descent, step mu; <= 0: default)."""
        self._check(self._L.redve_set_base(self._h, BASES[base], float(mu)))
        return self

    def set_precision_switch(self, delta: float):
        """BF16 form: FP32 banks once the relative change falls below delta (0: never)."""
        self._check(self._L.redve_set_precision_switch(self._h, float(delta)))
        return self

    def set_guard(self, gamma_cap: float):
        """Stability guard on sum |gamma| (<= 0: off)."""
        self._check(self._L.redve_set_guard(self._h, float(gamma_cap)))
        return self

    def set_autotune(self, auto: bool = True, cache_path=None):
        """Launch configuration: built-in rules (auto False) or timed per problem on first use."""
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self._L.redve_set_autotune(self._h, int(bool(auto)), path))
        return self

    def set_tuning(self, cfg=None):
        """Force a launch configuration (dict of Tuning fields, missing ones 0 = rule); None
        returns to the mode."""
        if cfg is None:
            self._check(self._L.redve_set_tuning(self._h, None))
        else:
            t = Tuning(**{k: int(v) for k, v in cfg.items()})
            self._check(self._L.redve_set_tuning(self._h, ctypes.byref(t)))
        return self

    def get_tuning(self, hx: int, wx: int):
        """(configuration dict, tuned FP-call microseconds or -1) for an hx x wx image."""
        t = Tuning()
        us = ctypes.c_double()
        self._check(self._L.redve_get_tuning(self._h, int(hx), int(wx), ctypes.byref(t),
                                             ctypes.byref(us)))
        return t.as_dict(), us.value

    def set_linear_solver(self, kind: str = "cg"):
        """Linear step of the FP call: "cg" (cg_iters iterations) or "fft" (exact, deblurring)."""
        self._check(self._L.redve_set_linear_solver(self._h, LINEAR[kind]))
        return self

    def configure(self, prob, precision="fp32", method=None, L=None, m=None, tol=None,
                  max_fp_calls=None, extra_fp=0):
        """Set everything from a workload.Problem."""
        self.set_operator(prob.psf, prob.decim).set_noise(prob.sigma).set_lambda(prob.lam)
        self.set_denoiser(prob.denoiser, precision)
        self.set_extrapolation(method if method is not None else prob.method,
                               L if L is not None else prob.L, m if m is not None else prob.m)
        self.set_solver(prob.cg_iters, max_fp_calls if max_fp_calls is not None else prob.max_fp_calls,
                        tol if tol is not None else prob.tol, extra_fp)
        return self

    # -- solve
    def solve(self, y, hx: int, wx: int, x0=None, out=None):
        torch = self._torch
        hy, wy = lr_shape(hx, wx, self.decim)
        if out is None:
            out = torch.empty((hx, wx), dtype=torch.float32, device=y.device)
        st = Stats()
        rc = self._L.redve_solve(self._h, _dev(y, (hy, wy)), hy, wy, _dev(x0, (hx, wx)),
                                 _dev(out, (hx, wx)), hx, wx, ctypes.byref(st))
        if rc != OK:  # the statistics of the failed solve travel with the error
            err = RedveError(rc, self._L.redve_last_error(self._h).decode())
            err.stats = st.as_dict()
            raise err
        return out, st.as_dict()

    # -- single steps
    def _empty(self, shape, like):
        return self._torch.empty(shape, dtype=self._torch.float32, device=like.device)

    def apply_H(self, x):
        hx, wx = x.shape
        y = self._empty(lr_shape(hx, wx, self.decim), x)
        self._check(self._L.redve_apply_H(self._h, _dev(x), hx, wx, _dev(y)))
        return y

    def apply_Ht(self, y, hx, wx):
        out = self._empty((hx, wx), y)
        self._check(self._L.redve_apply_Ht(self._h, _dev(y, lr_shape(hx, wx, self.decim)), hx, wx,
                                           _dev(out)))
        return out

    def apply_A(self, p):
        out = self._empty(p.shape, p)
        self._check(self._L.redve_apply_A(self._h, _dev(p), p.shape[0], p.shape[1], _dev(out)))
        return out

    def cg(self, rhs, x, iters):
        x = x.clone()
        self._check(self._L.redve_cg(self._h, _dev(rhs, x.shape), _dev(x), x.shape[0],
                                     x.shape[1], int(iters)))
        return x

    def denoise(self, x):
        out = self._empty(x.shape, x)
        self._check(self._L.redve_denoise(self._h, _dev(x), x.shape[0], x.shape[1], _dev(out)))
        return out

    def fp_step(self, y, x):
        out = self._empty(x.shape, x)
        hx, wx = x.shape
        self._check(self._L.redve_fp_step(self._h, _dev(y, lr_shape(hx, wx, self.decim)),
                                          _dev(x), hx, wx, _dev(out)))
        return out

    def make_item(self, y, hx, wx, psf, decim, sigma, lam, x0=None, out=None):
        """Describes one problem for solve_batch / Server.submit (keeps the host PSF alive)."""
        torch = self._torch
        if out is None:
            out = torch.empty((hx, wx), dtype=torch.float32, device=y.device)
        a, pp = _f64p(psf)
        it = Item(_dev(y, lr_shape(hx, wx, decim)), _dev(x0, (hx, wx)), _dev(out, (hx, wx)),
                  int(hx), int(wx), pp, a.shape[0], a.shape[1], int(decim), float(sigma),
                  float(lam))
        return it, out, a

    def solve_batch(self, problems):
        """problems: list of dicts with y, hx, wx, psf, decim, sigma, lam (and optional x0, out).
        Returns (outputs, stats) in the same order."""
        made = [self.make_item(**p) for p in problems]
        arr = (Item * len(made))(*[m[0] for m in made])
        st = (Stats * len(made))()
        rc = self._L.redve_solve_batch(self._h, len(made), arr, st)
        stats = [s.as_dict() for s in st]
        if rc != OK and not any(s["status"] for s in stats):
            self._check(rc)
        return [m[1] for m in made], stats

    def objective(self, y, x):
        """E(x) of eq. (4): ||Hx - y||^2 / (2 sigma^2) + (lambda/2) x^T (x - f(x))."""
        hx, wx = x.shape
        e = ctypes.c_double()
        self._check(self._L.redve_objective(self._h, _dev(y, lr_shape(hx, wx, self.decim)),
                                            _dev(x), hx, wx, ctypes.byref(e)))
        return e.value

    def extrapolate(self, xs):
        """xs: (L+1, h, w) stacked iterates -> (x_new, gamma, breakdown)."""
        n1, hx, wx = xs.shape
        L = n1 - 1
        out = self._empty((hx, wx), xs)
        g = np.zeros(L)
        bd = ctypes.c_int(0)
        self._check(self._L.redve_extrapolate(self._h, _dev(xs), L, hx, wx, _dev(out),
                                              g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              ctypes.byref(bd)))
        return out, g, bool(bd.value)

    def extrapolate_noalloc(self, xs, out=None):
        """As extrapolate, through the entry point that allocates no device memory (the
        library's fixed scratch array; h w at most extrapolate_noalloc_max(L))."""
        n1, hx, wx = xs.shape
        L = n1 - 1
        if out is None:
            out = self._empty((hx, wx), xs)
        g = np.zeros(L)
        bd = ctypes.c_int(0)
        self._check(self._L.redve_extrapolate_noalloc(
            self._h, _dev(xs), L, hx, wx, _dev(out, (hx, wx)),
            g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(bd)))
        return out, g, bool(bd.value)

    def extrapolate_noalloc_max(self, L: int) -> int:
        return int(self._L.redve_extrapolate_noalloc_max(int(L)))


class Server:
    """Continuous-batching restoration server (include/redve.h, redve_server_*). It copies the
    settings of a configured Restorer; requests are admitted by device-memory budget."""

    def __init__(self, proto: Restorer, hbm_budget: int, max_active: int = 64):
        self._L = proto._L
        self._proto = proto
        h = ctypes.c_void_p()
        rc = self._L.redve_server_create(ctypes.byref(h), proto._h, int(hbm_budget),
                                         int(max_active))
        if rc != OK:
            raise RedveError(rc, "redve_server_create failed")
        self._h = h
        self._keep = {}

    def submit(self, y, hx, wx, psf, decim, sigma, lam, x0=None, out=None):
        it, out, psf_arr = self._proto.make_item(y, hx, wx, psf, decim, sigma, lam, x0, out)
        t = ctypes.c_ulonglong()
        rc = self._L.redve_server_submit(self._h, ctypes.byref(it), ctypes.byref(t))
        if rc != OK:
            raise RedveError(rc, "redve_server_submit failed")
        self._keep[t.value] = (y, x0, out)
        return t.value, out

    def poll(self, ticket):
        done = ctypes.c_int()
        st = Stats()
        self._L.redve_server_poll(self._h, ctypes.c_ulonglong(ticket), ctypes.byref(done),
                                  ctypes.byref(st))
        return bool(done.value), (st.as_dict() if done.value else None)

    def wait(self, ticket):
        st = Stats()
        rc = self._L.redve_server_wait(self._h, ctypes.c_ulonglong(ticket), ctypes.byref(st))
        if rc != OK:
            raise RedveError(rc, "redve_server_wait failed")
        self._keep.pop(ticket, None)
        return st.as_dict()

    def counts(self):
        q, a, f, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
        self._L.redve_server_counts(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(f),
                                    ctypes.byref(r))
        return {"queued": q.value, "active": a.value, "finished": f.value, "rounds": r.value}

    def occupancy(self):
        """Pixel capacity of the budget, most pixels admitted at once, rounds with a request
        waiting."""
        c, p, w = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_longlong()
        self._L.redve_server_occupancy(self._h, ctypes.byref(c), ctypes.byref(p), ctypes.byref(w))
        return {"capacity_px": c.value, "peak_px": p.value, "waited_rounds": w.value}

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._L.redve_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
