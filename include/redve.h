/*
 * redve — RED restoration by fixed-point iteration with vector extrapolation, on MI355X.
 *
 * C ABI of the GPU library. It implements the method of Hong, Romano and Elad,
 * "Acceleration of RED via Vector Extrapolation":
 *   observation   y = H x + e, e white Gaussian of variance sigma^2          (Sec. II-A, eq. (1))
 *   FP iteration  x_{k+1} = [H^T H/sigma^2 + lambda I]^{-1}[H^T y/sigma^2 + lambda f(x_k)]
 *                                                                            (Sec. II-B, eq. (7))
 *   acceleration  MPE / RRE / SVD-MPE in full cycling                       (Sec. III, Alg. 1-3)
 * with the linear step of eq. (7) solved by conjugate gradients (eq. (7) footnote: iterative
 * methods) and f a TNRD-style reaction-diffusion denoiser (Sec. IV uses TNRD).
 *
 * Conventions
 *  - Images are row-major float32, H rows by W columns, dense (row pitch = W elements).
 *  - "device pointer": memory on the handle's GPU, owned by the caller, valid until the call
 *    returns. "host pointer": CPU memory, read during the call only (the library copies it).
 *  - Every call returns REDVE_OK (0) or a negative error code; redve_last_error() gives a
 *    message. No call throws. A handle is not thread-safe: use one handle per host thread.
 *  - Work is queued on the handle's HIP stream (the caller's); calls that return results to
 *    the host (solve statistics) synchronise that stream before returning.
 *  - Boundary: the blur H is periodic (block-circulant, footnote to eq. (7)); the denoiser
 *    extends images by half-sample symmetric mirroring.
 */
#ifndef REDVE_H
#define REDVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct redve_ctx* redve_t;

enum {
    REDVE_OK = 0,
    REDVE_E_ARG = -1,       /* invalid argument (null pointer, size, parameter range)       */
    REDVE_E_STATE = -2,     /* a required setter was not called before solve                 */
    REDVE_E_NOMEM = -3,     /* device allocation failed                                      */
    REDVE_E_HIP = -4,       /* a HIP runtime call failed                                     */
    REDVE_E_NONFINITE = -5, /* an iterate became NaN or infinite                             */
    REDVE_E_DIVERGED = -6   /* the relative change grew for 3 consecutive cycles/calls       */
};

enum { REDVE_VE_NONE = 0, REDVE_VE_MPE = 1, REDVE_VE_RRE = 2, REDVE_VE_SVD_MPE = 3 };
enum { REDVE_PREC_FP32 = 0, REDVE_PREC_BF16 = 1 };

/* Largest supported sizes. */
#define REDVE_MAX_PSF 15     /* PSF side (odd, 1..15)                              */
#define REDVE_MAX_DECIM 4    /* decimation factor s                                */
#define REDVE_MAX_L 16       /* difference columns per extrapolation (kappa + 1)   */
#define REDVE_MAX_FILTERS 32 /* denoiser filters per stage                         */
#define REDVE_MAX_RBF 127    /* Gaussian RBF centres per influence function        */

/* TNRD-style denoiser f (Sec. II-B; TNRD per Sec. IV). T stages; each stage t maps
 *   u_t = u_{t-1} - sum_i K_{t,i}^T phi_{t,i}(K_{t,i} u_{t-1}) - theta_t (u_{t-1} - f_in)
 * with K_{t,i} the 5x5 correlation of the mirror-extended image with filters[t][i], and
 * phi_{t,i}(z) = sum_j rbf_w[t][i][j] exp(-(z - mu0 - j dmu)^2 / (2 gamma^2)).
 * u_0 = f_in = the denoiser input; the output is u_T. All arrays are host pointers (copied). */
typedef struct {
    int stages;             /* T >= 0 (0: f is the identity)                      */
    int nfilt;              /* filters per stage, 1..REDVE_MAX_FILTERS            */
    int ksize;              /* filter side; must be 5                             */
    int nrbf;               /* RBF centres, 1..REDVE_MAX_RBF                      */
    double mu0, dmu, gamma; /* centre of index 0, spacing, width (> 0)            */
    const double* filters;  /* T*nfilt*ksize*ksize, row-major taps                */
    const double* rbf_w;    /* T*nfilt*nrbf                                       */
    const double* react;    /* T reaction weights theta_t                         */
    int precision;          /* REDVE_PREC_FP32 or REDVE_PREC_BF16 (filter banks)  */
} redve_tnrd_t;

/* Statistics of one solve (host struct written by redve_solve). */
typedef struct {
    int fp_calls;        /* FP calls made (one denoiser call + one CG solve each)        */
    int cycles;          /* extrapolations performed (Algorithm 3 cycles)                */
    int breakdowns;      /* extrapolations that did not exist (MPE/SVD-MPE, Sec. III-B)  */
    int status;          /* REDVE_OK, or the error the solve ended with                  */
    double final_delta;  /* last ||x_{k+1} - x_k|| / ||x_k|| of two FP iterates          */
    double max_gamma_l1; /* max over cycles of sum_i |gamma_i| (stability, eq. (21))     */
    double ms;           /* wall time of the solve on the host, milliseconds             */
} redve_stats_t;

/* ---- handle ------------------------------------------------------------------------- */

/* Create a handle on GPU `device`, queueing work on `hip_stream` (a hipStream_t; NULL = the
 * null stream). The handle owns its device workspace. */
int redve_create(redve_t* out, int device, void* hip_stream);
int redve_destroy(redve_t h);
int redve_set_stream(redve_t h, void* hip_stream);
const char* redve_last_error(redve_t h);
/* Bytes of device workspace a solve of an hx x wx image needs with the current settings. */
size_t redve_workspace_bytes(redve_t h, int hx, int wx);

/* ---- problem statement (Sec. II) ------------------------------------------------------ */

/* Operator H = S B of eq. (1): B blurs with the kh x kw PSF `psf` (host, row-major, odd sizes
 * up to REDVE_MAX_PSF), periodic boundary:
 *   (B x)[i,j] = sum_{a,b} psf[a+rh][b+rw] x[(i-a) mod H][(j-b) mod W];
 * S keeps samples (decim*i, decim*j) (decim = 1: deblurring; 3: super-resolution). */
int redve_set_operator(redve_t h, const double* psf, int kh, int kw, int decim);
/* Noise standard deviation sigma > 0 of eq. (1). */
int redve_set_noise(redve_t h, double sigma);
/* Trade-off weight lambda > 0 (the paper's alpha, eq. (2)). */
int redve_set_lambda(redve_t h, double lambda);
/* Denoiser f (see redve_tnrd_t). Filters must have zero mean (|sum| <= 1e-6 sum|k|). */
int redve_set_denoiser(redve_t h, const redve_tnrd_t* p);

/* ---- solver (Sec. III) --------------------------------------------------------------- */

/* Extrapolation method (Sec. III-B) with L = kappa + 1 difference columns (2..REDVE_MAX_L;
 * Algorithm 1 uses x_m .. x_{m+kappa+1}) and m >= 0 FP calls before each window
 * (Algorithm 3). method REDVE_VE_NONE runs plain FP. */
int redve_set_extrapolation(redve_t h, int method, int L, int m);
/* cg_iters >= 0 CG iterations per FP call (warm start from x_k); the solve stops after
 * max_fp_calls FP calls, or when ||x_{k+1} - x_k|| / ||x_k|| < tol (plain FP: after every call;
 * with extrapolation: for the last call of a cycle, Sec. III-C); extra_fp >= 0 FP calls
 * follow (Sec. III-C recommends some). Defaults: 15, 500, 1e-5, 0. */
int redve_set_solver(redve_t h, int cg_iters, int max_fp_calls, double tol, int extra_fp);

/* Solve: y (device, hy x wy) -> x (device, hx x wx), hy = ceil(hx/decim), wy = ceil(wx/decim).
 * x0 (device, hx x wx) is the initial vector, or NULL for the default (y when decim = 1,
 * decim^2 H^T y otherwise). x may alias x0. If the budget ends inside a cycle the last FP
 * iterate is returned; a completed cycle returns the extrapolated vector (Algorithm 3).
 * st (host, may be NULL) receives statistics. Synchronises the stream. */
int redve_solve(redve_t h, const float* y, int hy, int wy, const float* x0, float* x, int hx,
                int wx, redve_stats_t* st);

/* ---- single steps (device pointers; queued on the stream, not synchronised) ------------ */

/* y = H x (eq. (1)); x: hx x wx, y: ceil(hx/decim) x ceil(wx/decim). */
int redve_apply_H(redve_t h, const float* x, int hx, int wx, float* y);
/* out = H^T y; y: ceil(hx/decim) x ceil(wx/decim), out: hx x wx. */
int redve_apply_Ht(redve_t h, const float* y, int hx, int wx, float* out);
/* out = (H^T H / sigma^2 + lambda I) p, the matrix of eq. (7). */
int redve_apply_A(redve_t h, const float* p, int hx, int wx, float* out);
/* iters CG iterations on (H^T H/sigma^2 + lambda I) x = rhs, warm-started from x (in/out). */
int redve_cg(redve_t h, const float* rhs, float* x, int hx, int wx, int iters);
/* out = f(x), the denoiser. out must not alias x. */
int redve_denoise(redve_t h, const float* x, int hx, int wx, float* out);
/* One FP call of eq. (7): out = CG_{cg_iters}(A, b0 + lambda f(x); start x), where
 * b0 = H^T y / sigma^2 is computed from y (ceil(hx/decim) x ceil(wx/decim)). out may not alias x. */
int redve_fp_step(redve_t h, const float* y, const float* x, int hx, int wx, float* out);
/* One extrapolation (Algorithm 1 with the configured method) from the L+1 iterates
 * xs[0..L] (device, each hx x wx, stored consecutively): out = x_(0,kappa), or xs[L] if the
 * extrapolation does not exist. gamma (host, L doubles, may be NULL) receives gamma_0..kappa
 * (zeros on breakdown); *breakdown (host, may be NULL) receives 1 on breakdown.
 * Synchronises the stream. */
int redve_extrapolate(redve_t h, const float* xs, int L, int hx, int wx, float* out,
                      double* gamma, int* breakdown);

#ifdef __cplusplus
}
#endif
#endif
