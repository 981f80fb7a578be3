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
enum { REDVE_BASE_FP = 0, REDVE_BASE_SD = 1 };
enum { REDVE_LIN_CG = 0, REDVE_LIN_FFT = 1 };

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
    int precision;          /* REDVE_PREC_FP32 or REDVE_PREC_BF16 (filter banks);
                               BF16 needs 4 (576 + 400 z + nfilt (nrbf + 32)) bytes
                               of LDS per workgroup (the device's limit: 160 KiB on
                               gfx950, which every size within the limits fits),
                               z = 25 (nfilt <= 25) or 33 (else); REDVE_E_ARG if not.
                               On images of fewer than 512 16x16 tiles the BF16
                               stage reads phi from per-filter cubic tables (knots
                               gamma / 2 apart; error < 1e-3 of the weights) where
                               they fit that limit, else it sums the window   */
} redve_tnrd_t;

/* Statistics of one solve (host struct written by redve_solve). */
typedef struct {
    int fp_calls;        /* FP calls made (one denoiser call + one CG solve each)        */
    int cycles;          /* extrapolations performed (Algorithm 3 cycles)                */
    int breakdowns;      /* extrapolations that did not exist (MPE/SVD-MPE, Sec. III-B)  */
    int status;          /* REDVE_OK, or the error the solve ended with                  */
    double final_delta;  /* last ||x_{k+1} - x_k|| / ||x_k|| of two FP iterates          */
    double max_gamma_l1; /* max over accepted cycles of sum_i |gamma_i| (eq. (21))       */
    double ms;           /* wall time of the solve on the host, milliseconds             */
    int rejected;        /* extrapolations the stability guard rejected (redve_set_guard);
                            each is also counted in breakdowns                          */
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
/* Denoiser f (see redve_tnrd_t). Filters must have zero mean (|sum| <= 1e-6 sum|k|);
 * gamma / dmu in [1/3, 2.2]. Packs the MFMA operands and, for BF16, the influence-function
 * tables on the host (FP64), and uploads them: a setup call, not for the solve loop. */
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
/* Base iteration that Algorithm 3 accelerates (Sec. IV runs VE on the FP method and on
 * steepest descent). REDVE_BASE_FP (default): the FP map of eq. (7). REDVE_BASE_SD:
 * x_{k+1} = x_k - mu g(x_k), g = H^T (H x - y) / sigma^2 + lambda (x - f(x)) the gradient of
 * eq. (5), one denoiser call and no CG per step; mu > 0 a fixed step (the paper fixes it by
 * hand), mu <= 0 the default 1 / (||H||^2 / sigma^2 + 2 lambda) with ||H|| <= sum |h|
 * (computed per image in batches). Everything else (extrapolation, stopping, statistics) is
 * the same; "FP call" then counts SD steps. */
int redve_set_base(redve_t h, int base, double mu);
/* BF16 form only: once the relative change of two FP iterates falls below delta (> 0), the
 * remaining FP calls of that solve (of that image, in batches and servers) take the FP32 banks
 * and the FP32 window of the influence functions, so that the last cycles run above the BF16
 * operands' noise and stop at tolerances below it in fewer calls. 0 (default): BF16 banks
 * throughout. The batched engine switches only for denoisers whose FP32 MFMA stage fits 64 KiB
 * of LDS. Negative or non-finite: REDVE_E_ARG. */
int redve_set_precision_switch(redve_t h, double delta);
/* Stability guard (Sec. III-D, eq. (21)): VE is stable when sum_i |gamma_i| stays bounded
 * over the cycles, and the extrapolated vector sum_i gamma_i x_{m+i} carries the iterates'
 * errors magnified by up to that sum. An extrapolation whose sum |gamma| exceeds gamma_cap, or
 * is not finite, is rejected: the cycle continues from its last FP iterate x_{m+L} (as on a
 * breakdown, and counted in breakdowns and rejected). The default, +infinity, rejects only
 * non-finite coefficients (the paper rejects none; windows with sum |gamma| near 1e8 still
 * accelerate steepest descent); a finite cap bounds the magnification, e.g. 1e3 keeps it below
 * the 1e-4 relative bar for iterates rounded to FP32. gamma_cap <= 0 turns the guard off (a
 * non-finite sum then ends the solve with REDVE_E_NONFINITE). Applies to redve_solve,
 * redve_extrapolate(_noalloc), the batched solve and servers created afterwards.
 * NaN: REDVE_E_ARG. */
int redve_set_guard(redve_t h, double gamma_cap);
/* Linear step of the FP call (eq. (7); its footnote allows the Fourier domain for
 * block-circulant H, or iterative methods). REDVE_LIN_CG (default): cg_iters conjugate-
 * gradient iterations, warm-started. REDVE_LIN_FFT: the exact inverse in the Fourier domain,
 * d = F^-1[F(r0) / (|h_hat|^2 / sigma^2 + lambda)] on the FP64-accumulated residual r0, by the
 * library's own FP32 mixed-radix FFT kernels (any side length; lengths with a large prime
 * factor are slower), for deblurring only (decim = 1) and sides up to 4096: solve and fp_step
 * return REDVE_E_ARG otherwise. The batched engine and the server use CG and refuse it. */
int redve_set_linear_solver(redve_t h, int kind);

/* Solve: y (device, hy x wy) -> x (device, hx x wx), hy = ceil(hx/decim), wy = ceil(wx/decim).
 * x0 (device, hx x wx) is the initial vector, or NULL for the default (y when decim = 1,
 * decim^2 H^T y otherwise). x may alias x0. If the budget ends inside a cycle the last FP
 * iterate is returned; a completed cycle returns the extrapolated vector (Algorithm 3).
 * st (host, may be NULL) receives statistics. Returns once the statistics are on the host
 * (the handle waits for its stream after every pass of the loop); the final copy into x is
 * queued on the handle's stream, so work on that stream, or a synchronisation of it, sees x.
 * The observation is copied into the workspace at the start, and each pass of the loop (a
 * full cycle, or one FP call without extrapolation) is recorded into a HIP graph on first use
 * and replayed while the handle's settings and the image size are unchanged. */
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
/* One call of the base iteration: the FP map of eq. (7), out = CG_{cg_iters}(A, b0 + lambda
 * f(x); start x) with b0 = H^T y / sigma^2 computed from y (ceil(hx/decim) x ceil(wx/decim)),
 * or with REDVE_BASE_SD one steepest-descent step out = x - mu g(x). out may not alias x. */
int redve_fp_step(redve_t h, const float* y, const float* x, int hx, int wx, float* out);
/* The RED objective of eq. (4) with the data term of eq. (1): *E (host) =
 * ||Hx - y||^2 / (2 sigma^2) + (lambda / 2) x^T (x - f(x)), one denoiser call, FP64 sums of the
 * FP32 images. y: ceil(hx/decim) x ceil(wx/decim), x: hx x wx (device). Synchronises. */
int redve_objective(redve_t h, const float* y, const float* x, int hx, int wx, double* E);
/* One extrapolation (Algorithm 1 with the configured method) from the L+1 iterates
 * xs[0..L] (device, each hx x wx, stored consecutively): out = x_(0,kappa), or xs[L] if the
 * extrapolation does not exist. gamma (host, L doubles, may be NULL) receives gamma_0..kappa
 * (zeros on breakdown; the rejected values when the stability guard rejected them);
 * *breakdown (host, may be NULL) receives 1 on breakdown or rejection.
 * Synchronises the stream. */
int redve_extrapolate(redve_t h, const float* xs, int L, int hx, int wx, float* out,
                      double* gamma, int* breakdown);

/* ---- launch configuration (autotuning) -------------------------------------------------- */

/* Launch configuration of the single-image path's kernels. Every choice computes the same
 * quantities within the stated tolerances; they differ in speed by image size. */
typedef struct {
    int stage_threads; /* threads per 16x16 tile of the denoiser stage: 512 or 1024           */
    int phi_table;     /* 1: influence functions read from the per-filter cubic tables (BF16
                          banks, 1024 stage threads, tables fitting the LDS), 2: summed on
                          the exact window                                                   */
    int cg_per_launch; /* CG iterations per kernel launch: 1, or 2 (separable square 7x7 or
                          9x9 PSF without decimation, 3 or more iterations)                  */
    int cg_threads;    /* threads per 16x16 tile of the one-iteration CG kernel: 256 or 1024
                          (1024: separable square 7x7 or 9x9 PSF)                            */
    int fused_start;   /* 1: the FP call's last denoiser stage also forms the CG start (needs 2
                          iterations per launch, 1024 stage threads, and tables or FP32
                          banks), 2: a kernel of its own                                     */
    int cg_tile;       /* one-iteration CG kernel: 16 (16x16 tiles, r, A r, A p, p, d kept in
                          HBM) or 32 (32x32 tiles, only r, p, d kept: A r and A p recomputed;
                          separable square 7x7 or 9x9 PSF without decimation)               */
} redve_tuning_t;

enum { REDVE_TUNE_RULES = 0, REDVE_TUNE_AUTO = 1 };

/* REDVE_TUNE_RULES (default): built-in rules by image size (1024-thread stages with tables,
 * two CG iterations per launch and the fused start below 512 tiles). REDVE_TUNE_AUTO: the
 * first redve_solve or redve_fp_step of each problem (image size, denoiser shape and precision,
 * PSF, decimation, CG count, base iteration, linear step) times every valid configuration on
 * one FP call (one warm-up and three timed calls each, HIP events on the handle's stream) and
 * keeps the fastest for later calls. cache_path (may be NULL): a file of JSON lines, one per
 * tuned problem, read now (entries for other problems are kept) and appended to as problems
 * are tuned. */
int redve_set_autotune(redve_t h, int mode, const char* cache_path);
/* Forces a configuration for every later call (fields 0: the rule for that field), validated
 * against what the kernels support (REDVE_E_ARG otherwise); NULL returns to the mode. */
int redve_set_tuning(redve_t h, const redve_tuning_t* t);
/* The configuration the next solve of an hx x wx image would use with the current settings,
 * every field resolved. *us (may be NULL) receives the FP-call time it was tuned with, or -1
 * if it comes from a forced setting or the rules (not tuned yet). */
int redve_get_tuning(redve_t h, int hx, int wx, redve_tuning_t* out, double* us);

/* ---- without device allocation -------------------------------------------------------- */

/* Size of the library's fixed device scratch array (one per GPU, held until the process
 * ends). */
#define REDVE_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): redve_extrapolate with the same arguments, kernels,
 * results and synchronisation, but its difference columns, Gram partials and small-solve
 * result live in the library's fixed scratch array instead of the handle's workspace; it calls
 * no allocating routine. Limit: L * hx * wx <= redve_extrapolate_noalloc_max(L) values
 * (7,831,360 at REDVE_NOALLOC_SCRATCH_BYTES = 32 MiB, e.g. 1024 x 1024 with L = 7), else
 * REDVE_E_ARG with nothing queued. All calls on one GPU share that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (several handles or host threads, or
 * streams not ordered with each other) race and must be serialised by the caller. */
int redve_extrapolate_noalloc(redve_t h, const float* xs, int L, int hx, int wx, float* out,
                              double* gamma, int* breakdown);
/* Largest hx * wx redve_extrapolate_noalloc accepts for window L (0 if L is out of range). */
size_t redve_extrapolate_noalloc_max(int L);

/* ---- batched solve (many images of different sizes in one set of launches) ------------- */

/* One restoration of a batch or a serving request. Device pointers are caller-owned and must
 * stay valid until the call returns (batch) or the request is done (server). */
typedef struct {
    const float* y;     /* device, ceil(hx/decim) x ceil(wx/decim): observation of eq. (1)  */
    const float* x0;    /* device, hx x wx, or NULL: y (decim 1) or decim^2 H^T y            */
    float* x;           /* device, hx x wx: receives the result                              */
    int hx, wx;         /* image size (>= 2 each)                                            */
    const double* psf;  /* host, kh x kw (odd, <= 15): the blur of H = S B (copied by the call
                           or, for the server, at submit)                                  */
    int kh, kw;
    int decim;          /* S: 1 deblurring, 3 super-resolution (1..4)                        */
    double sigma;       /* noise standard deviation of eq. (1), > 0                          */
    double lambda;      /* weight lambda of eq. (2), > 0                                     */
} redve_item_t;

/* Solves n independent problems at once (the denoiser, extrapolation and solver settings of
 * the handle apply to all; the handle's operator, sigma and lambda are not used): every kernel
 * of an FP call (eq. (7)) runs once over a tile list of the running images, each FP call is one
 * replay of a captured HIP graph, and converged images drop out of the list. Reductions are per
 * image, in a fixed order, so each image's result does not depend on the other images in the
 * batch. Waits for the handle's stream before reading the inputs and runs on a stream of the
 * handle's own. The workspace (about 4 (14 + L) bytes per pixel) and the captured graphs are
 * kept in the handle for later calls that fit them with unchanged denoiser, extrapolation and
 * CG settings; otherwise they are rebuilt; redve_destroy frees them. st: n entries (host) or
 * NULL; st[i].status is the item's own outcome. Returns REDVE_OK, an argument/HIP error, or the
 * first non-OK item status. */
int redve_solve_batch(redve_t h, int n, const redve_item_t* items, redve_stats_t* st);

/* ---- serving: continuous batching of arriving requests --------------------------------- */

typedef struct redve_server* redve_server_t;

/* A scheduler thread with its own stream and a copy of proto's denoiser, extrapolation and
 * solver settings (proto must have a denoiser, must outlive the server and must keep its
 * denoiser while the server exists: the denoiser's device buffers are shared). The server allocates its whole workspace here, within
 * hbm_budget bytes (4 (14 + L) bytes per pixel of capacity); requests are admitted in arrival
 * order while their pixels fit (and at most max_active run at once). Every round advances each
 * admitted request by one FP call (one batched launch sequence), extrapolates those that
 * complete a window, retires the finished ones and admits queued ones. Each request's result
 * is the same alone and in any mix. */
int redve_server_create(redve_server_t* out, redve_t proto, size_t hbm_budget, int max_active);
/* Queues a request (does not wait for the GPU); *ticket identifies it. The inputs are read
 * after the work queued so far on proto's stream. The item's device buffers must live until
 * the request is done. REDVE_E_NOMEM: the request could never fit the server's capacity. */
int redve_server_submit(redve_server_t s, const redve_item_t* item, unsigned long long* ticket);
/* *done = 1 once the request finished; st (host, may be NULL) then receives its statistics
 * (st->ms = submit-to-completion latency). */
int redve_server_poll(redve_server_t s, unsigned long long ticket, int* done, redve_stats_t* st);
/* Blocks until the request finished. */
int redve_server_wait(redve_server_t s, unsigned long long ticket, redve_stats_t* st);
/* Requests queued, running, finished so far, and rounds executed. */
int redve_server_counts(redve_server_t s, int* queued, int* active, int* finished, long long* rounds);
/* Admission record: the pixel capacity the budget buys (hbm_budget / (4 (14 + L)) bytes),
 * the most pixels admitted at once so far (each request's range rounded up to 64), which
 * never exceeds it, and the rounds run while a request waited in the queue. */
int redve_server_occupancy(redve_server_t s, size_t* capacity_px, size_t* peak_px,
                           long long* waited_rounds);
/* Waits for every submitted request, stops the scheduler, frees everything. */
int redve_server_destroy(redve_server_t s);

#ifdef __cplusplus
}
#endif
#endif
