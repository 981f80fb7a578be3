/*
 * FP64 CPU oracle for RED restoration by fixed-point iteration (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, obviously correct double-precision reference of the operators used by the
 * fixed-point (FP) iteration of RED (Hong, Romano, Elad, "Acceleration of RED via Vector
 * Extrapolation", Sec. II-B, eq. (7)). Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it; the GPU library never does. It shares no code with the GPU
 * path.
 *
 * Images are row-major, H rows by W columns, values on the [0,255] scale.
 */
#ifndef RED_ORACLE_H
#define RED_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Number of OpenMP threads the oracle runs with (1 when built without OpenMP). */
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Blur with a kh x kw PSF (odd sizes), periodic boundary (block-circulant H, footnote to
 * eq. (7)): out[i,j] = sum_{a,b} psf[a+rh, b+rw] x[(i-a) mod H, (j-b) mod W]. */
void orc_blur(const double* x, int H, int W, const double* psf, int kh, int kw, double* out);
/* Adjoint of orc_blur: out[i,j] = sum_{a,b} psf[a+rh, b+rw] z[(i+a) mod H, (j+b) mod W]. */
void orc_blur_adj(const double* z, int H, int W, const double* psf, int kh, int kw, double* out);
/* Decimation by s keeping samples (s*i, s*j); out is ceil(H/s) x ceil(W/s). */
void orc_decimate(const double* x, int H, int W, int s, double* out);
/* Adjoint of orc_decimate: zero-fill onto the H x W grid. */
void orc_decimate_adj(const double* y, int H, int W, int s, double* out);
/* Degradation operator H = S B (s = 1: plain blur), eq. (1). out: ceil(H/s) x ceil(W/s). */
void orc_apply_H(const double* x, int H, int W, const double* psf, int kh, int kw, int s,
                 double* out);
/* H^T y = B^T S^T y. out: H x W. */
void orc_apply_Ht(const double* y, int H, int W, const double* psf, int kh, int kw, int s,
                  double* out);
/* System matrix of eq. (7): out = H^T H p / sigma^2 + lambda p. */
void orc_apply_A(const double* p, int H, int W, const double* psf, int kh, int kw, int s,
                 double sigma, double lambda, double* out);
/* n_iter conjugate-gradient iterations (Hestenes-Stiefel, no preconditioner) on
 * A x = rhs, starting from the x passed in (warm start); x is overwritten. */
void orc_cg(const double* rhs, double* x, int H, int W, const double* psf, int kh, int kw,
            int s, double sigma, double lambda, int n_iter);

/* TNRD-style denoiser parameters (T stages, F filters of k x k per stage, J RBF centres
 * mu_j = mu0 + j*dmu of width gamma, reaction weights theta_t). */
typedef struct {
    int stages, nfilt, ksize, nrbf;
    double mu0, dmu, gamma;
    const double* filters; /* T*F*k*k */
    const double* rbf_w;   /* T*F*J   */
    const double* react;   /* T       */
} orc_tnrd_t;

/* Forward filter: correlation of the symmetric (half-sample mirror) extension of u with k,
 * 'valid' part, H x W output. */
void orc_filter_fwd(const double* u, int H, int W, const double* k, int ks, double* out);
/* Exact adjoint of orc_filter_fwd (full convolution, then the extension's transpose folds
 * the border contributions back onto their mirror sources). */
void orc_filter_adj(const double* v, int H, int W, const double* k, int ks, double* out);
/* Influence function phi(z) = sum_j w_j exp(-(z - mu_j)^2 / (2 gamma^2)). */
double orc_phi(double z, const double* w, int J, double mu0, double dmu, double gamma);
/* One diffusion stage t: u_out = u - sum_i K_i^T phi_i(K_i u) - theta_t (u - f). */
void orc_tnrd_stage(const double* u, const double* f, int H, int W, const orc_tnrd_t* p,
                    int t, double* u_out);
/* Denoiser D(x) = u_T with u_0 = f = x. */
void orc_denoise(const double* x, int H, int W, const orc_tnrd_t* p, double* out);

/* One FP call, eq. (7): x_next = CG_{n_cg}(A, b0 + lambda D(x); start x). */
void orc_fp_step(const double* x, const double* b0, int H, int W, const double* psf, int kh,
                 int kw, int s, double sigma, double lambda, int n_cg, const orc_tnrd_t* p,
                 double* x_next);

#ifdef __cplusplus
}
#endif
#endif
