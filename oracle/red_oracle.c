/*
 * FP64 CPU oracle for RED restoration by fixed-point iteration (TEST INFRASTRUCTURE ONLY).
 *
 * Plain double-precision reference of "Acceleration of RED via Vector Extrapolation"
 * (Hong, Romano, Elad): the observation model (Sec. II-A, eq. (1)), the FP iteration
 * (Sec. II-B, eq. (7)) with its linear step solved by conjugate gradients (the footnote to
 * eq. (7) allows iterative methods), and a TNRD-style denoiser (Sec. IV names TNRD).
 * Every loop is the definition written out; there is no tiling, fusion or reordering.
 * OpenMP only splits independent outer loops (rows, filters); every reduction is a plain
 * sequential sum, so the results do not depend on the thread count.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg use this file.
 */
#include "red_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

static double* dalloc(size_t n) {
    double* p = (double*)calloc(n ? n : 1, sizeof(double));
    if (!p) abort();
    return p;
}

static double dot(const double* a, const double* b, size_t n) {
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ---------------------------------------------------------------------------------------
 * Degradation operator, eq. (1): y = H x + e with H = B (deblurring) or S B (SR).
 * B is block-circulant (periodic boundary), as the footnote to eq. (7) assumes.
 * ------------------------------------------------------------------------------------- */

void orc_blur(const double* x, int H, int W, const double* psf, int kh, int kw, double* out) {
    const int rh = (kh - 1) / 2, rw = (kw - 1) / 2;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double s = 0.0;
            for (int a = -rh; a <= rh; ++a)
                for (int b = -rw; b <= rw; ++b)
                    s += psf[(a + rh) * kw + (b + rw)] * x[(size_t)wrap(i - a, H) * W + wrap(j - b, W)];
            out[(size_t)i * W + j] = s;
        }
}

void orc_blur_adj(const double* z, int H, int W, const double* psf, int kh, int kw, double* out) {
    const int rh = (kh - 1) / 2, rw = (kw - 1) / 2;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double s = 0.0;
            for (int a = -rh; a <= rh; ++a)
                for (int b = -rw; b <= rw; ++b)
                    s += psf[(a + rh) * kw + (b + rw)] * z[(size_t)wrap(i + a, H) * W + wrap(j + b, W)];
            out[(size_t)i * W + j] = s;
        }
}

void orc_decimate(const double* x, int H, int W, int s, double* out) {
    const int h = (H + s - 1) / s, w = (W + s - 1) / s;
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) out[(size_t)i * w + j] = x[(size_t)(s * i) * W + s * j];
}

void orc_decimate_adj(const double* y, int H, int W, int s, double* out) {
    const int h = (H + s - 1) / s, w = (W + s - 1) / s;
    memset(out, 0, sizeof(double) * (size_t)H * W);
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < w; ++j) out[(size_t)(s * i) * W + s * j] = y[(size_t)i * w + j];
}

void orc_apply_H(const double* x, int H, int W, const double* psf, int kh, int kw, int s,
                 double* out) {
    double* t = dalloc((size_t)H * W);
    orc_blur(x, H, W, psf, kh, kw, t);
    orc_decimate(t, H, W, s, out);
    free(t);
}

void orc_apply_Ht(const double* y, int H, int W, const double* psf, int kh, int kw, int s,
                  double* out) {
    double* t = dalloc((size_t)H * W);
    orc_decimate_adj(y, H, W, s, t);
    orc_blur_adj(t, H, W, psf, kh, kw, out);
    free(t);
}

/* A = H^T H / sigma^2 + lambda I, the matrix inverted in eq. (7). */
void orc_apply_A(const double* p, int H, int W, const double* psf, int kh, int kw, int s,
                 double sigma, double lambda, double* out) {
    const int h = (H + s - 1) / s, w = (W + s - 1) / s;
    double* t = dalloc((size_t)h * w);
    orc_apply_H(p, H, W, psf, kh, kw, s, t);
    orc_apply_Ht(t, H, W, psf, kh, kw, s, out);
    const double is2 = 1.0 / (sigma * sigma);
    for (size_t i = 0; i < (size_t)H * W; ++i) out[i] = is2 * out[i] + lambda * p[i];
    free(t);
}

/* Conjugate gradients (Hestenes-Stiefel), warm-started from x, fixed iteration count.
 * Used for the linear step of eq. (7) (footnote: iterative methods for general H). */
void orc_cg(const double* rhs, double* x, int H, int W, const double* psf, int kh, int kw,
            int s, double sigma, double lambda, int n_iter) {
    const size_t n = (size_t)H * W;
    double* r = dalloc(n);
    double* p = dalloc(n);
    double* q = dalloc(n);
    orc_apply_A(x, H, W, psf, kh, kw, s, sigma, lambda, q);
    for (size_t i = 0; i < n; ++i) r[i] = rhs[i] - q[i];
    memcpy(p, r, sizeof(double) * n);
    double rho0 = dot(r, r, n);
    for (int it = 0; it < n_iter; ++it) {
        if (rho0 <= 1e-300) break;
        orc_apply_A(p, H, W, psf, kh, kw, s, sigma, lambda, q);
        const double alpha = rho0 / dot(p, q, n);
        for (size_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        const double rho1 = dot(r, r, n);
        const double beta = rho1 / rho0;
        for (size_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho0 = rho1;
    }
    free(r);
    free(p);
    free(q);
}

/* ---------------------------------------------------------------------------------------
 * TNRD-style denoiser f (Sec. II-B; Sec. IV uses TNRD): T gradient-type diffusion stages
 *   u_t = u_{t-1} - sum_i K_{t,i}^T phi_{t,i}(K_{t,i} u_{t-1}) - theta_t (u_{t-1} - f)
 * with K u = 'valid' correlation of the symmetric extension of u with a k x k filter.
 * ------------------------------------------------------------------------------------- */

/* Half-sample symmetric mirror: -1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2. */
static int mirror(int i, int n) {
    if (i < 0) return -i - 1;
    if (i >= n) return 2 * n - i - 1;
    return i;
}

void orc_filter_fwd(const double* u, int H, int W, const double* k, int ks, double* out) {
    const int r = (ks - 1) / 2;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double s = 0.0;
            for (int a = -r; a <= r; ++a)
                for (int b = -r; b <= r; ++b)
                    s += k[(a + r) * ks + (b + r)] * u[(size_t)mirror(i + a, H) * W + mirror(j + b, W)];
            out[(size_t)i * W + j] = s;
        }
}

/* K = C E with E the extension (H x W -> (H+2r) x (W+2r)) and C the valid correlation.
 * K^T v = E^T (C^T v): scatter every v[i,j] k[a,b] onto extended position (i+a, j+b), then
 * fold each extended position back onto the pixel it mirrors. */
void orc_filter_adj(const double* v, int H, int W, const double* k, int ks, double* out) {
    const int r = (ks - 1) / 2;
    const int He = H + 2 * r, We = W + 2 * r;
    double* e = dalloc((size_t)He * We);
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j)
            for (int a = -r; a <= r; ++a)
                for (int b = -r; b <= r; ++b)
                    e[(size_t)(i + a + r) * We + (j + b + r)] += k[(a + r) * ks + (b + r)] * v[(size_t)i * W + j];
    memset(out, 0, sizeof(double) * (size_t)H * W);
    for (int ie = 0; ie < He; ++ie)
        for (int je = 0; je < We; ++je)
            out[(size_t)mirror(ie - r, H) * W + mirror(je - r, W)] += e[(size_t)ie * We + je];
    free(e);
}

double orc_phi(double z, const double* w, int J, double mu0, double dmu, double gamma) {
    double s = 0.0;
    for (int j = 0; j < J; ++j) {
        const double d = z - (mu0 + dmu * j);
        s += w[j] * exp(-d * d / (2.0 * gamma * gamma));
    }
    return s;
}

void orc_tnrd_stage(const double* u, const double* f, int H, int W, const orc_tnrd_t* p,
                    int t, double* u_out) {
    const size_t n = (size_t)H * W;
    const int F = p->nfilt, ks = p->ksize, J = p->nrbf;
    double* g = dalloc(n * (size_t)F); /* K_i^T phi_i(K_i u), one plane per filter */
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < F; ++i) {
        const double* k = p->filters + ((size_t)t * F + i) * ks * ks;
        const double* w = p->rbf_w + ((size_t)t * F + i) * J;
        double* z = dalloc(n);
        orc_filter_fwd(u, H, W, k, ks, z);
        for (size_t q = 0; q < n; ++q) z[q] = orc_phi(z[q], w, J, p->mu0, p->dmu, p->gamma);
        orc_filter_adj(z, H, W, k, ks, g + (size_t)i * n);
        free(z);
    }
    const double th = p->react[t];
    for (size_t q = 0; q < n; ++q) {
        double s = 0.0;
        for (int i = 0; i < F; ++i) s += g[(size_t)i * n + q];
        u_out[q] = u[q] - s - th * (u[q] - f[q]);
    }
    free(g);
}

void orc_denoise(const double* x, int H, int W, const orc_tnrd_t* p, double* out) {
    const size_t n = (size_t)H * W;
    double* u = dalloc(n);
    double* un = dalloc(n);
    memcpy(u, x, sizeof(double) * n);
    for (int t = 0; t < p->stages; ++t) {
        orc_tnrd_stage(u, x, H, W, p, t, un);
        double* tmp = u;
        u = un;
        un = tmp;
    }
    memcpy(out, u, sizeof(double) * n);
    free(u);
    free(un);
}

/* ---------------------------------------------------------------------------------------
 * One FP call, eq. (7): x_{k+1} = [H^T H / sigma^2 + lambda I]^{-1} [H^T y / sigma^2 +
 * lambda f(x_k)], the inverse applied by n_cg CG iterations warm-started at x_k.
 * ------------------------------------------------------------------------------------- */
void orc_fp_step(const double* x, const double* b0, int H, int W, const double* psf, int kh,
                 int kw, int s, double sigma, double lambda, int n_cg, const orc_tnrd_t* p,
                 double* x_next) {
    const size_t n = (size_t)H * W;
    double* rhs = dalloc(n);
    orc_denoise(x, H, W, p, rhs);
    for (size_t i = 0; i < n; ++i) rhs[i] = b0[i] + lambda * rhs[i];
    memcpy(x_next, x, sizeof(double) * n);
    orc_cg(rhs, x_next, H, W, psf, kh, kw, s, sigma, lambda, n_cg);
    free(rhs);
}
