// Exact linear step of eq. (7) for periodic deblurring. With H = B block-circulant (the footnote
// to eq. (7)), A = H^T H / sigma^2 + lambda I is diagonal in the 2-D DFT basis with eigenvalues
// |h_hat(u, v)|^2 / sigma^2 + lambda, so the FP call's correction is
//   d = F^-1[ F(r0) / (|h_hat|^2 / sigma^2 + lambda) ],  x_{k+1} = x_k + d,
// with r0 = H^T (y - H x_k) / sigma^2 + lambda (f(x_k) - x_k) from the CG start kernel (FP64
// sums). The transforms are rocFFT's single-precision real-to-complex and complex-to-real
// plans on the half spectrum H x (W/2 + 1); the scale 1 / (A_hat H W) (eigenvalue and the
// inverse transform's normalisation) is built on the GPU in FP64 from the PSF, once per image
// size and operator.
#include <math.h>
#include <rocfft/rocfft.h>

#include <mutex>

#include "context.h"

using namespace redve;

namespace {

// scale[u][v] = 1 / ((|h_hat(u, v)|^2 / sigma^2 + lambda) H W), h_hat the DFT of the PSF placed
// with its centre at the origin (circular convolution, tap (a, b) at offset (a - kh/2, b - kw/2)).
__global__ __launch_bounds__(256) void k_fft_scale(const double* __restrict__ psf, int kh, int kw,
                                                   int H, int W, double inv_s2, double lambda,
                                                   float* __restrict__ scale) {
    const int wc = W / 2 + 1;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= H * wc) return;
    const int u = idx / wc, v = idx % wc;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < kh; ++a)
        for (int b = 0; b < kw; ++b) {
            // phase of offset (da, db), in half turns (sincospi), reduced to (-1, 1]
            const long pa = (long)u * (a - kh / 2), pb = (long)v * (b - kw / 2);
            const double t = 2.0 * ((double)(pa % H) / H + (double)(pb % W) / W);
            double sn, cs;
            sincospi(t, &sn, &cs);
            const double hv = psf[a * kw + b];
            re += hv * cs;
            im -= hv * sn;
        }
    scale[idx] = (float)(1.0 / (((re * re + im * im) * inv_s2 + lambda) * (double)H * W));
}

__global__ __launch_bounds__(256) void k_fft_apply(float2* __restrict__ spec,
                                                   const float* __restrict__ scale, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float s = scale[i];
    float2 z = spec[i];
    z.x *= s;
    z.y *= s;
    spec[i] = z;
}

__global__ __launch_bounds__(256) void k_add(const float* __restrict__ x,
                                             const float* __restrict__ d, float* __restrict__ out,
                                             int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = x[i] + d[i];
}

// Plans, work buffer, spectrum and scale for one image size and operator.
struct FftSolve {
    int H = 0, W = 0;
    unsigned long long op_gen = ~0ull;
    rocfft_plan fwd = nullptr, inv = nullptr;
    rocfft_execution_info info = nullptr;
    void* work = nullptr;
    size_t work_bytes = 0;
    float2* spec = nullptr;
    float* scale = nullptr;

    ~FftSolve() {
        if (fwd) rocfft_plan_destroy(fwd);
        if (inv) rocfft_plan_destroy(inv);
        if (info) rocfft_execution_info_destroy(info);
        if (work) hipFree(work);
        if (spec) hipFree(spec);
        if (scale) hipFree(scale);
    }
};

std::once_flag g_rocfft_once;

int make_plans(redve_t h, FftSolve& f, int H, int W) {
    std::call_once(g_rocfft_once, [] { rocfft_setup(); });
    const size_t len[2] = {(size_t)W, (size_t)H};  // fastest dimension first
    if (rocfft_plan_create(&f.fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                           rocfft_precision_single, 2, len, 1, nullptr) != rocfft_status_success ||
        rocfft_plan_create(&f.inv, rocfft_placement_notinplace, rocfft_transform_type_real_inverse,
                           rocfft_precision_single, 2, len, 1, nullptr) != rocfft_status_success ||
        rocfft_execution_info_create(&f.info) != rocfft_status_success) {
        h->err = "rocFFT plan creation failed";
        return REDVE_E_HIP;
    }
    size_t w1 = 0, w2 = 0;
    rocfft_plan_get_work_buffer_size(f.fwd, &w1);
    rocfft_plan_get_work_buffer_size(f.inv, &w2);
    f.work_bytes = std::max(w1, w2);
    const size_t nspec = (size_t)H * (W / 2 + 1);
    if ((f.work_bytes && hipMalloc(&f.work, f.work_bytes) != hipSuccess) ||
        hipMalloc(&f.spec, nspec * sizeof(float2)) != hipSuccess ||
        hipMalloc(&f.scale, nspec * sizeof(float)) != hipSuccess) {
        h->err = "FFT workspace allocation failed";
        return REDVE_E_NOMEM;
    }
    if (f.work_bytes &&
        rocfft_execution_info_set_work_buffer(f.info, f.work, f.work_bytes) != rocfft_status_success)
        return REDVE_E_HIP;
    f.H = H;
    f.W = W;
    return REDVE_OK;
}

}  // namespace

// d = F^-1[F(r0) / A_hat], x_out = x_in + d (d in the workspace). r0 may be overwritten.
int redve_fft_correction(redve_t h, float* r0, const float* x_in, float* x_out, float* d, int H,
                         int W) {
    FftSolve* f = (FftSolve*)h->fft;
    if (f && (f->H != H || f->W != W)) {
        h->fft_free(f);
        f = nullptr;
        h->fft = nullptr;
    }
    if (!f) {
        f = new FftSolve();
        h->fft = f;
        h->fft_free = [](void* p) { delete (FftSolve*)p; };
        const int rc = make_plans(h, *f, H, W);
        if (rc) return rc;
    }
    const int nspec = H * (W / 2 + 1), n = H * W;
    if (f->op_gen != h->op_gen) {
        k_fft_scale<<<(nspec + 255) / 256, 256, 0, h->stream>>>(
            h->d_psf64, h->kh, h->kw, H, W, 1.0 / (h->sigma * h->sigma), h->lambda, f->scale);
        if (hipGetLastError() != hipSuccess) return REDVE_E_HIP;
        f->op_gen = h->op_gen;
    }
    if (rocfft_execution_info_set_stream(f->info, h->stream) != rocfft_status_success)
        return REDVE_E_HIP;
    void* in1[1] = {r0};
    void* out1[1] = {f->spec};
    if (rocfft_execute(f->fwd, in1, out1, f->info) != rocfft_status_success) return REDVE_E_HIP;
    k_fft_apply<<<(nspec + 255) / 256, 256, 0, h->stream>>>(f->spec, f->scale, nspec);
    void* in2[1] = {f->spec};
    void* out2[1] = {d};
    if (rocfft_execute(f->inv, in2, out2, f->info) != rocfft_status_success) return REDVE_E_HIP;
    k_add<<<(n + 255) / 256, 256, 0, h->stream>>>(x_in, d, x_out, n);
    return hipGetLastError() == hipSuccess ? REDVE_OK : REDVE_E_HIP;
}
