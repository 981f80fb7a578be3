// Exact linear step of eq. (7) for periodic deblurring, on hand-written FFT kernels. With
// H = B block-circulant (the footnote to eq. (7)), A = H^T H / sigma^2 + lambda I is diagonal in
// the 2-D DFT basis with eigenvalues |h_hat(u, v)|^2 / sigma^2 + lambda, so the FP call's
// correction is
//   d = F^-1[ F(r0) / (|h_hat|^2 / sigma^2 + lambda) ],  x_{k+1} = x_k + d,
// with r0 = H^T (y - H x_k) / sigma^2 + lambda (f(x_k) - x_k) from the CG start kernel (FP64
// sums). Three launches per FP call:
//   rows, forward: two real rows packed as one complex row z = a + i b, one FFT of length W
//     in LDS, split into the half spectra of a and b (Hermitian symmetry), H x (W/2 + 1);
//   columns: blocks of adjacent spectrum columns in LDS, forward FFT of length H, times the
//     real factor 1 / (A_hat H W), inverse FFT (the spectrum never leaves the workgroup);
//   rows, inverse: the two half spectra recombined into one complex row, inverse FFT, and
//     x_out = x_in + d written from its real and imaginary parts.
// The transforms are a self-sorting (Stockham) mixed-radix FFT in one LDS buffer: each radix-p
// stage reads every element into registers, waits for the workgroup, and writes the p outputs
// of each butterfly to their sorted places, so no bit reversal and no second buffer. Radices
// 4, 2, 3 and 5 have closed-form butterflies; any other prime factor takes a direct DFT per
// output (its cost grows with the factor, so lengths with a large prime factor are slow but
// exact). Twiddles w_N^e = exp(-2 pi i e / N) come from per-length tables computed in FP64 on
// the host and rounded to FP32, which each workgroup copies into LDS beside its data (a stage
// reads them there instead of from memory); arithmetic is FP32 (relative error of order
// log2(N) 2^-24).
#include <math.h>

#include <type_traits>
#include <vector>

#include "context.h"

using namespace redve;

namespace redve {
namespace {

constexpr int kFftMaxStages = 24;
constexpr int kFftMaxSide = 4096;   // W: 256 threads x 16 elements; H: 512 threads x 8
constexpr int kColThreads = 512;
// complex elements per thread and stage: the registers a stage holds grow with it, so the column
// pass takes 8 (under 128 registers: two workgroups of 512 threads per CU, against one with 16)
constexpr int kColElems = 8;
static_assert(kColThreads * kColElems >= kFftMaxSide, "a workgroup holds a whole column");

// Radix stages of one transform length.
struct FftPlan {
    int n, nrad;
    int rad[kFftMaxStages];
};

FftPlan make_plan(int n) {
    FftPlan p{};
    p.n = n;
    int m = n;
    auto take = [&](int r) {
        while (m % r == 0) {
            p.rad[p.nrad++] = r;
            m /= r;
        }
    };
    take(4);
    take(2);
    take(3);
    take(5);
    int r = 7;
    while (m > 1) {  // take() divides m by every factor r it finds
        take(r);
        r += 2;
    }
    return p;
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiplication by -i (forward) or +i (inverse)
__device__ inline float2 rot(float2 a, bool inv) {
    return inv ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// y_k = sum_q a_q w_P^{q k}, w_P = exp(-+ 2 pi i / P), closed forms for P = 2, 3, 4, 5.
template <int P>
__device__ inline void dft(const float2 (&a)[P], float2 (&y)[P], bool inv) {
    if constexpr (P == 2) {
        y[0] = cadd(a[0], a[1]);
        y[1] = csub(a[0], a[1]);
    } else if constexpr (P == 4) {
        const float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
        const float2 s13 = cadd(a[1], a[3]), d13 = rot(csub(a[1], a[3]), inv);
        y[0] = cadd(s02, s13);
        y[1] = cadd(d02, d13);
        y[2] = csub(s02, s13);
        y[3] = csub(d02, d13);
    } else if constexpr (P == 3) {
        constexpr float h = 0.86602540378443865f;  // sin(2 pi / 3)
        const float2 t = cadd(a[1], a[2]);
        const float2 m0 = make_float2(a[0].x - 0.5f * t.x, a[0].y - 0.5f * t.y);
        const float2 s = rot(csub(a[1], a[2]), inv);  // -+ i (a1 - a2)
        y[0] = cadd(a[0], t);
        y[1] = make_float2(m0.x + h * s.x, m0.y + h * s.y);
        y[2] = make_float2(m0.x - h * s.x, m0.y - h * s.y);
    } else {
        static_assert(P == 5, "closed-form radices: 2, 3, 4, 5");
        // cos and sin of 2 pi k / 5
        constexpr float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
        constexpr float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
        const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
        const float2 u1 = rot(csub(a[1], a[4]), inv), u2 = rot(csub(a[2], a[3]), inv);
        y[0] = cadd(a[0], cadd(t1, t2));
        const float2 p1 = make_float2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
        const float2 p2 = make_float2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
        const float2 q1 = make_float2(s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y);
        const float2 q2 = make_float2(s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y);
        y[1] = cadd(p1, q1);
        y[4] = csub(p1, q1);
        y[2] = cadd(p2, q2);
        y[3] = csub(p2, q2);
    }
}

__device__ inline float2 twiddle(const float2* __restrict__ tw, int e, bool inv) {
    const float2 t = tw[e];
    return inv ? make_float2(t.x, -t.y) : t;
}

// One Stockham stage of radix P on NC = 2^lgnc interleaved transforms of length N in LDS
// (element i of transform c at X[i NC + c]). Before the stage the data are the DFTs of length
// l of the m = N / l decimated subsequences; butterfly (c', k1), c' < m / P, k1 < l, reads
// a_q = X[k1 m + c' + (m / P) q], twiddles it by w_N^{q k1 m / P} and writes its P outputs to
// X[(k1 + l k2) (m / P) + c'].
template <int P, int NT, int EL>
__device__ inline void stage(float2* X, int N, int lgnc, int l, int m,
                             const float2* __restrict__ tw, bool inv) {
    constexpr int NB = (EL + P - 1) / P;  // butterflies per thread
    const int mp = m / P;
    const int nbf = (N / P) << lgnc;
    float2 y[NB][P];
    int o[NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
        const int b = threadIdx.x + bi * NT;
        o[bi] = -1;
        if (b < nbf) {
            const int c = b & ((1 << lgnc) - 1), bb = b >> lgnc;
            const int cp = bb % mp, k1 = bb / mp;
            float2 a[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const float2 v = X[((k1 * m + cp + mp * q) << lgnc) + c];
                a[q] = q ? cmul(v, twiddle(tw, q * k1 * mp, inv)) : v;
            }
            dft<P>(a, y[bi], inv);
            o[bi] = ((k1 * mp + cp) << lgnc) + c;
        }
    }
    __syncthreads();
    const int ostep = (l * mp) << lgnc;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
        if (o[bi] >= 0) {
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) X[o[bi] + k2 * ostep] = y[bi][k2];
        }
    __syncthreads();
}

// A stage of any prime radix p: each output is the direct sum over its p inputs, with the
// combined twiddle w_N^{q k1 m/p + ((q k2) mod p) N/p}.
template <int NT, int EL>
__device__ inline void stage_any(float2* X, int N, int lgnc, int p, int l, int m,
                                 const float2* __restrict__ tw, bool inv) {
    const int mp = m / p, np = N / p;
    const int total = N << lgnc;
    float2 y[EL];
    int o[EL];
#pragma unroll
    for (int e = 0; e < EL; ++e) {
        const int oi = threadIdx.x + e * NT;
        o[e] = -1;
        if (oi < total) {
            const int c = oi & ((1 << lgnc) - 1), t = oi >> lgnc;
            const int cp = t % mp, kk = t / mp, k1 = kk % l, k2 = kk / l;
            float2 acc = make_float2(0.f, 0.f);
            int e1 = 0, e2 = 0;  // q k1 mp and ((q k2) mod p) np
            for (int q = 0; q < p; ++q) {
                const float2 v = X[((k1 * m + cp + mp * q) << lgnc) + c];
                int ex = e1 + e2;
                ex = ex >= N ? ex - N : ex;
                const float2 t2 = twiddle(tw, ex, inv);
                acc.x += v.x * t2.x - v.y * t2.y;
                acc.y += v.x * t2.y + v.y * t2.x;
                e1 += k1 * mp;
                e2 += k2 * np;
                e2 = e2 >= N ? e2 - N : e2;
            }
            y[e] = acc;
            o[e] = oi;
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EL; ++e)
        if (o[e] >= 0) X[o[e]] = y[e];
    __syncthreads();
}

// The whole transform (forward: w = exp(-2 pi i / N); inverse: conjugate, unnormalised).
// Expects the data in X and a workgroup barrier behind; ends with one.
template <int NT, int EL>
__device__ inline void fft_lds(float2* X, int lgnc, const FftPlan& plan,
                               const float2* __restrict__ tw, bool inv) {
    const int N = plan.n;
    int l = 1, m = N;
    for (int s = 0; s < plan.nrad; ++s) {
        const int p = plan.rad[s];
        switch (p) {
            case 4: stage<4, NT, EL>(X, N, lgnc, l, m, tw, inv); break;
            case 2: stage<2, NT, EL>(X, N, lgnc, l, m, tw, inv); break;
            case 3: stage<3, NT, EL>(X, N, lgnc, l, m, tw, inv); break;
            case 5: stage<5, NT, EL>(X, N, lgnc, l, m, tw, inv); break;
            default: stage_any<NT, EL>(X, N, lgnc, p, l, m, tw, inv); break;
        }
        l *= p;
        m /= p;
    }
}

// Rows 2g and 2g + 1 of r (the second may be absent) -> their half spectra in spec (H x wc).
template <int NT, int EL>
__global__ __launch_bounds__(NT) void k_fft_rows_fwd(const float* __restrict__ r, int H,
                                                             int W, FftPlan plan,
                                                             const float2* __restrict__ tw,
                                                             float2* __restrict__ spec) {
    extern __shared__ float2 X[];  // the row, then the twiddles
    float2* T = X + W;
    const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
    const bool two = r1 < H;
    for (int j = threadIdx.x; j < W; j += NT) {
        X[j] = make_float2(r[(size_t)r0 * W + j], two ? r[(size_t)r1 * W + j] : 0.f);
        T[j] = tw[j];
    }
    __syncthreads();
    fft_lds<NT, EL>(X, 0, plan, T, false);
    // Z = F(a + i b): A_k = (Z_k + conj Z_{-k}) / 2, B_k = (Z_k - conj Z_{-k}) / (2 i)
    const int wc = W / 2 + 1;
    for (int k = threadIdx.x; k < wc; k += NT) {
        const float2 z = X[k], w = X[k == 0 ? 0 : W - k];
        spec[(size_t)r0 * wc + k] = make_float2(0.5f * (z.x + w.x), 0.5f * (z.y - w.y));
        if (two) spec[(size_t)r1 * wc + k] = make_float2(0.5f * (z.y + w.y), 0.5f * (w.x - z.x));
    }
}

// Columns [c0, c0 + 2^lgnc) of the half spectrum: forward FFT of length H, times scale
// (1 / (A_hat H W)), inverse FFT. Blocks of adjacent columns go to the same XCD (xcd_tile):
// a block reads 2^lgnc x 8 bytes of each spectrum row, less than a cache line for narrow
// blocks on tall images, and its neighbours on the same L2 read the rest of the line. Bounded
// to 80 registers (six waves per SIMD): three workgroups fit a CU, so the 513 blocks of a
// 2048-row image run at once.
__global__ __launch_bounds__(kColThreads, 6) void k_fft_cols(float2* __restrict__ spec,
                                                         const float* __restrict__ scale, int H,
                                                         int wc, int lgnc, FftPlan plan,
                                                         const float2* __restrict__ tw) {
    extern __shared__ float2 X[];  // the columns, then the twiddles
    const int nc = 1 << lgnc, c0 = xcd_tile(blockIdx.x, gridDim.x) * nc;
    const int total = H << lgnc;
    float2* T = X + total;
    for (int e = threadIdx.x; e < total; e += kColThreads) {
        const int i = e >> lgnc, c = c0 + (e & (nc - 1));
        X[e] = c < wc ? spec[(size_t)i * wc + c] : make_float2(0.f, 0.f);
    }
    for (int e = threadIdx.x; e < H; e += kColThreads) T[e] = tw[e];
    __syncthreads();
    fft_lds<kColThreads, kColElems>(X, lgnc, plan, T, false);
    for (int e = threadIdx.x; e < total; e += kColThreads) {
        const int i = e >> lgnc, c = c0 + (e & (nc - 1));
        const float s = c < wc ? scale[(size_t)i * wc + c] : 0.f;
        X[e] = make_float2(X[e].x * s, X[e].y * s);
    }
    __syncthreads();
    fft_lds<kColThreads, kColElems>(X, lgnc, plan, T, true);
    for (int e = threadIdx.x; e < total; e += kColThreads) {
        const int i = e >> lgnc, c = c0 + (e & (nc - 1));
        if (c < wc) spec[(size_t)i * wc + c] = X[e];
    }
}

// Rows 2g and 2g + 1: Z = A + i B on the full length (A_{W-k} = conj A_k), inverse FFT, and
// x_out = x_in + (Re z, Im z) on the two rows.
template <int NT, int EL>
__global__ __launch_bounds__(NT) void k_fft_rows_inv(const float2* __restrict__ spec,
                                                             const float* __restrict__ x_in,
                                                             float* __restrict__ x_out, int H,
                                                             int W, FftPlan plan,
                                                             const float2* __restrict__ tw) {
    extern __shared__ float2 X[];  // the row, then the twiddles
    float2* T = X + W;
    const int r0 = 2 * blockIdx.x, r1 = r0 + 1;
    const bool two = r1 < H;
    const int wc = W / 2 + 1;
    for (int j = threadIdx.x; j < W; j += NT) {
        T[j] = tw[j];
        const bool lo = j < wc;
        const int k = lo ? j : W - j;
        float2 a = spec[(size_t)r0 * wc + k];
        float2 b = two ? spec[(size_t)r1 * wc + k] : make_float2(0.f, 0.f);
        if (!lo) {
            a.y = -a.y;
            b.y = -b.y;
        }
        X[j] = make_float2(a.x - b.y, a.y + b.x);
    }
    __syncthreads();
    fft_lds<NT, EL>(X, 0, plan, T, true);
    for (int j = threadIdx.x; j < W; j += NT) {
        const float2 z = X[j];
        x_out[(size_t)r0 * W + j] = x_in[(size_t)r0 * W + j] + z.x;
        if (two) x_out[(size_t)r1 * W + j] = x_in[(size_t)r1 * W + j] + z.y;
    }
}

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

// Columns per block of the column pass: two where the block fits the workgroup's elements
// (H <= 2048), else one. Wider blocks read longer row segments but give fewer workgroups: at
// 256x256 (129 columns) 16 columns per block left 9 workgroups for the whole pass (16.2 us
// against 8.8 us with two), at 2048x2048 four columns per block took 74.8 us against 70.8 us.
int col_lgnc(int H) { return (H << 1) <= kColThreads * kColElems ? 1 : 0; }

// Tables and buffers for one image size and operator.
struct FftSolve {
    int H = 0, W = 0;
    unsigned long long op_gen = ~0ull;
    FftPlan ph{}, pw{};
    float2 *tw_h = nullptr, *tw_w = nullptr;
    float2* spec = nullptr;
    float* scale = nullptr;

    ~FftSolve() {  // teardown: a failed free leaves nothing to recover
        (void)hipFree(tw_h);
        (void)hipFree(tw_w);
        (void)hipFree(spec);
        (void)hipFree(scale);
    }
};

int upload_twiddles(int n, float2** out, hipStream_t st) {
    std::vector<float2> t(n);
    for (int e = 0; e < n; ++e) {
        const double ang = 2.0 * 3.14159265358979323846 * (double)e / n;
        t[e] = make_float2((float)cos(ang), (float)-sin(ang));
    }
    if (hipMalloc(out, sizeof(float2) * n) != hipSuccess) return REDVE_E_NOMEM;
    if (hipMemcpyAsync(*out, t.data(), sizeof(float2) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return REDVE_E_HIP;
    return REDVE_OK;
}

int make_solve(redve_t h, FftSolve& f, int H, int W) {
    f.H = H;
    f.W = W;
    f.ph = make_plan(H);
    f.pw = make_plan(W);
    int rc;
    if ((rc = upload_twiddles(H, &f.tw_h, h->stream)) || (rc = upload_twiddles(W, &f.tw_w, h->stream)))
        return rc;
    const size_t nspec = (size_t)H * (W / 2 + 1);
    if (hipMalloc(&f.spec, nspec * sizeof(float2)) != hipSuccess ||
        hipMalloc(&f.scale, nspec * sizeof(float)) != hipSuccess)
        return REDVE_E_NOMEM;
    return REDVE_OK;
}

}  // namespace
}  // namespace redve

bool redve_fft_size_ok(int H, int W) { return H <= kFftMaxSide && W <= kFftMaxSide; }

// d = F^-1[F(r0) / A_hat], x_out = x_in + d. r0 is read only.
int redve_fft_correction(redve_t h, float* r0, const float* x_in, float* x_out, float* d, int H,
                         int W) {
    (void)d;
    if (!redve_fft_size_ok(H, W)) {
        h->err = "the Fourier linear step supports sides up to 4096";
        return REDVE_E_ARG;
    }
    FftSolve* f = (FftSolve*)h->fft;
    if (f && (f->H != H || f->W != W)) {
        // the buffers of the old size may still be in use by queued work
        if (hipStreamSynchronize(h->stream) != hipSuccess) return REDVE_E_HIP;
        h->fft_free(f);
        f = nullptr;
        h->fft = nullptr;
    }
    if (!f) {
        f = new FftSolve();
        h->fft = f;
        h->fft_free = [](void* p) { delete (FftSolve*)p; };
        const int rc = make_solve(h, *f, H, W);
        if (rc) {
            h->err = "Fourier step set-up failed";
            return rc;
        }
    }
    const int wc = W / 2 + 1, nspec = H * wc;
    if (f->op_gen != h->op_gen) {
        k_fft_scale<<<(nspec + 255) / 256, 256, 0, h->stream>>>(
            h->d_psf64, h->kh, h->kw, H, W, 1.0 / (h->sigma * h->sigma), h->lambda, f->scale);
        if (hipGetLastError() != hipSuccess) return REDVE_E_HIP;
        f->op_gen = h->op_gen;
    }
    const int rows = (H + 1) / 2;
    const size_t row_lds = sizeof(float2) * 2 * W;  // a row and its twiddles
    const int lgnc = col_lgnc(H);
    const size_t col_lds = sizeof(float2) * (((size_t)H << lgnc) + H);  // columns, twiddles
    // rows: four elements per thread on sides up to 2048 (256 or 512 threads), eight beyond
    const auto rows_fwd = [&](auto nt, auto el) {
        k_fft_rows_fwd<decltype(nt)::value, decltype(el)::value>
            <<<rows, decltype(nt)::value, row_lds, h->stream>>>(r0, H, W, f->pw, f->tw_w, f->spec);
    };
    const auto rows_inv = [&](auto nt, auto el) {
        k_fft_rows_inv<decltype(nt)::value, decltype(el)::value>
            <<<rows, decltype(nt)::value, row_lds, h->stream>>>(f->spec, x_in, x_out, H, W, f->pw,
                                                                f->tw_w);
    };
    using I256 = std::integral_constant<int, 256>;
    using I512 = std::integral_constant<int, 512>;
    using E4 = std::integral_constant<int, 4>;
    using E8 = std::integral_constant<int, 8>;
    static_assert(512 * 8 >= kFftMaxSide, "a workgroup holds a whole row");
    if (W <= 1024)
        rows_fwd(I256{}, E4{});
    else if (W <= 2048)
        rows_fwd(I512{}, E4{});
    else
        rows_fwd(I512{}, E8{});
    k_fft_cols<<<(wc + (1 << lgnc) - 1) >> lgnc, kColThreads, col_lds, h->stream>>>(
        f->spec, f->scale, H, wc, lgnc, f->ph, f->tw_h);
    if (W <= 1024)
        rows_inv(I256{}, E4{});
    else if (W <= 2048)
        rows_inv(I512{}, E4{});
    else
        rows_inv(I512{}, E8{});
    return hipGetLastError() == hipSuccess ? REDVE_OK : REDVE_E_HIP;
}
