// The residual that starts an FP call's CG (eq. (7) in residual form) at one 16x16 tile:
//   r = H^T (y - H x) / sigma^2 + lambda s,   s = f(x) - x,
// for a separable PSF of compile-time radius RS (H = S B, B = col (x) row), accumulated in FP64
// from the FP32 image, so r carries no rounding of the O(|x|) quantities H^T y and A x. Shared
// by the CG start kernel and the last denoiser stage (which has s at hand): the loads of x and
// y are issued first (residual_fetch) and the stencil passes run later (residual_bt), with the
// same operations in the same order in both.
#pragma once

#include "internal.h"

namespace redve {

constexpr int kResTH = 16, kResTW = 16;  // the tile (the CG's and the denoiser stage's)

// i mod n in [0, n) (one period outside [0, n) without a division).
__device__ inline int res_wrap(int i, int n) {
    int r = i < 0 ? i + n : (i >= n ? i - n : i);
    if ((unsigned)r >= (unsigned)n) {
        r = i % n;
        r = r < 0 ? r + n : r;
    }
    return r;
}

// Regions of one tile: x on P (tile + 2 RS), y - S B x on B (tile + RS); LDS rows of SW.
template <int RS, int NTH>
struct ResidualIn {
    static constexpr int ph = kResTH + 4 * RS, pw = kResTW + 4 * RS;
    static constexpr int bh = kResTH + 2 * RS, bw = kResTW + 2 * RS;
    static constexpr int SW = kResTW + 4 * RS;
    static constexpr int NX = (ph * pw + NTH - 1) / NTH, NY = (bh * bw + NTH - 1) / NTH;
    float xv[NX], yv[NY];
    bool ys[NY];
};

// LDS of the passes: sp (ph x SW floats), se (bh x SW doubles), sh (ph x SW doubles).
template <int RS>
constexpr size_t residual_lds_bytes() {
    return (size_t)(kResTH + 4 * RS) * (kResTW + 4 * RS) * (sizeof(float) + sizeof(double)) +
           (size_t)(kResTH + 2 * RS) * (kResTW + 4 * RS) * sizeof(double);
}

template <int RS, int NTH>
__device__ inline void residual_fetch(int dec, const float* __restrict__ x,
                                      const float* __restrict__ y, int H, int W, int r0, int c0,
                                      ResidualIn<RS, NTH>& in) {
    using C = ResidualIn<RS, NTH>;
    const int wy = (W + dec - 1) / dec;
#pragma unroll
    for (int i = 0; i < C::NX; ++i) {
        const int e = threadIdx.x + i * NTH;
        in.xv[i] = 0.f;
        if (e < C::ph * C::pw)
            in.xv[i] = x[(size_t)res_wrap(r0 - 2 * RS + e / C::pw, H) * W +
                         res_wrap(c0 - 2 * RS + e % C::pw, W)];
    }
#pragma unroll
    for (int i = 0; i < C::NY; ++i) {
        const int e = threadIdx.x + i * NTH;
        in.ys[i] = false;
        in.yv[i] = 0.f;
        if (e < C::bh * C::bw) {
            const int gr = res_wrap(r0 - RS + e / C::bw, H), gc = res_wrap(c0 - RS + e % C::bw, W);
            in.ys[i] = dec == 1 || (gr % dec == 0 && gc % dec == 0);
            if (in.ys[i]) in.yv[i] = y[(size_t)(gr / dec) * wy + gc / dec];
        }
    }
}

// B^T (y - S B x) (the sum before 1 / sigma^2) at the thread's pixel of the tile (threads
// below kResTH * kResTW; 0 for the others). x stays in sp (P region, row stride SW). Contains workgroup
// barriers: every thread of the workgroup calls it.
template <int RS, int NTH>
__device__ inline double residual_bt(const LinOp& op, const ResidualIn<RS, NTH>& in, float* sp,
                                     double* se, double* sh) {
    using C = ResidualIn<RS, NTH>;
    constexpr int SW = C::SW, K = 2 * RS + 1;
    constexpr int ph = C::ph, pw = C::pw, bh = C::bh, bw = C::bw;
#pragma unroll
    for (int i = 0; i < C::NX; ++i) {
        const int e = threadIdx.x + i * NTH;
        if (e < ph * pw) sp[(e / pw) * SW + e % pw] = in.xv[i];
    }
    __syncthreads();
    // B x: row pass over the P rows, then the column pass at the B region (FP64)
    for (int e = threadIdx.x; e < ph * bw; e += NTH) {
        const int pr = e / bw, bc = e % bw;
        const float* prow = sp + pr * SW + bc + 2 * RS;
        double a = 0.0;
#pragma unroll
        for (int b = 0; b < K; ++b) a += op.row_d[b] * (double)prow[-b];
        sh[pr * SW + bc] = a;
    }
    __syncthreads();
    // e = S^T (y - S B x) on the tile + RS halo
#pragma unroll
    for (int i = 0; i < C::NY; ++i) {
        const int e = threadIdx.x + i * NTH;
        if (e < bh * bw) {
            const int br = e / bw, bc = e % bw;
            double v = 0.0;
            if (in.ys[i]) {
                double bx = 0.0;
                const double* hcol = sh + (br + 2 * RS) * SW + bc;
#pragma unroll
                for (int a = 0; a < K; ++a) bx += op.col_d[a] * hcol[-a * SW];
                v = (double)in.yv[i] - bx;
            }
            se[br * SW + bc] = v;
        }
    }
    __syncthreads();
    // B^T e: row pass, then the column pass at the thread's pixel
    for (int e = threadIdx.x; e < bh * kResTW; e += NTH) {
        const int br = e / kResTW, c = e % kResTW;
        const double* erow = se + br * SW + c;
        double a = 0.0;
#pragma unroll
        for (int b = 0; b < K; ++b) a += op.row_d[b] * erow[b];
        sh[br * SW + c] = a;
    }
    __syncthreads();
    double bt = 0.0;
    if ((int)threadIdx.x < kResTH * kResTW) {
        const double* hcol = sh + (threadIdx.x / kResTW) * SW + threadIdx.x % kResTW;
#pragma unroll
        for (int a = 0; a < K; ++a) bt += op.col_d[a] * hcol[a * SW];
    }
    return bt;
}

}  // namespace redve
