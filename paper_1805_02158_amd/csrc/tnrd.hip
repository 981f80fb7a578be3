// TNRD-style reaction-diffusion denoiser f (the denoising engine of Sec. IV), one fused kernel
// per stage:
//   u_t = u_{t-1} - sum_i K_i^T phi_i(K_i u_{t-1}) - theta_t (u_{t-1} - f_in)
// K_i = 5x5 correlation of the half-sample mirror extension, K_i^T its exact adjoint,
// phi_i(z) = sum_j w_ij exp(-(z - mu_j)^2 / (2 gamma^2)).
// The stages carry the residual w_t = u_t - f (small next to u): the input tile is staged as
// f + w, the epilogue computes w_t = w_{t-1} - g - theta_t w_{t-1}, so the FP32 rounding of the
// carried state is relative to |w|, not to |u|. The FP call then uses f(x) - x = w_T directly.
//
// A workgroup owns a TH x TW output tile. It stages u on the tile + 4-pixel halo in LDS
// (2 for the forward bank, 2 for the adjoint). Every thread keeps the 5x5 window of u around
// each of its forward positions in registers, so the 24-filter forward bank reads LDS once.
// Per filter, v = phi(K u) on the tile + 2 halo goes to LDS and the adjoint accumulates in
// registers. The responses z and v never reach HBM: one read of u and f, one write of u_t.
#include "internal.h"

namespace redve {

namespace {

constexpr int TH = 16, TW = 16;
constexpr int UH = TH + 8, UW = TW + 8;  // u region: rows r0-4 .. r0+TH+3
constexpr int VH = TH + 4, VW = TW + 4;  // v region: rows r0-2 .. r0+TH+1
constexpr int NPOS = (VH * VW + kThreads - 1) / kThreads;  // forward positions per thread
constexpr int NOUT = TH * TW / kThreads;                    // outputs per thread
constexpr float LOG2E = 1.4426950408889634f;

// Half-sample symmetric mirror, valid for -2 <= i <= n+1 and n >= 2.
__device__ inline int mirror(int i, int n) { return i < 0 ? -i - 1 : (i >= n ? 2 * n - i - 1 : i); }

__global__ __launch_bounds__(kThreads) void k_tnrd_stage_f32(
    const float* __restrict__ w, const float* __restrict__ f, float* __restrict__ out, int H,
    int W, const float* __restrict__ filt /* F*25 */, const float* __restrict__ rbfw /* F*J */,
    int F, int J, float theta, float mu0, float dmu, float gscale /* log2(e)/(2 gamma^2) */,
    int out_mode) {
    __shared__ float su[UH * UW];
    __shared__ float sv[VH * VW];
    const int r0 = blockIdx.y * TH, c0 = blockIdx.x * TW;

    for (int e = threadIdx.x; e < UH * UW; e += kThreads) {
        const int er = r0 - 4 + e / UW, ec = c0 - 4 + e % UW;
        float val = 0.f;
        if (er >= -2 && er <= H + 1 && ec >= -2 && ec <= W + 1) {
            const size_t g = (size_t)mirror(er, H) * W + mirror(ec, W);
            val = w ? f[g] + w[g] : f[g];
        }
        su[e] = val;
    }
    __syncthreads();

    // 5x5 windows of u for this thread's forward positions (v region coordinates).
    float win[NPOS][25];
    bool inside[NPOS];
#pragma unroll
    for (int k = 0; k < NPOS; ++k) {
        const int pos = threadIdx.x + k * kThreads;
        const int vr = pos / VW, vc = pos % VW;  // v region row/col; image row r0-2+vr
        const int gr = r0 - 2 + vr, gc = c0 - 2 + vc;
        inside[k] = pos < VH * VW && gr >= 0 && gr < H && gc >= 0 && gc < W;
#pragma unroll
        for (int t = 0; t < 25; ++t) win[k][t] = 0.f;
        if (inside[k]) {
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = 0; b < 5; ++b) win[k][a * 5 + b] = su[(vr + a) * UW + vc + b];
        }
    }

    float g[NOUT];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) g[k] = 0.f;

    for (int i = 0; i < F; ++i) {
        const float* kf = filt + i * 25;
        const float* wi = rbfw + i * J;
#pragma unroll
        for (int k = 0; k < NPOS; ++k) {
            const int pos = threadIdx.x + k * kThreads;
            float v = 0.f;
            if (inside[k]) {
                float z = 0.f;
#pragma unroll
                for (int t = 0; t < 25; ++t) z += kf[t] * win[k][t];
                float acc = 0.f;
                for (int j = 0; j < J; ++j) {
                    const float d = z - (mu0 + dmu * (float)j);
                    acc += wi[j] * __builtin_amdgcn_exp2f(-(d * d) * gscale);
                }
                v = acc;
            }
            if (pos < VH * VW) sv[pos] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NOUT; ++k) {
            const int o = threadIdx.x + k * kThreads;
            const int tr = o / TW, tc = o % TW;
            const int gr = r0 + tr, gc = c0 + tc;
            // primary: extended position == the pixel itself; v outside the image is 0 in LDS
            float acc = 0.f;
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = 0; b < 5; ++b)
                    acc += kf[a * 5 + b] * sv[(tr + 4 - a) * VW + tc + 4 - b];
            // border pixels also receive the contributions of the extended positions that
            // mirror onto them (the transpose of the extension)
            if ((gr <= 1 || gr >= H - 2 || gc <= 1 || gc >= W - 2) && gr < H && gc < W) {
                const int cr[3] = {gr, -1 - gr, 2 * H - 1 - gr};
                const int cc[3] = {gc, -1 - gc, 2 * W - 1 - gc};
                for (int x = 0; x < 3; ++x) {
                    const int er = cr[x];
                    if (er < -2 || er > H + 1) continue;
                    for (int y = 0; y < 3; ++y) {
                        const int ec = cc[y];
                        if (ec < -2 || ec > W + 1) continue;
                        if (x == 0 && y == 0) continue;
                        for (int a = 0; a < 5; ++a) {
                            const int vr = er - a + 2;
                            if (vr < 0 || vr >= H) continue;
                            for (int b = 0; b < 5; ++b) {
                                const int vc = ec - b + 2;
                                if (vc < 0 || vc >= W) continue;
                                acc += kf[a * 5 + b] * sv[(vr - r0 + 2) * VW + vc - c0 + 2];
                            }
                        }
                    }
                }
            }
            g[k] += acc;
        }
        __syncthreads();
    }

#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int tr = o / TW, tc = o % TW;
        const int gr = r0 + tr, gc = c0 + tc;
        if (gr < H && gc < W) {
            const size_t gi = (size_t)gr * W + gc;
            const float wc = w ? w[gi] : 0.f;
            const float wn = wc - g[k] - theta * wc;
            out[gi] = out_mode ? f[gi] + wn : wn;
        }
    }
}

}  // namespace

int tnrd_grid(int H, int W) { return ((W + TW - 1) / TW) * ((H + TH - 1) / TH); }

void launch_tnrd_stage(const TnrdDev& d, int t, const float* w_prev, const float* f, float* out,
                       int H, int W, int out_mode, hipStream_t st) {
    dim3 grid((W + TW - 1) / TW, (H + TH - 1) / TH);
    const float gscale = LOG2E / (2.f * d.gamma * d.gamma);
    const float theta = d.theta[t];
    k_tnrd_stage_f32<<<grid, kThreads, 0, st>>>(w_prev, f, out, H, W,
                                                d.filters + (size_t)t * d.nfilt * 25,
                                                d.rbf_w + (size_t)t * d.nfilt * d.nrbf, d.nfilt,
                                                d.nrbf, theta, d.mu0, d.dmu, gscale, out_mode);
}

}  // namespace redve
