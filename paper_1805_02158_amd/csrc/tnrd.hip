// TNRD-style reaction-diffusion denoiser f (the denoising engine of Sec. IV), FP32 banks on the
// vector ALUs, one fused kernel per stage. The FP32 form runs on the MFMA stage of
// tnrd_mfma.hip; this one takes denoisers whose tile would not fit 64 KiB of LDS there (up to
// 32 filters of 127 centres):
//   u_t = u_{t-1} - sum_i K_i^T phi_i(K_i u_{t-1}) - theta_t (u_{t-1} - f_in)
// K_i = 5x5 correlation of the half-sample mirror extension, K_i^T its exact adjoint,
// phi_i(z) = sum_j w_ij exp(-(z - mu_j)^2 / (2 gamma^2)).
// The stages carry the residual w_t = u_t - f (small next to u): the input tile is staged as
// f + w, the epilogue computes w_t = w_{t-1} - g - theta_t w_{t-1}, so the FP32 rounding of the
// carried state is relative to |w|, not to |u|. The FP call then uses f(x) - x = w_T directly.
//
// Work decomposition (gfx950, wave64). A workgroup owns a 16x16 output tile and stages u on
// the tile + 4-pixel halo in LDS (2 for the forward bank, 2 for the adjoint). Its eight waves
// split the filters (wave q takes filters q, q+8, ...), so the filter loop needs no workgroup
// barrier. Forward bank: each lane keeps a 5x11 patch of u in registers and produces a 1x7
// strip of responses z for every filter of its wave (no LDS reads). Influence functions: the
// Gaussian RBF sum is evaluated exactly on the centres within 7.5 spacings of z (the rest
// contribute < 1e-12 of a weight), with one exp for the nearest term and a two-multiply
// recurrence for its neighbours. Adjoint: the wave's v plane goes to a wave-private LDS slab;
// each lane accumulates a 1x4 output strip from a 5x8 window of it. The eight waves' partial
// sums are added in fixed wave order at the end (deterministic). z and v never reach HBM:
// one read of f and w (plus halo), one write of w_t.
#include <math.h>

#include "internal.h"
#include "rbf.h"

namespace redve {

namespace {

constexpr int TH = 16, TW = 16;
constexpr int UH = TH + 8, UW = TW + 12;  // u region rows r0-4.., padded columns for the patches
constexpr int VH = TH + 4, VW = TW + 4;   // v region: rows r0-2 .. r0+TH+1
constexpr int NP = 7;                      // forward positions per lane (a 1x7 strip)
constexpr int SPR = (VW + NP - 1) / NP;    // strips per v row
constexpr int OS = 4;                      // adjoint outputs per lane (a 1x4 strip)
constexpr int NTHR = 512;                  // 8 waves: each takes every 8th filter
constexpr int NWAVE = NTHR / 64;
constexpr int WPAD = kRbfPad;  // zero padding on both sides of each weight row
static_assert(VH * SPR <= 64, "forward strips must fit one wave");
static_assert(TH * TW == 64 * OS, "adjoint strips must cover the tile with one wave");
static_assert((SPR - 1) * NP + NP + 4 <= UW, "patch columns must stay inside the u region");

// Half-sample symmetric mirror, valid for -2 <= i <= n+1 and n >= 2.
__device__ inline int mirror(int i, int n) { return i < 0 ? -i - 1 : (i >= n ? 2 * n - i - 1 : i); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// The stage on the 16x16 output tile at (r0, c0) of one image.
template <int KC>
__device__ inline void stage_tile(const float* __restrict__ w, const float* __restrict__ f,
                                  float* __restrict__ out, int H, int W, int r0, int c0,
                                  const float* __restrict__ filt, const float* __restrict__ rbfw,
                                  int F, const RbfParams& rc, float theta, int out_mode) {
    extern __shared__ float smem[];
    // The weight rows come first, so a lane's window of weights is within the immediate
    // offsets of one LDS address.
    const int wstride = rc.J + 2 * WPAD;
    float* sw = smem;                  // F * (J + 2 WPAD)
    float* su = sw + F * wstride;      // UH * UW
    float* sg = su + UH * UW;          // NWAVE * TH * TW (partial g)
    float* sv = sg + NWAVE * TH * TW;  // NWAVE * VH * VW
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    for (int e = threadIdx.x; e < UH * UW; e += NTHR) {
        const int er = r0 - 4 + e / UW, ec = c0 - 4 + e % UW;
        float val = 0.f;
        if (er >= -2 && er <= H + 1 && ec >= -2 && ec <= W + 1) {
            const size_t g = (size_t)mirror(er, H) * W + mirror(ec, W);
            val = w ? f[g] + w[g] : f[g];
        }
        su[e] = val;
    }
    for (int e = threadIdx.x; e < F * wstride; e += NTHR) sw[e] = rbfw[e];  // padded rows
    __syncthreads();

    // forward strip of this lane: v row fr, columns fc .. fc+NP-1
    const int fr = lane / SPR, fc = (lane % SPR) * NP;
    const bool fwd_lane = fr < VH;
    float patch[5][NP + 4];
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
        for (int b = 0; b < NP + 4; ++b) patch[a][b] = fwd_lane ? su[(fr + a) * UW + fc + b] : 0.f;
    bool fin[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int gr = r0 - 2 + fr, gc = c0 - 2 + fc + p;
        fin[p] = fwd_lane && fc + p < VW && gr >= 0 && gr < H && gc >= 0 && gc < W;
    }
    // adjoint strip of this lane: tile row ar, columns ac .. ac+OS-1
    const int ar = lane / (TW / OS), ac = (lane % (TW / OS)) * OS;
    float g[OS];
#pragma unroll
    for (int o = 0; o < OS; ++o) g[o] = 0.f;
    const int gra = r0 + ar;
    bool border[OS];
#pragma unroll
    for (int o = 0; o < OS; ++o) {
        const int gca = c0 + ac + o;
        border[o] = gra < H && gca < W && (gra <= 1 || gra >= H - 2 || gca <= 1 || gca >= W - 2);
    }
    float* my_v = sv + wave * VH * VW;

    for (int i = wave; i < F; i += NWAVE) {
        const float* kf = filt + i * 25;
        const float* wrow = sw + i * wstride;
        // forward bank + influence function on the strip
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            float z = 0.f;
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = 0; b < 5; ++b) z += kf[a * 5 + b] * patch[a][p + b];
            const float v = fin[p] ? phi_eval<KC>(z, wrow, rc) : 0.f;
            if (fwd_lane && fc + p < VW) my_v[fr * VW + fc + p] = v;
        }
        wave_sync();
        // adjoint: g(p) += sum_{a,b} k[a][b] v[p - (a-2, b-2)] on the strip
        float vw[5][OS + 4];
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int b = 0; b < OS + 4; ++b) vw[a][b] = my_v[(ar + a) * VW + ac + b];
#pragma unroll
        for (int o = 0; o < OS; ++o) {
            float acc = 0.f;
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = 0; b < 5; ++b) acc += kf[a * 5 + b] * vw[4 - a][o + 4 - b];
            g[o] += acc;
        }
        // border pixels also receive the contributions of the extended positions that mirror
        // onto them (the transpose of the extension)
        for (int o = 0; o < OS; ++o) {
            if (!border[o]) continue;
            const int gca = c0 + ac + o;
            const int cr[3] = {gra, -1 - gra, 2 * H - 1 - gra};
            const int cc[3] = {gca, -1 - gca, 2 * W - 1 - gca};
            float acc = 0.f;
            for (int x = 0; x < 3; ++x) {
                const int er = cr[x];
                if (er < -2 || er > H + 1) continue;
                for (int y = 0; y < 3; ++y) {
                    const int ec = cc[y];
                    if (ec < -2 || ec > W + 1 || (x == 0 && y == 0)) continue;
                    for (int a = 0; a < 5; ++a) {
                        const int vr = er - a + 2;
                        if (vr < 0 || vr >= H) continue;
                        for (int b = 0; b < 5; ++b) {
                            const int vc = ec - b + 2;
                            if (vc < 0 || vc >= W) continue;
                            acc += kf[a * 5 + b] * my_v[(vr - r0 + 2) * VW + vc - c0 + 2];
                        }
                    }
                }
            }
            g[o] += acc;
        }
        wave_sync();
    }

#pragma unroll
    for (int o = 0; o < OS; ++o) sg[wave * TH * TW + ar * TW + ac + o] = g[o];
    __syncthreads();
    // fixed-order sum of the wave partials and the reaction update
    for (int e = threadIdx.x; e < TH * TW; e += NTHR) {
        const int tr = e / TW, tc = e % TW;
        const int gr = r0 + tr, gc = c0 + tc;
        if (gr >= H || gc >= W) continue;
        float gs = 0.f;
#pragma unroll
        for (int q = 0; q < NWAVE; ++q) gs += sg[q * TH * TW + e];
        const size_t gi = (size_t)gr * W + gc;
        const float wc = w ? w[gi] : 0.f;
        const float wn = wc - gs - theta * wc;
        out[gi] = out_mode ? f[gi] + wn : wn;
    }
}

template <int KC>
__global__ __launch_bounds__(NTHR) void k_tnrd_stage_f32_valu(
    const float* __restrict__ w, const float* __restrict__ f, float* __restrict__ out, int H,
    int W, const float* __restrict__ filt, const float* __restrict__ rbfw, int F, RbfParams rc,
    float theta, int out_mode) {
    const int t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    stage_tile<KC>(w, f, out, H, W, (t / gridDim.x) * TH, (t % gridDim.x) * TW, filt, rbfw, F, rc, theta,
                   out_mode);
}

// Batched: one workgroup per tile of the batch's tile list. Vector v of image i lives at
// base_v + desc[i].off; w_base null means w = 0 (first stage).
template <int KC>
__global__ __launch_bounds__(NTHR) void k_tnrd_stage_f32_valu_batch(
    const ImgDesc* __restrict__ desc, const TileRef* __restrict__ tiles,
    const float* __restrict__ w_base, float* __restrict__ out_base,
    const float* __restrict__ filt, const float* __restrict__ rbfw, int F, RbfParams rc,
    float theta, int out_mode) {
    const TileRef e = tiles[blockIdx.x];
    const ImgDesc& d = desc[e.img];
    if (!d.active) return;
    const int t = e.t, ntx = (d.W + TW - 1) / TW;
    stage_tile<KC>(w_base ? w_base + d.off : nullptr, d.x_in, out_base + d.off, d.H, d.W,
                   (t / ntx) * TH, (t % ntx) * TW, filt, rbfw, F, rc, theta, out_mode);
}

}  // namespace

int tnrd_grid(int H, int W) { return ((W + TW - 1) / TW) * ((H + TH - 1) / TH); }

size_t tnrd_smem_bytes(int F, int J) {
    return sizeof(float) * ((size_t)UH * UW + NWAVE * TH * TW + NWAVE * VH * VW +
                            (size_t)F * (J + 2 * WPAD));
}


void launch_tnrd_stage_valu(const TnrdDev& d, int t, const float* w_prev, const float* f, float* out,
                       int H, int W, int out_mode, hipStream_t st) {
    dim3 grid((W + TW - 1) / TW, (H + TH - 1) / TH);
    const RbfParams rc = rbf_params(d);
    const size_t smem = tnrd_smem_bytes(d.nfilt, d.nrbf);
    const float* kf = d.filters + (size_t)t * d.nfilt * 25;
    const float* wf = d.rbf_w + (size_t)t * d.nfilt * (d.nrbf + 2 * kRbfPad);
    if (rc.K == 7)
        k_tnrd_stage_f32_valu<7><<<grid, NTHR, smem, st>>>(w_prev, f, out, H, W, kf, wf, d.nfilt, rc,
                                                      d.theta[t], out_mode);
    else
        k_tnrd_stage_f32_valu<0><<<grid, NTHR, smem, st>>>(w_prev, f, out, H, W, kf, wf, d.nfilt, rc,
                                                      d.theta[t], out_mode);
}

void launch_tnrd_stage_valu_batch(const TnrdDev& d, int t, const ImgDesc* desc, const TileRef* tiles,
                             int ntiles, const float* w_prev, float* out, int out_mode,
                             hipStream_t st) {
    const RbfParams rc = rbf_params(d);
    const size_t smem = tnrd_smem_bytes(d.nfilt, d.nrbf);
    const float* kf = d.filters + (size_t)t * d.nfilt * 25;
    const float* wf = d.rbf_w + (size_t)t * d.nfilt * (d.nrbf + 2 * kRbfPad);
    if (rc.K == 7)
        k_tnrd_stage_f32_valu_batch<7><<<ntiles, NTHR, smem, st>>>(desc, tiles, w_prev, out, kf,
                                                               wf, d.nfilt, rc, d.theta[t], out_mode);
    else
        k_tnrd_stage_f32_valu_batch<0><<<ntiles, NTHR, smem, st>>>(desc, tiles, w_prev, out, kf,
                                                               wf, d.nfilt, rc, d.theta[t], out_mode);
}

}  // namespace redve
