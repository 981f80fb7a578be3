// Denoiser stage with both 5x5 filter banks on MFMA, in two forms: BF16 operands
// (v_mfma_f32_16x16x32_bf16) or FP32 operands (v_mfma_f32_16x16x4_f32), FP32 accumulation in
// both; influence functions and the reaction update in FP32.
//
// The stage u_t = u_{t-1} - sum_i K_i^T phi_i(K_i u_{t-1}) - theta (u_{t-1} - f), carried as
// the residual w = u - f, is organised as two implicit GEMMs per 16x16 tile:
//   forward  Z[q][i] = sum_tap A[q][tap] Kf[tap][i]   q: 400 positions (tile + 2 halo, 25 groups
//            of 16), taps 25 -> 32 (BF16) or 28 (FP32), filters F -> 32; A[q][tap] =
//            u(q + tap) - u(q) (the filters have zero mean, so subtracting the window centre
//            is exact and keeps the operand small: in BF16 an image value of 100 carries an
//            error of 0.4, a local difference of 5 one of 0.02).
//   adjoint S[q][tap] = sum_i V[q][i] Kf[tap][i]    V = phi(Z) (FP32),
//            then g(p) = sum_tap S[p - off(tap)][tap] (shift-add in LDS) plus the mirror fold at
//            the image border.
// MFMA operand layout (checked on gfx950 for BF16): lane l holds row (A) or column (B) l % 16
// and the K values of slice l / 16 (eight for BF16, one for FP32); the accumulator holds
// column l % 16, rows 4 (l / 16) + 0..3. The filter fragments are prepacked on the host per
// stage. The FP32 form's stage is also in tnrd.hip (vector ALU banks), which takes denoisers
// whose tile would not fit 64 KiB of LDS here.
// Influence functions: on the exact window (KC = K > 0, or 0 for any K), or, in the BF16 form
// on images of fewer than 512 tiles where the tables fit the device's LDS, from the per-filter
// cubic tables (KC = -1; the tables take the place of the weight rows in LDS, and the
// workgroup has 1024 threads). The tables take 56 KiB per tile for the 24-filter denoiser, so a
// CU holds one such tile: on larger images, where two window tiles per CU overlap their
// phases, and in the batched engine (an image's result must not depend on the batch), the
// window is used.
#include <math.h>

#include <type_traits>

#include "../../include/redve.h"
#include "internal.h"
#include "rbf.h"
#include "residual.h"

namespace redve {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int TH = 16, TW = 16;
static_assert(TH == kResTH && TW == kResTW, "the residual's tile");
constexpr int UH = TH + 8, UW = TW + 8;  // u region: rows r0-4 .. r0+TH+3
constexpr int VH = TH + 4, VW = TW + 4;  // positions of z / v: rows r0-2 .. r0+TH+1
constexpr int NPOS = VH * VW;            // 400 = 25 groups of 16
constexpr int NGRP = NPOS / 16;
constexpr int WPAD = kRbfPad;
static_assert(NPOS % 16 == 0, "positions must fill MFMA groups");

__device__ inline int mirror(int i, int n) { return i < 0 ? -i - 1 : (i >= n ? 2 * n - i - 1 : i); }

__device__ inline bf16x8 load_frag(const uint16_t* p) {
    // eight packed BF16 values (16 bytes, aligned)
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    bf16x8 r;
    __builtin_memcpy(&r, &v, 16);
    return r;
}

// NT threads per workgroup: 512 where the image has tiles for every CU several times over,
// 1024 on small images (one tile per CU), where twice the waves hide twice the latency.
// ZS: the odd row stride of the per-position rows in LDS (z, v, then the tap sums), at least
// max(F, 25): 25 for up to 25 filters, 33 for up to 32.
// F32: FP32 operands on v_mfma_f32_16x16x4_f32 (the FP32 form) instead of BF16; bfwd / badj
// then hold FP32 fragments (forward 7 x 2, adjoint 8 x 2 slices of 64 lanes).
// RSR > 0: the last stage of an FP call also forms the CG start r = H^T (y - H x) / sigma^2 +
// lambda s at its pixels (x = f, s its output; PSF radius RSR): the loads of x and y are issued
// with the stage's own, the stencil passes run at the end in the freed per-position rows.
template <int KC, int NT, int ZS, bool F32, int RSR = 0>
__device__ inline void stage_tile_mfma(const float* __restrict__ w, const float* __restrict__ f,
                                       float* __restrict__ out, int H, int W, int r0, int c0,
                                       const void* __restrict__ bfwd,
                                       const void* __restrict__ badj,
                                       const float* __restrict__ rbfw, int F, const RbfParams& rc,
                                       float theta, int out_mode,
                                       const ResidualReq* __restrict__ rq = nullptr) {
    extern __shared__ __align__(16) float smem[];
    // One row per position holds z, then v = phi(z), then the 25 per-tap adjoint sums (a wave
    // overwrites the rows of its own MFMA group after loading them as an operand).
    // The weight rows come first, so a lane's window of weights is within the immediate
    // offsets of one LDS address.
    static_assert(ZS % 2 == 1 && ZS >= 25, "odd stride covering the 25 taps");
    // weight rows of J + 2 WPAD, or table rows of 4 tab_n (16-byte aligned)
    const int wstride = KC < 0 ? 4 * rc.tab_n : rc.J + 2 * WPAD;
    float* sw = smem;                 // F * wstride
    float* su = sw + F * wstride;     // UH * UW
    float* sz = su + UH * UW;         // NPOS * ZS
    float* ss = sz;
    constexpr int NWAVE = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the pixel's own w and f for the update, loaded first: the loads are in flight for the
    // whole stage instead of after its last barrier
    const int tr = threadIdx.x / TW, tc = threadIdx.x % TW;
    const int gr = r0 + tr, gc = c0 + tc;
    const bool pix = (int)threadIdx.x < TH * TW && gr < H && gc < W;
    const size_t gi = (size_t)gr * W + gc;
    const float wc = pix && w ? w[gi] : 0.f;
    const float fc = pix && out_mode ? f[gi] : 0.f;
    constexpr int RSX = RSR > 0 ? RSR : 1;
    ResidualIn<RSX, NT> rin;
    if constexpr (RSR > 0) residual_fetch<RSR, NT>(1, f, rq->y, H, W, r0, c0, rin);

    for (int e = threadIdx.x; e < UH * UW; e += NT) {
        const int er = r0 - 4 + e / UW, ec = c0 - 4 + e % UW;
        float val = 0.f;
        if (er >= -2 && er <= H + 1 && ec >= -2 && ec <= W + 1) {
            const size_t g = (size_t)mirror(er, H) * W + mirror(ec, W);
            val = w ? f[g] + w[g] : f[g];
        }
        su[e] = val;
    }
    if constexpr (KC < 0) {
        const float4* src = reinterpret_cast<const float4*>(rbfw);
        float4* dst = reinterpret_cast<float4*>(sw);
        for (int e = threadIdx.x; e < F * rc.tab_n; e += NT) dst[e] = src[e];
    } else {
        for (int e = threadIdx.x; e < F * wstride; e += NT) sw[e] = rbfw[e];  // padded rows
    }
    __syncthreads();

    const int m = lane & 15, sl = lane >> 4;  // fragment row/column, K slice
    // ---- forward bank: Z = A Kf on MFMA, one group of 16 positions per step
    if constexpr (F32) {
        // seven K slices of four taps, two blocks of 16 filters
        const float* fr = static_cast<const float*>(bfwd);
        float b[7][2];
#pragma unroll
        for (int k = 0; k < 7; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) b[k][h] = fr[(k * 2 + h) * 64 + lane];
        // the lane's tap offsets in the u region; taps past 25 read the centre (x = 0)
        int toff[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const int tap = 4 * k + sl;
            toff[k] = tap < 25 ? (tap / 5) * UW + tap % 5 : 2 * UW + 2;
        }
        for (int grp = wave; grp < NGRP; grp += NWAVE) {
            const int q = grp * 16 + m;
            const int qb = (q / VW) * UW + q % VW;
            const float centre = su[qb + 2 * UW + 2];
            f32x4 z0 = {0.f, 0.f, 0.f, 0.f}, z1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const float x = su[qb + toff[k]] - centre;
                z0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, b[k][0], z0, 0, 0, 0);
                z1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, b[k][1], z1, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int qq = grp * 16 + sl * 4 + i;
                sz[qq * ZS + m] = z0[i];
                if (m + 16 < F) sz[qq * ZS + m + 16] = z1[i];
            }
        }
    } else {
        const bf16x8 b0 = load_frag((const uint16_t*)bfwd + (0 * 64 + lane) * 8);
        const bf16x8 b1 = load_frag((const uint16_t*)bfwd + (1 * 64 + lane) * 8);
        // the lane's tap offsets in the u region; taps past 25 read the centre (x = 0)
        int toff[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int tap = sl * 8 + j;
            toff[j] = tap < 25 ? (tap / 5) * UW + tap % 5 : 2 * UW + 2;
        }
        // tabulated phi: the lane's two filters are fixed, so phi is applied to the
        // accumulators here and v is stored in place of z
        const float* tab0 = sw + m * wstride;
        const float* tab1 = sw + (m + 16) * wstride;
        for (int grp = wave; grp < NGRP; grp += NWAVE) {
            const int q = grp * 16 + m;
            const int qb = (q / VW) * UW + q % VW;
            const float centre = su[qb + 2 * UW + 2];
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)(su[qb + toff[j]] - centre);
            f32x4 z0 = {0.f, 0.f, 0.f, 0.f}, z1 = {0.f, 0.f, 0.f, 0.f};
            z0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, z0, 0, 0, 0);
            z1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, z1, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int qq = grp * 16 + sl * 4 + i;
                if constexpr (KC < 0) {
                    if (m < F) sz[qq * ZS + m] = phi_table(z0[i], tab0, rc);
                    if (m + 16 < F) sz[qq * ZS + m + 16] = phi_table(z1[i], tab1, rc);
                } else {
                    sz[qq * ZS + m] = z0[i];
                    if (m + 16 < F) sz[qq * ZS + m + 16] = z1[i];
                }
            }
        }
    }
    __syncthreads();
    // ---- influence functions on the window (tabulated: applied in the forward bank above),
    // dense over (filter, position) pairs, FP32, at every position (the adjoint bank zeroes
    // those outside the image). A wave takes filters wave, wave + NWAVE, ... and its lanes 64
    // consecutive positions at a time over the first QM positions: the lanes gather weights
    // from one LDS row, mostly at the same or nearby centres (broadcast instead of bank
    // conflicts), read z at the odd stride ZS (conflict-free), and step by an immediate offset;
    // the last QT positions of every filter are shared out over all threads afterwards.
    if constexpr (KC >= 0) {
        constexpr int QM = NPOS / 64 * 64, QT = NPOS - QM;
        for (int i = wave; i < F; i += NWAVE) {
            const float* wr = sw + i * wstride;
            float* zp = sz + lane * ZS + i;
#pragma unroll
            for (int s = 0; s < QM / 64; ++s) zp[s * 64 * ZS] = phi_eval<KC>(zp[s * 64 * ZS], wr, rc);
        }
        if constexpr (QT > 0) {
            for (int e = threadIdx.x; e < QT * F; e += NT) {
                const int q = QM + e % QT, i = e / QT;
                sz[q * ZS + i] = phi_eval<KC>(sz[q * ZS + i], sw + i * wstride, rc);
            }
        }
        __syncthreads();
    }
    // ---- adjoint bank: S = V Kf^T on MFMA
    if constexpr (F32) {
        // K slices of four filters (as many as F needs, at most eight), two blocks of 16 taps
        const float* fr = static_cast<const float*>(badj);
        float b[8][2];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) b[k][h] = 4 * k < F ? fr[(k * 2 + h) * 64 + lane] : 0.f;
        for (int grp = wave; grp < NGRP; grp += NWAVE) {
            const int q = grp * 16 + m;
            const int gr = r0 - 2 + q / VW, gc = c0 - 2 + q % VW;
            const bool qin = gr >= 0 && gr < H && gc >= 0 && gc < W;  // v = 0 outside the image
            f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (4 * k >= F) break;
                const int i = 4 * k + sl;
                const float x = i < F && qin ? sz[q * ZS + i] : 0.f;
                s0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, b[k][0], s0, 0, 0, 0);
                s1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x, b[k][1], s1, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int qq = grp * 16 + sl * 4 + i;
                ss[qq * ZS + m] = s0[i];
                if (m + 16 < 25) ss[qq * ZS + m + 16] = s1[i];
            }
        }
    } else {
        const bf16x8 b0 = load_frag((const uint16_t*)badj + (0 * 64 + lane) * 8);
        const bf16x8 b1 = load_frag((const uint16_t*)badj + (1 * 64 + lane) * 8);
        for (int grp = wave; grp < NGRP; grp += NWAVE) {
            const int q = grp * 16 + m;
            const int gr = r0 - 2 + q / VW, gc = c0 - 2 + q % VW;
            const bool qin = gr >= 0 && gr < H && gc >= 0 && gc < W;  // v = 0 outside the image
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = sl * 8 + j;
                a[j] = (__bf16)(i < F && qin ? sz[q * ZS + i] : 0.f);
            }
            f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
            s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, s0, 0, 0, 0);
            s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, s1, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int qq = grp * 16 + sl * 4 + i;
                ss[qq * ZS + m] = s0[i];
                if (m + 16 < 25) ss[qq * ZS + m + 16] = s1[i];
            }
        }
    }
    __syncthreads();
    // ---- shift-add of the tap sums, g(p) = sum_tap S[p + (2, 2) - tap][tap], and the
    // transpose of the mirror extension: a border pixel also receives t(e), the same sum at
    // each position e of the extension (outside the image, at most 2 away) that mirrors onto
    // it. S vanishes outside the image, and every S such a t(e) needs inside the image lies in
    // the position region. The first TH * TW threads take one pixel each; in a tile at the
    // border the others meanwhile write the t(e) to the u region (free after the forward bank).
    constexpr int EH = TH + 5, EW = TW + 5;  // rows r0-2 .. r0+TH+2, columns c0-2 .. c0+TW+2
    static_assert(EH * EW <= UH * UW, "extension sums fit the u region");
    static_assert(NT >= 2 * TH * TW, "threads for the pixels and for the extension");
    float* st = su;
    const bool edge = r0 < 2 || c0 < 2 || r0 + TH + 2 > H || c0 + TW + 2 > W;
    float g = 0.f;
    if (pix) {
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int b = 0; b < 5; ++b) g += ss[((tr + 4 - a) * VW + tc + 4 - b) * ZS + a * 5 + b];
    } else if (edge && (int)threadIdx.x >= TH * TW) {
        const int rend = min(r0 + TH, H), cend = min(c0 + TW, W);
        for (int e = threadIdx.x - TH * TW; e < EH * EW; e += NT - TH * TW) {
            const int lr = e / EW, lc = e % EW;
            const int er = r0 - 2 + lr, ec = c0 - 2 + lc;
            if (er < -2 || er > H + 1 || ec < -2 || ec > W + 1) continue;
            if (er >= 0 && er < H && ec >= 0 && ec < W) continue;  // inside the image
            const int mr = mirror(er, H), mc = mirror(ec, W);
            if (mr < r0 || mr >= rend || mc < c0 || mc >= cend) continue;  // not onto this tile
            // tap (a, b) reads position (lr + 2 - a, lc + 2 - b), counted where it lies in the
            // region (S vanishes there outside the image); the row and column offsets are
            // formed once, clamped into the region, and all 25 reads are issued before the
            // sum, which adds them in tap order
            int ro[5], co[5];
            bool rok[5], cok[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int qr = lr + 2 - k, qc = lc + 2 - k;
                rok[k] = qr >= 0 && qr < VH;
                cok[k] = qc >= 0 && qc < VW;
                ro[k] = (rok[k] ? qr : 0) * VW * ZS;
                co[k] = (cok[k] ? qc : 0) * ZS;
            }
            float v[25];
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = 0; b < 5; ++b) v[a * 5 + b] = ss[ro[a] + co[b] + a * 5 + b];
            float t = 0.f;
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = 0; b < 5; ++b) t += rok[a] && cok[b] ? v[a * 5 + b] : 0.f;
            st[e] = t;
        }
    }
    if (edge) __syncthreads();
    if (RSR == 0 && !pix) return;
    // rows -1-r (r <= 1) and 2H-1-r (r >= H-2) mirror onto row r, the same for columns, and the
    // corners of both (two of each on a side of 2 or 3 pixels); then the reaction update
    if (pix && (gr <= 1 || gr >= H - 2 || gc <= 1 || gc >= W - 2)) {
        // local rows / columns of the pixel and its mirror images, with their validity (fixed
        // indices, so the arrays stay in registers)
        const int lr[3] = {tr + 2, 1 - gr - r0, 2 * H + 1 - gr - r0};
        const int lc[3] = {tc + 2, 1 - gc - c0, 2 * W + 1 - gc - c0};
        const bool vr[3] = {true, gr <= 1, gr >= H - 2};
        const bool vc[3] = {true, gc <= 1, gc >= W - 2};
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int y = 0; y < 3; ++y)
                if ((x || y) && vr[x] && vc[y]) g += st[lr[x] * EW + lc[y]];
    }
    const float wn = wc - g - theta * wc;
    if (pix) out[gi] = out_mode ? fc + wn : wn;
    if constexpr (RSR > 0) {
        // the CG start, with s = wn: the passes in the per-position rows (free once every pixel
        // has its sum)
        __syncthreads();
        double* rl = reinterpret_cast<double*>(
            (reinterpret_cast<uintptr_t>(sz) + 15) & ~static_cast<uintptr_t>(15));
        constexpr int SW = ResidualIn<RSR, NT>::SW;
        constexpr int PH = TH + 4 * RSR, BH = TH + 2 * RSR;
        static_assert(residual_lds_bytes<RSR>() + 16 <= sizeof(float) * NPOS * 25,
                      "the residual's rows fit the per-position rows");
        double* se = rl;
        double* sh = se + BH * SW;
        float* sp = reinterpret_cast<float*>(sh + PH * SW);
        const double bt = residual_bt<RSR, NT>(rq->op, rin, sp, se, sh);
        if (pix) {
            double rv = rq->op.inv_s2_d * bt;
            rv += rq->op.lambda_d * (double)wn;
            rq->r[gi] = (float)rv;
        }
    }
}

template <int KC, int NT, int ZS>
__global__ __launch_bounds__(NT) void k_tnrd_stage_bf16(
    const float* __restrict__ w, const float* __restrict__ f, float* __restrict__ out, int H,
    int W, const void* __restrict__ bfwd, const void* __restrict__ badj,
    const float* __restrict__ rbfw, int F, RbfParams rc, float theta, int out_mode) {
    const int t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    stage_tile_mfma<KC, NT, ZS, false>(w, f, out, H, W, (t / gridDim.x) * TH,
                                       (t % gridDim.x) * TW, bfwd, badj, rbfw, F, rc, theta,
                                       out_mode);
}

template <int KC, int NT, int ZS>
__global__ __launch_bounds__(NT) void k_tnrd_stage_f32(
    const float* __restrict__ w, const float* __restrict__ f, float* __restrict__ out, int H,
    int W, const void* __restrict__ bfwd, const void* __restrict__ badj,
    const float* __restrict__ rbfw, int F, RbfParams rc, float theta, int out_mode) {
    const int t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    stage_tile_mfma<KC, NT, ZS, true>(w, f, out, H, W, (t / gridDim.x) * TH,
                                      (t % gridDim.x) * TW, bfwd, badj, rbfw, F, rc, theta,
                                      out_mode);
}

// The last stage of an FP call with the CG start (one tile per workgroup of 1024 threads).
template <int KC, int ZS, int RSR>
__global__ __launch_bounds__(1024) void k_tnrd_stage_bf16_res(
    const float* __restrict__ w, const float* __restrict__ f, float* __restrict__ out, int H,
    int W, const void* __restrict__ bfwd, const void* __restrict__ badj,
    const float* __restrict__ rbfw, int F, RbfParams rc, float theta, int out_mode,
    ResidualReq rq) {
    const int t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    stage_tile_mfma<KC, 1024, ZS, false, RSR>(w, f, out, H, W, (t / gridDim.x) * TH,
                                              (t % gridDim.x) * TW, bfwd, badj, rbfw, F, rc,
                                              theta, out_mode, &rq);
}

template <int KC, int ZS, int RSR>
__global__ __launch_bounds__(1024) void k_tnrd_stage_f32_res(
    const float* __restrict__ w, const float* __restrict__ f, float* __restrict__ out, int H,
    int W, const void* __restrict__ bfwd, const void* __restrict__ badj,
    const float* __restrict__ rbfw, int F, RbfParams rc, float theta, int out_mode,
    ResidualReq rq) {
    const int t = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    stage_tile_mfma<KC, 1024, ZS, true, RSR>(w, f, out, H, W, (t / gridDim.x) * TH,
                                             (t % gridDim.x) * TW, bfwd, badj, rbfw, F, rc,
                                             theta, out_mode, &rq);
}

template <int KC, int NT, int ZS, bool F32>
__device__ inline void stage_batch_tile(const ImgDesc* __restrict__ desc,
                                        const TileRef* __restrict__ tiles,
                                        const float* __restrict__ w_base,
                                        float* __restrict__ out_base, const void* bfwd,
                                        const void* badj, const float* __restrict__ rbfw, int F,
                                        const RbfParams& rc, float theta, int out_mode) {
    const TileRef e = tiles[blockIdx.x];
    const ImgDesc& d = desc[e.img];
    if (!d.active) return;
    const int t = e.t, ntx = (d.W + TW - 1) / TW;
    stage_tile_mfma<KC, NT, ZS, F32>(w_base ? w_base + d.off : nullptr, d.x_in,
                                      out_base + d.off, d.H, d.W, (t / ntx) * TH,
                                      (t % ntx) * TW, bfwd, badj, rbfw, F, rc, theta, out_mode);
}

template <int KC, int ZS>
__global__ __launch_bounds__(512) void k_tnrd_stage_bf16_batch(
    const ImgDesc* __restrict__ desc, const TileRef* __restrict__ tiles,
    const float* __restrict__ w_base, float* __restrict__ out_base, const void* __restrict__ bfwd,
    const void* __restrict__ badj, const float* __restrict__ rbfw, int F, RbfParams rc,
    float theta, int out_mode) {
    stage_batch_tile<KC, 512, ZS, false>(desc, tiles, w_base, out_base, bfwd, badj, rbfw, F, rc,
                                    theta, out_mode);
}

template <int KC, int ZS>
__global__ __launch_bounds__(512) void k_tnrd_stage_f32_batch(
    const ImgDesc* __restrict__ desc, const TileRef* __restrict__ tiles,
    const float* __restrict__ w_base, float* __restrict__ out_base, const void* __restrict__ bfwd,
    const void* __restrict__ badj, const float* __restrict__ rbfw, int F, RbfParams rc,
    float theta, int out_mode) {
    stage_batch_tile<KC, 512, ZS, true>(desc, tiles, w_base, out_base, bfwd, badj, rbfw, F, rc,
                                   theta, out_mode);
}

// Per tile, the image's form: BF16 banks on the KB window, or FP32 banks on the KF window.
template <int KB, int KF, int ZS>
__global__ __launch_bounds__(512) void k_tnrd_stage_mixed_batch(
    const ImgDesc* __restrict__ desc, const TileRef* __restrict__ tiles,
    const float* __restrict__ w_base, float* __restrict__ out_base, const void* __restrict__ bfwd,
    const void* __restrict__ badj, const void* __restrict__ ffwd, const void* __restrict__ fadj,
    const float* __restrict__ rbfw, int F, RbfParams rcb, RbfParams rcf, float theta,
    int out_mode) {
    if (desc[tiles[blockIdx.x].img].fp32_banks)
        stage_batch_tile<KF, 512, ZS, true>(desc, tiles, w_base, out_base, ffwd, fadj, rbfw, F,
                                            rcf, theta, out_mode);
    else
        stage_batch_tile<KB, 512, ZS, false>(desc, tiles, w_base, out_base, bfwd, badj, rbfw, F,
                                             rcb, theta, out_mode);
}

int row_stride(int F) { return F > 25 ? 33 : 25; }

constexpr int kWideStageBelow = 512;  // tiles: fewer than two per CU

// Arguments of one stage launch.
struct StageArgs {
    const float *w, *f;
    float* out;
    int H, W;
    const void *bf, *ba;
    const float* wf;
    int F;
    RbfParams rc;
    float theta;
    int out_mode;
    bool table;  // tabulated influence functions (BF16 form)
    const ResidualReq* rq;  // the CG start with the last stage (or null)
};

template <int KC, int ZS, bool F32>
void stage_single(bool wide, dim3 grid, size_t smem, hipStream_t st, const StageArgs& a) {
    // the stage with the CG start: BF16 tables (KC = -1) or the FP32 K = 7 window
    if constexpr ((!F32 && KC < 0) || (F32 && KC == 7)) {
        if (a.rq) {
#define REDVE_STAGE_RES(NAME, RS_)                                                          \
    NAME<KC, ZS, RS_><<<grid, 1024, smem, st>>>(a.w, a.f, a.out, a.H, a.W, a.bf, a.ba, a.wf, \
                                                a.F, a.rc, a.theta, a.out_mode, *a.rq)
            if constexpr (F32) {
                if (a.rq->rs == 4)
                    REDVE_STAGE_RES(k_tnrd_stage_f32_res, 4);
                else
                    REDVE_STAGE_RES(k_tnrd_stage_f32_res, 3);
            } else {
                if (a.rq->rs == 4)
                    REDVE_STAGE_RES(k_tnrd_stage_bf16_res, 4);
                else
                    REDVE_STAGE_RES(k_tnrd_stage_bf16_res, 3);
            }
#undef REDVE_STAGE_RES
            return;
        }
    }
#define REDVE_STAGE(NAME, NT)                                                                \
    NAME<KC, NT, ZS><<<grid, NT, smem, st>>>(a.w, a.f, a.out, a.H, a.W, a.bf, a.ba, a.wf, a.F, \
                                             a.rc, a.theta, a.out_mode)
    if constexpr (F32) {
        if (wide)
            REDVE_STAGE(k_tnrd_stage_f32, 1024);
        else
            REDVE_STAGE(k_tnrd_stage_f32, 512);
    } else {
        if (wide || KC < 0)
            REDVE_STAGE(k_tnrd_stage_bf16, 1024);
        else if constexpr (KC >= 0)
            REDVE_STAGE(k_tnrd_stage_bf16, 512);
    }
#undef REDVE_STAGE
}

template <int KC, int ZS, bool F32>
void stage_batch(int ntiles, size_t smem, hipStream_t st, const ImgDesc* desc,
                 const TileRef* tiles, const StageArgs& a) {
    if constexpr (F32)
        k_tnrd_stage_f32_batch<KC, ZS><<<ntiles, 512, smem, st>>>(
            desc, tiles, a.w, a.out, a.bf, a.ba, a.wf, a.F, a.rc, a.theta, a.out_mode);
    else if constexpr (KC >= 0)  // the batched engine evaluates phi on the window
        k_tnrd_stage_bf16_batch<KC, ZS><<<ntiles, 512, smem, st>>>(
            desc, tiles, a.w, a.out, a.bf, a.ba, a.wf, a.F, a.rc, a.theta, a.out_mode);
}

// Dispatch over the evaluation of phi (table, window K = 5, 7 or any) and the row stride.
template <bool F32, typename Launch>
void dispatch(const StageArgs& a, Launch&& go) {
    const bool z33 = row_stride(a.F) == 33;
    auto by_zs = [&](auto kc) {
        if (z33)
            go(kc, std::integral_constant<int, 33>{});
        else
            go(kc, std::integral_constant<int, 25>{});
    };
    if constexpr (!F32)
        if (a.table) {
            by_zs(std::integral_constant<int, -1>{});
            return;
        }
    if (a.rc.K == 5)
        by_zs(std::integral_constant<int, 5>{});
    else if (a.rc.K == 7)
        by_zs(std::integral_constant<int, 7>{});
    else
        by_zs(std::integral_constant<int, 0>{});
}

template <bool F32>
StageArgs stage_args(const TnrdDev& d, int t, const float* w_prev, const float* f, float* out,
                     int H, int W, int out_mode, bool allow_table) {
    StageArgs a;
    a.w = w_prev;
    a.f = f;
    a.out = out;
    a.H = H;
    a.W = W;
    if constexpr (F32) {
        a.bf = d.frag32_fwd + (size_t)t * kFrag32Fwd;
        a.ba = d.frag32_adj + (size_t)t * kFrag32Adj;
    } else {
        a.bf = d.frag_fwd + (size_t)t * 2 * 64 * 8;
        a.ba = d.frag_adj + (size_t)t * 2 * 64 * 8;
    }
    a.table = !F32 && allow_table && d.phi_tab;
    a.wf = a.table ? d.phi_tab + (size_t)t * d.nfilt * d.tab_n * 4
                   : d.rbf_w + (size_t)t * d.nfilt * (d.nrbf + 2 * kRbfPad);
    a.F = d.nfilt;
    a.rc = rbf_params(d);
    a.theta = d.theta[t];
    a.out_mode = out_mode;
    a.rq = nullptr;
    return a;
}

// Returns whether the launch formed the CG start of rq.
template <bool F32>
bool launch_single(const TnrdDev& d, int t, const float* w_prev, const float* f, float* out,
                   int H, int W, int out_mode, hipStream_t st, const ResidualReq* rq) {
    dim3 grid((W + TW - 1) / TW, (H + TH - 1) / TH);
    // rule: fewer tiles than two per CU take 1024 threads per tile, and the tables where there
    // are; a tuned configuration may choose otherwise (tables need 1024 threads)
    const bool wide = d.stage_threads ? d.stage_threads == 1024 : grid.x * grid.y < kWideStageBelow;
    const bool table = wide && d.phi_table != 2;
    StageArgs a = stage_args<F32>(d, t, w_prev, f, out, H, W, out_mode, table);
    // the residual kernels have 1024 threads and exist for the tables (BF16) or the K = 7
    // window (FP32)
    a.rq = wide && (F32 ? a.rc.K == 7 : a.table) ? rq : nullptr;
    const size_t smem = a.table ? tnrd_table_smem_bytes(d.nfilt, d.tab_n)
                                : tnrd_mfma_smem_bytes(d.nfilt, d.nrbf);
    dispatch<F32>(a, [&](auto kc, auto zs) {
        stage_single<decltype(kc)::value, decltype(zs)::value, F32>(wide, grid, smem, st, a);
    });
    return a.rq != nullptr;
}

template <bool F32>
void launch_batch(const TnrdDev& d, int t, const ImgDesc* desc, const TileRef* tiles,
                  int ntiles, const float* w_prev, float* out, int out_mode, hipStream_t st) {
    const StageArgs a = stage_args<F32>(d, t, w_prev, nullptr, out, 0, 0, out_mode, false);
    const size_t smem = a.table ? tnrd_table_smem_bytes(d.nfilt, d.tab_n)
                                : tnrd_mfma_smem_bytes(d.nfilt, d.nrbf);
    dispatch<F32>(a, [&](auto kc, auto zs) {
        stage_batch<decltype(kc)::value, decltype(zs)::value, F32>(ntiles, smem, st, desc, tiles,
                                                                   a);
    });
}

}  // namespace

size_t tnrd_mfma_smem_bytes(int F, int J) {
    return sizeof(float) *
           ((size_t)UH * UW + (size_t)NPOS * row_stride(F) + (size_t)F * (J + 2 * WPAD));
}

bool tnrd_mfma_fits(int F, int J) { return tnrd_mfma_smem_bytes(F, J) <= 64 * 1024; }

size_t tnrd_table_smem_bytes(int F, int tab_n) {
    return sizeof(float) * ((size_t)UH * UW + (size_t)NPOS * row_stride(F)) +
           16 * (size_t)F * tab_n;
}

int tnrd_table_intervals(double dmu, double gamma, int J) {
    const double span = (J - 1) * dmu + 2 * kTabReach * gamma;
    return (int)ceil(span / (kTabStep * gamma));
}

bool launch_tnrd_stage_bf16(const TnrdDev& d, int t, const float* w_prev, const float* f,
                            float* out, int H, int W, int out_mode, hipStream_t st,
                            const ResidualReq* rq) {
    return launch_single<false>(d, t, w_prev, f, out, H, W, out_mode, st, rq);
}

int tnrd_rule_threads(int H, int W) {
    return ((W + TW - 1) / TW) * ((H + TH - 1) / TH) < kWideStageBelow ? 1024 : 512;
}

void launch_tnrd_stage_mixed_batch(const TnrdDev& db, const TnrdDev& df, int t,
                                   const ImgDesc* desc, const TileRef* tiles, int ntiles,
                                   const float* w_prev, float* out, int out_mode, hipStream_t st) {
    const StageArgs b = stage_args<false>(db, t, w_prev, nullptr, out, 0, 0, out_mode, false);
    const StageArgs f = stage_args<true>(df, t, w_prev, nullptr, out, 0, 0, out_mode, false);
    const size_t smem = tnrd_mfma_smem_bytes(db.nfilt, db.nrbf);
    const bool z33 = row_stride(db.nfilt) == 33;
#define REDVE_MIXED(KB, KF, ZS)                                                                \
    k_tnrd_stage_mixed_batch<KB, KF, ZS><<<ntiles, 512, smem, st>>>(                             \
        desc, tiles, b.w, b.out, b.bf, b.ba, f.bf, f.ba, b.wf, b.F, b.rc, f.rc, b.theta, b.out_mode)
    const int kb = b.rc.K == 5 ? 5 : 0, kf = f.rc.K == 7 ? 7 : 0;
    if (kb == 5 && kf == 7) {
        if (z33) REDVE_MIXED(5, 7, 33); else REDVE_MIXED(5, 7, 25);
    } else {
        if (z33) REDVE_MIXED(0, 0, 33); else REDVE_MIXED(0, 0, 25);
    }
#undef REDVE_MIXED
}

bool tnrd_fuses_residual(const TnrdDev& d) {
    if (d.precision == REDVE_PREC_BF16) return d.phi_tab != nullptr;
    return tnrd_mfma_fits(d.nfilt, d.nrbf) && d.kwin == 7;
}

void launch_tnrd_stage_bf16_batch(const TnrdDev& d, int t, const ImgDesc* desc,
                                  const TileRef* tiles, int ntiles, const float* w_prev, float* out,
                                  int out_mode, hipStream_t st) {
    launch_batch<false>(d, t, desc, tiles, ntiles, w_prev, out, out_mode, st);
}

bool launch_tnrd_stage(const TnrdDev& d, int t, const float* w_prev, const float* f, float* out,
                       int H, int W, int out_mode, hipStream_t st, const ResidualReq* rq) {
    if (tnrd_mfma_fits(d.nfilt, d.nrbf))
        return launch_single<true>(d, t, w_prev, f, out, H, W, out_mode, st, rq);
    launch_tnrd_stage_valu(d, t, w_prev, f, out, H, W, out_mode, st);
    return false;
}

void launch_tnrd_stage_batch(const TnrdDev& d, int t, const ImgDesc* desc, const TileRef* tiles,
                             int ntiles, const float* w_prev, float* out, int out_mode,
                             hipStream_t st) {
    if (tnrd_mfma_fits(d.nfilt, d.nrbf))
        launch_batch<true>(d, t, desc, tiles, ntiles, w_prev, out, out_mode, st);
    else
        launch_tnrd_stage_valu_batch(d, t, desc, tiles, ntiles, w_prev, out, out_mode, st);
}

}  // namespace redve
