// Degradation operator H = S B (Sec. II-A, eq. (1)) and the conjugate-gradient linear step of
// the FP iteration (Sec. II-B, eq. (7); its footnote allows iterative solvers).
//
// Layout: images row-major FP32, dense rows. B is periodic (block-circulant).
// The CG matrix-vector product q = (H^T H / sigma^2 + lambda I) p is an LDS-tiled stencil: a
// workgroup loads a TH x TW tile of p plus a 2r halo (wrapped), forms B p on the tile plus an
// r halo, masks it by the decimation pattern S^T S, and applies B^T on the tile. A rank-1 PSF
// is applied as separate column and row passes (2 (kh + kw) taps per pixel instead of
// 2 kh kw). Reducing kernels loop over tiles with at most kMaxRedBlocks workgroups, publish
// one FP64 partial per workgroup, and the next kernel re-sums them (see reduce.h).
#include <algorithm>
#include <atomic>
#include <tuple>
#include <mutex>
#include <map>

#include "internal.h"
#include "reduce.h"
#include "residual.h"

namespace redve {

namespace {

constexpr int TH = 16, TW = 16;  // CG tile: 256 outputs per 256-thread workgroup
static_assert(TH == kResTH && TW == kResTW, "the residual's tile");
constexpr int MAXR = (kMaxPsf - 1) / 2;
constexpr int PH = TH + 4 * MAXR, PW = TW + 4 * MAXR;
constexpr int NO = TH * TW / kThreads;  // outputs per thread
constexpr int kWideThreadsBlk = 1024;  // threads of the two-iteration CG kernels

// i mod n in [0, n). Stencil indexes are at most one period outside [0, n) unless the image
// is smaller than the halo; only then is the division needed.
__device__ inline int wrapi(int i, int n) {
    int r = i < 0 ? i + n : (i >= n ? i - n : i);
    if ((unsigned)r >= (unsigned)n) {
        r = i % n;
        r = r < 0 ? r + n : r;
    }
    return r;
}

// y[i,j] = sum_{a,b} psf[a+rh][b+rw] x[(s i - a) mod H][(s j - b) mod W]
__global__ __launch_bounds__(kThreads) void k_apply_H(const float* __restrict__ x, int H, int W,
                                                      const float* __restrict__ psf, int kh,
                                                      int kw, int s, float* __restrict__ y) {
    const int h = (H + s - 1) / s, w = (W + s - 1) / s;
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx >= h * w) return;
    const int i = idx / w, j = idx % w;
    const int rh = kh / 2, rw = kw / 2;
    float acc = 0.f;
    for (int a = -rh; a <= rh; ++a) {
        const float* row = x + (size_t)wrapi(s * i - a, H) * W;
        for (int b = -rw; b <= rw; ++b) acc += psf[(a + rh) * kw + b + rw] * row[wrapi(s * j - b, W)];
    }
    y[idx] = acc;
}

// out[i,j] = scale * sum_{a,b} psf[a+rh][b+rw] (S^T y)[(i+a) mod H][(j+b) mod W]
__global__ __launch_bounds__(kThreads) void k_apply_Ht(const float* __restrict__ y, int H, int W,
                                                       const float* __restrict__ psf, int kh,
                                                       int kw, int s, float scale,
                                                       float* __restrict__ out) {
    const int w = (W + s - 1) / s;
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx >= H * W) return;
    const int i = idx / W, j = idx % W;
    const int rh = kh / 2, rw = kw / 2;
    float acc = 0.f;
    for (int a = -rh; a <= rh; ++a) {
        const int gi = wrapi(i + a, H);
        if (gi % s) continue;
        for (int b = -rw; b <= rw; ++b) {
            const int gj = wrapi(j + b, W);
            if (gj % s) continue;
            acc += psf[(a + rh) * kw + b + rw] * y[(size_t)(gi / s) * w + gj / s];
        }
    }
    out[idx] = scale * acc;
}

// LDS of one tile product, sized for stencil radius RS (RS = 0: any radius up to MAXR): the P
// region (tile + 2r halo), the row-pass results, and B P masked by S^T S on the tile + r halo.
template <int RS>
struct __align__(16) TileSmem {
    static constexpr int S = RS ? TW + 4 * RS : PW;   // row stride of every region
    static constexpr int RP = RS ? TH + 4 * RS : PH;  // rows of the P and row-pass regions
    static constexpr int RT = RS ? TH + 2 * RS : PH;  // rows of the B P region
    float p[RP * S];
    float h[RP * S];
    float t[RT * S];
};

// Row pass of B^T B over the rows of X (nr rows, stride xs) at nc output columns:
// out[r][c] = sum_j acr[j] X[r][c + j]. Each item is four adjacent outputs from one window of
// 4 RS + 4 values, read as 16-byte words (xs, nc multiples of 4, X 16-byte aligned): a
// quarter of the LDS reads of one output per item, the same sums in the same order.
template <int RS, int NTH>
__device__ inline void ac_rows(const LinOp& op, const float* X, int xs, int nr, int nc,
                               float* out) {
    constexpr int KA = 4 * RS + 1, NWIN = KA + 3;
    static_assert(NWIN % 4 == 0, "whole 16-byte words");
    const int nq = nc / 4;
    for (int e = threadIdx.x; e < nr * nq; e += NTH) {
        const int r = e / nq, c = (e % nq) * 4;
        const float4* x4 = reinterpret_cast<const float4*>(X + r * xs + c);
        float x[NWIN];
#pragma unroll
        for (int i = 0; i < NWIN / 4; ++i) {
            const float4 v = x4[i];
            x[4 * i] = v.x;
            x[4 * i + 1] = v.y;
            x[4 * i + 2] = v.z;
            x[4 * i + 3] = v.w;
        }
        float o0 = 0.f, o1 = 0.f, o2 = 0.f, o3 = 0.f;
#pragma unroll
        for (int j = 0; j < KA; ++j) {
            o0 += op.acr[j] * x[j];
            o1 += op.acr[j] * x[j + 1];
            o2 += op.acr[j] * x[j + 2];
            o3 += op.acr[j] * x[j + 3];
        }
        *reinterpret_cast<float4*>(out + r * nc + c) = make_float4(o0, o1, o2, o3);
    }
}

// Column pass completing A = B^T B / sigma^2 + lambda I at an nr x nc region: h holds the row
// pass (stride nc, nr + 4 RS rows), X the input (stride xs) whose point (r, c) of the output
// sits at X[r + 2 RS][c + 2 RS]. Each item is four outputs down one column (nr a multiple of
// 4), from one window of 4 RS + 4 values of h.
template <int RS, int NTH>
__device__ inline void ac_cols(const LinOp& op, const float* h, const float* X, int xs, int nr,
                               int nc, float* out) {
    constexpr int KA = 4 * RS + 1, NWIN = KA + 3;
    const int nq = nr / 4;
    for (int e = threadIdx.x; e < nq * nc; e += NTH) {
        const int r = (e / nc) * 4, c = e % nc;
        const float* hc = h + r * nc + c;
        float x[NWIN];
#pragma unroll
        for (int i = 0; i < NWIN; ++i) x[i] = hc[i * nc];
        float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < KA; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] += op.acc[i] * x[i + k];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            out[(r + k) * nc + c] =
                op.inv_s2 * o[k] + op.lambda * X[(r + k + 2 * RS) * xs + c + 2 * RS];
    }
}

// q = A P on the tile at (r0, c0). P must already be in sm.p on the tile + 2r halo (region
// origin (r0 - 2rh, c0 - 2rw)). Returns P and q at the thread's NO outputs. RS > 0: separable
// PSF of compile-time radius RS (fully unrolled passes); RS == 0: runtime sizes (separable or
// general 2-D). NTH threads share the passes; with NTH > kThreads (one output per thread of
// the first kThreads) the other threads only help with the halo passes and get no output.
template <int RS, int NTH = kThreads>
__device__ inline void tile_A_from_lds(const LinOp& op, int H, int W, int r0, int c0,
                                       TileSmem<RS>& sm, float (&pc)[NO], float (&q)[NO]) {
    constexpr int SW = TileSmem<RS>::S;
    const int rh = RS ? RS : op.kh / 2, rw = RS ? RS : op.kw / 2;
    const int kh = 2 * rh + 1, kw = 2 * rw + 1;
    const int ph = TH + 4 * rh;                    // P region rows
    const int bh = TH + 2 * rh, bw = TW + 2 * rw;  // B P region
    const int s = op.decim;
    if constexpr (RS > 0) {
        if (s == 1) {
            // no decimation: B^T B is separable with the autocorrelations of row and col
            // (4 RS + 1 taps): a row pass over the P rows at the tile's columns, then the
            // column pass at the tile
            constexpr int KA = 4 * RS + 1;
            ac_rows<RS, NTH>(op, sm.p, SW, ph, TW, sm.h);  // h: stride TW
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                const int o = threadIdx.x + k * kThreads;
                if (NTH > kThreads && o >= TH * TW) break;
                const int tr = o / TW, tc = o % TW;
                const float* hcol = sm.h + tr * TW + tc;
                float acc = 0.f;
#pragma unroll
                for (int i = 0; i < KA; ++i) acc += op.acc[i] * hcol[i * TW];
                pc[k] = sm.p[(tr + 2 * RS) * SW + tc + 2 * RS];
                q[k] = op.inv_s2 * acc + op.lambda * pc[k];
            }
            __syncthreads();
            return;
        }
    }
    if (RS || op.separable) {
        // row pass over all P rows, B columns: h[pr][bc] = sum_b row[b] P[pr][bc + 2rw - b]
        for (int e = threadIdx.x; e < ph * bw; e += NTH) {
            const int pr = e / bw, bc = e % bw;
            const float* prow = sm.p + pr * SW + bc + 2 * rw;
            float acc = 0.f;
#pragma unroll
            for (int b = 0; b < (RS ? 2 * RS + 1 : kMaxPsf); ++b) {
                if (!RS && b >= kw) break;
                acc += op.row[b] * prow[-b];
            }
            sm.h[pr * SW + bc] = acc;
        }
        __syncthreads();
        // column pass + decimation mask: t[br][bc] = m * sum_a col[a] h[br + 2rh - a][bc]
        for (int e = threadIdx.x; e < bh * bw; e += NTH) {
            const int br = e / bw, bc = e % bw;
            float acc = 0.f;
            bool keep = true;
            if (s > 1) {
                const int gr = wrapi(r0 - rh + br, H), gc = wrapi(c0 - rw + bc, W);
                keep = gr % s == 0 && gc % s == 0;
            }
            if (keep) {
                const float* hcol = sm.h + (br + 2 * rh) * SW + bc;
#pragma unroll
                for (int a = 0; a < (RS ? 2 * RS + 1 : kMaxPsf); ++a) {
                    if (!RS && a >= kh) break;
                    acc += op.col[a] * hcol[-a * SW];
                }
            }
            sm.t[br * SW + bc] = acc;
        }
        __syncthreads();
        // B^T row pass: h[br][tc] = sum_b row[b] t[br][tc + b]
        for (int e = threadIdx.x; e < bh * TW; e += NTH) {
            const int br = e / TW, tc = e % TW;
            const float* trow = sm.t + br * SW + tc;
            float acc = 0.f;
#pragma unroll
            for (int b = 0; b < (RS ? 2 * RS + 1 : kMaxPsf); ++b) {
                if (!RS && b >= kw) break;
                acc += op.row[b] * trow[b];
            }
            sm.h[br * SW + tc] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int o = threadIdx.x + k * kThreads;
            if (NTH > kThreads && o >= TH * TW) break;
            const int tr = o / TW, tc = o % TW;
            const float* hcol = sm.h + tr * SW + tc;
            float acc = 0.f;
#pragma unroll
            for (int a = 0; a < (RS ? 2 * RS + 1 : kMaxPsf); ++a) {
                if (!RS && a >= kh) break;
                acc += op.col[a] * hcol[a * SW];
            }
            pc[k] = sm.p[(tr + 2 * rh) * SW + tc + 2 * rw];
            q[k] = op.inv_s2 * acc + op.lambda * pc[k];
        }
    } else {
        for (int e = threadIdx.x; e < bh * bw; e += NTH) {
            const int br = e / bw, bc = e % bw;
            const int gr = wrapi(r0 - rh + br, H), gc = wrapi(c0 - rw + bc, W);
            float acc = 0.f;
            if (gr % s == 0 && gc % s == 0) {
                for (int a = -rh; a <= rh; ++a) {
                    const float* prow = sm.p + (br + rh - a) * SW + bc + rw;
                    const float* krow = op.psf + (a + rh) * op.kw + rw;
                    for (int b = -rw; b <= rw; ++b) acc += krow[b] * prow[-b];
                }
            }
            sm.t[br * SW + bc] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int o = threadIdx.x + k * kThreads;
            if (NTH > kThreads && o >= TH * TW) break;
            const int tr = o / TW, tc = o % TW;
            float acc = 0.f;
            for (int a = -rh; a <= rh; ++a) {
                const float* trow = sm.t + (tr + a + rh) * SW + tc + rw;
                const float* krow = op.psf + (a + rh) * op.kw + rw;
                for (int b = -rw; b <= rw; ++b) acc += krow[b] * trow[b];
            }
            pc[k] = sm.p[(tr + 2 * rh) * SW + tc + 2 * rw];
            q[k] = op.inv_s2 * acc + op.lambda * pc[k];
        }
    }
    __syncthreads();
}

// Loads f(g) for every position of the P region of the tile at (r0, c0) into sm.p.
template <int RS, typename F>
__device__ inline void tile_load(const LinOp& op, int H, int W, int r0, int c0, TileSmem<RS>& sm,
                                 F f) {
    constexpr int SW = TileSmem<RS>::S;
    const int rh = RS ? RS : op.kh / 2, rw = RS ? RS : op.kw / 2;
    const int ph = TH + 4 * rh, pw = TW + 4 * rw;
    for (int e = threadIdx.x; e < ph * pw; e += kThreads) {
        const int pr = e / pw, pcol = e % pw;
        const size_t g = (size_t)wrapi(r0 - 2 * rh + pr, H) * W + wrapi(c0 - 2 * rw + pcol, W);
        sm.p[pr * SW + pcol] = f(g);
    }
    __syncthreads();
}

__device__ inline void tile_origin(int t, int W, int& r0, int& c0) {
    const int ntx = (W + TW - 1) / TW;
    r0 = (t / ntx) * TH;
    c0 = (t % ntx) * TW;
}

__device__ inline int ntiles(int H, int W) { return ((H + TH - 1) / TH) * ((W + TW - 1) / TW); }

template <int RS>
__global__ __launch_bounds__(kThreads) void k_apply_A(const LinOp op, const float* __restrict__ p,
                                                      int H, int W, float* __restrict__ out) {
    __shared__ TileSmem<RS> sm;
    const int nt = ntiles(H, W);
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        int r0, c0;
        tile_origin(xcd_tile(t, nt), W, r0, c0);
        tile_load<RS>(op, H, W, r0, c0, sm, [&](size_t g) { return p[g]; });
        float pc[NO], q[NO];
        tile_A_from_lds<RS>(op, H, W, r0, c0, sm, pc, q);
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int o = threadIdx.x + k * kThreads;
            const int gr = r0 + o / TW, gc = c0 + o % TW;
            if (gr < H && gc < W) out[(size_t)gr * W + gc] = q[k];
        }
    }
}

// Generic CG start: r = rhs - A x_in.
template <int RS>
__global__ __launch_bounds__(kThreads) void k_cg_init(const LinOp op, const float* __restrict__ x_in,
                                                      const float* __restrict__ rhs,
                                                      float* __restrict__ r, int H, int W) {
    __shared__ TileSmem<RS> sm;
    const int nt = ntiles(H, W);
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        int r0, c0;
        tile_origin(xcd_tile(t, nt), W, r0, c0);
        tile_load<RS>(op, H, W, r0, c0, sm, [&](size_t g) { return x_in[g]; });
        float pc[NO], q[NO];
        tile_A_from_lds<RS>(op, H, W, r0, c0, sm, pc, q);
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int o = threadIdx.x + k * kThreads;
            const int gr = r0 + o / TW, gc = c0 + o % TW;
            if (gr < H && gc < W) {
                const size_t g = (size_t)gr * W + gc;
                r[g] = rhs[g] - q[k];
            }
        }
    }
}

// LDS of the FP64 residual start on one tile, sized for stencil radius RS (0: any radius up to
// MAXR): the P region of x, e on the tile + r halo, row-pass results.
template <int RS>
struct InitFpSmem {
    static constexpr int S = RS ? TW + 4 * RS : PW;
    static constexpr int RP = RS ? TH + 4 * RS : PH;
    static constexpr int RT = RS ? TH + 2 * RS : PH;
    float sp[RP * S];
    double se[RT * S];
    double sh[RP * S];
};

// r = H^T (y - H x) / sigma^2 + lambda s on the tile at (r0, c0); FP64 sums.
template <int RS>
__device__ inline void init_fp_tile(const LinOp& op, const float* __restrict__ x,
                                    const float* __restrict__ y, const float* __restrict__ s,
                                    float* __restrict__ r, int H, int W, int r0, int c0,
                                    InitFpSmem<RS>& sm, float* __restrict__ xo = nullptr) {
    constexpr int SW = InitFpSmem<RS>::S;
    float* sp = sm.sp;
    double* se = sm.se;
    double* sh = sm.sh;
    const int rh = op.kh / 2, rw = op.kw / 2, dec = op.decim;
    const int ph = TH + 4 * rh, pw = TW + 4 * rw;
    const int bh = TH + 2 * rh, bw = TW + 2 * rw;
    const int wy = (W + dec - 1) / dec;
    for (int e = threadIdx.x; e < ph * pw; e += kThreads) {
        const int pr = e / pw, pc = e % pw;
        sp[pr * SW + pc] = x[(size_t)wrapi(r0 - 2 * rh + pr, H) * W + wrapi(c0 - 2 * rw + pc, W)];
    }
    __syncthreads();
    if (op.separable) {
        for (int e = threadIdx.x; e < ph * bw; e += kThreads) {
            const int pr = e / bw, bc = e % bw;
            const float* prow = sp + pr * SW + bc + 2 * rw;
            double a = 0.0;
            for (int b = 0; b < op.kw; ++b) a += op.row_d[b] * (double)prow[-b];
            sh[pr * SW + bc] = a;
        }
        __syncthreads();
    }
    // e = S^T (y - S B x) on the tile + r halo, FP64
    for (int e = threadIdx.x; e < bh * bw; e += kThreads) {
        const int br = e / bw, bc = e % bw;
        const int gr = wrapi(r0 - rh + br, H), gc = wrapi(c0 - rw + bc, W);
        double v = 0.0;
        if (gr % dec == 0 && gc % dec == 0) {
            double bx = 0.0;
            if (op.separable) {
                const double* hcol = sh + (br + 2 * rh) * SW + bc;
                for (int a = 0; a < op.kh; ++a) bx += op.col_d[a] * hcol[-a * SW];
            } else {
                for (int a = -rh; a <= rh; ++a) {
                    const float* prow = sp + (br + rh - a) * SW + bc + rw;
                    const double* krow = op.psf64 + (a + rh) * op.kw + rw;
                    for (int b = -rw; b <= rw; ++b) bx += krow[b] * (double)prow[-b];
                }
            }
            v = (double)y[(size_t)(gr / dec) * wy + gc / dec] - bx;
        }
        se[br * SW + bc] = v;
    }
    __syncthreads();
    if (op.separable) {
        for (int e = threadIdx.x; e < bh * TW; e += kThreads) {
            const int br = e / TW, tc = e % TW;
            const double* erow = se + br * SW + tc;
            double a = 0.0;
            for (int b = 0; b < op.kw; ++b) a += op.row_d[b] * erow[b];
            sh[br * SW + tc] = a;
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int tr = o / TW, tc = o % TW;
        const int gr = r0 + tr, gc = c0 + tc;
        double bt = 0.0;
        if (op.separable) {
            const double* hcol = sh + tr * SW + tc;
            for (int a = 0; a < op.kh; ++a) bt += op.col_d[a] * hcol[a * SW];
        } else {
            for (int a = -rh; a <= rh; ++a) {
                const double* erow = se + (tr + a + rh) * SW + tc + rw;
                const double* krow = op.psf64 + (a + rh) * op.kw + rw;
                for (int b = -rw; b <= rw; ++b) bt += krow[b] * erow[b];
            }
        }
        if (gr < H && gc < W) {
            const size_t g = (size_t)gr * W + gc;
            double rv = op.inv_s2_d * bt;
            if (s) rv += op.lambda_d * (double)s[g];
            if (xo)  // steepest descent: x - mu g(x) = x + mu r, rounded once
                xo[g] = (float)((double)sp[(tr + 2 * rh) * SW + tc + 2 * rw] + op.sd_mu * rv);
            else
                r[g] = (float)rv;
        }
    }
    __syncthreads();
}

// init_fp_tile for a separable square PSF of compile-time radius RS (the same sums in the same
// order), with every global load issued at the start: x on the P region, y at the B region's
// sampled positions, s at the thread's pixel.
template <int RS>
__device__ inline void init_fp_tile_rs(const LinOp& op, const float* __restrict__ x,
                                       const float* __restrict__ y, const float* __restrict__ s,
                                       float* __restrict__ r, int H, int W, int r0, int c0,
                                       InitFpSmem<RS>& sm, float* __restrict__ xo) {
    static_assert(RS > 0 && NO == 1 && kThreads == TH * TW, "compile-time radius, one pixel per thread");
    static_assert(InitFpSmem<RS>::S == ResidualIn<RS, kThreads>::SW, "the shared layout");
    constexpr int SW = InitFpSmem<RS>::S;
    ResidualIn<RS, kThreads> in;
    residual_fetch<RS, kThreads>(op.decim, x, y, H, W, r0, c0, in);
    const int tr = threadIdx.x / TW, tc = threadIdx.x % TW;
    const int gr = r0 + tr, gc = c0 + tc;
    const bool pix = gr < H && gc < W;
    const float sv = (s && pix) ? s[(size_t)gr * W + gc] : 0.f;
    const double bt = residual_bt<RS, kThreads>(op, in, sm.sp, sm.se, sm.sh);
    if (pix) {
        const size_t g = (size_t)gr * W + gc;
        double rv = op.inv_s2_d * bt;
        if (s) rv += op.lambda_d * (double)sv;
        if (xo)  // steepest descent: x - mu g(x) = x + mu r, rounded once
            xo[g] = (float)((double)sm.sp[(tr + 2 * RS) * SW + tc + 2 * RS] + op.sd_mu * rv);
        else
            r[g] = (float)rv;
    }
    __syncthreads();
}

// CG start of one FP call (eq. (7)) in residual form. With rhs = H^T y / sigma^2 + lambda f(x),
//   r = rhs - A x = H^T (y - H x) / sigma^2 + lambda (f(x) - x),
// both terms small near the fixed point; the data term is accumulated in FP64 from the FP32
// image, so r carries no rounding of the O(|x|) quantities rhs and A x. s = f(x) - x (null:
// the identity denoiser, s = 0).
template <int RS>
__global__ __launch_bounds__(kThreads) void k_cg_init_fp(const LinOp op, const float* __restrict__ x,
                                                         const float* __restrict__ y,
                                                         const float* __restrict__ s,
                                                         float* __restrict__ r, int H, int W,
                                                         float* __restrict__ xo) {
    __shared__ InitFpSmem<RS> sm;
    const int nt = ntiles(H, W);
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        int r0, c0;
        tile_origin(xcd_tile(t, nt), W, r0, c0);
        if constexpr (RS > 0)
            init_fp_tile_rs<RS>(op, x, y, s, r, H, W, r0, c0, sm, xo);
        else
            init_fp_tile<RS>(op, x, y, s, r, H, W, r0, c0, sm, xo);
    }
}

// w0 = A r0 on one tile; accumulates r0.r0 and w0.r0.
template <int RS>
__device__ inline void w0_tile(const LinOp& op, const float* __restrict__ r, float* __restrict__ w,
                               int H, int W, int r0, int c0, TileSmem<RS>& sm, double (&acc)[2]) {
    tile_load<RS>(op, H, W, r0, c0, sm, [&](size_t g) { return r[g]; });
    float pc[NO], q[NO];
    tile_A_from_lds<RS>(op, H, W, r0, c0, sm, pc, q);
#pragma unroll
    for (int k = 0; k < NO; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int gr = r0 + o / TW, gc = c0 + o % TW;
        if (gr < H && gc < W) {
            w[(size_t)gr * W + gc] = q[k];
            acc[0] += (double)pc[k] * (double)pc[k];
            acc[1] += (double)q[k] * (double)pc[k];
        }
    }
}

// Second half of the CG start: w0 = A r0; publishes rho0 = r0.r0 and mu0 = w0.r0.
template <int RS>
__global__ __launch_bounds__(kThreads) void k_cg_w0(const LinOp op, const float* __restrict__ r,
                                                    float* __restrict__ w, int H, int W,
                                                    double* __restrict__ part) {
    __shared__ TileSmem<RS> sm;
    __shared__ double sred[2 * kThreads / 64];
    double acc[2] = {0.0, 0.0};
    const int nt = ntiles(H, W);
    if (nt <= (int)gridDim.x) {  // one tile per workgroup: the sums before the store
        int r0, c0;
        tile_origin(xcd_tile(blockIdx.x, nt), W, r0, c0);
        tile_load<RS>(op, H, W, r0, c0, sm, [&](size_t g) { return r[g]; });
        float pc[NO], q[NO];
        tile_A_from_lds<RS>(op, H, W, r0, c0, sm, pc, q);
        const int gr = r0 + threadIdx.x / TW, gc = c0 + threadIdx.x % TW;
        const bool pix = gr < H && gc < W;
        if (pix) {
            acc[0] += (double)pc[0] * (double)pc[0];
            acc[1] += (double)q[0] * (double)pc[0];
        }
        block_sum<2>(acc, sred);
        if (pix) w[(size_t)gr * W + gc] = q[0];
        publish<2>(acc, part, kMaxRedBlocks, blockIdx.x);
        return;
    }
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        int r0, c0;
        tile_origin(xcd_tile(t, nt), W, r0, c0);
        w0_tile<RS>(op, r, w, H, W, r0, c0, sm, acc);
    }
    block_sum<2>(acc, sred);
    publish<2>(acc, part, kMaxRedBlocks, blockIdx.x);
}

// Step lengths of the single-reduction CG from rho_k, mu_k and the previous iteration's
// alpha and rho (a vanished residual gives alpha = beta = 0: the iteration stops moving).
__device__ inline void cg_scalars(int k, double rho, double mu, double alpha_prev, double rho_prev,
                                  double& alpha, double& beta) {
    alpha = 0.0;
    beta = 0.0;
    if (rho > 1e-300) {
        if (k == 0) {
            alpha = mu > 0.0 ? rho / mu : 0.0;
        } else {
            // beta rho / alpha_prev as rho^2 / (rho_prev alpha_prev): two divisions in parallel,
            // then the third
            const bool prev = rho_prev > 1e-300;
            beta = prev ? rho / rho_prev : 0.0;
            const double t = prev && alpha_prev != 0.0 ? (rho * rho) / (rho_prev * alpha_prev) : 0.0;
            const double den = alpha_prev != 0.0 ? mu - t : 0.0;
            alpha = den > 0.0 ? rho / den : 0.0;
        }
    }
}

// One single-reduction CG iteration on one tile (see k_cg_iter); accumulates rho_{k+1}, mu_{k+1}.
template <int RS>
__device__ inline void cg_iter_tile(const LinOp& op, int H, int W, int r0, int c0, int k,
                                    float alpha, float beta, const float* __restrict__ r_in,
                                    const float* __restrict__ w_in, const float* __restrict__ s_in,
                                    float* __restrict__ r_out, float* __restrict__ w_out,
                                    float* __restrict__ s_out, float* __restrict__ p,
                                    float* __restrict__ d, TileSmem<RS>& sm, double (&acc)[2]) {
    tile_load<RS>(op, H, W, r0, c0, sm, [&](size_t g) {
        const float sk = k ? w_in[g] + beta * s_in[g] : w_in[g];
        return r_in[g] - alpha * sk;
    });
    float r1[NO], w1[NO];
    tile_A_from_lds<RS>(op, H, W, r0, c0, sm, r1, w1);
#pragma unroll
    for (int kk = 0; kk < NO; ++kk) {
        const int o = threadIdx.x + kk * kThreads;
        const int gr = r0 + o / TW, gc = c0 + o % TW;
        if (gr < H && gc < W) {
            const size_t g = (size_t)gr * W + gc;
            const float rk = r_in[g];
            const float sk = k ? w_in[g] + beta * s_in[g] : w_in[g];
            const float pk = k ? rk + beta * p[g] : rk;
            const float dn = k ? d[g] + alpha * pk : alpha * pk;
            s_out[g] = sk;
            p[g] = pk;
            d[g] = dn;
            r_out[g] = r1[kk];
            w_out[g] = w1[kk];
            acc[0] += (double)r1[kk] * (double)r1[kk];
            acc[1] += (double)w1[kk] * (double)r1[kk];
        }
    }
}

// The last iteration on one tile: only x_out = x_in + d_k + alpha p_k.
__device__ inline void cg_last_tile(int H, int W, int r0, int c0, int k, float alpha, float beta,
                                    const float* __restrict__ r_in, const float* __restrict__ p,
                                    const float* __restrict__ d, const float* __restrict__ x_in,
                                    float* __restrict__ x_out) {
#pragma unroll
    for (int kk = 0; kk < NO; ++kk) {
        const int o = threadIdx.x + kk * kThreads;
        const int gr = r0 + o / TW, gc = c0 + o % TW;
        if (gr < H && gc < W) {
            const size_t g = (size_t)gr * W + gc;
            const float pk = k ? r_in[g] + beta * p[g] : r_in[g];
            const float dn = k ? d[g] + alpha * pk : alpha * pk;
            x_out[g] = x_in[g] + dn;
        }
    }
}

// Raw inputs of one CG iteration on one tile, loaded before the step lengths are known so that
// these loads overlap the reduction that produces alpha and beta: r_k, w_k, s_{k-1} on the P
// region (tile + 2r halo) and r_k, w_k, s_{k-1}, p_{k-1}, d_k at the thread's output pixel.
template <int RS, int NTH = kThreads>
struct CgIn {
    static constexpr int PHr = TH + 4 * RS, PWr = TW + 4 * RS;
    static constexpr int NE = (PHr * PWr + NTH - 1) / NTH;
    float r[NE], w[NE], s[NE];
    float ro, wo, so, po, dn;
};
static_assert(NO == 1, "one output pixel per thread");

template <int RS, int NTH = kThreads>
__device__ inline void cg_fetch(int H, int W, int r0, int c0, int k, const float* __restrict__ r_in,
                                const float* __restrict__ w_in, const float* __restrict__ s_in,
                                const float* __restrict__ p, const float* __restrict__ d,
                                CgIn<RS, NTH>& f) {
    using C = CgIn<RS, NTH>;
#pragma unroll
    for (int i = 0; i < C::NE; ++i) {
        const int e = threadIdx.x + i * NTH;
        f.r[i] = f.w[i] = f.s[i] = 0.f;
        if (e < C::PHr * C::PWr) {
            const int pr = e / C::PWr, pc = e % C::PWr;
            const size_t g =
                (size_t)wrapi(r0 - 2 * RS + pr, H) * W + wrapi(c0 - 2 * RS + pc, W);
            f.r[i] = r_in[g];
            f.w[i] = w_in[g];
            if (k) f.s[i] = s_in[g];
        }
    }
    f.ro = f.wo = f.so = f.po = f.dn = 0.f;
    const int gr = r0 + threadIdx.x / TW, gc = c0 + threadIdx.x % TW;
    if ((NTH == kThreads || threadIdx.x < TH * TW) && gr < H && gc < W) {
        const size_t g = (size_t)gr * W + gc;
        f.ro = r_in[g];
        f.wo = w_in[g];
        if (k) {
            f.so = s_in[g];
            f.po = p[g];
            f.dn = d[g];
        }
    }
}

// Outputs of one CG iteration at a thread's pixel g (valid: the thread has a pixel in the image).
struct CgOut {
    size_t g;
    float s, p, d, r, w;
    bool valid;
};

// cg_iter_tile on prefetched inputs (the same arithmetic), returning the outputs unstored.
template <int RS, int NTH = kThreads>
__device__ inline CgOut cg_iter_compute(const LinOp& op, int H, int W, int r0, int c0, int k,
                                        float alpha, float beta, const CgIn<RS, NTH>& f,
                                        TileSmem<RS>& sm, double (&acc)[2]) {
    using C = CgIn<RS, NTH>;
    constexpr int SW = TileSmem<RS>::S;
#pragma unroll
    for (int i = 0; i < C::NE; ++i) {
        const int e = threadIdx.x + i * NTH;
        if (e < C::PHr * C::PWr) {
            const float sk = k ? f.w[i] + beta * f.s[i] : f.w[i];
            sm.p[(e / C::PWr) * SW + e % C::PWr] = f.r[i] - alpha * sk;
        }
    }
    __syncthreads();
    float r1[NO], w1[NO];
    tile_A_from_lds<RS, NTH>(op, H, W, r0, c0, sm, r1, w1);
    CgOut o{};
    const int gr = r0 + threadIdx.x / TW, gc = c0 + threadIdx.x % TW;
    if ((NTH == kThreads || threadIdx.x < TH * TW) && gr < H && gc < W) {
        o.g = (size_t)gr * W + gc;
        o.s = k ? f.wo + beta * f.so : f.wo;
        o.p = k ? f.ro + beta * f.po : f.ro;
        o.d = k ? f.dn + alpha * o.p : alpha * o.p;
        o.r = r1[0];
        o.w = w1[0];
        o.valid = true;
        acc[0] += (double)r1[0] * (double)r1[0];
        acc[1] += (double)w1[0] * (double)r1[0];
    }
    return o;
}

__device__ inline void cg_store(const CgOut& o, float* __restrict__ r_out,
                                float* __restrict__ w_out, float* __restrict__ s_out,
                                float* __restrict__ p, float* __restrict__ d) {
    if (o.valid) {
        s_out[o.g] = o.s;
        p[o.g] = o.p;
        d[o.g] = o.d;
        r_out[o.g] = o.r;
        w_out[o.g] = o.w;
    }
}

template <int RS, int NTH = kThreads>
__device__ inline void cg_iter_fetched(const LinOp& op, int H, int W, int r0, int c0, int k,
                                       float alpha, float beta, const CgIn<RS, NTH>& f,
                                       float* __restrict__ r_out, float* __restrict__ w_out,
                                       float* __restrict__ s_out, float* __restrict__ p,
                                       float* __restrict__ d, TileSmem<RS>& sm,
                                       double (&acc)[2]) {
    cg_store(cg_iter_compute<RS, NTH>(op, H, W, r0, c0, k, alpha, beta, f, sm, acc), r_out, w_out,
             s_out, p, d);
}

// One conjugate-gradient iteration in the single-reduction (Chronopoulos-Gear) form: with
// r_k, w_k = A r_k, rho_k = r_k.r_k, mu_k = w_k.r_k (published by the previous kernel) and
// alpha_{k-1}, rho_{k-1} (hist):
//   beta = rho_k / rho_{k-1},  alpha = rho_k / (mu_k - beta rho_k / alpha_{k-1})  (k = 0:
//   beta = 0, alpha = rho_0 / mu_0)
//   p_k = r_k + beta p_{k-1},  s_k = w_k + beta s_{k-1}  (s = A p)
//   d_{k+1} = d_k + alpha p_k,  r_{k+1} = r_k - alpha s_k,  w_{k+1} = A r_{k+1}
// and publishes rho_{k+1}, mu_{k+1}. In exact arithmetic these are the Hestenes-Stiefel
// iterates; one grid-wide reduction per iteration instead of two. r_{k+1} is formed on the
// tile + halo from r_k, w_k and s_{k-1}, then w_{k+1} is its stencil. On the last iteration
// only x_out = x_in + d_{k+1} is written.
//
// NTH = kThreads: one output pixel per thread. NTH > kThreads (RS > 0, not the last
// iteration): the extra threads share the loads and the halo passes of the tile, for small
// images whose tiles give each CU a single workgroup.
template <int RS, int NTH>
__global__ __launch_bounds__(NTH) void k_cg_iter(
    const LinOp op, int H, int W, int k, int last, const float* __restrict__ r_in,
    const float* __restrict__ w_in, const float* __restrict__ s_in, float* __restrict__ r_out,
    float* __restrict__ w_out, float* __restrict__ s_out, float* __restrict__ p,
    float* __restrict__ d, const float* __restrict__ x_in, float* __restrict__ x_out,
    Partials rm, const double* __restrict__ hist_prev, double* __restrict__ hist_cur,
    double* __restrict__ part) {
    static_assert(NTH == kThreads || RS > 0, "wide workgroups need a compile-time radius");
    __shared__ TileSmem<RS> sm;
    __shared__ double sred[2 * NTH / 64];
    __shared__ double bc[2];
    const int nt = ntiles(H, W);
    int r0 = 0, c0 = 0;
    // Loads in order of need: the published partials and (alpha, rho) of the previous
    // iteration first, then the tile's inputs, so that the step lengths do not wait for those.
    Early2 early;
    const bool early_ok = rm.n <= kEarlyPartials;
    if (early_ok) consume2_issue(rm.p, kMaxRedBlocks, rm.n, early);
    const double alpha_prev = k ? hist_prev[0] : 0.0, rho_prev = k ? hist_prev[1] : 0.0;
    CgIn<RS, NTH> f;
    if constexpr (RS > 0) {
        if (!last && (int)blockIdx.x < nt) {
            tile_origin(xcd_tile(blockIdx.x, nt), W, r0, c0);
            cg_fetch<RS, NTH>(H, W, r0, c0, k, r_in, w_in, s_in, p, d, f);
        }
    }
    double rho, mu;
    if (early_ok)
        consume2_finish(early, bc, rho, mu);
    else
        consume2(rm.p, kMaxRedBlocks, rm.n, bc, rho, mu);
    double alpha_d, beta_d;
    cg_scalars(k, rho, mu, alpha_prev, rho_prev, alpha_d, beta_d);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hist_cur[0] = alpha_d;
        hist_cur[1] = rho;
    }
    const float alpha = (float)alpha_d, beta = (float)beta_d;
    double acc[2] = {0.0, 0.0};
    if constexpr (RS > 0) {
        if (!last && nt <= (int)gridDim.x) {
            // one tile per workgroup: the workgroup sum first, then every store at once
            const CgOut o = cg_iter_compute<RS, NTH>(op, H, W, r0, c0, k, alpha, beta, f, sm, acc);
            block_sum<2, NTH, kThreads>(acc, sred);  // outputs sit in the first kThreads
            cg_store(o, r_out, w_out, s_out, p, d);
            publish<2>(acc, part, kMaxRedBlocks, blockIdx.x);
            return;
        }
    }
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        tile_origin(xcd_tile(t, nt), W, r0, c0);
        if (last) {
            if constexpr (NTH == kThreads)
                cg_last_tile(H, W, r0, c0, k, alpha, beta, r_in, p, d, x_in, x_out);
        } else if constexpr (RS > 0) {
            if (t != (int)blockIdx.x)
                cg_fetch<RS, NTH>(H, W, r0, c0, k, r_in, w_in, s_in, p, d, f);
            cg_iter_fetched<RS, NTH>(op, H, W, r0, c0, k, alpha, beta, f, r_out, w_out, s_out, p,
                                     d, sm, acc);
        } else {
            cg_iter_tile<RS>(op, H, W, r0, c0, k, alpha, beta, r_in, w_in, s_in, r_out, w_out,
                             s_out, p, d, sm, acc);
        }
    }
    if (last) return;
    block_sum<2, NTH>(acc, sred);
    publish<2>(acc, part, kMaxRedBlocks, blockIdx.x);
}

// ---- CG iteration on 32x32 tiles keeping only r, p and d in HBM (large images) ------------
//
// The single-reduction iteration above stores w = A r and s = A p beside r, p, d (40 B per pixel
// and iteration). Here s is recomputed instead, and w is not formed at all: mu = r.A r =
// ||B^T r||^2 / sigma^2 + lambda ||r||^2 for A = B^T B / sigma^2 + lambda I, and with the
// periodic boundary B is circulant, hence normal (B^T B = B B^T), so ||B^T r|| = ||B r||.
// With r_k and p_{k-1} read on the tile + 3 RS halo (2 RS: the radius of A; RS: that of B),
//   p_k = r_k + beta p_{k-1}                  on the tile + 3 RS   (P region)
//   s_k = A p_k,  r_{k+1} = r_k - alpha s_k    on the tile + RS     (S region)
//   q = B^T r_{k+1} (the PSF's correlation)   at the tile's pixels
//   d_{k+1} = d_k + alpha p_k,  rho_{k+1} = r.r,  mu_{k+1} = q.q / sigma^2 + lambda rho
// storing r_{k+1}, p_k (double-buffered: neighbours read p_{k-1} on their halos) and d_{k+1}:
// 24 B per pixel and iteration, the algorithm's own traffic, for one application of A on a
// region 1.56x (RS = 4) the tile and one of B on the tile. The scalars alpha_k, beta_k come from
// rho_k, mu_k as in k_cg_iter, so the iterates are those of the single-reduction form in exact
// arithmetic. Region sides are rounded up to multiples of 4 (16-byte LDS rows; the extra rows
// and columns are halo that no output uses).
constexpr int T32 = 32;
constexpr int kCg32Threads = 512;

template <int RS>
struct __align__(16) Cg32Smem {
    static constexpr int PR = (T32 + 6 * RS + 3) / 4 * 4;  // P region side (origin tile - 3 RS)
    static constexpr int SR = (T32 + 2 * RS + 3) / 4 * 4;  // S region side (origin tile - RS)
    static_assert(PR >= SR + 4 * RS, "the S region's A reads stay in the P region");
    static_assert(SR >= T32 + 2 * RS, "the tile's B reads stay in the S region");
    // the loader: thread t < LR * PR takes column t % PR of rows t / PR + LR i, i < NL; rows
    // PR .. LR NL - 1 are stored too (they repeat row PR - 1) and never read
    static constexpr int LR = kCg32Threads / PR, NL = (PR + LR - 1) / LR, PRX = LR * NL;
    // row strides: an odd number of 16-byte words (16 lanes reading one word each from 16
    // consecutive rows hit 16 different groups of four LDS banks); r is stored RO columns to
    // the right, so that its S region starts on a 16-byte boundary
    static constexpr int RO = (4 - (2 * RS) % 4) % 4;
    static constexpr int odd_words(int n) { return (n / 4) % 2 ? n : n + 4; }
    static constexpr int PS = odd_words(PR);
    static constexpr int RSS = odd_words((PR + RO + 3) / 4 * 4);
    static constexpr int HS = odd_words(SR);
    float p[PRX * PS];   // p_k on the P region
    float r[PRX * RSS];  // r_k on the P region, then r_{k+1} on its S part
    float h[PR * HS];    // A's row pass over the P rows at the S columns, then B's over the S rows
};

// A's row pass over the P rows at the S columns (the autocorrelation of the PSF's row factor),
// into h: four outputs per item from one window of 4 RS + 4 values read as 16-byte words,
// consecutive lanes on consecutive rows. The item loop stays rolled: an unrolled pair of items
// doubles the live window.
template <int RS, int NT>
__device__ inline void cg32_a_rows(const LinOp& op, Cg32Smem<RS>& sm) {
    using M = Cg32Smem<RS>;
    constexpr int SR = M::SR, PR = M::PR, PS = M::PS, HS = M::HS, KA = 4 * RS + 1, NWIN = KA + 3;
    static_assert(NWIN % 4 == 0, "whole 16-byte words");
    constexpr int NQ = SR / 4;
#pragma unroll 1
    for (int e = threadIdx.x; e < PR * NQ; e += NT) {
        const int r = e % PR, c = (e / PR) * 4;
        const float4* x4 = reinterpret_cast<const float4*>(sm.p + r * PS + c);
        float x[NWIN];
#pragma unroll
        for (int i = 0; i < NWIN / 4; ++i) {
            const float4 v = x4[i];
            x[4 * i] = v.x;
            x[4 * i + 1] = v.y;
            x[4 * i + 2] = v.z;
            x[4 * i + 3] = v.w;
        }
        float o0 = 0.f, o1 = 0.f, o2 = 0.f, o3 = 0.f;
#pragma unroll
        for (int j = 0; j < KA; ++j) {
            o0 += op.acr[j] * x[j];
            o1 += op.acr[j] * x[j + 1];
            o2 += op.acr[j] * x[j + 2];
            o3 += op.acr[j] * x[j + 3];
        }
        *reinterpret_cast<float4*>(sm.h + r * HS + c) = make_float4(o0, o1, o2, o3);
    }
}

// r_{k+1} = r_k - alpha (A p)_k on the S region, in place in sm.r: the column pass of A from
// its row pass h, four outputs down a column per item.
template <int RS, int NT>
__device__ inline void cg32_update_r(const LinOp& op, Cg32Smem<RS>& sm, float alpha) {
    using M = Cg32Smem<RS>;
    constexpr int SR = M::SR, PS = M::PS, RSS = M::RSS, HS = M::HS, RO = M::RO;
    constexpr int KA = 4 * RS + 1, NWIN = KA + 3;
#pragma unroll 1
    for (int e = threadIdx.x; e < (SR / 4) * SR; e += NT) {
        const int r = (e / SR) * 4, c = e % SR;
        const float* hc = sm.h + r * HS + c;
        float x[NWIN];
#pragma unroll
        for (int i = 0; i < NWIN; ++i) x[i] = hc[i * HS];
        float o[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < KA; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] += op.acc[i] * x[i + k];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float sv =
                op.inv_s2 * o[k] + op.lambda * sm.p[(r + k + 2 * RS) * PS + c + 2 * RS];
            float& rv = sm.r[(r + k + 2 * RS) * RSS + c + 2 * RS + RO];
            rv = rv - alpha * sv;
        }
    }
}

// B^T's row pass over the S rows at the tile's columns (the PSF's row factor, correlation
// form), into h with stride T32: four outputs per item from three 16-byte LDS reads.
template <int RS, int NT>
__device__ inline void cg32_b_rows(const LinOp& op, Cg32Smem<RS>& sm) {
    using M = Cg32Smem<RS>;
    constexpr int SR = M::SR, RSS = M::RSS, RO = M::RO, KB = 2 * RS + 1;
    constexpr int NWIN = (KB + 3 + 3) / 4 * 4;
    static_assert(T32 - 4 + NWIN <= SR, "the window stays in the S row");
    static_assert((2 * RS + RO) % 4 == 0 && RSS % 4 == 0, "16-byte aligned S rows");
#pragma unroll 1
    for (int e = threadIdx.x; e < SR * (T32 / 4); e += NT) {
        const int r = e / (T32 / 4), c = (e % (T32 / 4)) * 4;
        const float4* x4 =
            reinterpret_cast<const float4*>(sm.r + (r + 2 * RS) * RSS + c + 2 * RS + RO);
        float x[NWIN];
#pragma unroll
        for (int i = 0; i < NWIN / 4; ++i) {
            const float4 v = x4[i];
            x[4 * i] = v.x;
            x[4 * i + 1] = v.y;
            x[4 * i + 2] = v.z;
            x[4 * i + 3] = v.w;
        }
        float o0 = 0.f, o1 = 0.f, o2 = 0.f, o3 = 0.f;
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            o0 += op.row[j] * x[j];
            o1 += op.row[j] * x[j + 1];
            o2 += op.row[j] * x[j + 2];
            o3 += op.row[j] * x[j + 3];
        }
        *reinterpret_cast<float4*>(sm.h + r * T32 + c) = make_float4(o0, o1, o2, o3);
    }
}

// The per-tile steps, shared by the single-image kernel (a loop over tiles) and the batched
// one (one tile per workgroup).
template <int RS>
struct Cg32Geo {
    using M = Cg32Smem<RS>;
    static constexpr int NT = kCg32Threads, PR = M::PR, SR = M::SR, PS = M::PS, RSS = M::RSS;
    static constexpr int LR = M::LR, NL = M::NL, RO = M::RO;
    static constexpr int NOUT = T32 * T32 / NT;  // tile pixels per thread
};

// r_k and p_{k-1} of the tile at (r0, c0) on its P region into the loader's registers (p only
// for k > 0). Straight-line loads: the rows past the region repeat its last row. Indexes wrap
// periodically.
template <int RS>
__device__ inline void cg32_fetch(int H, int W, int r0, int c0, int k, const float* r_in,
                                  const float* p_in, float (&fr)[Cg32Geo<RS>::NL],
                                  float (&fp)[Cg32Geo<RS>::NL]) {
    using G = Cg32Geo<RS>;
    constexpr int PR = G::PR, LR = G::LR, NL = G::NL;
    const int lcol = threadIdx.x % PR, lrow = threadIdx.x / PR;
    if (lrow >= LR) return;
    const int pr0 = r0 - 3 * RS, pc0 = c0 - 3 * RS;
    size_t g[NL];
    if (pr0 >= 0 && pc0 >= 0 && pr0 + PR <= H && pc0 + PR <= W) {
        // the region lies inside the image (every tile but those at the border)
        const size_t base = (size_t)(pr0 + lrow) * W + pc0 + lcol;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int dr = i == NL - 1 ? min(LR * i, PR - 1 - lrow) : LR * i;
            g[i] = base + (size_t)dr * W;
        }
    } else {
        const size_t gc = wrapi(pc0 + lcol, W);
#pragma unroll
        for (int i = 0; i < NL; ++i)
            g[i] = (size_t)wrapi(pr0 + min(lrow + LR * i, PR - 1), H) * W + gc;
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) fr[i] = r_in[g[i]];
    if (k) {
#pragma unroll
        for (int i = 0; i < NL; ++i) fp[i] = p_in[g[i]];
    }
}

// p_k = r_k + beta p_{k-1} and r_k into the P region (from the loader's registers); the caller
// synchronizes.
template <int RS>
__device__ inline void cg32_stage(int k, float beta, const float (&fr)[Cg32Geo<RS>::NL],
                                  const float (&fp)[Cg32Geo<RS>::NL], Cg32Smem<RS>& sm) {
    using G = Cg32Geo<RS>;
    constexpr int PR = G::PR, PS = G::PS, RSS = G::RSS, RO = G::RO, LR = G::LR, NL = G::NL;
    const int lcol = threadIdx.x % PR, lrow = threadIdx.x / PR;
    if (lrow >= LR) return;
    float* pp = sm.p + lrow * PS + lcol;
    float* rr = sm.r + lrow * RSS + lcol + RO;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        pp[LR * i * PS] = k ? fr[i] + beta * fp[i] : fr[i];
        rr[LR * i * RSS] = fr[i];
    }
}

// d_k at the thread's pixels of the tile (0 for k = 0 and outside the image).
template <int RS>
__device__ inline void cg32_load_d(int H, int W, int r0, int c0, int k, const float* d,
                                   float (&dk)[Cg32Geo<RS>::NOUT]) {
#pragma unroll
    for (int o = 0; o < Cg32Geo<RS>::NOUT; ++o) {
        const int idx = threadIdx.x + o * kCg32Threads, gr = r0 + idx / T32, gc = c0 + idx % T32;
        dk[o] = k && gr < H && gc < W ? d[(size_t)gr * W + gc] : 0.f;
    }
}

// With p_k and r_k staged: r_{k+1} = r_k - alpha A p_k on the S region, q = B^T r_{k+1} at the
// tile, then the stores of r_{k+1}, p_k, d_{k+1} and the sums r.r and q.q. Leaves the
// workgroup synchronized (LDS free for the next tile).
template <int RS>
__device__ inline void cg32_finish(const LinOp& op, int H, int W, int r0, int c0, int k,
                                   float alpha, Cg32Smem<RS>& sm,
                                   const float (&dk)[Cg32Geo<RS>::NOUT], float* r_out,
                                   float* p_out, float* d, double (&acc)[2]) {
    using G = Cg32Geo<RS>;
    constexpr int NT = G::NT, PS = G::PS, RSS = G::RSS, RO = G::RO, KB = 2 * RS + 1;
    cg32_a_rows<RS, NT>(op, sm);
    __syncthreads();
    cg32_update_r<RS, NT>(op, sm, alpha);  // r_{k+1} on the S region
    __syncthreads();
    cg32_b_rows<RS, NT>(op, sm);
    __syncthreads();
#pragma unroll
    for (int o = 0; o < G::NOUT; ++o) {
        const int idx = threadIdx.x + o * NT, tr = idx / T32, tc = idx % T32;
        const int gr = r0 + tr, gc = c0 + tc;
        float q = 0.f;  // B^T r_{k+1}: the column pass at this pixel
#pragma unroll
        for (int i = 0; i < KB; ++i) q += op.col[i] * sm.h[(tr + i) * T32 + tc];
        if (gr < H && gc < W) {
            const size_t g = (size_t)gr * W + gc;
            const float rv = sm.r[(tr + 3 * RS) * RSS + tc + 3 * RS + RO];
            const float pv = sm.p[(tr + 3 * RS) * PS + tc + 3 * RS];
            r_out[g] = rv;
            p_out[g] = pv;
            d[g] = k ? dk[o] + alpha * pv : alpha * pv;
            acc[0] += (double)rv * (double)rv;
            acc[1] += (double)q * (double)q;
        }
    }
    __syncthreads();
}

template <int RS>
__global__ __launch_bounds__(kCg32Threads) void k_cg_iter32(
    const LinOp op, int H, int W, int k, const float* __restrict__ r_in,
    const float* __restrict__ p_in, float* __restrict__ r_out, float* __restrict__ p_out,
    float* __restrict__ d, Partials rm, const double* __restrict__ hist_prev,
    double* __restrict__ hist_cur, double* __restrict__ part) {
    using G = Cg32Geo<RS>;
    constexpr int NT = G::NT;
    __shared__ Cg32Smem<RS> sm;
    __shared__ double sred[2 * NT / 64];
    __shared__ double bc[2];
    const int ntx = (W + T32 - 1) / T32, nt = ntx * ((H + T32 - 1) / T32);
    // the published partials and the previous step lengths first
    Early2 early;
    const bool early_ok = rm.n <= kEarlyPartials;
    if (early_ok) consume2_issue(rm.p, kMaxRedBlocks, rm.n, early);
    const double alpha_prev = k ? hist_prev[0] : 0.0, rho_prev = k ? hist_prev[1] : 0.0;
    float fr[G::NL], fp[G::NL];
    int r0 = 0, c0 = 0;
    auto origin = [&](int t) {
        const int tt = xcd_tile(t, nt);
        r0 = (tt / ntx) * T32;
        c0 = (tt % ntx) * T32;
    };
    double rho, mu;
    if (early_ok)
        consume2_finish(early, bc, rho, mu);
    else
        consume2(rm.p, kMaxRedBlocks, rm.n, bc, rho, mu);
    double alpha_d, beta_d;
    cg_scalars(k, rho, mu, alpha_prev, rho_prev, alpha_d, beta_d);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hist_cur[0] = alpha_d;
        hist_cur[1] = rho;
    }
    const float alpha = (float)alpha_d, beta = (float)beta_d;
    double acc[2] = {0.0, 0.0};  // r.r, (B^T r).(B^T r)
    // one tile at a time: three workgroups per CU overlap one another's loads and passes (a
    // prefetch of the next tile into registers cost the registers of the third workgroup)
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        origin(t);
        float dk[G::NOUT];
        cg32_load_d<RS>(H, W, r0, c0, k, d, dk);
        cg32_fetch<RS>(H, W, r0, c0, k, r_in, p_in, fr, fp);
        cg32_stage<RS>(k, beta, fr, fp, sm);
        __syncthreads();
        cg32_finish<RS>(op, H, W, r0, c0, k, alpha, sm, dk, r_out, p_out, d, acc);
    }
    block_sum<2, NT>(acc, sred);
    // mu's partial: ||B^T r||^2 / sigma^2 + lambda ||r||^2 over this workgroup's pixels
    acc[1] = op.inv_s2_d * acc[1] + op.lambda_d * acc[0];
    publish<2>(acc, part, kMaxRedBlocks, blockIdx.x);
}

// Batched form: one workgroup per entry of the 32x32 tile list (image, tile t of ceil(W/32)
// per row); images whose 32x32 tiles are in the list have cg32 set. The tile's sums go to
// partial index tile0 + t of its image (one per 32x32 tile), summed by k_cg_fin_batch.
template <int RS>
__global__ __launch_bounds__(kCg32Threads) void k_cg_iter32_batch(
    const ImgDesc* __restrict__ desc, const TileRef* __restrict__ tiles, int k,
    const CgImg* __restrict__ cg, const float* __restrict__ r_in, const float* __restrict__ p_in,
    float* __restrict__ r_out, float* __restrict__ p_out, float* __restrict__ dd,
    double* __restrict__ part, int cap) {
    using G = Cg32Geo<RS>;
    __shared__ Cg32Smem<RS> sm;
    __shared__ double sred[2 * G::NT / 64];
    const TileRef e = tiles[blockIdx.x];
    const ImgDesc* d = desc + e.img;
    if (!d->active || !d->cg32) return;
    const int H = d->H, W = d->W, ntx = (W + T32 - 1) / T32;
    const int r0 = (e.t / ntx) * T32, c0 = (e.t % ntx) * T32;
    const size_t o = d->off;
    float fr[G::NL], fp[G::NL], dk[G::NOUT];
    cg32_load_d<RS>(H, W, r0, c0, k, dd + o, dk);
    cg32_fetch<RS>(H, W, r0, c0, k, r_in + o, p_in + o, fr, fp);
    const CgImg c = cg[e.img];
    cg32_stage<RS>(k, (float)c.beta, fr, fp, sm);
    __syncthreads();
    double acc[2] = {0.0, 0.0};
    cg32_finish<RS>(d->op, H, W, r0, c0, k, (float)c.alpha, sm, dk, r_out + o, p_out + o,
                    dd + o, acc);
    block_sum<2, G::NT>(acc, sred);
    acc[1] = d->op.inv_s2_d * acc[1] + d->op.lambda_d * acc[0];
    publish<2>(acc, part, cap, d->tile0 + e.t);
}

// The last CG iteration of an FP call and the difference pass of vector extrapolation
// (Algorithm 1, step 1) in one pass over the pixels: x_out = x_in + d_k + alpha_k p_k, then
// u = x_out - x_in, stored as column NC of U (U null: not stored), its inner products with the
// NC earlier columns, ||u||^2 and ||x_in||^2, published as per-workgroup FP64 partials. Each
// pixel's arithmetic, the pixel order and the sums are those of the two separate passes (the
// last iteration, then k_diff_gram on the same grid), so the results are bitwise theirs.
template <int NC>
__global__ __launch_bounds__(kThreads) void k_cg_last_diff(
    int n, int k, const float* __restrict__ r_in, const float* __restrict__ p,
    const float* __restrict__ d, const float* __restrict__ x_in, float* __restrict__ x_out,
    Partials rm, const double* __restrict__ hist_prev, float* __restrict__ U,
    double* __restrict__ part) {
    constexpr int NV = NC + 2;
    __shared__ double sred[NV * kThreads / 64];
    __shared__ double bc[2];
    Early2 early;
    const bool early_ok = rm.n <= kEarlyPartials;
    if (early_ok) consume2_issue(rm.p, kMaxRedBlocks, rm.n, early);
    const double alpha_prev = k ? hist_prev[0] : 0.0, rho_prev = k ? hist_prev[1] : 0.0;
    double rho, mu;
    if (early_ok)
        consume2_finish(early, bc, rho, mu);
    else
        consume2(rm.p, kMaxRedBlocks, rm.n, bc, rho, mu);
    double alpha_d, beta_d;
    cg_scalars(k, rho, mu, alpha_prev, rho_prev, alpha_d, beta_d);
    const float alpha = (float)alpha_d, beta = (float)beta_d;
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    const int stride = gridDim.x * kThreads;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const float pk = k ? r_in[i] + beta * p[i] : r_in[i];
        const float dn = k ? d[i] + alpha * pk : alpha * pk;
        const float xo = x_in[i];
        const float xn = xo + dn;
        x_out[i] = xn;
        const float uv = xn - xo;
        if (U) U[(size_t)NC * n + i] = uv;
#pragma unroll
        for (int j = 0; j < NC; ++j) acc[j] += (double)uv * (double)U[(size_t)j * n + i];
        acc[NC] += (double)uv * (double)uv;
        acc[NC + 1] += (double)xo * (double)xo;
    }
    block_sum<NV>(acc, sred);
    publish<NV>(acc, part, kMaxRedBlocks, blockIdx.x);
}

// ---- the RED objective E(x) = ||Hx - y||^2 / (2 sigma^2) + (lambda/2) x^T (x - f(x)), eq. (4)

// Per-workgroup FP64 partials of ||Hx - y||^2 (over the decimated grid; H x summed in FP64 from
// the FP32 image) and of x.s (s = f(x) - x; null: the identity denoiser).
__global__ __launch_bounds__(kThreads) void k_objective(const LinOp op, const float* __restrict__ x,
                                                        const float* __restrict__ y,
                                                        const float* __restrict__ s, int H,
                                                        int W, double* __restrict__ part) {
    __shared__ double sred[2 * kThreads / 64];
    const int dec = op.decim, h = (H + dec - 1) / dec, w = (W + dec - 1) / dec;
    const int rh = op.kh / 2, rw = op.kw / 2;
    const int n = max(h * w, H * W), stride = gridDim.x * kThreads;
    double acc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        if (i < h * w) {
            const int ii = i / w, jj = i % w;
            double hx = 0.0;
            for (int a = -rh; a <= rh; ++a) {
                const float* row = x + (size_t)wrapi(dec * ii - a, H) * W;
                for (int b = -rw; b <= rw; ++b)
                    hx += op.psf64[(a + rh) * op.kw + b + rw] * (double)row[wrapi(dec * jj - b, W)];
            }
            const double rr = hx - (double)y[i];
            acc[0] += rr * rr;
        }
        if (s && i < H * W) acc[1] += (double)x[i] * (double)s[i];
    }
    block_sum<2>(acc, sred);
    publish<2>(acc, part, kMaxRedBlocks, blockIdx.x);
}

__global__ __launch_bounds__(64) void k_objective_fin(const double* __restrict__ part, int nblk,
                                                      double* __restrict__ out) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 64) {
        s0 += part[i];
        s1 += part[kMaxRedBlocks + i];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
    }
}

// ---- batched kernels: one workgroup per tile of the batch tile list ----------------------

// This workgroup's list entry: its image, the tile's origin, and bt, the index its per-tile
// partials are published at; null for an inactive image.
__device__ inline const ImgDesc* batch_tile(const ImgDesc* desc, const TileRef* tiles, int& bt,
                                            int& r0, int& c0) {
    const TileRef e = tiles[blockIdx.x];
    const ImgDesc* d = desc + e.img;
    if (!d->active) return nullptr;
    const int t = e.t, ntx = (d->W + TW - 1) / TW;
    bt = d->tile0 + t;
    r0 = (t / ntx) * TH;
    c0 = (t % ntx) * TW;
    return d;
}

template <int RS>
__global__ __launch_bounds__(kThreads) void k_cg_init_fp_batch(const ImgDesc* __restrict__ desc,
                                                               const TileRef* __restrict__ tiles,
                                                               const float* __restrict__ sres,
                                                               float* __restrict__ r, int sd) {
    __shared__ InitFpSmem<RS> sm;
    int bt, r0, c0;
    const ImgDesc* d = batch_tile(desc, tiles, bt, r0, c0);
    if (!d) return;
    if constexpr (RS > 0)  // every operator of the batch is padded to this radius
        init_fp_tile_rs<RS>(d->op, d->x_in, d->y, sres ? sres + d->off : nullptr,
                            sd ? nullptr : r + d->off, d->H, d->W, r0, c0, sm,
                            sd ? d->x_out : nullptr);
    else
        init_fp_tile<RS>(d->op, d->x_in, d->y, sres ? sres + d->off : nullptr,
                         sd ? nullptr : r + d->off, d->H, d->W, r0, c0, sm,
                         sd ? d->x_out : nullptr);
}

template <int RS>
__global__ __launch_bounds__(kThreads) void k_cg_w0_batch(const ImgDesc* __restrict__ desc,
                                                          const TileRef* __restrict__ tiles,
                                                          const float* __restrict__ r,
                                                          float* __restrict__ w,
                                                          double* __restrict__ part, int cap) {
    __shared__ TileSmem<RS> sm;
    __shared__ double sred[2 * kThreads / 64];
    int bt, r0, c0;
    const ImgDesc* d = batch_tile(desc, tiles, bt, r0, c0);
    if (!d) return;
    double acc[2] = {0.0, 0.0};
    w0_tile<RS>(d->op, r + d->off, w + d->off, d->H, d->W, r0, c0, sm, acc);
    block_sum<2>(acc, sred);
    publish<2>(acc, part, cap, bt);
}

// Per-image CG scalars: sums the image's tile partials (rho on threads 0..255, mu on 256..511;
// each thread four independent chains, so the loads of a chain overlap; the summation order
// depends only on the image's tile count, hence on nothing else in the batch), then alpha_k,
// beta_k.
__global__ __launch_bounds__(512) void k_cg_fin_batch(const ImgDesc* __restrict__ desc, int k,
                                                      const double* __restrict__ part, int cap,
                                                      CgImg* __restrict__ cg) {
    __shared__ double sums[8];
    const ImgDesc& d = desc[blockIdx.x];
    if (!d.active) return;
    const int v = threadIdx.x >> 8, tid = threadIdx.x & 255;
    const double* pv = part + (size_t)v * cap + d.tile0;
    // partials of the previous kernel: one per 16x16 tile, or per 32x32 tile after an
    // iteration of the 32x32 form (every iteration but the first: k_cg_w0_batch runs on 16x16)
    const int n = d.cg32 && k > 0 ? ((d.H + T32 - 1) / T32) * ((d.W + T32 - 1) / T32) : d.ntiles;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = tid;
    for (; i + 768 < n; i += 1024) {
        a0 += pv[i];
        a1 += pv[i + 256];
        a2 += pv[i + 512];
        a3 += pv[i + 768];
    }
    for (; i < n; i += 256) a0 += pv[i];
    const double s = wave_sum((a0 + a1) + (a2 + a3));
    if ((threadIdx.x & 63) == 0) sums[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double rho = (sums[0] + sums[1]) + (sums[2] + sums[3]);
        const double mu = (sums[4] + sums[5]) + (sums[6] + sums[7]);
        CgImg c = cg[blockIdx.x];
        double alpha, beta;
        cg_scalars(k, rho, mu, c.alpha_prev, c.rho_prev, alpha, beta);
        c.alpha = alpha;
        c.beta = beta;
        c.alpha_prev = alpha;
        c.rho_prev = rho;
        cg[blockIdx.x] = c;
    }
}

template <int RS>
__global__ __launch_bounds__(kThreads) void k_cg_iter_batch(
    const ImgDesc* __restrict__ desc, const TileRef* __restrict__ tiles, int k, int last,
    const CgImg* __restrict__ cg, const float* __restrict__ r_in, const float* __restrict__ w_in,
    const float* __restrict__ s_in, float* __restrict__ r_out, float* __restrict__ w_out,
    float* __restrict__ s_out, float* __restrict__ p, float* __restrict__ dd,
    double* __restrict__ part, int cap) {
    __shared__ TileSmem<RS> sm;
    __shared__ double sred[2 * kThreads / 64];
    int bt, r0, c0;
    const ImgDesc* d = batch_tile(desc, tiles, bt, r0, c0);
    if (!d) return;
    const size_t o = d->off;
    if (last) {
        // p_{k-1}: the 32x32 form keeps it double-buffered in the s arrays (this call's s_out)
        const CgImg c = cg[d - desc];
        cg_last_tile(d->H, d->W, r0, c0, k, (float)c.alpha, (float)c.beta, r_in + o,
                     (d->cg32 ? s_out : p) + o, dd + o, d->x_in, d->x_out);
        return;
    }
    if (d->cg32) return;  // the 32x32 tile list takes this image's iteration
    double acc[2] = {0.0, 0.0};
    if constexpr (RS > 0) {
        // the workgroup sum first, then every store of the tile at once
        const CgImg c = cg[d - desc];
        CgIn<RS> f;
        cg_fetch<RS>(d->H, d->W, r0, c0, k, r_in + o, w_in + o, s_in + o, p + o, dd + o, f);
        const CgOut out = cg_iter_compute<RS>(d->op, d->H, d->W, r0, c0, k, (float)c.alpha,
                                              (float)c.beta, f, sm, acc);
        block_sum<2>(acc, sred);
        cg_store(out, r_out + o, w_out + o, s_out + o, p + o, dd + o);
        publish<2>(acc, part, cap, bt);
        return;
    } else {
        const CgImg c = cg[d - desc];
        cg_iter_tile<RS>(d->op, d->H, d->W, r0, c0, k, (float)c.alpha, (float)c.beta, r_in + o,
                         w_in + o, s_in + o, r_out + o, w_out + o, s_out + o, p + o, dd + o, sm,
                         acc);
    }
    block_sum<2>(acc, sred);
    publish<2>(acc, part, cap, bt);
}

// ---- two CG iterations per kernel (undecimated, separable square PSF) --------------------
//
// The single-reduction iteration above needs one grid-wide sum per iteration. Two iterations
// k, k+1 need only the sums available at k if the kernel also carries a = A w and b = A s:
// with V = [r_k, w_k, s_{k-1}, a_k, b_{k-1}] (w = A r, s = A p, a = A w, b = A s) and G its
// Gram matrix,
//   s_k = w + beta_{k-1} s,  A s_k = a + beta_{k-1} b,
//   r_{k+1} = r - alpha_k s_k,  w_{k+1} = w - alpha_k A s_k        (linear in V)
//   rho_{k+1} = r_{k+1}.r_{k+1},  mu_{k+1} = w_{k+1}.r_{k+1}      (quadratic forms in G)
// give alpha_{k+1} and beta_k without a second sum, then
//   s_{k+1} = w_{k+1} + beta_k s_k,  r_{k+2} = r_{k+1} - alpha_{k+1} s_{k+1}   (linear in V)
//   p_k = r_k + beta_{k-1} p_{k-1},  p_{k+1} = r_{k+1} + beta_k p_k,
//   d_{k+2} = d_k + alpha_k p_k + alpha_{k+1} p_{k+1},
// and the stencils w_{k+2} = A r_{k+2}, a_{k+2} = A w_{k+2}, b_{k+1} = A s_{k+1} complete the
// next V, whose Gram sums are the kernel's only reduction. rho_{k+1} and mu_{k+1} use nine of
// them, with r.a = w.w, r.b = w.s and w.b = a.s (A symmetric): r.r, w.r, w.w, s.r, s.w, s.s,
// a.w, a.s, b.s, stored in that order (entry 0 is rho = r.r, entry 1 mu = w.r, so the
// single-iteration kernel can follow a block). In exact arithmetic the iterates are those of
// CG; with FP32 vectors and FP64 sums the rounding is of the same size. A is applied in the
// autocorrelation form (a row pass and a column pass of 4 RS + 1 taps), so r_{k+2} is formed
// on the tile plus a 4 RS halo, and s_{k+1}, w_{k+2} on a 2 RS halo.
constexpr int kGram = 9;
enum GramEntry { G_RR, G_WR, G_WW, G_SR, G_SW, G_SS, G_AW, G_AS, G_BS };

template <int RS>
struct __align__(16) BlkSmem {
    static constexpr int RH = TH + 8 * RS, RW = TW + 8 * RS;  // r_{k+2} region
    static constexpr int QH = TH + 4 * RS, QW = TW + 4 * RS;  // s_{k+1}, w_{k+2} regions
    float R[RH * RW];
    float hR[RH * QW];
    float Wn[QH * QW];
    float S[QH * QW];
    float hS[QH * TW];
    float hw[QH * TW];
    float Bn[TH * TW];
    float An[TH * TW];
    float T0[TH * TW];  // r_k at the tile's pixels
    float T1[TH * TW];  // r_{k+1} there
    // the Gram sums' per-thread values once the tile loop is done (the regions are free then)
    __device__ double* sums() { return reinterpret_cast<double*>(this); }
};
static_assert(sizeof(BlkSmem<3>) >= sizeof(double) * kGram * TH * TW,
              "the Gram sums' values fit the regions");

// The published Gram sums: wave v < kGram sums array v, in partial order (as consume2). For at most
// kEarlyPartials partials the loads are issued first (gram_issue, before the tile's loads) and
// summed later (gram_finish); beyond that gram_finish loads them itself.
struct GramEarly {
    double a[4];
};

template <int NTH>
__device__ inline void gram_issue(const double* part, int n, GramEarly& q) {
    static_assert(NTH / 64 >= kGram, "one wave per Gram entry");
    const int v = threadIdx.x >> 6;
    if (v < kGram && n <= kEarlyPartials) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = (threadIdx.x & 63) + 64 * i;
            q.a[i] = j < n ? part[(size_t)v * kMaxRedBlocks + j] : 0.0;
        }
    }
}

template <int NTH>
__device__ inline void gram_finish(const double* part, int n, const GramEarly& q,
                                   double* bc /* kGram */) {
    const int v = threadIdx.x >> 6;
    if (v < kGram) {
        double s = 0.0;
        if (n <= kEarlyPartials) {
#pragma unroll
            for (int i = 0; i < 4; ++i) s += q.a[i];
        } else {
            for (int i = threadIdx.x & 63; i < n; i += 64) s += part[(size_t)v * kMaxRedBlocks + i];
        }
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) bc[v] = s;
    }
    __syncthreads();
}

// Scalars of the two iterations from G, and the coefficient rows over V of r_{k+1}, s_{k+1},
// r_{k+2}.
struct BlkScalars {
    double a0, b1, a1, b2, rho1;
    float cr1[5], cs1[5], cr2[5];
};

__device__ inline BlkScalars blk_scalars(int k, const double* G, double alpha_prev,
                                         double rho_prev) {
    BlkScalars q;
    cg_scalars(k, G[0], G[1], alpha_prev, rho_prev, q.a0, q.b1);
    // r_{k+1} = r - x w - y s, w_{k+1} = w - x a - y b with x = alpha_k, y = alpha_k beta_{k-1}
    const double x = q.a0, y = q.a0 * q.b1;
    const double rho1 = (G[G_RR] - 2.0 * (x * G[G_WR] + y * G[G_SR])) +
                        (x * x * G[G_WW] + 2.0 * x * y * G[G_SW] + y * y * G[G_SS]);
    const double mu1 = (G[G_WR] - x * G[G_WW] - y * G[G_SW]) -
                       x * (G[G_WW] - x * G[G_AW] - y * G[G_AS]) -
                       y * (G[G_SW] - x * G[G_AS] - y * G[G_BS]);
    const double c1[5] = {1.0, -x, -y, 0.0, 0.0};
    q.rho1 = rho1;
    cg_scalars(k + 1, rho1, mu1, q.a0, G[0], q.a1, q.b2);
    const double cs[5] = {0.0, 1.0 + q.b2, q.b2 * q.b1, -q.a0, -q.a0 * q.b1};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        q.cr1[i] = (float)c1[i];
        q.cs1[i] = (float)cs[i];
        q.cr2[i] = (float)(c1[i] - q.a1 * cs[i]);
    }
    return q;
}

// V on the r_{k+2} region of one tile (NE positions per thread), and p, d at the pixel (V
// there is part of the region).
template <int RS, int NTH>
struct BlkIn {
    static constexpr int RH = TH + 8 * RS, RW = TW + 8 * RS;
    static constexpr int NE = (RH * RW + NTH - 1) / NTH;
    float v[NE][5];
    float po, dn;
};

template <int RS, int NTH>
__device__ inline void blk_fetch(int H, int W, int r0, int c0, int k, const float* const* vin,
                                 const float* __restrict__ p, const float* __restrict__ d,
                                 BlkIn<RS, NTH>& f) {
    using C = BlkIn<RS, NTH>;
    const int nv = k ? 5 : 4;  // s_{-1} = b_{-1} = 0: the loads of s and b are skipped at k = 0
#pragma unroll
    for (int i = 0; i < C::NE; ++i) {
        const int e = threadIdx.x + i * NTH;
#pragma unroll
        for (int j = 0; j < 5; ++j) f.v[i][j] = 0.f;
        if (e < C::RH * C::RW) {
            const size_t g = (size_t)wrapi(r0 - 4 * RS + e / C::RW, H) * W +
                             wrapi(c0 - 4 * RS + e % C::RW, W);
#pragma unroll
            for (int j = 0; j < 5; ++j)
                if (j != 2 && j != 4 ? true : nv == 5) f.v[i][j] = vin[j][g];
        }
    }
    f.po = f.dn = 0.f;
    const int gr = r0 + threadIdx.x / TW, gc = c0 + threadIdx.x % TW;
    if (k && (int)threadIdx.x < TH * TW && gr < H && gc < W) {
        const size_t g = (size_t)gr * W + gc;
        f.po = p[g];
        f.dn = d[g];
    }
}

// Two CG iterations k, k + 1 on one tile (see above); accumulates the Gram matrix of the next
// V at the tile's pixels.
template <int RS, int NTH>
__device__ inline void blk_tile(const LinOp& op, int H, int W, int r0, int c0,
                                const BlkScalars& q, const BlkIn<RS, NTH>& f,
                                float* const* vout, float* __restrict__ p, float* __restrict__ d,
                                BlkSmem<RS>& sm, double (&g)[kGram]) {
    using M = BlkSmem<RS>;
    using C = BlkIn<RS, NTH>;
    // r_{k+2} on the whole region, s_{k+1} on its inner 2 RS halo, r_k and r_{k+1} at the
    // tile's pixels (the region covers them)
#pragma unroll
    for (int i = 0; i < C::NE; ++i) {
        const int e = threadIdx.x + i * NTH;
        if (e < M::RH * M::RW) {
            const int rr = e / M::RW, rc = e % M::RW;
            float rv = 0.f, sv = 0.f;
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                rv += q.cr2[j] * f.v[i][j];
                sv += q.cs1[j] * f.v[i][j];
            }
            sm.R[e] = rv;
            const int qr = rr - 2 * RS, qc = rc - 2 * RS;
            if (qr >= 0 && qr < M::QH && qc >= 0 && qc < M::QW) sm.S[qr * M::QW + qc] = sv;
            const int tr = rr - 4 * RS, tc = rc - 4 * RS;
            if (tr >= 0 && tr < TH && tc >= 0 && tc < TW) {
                float r1 = 0.f;
#pragma unroll
                for (int j = 0; j < 5; ++j) r1 += q.cr1[j] * f.v[i][j];
                sm.T0[tr * TW + tc] = f.v[i][0];
                sm.T1[tr * TW + tc] = r1;
            }
        }
    }
    __syncthreads();
    ac_rows<RS, NTH>(op, sm.R, M::RW, M::RH, M::QW, sm.hR);
    ac_rows<RS, NTH>(op, sm.S, M::QW, M::QH, TW, sm.hS);
    __syncthreads();
    ac_cols<RS, NTH>(op, sm.hR, sm.R, M::RW, M::QH, M::QW, sm.Wn);  // w_{k+2} = A r_{k+2}
    ac_cols<RS, NTH>(op, sm.hS, sm.S, M::QW, TH, TW, sm.Bn);        // b_{k+1} = A s_{k+1}
    __syncthreads();
    ac_rows<RS, NTH>(op, sm.Wn, M::QW, M::QH, TW, sm.hw);
    __syncthreads();
    ac_cols<RS, NTH>(op, sm.hw, sm.Wn, M::QW, TH, TW, sm.An);  // a_{k+2} = A w_{k+2}
    __syncthreads();
    const int tr = threadIdx.x / TW, tc = threadIdx.x % TW;
    const int gr = r0 + tr, gc = c0 + tc;
    if ((int)threadIdx.x < TH * TW && gr < H && gc < W) {
        const size_t gi = (size_t)gr * W + gc;
        const float r1 = sm.T1[tr * TW + tc];
        const float pk = sm.T0[tr * TW + tc] + (float)q.b1 * f.po;
        const float pk1 = r1 + (float)q.b2 * pk;
        const float dn = f.dn + (float)q.a0 * pk + (float)q.a1 * pk1;
        const float v[5] = {sm.R[(tr + 4 * RS) * M::RW + tc + 4 * RS],
                            sm.Wn[(tr + 2 * RS) * M::QW + tc + 2 * RS],
                            sm.S[(tr + 2 * RS) * M::QW + tc + 2 * RS], sm.An[tr * TW + tc],
                            sm.Bn[tr * TW + tc]};
#pragma unroll
        for (int i = 0; i < 5; ++i) vout[i][gi] = v[i];
        const double dr = v[0], dw = v[1], ds = v[2], da = v[3], db = v[4];
        g[G_RR] += dr * dr;
        g[G_WR] += dw * dr;
        g[G_WW] += dw * dw;
        g[G_SR] += ds * dr;
        g[G_SW] += ds * dw;
        g[G_SS] += ds * ds;
        g[G_AW] += da * dw;
        g[G_AS] += da * ds;
        g[G_BS] += db * ds;
        p[gi] = pk1;
        d[gi] = dn;
    }
    __syncthreads();
}

// Pointers of V = [r, w, s, a, b] (kernel argument).
struct VecSet {
    const float* in[5];
    float* out[5];
};

template <int RS>
__global__ __launch_bounds__(kWideThreadsBlk) void k_cg_block(
    const LinOp op, int H, int W, int k, VecSet vs, float* __restrict__ p, float* __restrict__ d,
    Partials rm, const double* __restrict__ hist_prev, double* __restrict__ hist_cur,
    double* __restrict__ part) {
    constexpr int NTH = kWideThreadsBlk;
    __shared__ BlkSmem<RS> sm;
    __shared__ double bc[kGram];
    const int nt = ntiles(H, W);
    GramEarly early;
    gram_issue<NTH>(rm.p, rm.n, early);
    const double alpha_prev = k ? hist_prev[0] : 0.0, rho_prev = k ? hist_prev[1] : 0.0;
    int r0 = 0, c0 = 0;
    BlkIn<RS, NTH> f;
    if ((int)blockIdx.x < nt) {
        tile_origin(xcd_tile(blockIdx.x, nt), W, r0, c0);
        blk_fetch<RS, NTH>(H, W, r0, c0, k, vs.in, p, d, f);
    }
    gram_finish<NTH>(rm.p, rm.n, early, bc);
    const BlkScalars q = blk_scalars(k, bc, alpha_prev, rho_prev);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hist_cur[0] = q.a1;
        hist_cur[1] = q.rho1;
    }
    double g[kGram];
#pragma unroll
    for (int i = 0; i < kGram; ++i) g[i] = 0.0;
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        tile_origin(xcd_tile(t, nt), W, r0, c0);
        if (t != (int)blockIdx.x) blk_fetch<RS, NTH>(H, W, r0, c0, k, vs.in, p, d, f);
        blk_tile<RS, NTH>(op, H, W, r0, c0, q, f, vs.out, p, d, sm, g);
    }
    block_sum_publish<kGram, NTH, TH * TW>(g, sm.sums(), part, kMaxRedBlocks, blockIdx.x);
}

// Block start at k = 0: from r_0, w_0 = A r_0 and a_0 = A w_0 on the tile and the Gram sums
// of V_0 = [r_0, w_0, 0, a_0, 0] (s_{-1} = b_{-1} = 0).
template <int RS>
__global__ __launch_bounds__(kWideThreadsBlk) void k_cg_w0_block(
    const LinOp op, int H, int W, const float* __restrict__ r, float* __restrict__ w,
    float* __restrict__ a, double* __restrict__ part) {
    constexpr int NTH = kWideThreadsBlk;
    using M = BlkSmem<RS>;
    __shared__ BlkSmem<RS> sm;
    const int nt = ntiles(H, W);
    double g[kGram];
#pragma unroll
    for (int i = 0; i < kGram; ++i) g[i] = 0.0;
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        int r0, c0;
        tile_origin(xcd_tile(t, nt), W, r0, c0);
        // w_0 = A r_0 is needed on the tile plus 2 RS (for a_0): r_0 on 4 RS
        for (int e = threadIdx.x; e < M::RH * M::RW; e += NTH)
            sm.R[e] = r[(size_t)wrapi(r0 - 4 * RS + e / M::RW, H) * W +
                        wrapi(c0 - 4 * RS + e % M::RW, W)];
        __syncthreads();
        ac_rows<RS, NTH>(op, sm.R, M::RW, M::RH, M::QW, sm.hR);
        __syncthreads();
        ac_cols<RS, NTH>(op, sm.hR, sm.R, M::RW, M::QH, M::QW, sm.Wn);
        __syncthreads();
        ac_rows<RS, NTH>(op, sm.Wn, M::QW, M::QH, TW, sm.hw);
        __syncthreads();
        ac_cols<RS, NTH>(op, sm.hw, sm.Wn, M::QW, TH, TW, sm.An);
        __syncthreads();
        const int tr = threadIdx.x / TW, tc = threadIdx.x % TW;
        const int gr = r0 + tr, gc = c0 + tc;
        if ((int)threadIdx.x < TH * TW && gr < H && gc < W) {
            const size_t gi = (size_t)gr * W + gc;
            const float rv = sm.R[(tr + 4 * RS) * M::RW + tc + 4 * RS];
            const float wv = sm.Wn[(tr + 2 * RS) * M::QW + tc + 2 * RS];
            const float av = sm.An[tr * TW + tc];
            w[gi] = wv;
            a[gi] = av;
            g[G_RR] += (double)rv * rv;
            g[G_WR] += (double)wv * rv;
            g[G_WW] += (double)wv * wv;
            g[G_AW] += (double)av * wv;
        }
        __syncthreads();
    }
    block_sum_publish<kGram, NTH, TH * TW>(g, sm.sums(), part, kMaxRedBlocks, blockIdx.x);
}

inline int ntiles_host(int H, int W) { return ((H + TH - 1) / TH) * ((W + TW - 1) / TW); }

inline int tile_blocks(int H, int W) {
    const int nt = ntiles_host(H, W);
    return nt < kMaxRedBlocks ? nt : kMaxRedBlocks;
}

// Images with fewer tiles than this run the CG iteration with kWideThreads per tile.
constexpr int kWideThreads = 1024;
constexpr int kWideBelowTiles = 512;

inline int upd_blocks(int n) {
    const int b = (n + kThreads - 1) / kThreads;
    return b < kMaxRedBlocks ? (b > 0 ? b : 1) : kMaxRedBlocks;
}

}  // namespace

void launch_apply_H(const LinOp& op, const float* x, int H, int W, float* y, hipStream_t st) {
    const int n = ((H + op.decim - 1) / op.decim) * ((W + op.decim - 1) / op.decim);
    k_apply_H<<<(n + kThreads - 1) / kThreads, kThreads, 0, st>>>(x, H, W, op.psf, op.kh, op.kw,
                                                                   op.decim, y);
}

void launch_apply_Ht(const LinOp& op, const float* y, int H, int W, float scale, float* out,
                     hipStream_t st) {
    const int n = H * W;
    k_apply_Ht<<<(n + kThreads - 1) / kThreads, kThreads, 0, st>>>(y, H, W, op.psf, op.kh, op.kw,
                                                                    op.decim, scale, out);
}

void launch_apply_A(const LinOp& op, const float* p, int H, int W, float* out, hipStream_t st) {
    const int g = tile_blocks(H, W);
    const int rr = op.separable && op.kh == op.kw ? op.kh / 2 : 0;
    if (rr == 4)
        k_apply_A<4><<<g, kThreads, 0, st>>>(op, p, H, W, out);
    else if (rr == 3)
        k_apply_A<3><<<g, kThreads, 0, st>>>(op, p, H, W, out);
    else
        k_apply_A<0><<<g, kThreads, 0, st>>>(op, p, H, W, out);
}

void launch_cg_init(const LinOp& op, const float* x_in, const float* rhs, float* r, int H, int W,
                    hipStream_t st) {
    const int g = tile_blocks(H, W);
    const int rr = op.separable && op.kh == op.kw ? op.kh / 2 : 0;
    if (rr == 4)
        k_cg_init<4><<<g, kThreads, 0, st>>>(op, x_in, rhs, r, H, W);
    else if (rr == 3)
        k_cg_init<3><<<g, kThreads, 0, st>>>(op, x_in, rhs, r, H, W);
    else
        k_cg_init<0><<<g, kThreads, 0, st>>>(op, x_in, rhs, r, H, W);
}

static void init_fp(const LinOp& op, const float* x, const float* y, const float* s, float* r,
                    float* xo, int H, int W, hipStream_t st) {
    const int g = tile_blocks(H, W);
    const int rr = op.separable && op.kh == op.kw ? op.kh / 2 : 0;
    if (rr == 4)
        k_cg_init_fp<4><<<g, kThreads, 0, st>>>(op, x, y, s, r, H, W, xo);
    else if (rr == 3)
        k_cg_init_fp<3><<<g, kThreads, 0, st>>>(op, x, y, s, r, H, W, xo);
    else
        k_cg_init_fp<0><<<g, kThreads, 0, st>>>(op, x, y, s, r, H, W, xo);
}

void launch_objective(const LinOp& op, const float* x, const float* y, const float* s, int H,
                      int W, double* part, double* out, hipStream_t st) {
    const int h = (H + op.decim - 1) / op.decim, w = (W + op.decim - 1) / op.decim;
    const int g = upd_blocks(std::max(h * w, H * W));
    k_objective<<<g, kThreads, 0, st>>>(op, x, y, s, H, W, part);
    k_objective_fin<<<1, 64, 0, st>>>(part, g, out);
}

void launch_cg_init_fp(const LinOp& op, const float* x, const float* y, const float* s, float* r,
                       int H, int W, hipStream_t st) {
    init_fp(op, x, y, s, r, nullptr, H, W, st);
}

void launch_sd_step(const LinOp& op, const float* x, const float* y, const float* s,
                    float* x_out, int H, int W, hipStream_t st) {
    init_fp(op, x, y, s, nullptr, x_out, H, W, st);
}

Partials launch_cg_w0(const LinOp& op, const float* r, float* w, int H, int W, double* part,
                      hipStream_t st) {
    const int g = tile_blocks(H, W);
    const int rr = op.separable && op.kh == op.kw ? op.kh / 2 : 0;
    if (rr == 4)
        k_cg_w0<4><<<g, kThreads, 0, st>>>(op, r, w, H, W, part);
    else if (rr == 3)
        k_cg_w0<3><<<g, kThreads, 0, st>>>(op, r, w, H, W, part);
    else
        k_cg_w0<0><<<g, kThreads, 0, st>>>(op, r, w, H, W, part);
    return Partials{part, g};
}

// The two-iteration kernels exist for separable square 7x7 and 9x9 PSFs without decimation.
static bool cg_block_eligible(const LinOp& op, int iters) {
    return op.decim == 1 && op.separable && op.kh == op.kw && (op.kh == 7 || op.kh == 9) &&
           iters >= 3;
}

int cg_rule_pack(const LinOp& op, int iters, int H, int W) {
    // small images only: there the per-kernel latency dominates; on large ones the wider
    // halos of the two-iteration kernel cost more than the launch they save
    return cg_block_eligible(op, iters) && ntiles_host(H, W) < kWideBelowTiles ? 2 : 1;
}

int cg_rule_threads(const LinOp& op, int H, int W) {
    const bool rs = op.separable && op.kh == op.kw && (op.kh == 7 || op.kh == 9);
    return rs && ntiles_host(H, W) < kWideBelowTiles ? kWideThreads : kThreads;
}

bool cg_block_ok(const LinOp& op, int iters, int H, int W) {
    if (!cg_block_eligible(op, iters)) return false;
    return op.cg_pack ? op.cg_pack == 2 : cg_rule_pack(op, iters, H, W) == 2;
}

Partials launch_cg_w0_block(const LinOp& op, const float* r, float* w, float* a, int H, int W,
                            double* part, hipStream_t st) {
    const int g = tile_blocks(H, W);
    if (op.kh == 9)
        k_cg_w0_block<4><<<g, kWideThreadsBlk, 0, st>>>(op, H, W, r, w, a, part);
    else
        k_cg_w0_block<3><<<g, kWideThreadsBlk, 0, st>>>(op, H, W, r, w, a, part);
    return Partials{part, g};
}

Partials launch_cg_block(const LinOp& op, int H, int W, int k, const float* const* vin,
                         float* const* vout, float* p, float* d, Partials rm,
                         const double* hist_prev, double* hist_cur, double* part,
                         hipStream_t st) {
    const int g = tile_blocks(H, W);
    VecSet vs;
    for (int j = 0; j < 5; ++j) {
        vs.in[j] = vin[j];
        vs.out[j] = vout[j];
    }
    if (op.kh == 9)
        k_cg_block<4><<<g, kWideThreadsBlk, 0, st>>>(op, H, W, k, vs, p, d, rm, hist_prev,
                                                     hist_cur, part);
    else
        k_cg_block<3><<<g, kWideThreadsBlk, 0, st>>>(op, H, W, k, vs, p, d, rm, hist_prev,
                                                     hist_cur, part);
    return Partials{part, g};
}

Partials launch_cg_iter(const LinOp& op, int H, int W, int k, int last, const float* r_in,
                        const float* w_in, const float* s_in, float* r_out, float* w_out,
                        float* s_out, float* p, float* d, const float* x_in, float* x_out,
                        Partials rm, const double* hist_prev, double* hist_cur, double* part,
                        hipStream_t st) {
    const int g = last ? upd_blocks(H * W) : tile_blocks(H, W);
    const int rr = op.separable && op.kh == op.kw ? op.kh / 2 : 0;
    // fewer tiles than two per CU: wide workgroups (see k_cg_iter), or the tuned choice
    const bool wide = !last && (op.cg_threads ? op.cg_threads == kWideThreads
                                              : ntiles_host(H, W) < kWideBelowTiles);
#define REDVE_CG_ITER(RS, NTH)                                                                 \
    k_cg_iter<RS, NTH><<<g, NTH, 0, st>>>(op, H, W, k, last, r_in, w_in, s_in, r_out, w_out, \
                                          s_out, p, d, x_in, x_out, rm, hist_prev, hist_cur, part)
    if (rr == 4) {
        if (wide)
            REDVE_CG_ITER(4, kWideThreads);
        else
            REDVE_CG_ITER(4, kThreads);
    } else if (rr == 3) {
        if (wide)
            REDVE_CG_ITER(3, kWideThreads);
        else
            REDVE_CG_ITER(3, kThreads);
    } else {
        REDVE_CG_ITER(0, kThreads);
    }
#undef REDVE_CG_ITER
    return Partials{part, g};
}

bool cg_iter32_ok(const LinOp& op, int iters, int H, int W) {
    const bool eligible = op.decim == 1 && op.separable && op.kh == op.kw &&
                          (op.kh == 7 || op.kh == 9) && iters >= 2;
    if (!eligible) return false;
    // rule (measured at 512^2 to 4096^2): the 32x32 form from 512 16x16 tiles (two per CU);
    // below, the two-iteration kernel
    return op.cg_tile ? op.cg_tile == 32 : ntiles_host(H, W) >= kWideBelowTiles;
}

// Workgroups of the 32x32 kernel: as many as the device holds at once (at most kMaxRedBlocks),
// so that every workgroup runs from the start and takes an equal run of tiles; a grid beyond
// that leaves a second, partial wave of workgroups.
template <int RS>
static int cg32_resident() {
    return std::min(kMaxRedBlocks,
                    resident_workgroups(reinterpret_cast<const void*>(k_cg_iter32<RS>),
                                        kCg32Threads, 0));
}

Partials launch_cg_iter32(const LinOp& op, int H, int W, int k, const float* r_in,
                          const float* p_in, float* r_out, float* p_out, float* d, Partials rm,
                          const double* hist_prev, double* hist_cur, double* part,
                          hipStream_t st) {
    const int nt = ((H + T32 - 1) / T32) * ((W + T32 - 1) / T32);
    int cap = op.kh == 9 ? cg32_resident<4>() : cg32_resident<3>();
    if (cap >= kXcds) cap -= cap % kXcds;
    const int g = nt < cap ? nt : cap;
    if (op.kh == 9)
        k_cg_iter32<4><<<g, kCg32Threads, 0, st>>>(op, H, W, k, r_in, p_in, r_out, p_out, d, rm,
                                                   hist_prev, hist_cur, part);
    else
        k_cg_iter32<3><<<g, kCg32Threads, 0, st>>>(op, H, W, k, r_in, p_in, r_out, p_out, d, rm,
                                                   hist_prev, hist_cur, part);
    return Partials{part, g};
}

void launch_cg_iter32_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int k,
                            const CgImg* cg, const float* r_in, const float* p_in, float* r_out,
                            float* p_out, float* d, double* part, int cap, hipStream_t st) {
    k_cg_iter32_batch<4><<<ntiles, kCg32Threads, 0, st>>>(desc, tiles, k, cg, r_in, p_in, r_out,
                                                          p_out, d, part, cap);
}

int launch_cg_last_diff(int n, int k, const float* r_in, const float* p, const float* d,
                        const float* x_in, float* x_out, Partials rm, const double* hist_prev,
                        float* U, int j, double* part, hipStream_t st) {
    const int g = upd_blocks(n);
#define REDVE_LD(J)                                                                         \
    case J:                                                                                 \
        k_cg_last_diff<J><<<g, kThreads, 0, st>>>(n, k, r_in, p, d, x_in, x_out, rm, hist_prev, \
                                                  U, part);                                 \
        break;
    switch (j) {
        REDVE_LD(0) REDVE_LD(1) REDVE_LD(2) REDVE_LD(3) REDVE_LD(4) REDVE_LD(5) REDVE_LD(6)
        REDVE_LD(7) REDVE_LD(8) REDVE_LD(9) REDVE_LD(10) REDVE_LD(11) REDVE_LD(12) REDVE_LD(13)
        REDVE_LD(14) REDVE_LD(15)
        default: return 0;
    }
#undef REDVE_LD
    return g;
}

static void init_fp_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs,
                          const float* sres, float* r, int sd, hipStream_t st) {
    if (rs == 4)
        k_cg_init_fp_batch<4><<<ntiles, kThreads, 0, st>>>(desc, tiles, sres, r, sd);
    else if (rs == 3)
        k_cg_init_fp_batch<3><<<ntiles, kThreads, 0, st>>>(desc, tiles, sres, r, sd);
    else
        k_cg_init_fp_batch<0><<<ntiles, kThreads, 0, st>>>(desc, tiles, sres, r, sd);
}

void launch_cg_init_fp_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs,
                             const float* sres, float* r, hipStream_t st) {
    init_fp_batch(desc, tiles, ntiles, rs, sres, r, 0, st);
}

void launch_sd_step_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs,
                          const float* sres, hipStream_t st) {
    init_fp_batch(desc, tiles, ntiles, rs, sres, nullptr, 1, st);
}

void launch_cg_w0_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs,
                        const float* r, float* w, double* part, int cap, hipStream_t st) {
    if (rs == 4)
        k_cg_w0_batch<4><<<ntiles, kThreads, 0, st>>>(desc, tiles, r, w, part, cap);
    else if (rs == 3)
        k_cg_w0_batch<3><<<ntiles, kThreads, 0, st>>>(desc, tiles, r, w, part, cap);
    else
        k_cg_w0_batch<0><<<ntiles, kThreads, 0, st>>>(desc, tiles, r, w, part, cap);
}

void launch_cg_fin_batch(const ImgDesc* desc, int nimg, int k, const double* part, int cap,
                         CgImg* cg, hipStream_t st) {
    k_cg_fin_batch<<<nimg, 512, 0, st>>>(desc, k, part, cap, cg);
}

void launch_cg_iter_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs, int k,
                          int last, const CgImg* cg, const float* r_in, const float* w_in,
                          const float* s_in, float* r_out, float* w_out, float* s_out, float* p,
                          float* d, double* part, int cap, hipStream_t st) {
    if (rs == 4)
        k_cg_iter_batch<4><<<ntiles, kThreads, 0, st>>>(desc, tiles, k, last, cg, r_in, w_in,
                                                        s_in, r_out, w_out, s_out, p, d, part, cap);
    else if (rs == 3)
        k_cg_iter_batch<3><<<ntiles, kThreads, 0, st>>>(desc, tiles, k, last, cg, r_in, w_in,
                                                        s_in, r_out, w_out, s_out, p, d, part, cap);
    else
        k_cg_iter_batch<0><<<ntiles, kThreads, 0, st>>>(desc, tiles, k, last, cg, r_in, w_in,
                                                        s_in, r_out, w_out, s_out, p, d, part, cap);
}

// Workgroups of `fn` (threads per workgroup, dynamic LDS bytes) the current device holds at once,
// a multiple of the XCD count: CUs x per-CU residency, where the per-CU figure is the larger of
// the occupancy query and the kernel's own register and LDS limits (the query reported 2 on
// gfx950 where 3 ran together; a grid matching what runs together was 1.2-1.3x faster for the
// 32x32 CG kernel than one of 1024). Cached per device, kernel and configuration.
int resident_workgroups(const void* fn, int threads, size_t dyn_smem) {
    struct Key {
        int device;
        const void* fn;
        int threads;
        size_t smem;
        bool operator<(const Key& o) const {
            return std::tie(device, fn, threads, smem) < std::tie(o.device, o.fn, o.threads, o.smem);
        }
    };
    static std::mutex mu;
    static std::map<Key, int> cache;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 1024;
    const Key key{device, fn, threads, dyn_smem};
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int cus = 0, per_cu = 0, lds_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, dyn_smem) !=
            hipSuccess ||
        cus <= 0 || per_cu <= 0)
        return 1024;
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, fn) == hipSuccess &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                              device) == hipSuccess &&
        fa.numRegs > 0 && lds_cu > 0) {
        constexpr int kWavesPerSimd = 8, kVgprsPerLane = 512, kSimds = 4;
        const int regs = (fa.numRegs + 7) / 8 * 8;
        const int waves = (threads + 63) / 64;
        const int wg_waves_per_simd = (waves + kSimds - 1) / kSimds;
        const int by_regs = std::min(kWavesPerSimd, kVgprsPerLane / regs) / wg_waves_per_simd;
        const size_t lds = fa.sharedSizeBytes + dyn_smem;
        const int by_lds = lds > 0 ? (int)(lds_cu / lds) : by_regs;
        per_cu = std::max(per_cu, std::min(by_regs, by_lds));
    }
    int g = cus * per_cu;
    if (g >= kXcds) g -= g % kXcds;
    std::lock_guard<std::mutex> lock(mu);
    cache[key] = g;
    return g;
}

}  // namespace redve
