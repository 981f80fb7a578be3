// Degradation operator H = S B (Sec. II-A, eq. (1)) and the conjugate-gradient linear step of
// the FP iteration (Sec. II-B, eq. (7); its footnote allows iterative solvers).
//
// Layout: images row-major FP32, dense rows. B is periodic (block-circulant).
// The CG matrix-vector product q = (H^T H / sigma^2 + lambda I) p is an LDS-tiled stencil: a
// workgroup loads its TH x TW tile of p plus a 2r halo (wrapped), forms B p on the tile plus an
// r halo, masks it by the decimation pattern S^T S, and applies B^T on the tile. One HBM read
// of p (plus halo) and one write of q per iteration; the dot products are FP64.
#include "internal.h"
#include "reduce.h"

namespace redve {

namespace {

constexpr int TH = 16, TW = 32;  // CG tile: 512 outputs per 256-thread workgroup
constexpr int MAXR = 7;           // PSF half-size limit (15 x 15)
constexpr int PH = TH + 4 * MAXR, PW = TW + 4 * MAXR;

__device__ inline int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
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

// Shared body of the tiled A-product. Loads P = src0 + beta * src1 (src1 may be null) on the
// tile + 2r halo, computes q = A P on the tile. Returns P and q at the thread's outputs.
struct TileIO {
    float p[TH * TW / kThreads];
    float q[TH * TW / kThreads];
};

__device__ inline void tile_apply_A(const LinOp op, const float* __restrict__ src0,
                                    const float* __restrict__ src1, float beta, int H, int W,
                                    int r0, int c0, float* sp, float* sb, TileIO& io) {
    const int rh = op.kh / 2, rw = op.kw / 2;
    const int ph = TH + 4 * rh, pw = TW + 4 * rw;  // P region
    const int bh = TH + 2 * rh, bw = TW + 2 * rw;  // B P region
    for (int e = threadIdx.x; e < ph * pw; e += kThreads) {
        const int pr = e / pw, pc = e % pw;
        const size_t g = (size_t)wrapi(r0 - 2 * rh + pr, H) * W + wrapi(c0 - 2 * rw + pc, W);
        float v = src0[g];
        if (src1) v += beta * src1[g];
        sp[pr * PW + pc] = v;
    }
    __syncthreads();
    const int s = op.decim;
    for (int e = threadIdx.x; e < bh * bw; e += kThreads) {
        const int br = e / bw, bc = e % bw;
        const int gr = wrapi(r0 - rh + br, H), gc = wrapi(c0 - rw + bc, W);
        float acc = 0.f;
        if (gr % s == 0 && gc % s == 0) {
            for (int a = -rh; a <= rh; ++a) {
                const float* prow = sp + (br + rh - a) * PW + bc + rw;
                const float* krow = op.psf + (a + rh) * op.kw + rw;
                for (int b = -rw; b <= rw; ++b) acc += krow[b] * prow[-b];
            }
        }
        sb[br * PW + bc] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TH * TW / kThreads; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int tr = o / TW, tc = o % TW;
        float acc = 0.f;
        for (int a = -rh; a <= rh; ++a) {
            const float* brow = sb + (tr + a + rh) * PW + tc + rw;
            const float* krow = op.psf + (a + rh) * op.kw + rw;
            for (int b = -rw; b <= rw; ++b) acc += krow[b] * brow[b];
        }
        const float pc = sp[(tr + 2 * rh) * PW + tc + 2 * rw];
        io.p[k] = pc;
        io.q[k] = op.inv_s2 * acc + op.lambda * pc;
    }
}

__global__ __launch_bounds__(kThreads) void k_apply_A(const LinOp op, const float* __restrict__ p,
                                                      int H, int W, float* __restrict__ out) {
    __shared__ float sp[PH * PW];
    __shared__ float sb[PH * PW];
    const int r0 = blockIdx.y * TH, c0 = blockIdx.x * TW;
    TileIO io;
    tile_apply_A(op, p, nullptr, 0.f, H, W, r0, c0, sp, sb, io);
#pragma unroll
    for (int k = 0; k < TH * TW / kThreads; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int gr = r0 + o / TW, gc = c0 + o % TW;
        if (gr < H && gc < W) out[(size_t)gr * W + gc] = io.q[k];
    }
}

// CG start for A x = rhs warm-started at x: r = rhs - A x, p = r, rho0 = r.r, beta = 0.
// The iterations then accumulate the correction d (x_out = x + d).
__global__ __launch_bounds__(kThreads) void k_cg_init(const LinOp op, const float* __restrict__ x_in,
                                                      const float* __restrict__ rhs,
                                                      float* __restrict__ r,
                                                      float* __restrict__ p, int H, int W,
                                                      Reduction red, CgScalars* sc) {
    __shared__ float sp[PH * PW];
    __shared__ float sb[PH * PW];
    __shared__ double sred[kThreads / 64];
    const int r0 = blockIdx.y * TH, c0 = blockIdx.x * TW;
    TileIO io;
    tile_apply_A(op, x_in, nullptr, 0.f, H, W, r0, c0, sp, sb, io);
    double acc[1] = {0.0};
#pragma unroll
    for (int k = 0; k < TH * TW / kThreads; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int gr = r0 + o / TW, gc = c0 + o % TW;
        if (gr < H && gc < W) {
            const size_t g = (size_t)gr * W + gc;
            const float rv = rhs[g] - io.q[k];
            r[g] = rv;
            p[g] = rv;
            acc[0] += (double)rv * (double)rv;
        }
    }
    block_sum<1>(acc, sred);
    double tot[1];
    const int blk = blockIdx.y * gridDim.x + blockIdx.x, nblk = gridDim.x * gridDim.y;
    if (grid_sum<1>(acc, tot, red, blk, nblk, sred) && threadIdx.x == 0) {
        sc->rho0 = tot[0];
        sc->beta = 0.0;
    }
}

// CG start of one FP call (eq. (7)) in residual form. With rhs = H^T y / sigma^2 + lambda f(x),
//   r = rhs - A x = H^T (y - H x) / sigma^2 + lambda (f(x) - x),
// both terms small near the fixed point; the data term is accumulated in FP64 from the FP32
// image, so r carries no rounding of the O(|x|) quantities rhs and A x. s = f(x) - x (null:
// the identity denoiser, s = 0). p = r, rho0 = r.r, beta = 0.
__global__ __launch_bounds__(kThreads) void k_cg_init_fp(const LinOp op, const double* __restrict__ psf64,
                                                         const float* __restrict__ x,
                                                         const float* __restrict__ y,
                                                         const float* __restrict__ s,
                                                         float* __restrict__ r,
                                                         float* __restrict__ p, int H, int W,
                                                         Reduction red, CgScalars* sc) {
    __shared__ float sp[PH * PW];
    __shared__ double se[PH * PW];
    __shared__ double sred[kThreads / 64];
    const int r0 = blockIdx.y * TH, c0 = blockIdx.x * TW;
    const int rh = op.kh / 2, rw = op.kw / 2, dec = op.decim;
    const int ph = TH + 4 * rh, pw = TW + 4 * rw;
    const int bh = TH + 2 * rh, bw = TW + 2 * rw;
    const int wy = (W + dec - 1) / dec;
    for (int e = threadIdx.x; e < ph * pw; e += kThreads) {
        const int pr = e / pw, pc = e % pw;
        sp[pr * PW + pc] = x[(size_t)wrapi(r0 - 2 * rh + pr, H) * W + wrapi(c0 - 2 * rw + pc, W)];
    }
    __syncthreads();
    // e = S^T (y - S B x) on the tile + r halo, FP64
    for (int e = threadIdx.x; e < bh * bw; e += kThreads) {
        const int br = e / bw, bc = e % bw;
        const int gr = wrapi(r0 - rh + br, H), gc = wrapi(c0 - rw + bc, W);
        double v = 0.0;
        if (gr % dec == 0 && gc % dec == 0) {
            double bx = 0.0;
            for (int a = -rh; a <= rh; ++a) {
                const float* prow = sp + (br + rh - a) * PW + bc + rw;
                const double* krow = psf64 + (a + rh) * op.kw + rw;
                for (int b = -rw; b <= rw; ++b) bx += krow[b] * (double)prow[-b];
            }
            v = (double)y[(size_t)(gr / dec) * wy + gc / dec] - bx;
        }
        se[br * PW + bc] = v;
    }
    __syncthreads();
    const double is2 = op.inv_s2_d;
    double acc[1] = {0.0};
#pragma unroll
    for (int k = 0; k < TH * TW / kThreads; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int tr = o / TW, tc = o % TW;
        const int gr = r0 + tr, gc = c0 + tc;
        double bt = 0.0;
        for (int a = -rh; a <= rh; ++a) {
            const double* erow = se + (tr + a + rh) * PW + tc + rw;
            const double* krow = psf64 + (a + rh) * op.kw + rw;
            for (int b = -rw; b <= rw; ++b) bt += krow[b] * erow[b];
        }
        if (gr < H && gc < W) {
            const size_t g = (size_t)gr * W + gc;
            double rv = is2 * bt;
            if (s) rv += op.lambda_d * (double)s[g];
            const float rf = (float)rv;
            r[g] = rf;
            p[g] = rf;
            acc[0] += (double)rf * (double)rf;
        }
    }
    block_sum<1>(acc, sred);
    double tot[1];
    const int blk = blockIdx.y * gridDim.x + blockIdx.x, nblk = gridDim.x * gridDim.y;
    if (grid_sum<1>(acc, tot, red, blk, nblk, sred) && threadIdx.x == 0) {
        sc->rho0 = tot[0];
        sc->beta = 0.0;
    }
}

// CG direction + product: p_new = r + beta p_old (on the fly, halo included), q = A p_new,
// pq = p_new . q, alpha = rho0 / pq (0 once the residual vanished).
__global__ __launch_bounds__(kThreads) void k_cg_q(const LinOp op, const float* __restrict__ r,
                                                   const float* __restrict__ p_old,
                                                   float* __restrict__ p_new,
                                                   float* __restrict__ q, int H, int W,
                                                   Reduction red, CgScalars* sc) {
    __shared__ float sp[PH * PW];
    __shared__ float sb[PH * PW];
    __shared__ double sred[kThreads / 64];
    const int r0 = blockIdx.y * TH, c0 = blockIdx.x * TW;
    const float beta = (float)sc->beta;
    TileIO io;
    tile_apply_A(op, r, p_old, beta, H, W, r0, c0, sp, sb, io);
    double acc[1] = {0.0};
#pragma unroll
    for (int k = 0; k < TH * TW / kThreads; ++k) {
        const int o = threadIdx.x + k * kThreads;
        const int gr = r0 + o / TW, gc = c0 + o % TW;
        if (gr < H && gc < W) {
            const size_t g = (size_t)gr * W + gc;
            p_new[g] = io.p[k];
            q[g] = io.q[k];
            acc[0] += (double)io.p[k] * (double)io.q[k];
        }
    }
    block_sum<1>(acc, sred);
    double tot[1];
    const int blk = blockIdx.y * gridDim.x + blockIdx.x, nblk = gridDim.x * gridDim.y;
    if (grid_sum<1>(acc, tot, red, blk, nblk, sred) && threadIdx.x == 0) {
        const double rho0 = sc->rho0;
        sc->pq = tot[0];
        sc->alpha = (rho0 > 1e-300 && tot[0] > 0.0) ? rho0 / tot[0] : 0.0;
    }
}

// CG update on the correction: d += alpha p (d = alpha p on the first iteration),
// r -= alpha q, rho1 = r.r, beta = rho1 / rho0, rho0 = rho1. On the last iteration the new
// iterate x_out = x_in + d is written instead of d (one rounding of the O(|x|) quantity).
constexpr int UPD_PER_THREAD = 4;
__global__ __launch_bounds__(kThreads) void k_cg_update(float* __restrict__ d, float* __restrict__ r,
                                                        const float* __restrict__ p,
                                                        const float* __restrict__ q, int n,
                                                        int first, const float* __restrict__ x_in,
                                                        float* __restrict__ x_out,
                                                        Reduction red, CgScalars* sc) {
    __shared__ double sred[kThreads / 64];
    const float alpha = (float)sc->alpha;
    double acc[1] = {0.0};
    const int base = blockIdx.x * kThreads * UPD_PER_THREAD + threadIdx.x;
#pragma unroll
    for (int k = 0; k < UPD_PER_THREAD; ++k) {
        const int i = base + k * kThreads;
        if (i < n) {
            const float dv = first ? alpha * p[i] : d[i] + alpha * p[i];
            if (x_out)
                x_out[i] = x_in[i] + dv;
            else
                d[i] = dv;
            const float rv = r[i] - alpha * q[i];
            r[i] = rv;
            acc[0] += (double)rv * (double)rv;
        }
    }
    block_sum<1>(acc, sred);
    double tot[1];
    if (grid_sum<1>(acc, tot, red, blockIdx.x, gridDim.x, sred) && threadIdx.x == 0) {
        const double rho0 = sc->rho0;
        sc->beta = rho0 > 1e-300 ? tot[0] / rho0 : 0.0;
        sc->rho0 = tot[0];
    }
}

// out = b0 + lambda u (right-hand side of eq. (7) when the denoiser has no stages).
__global__ __launch_bounds__(kThreads) void k_axpb(const float* __restrict__ b0,
                                                   const float* __restrict__ u, float lambda,
                                                   float* __restrict__ out, int n) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = b0[i] + lambda * u[i];
}

inline dim3 tile_grid(int H, int W) { return dim3((W + TW - 1) / TW, (H + TH - 1) / TH); }

}  // namespace

int linop_grid(int H, int W) {
    dim3 g = tile_grid(H, W);
    return (int)(g.x * g.y);
}

int cg_update_grid(int n) { return (n + kThreads * UPD_PER_THREAD - 1) / (kThreads * UPD_PER_THREAD); }

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
    k_apply_A<<<tile_grid(H, W), kThreads, 0, st>>>(op, p, H, W, out);
}

void launch_cg_init(const LinOp& op, const float* x_in, const float* rhs, float* r, float* p,
                    int H, int W, Reduction red, CgScalars* sc, hipStream_t st) {
    k_cg_init<<<tile_grid(H, W), kThreads, 0, st>>>(op, x_in, rhs, r, p, H, W, red, sc);
}

void launch_cg_init_fp(const LinOp& op, const double* psf64, const float* x, const float* y,
                       const float* s, float* r, float* p, int H, int W, Reduction red,
                       CgScalars* sc, hipStream_t st) {
    k_cg_init_fp<<<tile_grid(H, W), kThreads, 0, st>>>(op, psf64, x, y, s, r, p, H, W, red, sc);
}

void launch_cg_q(const LinOp& op, const float* r, const float* p_old, float* p_new, float* q,
                 int H, int W, Reduction red, CgScalars* sc, hipStream_t st) {
    k_cg_q<<<tile_grid(H, W), kThreads, 0, st>>>(op, r, p_old, p_new, q, H, W, red, sc);
}

void launch_cg_update(float* d, float* r, const float* p, const float* q, int n, int first,
                      const float* x_in, float* x_out, Reduction red, CgScalars* sc,
                      hipStream_t st) {
    k_cg_update<<<cg_update_grid(n), kThreads, 0, st>>>(d, r, p, q, n, first, x_in, x_out, red, sc);
}

void launch_axpb(const float* b0, const float* u, float lambda, float* out, int n,
                 hipStream_t st) {
    k_axpb<<<(n + kThreads - 1) / kThreads, kThreads, 0, st>>>(b0, u, lambda, out, n);
}

}  // namespace redve
