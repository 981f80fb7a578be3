// Vector extrapolation on the GPU (Sec. III-B): MPE (Algorithm 1), RRE (eq. (19)), SVD-MPE.
//
// The N x (kappa+1) difference matrix U (Algorithm 1, step 1) lives in HBM, one FP32 image per
// column, written as each FP iterate arrives (the in-place storage remark of Sec. III-B keeps
// kappa+2 vectors; here: x_m plus the columns). Instead of running modified Gram-Schmidt
// (Algorithm 2) over the tall matrix, which would need kappa+1 dependent passes, each new
// column's FP64 inner products with the previous columns are accumulated in the same pass that
// forms it: the Gram matrix G = U^T U. Its Cholesky factor is the R of Algorithm 2 (QR of U
// gives U^T U = R^T R with the same positive-diagonal R), and Algorithm 1 only needs R and
// Q_{kappa-1} eta = U_{kappa-1} R_{kappa-1}^{-1} eta = U_{kappa-1} xi. So the extrapolated vector
// is x_m + U_{kappa-1} xi, one more streaming pass. The L x L work is one FP64 thread.
#include <math.h>

#include "internal.h"
#include "reduce.h"

namespace redve {

namespace {

// One pass over two consecutive iterates: u = x_new - x_old, its inner products with the
// NC earlier columns, ||u||^2 and ||x_old||^2, published as per-workgroup partials.
template <int NC>
__global__ __launch_bounds__(kThreads) void k_diff_gram(const float* __restrict__ x_new,
                                                        const float* __restrict__ x_old,
                                                        float* __restrict__ U, int n,
                                                        double* __restrict__ part) {
    constexpr int NV = NC + 2;
    __shared__ double sred[NV * kThreads / 64];
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const int stride = gridDim.x * kThreads;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const float xo = x_old[i];
        const float uv = x_new[i] - xo;
        if (U) U[(size_t)NC * n + i] = uv;
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] += (double)uv * (double)U[(size_t)k * n + i];
        acc[NC] += (double)uv * (double)uv;
        acc[NC + 1] += (double)xo * (double)xo;
    }
    block_sum<NV>(acc, sred);
    publish<NV>(acc, part, kMaxRedBlocks, blockIdx.x);
}

// ---- small dense FP64 algebra, one thread ----------------------------------------------

constexpr int MAXL = 16;  // REDVE_MAX_L

// Work area of the one-thread L x L solver, in LDS (private arrays indexed at run time would
// live in scratch memory).
struct SolveWork {
    double R[MAXL][MAXL];
    double A[MAXL][MAXL], V[MAXL][MAXL];  // SVD-MPE
    double t0[MAXL], t1[MAXL], t2[MAXL];  // vectors of the triangular solves
    double gamma[MAXL];
};

__device__ void back_sub(const double (*R)[MAXL], int k, const double* b, double* x) {
    for (int i = k - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < k; ++j) s -= R[i][j] * x[j];
        x[i] = s / R[i][i];
    }
}

__device__ void fwd_sub_t(const double (*R)[MAXL], int k, const double* b, double* x) {
    for (int i = 0; i < k; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= R[j][i] * x[j];
        x[i] = s / R[i][i];
    }
}

__device__ bool full_rank(const double (*R)[MAXL], int k, double eps) {
    if (k == 0) return true;
    if (!(R[0][0] > 0.0)) return false;
    for (int j = 0; j < k; ++j)
        if (!(fabs(R[j][j]) > eps * R[0][0])) return false;
    return true;
}

// MPE (Algorithm 1, step 2): R_{k-1} c' = -r_{k+1}, c = (c', 1), gamma = c / sum(c).
__device__ bool mpe(const double (*R)[MAXL], int k, double eps, double* gamma, SolveWork& ws) {
    if (!full_rank(R, k, eps)) return false;
    double* c = ws.t0;
    double* rhs = ws.t1;
    for (int i = 0; i < k; ++i) rhs[i] = -R[i][k];
    back_sub(R, k, rhs, c);
    c[k] = 1.0;
    double s = 0.0, a = 0.0;
    for (int i = 0; i <= k; ++i) {
        s += c[i];
        a += fabs(c[i]);
    }
    if (!(fabs(s) > 1e-12 * a)) return false;
    for (int i = 0; i <= k; ++i) gamma[i] = c[i] / s;
    return true;
}

// RRE on the leading k + 1 columns of a full-rank R (eq. (19)): R^T R d = 1 by forward then
// backward substitution, gamma = d / sum(d).
__device__ __noinline__ void rre_full(const double (*R)[MAXL], int k, double* gamma,
                                      SolveWork& ws) {
    double* ones = ws.t0;
    double* w = ws.t1;
    double* d = ws.t2;
    for (int i = 0; i <= k; ++i) ones[i] = 1.0;
    fwd_sub_t(R, k + 1, ones, w);
    back_sub(R, k + 1, w, d);
    double s = 0.0;
    for (int i = 0; i <= k; ++i) s += d[i];
    for (int i = 0; i <= k; ++i) gamma[i] = d[i] / s;
}

// RRE (eq. (19)). A dependent last column: MPE's null vector attains ||U gamma|| = 0; if MPE
// does not exist either, RRE_k = RRE_{k-1} (Sec. III-B). Returns the kappa used. The column
// count of each attempt is a loop variable of its own: the form that decremented the argument
// in an unbounded loop was compiled for gfx950 (run-time window sizes) into code that solved
// with one column count and returned another.
__device__ int rre(const double (*R)[MAXL], int k, double eps, double* gamma, SolveWork& ws) {
    for (int kk = k; kk >= 1; --kk) {
        if (full_rank(R, kk + 1, eps)) {
            rre_full(R, kk, gamma, ws);
            return kk;
        }
        if (mpe(R, kk, eps, gamma, ws)) return kk;
    }
    if (full_rank(R, 1, eps)) {
        rre_full(R, 0, gamma, ws);
    } else {
        gamma[0] = 1.0;
    }
    return 0;
}

// SVD-MPE (Sec. III-B): gamma = v / sum(v), v the right singular vector of the smallest
// singular value of R, by one-sided Jacobi rotations on the columns of R.
__device__ bool svd_mpe(const double (*R)[MAXL], int k, double* gamma, SolveWork& ws) {
    const int n = k + 1;
    double(*A)[MAXL] = ws.A;
    double(*V)[MAXL] = ws.V;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            A[i][j] = (j >= i) ? R[i][j] : 0.0;
            V[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < n; ++i) {
                    al += A[i][p] * A[i][p];
                    be += A[i][q] * A[i][q];
                    ga += A[i][p] * A[i][q];
                }
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                off = fmax(off, fabs(ga) / sqrt(al * be));
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < n; ++i) {
                    const double ap = A[i][p], aq = A[i][q];
                    A[i][p] = c * ap - s * aq;
                    A[i][q] = s * ap + c * aq;
                    const double vp = V[i][p], vq = V[i][q];
                    V[i][p] = c * vp - s * vq;
                    V[i][q] = s * vp + c * vq;
                }
            }
        if (off <= 1e-15) break;
    }
    int jmin = 0;
    double smin = INFINITY;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += A[i][j] * A[i][j];
        if (s < smin) {
            smin = s;
            jmin = j;
        }
    }
    double s = 0.0, a = 0.0;
    for (int i = 0; i < n; ++i) {
        s += V[i][jmin];
        a += fabs(V[i][jmin]);
    }
    if (!(fabs(s) > 1e-12 * a)) return false;
    for (int i = 0; i < n; ++i) gamma[i] = V[i][jmin] / s;
    return true;
}

// The L x L work of Algorithm 1 on one thread: Cholesky of the Gram matrix (= the R of
// Algorithm 2), MPE / RRE / SVD-MPE coefficients, xi; writes gamma, xi, ncols, breakdown.
__device__ void small_solve(const double* G, int ldG, int L, int method, double rank_eps,
                            VeInfo* __restrict__ info, SolveWork& ws) {
    // Cholesky G = R^T R (upper R). A column whose pivot falls under the rank threshold gets
    // R_ii = 0 and a zero row, as modified Gram-Schmidt gives a zero q_i for it.
    double(*R)[MAXL] = ws.R;
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) R[i][j] = 0.0;
    for (int i = 0; i < L; ++i) {
        double d = G[i * ldG + i];
        for (int k = 0; k < i; ++k) d -= R[k][i] * R[k][i];
        double rii = sqrt(fmax(d, 0.0));
        if (i > 0 && !(rii > rank_eps * R[0][0])) rii = 0.0;
        R[i][i] = rii;
        for (int j = i + 1; j < L; ++j) {
            double s = G[i * ldG + j];
            for (int k = 0; k < i; ++k) s -= R[k][i] * R[k][j];
            R[i][j] = rii > 0.0 ? s / rii : 0.0;
        }
    }
    double* gamma = ws.gamma;
    int k = L - 1;
    bool ok;
    if (method == 1) {
        ok = mpe(R, k, rank_eps, gamma, ws);
    } else if (method == 2) {
        k = rre(R, k, rank_eps, gamma, ws);
        ok = true;
    } else {
        ok = svd_mpe(R, k, gamma, ws);
    }
    for (int i = 0; i < MAXL; ++i) {
        info->xi[i] = 0.0;
        info->gamma[i] = 0.0;
    }
    info->guarded = 0;
    if (!ok) {
        // no extrapolation: x_m + sum of all L differences = the last FP iterate
        for (int j = 0; j < L; ++j) info->xi[j] = 1.0;
        info->ncols = L;
        info->breakdown = 1;
        info->kappa_used = L - 1;
        info->gamma_l1 = 0.0;
        return;
    }
    // Algorithm 1, step 3: xi_0 = 1 - gamma_0, xi_j = xi_{j-1} - gamma_j (j < kappa)
    double acc = 1.0, l1 = 0.0;
    for (int j = 0; j < k; ++j) {
        acc -= gamma[j];
        info->xi[j] = acc;
    }
    for (int j = 0; j <= k; ++j) {
        info->gamma[j] = gamma[j];
        l1 += fabs(gamma[j]);
    }
    info->ncols = k;
    info->breakdown = 0;
    info->kappa_used = k;
    info->gamma_l1 = l1;
}

// The same L x L work for MPE and RRE on a window of L <= 6 with the matrices in registers
// (every loop has compile-time bounds): the operations and their order are small_solve's, so
// the results are bitwise its own. Returns false, having written nothing, where the window is
// rank deficient; small_solve then handles the breakdown rules.
template <int L>
__device__ bool small_solve_reg(const double* G, int ldG, int method, double rank_eps,
                                VeInfo* __restrict__ info) {
    double R[L][L];
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
        for (int j = 0; j < L; ++j) R[i][j] = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
        double d = G[i * ldG + i];
#pragma unroll
        for (int k = 0; k < i; ++k) d -= R[k][i] * R[k][i];
        double rii = sqrt(fmax(d, 0.0));
        if (i > 0 && !(rii > rank_eps * R[0][0])) rii = 0.0;
        R[i][i] = rii;
#pragma unroll
        for (int j = i + 1; j < L; ++j) {
            double sum = G[i * ldG + j];
#pragma unroll
            for (int k = 0; k < i; ++k) sum -= R[k][i] * R[k][j];
            R[i][j] = rii > 0.0 ? sum / rii : 0.0;
        }
    }
    // full rank of the leading n = k (MPE) or k + 1 (RRE) columns, as full_rank above
    constexpr int k = L - 1;
    const int n = method == 1 ? k : k + 1;
    bool full = n == 0 || R[0][0] > 0.0;
#pragma unroll
    for (int j = 0; j < L; ++j)
        if (j < n && !(fabs(R[j][j]) > rank_eps * R[0][0])) full = false;
    if (!full) return false;
    double gamma[L];
    if (method == 1) {  // MPE: R_{k-1} c' = -r_{k}, c = (c', 1)
        double c[L];
#pragma unroll
        for (int i = k - 1; i >= 0; --i) {
            double sum = -R[i][k];
#pragma unroll
            for (int j = i + 1; j < k; ++j) sum -= R[i][j] * c[j];
            c[i] = sum / R[i][i];
        }
        c[k] = 1.0;
        double sc = 0.0, ac = 0.0;
#pragma unroll
        for (int i = 0; i <= k; ++i) {
            sc += c[i];
            ac += fabs(c[i]);
        }
        if (!(fabs(sc) > 1e-12 * ac)) return false;
#pragma unroll
        for (int i = 0; i <= k; ++i) gamma[i] = c[i] / sc;
    } else {  // RRE: R^T R d = 1
        double wv[L], dv[L];
#pragma unroll
        for (int i = 0; i <= k; ++i) {
            double sum = 1.0;
#pragma unroll
            for (int j = 0; j < i; ++j) sum -= R[j][i] * wv[j];
            wv[i] = sum / R[i][i];
        }
#pragma unroll
        for (int i = k; i >= 0; --i) {
            double sum = wv[i];
#pragma unroll
            for (int j = i + 1; j <= k; ++j) sum -= R[i][j] * dv[j];
            dv[i] = sum / R[i][i];
        }
        double sd = 0.0;
#pragma unroll
        for (int i = 0; i <= k; ++i) sd += dv[i];
#pragma unroll
        for (int i = 0; i <= k; ++i) gamma[i] = dv[i] / sd;
    }
    for (int i = 0; i < MAXL; ++i) {
        info->xi[i] = 0.0;
        info->gamma[i] = 0.0;
    }
    // Algorithm 1, step 3
    double acc = 1.0, l1 = 0.0;
#pragma unroll
    for (int j = 0; j < k; ++j) {
        acc -= gamma[j];
        info->xi[j] = acc;
    }
#pragma unroll
    for (int j = 0; j <= k; ++j) {
        info->gamma[j] = gamma[j];
        l1 += fabs(gamma[j]);
    }
    info->ncols = k;
    info->breakdown = 0;
    info->kappa_used = k;
    info->gamma_l1 = l1;
    info->guarded = 0;
    return true;
}

__device__ bool small_solve_fast(const double* G, int ldG, int L, int method, double rank_eps,
                                 VeInfo* __restrict__ info) {
    if (method != 1 && method != 2) return false;
    switch (L) {
        case 2: return small_solve_reg<2>(G, ldG, method, rank_eps, info);
        case 3: return small_solve_reg<3>(G, ldG, method, rank_eps, info);
        case 4: return small_solve_reg<4>(G, ldG, method, rank_eps, info);
        case 5: return small_solve_reg<5>(G, ldG, method, rank_eps, info);
        case 6: return small_solve_reg<6>(G, ldG, method, rank_eps, info);
        default: return false;
    }
}

// Stability guard (Sec. III-D, eq. (21): the extrapolated vector sum_i gamma_i x_{m+i} carries
// the iterates' errors magnified by up to sum |gamma_i|). With cap > 0, coefficients whose
// sum |gamma| exceeds cap, or is not finite, are rejected: the cycle continues from its last FP
// iterate x_{m+L} (xi = 1 on all L columns), counted as a breakdown; gamma and gamma_l1 keep
// the rejected values for the statistics.
__device__ void guard_extrapolation(VeInfo* __restrict__ info, int L, double cap) {
    if (!(cap > 0.0) || info->breakdown || info->gamma_l1 <= cap) return;
    for (int j = 0; j < MAXL; ++j) info->xi[j] = j < L ? 1.0 : 0.0;
    info->ncols = L;
    info->breakdown = 1;
    info->guarded = 1;
}

// Sums the window's published partials into the Gram matrix (fixed order, FP64; one wave per
// entry, 16 waves), then the L x L work on one thread.
constexpr int kSolveThreads = 1024;

__global__ __launch_bounds__(kSolveThreads) void k_ve_solve(const double* __restrict__ part,
                                                            size_t win_stride, int nblk, int L,
                                                            int method, double rank_eps,
                                                            double gamma_cap,
                                                            VeInfo* __restrict__ info) {
    __shared__ double G[MAXL * MAXL];
    __shared__ double norms[2];
    __shared__ SolveWork ws;
    // column j's pass published values k < j (u_j . u_k), j (u_j . u_j), j + 1 (x . x)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int npairs = L * (L + 3) / 2;  // sum over j of (j + 2)
    constexpr int NW = kSolveThreads / 64;
    // a wave sums the published values q and q + NW together (their loads in flight at once)
    for (int q0 = wave; q0 < npairs; q0 += 2 * NW) {
        int jj[2], kk[2];
        const double* pp[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = q0 + h * NW < npairs ? q0 + h * NW : q0;
            int j = 0, base = 0;
            while (base + j + 2 <= q) {
                base += j + 2;
                ++j;
            }
            jj[h] = j;
            kk[h] = q - base;
            pp[h] = part + (size_t)j * win_stride + (size_t)kk[h] * kMaxRedBlocks;
        }
        double sum[2] = {0.0, 0.0};
        for (int i = lane; i < nblk; i += 64) {
            sum[0] += pp[0][i];
            sum[1] += pp[1][i];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && q0 + NW >= npairs) break;
            const double sv = wave_sum(sum[h]);
            const int j = jj[h], k = kk[h];
            if (lane == 0) {
                if (k <= j) {
                    G[j * MAXL + k] = sv;
                    G[k * MAXL + j] = sv;
                    if (k == j && j == L - 1) norms[0] = sv;
                } else if (j == L - 1) {
                    norms[1] = sv;
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    info->uu = norms[0];
    info->xx = norms[1];
    if (!small_solve_fast(G, MAXL, L, method, rank_eps, info))
        small_solve(G, MAXL, L, method, rank_eps, info, ws);
    guard_extrapolation(info, L, gamma_cap);
}

// Algorithm 1, step 4: x_(m,kappa) = x_m + U_{kappa-1} xi (= x_m + Q_{kappa-1} eta).
__global__ __launch_bounds__(kThreads) void k_ve_combine(const float* __restrict__ x_m,
                                                         const float* __restrict__ U, int n,
                                                         const VeInfo* __restrict__ info,
                                                         float* __restrict__ out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int nc = info->ncols;
    double acc = (double)x_m[i];
    for (int j = 0; j < nc; ++j) acc += info->xi[j] * (double)U[(size_t)j * n + i];
    out[i] = (float)acc;
}

// Relative change of one FP call: sums a single difference pass (j = 0) into uu, xx.
__global__ __launch_bounds__(64) void k_delta(const double* __restrict__ part, int nblk,
                                              VeInfo* __restrict__ info) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 64) {
        s0 += part[i];
        s1 += part[kMaxRedBlocks + i];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (threadIdx.x == 0) {
        info->uu = s0;
        info->xx = s1;
    }
}

// ---- batched kernels ----------------------------------------------------------------------

// One tile of one image: u = x_out - x_in (stored as window column wj when wj >= 0), its inner
// products with window columns 0..wj, ||u||^2, ||x_in||^2; NL + 2 per-tile partials.
template <int NL>
__global__ __launch_bounds__(kThreads) void k_diff_gram_batch(const ImgDesc* __restrict__ desc,
                                                              const TileRef* __restrict__ tiles,
                                                              float* __restrict__ U,
                                                              size_t ustride,
                                                              double* __restrict__ part, int cap) {
    constexpr int NV = NL + 2;
    __shared__ double sred[NV * kThreads / 64];
    const TileRef e = tiles[blockIdx.x];
    const ImgDesc& d = desc[e.img];
    if (!d.active) return;
    const int t = e.t, ntx = (d.W + kBatchTile - 1) / kBatchTile, bt = d.tile0 + t;
    const int gr = (t / ntx) * kBatchTile + threadIdx.x / kBatchTile;
    const int gc = (t % ntx) * kBatchTile + threadIdx.x % kBatchTile;
    const int j = d.wj;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    if (gr < d.H && gc < d.W) {
        const size_t g = (size_t)gr * d.W + gc;
        const float xo = d.x_in[g];
        const float uv = d.x_out[g] - xo;
        float* Ui = U + d.off + g;
        if (j >= 0) Ui[(size_t)j * ustride] = uv;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            if (k < j) acc[k] = (double)uv * (double)Ui[(size_t)k * ustride];
            else if (k == j) acc[k] = (double)uv * (double)uv;
        }
        acc[NL] = (double)uv * (double)uv;
        acc[NL + 1] = (double)xo * (double)xo;
    }
    block_sum<NV>(acc, sred);
    publish<NV>(acc, part, cap, bt);
}

// Per image: sums the tile partials in tile order into Gram row wj and the norms (one wave
// per value; each value summed in the same fixed order).
__global__ __launch_bounds__(256) void k_diff_fin_batch(const ImgDesc* __restrict__ desc, int L,
                                                        const double* __restrict__ part, int cap,
                                                        double* __restrict__ G,
                                                        ImgStat* __restrict__ stat) {
    const ImgDesc& d = desc[blockIdx.x];
    if (!d.active) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* Gi = G + (size_t)blockIdx.x * MAXL * MAXL;
    for (int v = wave; v < L + 2; v += 4) {
        const bool gram = v < L && v <= d.wj;
        if (v < L && !gram) continue;
        double sum = 0.0;
        for (int i = lane; i < d.ntiles; i += 64) sum += part[(size_t)v * cap + d.tile0 + i];
        sum = wave_sum(sum);
        if (lane == 0) {
            if (gram) {
                Gi[d.wj * MAXL + v] = sum;
                Gi[v * MAXL + d.wj] = sum;
            } else if (v == L) {
                stat[blockIdx.x].uu = sum;
            } else {
                stat[blockIdx.x].xx = sum;
            }
        }
    }
}

// Per image that completes its window this round: the L x L solve.
__global__ __launch_bounds__(64) void k_ve_solve_batch(const ImgDesc* __restrict__ desc, int L,
                                                       int method, double rank_eps,
                                                       double gamma_cap,
                                                       const double* __restrict__ G,
                                                       VeInfo* __restrict__ info,
                                                       ImgStat* __restrict__ stat) {
    __shared__ SolveWork ws;
    const ImgDesc& d = desc[blockIdx.x];
    if (!d.active || !d.do_ve || threadIdx.x != 0) return;
    VeInfo* in = info + blockIdx.x;
    small_solve(G + (size_t)blockIdx.x * MAXL * MAXL, MAXL, L, method, rank_eps, in, ws);
    guard_extrapolation(in, L, gamma_cap);
    stat[blockIdx.x].gamma_l1 = in->gamma_l1;
    stat[blockIdx.x].breakdown = in->breakdown;
    stat[blockIdx.x].guarded = in->guarded;
}

// x_m = x_m + U_{kappa-1} xi on one tile of an image that extrapolates this round.
__global__ __launch_bounds__(kThreads) void k_ve_combine_batch(const ImgDesc* __restrict__ desc,
                                                               const TileRef* __restrict__ tiles,
                                                               const float* __restrict__ U,
                                                               size_t ustride,
                                                               const VeInfo* __restrict__ info) {
    const TileRef e = tiles[blockIdx.x];
    const int img = e.img;
    const ImgDesc& d = desc[img];
    if (!d.active || !d.do_ve) return;
    const int t = e.t, ntx = (d.W + kBatchTile - 1) / kBatchTile;
    const int gr = (t / ntx) * kBatchTile + threadIdx.x / kBatchTile;
    const int gc = (t % ntx) * kBatchTile + threadIdx.x % kBatchTile;
    if (gr >= d.H || gc >= d.W) return;
    const size_t g = (size_t)gr * d.W + gc;
    const VeInfo& in = info[img];
    double acc = (double)d.x_m[g];
    for (int j = 0; j < in.ncols; ++j) acc += in.xi[j] * (double)U[(size_t)j * ustride + d.off + g];
    d.x_m[g] = (float)acc;
}

}  // namespace

int launch_diff_gram(const float* x_new, const float* x_old, float* U, int j, int n, double* part,
                     hipStream_t st) {
    int g = (n + kThreads - 1) / kThreads;
    g = g < kMaxRedBlocks ? (g > 0 ? g : 1) : kMaxRedBlocks;
#define REDVE_DG(J)                                                                   \
    case J:                                                                           \
        k_diff_gram<J><<<g, kThreads, 0, st>>>(x_new, x_old, U, n, part);             \
        break;
    switch (j) {
        REDVE_DG(0) REDVE_DG(1) REDVE_DG(2) REDVE_DG(3) REDVE_DG(4) REDVE_DG(5) REDVE_DG(6)
        REDVE_DG(7) REDVE_DG(8) REDVE_DG(9) REDVE_DG(10) REDVE_DG(11) REDVE_DG(12) REDVE_DG(13)
        REDVE_DG(14) REDVE_DG(15)
        default: break;
    }
#undef REDVE_DG
    return g;
}

void launch_delta(const double* part, int nblk, VeInfo* info, hipStream_t st) {
    k_delta<<<1, 64, 0, st>>>(part, nblk, info);
}

void launch_ve_solve(const double* part, size_t win_stride, int nblk, int L, int method,
                     double rank_eps, double gamma_cap, VeInfo* info, hipStream_t st) {
    k_ve_solve<<<1, kSolveThreads, 0, st>>>(part, win_stride, nblk, L, method, rank_eps,
                                             gamma_cap, info);
}

void launch_ve_combine(const float* x_m, const float* U, int n, const VeInfo* info, float* out,
                       hipStream_t st) {
    k_ve_combine<<<(n + kThreads - 1) / kThreads, kThreads, 0, st>>>(x_m, U, n, info, out);
}

void launch_diff_gram_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int L, float* U,
                            size_t ustride, double* part, int cap, hipStream_t st) {
#define REDVE_DGB(N)                                                                       \
    case N:                                                                                \
        k_diff_gram_batch<N><<<ntiles, kThreads, 0, st>>>(desc, tiles, U, ustride, part, cap); \
        break;
    switch (L) {
        REDVE_DGB(1) REDVE_DGB(2) REDVE_DGB(3) REDVE_DGB(4) REDVE_DGB(5) REDVE_DGB(6) REDVE_DGB(7)
        REDVE_DGB(8) REDVE_DGB(9) REDVE_DGB(10) REDVE_DGB(11) REDVE_DGB(12) REDVE_DGB(13)
        REDVE_DGB(14) REDVE_DGB(15) REDVE_DGB(16)
        default: break;
    }
#undef REDVE_DGB
}

void launch_diff_fin_batch(const ImgDesc* desc, int nimg, int L, const double* part, int cap,
                           double* G, ImgStat* stat, hipStream_t st) {
    k_diff_fin_batch<<<nimg, 256, 0, st>>>(desc, L, part, cap, G, stat);
}

void launch_ve_solve_batch(const ImgDesc* desc, int nimg, int L, int method, double rank_eps,
                           double gamma_cap, const double* G, VeInfo* info, ImgStat* stat,
                           hipStream_t st) {
    k_ve_solve_batch<<<nimg, 64, 0, st>>>(desc, L, method, rank_eps, gamma_cap, G, info, stat);
}

void launch_ve_combine_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, const float* U,
                             size_t ustride, const VeInfo* info, hipStream_t st) {
    k_ve_combine_batch<<<ntiles, kThreads, 0, st>>>(desc, tiles, U, ustride, info);
}

}  // namespace redve
