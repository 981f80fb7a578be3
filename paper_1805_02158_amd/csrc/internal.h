// Internal declarations of the redve GPU library: device launchers and shared device helpers.
// gfx950 (CDNA4) only: wave64, FP64 reductions, LDS-tiled stencils.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace redve {

constexpr int kThreads = 256;  // threads per workgroup of every tiled kernel (4 waves)
constexpr int kMaxStages = 16; // denoiser stages

// Scalars of one CG solve, device resident. Read by every workgroup of the next kernel;
// written by the last workgroup of the kernel that finishes the corresponding reduction.
struct CgScalars {
    double rho0;   // r.r of the current residual
    double pq;     // p.(A p)
    double alpha;  // step length
    double beta;   // direction update weight
};

// Grid-wide deterministic reduction: per-workgroup FP64 partials plus a completion counter.
// The last workgroup to finish sums the partials in workgroup order and resets the counter.
struct Reduction {
    double* partials;   // nvals * capacity doubles
    unsigned* counter;  // one counter, zero between kernels
    int capacity;       // max workgroups
};

// Linear operator H = S B (eq. (1)) and the CG pieces (footnote to eq. (7)).
struct LinOp {
    const float* psf;  // device copy, kh*kw, row-major
    int kh, kw, decim;
    float inv_s2;      // 1 / sigma^2
    float lambda;
    double inv_s2_d;   // the same in FP64 (residual accumulation)
    double lambda_d;
};

// Denoiser parameters on the device (FP32; BF16 copies of the filters for the MFMA path).
struct TnrdDev {
    int stages, nfilt, nrbf;
    float mu0, dmu, gamma;
    const float* filters;    // T*F*25
    const float* rbf_w;      // T*F*J
    float theta[kMaxStages]; // reaction weights theta_t (kernel arguments)
    const uint16_t* filt_bf16;  // T*F*25 bf16 bits
    int precision;
};

// ---- launchers (all asynchronous on `st`) ----------------------------------------------
void launch_apply_H(const LinOp& op, const float* x, int H, int W, float* y, hipStream_t st);
void launch_apply_Ht(const LinOp& op, const float* y, int H, int W, float scale, float* out,
                     hipStream_t st);
void launch_apply_A(const LinOp& op, const float* p, int H, int W, float* out, hipStream_t st);
int linop_grid(int H, int W);  // workgroups of the tiled CG kernels
// CG on A x = rhs warm-started at x_in (generic right-hand side).
void launch_cg_init(const LinOp& op, const float* x_in, const float* rhs, float* r, float* p,
                    int H, int W, Reduction red, CgScalars* sc, hipStream_t st);
// CG start of one FP call: r = H^T (y - H x) / sigma^2 + lambda s, s = f(x) - x (may be null).
void launch_cg_init_fp(const LinOp& op, const double* psf64, const float* x, const float* y,
                       const float* s, float* r, float* p, int H, int W, Reduction red,
                       CgScalars* sc, hipStream_t st);
void launch_cg_q(const LinOp& op, const float* r, const float* p_old, float* p_new, float* q,
                 int H, int W, Reduction red, CgScalars* sc, hipStream_t st);
// d (+)= alpha p, r -= alpha q; with x_out != null: x_out = x_in + d instead of storing d.
void launch_cg_update(float* d, float* r, const float* p, const float* q, int n, int first,
                      const float* x_in, float* x_out, Reduction red, CgScalars* sc,
                      hipStream_t st);
int cg_update_grid(int n);
void launch_axpb(const float* b0, const float* u, float lambda, float* out, int n,
                 hipStream_t st);

int tnrd_grid(int H, int W);
// One denoiser stage in residual form: w_t = w_{t-1} - sum_i K_i^T phi_i(K_i (f + w_{t-1}))
// - theta_t w_{t-1}, with w = u - f (w_prev null: w_0 = 0). out_mode 0 writes w_t, 1 writes
// f + w_t (= u_t).
void launch_tnrd_stage(const TnrdDev& d, int t, const float* w_prev, const float* f, float* out,
                       int H, int W, int out_mode, hipStream_t st);

// Differences, Gram row and norms of two consecutive iterates.
//   u = x_new - x_old (stored in U + j*n when U != nullptr),
//   G[j][i] = G[i][j] = u . U_i for i < j, G[j][j] = u . u,
//   norms[0] = ||u||^2, norms[1] = ||x_old||^2.
int diff_grid(int n);
void launch_diff_gram(const float* x_new, const float* x_old, float* U, int j, int ldG, int n,
                      double* G, double* norms, Reduction red, hipStream_t st);
// Small FP64 solve on the L x L Gram matrix: gamma, xi, number of columns to combine, info.
struct VeInfo {
    double xi[32];
    double gamma[32];
    double gamma_l1;
    int ncols;       // columns of U combined (kappa, or L on breakdown)
    int breakdown;   // 1 if the extrapolation did not exist
    int kappa_used;  // kappa after any RRE column drops
    int pad;
};
void launch_ve_solve(const double* G, int ldG, int L, int method, double rank_eps, VeInfo* info,
                     hipStream_t st);
void launch_ve_combine(const float* x_m, const float* U, int n, const VeInfo* info, float* out,
                       hipStream_t st);

}  // namespace redve
