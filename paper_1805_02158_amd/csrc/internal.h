// Internal declarations of the redve GPU library: device launchers and shared device helpers.
// gfx950 (CDNA4) only: wave64, FP64 reductions, LDS-tiled stencils.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace redve {

constexpr int kThreads = 256;  // threads per workgroup of every tiled kernel (4 waves)
constexpr int kMaxStages = 16; // denoiser stages
constexpr int kMaxRbfWindow = 16;  // half-width (in centres) of the exact RBF window
constexpr int kRbfPad = kMaxRbfWindow;  // zeros on both sides of each RBF weight row

constexpr int kMaxRedBlocks = 1024;  // workgroups of any kernel that publishes partial sums
constexpr int kMaxPsf = 15;
constexpr int kMaxAc = 17;  // autocorrelation taps of a PSF side of at most 9

// Linear operator H = S B (eq. (1)) and the CG pieces (footnote to eq. (7)). Passed by value:
// the PSF taps live in kernel-argument registers. A rank-1 PSF (both blurs of the paper's
// experiments) is applied as a column pass and a row pass: psf[a][b] = col[a] * row[b].
struct LinOp {
    const float* psf;  // device copy, kh*kw, row-major (general 2-D path)
    const double* psf64;
    int kh, kw, decim;
    int separable;
    float inv_s2;      // 1 / sigma^2
    float lambda;
    double inv_s2_d;   // the same in FP64 (residual accumulation)
    double lambda_d;
    double sd_mu;      // step of the steepest-descent base iteration
    float row[kMaxPsf], col[kMaxPsf];
    double row_d[kMaxPsf], col_d[kMaxPsf];
    // B^T B for a separable square PSF of side <= 9: the separable filter of the
    // autocorrelations of col and row (2 kh - 1 taps each; see set_autocorrelations)
    float acr[kMaxAc], acc[kMaxAc];
    // launch configuration of the CG kernels (0: the built-in rule by image size):
    // cg_pack 1 or 2 CG iterations per launch, cg_threads 256 or 1024 per single-iteration tile,
    // cg_tile 16 (k_cg_iter: r, w, s, p, d in HBM) or 32 (k_cg_iter32: r, p, d only)
    int cg_pack, cg_threads, cg_tile;
};

// acr[j] = sum_b row[b] row[b + j - (kw - 1)], acc likewise from col, j = 0 .. 2 (kw - 1), in
// FP64 rounded once: (B^T B p)(y) = sum_{i,j} acc[i] acr[j] p(y + (i, j) - (kh - 1, kw - 1))
// for B = col (x) row. Zero unless the PSF is separable, square and at most 9 x 9.
inline void set_autocorrelations(LinOp& op) {
    for (int j = 0; j < kMaxAc; ++j) op.acr[j] = op.acc[j] = 0.f;
    if (!op.separable || op.kh != op.kw || 2 * op.kh - 1 > kMaxAc) return;
    const int k = op.kh, r2 = k - 1;
    for (int j = 0; j <= 2 * r2; ++j) {
        double sr = 0.0, sc = 0.0;
        for (int b = 0; b < k; ++b) {
            const int b2 = b + j - r2;
            if (b2 < 0 || b2 >= k) continue;
            sr += op.row_d[b] * op.row_d[b2];
            sc += op.col_d[b] * op.col_d[b2];
        }
        op.acr[j] = (float)sr;
        op.acc[j] = (float)sc;
    }
}

// One image of a batch (batched kernels take a device array of these and a tile list that gives
// each workgroup a 16x16 tile of an image).
struct ImgDesc {
    int H, W;          // image size
    int tile0, ntiles; // this image's range in the batch tile list
    int active;        // 0: every batched kernel skips the image
    int wj;            // window column the difference pass of this FP call writes (-1: none)
    int do_ve;         // 1: this round completes the image's window: extrapolate
    int fp32_banks;    // 1: this image's denoiser stages take FP32 banks (BF16 form, finishing)
    int cg32;          // 1: this image's CG iterations but the last run on the 32x32 tile list
    size_t off;        // element offset of the image in every per-image workspace array
    const float* y;    // observation (caller-owned device memory)
    const float* x_in; // this FP call's input iterate
    float* x_out;      // this FP call's output iterate
    float* x_m;        // window base x_m (extrapolation combines into it)
    LinOp op;
};
constexpr int kBatchTile = 16;  // side of the tiles of the batch tile list

// Entry of the batch tile list: image img, its row-major tile t (of ceil(W/16) per row). The
// host orders the list for dispatch (see the batched engine); per-tile partial sums go to index
// desc[img].tile0 + t, contiguous per image.
struct TileRef {
    int img, t;
};

constexpr int kXcds = 8;  // accelerator dies of the MI355X, each with its own L2
// The tile workgroup b processes, out of n. Workgroups are dispatched round-robin over the
// XCDs (b on XCD b mod 8); XCD x gets the contiguous x-th chunk of the tiles, so tiles that
// share halo rows and columns are fetched through the same L2. A bijection of [0, n).
__device__ inline int xcd_tile(int b, int n) {
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, i = b / kXcds;
    return x * q + (x < r ? x : r) + i;
}

struct VeInfo;

// Per-image results of a batched round, read back by the host.
struct ImgStat {
    double uu, xx;     // ||x_out - x_in||^2, ||x_in||^2 of this FP call
    double gamma_l1;   // sum |gamma| of the extrapolation (0 if none)
    int breakdown;     // 1 if the extrapolation did not exist (or was rejected)
    int guarded;       // 1 if the stability guard rejected it
};
// Per-image CG scalars of the batched single-reduction CG.
struct CgImg {
    double alpha, beta;            // this iteration's step and direction weights
    double alpha_prev, rho_prev;   // the previous iteration's alpha and rho
};

// Batched CG (see linear.hip). Partials are per tile (value v of tile T at part[v * cap + T]).
void launch_cg_init_fp_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs,
                             const float* sres /* null: f = identity */, float* r, hipStream_t st);
// Steepest-descent step of every active image: x_out = x_in + mu (H^T (y - H x_in) / sigma^2
// + lambda s), FP64 sums, mu = op.sd_mu.
void launch_sd_step_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs,
                          const float* sres, hipStream_t st);
void launch_cg_w0_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs,
                        const float* r, float* w, double* part, int cap, hipStream_t st);
void launch_cg_fin_batch(const ImgDesc* desc, int nimg, int k, const double* part, int cap,
                         CgImg* cg, hipStream_t st);
void launch_cg_iter_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int rs, int k,
                          int last, const CgImg* cg, const float* r_in, const float* w_in,
                          const float* s_in, float* r_out, float* w_out, float* s_out, float* p,
                          float* d, double* part, int cap, hipStream_t st);
// Workgroups of kernel `fn` the current device holds at once (a multiple of the XCD count).
int resident_workgroups(const void* fn, int threads, size_t dyn_smem);
// The CG iterations but the last of the images with cg32 set, over the 32x32 tile list (PSF
// padded to 9x9, no decimation): r and p double-buffered, d in place.
void launch_cg_iter32_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int k,
                            const CgImg* cg, const float* r_in, const float* p_in, float* r_out,
                            float* p_out, float* d, double* part, int cap, hipStream_t st);
// Batched VE (see ve.hip).
void launch_diff_gram_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, int L, float* U,
                            size_t ustride, double* part, int cap, hipStream_t st);
void launch_diff_fin_batch(const ImgDesc* desc, int nimg, int L, const double* part, int cap,
                           double* G, ImgStat* stat, hipStream_t st);
void launch_ve_solve_batch(const ImgDesc* desc, int nimg, int L, int method, double rank_eps,
                           double gamma_cap, const double* G, VeInfo* info, ImgStat* stat,
                           hipStream_t st);
void launch_ve_combine_batch(const ImgDesc* desc, const TileRef* tiles, int ntiles, const float* U,
                             size_t ustride, const VeInfo* info, hipStream_t st);

// Denoiser parameters on the device (FP32; BF16 copies of the filters for the MFMA path).
// FP32 MFMA operand fragments per stage (v_mfma_f32_16x16x4_f32, B operand, 64 lanes per
// slice): forward 7 slices of four taps x 2 blocks of 16 filters, adjoint 8 slices of four
// filters x 2 blocks of 16 taps.
constexpr int kFrag32Fwd = 7 * 2 * 64;
constexpr int kFrag32Adj = 8 * 2 * 64;

struct TnrdDev {
    int stages, nfilt, nrbf;
    float mu0, dmu, gamma;
    const float* filters;    // T*F*25
    const float* rbf_w;      // T*F rows of J + 2 kRbfPad: the weights, zero-padded both sides
    float theta[kMaxStages]; // reaction weights theta_t (kernel arguments)
    const uint16_t* frag_fwd;   // per stage: 2 x 64 lanes x 8 BF16 forward-bank MFMA operands
    const uint16_t* frag_adj;   // per stage: 2 x 64 lanes x 8 BF16 adjoint-bank MFMA operands
    const float* frag32_fwd;    // per stage: kFrag32Fwd FP32 forward-bank MFMA operands
    const float* frag32_adj;    // per stage: kFrag32Adj FP32 adjoint-bank MFMA operands
    int precision;
    int kwin;                   // RBF window half-width: centres beyond it add < eps w
                                // (1e-12 for the FP32 form, 1e-6 for BF16)
    // BF16 form, tabulated influence functions (null: evaluated on the window): per stage and
    // filter tab_n intervals of width h, each the cubic (a0, a1, a2, a3) in u in [0, 1) of the
    // Hermite interpolant of phi on [lo + k h, lo + (k + 1) h]; k = floor(t), u = t - k with
    // t = z tab_scale + tab_off = (z - lo) / h.
    const float* phi_tab;
    int tab_n;
    float tab_scale, tab_off;
    // launch configuration of the single-image MFMA stage (0: the built-in rule by image size):
    // stage_threads 512 or 1024 per tile; phi_table 1 tables (BF16, 1024 threads), 2 window
    int stage_threads, phi_table;
};

// Influence-function table of the BF16 form: spacing h = gamma / 2, range the centres widened
// by 5.2565 gamma on both sides (outside it every term is below 1e-6 of its weight).
constexpr double kTabStep = 0.5, kTabReach = 5.2565;
int tnrd_table_intervals(double dmu, double gamma, int J);

// ---- launchers (all asynchronous on `st`) ----------------------------------------------
void launch_apply_H(const LinOp& op, const float* x, int H, int W, float* y, hipStream_t st);
void launch_apply_Ht(const LinOp& op, const float* y, int H, int W, float scale, float* out,
                     hipStream_t st);
void launch_apply_A(const LinOp& op, const float* p, int H, int W, float* out, hipStream_t st);

// CG with reductions split across kernels: every reducing kernel publishes FP64 partials per
// workgroup (grid <= kMaxRedBlocks) and the next kernel re-sums them. `Partials` names a
// published array (value v at p + v * kMaxRedBlocks) and the number of workgroups that wrote it.
struct Partials {
    double* p;
    int n;
};
// CG start for A x = rhs warm-started at x_in (generic right-hand side): r = rhs - A x_in.
void launch_cg_init(const LinOp& op, const float* x_in, const float* rhs, float* r, int H, int W,
                    hipStream_t st);
// CG start of one FP call: r = H^T (y - H x) / sigma^2 + lambda s, s = f(x) - x (may be null).
// out[0] = ||Hx - y||^2, out[1] = x.s (device, FP64); part: 2 x kMaxRedBlocks doubles.
void launch_objective(const LinOp& op, const float* x, const float* y, const float* s, int H,
                      int W, double* part, double* out, hipStream_t st);
// Step of the steepest-descent base iteration (mu > 0: mu; else 1 / (psf_l1^2/sigma^2 + 2 lambda)).
double sd_step(double mu, double psf_l1, double sigma, double lambda);
// x_out = x + op.sd_mu (H^T (y - H x) / sigma^2 + lambda s): one steepest-descent step.
void launch_sd_step(const LinOp& op, const float* x, const float* y, const float* s,
                    float* x_out, int H, int W, hipStream_t st);
// Last CG iteration k of an FP call fused with the difference pass of column j (0..15) of
// vector extrapolation: x_out = x_in + d + alpha p, u = x_out - x_in (stored in U unless null),
// and the partials of u with the j earlier columns, ||u||^2, ||x_in||^2 (j + 2 values at
// part + v kMaxRedBlocks, as launch_diff_gram). Returns the number of partials per value.
int launch_cg_last_diff(int n, int k, const float* r_in, const float* p, const float* d,
                        const float* x_in, float* x_out, Partials rm, const double* hist_prev,
                        float* U, int j, double* part, hipStream_t st);
void launch_cg_init_fp(const LinOp& op, const float* x, const float* y, const float* s, float* r,
                       int H, int W, hipStream_t st);
// w0 = A r0; publishes r0.r0 and w0.r0.
Partials launch_cg_w0(const LinOp& op, const float* r, float* w, int H, int W, double* part,
                      hipStream_t st);
// Two CG iterations per kernel for an undecimated, separable, square PSF of side 7 or 9 (see
// linear.hip): cg_block_ok says whether they apply to iters iterations on an H x W image.
// The block start writes w_0 = A r_0, a_0 = A w_0 and publishes nine Gram sums of
// [r, w, s, a, b] (entry 0 rho, entry 1 mu, so a single iteration can follow); a block takes
// iterations k and k + 1.
constexpr int kCgSums = 16;  // partial arrays per CG slot
bool cg_block_ok(const LinOp& op, int iters, int H, int W);
Partials launch_cg_w0_block(const LinOp& op, const float* r, float* w, float* a, int H, int W,
                            double* part, hipStream_t st);
Partials launch_cg_block(const LinOp& op, int H, int W, int k, const float* const* vin,
                         float* const* vout, float* p, float* d, Partials rm,
                         const double* hist_prev, double* hist_cur, double* part,
                         hipStream_t st);
// One single-reduction CG iteration k (see linear.hip); hist_prev holds (alpha, rho) of
// iteration k-1, hist_cur receives those of iteration k. The last iteration writes
// x_out = x_in + d only.
// One CG iteration (not the last) on 32x32 tiles keeping only r, p and d in HBM: reads r_in and
// p_in (p_{k-1}) on halos, writes r_out, p_out (p_k) and d in place; separable square 7x7 or
// 9x9 PSF without decimation. cg_iter32_ok: whether the FP call takes it (the rule: images of
// 512 or more 16x16 tiles; or the tuned cg_tile).
bool cg_iter32_ok(const LinOp& op, int iters, int H, int W);
Partials launch_cg_iter32(const LinOp& op, int H, int W, int k, const float* r_in,
                          const float* p_in, float* r_out, float* p_out, float* d, Partials rm,
                          const double* hist_prev, double* hist_cur, double* part,
                          hipStream_t st);
Partials launch_cg_iter(const LinOp& op, int H, int W, int k, int last, const float* r_in,
                        const float* w_in, const float* s_in, float* r_out, float* w_out,
                        float* s_out, float* p, float* d, const float* x_in, float* x_out,
                        Partials rm, const double* hist_prev, double* hist_cur, double* part,
                        hipStream_t st);

int tnrd_grid(int H, int W);
size_t tnrd_smem_bytes(int F, int J);
// Batched stage over the tile list; vectors are base pointers of per-image arrays.
// f is each image's x_in (from its descriptor).
void launch_tnrd_stage_batch(const TnrdDev& d, int t, const ImgDesc* desc, const TileRef* tiles,
                             int ntiles, const float* w_prev, float* out, int out_mode,
                             hipStream_t st);
void launch_tnrd_stage_bf16_batch(const TnrdDev& d, int t, const ImgDesc* desc,
                                  const TileRef* tiles, int ntiles, const float* w_prev, float* out,
                                  int out_mode, hipStream_t st);
// The BF16 form with a per-image switch to FP32 banks (ImgDesc::fp32_banks): one launch, each
// tile's workgroup takes its image's form (db: the BF16 denoiser, df: the same denoiser with
// FP32 banks and its window).
void launch_tnrd_stage_mixed_batch(const TnrdDev& db, const TnrdDev& df, int t,
                                   const ImgDesc* desc, const TileRef* tiles, int ntiles,
                                   const float* w_prev, float* out, int out_mode, hipStream_t st);
// The CG start an FP call's last denoiser stage can form as it finishes (single image, the
// two-iteration CG path): r = H^T (y - H x) / sigma^2 + lambda s with s the stage's output and
// x its input f, into r; rs the PSF radius (3 or 4, separable, no decimation).
struct ResidualReq {
    LinOp op;
    const float* y;
    float* r;
    int rs;
};
// Whether the stage kernels form it for this denoiser (MFMA stage, BF16 tables or the FP32
// K = 7 window).
bool tnrd_fuses_residual(const TnrdDev& d);
// Mixed-precision stage (BF16 filter banks on MFMA, FP32 influence functions and update).
// Returns whether the launch also formed the CG start of rq (the kernels with 1024 threads and
// tabulated phi, or the FP32 K = 7 window, take it; otherwise the caller must form it).
bool launch_tnrd_stage_bf16(const TnrdDev& d, int t, const float* w_prev, const float* f,
                            float* out, int H, int W, int out_mode, hipStream_t st,
                            const ResidualReq* rq = nullptr);
// LDS of one MFMA stage tile (either form) with the influence functions evaluated on the
// window, and whether it fits in 64 KiB (the FP32 form takes the vector-ALU stage beyond; the
// BF16 form runs up to the device's per-workgroup limit); LDS of a BF16 tile with tabulated
// influence functions (tab_n intervals per filter), used where it fits that limit.
size_t tnrd_mfma_smem_bytes(int F, int J);
bool tnrd_mfma_fits(int F, int J);
size_t tnrd_table_smem_bytes(int F, int tab_n);
// The FP32 form's stage on the vector ALUs (tnrd.hip), for denoisers whose MFMA tile does not
// fit; launch_tnrd_stage / launch_tnrd_stage_batch choose between the two.
void launch_tnrd_stage_valu(const TnrdDev& d, int t, const float* w_prev, const float* f,
                            float* out, int H, int W, int out_mode, hipStream_t st);
void launch_tnrd_stage_valu_batch(const TnrdDev& d, int t, const ImgDesc* desc,
                                  const TileRef* tiles, int ntiles, const float* w_prev,
                                  float* out, int out_mode, hipStream_t st);
// One denoiser stage in residual form: w_t = w_{t-1} - sum_i K_i^T phi_i(K_i (f + w_{t-1}))
// - theta_t w_{t-1}, with w = u - f (w_prev null: w_0 = 0). out_mode 0 writes w_t, 1 writes
// f + w_t (= u_t). Returns whether the CG start of rq was formed (as launch_tnrd_stage_bf16).
bool launch_tnrd_stage(const TnrdDev& d, int t, const float* w_prev, const float* f, float* out,
                       int H, int W, int out_mode, hipStream_t st,
                       const ResidualReq* rq = nullptr);
// The stage configuration the built-in rule picks for an H x W image: threads per tile (512 or
// 1024) and whether phi is tabulated.
int tnrd_rule_threads(int H, int W);
// The CG configuration the built-in rule picks: iterations per launch and single-iteration
// threads per tile.
int cg_rule_pack(const LinOp& op, int iters, int H, int W);
int cg_rule_threads(const LinOp& op, int H, int W);

// Differences, Gram row and norms of two consecutive iterates, as published partials:
//   u = x_new - x_old (stored in U + j*n when U != nullptr),
//   values k < j: u . U_k;  value j: u . u;  value j+1: x_old . x_old.
// Writes (j + 2) arrays of kMaxRedBlocks partials at part; returns the workgroup count.
int launch_diff_gram(const float* x_new, const float* x_old, float* U, int j, int n, double* part,
                     hipStream_t st);
// Result of the small FP64 solve on the L x L Gram matrix.
struct VeInfo {
    double xi[32];
    double gamma[32];
    double gamma_l1;
    double uu, xx;   // ||u_last||^2, ||x_prev||^2 of the last difference (relative change)
    int ncols;       // columns of U combined (kappa, or L on breakdown)
    int breakdown;   // 1 if the extrapolation did not exist, or the stability guard rejected it
    int kappa_used;  // kappa after any RRE column drops
    int guarded;     // 1 if the stability guard rejected the coefficients (gamma, gamma_l1 kept)
};
// Sums the partials of the L difference passes (column j's at part + j * win_stride, each
// written by nblk workgroups) into G, then Cholesky / MPE / RRE / SVD-MPE; coefficients with
// sum |gamma| above gamma_cap (or not finite) are rejected when gamma_cap > 0.
void launch_ve_solve(const double* part, size_t win_stride, int nblk, int L, int method,
                     double rank_eps, double gamma_cap, VeInfo* info, hipStream_t st);
// Sums the partials of a single difference pass (j = 0) into info->uu, info->xx.
void launch_delta(const double* part, int nblk, VeInfo* info, hipStream_t st);
void launch_ve_combine(const float* x_m, const float* U, int n, const VeInfo* info, float* out,
                       hipStream_t st);

}  // namespace redve
