// Private definition of the library handle (shared by the single-image runtime and the
// batched / serving engine).
#pragma once

#include <math.h>

#include <string>
#include <vector>

#include "../../include/redve.h"
#include "internal.h"

namespace redve_detail {

using redve::VeInfo;
constexpr size_t kAlign = 256;

struct Workspace {
    void* arena = nullptr;
    size_t bytes = 0;
    size_t cap_px = 0;
    int cap_L = 0;
    float *xa, *xb, *xc, *sres, *u0, *u1, *r[2], *w[2], *s[2], *p, *d, *U;
    float *a[2], *b[2];  // A w and A s of the two-iteration CG kernels
    float* yw;        // the solve's copy of the observation (captured passes read it)
    double* cg_part;  // two slots of published CG partials, kCgSums arrays each
    double* cg_hist;  // two slots of (alpha, rho) of the previous CG iteration
    double* ve_part;  // window partials: column j at j * win_stride
    size_t win_stride;
    VeInfo* info;
};

// A captured pass of the single-image solve loop (a full extrapolation cycle, or one FP call
// with its relative-change pass), replayed while everything it recorded is unchanged: the
// start vector, the image size, the workspace, the settings generations, m and the SD step.
struct PassGraph {
    hipGraphExec_t exec = nullptr;
    const float* from = nullptr;
    float* next = nullptr;  // where the pass leaves its iterate
    int hx = 0, wx = 0, m = 0;
    double sd_mu = 0.0;
    unsigned long long gen = 0, op_gen = 0;
    const void* arena = nullptr;
    redve_tuning_t tune{};  // the launch configuration it recorded
    bool finish_fp32 = false;  // the filter banks it recorded (BF16 form: FP32 finishing)
};
constexpr int kPassGraphs = 4;

// A tuned launch configuration and the problem it was measured on.
struct TuneEntry {
    int key[13];  // hx, wx, precision, T, F, J, kh, kw, decim, separable, cg_iters, base, linear
    redve_tuning_t cfg;
    double us;    // FP-call time measured for cfg
};

struct HostMirror {
    VeInfo info;
    double obj[2];  // ||Hx - y||^2, x.(f(x) - x)
};

}  // namespace redve_detail

using redve_detail::kAlign;
using redve_detail::Workspace;
using redve_detail::HostMirror;
using redve_detail::PassGraph;
using redve_detail::kPassGraphs;
using redve_detail::TuneEntry;

struct redve_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int lds_max = 64 * 1024;  // LDS one workgroup may use on this device (queried)
    hipStream_t bstream = nullptr;  // the batched engine's own stream (created on first use)
    std::string err;
    // operator H = S B
    bool have_op = false;
    std::vector<float> psf;
    int kh = 0, kw = 0, decim = 1;
    float* d_psf = nullptr;
    double* d_psf64 = nullptr;
    int separable = 0;
    double row[REDVE_MAX_PSF], col[REDVE_MAX_PSF];  // psf = col (x) row when separable
    // sigma, lambda
    double sigma = -1.0, lambda = -1.0;
    // denoiser
    bool have_den = false;
    int T = 0, F = 0, J = 0, precision = REDVE_PREC_FP32, kwin = 7;
    int kwin32 = 7;            // the window of the FP32 banks (the BF16 form's finishing calls)
    double prec_switch = 0.0;  // BF16 form: FP32 banks once the relative change is below this
    bool finish_fp32 = false;  // the current solve has switched (single image)
    double mu0 = 0, dmu = 0, gamma = 1;
    std::vector<float> theta;
    float* d_filt = nullptr;
    float* d_rbfw = nullptr;
    uint16_t* d_frag = nullptr;  // BF16 MFMA operand fragments: forward then adjoint, per stage
    float* d_frag32 = nullptr;   // FP32 MFMA operand fragments: forward then adjoint, per stage
    float* d_phitab = nullptr;   // BF16 form: influence-function tables per stage (or null)
    int tab_n = 0;
    double tab_lo = 0, tab_h = 1;
    // solver
    int method = REDVE_VE_NONE, L = 5, m = 0;
    int cg_iters = 15, max_fp = 500, extra_fp = 0;
    double tol = 1e-5;
    int base = REDVE_BASE_FP;  // base iteration of Algorithm 3
    double sd_mu = 0.0;        // steepest-descent step (<= 0: 1 / (||H||^2/sigma^2 + 2 lambda))
    double psf_l1 = 1.0;       // sum |h|, a bound on ||H||
    double rank_eps = 1e-7;  // R_jj <= rank_eps * R_00 counts as rank deficient (FP32 data)
    double gamma_cap = INFINITY;  // stability guard on sum |gamma| (<= 0: off)
    Workspace ws;
    HostMirror* host = nullptr;  // pinned
    // Settings generation: bumped by every setter that changes what a captured batched round
    // records (denoiser buffers and stages, precision, extrapolation method and window, CG
    // iterations). The batched engine kept between redve_solve_batch calls is rebuilt when it
    // was made for another generation.
    unsigned long long gen = 0;
    void* batch = nullptr;                 // the kept batched engine (batch.hip)
    void (*batch_free)(void*) = nullptr;   // its destructor
    // linear step of the FP call
    int lin = REDVE_LIN_CG;
    unsigned long long op_gen = 0;         // bumped by set_operator / set_noise / set_lambda
    void* fft = nullptr;                   // Fourier solve plans and tables (fft.hip)
    void (*fft_free)(void*) = nullptr;
    // captured passes of redve_solve, their capture stream, and whether capture failed once
    PassGraph pass[kPassGraphs];
    int pass_next = 0;
    hipStream_t gstream = nullptr;
    bool graphs_off = false;
    // launch configuration of the single-image kernels: cur is applied to the launches (zero
    // fields: the built-in rule); forced (set by redve_set_tuning) wins over the mode; in
    // REDVE_TUNE_AUTO the first solve or FP step of a problem times the candidates and caches
    // the fastest in tune_cache (and in the JSON lines file tune_path, if set)
    redve_tuning_t cur{};
    redve_tuning_t forced{};
    bool have_forced = false;
    int tune_mode = REDVE_TUNE_RULES;
    std::vector<TuneEntry> tune_cache;
    std::string tune_path;
};

// Whether the Fourier linear step supports an hx x wx image (fft.hip).
bool redve_fft_size_ok(int H, int W);
// d = F^-1[F(r0) / A_hat], x_out = x_in + d for periodic deblurring (fft.hip).
int redve_fft_correction(redve_t h, float* r0, const float* x_in, float* x_out, float* d, int H,
                         int W);

// Resolves the no-allocation scratch array on `device` (current) once (noalloc.hip).
int redve_noalloc_resolve(int device);

// Device view of the handle's denoiser (runtime.hip).
redve::TnrdDev redve_tnrd_dev(redve_t h);

