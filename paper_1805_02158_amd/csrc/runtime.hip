// Host runtime of the redve library: handle, parameter validation, device workspace, and the
// driver of the FP iteration (Sec. II-B, eq. (7)) with full-cycling vector extrapolation
// (Sec. III-C, Algorithm 3). Every arithmetic step runs in the HIP kernels; the host only
// orders launches and reads back a few scalars (relative change, extrapolation info).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "../../include/redve.h"
#include "internal.h"

using namespace redve;

#include "context.h"

namespace {

int fail(redve_t h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIP_TRY(h, expr)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(h, REDVE_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK(h) HIP_TRY(h, hipGetLastError())

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of the workspace arena for cap_px pixels and a window of cap_L.
struct Layout {
    static constexpr int kVecs = 19;
    size_t vec, win_stride, o_cg, o_hist, o_ve, o_info, bytes;
    Layout(size_t cap_px, int cap_L) {
        vec = align_up(cap_px * sizeof(float));
        win_stride = (size_t)(cap_L + 1) * kMaxRedBlocks;
        bytes = vec * (kVecs + (size_t)cap_L);
        o_cg = bytes;
        bytes += align_up(2 * kCgSums * kMaxRedBlocks * sizeof(double));
        o_hist = bytes;
        bytes += kAlign;
        o_ve = bytes;
        bytes += align_up((size_t)cap_L * win_stride * sizeof(double));
        o_info = bytes;
        bytes += align_up(sizeof(VeInfo));
    }
};

int ensure_workspace(redve_t h, int hx, int wx, int L) {
    const size_t npx = (size_t)hx * wx;
    Workspace& w = h->ws;
    if (w.arena && w.cap_px >= npx && w.cap_L >= L) return REDVE_OK;
    if (w.arena) {
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        HIP_TRY(h, hipFree(w.arena));
        w.arena = nullptr;
    }
    const size_t cap_px = std::max(npx, w.cap_px);
    const int cap_L = std::max(std::max(L, w.cap_L), 1);
    const Layout lay(cap_px, cap_L);
    void* arena = nullptr;
    if (hipMalloc(&arena, lay.bytes) != hipSuccess)
        return fail(h, REDVE_E_NOMEM, "device workspace allocation of " +
                                          std::to_string(lay.bytes) + " bytes failed");
    char* base = (char*)arena;
    float** vecs[Layout::kVecs] = {&w.xa,   &w.xb,   &w.xc,   &w.sres, &w.u0,   &w.u1,   &w.r[0],
                                   &w.r[1], &w.w[0], &w.w[1], &w.s[0], &w.s[1], &w.p,    &w.d,
                                   &w.yw,   &w.a[0], &w.a[1], &w.b[0], &w.b[1]};
    for (int i = 0; i < Layout::kVecs; ++i) *vecs[i] = (float*)(base + lay.vec * i);
    w.U = (float*)(base + lay.vec * Layout::kVecs);
    w.cg_part = (double*)(base + lay.o_cg);
    w.cg_hist = (double*)(base + lay.o_hist);
    w.ve_part = (double*)(base + lay.o_ve);
    w.win_stride = lay.win_stride;
    w.info = (VeInfo*)(base + lay.o_info);
    w.arena = arena;
    w.bytes = lay.bytes;
    w.cap_px = cap_px;
    w.cap_L = cap_L;
    return REDVE_OK;
}

}  // namespace

// Step of the steepest-descent base iteration: mu if mu > 0, else 1 / L with
// L = ||H||^2 / sigma^2 + 2 lambda (gradient Lipschitz bound for a strongly passive denoiser,
// Sec. II-B), ||H|| <= psf_l1 = sum |h|.
double redve::sd_step(double mu, double psf_l1, double sigma, double lambda) {
    if (mu > 0) return mu;
    return 1.0 / (psf_l1 * psf_l1 / (sigma * sigma) + 2.0 * lambda);
}

namespace {

LinOp linop_of(redve_t h) {
    const double is2 = 1.0 / (h->sigma * h->sigma);
    LinOp op{};
    op.psf = h->d_psf;
    op.psf64 = h->d_psf64;
    op.kh = h->kh;
    op.kw = h->kw;
    op.decim = h->decim;
    op.separable = h->separable;
    op.inv_s2 = (float)is2;
    op.lambda = (float)h->lambda;
    op.inv_s2_d = is2;
    op.lambda_d = h->lambda;
    op.sd_mu = sd_step(h->sd_mu, h->psf_l1, h->sigma, h->lambda);
    for (int i = 0; i < h->kh; ++i) {
        op.col_d[i] = h->col[i];
        op.col[i] = (float)h->col[i];
    }
    for (int j = 0; j < h->kw; ++j) {
        op.row_d[j] = h->row[j];
        op.row[j] = (float)h->row[j];
    }
    set_autocorrelations(op);
    op.cg_pack = h->cur.cg_per_launch;
    op.cg_threads = h->cur.cg_threads;
    op.cg_tile = h->cur.cg_tile;
    return op;
}

}  // namespace

TnrdDev redve_tnrd_dev(redve_t h) {
    TnrdDev d{};
    d.stages = h->T;
    d.nfilt = h->F;
    d.nrbf = h->J;
    d.mu0 = (float)h->mu0;
    d.dmu = (float)h->dmu;
    d.gamma = (float)h->gamma;
    d.filters = h->d_filt;
    d.rbf_w = h->d_rbfw;
    for (int t = 0; t < h->T && t < kMaxStages; ++t) d.theta[t] = h->theta[t];
    d.frag_fwd = h->d_frag;
    d.frag_adj = h->d_frag ? h->d_frag + (size_t)h->T * 2 * 64 * 8 : nullptr;
    d.frag32_fwd = h->d_frag32;
    d.frag32_adj = h->d_frag32 ? h->d_frag32 + (size_t)h->T * kFrag32Fwd : nullptr;
    d.precision = h->precision;
    d.kwin = h->kwin;
    d.phi_tab = h->d_phitab;
    d.tab_n = h->d_phitab ? h->tab_n : 0;
    d.tab_scale = (float)(1.0 / h->tab_h);
    d.tab_off = (float)(-h->tab_lo / h->tab_h);
    return d;
}

namespace {

// The handle's denoiser with the single-image launch configuration; in the BF16 form's
// finishing FP calls, the same denoiser with FP32 banks and the FP32 window.
TnrdDev tnrd_of(redve_t h) {
    TnrdDev d = redve_tnrd_dev(h);
    d.stage_threads = h->cur.stage_threads;
    d.phi_table = h->cur.phi_table;
    if (h->finish_fp32 && d.precision == REDVE_PREC_BF16) {
        d.precision = REDVE_PREC_FP32;
        d.kwin = h->kwin32;
        d.phi_tab = nullptr;
        d.tab_n = 0;
    }
    return d;
}

int check_ready(redve_t h, bool need_den) {
    if (!h->have_op) return fail(h, REDVE_E_STATE, "redve_set_operator was not called");
    if (h->sigma <= 0) return fail(h, REDVE_E_STATE, "redve_set_noise was not called");
    if (h->lambda <= 0) return fail(h, REDVE_E_STATE, "redve_set_lambda was not called");
    if (need_den && !h->have_den) return fail(h, REDVE_E_STATE, "redve_set_denoiser was not called");
    return REDVE_OK;
}

// The Fourier linear step diagonalises A only for H = B (decim 1, Sec. II-B footnote).
int check_linear(redve_t h) {
    if (h->lin == REDVE_LIN_FFT && h->base == REDVE_BASE_FP && h->decim != 1)
        return fail(h, REDVE_E_ARG, "the Fourier linear step needs decim = 1 (deblurring)");
    return REDVE_OK;
}

int check_image(redve_t h, int hx, int wx) {
    if (hx < 2 || wx < 2) return fail(h, REDVE_E_ARG, "image sides must be >= 2");
    if ((long long)hx * wx > (1LL << 30)) return fail(h, REDVE_E_ARG, "image too large");
    return REDVE_OK;
}

// The Fourier linear step's transforms hold a row or a block of columns in LDS.
int check_fft_size(redve_t h, int hx, int wx) {
    if (h->lin == REDVE_LIN_FFT && h->base == REDVE_BASE_FP && !redve_fft_size_ok(hx, wx))
        return fail(h, REDVE_E_ARG, "the Fourier linear step supports sides up to 4096");
    return REDVE_OK;
}

// Denoiser f. residual = true writes f(x) - x (nothing, and *out_null = true, for T = 0);
// otherwise f(x). With rq, *rq_done tells whether the last stage also formed the CG start.
int run_denoiser(redve_t h, const float* x, int H, int W, float* out, bool residual,
                 bool* out_null, const ResidualReq* rq = nullptr, bool* rq_done = nullptr) {
    Workspace& w = h->ws;
    const int n = H * W;
    TnrdDev d = tnrd_of(h);
    if (out_null) *out_null = false;
    if (rq_done) *rq_done = false;
    if (h->T == 0) {
        if (residual) {
            if (out_null) *out_null = true;
        } else {
            HIP_TRY(h, hipMemcpyAsync(out, x, sizeof(float) * n, hipMemcpyDeviceToDevice, h->stream));
        }
        return REDVE_OK;
    }
    const float* wprev = nullptr;
    for (int t = 0; t < h->T; ++t) {
        const bool last = t == h->T - 1;
        float* dst = last ? out : ((t & 1) ? w.u1 : w.u0);
        const int mode = (last && !residual) ? 1 : 0;
        const ResidualReq* q = last ? rq : nullptr;
        const bool done = d.precision == REDVE_PREC_BF16
                              ? launch_tnrd_stage_bf16(d, t, wprev, x, dst, H, W, mode, h->stream, q)
                              : launch_tnrd_stage(d, t, wprev, x, dst, H, W, mode, h->stream, q);
        if (q && rq_done) *rq_done = done;
        LAUNCH_CHECK(h);
        wprev = dst;
    }
    return REDVE_OK;
}

// The difference pass of vector extrapolation to fuse into the last CG iteration of an FP call:
// column j of U (U null: the relative change only), partials at part; nblk is set when fused.
struct DiffReq {
    float* U;
    int j;
    double* part;
    int nblk;
};

// CG iterations in single-reduction form on the correction d (A d = r0 from d = 0), r0 in
// ws.r[0]; the last iteration writes x_out = x_in + d.
int cg_iterate(redve_t h, const float* x_in, float* x_out, int H, int W, int iters,
               DiffReq* dq = nullptr) {
    Workspace& w = h->ws;
    LinOp op = linop_of(h);
    double* slot[2] = {w.cg_part, w.cg_part + kCgSums * kMaxRedBlocks};
    Partials rm;
    int k = 0, a = 0;
    if (cg_block_ok(op, iters, H, W)) {
        // two iterations per kernel while at least one iteration remains after the pair
        rm = launch_cg_w0_block(op, w.r[0], w.w[0], w.a[0], H, W, slot[0], h->stream);
        LAUNCH_CHECK(h);
        for (; k + 2 <= iters - 1; k += 2) {
            const int b = a ^ 1;
            const float* vin[5] = {w.r[a], w.w[a], w.s[a], w.a[a], w.b[a]};
            float* vout[5] = {w.r[b], w.w[b], w.s[b], w.a[b], w.b[b]};
            rm = launch_cg_block(op, H, W, k, vin, vout, w.p, w.d, rm, w.cg_hist + 2 * a,
                                 w.cg_hist + 2 * b, slot[b], h->stream);
            LAUNCH_CHECK(h);
            a = b;
        }
    } else if (cg_iter32_ok(op, iters, H, W)) {
        // 32x32 tiles keeping only r, p, d: p double-buffered in the s buffers, which this
        // form does not otherwise use; the last iteration below reads p_{n-2} from pb[a]
        rm = launch_cg_w0(op, w.r[0], w.w[0], H, W, slot[0], h->stream);
        LAUNCH_CHECK(h);
        float* pb[2] = {w.s[0], w.s[1]};
        for (; k < iters - 1; ++k) {
            const int b = a ^ 1;
            rm = launch_cg_iter32(op, H, W, k, w.r[a], pb[a], w.r[b], pb[b], w.d, rm,
                                  w.cg_hist + 2 * a, w.cg_hist + 2 * b, slot[b], h->stream);
            LAUNCH_CHECK(h);
            a = b;
        }
        if (dq) {
            dq->nblk = launch_cg_last_diff(H * W, k, w.r[a], pb[a], w.d, x_in, x_out, rm,
                                           w.cg_hist + 2 * a, dq->U, dq->j, dq->part, h->stream);
        } else {
            launch_cg_iter(op, H, W, k, 1, w.r[a], w.w[a], w.s[a], w.r[a ^ 1], w.w[a ^ 1],
                           w.s[a ^ 1], pb[a], w.d, x_in, x_out, rm, w.cg_hist + 2 * a,
                           w.cg_hist + 2 * (a ^ 1), slot[a ^ 1], h->stream);
        }
        LAUNCH_CHECK(h);
        return REDVE_OK;
    } else {
        rm = launch_cg_w0(op, w.r[0], w.w[0], H, W, slot[0], h->stream);
        LAUNCH_CHECK(h);
    }
    // single iterations (the last writes x_out = x_in + d); the vectors of iteration k are in
    // buffer set a, the previous step lengths in hist slot a
    for (; k < iters; ++k) {
        const int b = a ^ 1;
        if (dq && k == iters - 1) {  // the last iteration with the difference pass
            dq->nblk = launch_cg_last_diff(H * W, k, w.r[a], w.p, w.d, x_in, x_out, rm,
                                           w.cg_hist + 2 * a, dq->U, dq->j, dq->part, h->stream);
            LAUNCH_CHECK(h);
            break;
        }
        rm = launch_cg_iter(op, H, W, k, k == iters - 1, w.r[a], w.w[a], w.s[a], w.r[b], w.w[b],
                            w.s[b], w.p, w.d, x_in, x_out, rm, w.cg_hist + 2 * a,
                            w.cg_hist + 2 * b, slot[b], h->stream);
        LAUNCH_CHECK(h);
        a = b;
    }
    return REDVE_OK;
}

// iters CG iterations on A x = rhs: x_out starts at x_in (x_in != x_out).
int run_cg(redve_t h, const float* rhs, const float* x_in, float* x_out, int H, int W, int iters) {
    Workspace& w = h->ws;
    const int n = H * W;
    if (iters <= 0) {
        HIP_TRY(h, hipMemcpyAsync(x_out, x_in, sizeof(float) * n, hipMemcpyDeviceToDevice, h->stream));
        return REDVE_OK;
    }
    launch_cg_init(linop_of(h), x_in, rhs, w.r[0], H, W, h->stream);
    LAUNCH_CHECK(h);
    return cg_iterate(h, x_in, x_out, H, W, iters);
}

// One FP call, eq. (7): x_out = CG_{n_cg}(A, H^T y / sigma^2 + lambda f(x_in); start x_in),
// computed as x_in + d with d the CG solution of A d = r0 from d = 0 (the same Krylov iterates),
// r0 = H^T (y - H x_in) / sigma^2 + lambda (f(x_in) - x_in).
int fp_call(redve_t h, const float* y, const float* x_in, float* x_out, int H, int W,
            DiffReq* dq = nullptr) {
    Workspace& w = h->ws;
    const int n = H * W;
    bool s_null = false;
    // on the two-iteration CG path the last denoiser stage can also form the CG start r_0;
    // the stage reports whether it did, and the start kernel runs otherwise
    const LinOp op = linop_of(h);
    const bool fuse = h->base == REDVE_BASE_FP && h->lin == REDVE_LIN_CG && h->cg_iters > 0 &&
                      h->T > 0 && h->cur.fused_start != 2 &&
                      cg_block_ok(op, h->cg_iters, H, W) && tnrd_fuses_residual(tnrd_of(h));
    const ResidualReq rq{op, y, w.r[0], op.kh / 2};
    bool started = false;
    int rc = run_denoiser(h, x_in, H, W, w.sres, true, &s_null, fuse ? &rq : nullptr, &started);
    if (rc) return rc;
    if (h->base == REDVE_BASE_SD) {  // x - mu g(x): the same residual, no linear solve
        launch_sd_step(linop_of(h), x_in, y, s_null ? nullptr : w.sres, x_out, H, W, h->stream);
        LAUNCH_CHECK(h);
        return REDVE_OK;
    }
    if (h->lin == REDVE_LIN_FFT) {  // the exact solve of A d = r0 in the Fourier domain
        launch_cg_init_fp(linop_of(h), x_in, y, s_null ? nullptr : w.sres, w.r[0], H, W, h->stream);
        LAUNCH_CHECK(h);
        if ((rc = redve_fft_correction(h, w.r[0], x_in, x_out, w.d, H, W)))
            return fail(h, rc, "Fourier linear step failed");
        return REDVE_OK;
    }
    if (h->cg_iters <= 0) {
        HIP_TRY(h, hipMemcpyAsync(x_out, x_in, sizeof(float) * n, hipMemcpyDeviceToDevice, h->stream));
        return REDVE_OK;
    }
    if (!started) {
        launch_cg_init_fp(op, x_in, y, s_null ? nullptr : w.sres, w.r[0], H, W, h->stream);
        LAUNCH_CHECK(h);
    }
    return cg_iterate(h, x_in, x_out, H, W, h->cg_iters, dq);
}

// One FP call and the difference pass of column j (U null: relative change only), fused into
// its last CG iteration where it ends with one; returns the number of partials.
int fp_call_diff(redve_t h, const float* y, const float* x_in, float* x_out, int H, int W,
                 float* U, int j, double* part, int* nblk) {
    DiffReq dq{U, j, part, 0};
    int rc = fp_call(h, y, x_in, x_out, H, W, &dq);
    if (rc) return rc;
    *nblk = dq.nblk > 0 ? dq.nblk : launch_diff_gram(x_out, x_in, U, j, H * W, part, h->stream);
    LAUNCH_CHECK(h);
    return REDVE_OK;
}

int read_back(redve_t h) {
    HIP_TRY(h, hipMemcpyAsync(&h->host->info, h->ws.info, sizeof(VeInfo), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return REDVE_OK;
}

float* third(float* a, float* b, float* c, float* not1, float* not2) {
    if (a != not1 && a != not2) return a;
    if (b != not1 && b != not2) return b;
    return c;
}

// Waits for the handle's stream by polling it: a solve waits once per pass, and a sleeping
// wait adds the host's wake-up latency to each.
int wait_stream(redve_t h) {
    for (;;) {
        const hipError_t e = hipStreamQuery(h->stream);
        if (e == hipSuccess) return REDVE_OK;
        if (e != hipErrorNotReady) return fail(h, REDVE_E_HIP, hipGetErrorString(e));
    }
}

// Enqueues one pass of the solve loop from x_cur on h->stream: with extrapolation a full cycle
// of Algorithm 3 (m + L FP calls, whose last L differences form U, the small solve, and the
// combination written over x_(m,kappa)); without, one FP call and its relative-change pass.
// Ends with the copy of VeInfo to the host mirror; *next is where the pass leaves its iterate.
int enqueue_pass(redve_t h, const float* y, float* x_cur, int hx, int wx, float** next) {
    Workspace& w = h->ws;
    const int n = hx * wx;
    int rc;
    if (h->method == REDVE_VE_NONE) {
        float* nxt = x_cur == w.xa ? w.xb : w.xa;
        int nb = 0;
        if ((rc = fp_call_diff(h, y, x_cur, nxt, hx, wx, nullptr, 0, w.ve_part, &nb))) return rc;
        launch_delta(w.ve_part, nb, w.info, h->stream);
        LAUNCH_CHECK(h);
        *next = nxt;
    } else {
        float* wbase = h->m == 0 ? x_cur : nullptr;
        float* cur = x_cur;
        int nblk = 1;
        for (int i = 0; i < h->m + h->L; ++i) {
            float* nxt = third(w.xa, w.xb, w.xc, cur, wbase ? wbase : cur);
            if (i >= h->m) {
                if ((rc = fp_call_diff(h, y, cur, nxt, hx, wx, w.U, i - h->m,
                                       w.ve_part + (i - h->m) * w.win_stride, &nblk)))
                    return rc;
            } else if ((rc = fp_call(h, y, cur, nxt, hx, wx))) {
                return rc;
            }
            cur = nxt;
            if (i == h->m - 1) wbase = cur;
        }
        launch_ve_solve(w.ve_part, w.win_stride, nblk, h->L, h->method, h->rank_eps,
                        h->gamma_cap, w.info, h->stream);
        launch_ve_combine(wbase, w.U, n, w.info, wbase, h->stream);
        LAUNCH_CHECK(h);
        *next = wbase;
    }
    HIP_TRY(h, hipMemcpyAsync(&h->host->info, w.info, sizeof(VeInfo), hipMemcpyDeviceToHost,
                              h->stream));
    return REDVE_OK;
}

// Captures enqueue_pass into a graph on the handle's capture stream (the null stream cannot
// be captured). On a capture failure graphs stay off for the handle and the caller enqueues
// the pass itself.
int capture_pass(redve_t h, const float* y, float* x_cur, int hx, int wx, PassGraph& g) {
    if (!h->gstream && hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking) != hipSuccess) {
        h->gstream = nullptr;
        return REDVE_E_HIP;
    }
    hipStream_t user = h->stream;
    h->stream = h->gstream;
    if (hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        h->stream = user;
        return REDVE_E_HIP;
    }
    float* next = nullptr;
    const int rc = enqueue_pass(h, y, x_cur, hx, wx, &next);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->gstream, &graph);
    h->stream = user;
    hipGraphExec_t exec = nullptr;
    const bool ok = rc == REDVE_OK && ec == hipSuccess && graph &&
                    hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!ok) {
        (void)hipGetLastError();
        return rc ? rc : REDVE_E_HIP;
    }
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = exec;
    g.from = x_cur;
    g.next = next;
    g.hx = hx;
    g.wx = wx;
    g.m = h->m;
    g.sd_mu = h->sd_mu;
    g.gen = h->gen;
    g.op_gen = h->op_gen;
    g.arena = h->ws.arena;
    g.tune = h->cur;
    g.finish_fp32 = h->finish_fp32;
    return REDVE_OK;
}

// Runs one pass from x_cur (replaying its captured graph, capturing it on first use) and
// waits for it; the host mirror then holds its VeInfo.
int run_pass(redve_t h, const float* y, float* x_cur, int hx, int wx, float** next) {
    PassGraph* g = nullptr;
    if (!h->graphs_off && h->lin == REDVE_LIN_CG) {
        for (auto& e : h->pass)
            if (e.exec && e.from == x_cur && e.hx == hx && e.wx == wx && e.m == h->m &&
                e.sd_mu == h->sd_mu && e.gen == h->gen && e.op_gen == h->op_gen &&
                e.arena == h->ws.arena && !memcmp(&e.tune, &h->cur, sizeof(h->cur)) &&
                e.finish_fp32 == h->finish_fp32)
                g = &e;
        if (!g) {
            PassGraph& slot = h->pass[h->pass_next];
            const int rc = capture_pass(h, y, x_cur, hx, wx, slot);
            if (rc == REDVE_OK) {
                g = &slot;
                h->pass_next = (h->pass_next + 1) % kPassGraphs;
            } else if (rc == REDVE_E_HIP) {
                h->graphs_off = true;
            } else {
                return rc;
            }
        }
    }
    if (g) {
        HIP_TRY(h, hipGraphLaunch(g->exec, h->stream));
        *next = g->next;
    } else {
        const int rc = enqueue_pass(h, y, x_cur, hx, wx, next);
        if (rc) return rc;
    }
    return wait_stream(h);
}

// ---- launch configuration: rules, candidates, autotuning ------------------------------------

void tune_key(redve_t h, int hx, int wx, int (&k)[13]) {
    const int v[13] = {hx, wx, h->precision, h->T, h->F, h->J, h->kh, h->kw, h->decim,
                       h->separable, h->cg_iters, h->base, h->lin};
    for (int i = 0; i < 13; ++i) k[i] = v[i];
}

// Whether the denoiser's last stage can form the CG start with 1024-thread tiles.
bool stage_forms_start(redve_t h, int phi_table) {
    if (h->T == 0) return false;
    if (h->precision == REDVE_PREC_BF16) return h->d_phitab && phi_table == 1;
    return tnrd_mfma_fits(h->F, h->J) && h->kwin == 7;
}

// Every field of c resolved to what the launches do for an hx x wx image (0: the rule).
redve_tuning_t resolve_tuning(redve_t h, int hx, int wx, redve_tuning_t c) {
    redve_tuning_t r{};
    const LinOp op = linop_of(h);  // cur's CG fields are overridden below
    r.stage_threads = c.stage_threads ? c.stage_threads : tnrd_rule_threads(hx, wx);
    const bool tables = h->precision == REDVE_PREC_BF16 && h->d_phitab && r.stage_threads == 1024;
    r.phi_table = tables && c.phi_table != 2 ? 1 : 2;
    LinOp o2 = op;
    o2.cg_pack = c.cg_per_launch;
    const bool cg = h->base == REDVE_BASE_FP && h->lin == REDVE_LIN_CG && h->cg_iters > 0;
    r.cg_per_launch = cg && cg_block_ok(o2, h->cg_iters, hx, wx) ? 2 : 1;
    const int rule_threads = cg_rule_threads(op, hx, wx);
    const bool wide_ok = op.separable && op.kh == op.kw && (op.kh == 7 || op.kh == 9);
    r.cg_threads = c.cg_threads ? (c.cg_threads == 1024 && wide_ok ? 1024 : 256) : rule_threads;
    LinOp o3 = op;
    o3.cg_pack = 1;
    o3.cg_tile = c.cg_tile;
    r.cg_tile = cg && r.cg_per_launch == 1 && cg_iter32_ok(o3, h->cg_iters, hx, wx) ? 32 : 16;
    if (r.cg_tile == 32) r.cg_threads = 256;  // the 32x32 kernel has its own; the last is 256
    r.fused_start = cg && c.fused_start != 2 && r.cg_per_launch == 2 &&
                            r.stage_threads == 1024 && stage_forms_start(h, r.phi_table)
                        ? 1
                        : 2;
    return r;
}

const TuneEntry* find_tuned(redve_t h, const int (&k)[13]) {
    for (const TuneEntry& e : h->tune_cache)
        if (!memcmp(e.key, k, sizeof(k))) return &e;
    return nullptr;
}

void put_tuned(redve_t h, const TuneEntry& t) {
    for (TuneEntry& e : h->tune_cache)
        if (!memcmp(e.key, t.key, sizeof(t.key))) {
            e = t;
            return;
        }
    h->tune_cache.push_back(t);
}

// One JSON line per tuned problem.
void write_tuned(const std::string& path, const TuneEntry& t) {
    FILE* f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "{\"key\": [");
    for (int i = 0; i < 13; ++i) fprintf(f, i ? ", %d" : "%d", t.key[i]);
    fprintf(f,
            "], \"stage_threads\": %d, \"phi_table\": %d, \"cg_per_launch\": %d, "
            "\"cg_threads\": %d, \"fused_start\": %d, \"cg_tile\": %d, \"us\": %.3f}\n",
            t.cfg.stage_threads, t.cfg.phi_table, t.cfg.cg_per_launch, t.cfg.cg_threads,
            t.cfg.fused_start, t.cfg.cg_tile, t.us);
    fclose(f);
}

void read_tuned(redve_t h, const std::string& path) {
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return;
    char line[1024];
    while (fgets(line, sizeof(line), f)) {
        TuneEntry t{};
        int* k = t.key;
        const int n = sscanf(line,
                             "{\"key\": [%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d], "
                             "\"stage_threads\": %d, \"phi_table\": %d, \"cg_per_launch\": %d, "
                             "\"cg_threads\": %d, \"fused_start\": %d, \"cg_tile\": %d, "
                             "\"us\": %lf}",
                             &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6], &k[7], &k[8], &k[9],
                             &k[10], &k[11], &k[12], &t.cfg.stage_threads, &t.cfg.phi_table,
                             &t.cfg.cg_per_launch, &t.cfg.cg_threads, &t.cfg.fused_start,
                             &t.cfg.cg_tile, &t.us);
        if (n == 20) put_tuned(h, t);
    }
    fclose(f);
}

// The distinct valid configurations for an hx x wx image.
std::vector<redve_tuning_t> tuning_candidates(redve_t h, int hx, int wx) {
    std::vector<redve_tuning_t> out;
    for (int st : {512, 1024})
        for (int tab : {1, 2})
            for (int pk : {1, 2})
                for (int ct : {256, 1024})
                    for (int fs : {1, 2})
                        for (int tl : {16, 32}) {
                            const redve_tuning_t r =
                                resolve_tuning(h, hx, wx, {st, tab, pk, ct, fs, tl});
                            if (r.stage_threads != st || r.phi_table != tab ||
                                r.cg_per_launch != pk || r.fused_start != fs)
                                continue;  // not valid as asked
                            bool dup = false;
                            for (const auto& o : out) dup = dup || !memcmp(&o, &r, sizeof(r));
                            if (!dup) out.push_back(r);
                        }
    return out;
}

// Times every candidate on FP calls from x_in (into x_out, a scratch buffer) and keeps the
// fastest: one warm-up call, then three timed calls between HIP events on the handle's stream.
int autotune(redve_t h, const float* y, const float* x_in, float* x_out, int hx, int wx,
             TuneEntry& best) {
    const auto cands = tuning_candidates(h, hx, wx);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    int rc = REDVE_OK;
    best.us = -1.0;
    for (const redve_tuning_t& c : cands) {
        h->cur = c;
        if ((rc = fp_call(h, y, x_in, x_out, hx, wx, nullptr))) break;
        if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = REDVE_E_HIP; break; }
        for (int i = 0; i < 3 && !rc; ++i) rc = fp_call(h, y, x_in, x_out, hx, wx, nullptr);
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = REDVE_E_HIP;
            break;
        }
        const double us = ms * 1e3 / 3.0;
        if (best.us < 0 || us < best.us) {
            best.cfg = c;
            best.us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return fail(h, rc, "autotuning failed: " + h->err);
    tune_key(h, hx, wx, best.key);
    return REDVE_OK;
}

// Sets h->cur for an hx x wx problem: the forced configuration, else (AUTO) the cached or
// newly tuned one (tuning needs y, x_in and a scratch x_out; without them the rules), else the
// rules.
int select_tuning(redve_t h, int hx, int wx, const float* y = nullptr, const float* x_in = nullptr,
                  float* x_out = nullptr) {
    if (h->have_forced) {
        h->cur = h->forced;
        return REDVE_OK;
    }
    h->cur = redve_tuning_t{};
    if (h->tune_mode != REDVE_TUNE_AUTO) return REDVE_OK;
    int k[13];
    tune_key(h, hx, wx, k);
    if (const TuneEntry* e = find_tuned(h, k)) {
        h->cur = e->cfg;
        return REDVE_OK;
    }
    if (!y || !x_in || !x_out) return REDVE_OK;
    TuneEntry best{};
    const int rc = autotune(h, y, x_in, x_out, hx, wx, best);
    if (rc) {
        h->cur = redve_tuning_t{};
        return rc;
    }
    put_tuned(h, best);
    if (!h->tune_path.empty()) write_tuned(h->tune_path, best);
    h->cur = best.cfg;
    return REDVE_OK;
}

struct Progress {
    double last = -1.0;
    int grow = 0;
    // returns 0, or an error code for a non-finite or clearly diverging relative change
    int check(double d) {
        if (!std::isfinite(d)) return REDVE_E_NONFINITE;
        grow = (last >= 0 && d > last) ? grow + 1 : 0;
        last = d;
        if (grow >= 3 && d > 1.0) return REDVE_E_DIVERGED;
        return REDVE_OK;
    }
};

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================

extern "C" {

int redve_create(redve_t* out, int device, void* hip_stream) {
    if (!out) return REDVE_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return REDVE_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return REDVE_E_HIP;
    if (redve_noalloc_resolve(device) != REDVE_OK) return REDVE_E_HIP;
    redve_t h = new redve_ctx();
    h->device = device;
    h->stream = (hipStream_t)hip_stream;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess &&
        lds > h->lds_max)
        h->lds_max = lds;
    if (hipHostMalloc((void**)&h->host, sizeof(HostMirror), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return REDVE_E_NOMEM;
    }
    *out = h;
    return REDVE_OK;
}

int redve_destroy(redve_t h) {
    if (!h) return REDVE_E_ARG;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->batch && h->batch_free) h->batch_free(h->batch);
    h->batch = nullptr;
    if (h->fft && h->fft_free) h->fft_free(h->fft);
    h->fft = nullptr;
    if (h->ws.arena) (void)hipFree(h->ws.arena);
    (void)hipFree(h->d_psf);
    (void)hipFree(h->d_psf64);
    (void)hipFree(h->d_filt);
    (void)hipFree(h->d_rbfw);
    (void)hipFree(h->d_frag);
    (void)hipFree(h->d_frag32);
    (void)hipFree(h->d_phitab);
    if (h->bstream) (void)hipStreamDestroy(h->bstream);
    for (auto& g : h->pass)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    (void)hipHostFree(h->host);
    delete h;
    return REDVE_OK;
}

int redve_set_stream(redve_t h, void* hip_stream) {
    if (!h) return REDVE_E_ARG;
    h->stream = (hipStream_t)hip_stream;
    return REDVE_OK;
}

const char* redve_last_error(redve_t h) { return h ? h->err.c_str() : "null handle"; }

size_t redve_workspace_bytes(redve_t h, int hx, int wx) {
    if (!h || hx <= 0 || wx <= 0) return 0;
    return Layout((size_t)hx * wx, std::max(h->L, 1)).bytes;
}

int redve_set_operator(redve_t h, const double* psf, int kh, int kw, int decim) {
    if (!h) return REDVE_E_ARG;
    if (!psf || kh < 1 || kw < 1 || !(kh & 1) || !(kw & 1) || kh > REDVE_MAX_PSF ||
        kw > REDVE_MAX_PSF)
        return fail(h, REDVE_E_ARG, "psf must be odd-sized, at most 15 x 15");
    if (decim < 1 || decim > REDVE_MAX_DECIM) return fail(h, REDVE_E_ARG, "decim must be in 1..4");
    for (int i = 0; i < kh * kw; ++i)
        if (!std::isfinite(psf[i])) return fail(h, REDVE_E_ARG, "psf has non-finite taps");
    HIP_TRY(h, hipSetDevice(h->device));
    h->psf.assign(kh * kw, 0.f);
    for (int i = 0; i < kh * kw; ++i) h->psf[i] = (float)psf[i];
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (h->d_psf) HIP_TRY(h, hipFree(h->d_psf));
    if (h->d_psf64) HIP_TRY(h, hipFree(h->d_psf64));
    h->d_psf = nullptr;
    h->d_psf64 = nullptr;
    HIP_TRY(h, hipMalloc(&h->d_psf, sizeof(float) * kh * kw));
    HIP_TRY(h, hipMalloc(&h->d_psf64, sizeof(double) * kh * kw));
    HIP_TRY(h, hipMemcpy(h->d_psf, h->psf.data(), sizeof(float) * kh * kw, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->d_psf64, psf, sizeof(double) * kh * kw, hipMemcpyHostToDevice));
    h->kh = kh;
    h->kw = kw;
    h->decim = decim;
    h->psf_l1 = 0.0;
    for (int i = 0; i < kh * kw; ++i) h->psf_l1 += fabs(psf[i]);
    ++h->op_gen;
    // rank-1 test: psf = col (x) row with col = the column through the largest tap and
    // row = that tap's row divided by it (exact for any rank-1 matrix)
    int im = 0;
    for (int i = 1; i < kh * kw; ++i)
        if (fabs(psf[i]) > fabs(psf[im])) im = i;
    const int ai = im / kw, bj = im % kw;
    double amax = fabs(psf[im]), err = 0.0;
    for (int a = 0; a < kh; ++a) h->col[a] = psf[a * kw + bj];
    for (int b = 0; b < kw; ++b) h->row[b] = amax > 0 ? psf[ai * kw + b] / psf[im] : 0.0;
    for (int a = 0; a < kh; ++a)
        for (int b = 0; b < kw; ++b) err = fmax(err, fabs(psf[a * kw + b] - h->col[a] * h->row[b]));
    h->separable = (amax > 0 && err <= 1e-12 * amax) ? 1 : 0;
    h->have_op = true;
    return REDVE_OK;
}

int redve_set_noise(redve_t h, double sigma) {
    if (!h) return REDVE_E_ARG;
    if (!(sigma > 0) || !std::isfinite(sigma)) return fail(h, REDVE_E_ARG, "sigma must be > 0");
    h->sigma = sigma;
    ++h->op_gen;
    return REDVE_OK;
}

int redve_set_lambda(redve_t h, double lambda) {
    if (!h) return REDVE_E_ARG;
    if (!(lambda > 0) || !std::isfinite(lambda)) return fail(h, REDVE_E_ARG, "lambda must be > 0");
    h->lambda = lambda;
    ++h->op_gen;
    return REDVE_OK;
}

int redve_set_denoiser(redve_t h, const redve_tnrd_t* p) {
    if (!h) return REDVE_E_ARG;
    ++h->gen;
    if (!p) return fail(h, REDVE_E_ARG, "null denoiser");
    if (p->stages < 0 || p->stages > kMaxStages) return fail(h, REDVE_E_ARG, "stages must be 0..16");
    if (p->ksize != 5) return fail(h, REDVE_E_ARG, "ksize must be 5");
    if (p->stages > 0) {
        if (p->nfilt < 1 || p->nfilt > REDVE_MAX_FILTERS) return fail(h, REDVE_E_ARG, "nfilt out of range");
        if (p->nrbf < 1 || p->nrbf > REDVE_MAX_RBF) return fail(h, REDVE_E_ARG, "nrbf out of range");
        if (!(p->gamma > 0) || !(p->dmu > 0) || !std::isfinite(p->mu0) || !std::isfinite(p->dmu))
            return fail(h, REDVE_E_ARG, "bad RBF grid");
        // exact window: centres farther than (K + 1/2) dmu from z add < 1e-12 of a weight,
        // i.e. (K + 1/2) dmu / gamma >= sqrt(2 ln 1e12) = 7.43
        const double ratio = p->gamma / p->dmu;
        if (ratio < 1.0 / 3.0 || ratio > 2.2)
            return fail(h, REDVE_E_ARG, "gamma / dmu must be in [1/3, 2.2]");
        if (!p->filters || !p->rbf_w || !p->react) return fail(h, REDVE_E_ARG, "null denoiser array");
        const int ks2 = 25;
        for (int f = 0; f < p->stages * p->nfilt; ++f) {
            double s = 0, a = 0;
            for (int k = 0; k < ks2; ++k) {
                const double v = p->filters[(size_t)f * ks2 + k];
                if (!std::isfinite(v)) return fail(h, REDVE_E_ARG, "non-finite filter tap");
                s += v;
                a += fabs(v);
            }
            if (fabs(s) > 1e-6 * a) return fail(h, REDVE_E_ARG, "filters must have zero mean");
        }
        for (size_t i = 0; i < (size_t)p->stages * p->nfilt * p->nrbf; ++i)
            if (!std::isfinite(p->rbf_w[i])) return fail(h, REDVE_E_ARG, "non-finite RBF weight");
        for (int t = 0; t < p->stages; ++t)
            if (!std::isfinite(p->react[t])) return fail(h, REDVE_E_ARG, "non-finite reaction weight");
    }
    if (p->precision != REDVE_PREC_FP32 && p->precision != REDVE_PREC_BF16)
        return fail(h, REDVE_E_ARG, "precision must be FP32 or BF16");
    // a BF16 stage keeps a tile's per-position rows (z, v, tap sums) in LDS with the weight
    // rows (window evaluation; every image) and, on small images, with the influence-function
    // tables instead, which are built where they fit the device's workgroup LDS
    const int tab_n = p->stages > 0 ? tnrd_table_intervals(p->dmu, p->gamma, p->nrbf) : 0;
    const bool use_tab = p->stages > 0 && p->precision == REDVE_PREC_BF16 &&
                         tnrd_table_smem_bytes(p->nfilt, tab_n) <= (size_t)h->lds_max;
    if (p->stages > 0 && p->precision == REDVE_PREC_BF16 &&
        tnrd_mfma_smem_bytes(p->nfilt, p->nrbf) > (size_t)h->lds_max)
        return fail(h, REDVE_E_ARG, "BF16 stage: nfilt and nrbf exceed the LDS of a workgroup (use FP32)");
    HIP_TRY(h, hipSetDevice(h->device));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    (void)hipFree(h->d_filt);
    (void)hipFree(h->d_rbfw);
    (void)hipFree(h->d_frag);
    (void)hipFree(h->d_frag32);
    (void)hipFree(h->d_phitab);
    h->d_filt = h->d_rbfw = nullptr;
    h->d_frag = nullptr;
    h->d_frag32 = nullptr;
    h->d_phitab = nullptr;
    h->tab_n = 0;
    h->T = p->stages;
    h->F = p->stages > 0 ? p->nfilt : 0;
    h->J = p->stages > 0 ? p->nrbf : 0;
    h->mu0 = p->mu0;
    h->dmu = p->dmu;
    h->gamma = p->gamma;
    h->precision = p->precision;
    // RBF window: the centres beyond (K + 1/2) dmu from z add less than eps of a weight each,
    // (K + 1/2) dmu / gamma >= sqrt(2 ln(1/eps)): eps = 1e-12 for the FP32 form (7.4338), and
    // 1e-6 for the BF16 form (5.2565), far below the BF16 operands' own 3.9e-3
    const double reach = p->precision == REDVE_PREC_BF16 ? 5.2565 : 7.4338;
    h->kwin = p->stages > 0 ? std::max(1, (int)ceil(reach * p->gamma / p->dmu - 0.5)) : 1;
    h->kwin32 = p->stages > 0 ? std::max(1, (int)ceil(7.4338 * p->gamma / p->dmu - 0.5)) : 1;
    h->theta.assign(h->T, 0.f);
    if (h->T > 0) {
        // weights as rows of J + 2 kRbfPad, zero-padded both sides (the stage kernels copy
        // them to LDS as they are)
        const size_t ws = (size_t)h->J + 2 * kRbfPad;
        const size_t nf = (size_t)h->T * h->F * 25, nw = (size_t)h->T * h->F * ws;
        std::vector<float> f(nf), w(nw, 0.f);
        for (size_t i = 0; i < nf; ++i) f[i] = (float)p->filters[i];
        for (size_t r = 0; r < (size_t)h->T * h->F; ++r)
            for (int j = 0; j < h->J; ++j) w[r * ws + kRbfPad + j] = (float)p->rbf_w[r * h->J + j];
        for (int t = 0; t < h->T; ++t) h->theta[t] = (float)p->react[t];
        // MFMA operand fragments (v_mfma_f32_16x16x32_bf16, B operand): lane l of half hf holds
        // column n = l % 16 + 16 hf and the K values 8 (l / 16) + j. Forward: K = tap, n = filter;
        // adjoint: K = filter, n = tap. Round to nearest even.
        auto bf16 = [](double x) {
            float v = (float)x;
            uint32_t bits;
            memcpy(&bits, &v, 4);
            bits += 0x7FFFu + ((bits >> 16) & 1u);
            return (uint16_t)(bits >> 16);
        };
        const size_t per = 2 * 64 * 8;
        std::vector<uint16_t> frag(2 * (size_t)h->T * per, 0);
        for (int t = 0; t < h->T; ++t)
            for (int hf = 0; hf < 2; ++hf)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        const int kk = 8 * (l / 16) + j, n = l % 16 + 16 * hf;
                        const size_t o = (size_t)t * per + ((size_t)hf * 64 + l) * 8 + j;
                        const double* ft = p->filters + (size_t)t * h->F * 25;
                        if (kk < 25 && n < h->F) frag[o] = bf16(ft[n * 25 + kk]);
                        if (kk < h->F && n < 25) frag[(size_t)h->T * per + o] = bf16(ft[kk * 25 + n]);
                    }
        // FP32 fragments (v_mfma_f32_16x16x4_f32, B operand): lane l of block hf holds column
        // n = l % 16 + 16 hf and K value 4 k + l / 16 of slice k. Forward: K = tap, n = filter;
        // adjoint: K = filter, n = tap.
        std::vector<float> frag32((size_t)h->T * (kFrag32Fwd + kFrag32Adj), 0.f);
        for (int t = 0; t < h->T; ++t) {
            const double* ft = p->filters + (size_t)t * h->F * 25;
            float* fw = frag32.data() + (size_t)t * kFrag32Fwd;
            float* fa = frag32.data() + (size_t)h->T * kFrag32Fwd + (size_t)t * kFrag32Adj;
            for (int k = 0; k < 8; ++k)
                for (int hf = 0; hf < 2; ++hf)
                    for (int l = 0; l < 64; ++l) {
                        const int kk = 4 * k + l / 16, n = l % 16 + 16 * hf;
                        const size_t o = ((size_t)k * 2 + hf) * 64 + l;
                        if (k < 7 && kk < 25 && n < h->F) fw[o] = (float)ft[n * 25 + kk];
                        if (kk < h->F && n < 25) fa[o] = (float)ft[kk * 25 + n];
                    }
        }
        // influence-function tables (BF16 form): per stage and filter, the cubic Hermite
        // interpolant of phi between knots z_k = lo + k h, from phi and h phi' at the knots
        // (all J terms, FP64), as (a0, a1, a2, a3) with phi ~ a0 + a1 u + a2 u^2 + a3 u^3
        if (use_tab) {
            const double hs = kTabStep * p->gamma, lo = p->mu0 - kTabReach * p->gamma;
            const double g2 = p->gamma * p->gamma;
            std::vector<float> tab((size_t)h->T * h->F * tab_n * 4);
            std::vector<double> v(tab_n + 1), dv(tab_n + 1);
            for (size_t r = 0; r < (size_t)h->T * h->F; ++r) {
                const double* wr = p->rbf_w + r * h->J;
                for (int k = 0; k <= tab_n; ++k) {
                    const double z = lo + k * hs;
                    double s0 = 0, s1 = 0;
                    for (int j = 0; j < h->J; ++j) {
                        const double e = z - (p->mu0 + j * p->dmu);
                        const double term = wr[j] * exp(-e * e / (2.0 * g2));
                        s0 += term;
                        s1 -= term * e / g2;
                    }
                    v[k] = s0;
                    dv[k] = s1 * hs;
                }
                for (int k = 0; k < tab_n; ++k) {
                    float* c = tab.data() + (r * tab_n + k) * 4;
                    c[0] = (float)v[k];
                    c[1] = (float)dv[k];
                    c[2] = (float)(3.0 * (v[k + 1] - v[k]) - 2.0 * dv[k] - dv[k + 1]);
                    c[3] = (float)(2.0 * (v[k] - v[k + 1]) + dv[k] + dv[k + 1]);
                }
            }
            HIP_TRY(h, hipMalloc(&h->d_phitab, tab.size() * sizeof(float)));
            HIP_TRY(h, hipMemcpy(h->d_phitab, tab.data(), tab.size() * sizeof(float),
                                 hipMemcpyHostToDevice));
            h->tab_n = tab_n;
            h->tab_lo = lo;
            h->tab_h = hs;
        }
        HIP_TRY(h, hipMalloc(&h->d_frag32, frag32.size() * sizeof(float)));
        HIP_TRY(h, hipMemcpy(h->d_frag32, frag32.data(), frag32.size() * sizeof(float),
                             hipMemcpyHostToDevice));
        HIP_TRY(h, hipMalloc(&h->d_filt, nf * sizeof(float)));
        HIP_TRY(h, hipMalloc(&h->d_rbfw, nw * sizeof(float)));
        HIP_TRY(h, hipMalloc(&h->d_frag, frag.size() * sizeof(uint16_t)));
        HIP_TRY(h, hipMemcpy(h->d_filt, f.data(), nf * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(h->d_rbfw, w.data(), nw * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemcpy(h->d_frag, frag.data(), frag.size() * sizeof(uint16_t),
                             hipMemcpyHostToDevice));
    }
    h->have_den = true;
    return REDVE_OK;
}

int redve_set_extrapolation(redve_t h, int method, int L, int m) {
    if (!h) return REDVE_E_ARG;
    if (method < REDVE_VE_NONE || method > REDVE_VE_SVD_MPE) return fail(h, REDVE_E_ARG, "bad method");
    if (L < 2 || L > REDVE_MAX_L) return fail(h, REDVE_E_ARG, "L must be 2..16");
    if (m < 0) return fail(h, REDVE_E_ARG, "m must be >= 0");
    if (method != h->method || L != h->L) ++h->gen;
    h->method = method;
    h->L = L;
    h->m = m;
    return REDVE_OK;
}

int redve_set_precision_switch(redve_t h, double delta) {
    if (!h) return REDVE_E_ARG;
    if (!(delta >= 0) || !std::isfinite(delta))
        return fail(h, REDVE_E_ARG, "the switch must be finite and >= 0");
    if (delta != h->prec_switch) ++h->gen;  // the batched rounds record their stage kernel
    h->prec_switch = delta;
    return REDVE_OK;
}

int redve_set_guard(redve_t h, double gamma_cap) {
    if (!h) return REDVE_E_ARG;
    if (std::isnan(gamma_cap)) return fail(h, REDVE_E_ARG, "gamma_cap must not be NaN");
    const double cap = gamma_cap > 0.0 ? gamma_cap : 0.0;
    if (cap != h->gamma_cap) ++h->gen;  // captured passes and batched rounds record it
    h->gamma_cap = cap;
    return REDVE_OK;
}

int redve_set_autotune(redve_t h, int mode, const char* cache_path) {
    if (!h) return REDVE_E_ARG;
    if (mode != REDVE_TUNE_RULES && mode != REDVE_TUNE_AUTO)
        return fail(h, REDVE_E_ARG, "mode must be REDVE_TUNE_RULES or REDVE_TUNE_AUTO");
    h->tune_mode = mode;
    h->tune_path = cache_path ? cache_path : "";
    if (cache_path) read_tuned(h, h->tune_path);
    return REDVE_OK;
}

int redve_set_tuning(redve_t h, const redve_tuning_t* t) {
    if (!h) return REDVE_E_ARG;
    if (!t) {
        h->have_forced = false;
        return REDVE_OK;
    }
    const bool ok = (t->stage_threads == 0 || t->stage_threads == 512 || t->stage_threads == 1024) &&
                    t->phi_table >= 0 && t->phi_table <= 2 && t->cg_per_launch >= 0 &&
                    t->cg_per_launch <= 2 &&
                    (t->cg_threads == 0 || t->cg_threads == 256 || t->cg_threads == 1024) &&
                    t->fused_start >= 0 && t->fused_start <= 2 &&
                    (t->cg_tile == 0 || t->cg_tile == 16 || t->cg_tile == 32);
    if (!ok) return fail(h, REDVE_E_ARG, "tuning field out of range");
    if (t->phi_table == 1 && t->stage_threads == 512)
        return fail(h, REDVE_E_ARG, "tabulated influence functions need 1024 stage threads");
    if (t->fused_start == 1 && (t->cg_per_launch == 1 || t->stage_threads == 512))
        return fail(h, REDVE_E_ARG,
                    "the fused CG start needs two CG iterations per launch and 1024 stage threads");
    h->forced = *t;
    h->have_forced = true;
    return REDVE_OK;
}

int redve_get_tuning(redve_t h, int hx, int wx, redve_tuning_t* out, double* us) {
    if (!h) return REDVE_E_ARG;
    if (!out) return fail(h, REDVE_E_ARG, "null pointer");
    int rc = check_image(h, hx, wx);
    if (rc) return rc;
    redve_tuning_t c{};
    double u = -1.0;
    if (h->have_forced) {
        c = h->forced;
    } else if (h->tune_mode == REDVE_TUNE_AUTO) {
        int k[13];
        tune_key(h, hx, wx, k);
        if (const TuneEntry* e = find_tuned(h, k)) {
            c = e->cfg;
            u = e->us;
        }
    }
    *out = resolve_tuning(h, hx, wx, c);
    if (us) *us = u;
    return REDVE_OK;
}

int redve_set_linear_solver(redve_t h, int kind) {
    if (!h) return REDVE_E_ARG;
    if (kind != REDVE_LIN_CG && kind != REDVE_LIN_FFT) return fail(h, REDVE_E_ARG, "bad solver");
    h->lin = kind;
    return REDVE_OK;
}

int redve_set_base(redve_t h, int base, double mu) {
    if (!h) return REDVE_E_ARG;
    if (base != REDVE_BASE_FP && base != REDVE_BASE_SD) return fail(h, REDVE_E_ARG, "bad base");
    if (!std::isfinite(mu)) return fail(h, REDVE_E_ARG, "mu must be finite");
    if (base != h->base) ++h->gen;
    h->base = base;
    h->sd_mu = mu;
    return REDVE_OK;
}

int redve_set_solver(redve_t h, int cg_iters, int max_fp_calls, double tol, int extra_fp) {
    if (!h) return REDVE_E_ARG;
    if (cg_iters < 0 || max_fp_calls < 0 || extra_fp < 0 || !(tol >= 0) || !std::isfinite(tol))
        return fail(h, REDVE_E_ARG, "solver settings out of range");
    if (cg_iters != h->cg_iters) ++h->gen;
    h->cg_iters = cg_iters;
    h->max_fp = max_fp_calls;
    h->tol = tol;
    h->extra_fp = extra_fp;
    return REDVE_OK;
}

int redve_apply_H(redve_t h, const float* x, int hx, int wx, float* y) {
    if (!h) return REDVE_E_ARG;
    if (!x || !y) return fail(h, REDVE_E_ARG, "null pointer");
    int rc = check_image(h, hx, wx);
    if (rc) return rc;
    if (!h->have_op) return fail(h, REDVE_E_STATE, "redve_set_operator was not called");
    HIP_TRY(h, hipSetDevice(h->device));
    LinOp op = linop_of(h);
    launch_apply_H(op, x, hx, wx, y, h->stream);
    LAUNCH_CHECK(h);
    return REDVE_OK;
}

int redve_apply_Ht(redve_t h, const float* y, int hx, int wx, float* out) {
    if (!h) return REDVE_E_ARG;
    if (!y || !out) return fail(h, REDVE_E_ARG, "null pointer");
    int rc = check_image(h, hx, wx);
    if (rc) return rc;
    if (!h->have_op) return fail(h, REDVE_E_STATE, "redve_set_operator was not called");
    HIP_TRY(h, hipSetDevice(h->device));
    LinOp op = linop_of(h);
    launch_apply_Ht(op, y, hx, wx, 1.0f, out, h->stream);
    LAUNCH_CHECK(h);
    return REDVE_OK;
}

int redve_apply_A(redve_t h, const float* p, int hx, int wx, float* out) {
    if (!h) return REDVE_E_ARG;
    if (!p || !out) return fail(h, REDVE_E_ARG, "null pointer");
    int rc = check_image(h, hx, wx);
    if (rc || (rc = check_ready(h, false))) return rc;
    HIP_TRY(h, hipSetDevice(h->device));
    launch_apply_A(linop_of(h), p, hx, wx, out, h->stream);
    LAUNCH_CHECK(h);
    return REDVE_OK;
}

int redve_cg(redve_t h, const float* rhs, float* x, int hx, int wx, int iters) {
    if (!h) return REDVE_E_ARG;
    if (!rhs || !x || iters < 0) return fail(h, REDVE_E_ARG, "bad argument");
    int rc = check_image(h, hx, wx);
    if (rc || (rc = check_ready(h, false))) return rc;
    HIP_TRY(h, hipSetDevice(h->device));
    if ((rc = ensure_workspace(h, hx, wx, h->L)) || (rc = select_tuning(h, hx, wx))) return rc;
    const size_t n = (size_t)hx * wx;
    HIP_TRY(h, hipMemcpyAsync(h->ws.xa, x, n * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
    return run_cg(h, rhs, h->ws.xa, x, hx, wx, iters);
}

int redve_objective(redve_t h, const float* y, const float* x, int hx, int wx, double* E) {
    if (!h) return REDVE_E_ARG;
    if (!y || !x || !E) return fail(h, REDVE_E_ARG, "null pointer");
    int rc = check_image(h, hx, wx);
    if (rc || (rc = check_ready(h, true))) return rc;
    HIP_TRY(h, hipSetDevice(h->device));
    if ((rc = ensure_workspace(h, hx, wx, h->L)) || (rc = select_tuning(h, hx, wx))) return rc;
    Workspace& w = h->ws;
    bool s_null = false;
    if ((rc = run_denoiser(h, x, hx, wx, w.sres, true, &s_null))) return rc;
    double* out = w.ve_part + 2 * kMaxRedBlocks;  // the window partials are free here
    launch_objective(linop_of(h), x, y, s_null ? nullptr : w.sres, hx, wx, w.ve_part, out,
                     h->stream);
    LAUNCH_CHECK(h);
    HIP_TRY(h, hipMemcpyAsync(h->host->obj, out, 2 * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    *E = h->host->obj[0] / (2.0 * h->sigma * h->sigma) - 0.5 * h->lambda * h->host->obj[1];
    return REDVE_OK;
}

int redve_denoise(redve_t h, const float* x, int hx, int wx, float* out) {
    if (!h) return REDVE_E_ARG;
    if (!x || !out || x == out) return fail(h, REDVE_E_ARG, "bad pointers");
    int rc = check_image(h, hx, wx);
    if (rc) return rc;
    if (!h->have_den) return fail(h, REDVE_E_STATE, "redve_set_denoiser was not called");
    HIP_TRY(h, hipSetDevice(h->device));
    if ((rc = ensure_workspace(h, hx, wx, h->L)) || (rc = select_tuning(h, hx, wx))) return rc;
    return run_denoiser(h, x, hx, wx, out, false, nullptr);
}

int redve_fp_step(redve_t h, const float* y, const float* x, int hx, int wx, float* out) {
    if (!h) return REDVE_E_ARG;
    if (!y || !x || !out || x == out) return fail(h, REDVE_E_ARG, "bad pointers");
    int rc = check_image(h, hx, wx);
    if (rc || (rc = check_ready(h, true)) || (rc = check_linear(h)) ||
        (rc = check_fft_size(h, hx, wx)))
        return rc;
    HIP_TRY(h, hipSetDevice(h->device));
    if ((rc = ensure_workspace(h, hx, wx, h->L)) ||
        (rc = select_tuning(h, hx, wx, y, x, h->ws.xb)))
        return rc;
    return fp_call(h, y, x, out, hx, wx);
}

int redve_extrapolate(redve_t h, const float* xs, int L, int hx, int wx, float* out,
                      double* gamma, int* breakdown) {
    if (!h) return REDVE_E_ARG;
    if (!xs || !out) return fail(h, REDVE_E_ARG, "null pointer");
    if (L < 2 || L > REDVE_MAX_L) return fail(h, REDVE_E_ARG, "L must be 2..16");
    if (h->method == REDVE_VE_NONE) return fail(h, REDVE_E_STATE, "no extrapolation method set");
    int rc = check_image(h, hx, wx);
    if (rc) return rc;
    HIP_TRY(h, hipSetDevice(h->device));
    if ((rc = ensure_workspace(h, hx, wx, L))) return rc;
    const int n = hx * wx;
    Workspace& w = h->ws;
    int nblk = 1;
    for (int j = 0; j < L; ++j) {
        nblk = launch_diff_gram(xs + (size_t)(j + 1) * n, xs + (size_t)j * n, w.U, j, n,
                                w.ve_part + j * w.win_stride, h->stream);
        LAUNCH_CHECK(h);
    }
    launch_ve_solve(w.ve_part, w.win_stride, nblk, L, h->method, h->rank_eps, h->gamma_cap, w.info,
                    h->stream);
    launch_ve_combine(xs, w.U, n, w.info, out, h->stream);
    LAUNCH_CHECK(h);
    if ((rc = read_back(h))) return rc;
    if (gamma)
        for (int j = 0; j < L; ++j) gamma[j] = h->host->info.gamma[j];
    if (breakdown) *breakdown = h->host->info.breakdown;
    return REDVE_OK;
}

int redve_solve(redve_t h, const float* y, int hy, int wy, const float* x0, float* x, int hx,
                int wx, redve_stats_t* st) {
    if (!h) return REDVE_E_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    if (st) memset(st, 0, sizeof(*st));
    if (!y || !x) return fail(h, REDVE_E_ARG, "null pointer");
    int rc = check_image(h, hx, wx);
    if (rc || (rc = check_ready(h, true)) || (rc = check_linear(h)) ||
        (rc = check_fft_size(h, hx, wx)))
        return rc;
    if (hy != (hx + h->decim - 1) / h->decim || wy != (wx + h->decim - 1) / h->decim)
        return fail(h, REDVE_E_ARG, "observation size does not match ceil(x size / decim)");
    HIP_TRY(h, hipSetDevice(h->device));
    const int L = h->method == REDVE_VE_NONE ? 1 : h->L;
    if ((rc = ensure_workspace(h, hx, wx, L))) return rc;
    Workspace& w = h->ws;
    const int n = hx * wx;
    const size_t bytes = sizeof(float) * n;
    LinOp op = linop_of(h);

    // x0 (default: y, or decim^2 H^T y for SR)
    if (x0)
        HIP_TRY(h, hipMemcpyAsync(w.xa, x0, bytes, hipMemcpyDeviceToDevice, h->stream));
    else if (h->decim == 1)
        HIP_TRY(h, hipMemcpyAsync(w.xa, y, bytes, hipMemcpyDeviceToDevice, h->stream));
    else {
        launch_apply_Ht(op, y, hx, wx, (float)(h->decim * h->decim), w.xa, h->stream);
        LAUNCH_CHECK(h);
    }

    // the passes read the observation from the workspace, so a captured pass serves any y
    HIP_TRY(h, hipMemcpyAsync(w.yw, y, sizeof(float) * (size_t)hy * wy, hipMemcpyDeviceToDevice,
                              h->stream));
    const float* yw = w.yw;
    // the launch configuration (AUTO: tuned on FP calls from x0 on first use of this problem)
    if ((rc = select_tuning(h, hx, wx, yw, w.xa, w.xb))) return rc;

    int calls = 0, cycles = 0, breakdowns = 0, rejected = 0, status = REDVE_OK;
    double delta = INFINITY, gl1max = 0.0;
    Progress prog;
    float* x_cur = w.xa;
    // BF16 form: FP32 banks for the FP calls after the relative change first falls below the
    // switch (prec_switch > 0)
    h->finish_fp32 = false;
    auto maybe_switch = [&] {
        if (h->prec_switch > 0 && h->precision == REDVE_PREC_BF16 && delta < h->prec_switch)
            h->finish_fp32 = true;
    };

    if (h->method == REDVE_VE_NONE) {
        while (calls < h->max_fp) {
            float* nxt = nullptr;
            if ((rc = run_pass(h, yw, x_cur, hx, wx, &nxt))) return rc;
            ++calls;
            delta = sqrt(h->host->info.uu / h->host->info.xx);
            x_cur = nxt;
            if ((status = prog.check(delta))) break;
            if (delta < h->tol) break;
            maybe_switch();
        }
    } else {
        // Algorithm 3 (full cycling): m FP calls, then L = kappa+1 more whose differences form
        // U; extrapolate (Algorithm 1) and restart from x_(m,kappa).
        while (calls < h->max_fp) {
            if (calls + h->m + L > h->max_fp) {
                // the FP-call budget ends inside this cycle: its FP calls, no extrapolation
                float* wbase = h->m == 0 ? x_cur : nullptr;
                float* cur = x_cur;
                for (int i = 0; i < h->m + L && calls < h->max_fp; ++i) {
                    float* nxt = third(w.xa, w.xb, w.xc, cur, wbase ? wbase : cur);
                    if ((rc = fp_call(h, yw, cur, nxt, hx, wx))) return rc;
                    ++calls;
                    cur = nxt;
                    if (i == h->m - 1) wbase = cur;
                }
                x_cur = cur;
                break;
            }
            float* next = nullptr;
            if ((rc = run_pass(h, yw, x_cur, hx, wx, &next))) return rc;
            calls += h->m + L;
            x_cur = next;
            ++cycles;
            const VeInfo& vi = h->host->info;
            if (vi.breakdown)
                ++breakdowns;
            else
                gl1max = std::max(gl1max, vi.gamma_l1);
            if (vi.guarded) ++rejected;
            delta = sqrt(vi.uu / vi.xx);
            // rejected coefficients are not used; a non-finite iterate shows in delta
            if (!vi.guarded && !std::isfinite(vi.gamma_l1)) {
                status = REDVE_E_NONFINITE;
                break;
            }
            if ((status = prog.check(delta))) break;
            if (delta < h->tol) break;
            maybe_switch();
        }
    }
    if (status == REDVE_OK) {
        for (int e = 0; e < h->extra_fp; ++e) {
            float* nxt = third(w.xa, w.xb, w.xc, x_cur, x_cur);
            if ((rc = fp_call(h, yw, x_cur, nxt, hx, wx))) return rc;
            ++calls;
            x_cur = nxt;
        }
    }
    h->finish_fp32 = false;
    // the result is queued in stream order; the statistics are already on the host
    HIP_TRY(h, hipMemcpyAsync(x, x_cur, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (st) {
        st->fp_calls = calls;
        st->cycles = cycles;
        st->breakdowns = breakdowns;
        st->rejected = rejected;
        st->status = status;
        st->final_delta = delta;
        st->max_gamma_l1 = gl1max;
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status != REDVE_OK)
        return fail(h, status, status == REDVE_E_NONFINITE ? "iterate became non-finite"
                                                            : "iteration diverged");
    return REDVE_OK;
}

}  // extern "C"
