// Batched and serving engine: many independent restorations advance together, one FP call
// (eq. (7)) per round, each with its own full-cycling state (Algorithm 3).
//
// Every kernel of a round runs once over a tile list covering the running images (16x16
// tiles, padded to a power-of-two length with entries that point at an always-inactive image),
// so a round is a fixed launch sequence per (stencil class, list length): it is captured once
// as a HIP graph and replayed. The list is in dispatch order: workgroups go round-robin over
// the 8 XCDs, and the workgroups of each XCD take a contiguous run of the live tiles (image by
// image, row-major) and then an equal share of the padding, so neighbouring tiles share an L2
// and every XCD gets the same amount of work. What changes between rounds (which
// buffers hold x_in / x_out / x_m, the window column, whether to extrapolate, which images are
// active, where an image's tiles start in the list) lives in the per-image descriptors,
// uploaded before each replay. Per-image reductions sum per-tile partials in tile order, so an
// image's result does not depend on the rest of the batch. Device memory is one arena per named
// vector; an image occupies the same element range in each (first-fit over a fixed capacity),
// which is what the serving loop admits against.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "context.h"

using namespace redve;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kVecs = 14;  // x[3], sres, u0, u1, r[2], w[2], s[2], p, d

size_t align64(size_t n) { return (n + 63) / 64 * 64; }
int tiles_of(int h, int w) { return ((h + kBatchTile - 1) / kBatchTile) * ((w + kBatchTile - 1) / kBatchTile); }

// First-fit allocator of [0, cap) ranges.
struct RangeAlloc {
    size_t cap = 0;
    std::map<size_t, size_t> used;  // start -> length
    bool alloc(size_t n, size_t& out) {
        size_t pos = 0;
        for (auto& kv : used) {
            if (kv.first - pos >= n) break;
            pos = kv.first + kv.second;
        }
        if (pos + n > cap) return false;
        used[pos] = n;
        out = pos;
        return true;
    }
    void release(size_t start) { used.erase(start); }
};

struct Progress {
    double last = -1.0;
    int grow = 0;
    int check(double d) {
        if (!std::isfinite(d)) return REDVE_E_NONFINITE;
        grow = (last >= 0 && d > last) ? grow + 1 : 0;
        last = d;
        if (grow >= 3 && d > 1.0) return REDVE_E_DIVERGED;
        return REDVE_OK;
    }
};

struct Slot {
    bool used = false, running = false, finished = false;
    redve_item_t item{};
    size_t off = 0, npx = 0;
    int tile0 = 0, ntiles = 0;  // tile0: start in the packed tile list (set at each repack)
    LinOp op{};
    int padded = 0;        // the operator fits the radius-4 separable fast path
    int cg32 = 0;          // ... without decimation: CG on the 32x32 tile list (r, p, d only)
    // Algorithm 3 state
    int cur = 0, base = 0, phase = 0, extra_left = 0;
    bool extra = false;
    int calls = 0, cycles = 0, breakdowns = 0, rejected = 0, status = REDVE_OK;
    double delta = INFINITY, gl1max = 0.0;
    bool finish_fp32 = false;  // BF16 form: this image has switched to FP32 banks
    Progress prog;
    // round bookkeeping
    int next = 0;
    bool in_window = false, do_ve = false;
    unsigned long long ticket = 0;
    Clock::time_point t_submit;
    double ms = 0.0;
};

struct Engine {
    redve_t h = nullptr;      // settings (denoiser, method, solver)
    // the first failure of a copy or wait queued outside a round (admission, retirement); the
    // next round, and the end of a batch, report it as REDVE_E_HIP
    hipError_t queue_err = hipSuccess;
    void note(hipError_t e) {
        if (e != hipSuccess && queue_err == hipSuccess) queue_err = e;
    }
    unsigned long long gen = 0;  // the settings generation the graphs were recorded for
    hipStream_t st = nullptr; // the engine's own stream (capturable; never the null stream)
    int cap_img = 0, cap_tiles = 0, L = 1;
    size_t cap_px = 0;
    RangeAlloc px_alloc;
    int tiles_used = 0;    // tiles of the admitted images
    int launch_tiles = 0;  // length of the packed, padded tile list
    int launch_tiles32 = 0;  // length of the 32x32 tile list (0: no image takes that form)
    int launch_tiles16r = 0;  // length of the 16x16 list of the other images (0: none)
    void* arena = nullptr;
    float* vec[kVecs] = {};
    float* U = nullptr;
    ImgDesc* d_desc = nullptr;
    TileRef* d_tile = nullptr;
    TileRef* d_tile32 = nullptr;  // 32x32 tiles of the cg32 images (at most cap_tiles)
    TileRef* d_tile16r = nullptr;  // 16x16 tiles of the images not on the 32x32 CG form
    CgImg* d_cg = nullptr;
    double* d_part = nullptr;
    double* d_G = nullptr;
    VeInfo* d_info = nullptr;
    ImgStat* d_stat = nullptr;
    float* d_psf = nullptr;     // per slot: 15 x 15 floats
    double* d_psf64 = nullptr;  // per slot: 15 x 15 doubles
    ImgDesc* h_desc = nullptr;  // pinned
    ImgStat* h_stat = nullptr;  // pinned
    TileRef* h_tile = nullptr;  // pinned
    TileRef* h_tile32 = nullptr;   // pinned
    TileRef* h_tile16r = nullptr;  // pinned
    // live tiles in partial-index order (repack scratch): all, 32x32 of the cg32 images, 16x16
    // of the others
    std::vector<TileRef> live, live32, live16r;
    bool tiles_dirty = true;
    std::vector<Slot> slots;
    // graphs keyed by (stencil radius class, lengths of the tile list, the 32x32 list and the
    // 16x16 list of the images not on the 32x32 form)
    using GraphKey = std::tuple<int, int, int, int>;
    std::map<GraphKey, hipGraphExec_t> fp_graph, ve_graph;
    int part_vals = 2;

    float* x(int b) { return vec[b]; }
    float* sres() { return vec[3]; }
    float* u0() { return vec[4]; }
    float* u1() { return vec[5]; }
    float* r(int i) { return vec[6 + i]; }
    float* w(int i) { return vec[8 + i]; }
    float* s(int i) { return vec[10 + i]; }
    float* p() { return vec[12]; }
    float* dd() { return vec[13]; }

    ~Engine() { release(); }

    void release() {
        for (auto& kv : fp_graph) (void)hipGraphExecDestroy(kv.second);
        for (auto& kv : ve_graph) (void)hipGraphExecDestroy(kv.second);
        fp_graph.clear();
        ve_graph.clear();
        if (arena) (void)hipFree(arena);
        if (h_desc) (void)hipHostFree(h_desc);
        if (h_stat) (void)hipHostFree(h_stat);
        if (h_tile) (void)hipHostFree(h_tile);
        if (h_tile32) (void)hipHostFree(h_tile32);
        if (h_tile16r) (void)hipHostFree(h_tile16r);
        arena = nullptr;
        h_desc = nullptr;
        h_stat = nullptr;
        h_tile = nullptr;
        h_tile32 = nullptr;
        h_tile16r = nullptr;
    }

    // Allocates capacity for cap_img images, cap_px pixels, cap_tiles tiles.
    int init(redve_t hh, hipStream_t stream, int nimg, size_t npx, int ntiles) {
        h = hh;
        st = stream;
        L = h->method == REDVE_VE_NONE ? 1 : h->L;
        cap_img = nimg;
        cap_px = align64(npx);
        cap_tiles = (std::max(ntiles, 1) + kXcds - 1) / kXcds * kXcds;
        part_vals = std::max(L + 2, 2);
        px_alloc.cap = cap_px;
        tiles_used = 0;
        const size_t vbytes = cap_px * sizeof(float);
        size_t bytes = 0;
        auto take = [&](size_t n) {
            const size_t o = bytes;
            bytes += (n + 255) / 256 * 256;
            return o;
        };
        size_t o_vec[kVecs];
        for (int i = 0; i < kVecs; ++i) o_vec[i] = take(vbytes);
        const size_t o_U = take(vbytes * L);
        const size_t o_desc = take(sizeof(ImgDesc) * (cap_img + 1));
        const size_t o_tile = take(sizeof(TileRef) * cap_tiles);
        const size_t o_tile32 = take(sizeof(TileRef) * cap_tiles);
        const size_t o_tile16r = take(sizeof(TileRef) * cap_tiles);
        const size_t o_cg = take(sizeof(CgImg) * (cap_img + 1));
        const size_t o_part = take(sizeof(double) * (size_t)part_vals * cap_tiles);
        const size_t o_G = take(sizeof(double) * 256 * (cap_img + 1));
        const size_t o_info = take(sizeof(VeInfo) * (cap_img + 1));
        const size_t o_stat = take(sizeof(ImgStat) * (cap_img + 1));
        const size_t o_psf = take(sizeof(float) * 225 * (cap_img + 1));
        const size_t o_psf64 = take(sizeof(double) * 225 * (cap_img + 1));
        if (hipMalloc(&arena, bytes) != hipSuccess) {
            arena = nullptr;
            return REDVE_E_NOMEM;
        }
        char* b = (char*)arena;
        for (int i = 0; i < kVecs; ++i) vec[i] = (float*)(b + o_vec[i]);
        U = (float*)(b + o_U);
        d_desc = (ImgDesc*)(b + o_desc);
        d_tile = (TileRef*)(b + o_tile);
        d_tile32 = (TileRef*)(b + o_tile32);
        d_tile16r = (TileRef*)(b + o_tile16r);
        d_cg = (CgImg*)(b + o_cg);
        d_part = (double*)(b + o_part);
        d_G = (double*)(b + o_G);
        d_info = (VeInfo*)(b + o_info);
        d_stat = (ImgStat*)(b + o_stat);
        d_psf = (float*)(b + o_psf);
        d_psf64 = (double*)(b + o_psf64);
        if (hipHostMalloc((void**)&h_desc, sizeof(ImgDesc) * (cap_img + 1), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void**)&h_stat, sizeof(ImgStat) * (cap_img + 1), hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void**)&h_tile, sizeof(TileRef) * cap_tiles, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void**)&h_tile32, sizeof(TileRef) * cap_tiles, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void**)&h_tile16r, sizeof(TileRef) * cap_tiles, hipHostMallocDefault) !=
                hipSuccess)
            return REDVE_E_NOMEM;
        memset(h_desc, 0, sizeof(ImgDesc) * (cap_img + 1));
        memset(h_stat, 0, sizeof(ImgStat) * (cap_img + 1));
        // zero the whole arena once (outside any graph): window columns never hold garbage
        if (hipMemsetAsync(arena, 0, bytes, st) != hipSuccess) return REDVE_E_HIP;
        slots.assign(cap_img, Slot{});
        tiles_dirty = true;
        return REDVE_OK;
    }

    // Forgets every image (keeps buffers and graphs) for the next batch.
    void reset() {
        queue_err = hipSuccess;
        slots.assign(cap_img, Slot{});
        px_alloc.used.clear();
        tiles_used = 0;
        tiles_dirty = true;
    }

    static bool valid_item(const redve_item_t& it) {
        return it.y && it.x && it.hx >= 2 && it.wx >= 2 && it.psf && it.kh >= 1 && it.kw >= 1 &&
               (it.kh & 1) && (it.kw & 1) && it.kh <= REDVE_MAX_PSF && it.kw <= REDVE_MAX_PSF &&
               it.decim >= 1 && it.decim <= REDVE_MAX_DECIM && it.sigma > 0 &&
               std::isfinite(it.sigma) && it.lambda > 0 && std::isfinite(it.lambda) &&
               (long long)it.hx * it.wx <= (1LL << 30);
    }

    static size_t bytes_per_px(int L) { return sizeof(float) * (kVecs + L); }

    // Operator of one slot: rank-1 PSFs of radius <= 4 are zero-padded to 9x9 (exactly the
    // same sums: the extra taps add 0) so that every image can share the radius-4 stencil.
    void set_operator(int i, const redve_item_t& it) {
        Slot& sl = slots[i];
        LinOp op{};
        const int kh = it.kh, kw = it.kw;
        std::vector<float> pf(kh * kw);
        for (int k = 0; k < kh * kw; ++k) pf[k] = (float)it.psf[k];
        note(hipMemcpyAsync(d_psf + (size_t)i * 225, pf.data(), sizeof(float) * kh * kw,
                            hipMemcpyHostToDevice, st));
        note(hipMemcpyAsync(d_psf64 + (size_t)i * 225, it.psf, sizeof(double) * kh * kw,
                            hipMemcpyHostToDevice, st));
        note(hipStreamSynchronize(st));  // pf is a host temporary
        op.psf = d_psf + (size_t)i * 225;
        op.psf64 = d_psf64 + (size_t)i * 225;
        op.decim = it.decim;
        const double is2 = 1.0 / (it.sigma * it.sigma);
        op.inv_s2 = (float)is2;
        op.lambda = (float)it.lambda;
        op.inv_s2_d = is2;
        op.lambda_d = it.lambda;
        double l1 = 0.0;
        for (int k = 0; k < kh * kw; ++k) l1 += fabs(it.psf[k]);
        op.sd_mu = sd_step(h->sd_mu, l1, it.sigma, it.lambda);
        int im = 0;
        for (int k = 1; k < kh * kw; ++k)
            if (fabs(it.psf[k]) > fabs(it.psf[im])) im = k;
        const int ai = im / kw, bj = im % kw;
        const double amax = fabs(it.psf[im]);
        double col[REDVE_MAX_PSF], row[REDVE_MAX_PSF], err = 0.0;
        for (int a = 0; a < kh; ++a) col[a] = it.psf[a * kw + bj];
        for (int b = 0; b < kw; ++b) row[b] = amax > 0 ? it.psf[ai * kw + b] / it.psf[im] : 0.0;
        for (int a = 0; a < kh; ++a)
            for (int b = 0; b < kw; ++b) err = fmax(err, fabs(it.psf[a * kw + b] - col[a] * row[b]));
        op.separable = (amax > 0 && err <= 1e-12 * amax) ? 1 : 0;
        sl.padded = op.separable && kh <= 9 && kw <= 9;
        sl.cg32 = sl.padded && op.decim == 1;
        if (sl.padded) {
            op.kh = op.kw = 9;
            const int oh = 4 - kh / 2, ow = 4 - kw / 2;
            for (int a = 0; a < 9; ++a) {
                const double v = (a >= oh && a < oh + kh) ? col[a - oh] : 0.0;
                op.col_d[a] = v;
                op.col[a] = (float)v;
            }
            for (int b = 0; b < 9; ++b) {
                const double v = (b >= ow && b < ow + kw) ? row[b - ow] : 0.0;
                op.row_d[b] = v;
                op.row[b] = (float)v;
            }
        } else {
            op.kh = kh;
            op.kw = kw;
            for (int a = 0; a < kh; ++a) {
                op.col_d[a] = col[a];
                op.col[a] = (float)col[a];
            }
            for (int b = 0; b < kw; ++b) {
                op.row_d[b] = row[b];
                op.row[b] = (float)row[b];
            }
        }
        set_autocorrelations(op);
        sl.op = op;
    }

    // Places an item in a free slot; false if it does not fit now.
    bool admit(const redve_item_t& it, unsigned long long ticket, Clock::time_point t_submit,
               int& slot_out) {
        int i = -1;
        for (int k = 0; k < cap_img; ++k)
            if (!slots[k].used) {
                i = k;
                break;
            }
        if (i < 0) return false;
        const size_t npx = align64((size_t)it.hx * it.wx);
        const int nt = tiles_of(it.hx, it.wx);
        size_t off;
        if (tiles_used + nt > cap_tiles || !px_alloc.alloc(npx, off)) return false;
        tiles_used += nt;
        Slot& sl = slots[i];
        sl = Slot{};
        sl.used = sl.running = true;
        sl.item = it;
        sl.off = off;
        sl.npx = npx;
        sl.ntiles = nt;
        sl.ticket = ticket;
        sl.t_submit = t_submit;
        tiles_dirty = true;
        // a fresh CG state for the slot, then the operator (set_operator waits for the stream,
        // so both host-to-device copies are done before their host sources go away)
        CgImg z{};
        note(hipMemcpyAsync(d_cg + i, &z, sizeof(CgImg), hipMemcpyHostToDevice, st));
        set_operator(i, it);
        // initial vector: x0, y (deblurring) or decim^2 H^T y (needs the operator above)
        const size_t bytes = sizeof(float) * it.hx * it.wx;
        float* x0 = x(0) + off;
        if (it.x0)
            note(hipMemcpyAsync(x0, it.x0, bytes, hipMemcpyDeviceToDevice, st));
        else if (it.decim == 1)
            note(hipMemcpyAsync(x0, it.y, bytes, hipMemcpyDeviceToDevice, st));
        else {
            LinOp o2 = sl.op;
            o2.kh = it.kh;
            o2.kw = it.kw;
            if (!o2.psf || o2.decim != it.decim) {  // set_operator must have run
                px_alloc.release(off);
                tiles_used -= nt;
                sl = Slot{};
                return false;
            }
            launch_apply_Ht(o2, it.y, it.hx, it.wx, (float)(it.decim * it.decim), x0, st);
        }
        sl.cur = sl.base = 0;
        slot_out = i;
        return true;
    }

    void retire(int i) {
        Slot& sl = slots[i];
        const size_t bytes = sizeof(float) * sl.item.hx * sl.item.wx;
        note(hipMemcpyAsync(sl.item.x, x(sl.cur) + sl.off, bytes, hipMemcpyDeviceToDevice, st));
        px_alloc.release(sl.off);
        tiles_used -= sl.ntiles;
        tiles_dirty = true;
        sl.running = false;
        sl.finished = true;
    }

    static int third(int a, int b) {
        for (int k = 0; k < 3; ++k)
            if (k != a && k != b) return k;
        return 0;
    }

    // Builds the tile list: the running images' tiles in slot order get partial indices
    // 0..pos-1 (each image a contiguous range from its tile0); the list length B is a power of
    // two (at least 64, at most the capacity; both multiples of 8). Workgroup b runs on XCD
    // b mod 8; XCD x's workgroups take the x-th contiguous chunk of the live tiles, then padding.
    // The CG iterations but the last take two more lists, built the same way (length 0 when
    // empty): the 32x32 tiles of the images on that form, the 16x16 tiles of the others.
    int repack() {
        live.clear();
        live32.clear();
        live16r.clear();
        for (int i = 0; i < cap_img; ++i) {
            Slot& sl = slots[i];
            if (!sl.running) continue;
            sl.tile0 = (int)live.size();
            for (int t = 0; t < sl.ntiles; ++t) live.push_back(TileRef{i, t});
            if (takes_cg32(sl)) {
                const int n32 = tiles32_of(sl.item.hx, sl.item.wx);
                for (int t = 0; t < n32; ++t) live32.push_back(TileRef{i, t});
            } else {
                for (int t = 0; t < sl.ntiles; ++t) live16r.push_back(TileRef{i, t});
            }
        }
        launch_tiles = pack(live, h_tile);
        launch_tiles32 = live32.empty() ? 0 : pack(live32, h_tile32);
        launch_tiles16r = live16r.empty() ? 0 : pack(live16r, h_tile16r);
        if (hipMemcpyAsync(d_tile, h_tile, sizeof(TileRef) * launch_tiles, hipMemcpyHostToDevice,
                           st) != hipSuccess ||
            (launch_tiles32 && hipMemcpyAsync(d_tile32, h_tile32, sizeof(TileRef) * launch_tiles32,
                                              hipMemcpyHostToDevice, st) != hipSuccess) ||
            (launch_tiles16r &&
             hipMemcpyAsync(d_tile16r, h_tile16r, sizeof(TileRef) * launch_tiles16r,
                            hipMemcpyHostToDevice, st) != hipSuccess))
            return REDVE_E_HIP;
        return REDVE_OK;
    }

    // Dispatch order of a list of n live tiles padded to B (a power of two, at least 64, at most
    // the capacity): returns B.
    int pack(const std::vector<TileRef>& lv, TileRef* out) const {
        const int pos = (int)lv.size();
        int B = 64;
        while (B < pos) B *= 2;
        B = std::min(B, cap_tiles);
        const int nb = B / kXcds, q = pos / kXcds, r = pos % kXcds;
        for (int x = 0; x < kXcds; ++x) {
            const int start = x * q + std::min(x, r), len = q + (x < r ? 1 : 0);
            for (int i = 0; i < nb; ++i)
                out[x + kXcds * i] = i < len ? lv[start + i] : TileRef{cap_img, 0};
        }
        return B;
    }

    static int tiles32_of(int H, int W) { return ((H + 31) / 32) * ((W + 31) / 32); }

    // CG on the 32x32 tile list: a padded, undecimated operator, and at least one iteration
    // before the last (which runs on the 16x16 list for every image)
    bool takes_cg32(const Slot& sl) const {
        return sl.cg32 && h->base != REDVE_BASE_SD && h->cg_iters >= 2;
    }

    // The BF16 form with the switch to FP32 banks (one kernel takes each image's form).
    bool mixed() const {
        return h->precision == REDVE_PREC_BF16 && h->prec_switch > 0 && h->T > 0 &&
               tnrd_mfma_fits(h->F, h->J);
    }

    // The launches of one round (captured): denoiser stages, CG, differences + Gram, over the
    // first nt entries of the tile list.
    int record_fp(int rs, int nt, int nt32, int nt16r) {
        TnrdDev d = redve_tnrd_dev(h);
        const float* s_in = nullptr;
        if (h->T > 0) {
            const float* wprev = nullptr;
            for (int t = 0; t < h->T; ++t) {
                float* dst = (t == h->T - 1) ? sres() : ((t & 1) ? u1() : u0());
                if (mixed()) {
                    TnrdDev df = d;
                    df.precision = REDVE_PREC_FP32;
                    df.kwin = h->kwin32;
                    df.phi_tab = nullptr;
                    df.tab_n = 0;
                    launch_tnrd_stage_mixed_batch(d, df, t, d_desc, d_tile, nt, wprev, dst, 0, st);
                } else if (h->precision == REDVE_PREC_BF16) {
                    launch_tnrd_stage_bf16_batch(d, t, d_desc, d_tile, nt, wprev, dst, 0, st);
                } else {
                    launch_tnrd_stage_batch(d, t, d_desc, d_tile, nt, wprev, dst, 0, st);
                }
                wprev = dst;
            }
            s_in = sres();
        }
        const int n = h->cg_iters;
        if (h->base == REDVE_BASE_SD) {
            launch_sd_step_batch(d_desc, d_tile, nt, rs, s_in, st);
        } else if (n > 0) {
            launch_cg_init_fp_batch(d_desc, d_tile, nt, rs, s_in, r(0), st);
            launch_cg_w0_batch(d_desc, d_tile, nt, rs, r(0), w(0), d_part, cap_tiles, st);
            for (int k = 0; k < n; ++k) {
                const int a = k & 1, b = a ^ 1;
                launch_cg_fin_batch(d_desc, cap_img, k, d_part, cap_tiles, d_cg, st);
                if (k == n - 1) {  // the last iteration: every image on the 16x16 list
                    launch_cg_iter_batch(d_desc, d_tile, nt, rs, k, 1, d_cg, r(a), w(a), s(b),
                                         r(b), w(b), s(a), p(), dd(), d_part, cap_tiles, st);
                    continue;
                }
                if (nt16r > 0)
                    launch_cg_iter_batch(d_desc, d_tile16r, nt16r, rs, k, 0, d_cg, r(a), w(a),
                                         s(b), r(b), w(b), s(a), p(), dd(), d_part, cap_tiles, st);
                // the cg32 images: p_{k-1} in s(a), p_k to s(b), which the last iteration's
                // 16x16 kernel reads as its s_out
                if (nt32 > 0)
                    launch_cg_iter32_batch(d_desc, d_tile32, nt32, k, d_cg, r(a), s(a), r(b), s(b),
                                           dd(), d_part, cap_tiles, st);
            }
        }
        launch_diff_gram_batch(d_desc, d_tile, nt, L, U, cap_px, d_part, cap_tiles, st);
        launch_diff_fin_batch(d_desc, cap_img, L, d_part, cap_tiles, d_G, d_stat, st);
        return hipGetLastError() == hipSuccess ? REDVE_OK : REDVE_E_HIP;
    }

    int record_ve(int nt) {
        launch_ve_solve_batch(d_desc, cap_img, L, h->method, h->rank_eps, h->gamma_cap, d_G,
                              d_info, d_stat, st);
        launch_ve_combine_batch(d_desc, d_tile, nt, U, cap_px, d_info, st);
        return hipGetLastError() == hipSuccess ? REDVE_OK : REDVE_E_HIP;
    }

    int graph(std::map<GraphKey, hipGraphExec_t>& cache, GraphKey key, bool fp) {
        if (cache.count(key)) return REDVE_OK;
        hipGraph_t g;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return REDVE_E_HIP;
        const int rc = fp ? record_fp(std::get<0>(key), std::get<1>(key), std::get<2>(key),
                                      std::get<3>(key))
                          : record_ve(std::get<1>(key));
        if (hipStreamEndCapture(st, &g) != hipSuccess || rc) return REDVE_E_HIP;
        hipGraphExec_t ex;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return REDVE_E_HIP;
        cache[key] = ex;
        return REDVE_OK;
    }

    // Host-side consistency of what the next replay will read: every running image's
    // descriptor (buffers, ranges, operator) and the tile list. A failure here is a bug of the
    // engine; it is reported instead of being launched.
    bool valid_round() const {
        int pos = 0;
        for (int i = 0; i < cap_img; ++i) {
            const Slot& sl = slots[i];
            if (!sl.running) continue;
            const ImgDesc& d = h_desc[i];
            const LinOp& o = d.op;
            if (!d.active || !d.y || !d.x_in || !d.x_out || !d.x_m || d.H < 2 || d.W < 2 ||
                d.off + (size_t)d.H * d.W > cap_px || d.ntiles != tiles_of(d.H, d.W) ||
                d.tile0 != pos || d.wj >= L || !o.psf || !o.psf64 || o.decim < 1 ||
                o.decim > REDVE_MAX_DECIM || o.kh < 1 || o.kw < 1 || !(o.kh & 1) || !(o.kw & 1) ||
                o.kh > REDVE_MAX_PSF || o.kw > REDVE_MAX_PSF)
                return false;
            pos += d.ntiles;
        }
        if (pos > launch_tiles || launch_tiles > cap_tiles || launch_tiles % kXcds) return false;
        // every live tile exactly once, every other entry the inactive image
        std::vector<char> seen(pos, 0);
        for (int b = 0; b < launch_tiles; ++b) {
            const TileRef e = h_tile[b];
            if (e.img == cap_img) continue;
            if (e.img < 0 || e.img > cap_img || !slots[e.img].running || e.t < 0 ||
                e.t >= h_desc[e.img].ntiles)
                return false;
            const int pi = h_desc[e.img].tile0 + e.t;
            if (seen[pi]) return false;
            seen[pi] = 1;
        }
        for (char c : seen)
            if (!c) return false;
        // the 32x32 list: every 32x32 tile of the cg32 images exactly once, nothing else
        if (launch_tiles32 > cap_tiles || launch_tiles32 % kXcds) return false;
        std::fill(seen.begin(), seen.end(), 0);
        int want32 = 0, got32 = 0;
        for (int i = 0; i < cap_img; ++i)
            if (slots[i].running && h_desc[i].cg32) want32 += tiles32_of(h_desc[i].H, h_desc[i].W);
        if ((want32 > 0) != (launch_tiles32 > 0) || want32 > launch_tiles32) return false;
        for (int b = 0; b < launch_tiles32; ++b) {
            const TileRef e = h_tile32[b];
            if (e.img == cap_img) continue;
            if (e.img < 0 || e.img > cap_img || !slots[e.img].running || !h_desc[e.img].cg32 ||
                e.t < 0 || e.t >= tiles32_of(h_desc[e.img].H, h_desc[e.img].W))
                return false;
            const int pi = h_desc[e.img].tile0 + e.t;  // n32 <= ntiles: inside the image's range
            if (seen[pi]) return false;
            seen[pi] = 1;
            ++got32;
        }
        if (got32 != want32) return false;
        // the 16x16 list of the other images: each of their tiles exactly once, nothing else
        if (launch_tiles16r > cap_tiles || launch_tiles16r % kXcds) return false;
        std::fill(seen.begin(), seen.end(), 0);
        int want16r = 0, got16r = 0;
        for (int i = 0; i < cap_img; ++i)
            if (slots[i].running && !h_desc[i].cg32) want16r += h_desc[i].ntiles;
        if ((want16r > 0) != (launch_tiles16r > 0) || want16r > launch_tiles16r) return false;
        for (int b = 0; b < launch_tiles16r; ++b) {
            const TileRef e = h_tile16r[b];
            if (e.img == cap_img) continue;
            if (e.img < 0 || e.img > cap_img || !slots[e.img].running || h_desc[e.img].cg32 ||
                e.t < 0 || e.t >= h_desc[e.img].ntiles)
                return false;
            const int pi = h_desc[e.img].tile0 + e.t;
            if (seen[pi]) return false;
            seen[pi] = 1;
            ++got16r;
        }
        if (got16r != want16r) return false;
        return !h_desc[cap_img].active;
    }

    bool any_running() const {
        for (auto& sl : slots)
            if (sl.running) return true;
        return false;
    }

    // One FP call for every running slot, extrapolation for those completing a window, and the
    // Algorithm 3 bookkeeping. Returns an error code for HIP failures only.
    int round() {
        if (queue_err != hipSuccess) return REDVE_E_HIP;
        const int m = h->m;
        const bool ve = h->method != REDVE_VE_NONE;
        bool all_padded = true, any_ve = false;
        for (int i = 0; i <= cap_img; ++i) h_desc[i].active = 0;
        for (int i = 0; i < cap_img; ++i) {
            Slot& sl = slots[i];
            if (!sl.running) continue;
            all_padded = all_padded && sl.padded;
            sl.in_window = ve && !sl.extra && sl.phase >= m;
            const int wj = sl.in_window ? sl.phase - m : -1;
            sl.do_ve = sl.in_window && wj == L - 1;
            sl.next = third(sl.cur, sl.in_window ? sl.base : sl.cur);
            any_ve = any_ve || sl.do_ve;
            ImgDesc& d = h_desc[i];
            d.H = sl.item.hx;
            d.W = sl.item.wx;
            d.ntiles = sl.ntiles;
            d.active = 1;
            d.wj = ve ? wj : -1;
            d.do_ve = sl.do_ve ? 1 : 0;
            d.off = sl.off;
            d.y = sl.item.y;
            d.x_in = x(sl.cur) + sl.off;
            d.x_out = x(sl.next) + sl.off;
            d.x_m = x(sl.base) + sl.off;
            d.op = sl.op;
            d.fp32_banks = sl.finish_fp32 ? 1 : 0;
            d.cg32 = takes_cg32(sl) ? 1 : 0;
        }
        const int rs = all_padded ? 4 : 0;
        int rc;
        if (tiles_dirty) {
            if ((rc = repack())) return rc;
            tiles_dirty = false;
        }
        for (int i = 0; i < cap_img; ++i)
            if (slots[i].running) h_desc[i].tile0 = slots[i].tile0;
        if (!valid_round()) return REDVE_E_STATE;
        if (hipMemcpyAsync(d_desc, h_desc, sizeof(ImgDesc) * (cap_img + 1), hipMemcpyHostToDevice,
                           st) != hipSuccess)
            return REDVE_E_HIP;
        const GraphKey kf{rs, launch_tiles, launch_tiles32, launch_tiles16r},
            kv{0, launch_tiles, 0, 0};
        if ((rc = graph(fp_graph, kf, true))) return rc;
        if (hipGraphLaunch(fp_graph[kf], st) != hipSuccess) return REDVE_E_HIP;
        if (any_ve) {
            if ((rc = graph(ve_graph, kv, false))) return rc;
            if (hipGraphLaunch(ve_graph[kv], st) != hipSuccess) return REDVE_E_HIP;
        }
        if (hipMemcpyAsync(h_stat, d_stat, sizeof(ImgStat) * cap_img, hipMemcpyDeviceToHost, st) !=
            hipSuccess)
            return REDVE_E_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return REDVE_E_HIP;
        // Algorithm 3 bookkeeping per slot
        for (int i = 0; i < cap_img; ++i) {
            Slot& sl = slots[i];
            if (!sl.running) continue;
            const ImgStat& s = h_stat[i];
            sl.calls++;
            sl.delta = sqrt(s.uu / s.xx);
            // BF16 form: FP32 banks once the relative change falls below the switch (tested
            // at every call without extrapolation, at cycle ends with it, as in the solve)
            const bool test_now = !ve || sl.do_ve;
            if (test_now && mixed() && sl.delta < h->prec_switch) sl.finish_fp32 = true;
            sl.cur = sl.next;
            bool stop = false;
            if (sl.extra) {
                if (--sl.extra_left <= 0) stop = true;
            } else if (!ve) {
                if ((sl.status = sl.prog.check(sl.delta))) stop = true;
                else if (sl.delta < h->tol || sl.calls >= h->max_fp) stop = true;
                if (stop && sl.status == REDVE_OK && h->extra_fp > 0) {
                    stop = false;
                    sl.extra = true;
                    sl.extra_left = h->extra_fp;
                }
            } else {
                sl.phase++;
                if (sl.phase == m && m > 0) sl.base = sl.cur;
                if (sl.do_ve) {
                    sl.cycles++;
                    if (s.breakdown)
                        sl.breakdowns++;
                    else
                        sl.gl1max = std::max(sl.gl1max, s.gamma_l1);
                    if (s.guarded) sl.rejected++;
                    sl.cur = sl.base;  // x_(m,kappa) was combined into the window base
                    sl.phase = 0;
                    if (!s.guarded && !std::isfinite(s.gamma_l1)) sl.status = REDVE_E_NONFINITE;
                    else sl.status = sl.prog.check(sl.delta);
                    if (sl.status || sl.delta < h->tol || sl.calls >= h->max_fp) stop = true;
                } else if (sl.calls >= h->max_fp) {
                    stop = true;  // budget ends inside a cycle: the last FP iterate
                }
                if (sl.phase == 0 && !stop) sl.base = sl.cur;
                if (stop && sl.status == REDVE_OK && h->extra_fp > 0) {
                    stop = false;
                    sl.extra = true;
                    sl.extra_left = h->extra_fp;
                }
            }
            if (stop) retire(i);
        }
        return REDVE_OK;
    }

    void fill_stats(const Slot& sl, redve_stats_t* st) const {
        st->fp_calls = sl.calls;
        st->cycles = sl.cycles;
        st->breakdowns = sl.breakdowns;
        st->rejected = sl.rejected;
        st->status = sl.status;
        st->final_delta = sl.delta;
        st->max_gamma_l1 = sl.gl1max;
        st->ms = sl.ms;
    }
};

int check_settings(redve_t h) {
    if (!h->have_den) {
        h->err = "redve_set_denoiser was not called";
        return REDVE_E_STATE;
    }
    if (h->base == REDVE_BASE_FP && h->cg_iters < 1) {
        h->err = "the batched FP iteration needs cg_iters >= 1";
        return REDVE_E_ARG;
    }
    if (h->lin != REDVE_LIN_CG) {
        h->err = "the batched engine solves the linear step with CG";
        return REDVE_E_ARG;
    }
    return REDVE_OK;
}

}  // namespace

// ======================================================================================
// Batched solve
// ======================================================================================

extern "C" int redve_solve_batch(redve_t h, int n, const redve_item_t* items, redve_stats_t* st) {
    if (!h) return REDVE_E_ARG;
    if (n < 1 || !items) {
        h->err = "need n >= 1 items";
        return REDVE_E_ARG;
    }
    int rc = check_settings(h);
    if (rc) return rc;
    size_t npx = 0;
    int ntiles = 0;
    for (int i = 0; i < n; ++i) {
        if (!Engine::valid_item(items[i])) {
            h->err = "batch item " + std::to_string(i) + " is invalid";
            return REDVE_E_ARG;
        }
        npx += align64((size_t)items[i].hx * items[i].wx);
        ntiles += tiles_of(items[i].hx, items[i].wx);
    }
    if (hipSetDevice(h->device) != hipSuccess) return REDVE_E_HIP;
    // non-blocking: work on the legacy null stream (any thread) must not implicitly join a
    // stream while a round is being captured on it; ordering is explicit (synchronisations)
    if (!h->bstream && hipStreamCreateWithFlags(&h->bstream, hipStreamNonBlocking) != hipSuccess)
        return REDVE_E_HIP;
    // inputs were produced on the caller's stream
    if (hipStreamSynchronize(h->stream) != hipSuccess) return REDVE_E_HIP;
    const auto t0 = Clock::now();
    // the engine (workspace + captured graphs) is kept in the handle while the settings stay
    // the same and the batch fits its capacity
    Engine* eng = (Engine*)h->batch;
    if (eng && !(eng->gen == h->gen && eng->cap_img >= n && eng->cap_px >= npx &&
                 eng->cap_tiles >= ntiles)) {
        delete eng;
        eng = nullptr;
        h->batch = nullptr;
    }
    if (eng) {
        eng->reset();
    } else {
        eng = new Engine();
        if ((rc = eng->init(h, h->bstream, n, npx, ntiles))) {
            delete eng;
            h->err = "batch workspace allocation failed";
            return rc;
        }
        eng->gen = h->gen;
        h->batch = eng;
        h->batch_free = [](void* p) { delete (Engine*)p; };
    }
    auto drop = [&](int code, const char* msg) {
        delete eng;
        h->batch = nullptr;
        h->err = msg;
        return code;
    };
    for (int i = 0; i < n; ++i) {
        int slot;
        if (!eng->admit(items[i], (unsigned long long)i, t0, slot) || slot != i)
            return drop(REDVE_E_STATE, "internal: batch item did not fit its own capacity");
    }
    while (eng->any_running()) {
        if ((rc = eng->round()))
            return drop(rc, rc == REDVE_E_STATE ? "internal: inconsistent batched round (not launched)"
                                                : "HIP failure in a batched round");
    }
    if (hipStreamSynchronize(h->bstream) != hipSuccess || eng->queue_err != hipSuccess)
        return drop(REDVE_E_HIP, "HIP failure");
    const double ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    int worst = REDVE_OK;
    for (int i = 0; i < n; ++i) {
        eng->slots[i].ms = ms;
        if (st) eng->fill_stats(eng->slots[i], st + i);
        if (eng->slots[i].status && !worst) worst = eng->slots[i].status;
    }
    if (worst) h->err = "at least one batch item did not converge (see its status)";
    return worst;
}

// ======================================================================================
// Serving
// ======================================================================================

struct redve_server {
    redve_ctx ctx;               // private copy of the settings, own stream and workspace
    Engine eng;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    hipStream_t caller = nullptr;  // the prototype's stream: requests' inputs are made there
    struct Req {
        redve_item_t item;
        std::vector<double> psf;  // copied at submit
        unsigned long long ticket;
        Clock::time_point t_submit;
        hipEvent_t ready;  // recorded on the caller's stream at submit
    };
    std::deque<Req> queue;
    std::map<unsigned long long, redve_stats_t> results;
    unsigned long long next_ticket = 1;
    bool stop = false;
    int max_active = 0;
    int active = 0;  // running requests (the worker's count, published under mu)
    long long rounds = 0;
    int error = REDVE_OK;
    size_t peak_px = 0;       // most pixels admitted at once (allocated ranges, 64-aligned)
    long long waited = 0;     // rounds run while a request waited in the queue

    // The worker: admits queued requests in arrival order while the head fits (slots, device
    // memory, tiles), runs one round, publishes finished requests. Engine state is touched by
    // this thread only; everything the API functions read is published under mu.
    void run() {
        eng.note(hipSetDevice(ctx.device));  // a failure fails the first round
        while (true) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !queue.empty() || active > 0; });
                if (stop && queue.empty() && active == 0) break;
                while (!queue.empty() && active < max_active) {
                    int slot;
                    Req& q = queue.front();
                    q.item.psf = q.psf.data();
                    eng.note(hipStreamWaitEvent(eng.st, q.ready, 0));  // inputs: caller's stream
                    if (!eng.admit(q.item, q.ticket, q.t_submit, slot)) break;
                    (void)hipEventDestroy(q.ready);
                    queue.pop_front();
                    ++active;
                }
                size_t px = 0;
                for (const auto& sl : eng.slots)
                    if (sl.used) px += (sl.npx + 63) / 64 * 64;
                peak_px = std::max(peak_px, px);
                if (!queue.empty() && active > 0) ++waited;
            }
            if (active == 0) continue;  // cannot happen: an empty engine admits any queued head
            int rc = eng.round();
            if (rc == REDVE_OK) eng.note(hipStreamSynchronize(eng.st));  // the retire copies
            if (rc == REDVE_OK && eng.queue_err != hipSuccess) rc = REDVE_E_HIP;
            std::lock_guard<std::mutex> lk(mu);
            ++rounds;
            if (rc) {
                // fail every running and queued request; the server takes no more work
                error = rc;
                for (auto& sl : eng.slots)
                    if (sl.running) {
                        sl.running = false;
                        sl.status = rc;
                        sl.finished = true;
                    }
                for (auto& q : queue) {
                    redve_stats_t s{};
                    s.status = rc;
                    results[q.ticket] = s;
                    (void)hipEventDestroy(q.ready);
                }
                queue.clear();
            }
            for (auto& sl : eng.slots) {
                if (sl.used && sl.finished) {
                    sl.ms = std::chrono::duration<double, std::milli>(Clock::now() - sl.t_submit).count();
                    redve_stats_t s{};
                    eng.fill_stats(sl, &s);
                    results[sl.ticket] = s;
                    sl.used = false;
                    sl.finished = false;
                    --active;
                }
            }
            done_cv.notify_all();
        }
    }
};

extern "C" int redve_server_create(redve_server_t* out, redve_t proto, size_t hbm_budget,
                                   int max_active) {
    if (!out || !proto || max_active < 1 || max_active > 4096) return REDVE_E_ARG;
    *out = nullptr;
    if (!proto->have_den) return REDVE_E_STATE;
    if (proto->base == REDVE_BASE_FP && proto->cg_iters < 1) return REDVE_E_ARG;
    if (proto->lin != REDVE_LIN_CG) return REDVE_E_ARG;
    auto s = std::make_unique<redve_server>();
    // copy the settings; device buffers of the denoiser are shared read-only with proto
    redve_ctx& c = s->ctx;
    c.device = proto->device;
    c.T = proto->T;
    c.F = proto->F;
    c.J = proto->J;
    c.precision = proto->precision;
    c.kwin = proto->kwin;
    c.mu0 = proto->mu0;
    c.dmu = proto->dmu;
    c.gamma = proto->gamma;
    c.theta = proto->theta;
    c.d_filt = proto->d_filt;
    c.d_rbfw = proto->d_rbfw;
    c.d_frag = proto->d_frag;
    c.d_frag32 = proto->d_frag32;
    c.d_phitab = proto->d_phitab;
    c.tab_n = proto->tab_n;
    c.tab_lo = proto->tab_lo;
    c.tab_h = proto->tab_h;
    c.lds_max = proto->lds_max;
    c.have_den = true;
    c.method = proto->method;
    c.L = proto->L;
    c.m = proto->m;
    c.cg_iters = proto->cg_iters;
    c.max_fp = proto->max_fp;
    c.extra_fp = proto->extra_fp;
    c.tol = proto->tol;
    c.rank_eps = proto->rank_eps;
    c.gamma_cap = proto->gamma_cap;
    c.prec_switch = proto->prec_switch;
    c.kwin32 = proto->kwin32;
    c.base = proto->base;
    c.sd_mu = proto->sd_mu;
    if (hipSetDevice(c.device) != hipSuccess) return REDVE_E_HIP;
    // non-blocking (see redve_solve_batch); inputs are ordered by an event per request
    if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) return REDVE_E_HIP;
    s->caller = proto->stream;
    const int L = c.method == REDVE_VE_NONE ? 1 : c.L;
    const size_t per_px = Engine::bytes_per_px(L);
    const size_t cap_px = hbm_budget / per_px;
    if (cap_px < 64 * 64) {
        (void)hipStreamDestroy(c.stream);
        return REDVE_E_ARG;
    }
    s->max_active = max_active;
    // tiles: a request of p pixels needs (h / 16 + 1)(w / 16 + 1) <= p / 256 + (h + w) / 16 + 1;
    // requests thinner than 4 pixels may need more than cap_px / 64 and are refused at submit
    const int cap_tiles = (int)std::min<size_t>(cap_px / 64 + 64 * (size_t)max_active, 1 << 26);
    if (s->eng.init(&c, c.stream, max_active, cap_px, cap_tiles)) {
        (void)hipStreamDestroy(c.stream);
        return REDVE_E_NOMEM;
    }
    redve_server* raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return REDVE_OK;
}

extern "C" int redve_server_submit(redve_server_t s, const redve_item_t* item,
                                   unsigned long long* ticket) {
    if (!s || !item || !ticket) return REDVE_E_ARG;
    if (!Engine::valid_item(*item)) return REDVE_E_ARG;
    // a request must fit the empty engine, or it could never be admitted
    if ((size_t)item->hx * item->wx + 64 > s->eng.cap_px ||
        tiles_of(item->hx, item->wx) > s->eng.cap_tiles)
        return REDVE_E_NOMEM;
    if (hipSetDevice(s->ctx.device) != hipSuccess) return REDVE_E_HIP;
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return REDVE_E_HIP;
    if (hipEventRecord(ev, s->caller) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return REDVE_E_HIP;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error) {
        (void)hipEventDestroy(ev);
        return s->error;
    }
    *ticket = s->next_ticket++;
    redve_server::Req q;
    q.ready = ev;
    q.item = *item;
    q.psf.assign(item->psf, item->psf + (size_t)item->kh * item->kw);
    q.item.psf = nullptr;
    q.ticket = *ticket;
    q.t_submit = Clock::now();
    s->queue.push_back(std::move(q));
    s->cv.notify_all();
    return REDVE_OK;
}

extern "C" int redve_server_poll(redve_server_t s, unsigned long long ticket, int* done,
                                 redve_stats_t* st) {
    if (!s || !done) return REDVE_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    *done = it != s->results.end();
    if (*done && st) *st = it->second;
    return REDVE_OK;
}

extern "C" int redve_server_wait(redve_server_t s, unsigned long long ticket, redve_stats_t* st) {
    if (!s) return REDVE_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket) return REDVE_E_ARG;
    s->done_cv.wait(lk, [&] { return s->results.count(ticket) > 0; });
    if (st) *st = s->results[ticket];
    return REDVE_OK;
}

extern "C" int redve_server_counts(redve_server_t s, int* queued, int* active, int* finished,
                                   long long* rounds) {
    if (!s) return REDVE_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int)s->queue.size();
    if (active) *active = s->active;
    if (finished) *finished = (int)s->results.size();
    if (rounds) *rounds = s->rounds;
    return REDVE_OK;
}

extern "C" int redve_server_occupancy(redve_server_t s, size_t* capacity_px, size_t* peak_px,
                                      long long* waited_rounds) {
    if (!s) return REDVE_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (capacity_px) *capacity_px = s->eng.cap_px;
    if (peak_px) *peak_px = s->peak_px;
    if (waited_rounds) *waited_rounds = s->waited;
    return REDVE_OK;
}

extern "C" int redve_server_destroy(redve_server_t s) {
    if (!s) return REDVE_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx.device);
    (void)hipStreamSynchronize(s->ctx.stream);
    s->eng.release();
    (void)hipStreamDestroy(s->ctx.stream);
    // the denoiser buffers belong to the prototype handle
    s->ctx.d_filt = nullptr;
    s->ctx.d_rbfw = nullptr;
    s->ctx.d_frag = nullptr;
    s->ctx.d_frag32 = nullptr;
    s->ctx.d_phitab = nullptr;
    delete s;
    return REDVE_OK;
}
