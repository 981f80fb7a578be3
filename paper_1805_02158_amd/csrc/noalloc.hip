// Vector extrapolation without device allocation: the variant of redve_extrapolate for callers
// that cannot allocate (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc). It runs the same kernels in the same order as redve_extrapolate
// (difference passes with their FP64 Gram partials, the small solve, the combination;
// Algorithm 1 / eq. (19) / SVD-MPE of Sec. III-B), with the difference columns, the partials
// and the small solve's result in one fixed device array of this file instead of the handle's
// workspace.
//
// The array is resolved to a device address once per device at handle creation
// (hipGetSymbolAddress with that device current); host code only ever passes that address,
// never the array's name, to kernels and copies.
#include <mutex>
#include <string>

#include "../../include/redve.h"
#include "internal.h"
#include "context.h"

using namespace redve;

namespace {

constexpr size_t kScratchBytes = REDVE_NOALLOC_SCRATCH_BYTES;
constexpr size_t kAlignBytes = 256;
constexpr size_t align_up(size_t x) { return (x + kAlignBytes - 1) / kAlignBytes * kAlignBytes; }

// Layout: the window partials for the largest window (column j at j * win_stride, win_stride =
// (REDVE_MAX_L + 1) kMaxRedBlocks doubles), the small solve's VeInfo, then the columns of U.
constexpr size_t kWinStride = (size_t)(REDVE_MAX_L + 1) * kMaxRedBlocks;
constexpr size_t kPartBytes = align_up((size_t)REDVE_MAX_L * kWinStride * sizeof(double));
constexpr size_t kInfoOff = kPartBytes;
constexpr size_t kUOff = kInfoOff + align_up(sizeof(VeInfo));
static_assert(kUOff < kScratchBytes, "scratch too small for its fixed part");

// The library's fixed scratch array. Each GPU holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

int fail(redve_t h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

}  // namespace

// Resolves the scratch array's address on `device` (the current device) once; called by
// redve_create.
int redve_noalloc_resolve(int device) {
    if (device < 0 || device >= kMaxDevices) return REDVE_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return REDVE_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return REDVE_E_HIP;
    g_scratch[device] = p;
    return REDVE_OK;
}

extern "C" {

size_t redve_extrapolate_noalloc_max(int L) {
    if (L < 2 || L > REDVE_MAX_L) return 0;
    return (kScratchBytes - kUOff) / ((size_t)L * sizeof(float));
}

int redve_extrapolate_noalloc(redve_t h, const float* xs, int L, int hx, int wx, float* out,
                              double* gamma, int* breakdown) {
    if (!h) return REDVE_E_ARG;
    if (!xs || !out) return fail(h, REDVE_E_ARG, "null pointer");
    if (L < 2 || L > REDVE_MAX_L) return fail(h, REDVE_E_ARG, "L must be 2..16");
    if (h->method == REDVE_VE_NONE) return fail(h, REDVE_E_STATE, "no extrapolation method set");
    if (hx < 2 || wx < 2) return fail(h, REDVE_E_ARG, "image sides must be >= 2");
    const size_t n = (size_t)hx * wx;
    if (n > redve_extrapolate_noalloc_max(L))
        return fail(h, REDVE_E_ARG,
                    "image too large for the fixed scratch: L * h * w must be at most " +
                        std::to_string((kScratchBytes - kUOff) / sizeof(float)) + " (got " +
                        std::to_string((size_t)L * n) + ")");
    if (h->device < 0 || h->device >= kMaxDevices || !g_scratch[h->device])
        return fail(h, REDVE_E_STATE, "scratch address not resolved for this device");
    if (hipSetDevice(h->device) != hipSuccess) return fail(h, REDVE_E_HIP, "hipSetDevice failed");
    char* base = (char*)g_scratch[h->device];
    double* part = (double*)base;
    VeInfo* info = (VeInfo*)(base + kInfoOff);
    float* U = (float*)(base + kUOff);
    // every partial the small solve reads and every VeInfo field the combination reads are
    // written by this call's kernels, so nothing is cleared
    int nblk = 1;
    for (int j = 0; j < L; ++j)
        nblk = launch_diff_gram(xs + (size_t)(j + 1) * n, xs + (size_t)j * n, U, j, (int)n,
                                part + j * kWinStride, h->stream);
    launch_ve_solve(part, kWinStride, nblk, L, h->method, h->rank_eps, h->gamma_cap, info,
                    h->stream);
    launch_ve_combine(xs, U, (int)n, info, out, h->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(h, REDVE_E_HIP, std::string("launch: ") + hipGetErrorString(e));
    e = hipMemcpyAsync(&h->host->info, info, sizeof(VeInfo), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, REDVE_E_HIP, std::string("read-back: ") + hipGetErrorString(e));
    if (gamma)
        for (int j = 0; j < L; ++j) gamma[j] = h->host->info.gamma[j];
    if (breakdown) *breakdown = h->host->info.breakdown;
    return REDVE_OK;
}

}  // extern "C"
