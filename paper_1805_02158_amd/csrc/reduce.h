// Deterministic FP64 reductions for wave64 (gfx950) without atomics or fences.
//
// A grid-wide sum is split across a kernel boundary: the producing kernel writes one FP64
// partial per workgroup (plain stores), and every workgroup of the consuming kernel re-sums
// those partials itself, in workgroup-index order. The kernel boundary makes the partials
// visible, so no device-scope atomic, fence or last-workgroup protocol is needed; every
// consumer workgroup computes the bitwise-identical total. The order of summation is fixed by
// the data-to-thread mapping, the DPP scan inside a wavefront and the wave order inside a
// workgroup, so results are reproducible run to run.
#pragma once

#include "internal.h"

namespace redve {

// One DPP move of both halves of a double (bound_ctrl: lanes whose source is outside the row,
// and rows outside ROW_MASK, read zero).
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active), returned in every lane: an
// inclusive scan by DPP row shifts (1, 2, 4, 8 lanes) and the two row broadcasts (lane 15
// into the next row, lane 31 into rows 2 and 3), after which lane 63 holds the total. Cross-
// lane moves without the LDS unit; a fixed order of additions.
__device__ inline double wave_sum(double v) {
    v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
    v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
    v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
    v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
    v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15
    v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sums NV values across a workgroup of NTH threads; the result is valid in thread 0 only.
// Only the first NACT threads may hold nonzero values (the other waves skip the wave sums).
template <int NV, int NTH = kThreads, int NACT = NTH>
__device__ inline void block_sum(double (&v)[NV], double* scratch /* NV * NACT/64 */) {
    constexpr int NW = NACT / 64;
    static_assert(NACT % 64 == 0 && NACT <= NTH, "active waves");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w < NW) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double s = wave_sum(v[k]);
            if (lane == 0) scratch[k * NW + w] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int i = 0; i < NW; ++i) s += scratch[k * NW + i];
            v[k] = s;
        }
    }
    __syncthreads();
}

// block_sum and publish of many values at once: every active thread stores its NV values to
// LDS, then wave v < NV sums value v (lane l adds the values of threads l, l + 64, ... in that
// order, then the DPP wave sum) and writes it to part[v * stride + blk]. One DPP sum per wave,
// in parallel over the values, instead of NV sums in a row in each active wave.
template <int NV, int NTH, int NACT>
__device__ inline void block_sum_publish(const double (&v)[NV], double* scratch /* NV * NACT */,
                                         double* part, int stride, int blk) {
    static_assert(NACT % 64 == 0 && NACT <= NTH && NV <= NTH / 64, "one wave per value");
    if ((int)threadIdx.x < NACT) {
#pragma unroll
        for (int k = 0; k < NV; ++k) scratch[k * NACT + threadIdx.x] = v[k];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w < NV) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NACT / 64; ++i) s += scratch[w * NACT + i * 64 + lane];
        s = wave_sum(s);
        if (lane == 0) part[(size_t)w * stride + blk] = s;
    }
}

// Writes this workgroup's NV partials (valid in thread 0) to part[k * stride + blk].
template <int NV>
__device__ inline void publish(const double (&v)[NV], double* part, int stride, int blk) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[(size_t)k * stride + blk] = v[k];
    }
}

// Total of n partials, summed by the first wave in a fixed order and broadcast to the whole
// workgroup. Call from every thread (contains a workgroup barrier).
__device__ inline double consume(const double* part, int n, double* bcast /* one double */) {
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += 64) s += part[i];
        s = wave_sum(s);
        if (threadIdx.x == 0) *bcast = s;
    }
    __syncthreads();
    const double r = *bcast;
    __syncthreads();
    return r;
}

// Totals of two partial arrays (part[i] and part[stride + i]) in one pass: the same sums, in
// the same order, as two calls of consume, with one memory latency instead of two.
__device__ inline void consume2(const double* part, int stride, int n, double* bcast /* two */,
                                double& a, double& b) {
    if (threadIdx.x < 64) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = threadIdx.x; i < n; i += 64) {
            s0 += part[i];
            s1 += part[stride + i];
        }
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        if (threadIdx.x == 0) {
            bcast[0] = s0;
            bcast[1] = s1;
        }
    }
    __syncthreads();
    a = bcast[0];
    b = bcast[1];
    __syncthreads();
}

// consume2 split in two for at most 4 * 64 partials: the loads (wave 0, four per lane), to be
// issued before the caller's other loads so that waiting for them does not also wait for
// those, and the sums. The same sums, in the same order, as consume2 (absent partials add an
// exact zero).
struct Early2 {
    double a[4], b[4];
};
constexpr int kEarlyPartials = 4 * 64;

__device__ inline void consume2_issue(const double* part, int stride, int n, Early2& q) {
    if (threadIdx.x < 64) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = threadIdx.x + 64 * i;
            q.a[i] = j < n ? part[j] : 0.0;
            q.b[i] = j < n ? part[stride + j] : 0.0;
        }
    }
}

__device__ inline void consume2_finish(const Early2& q, double* bcast /* two */, double& a,
                                       double& b) {
    if (threadIdx.x < 64) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            s0 += q.a[i];
            s1 += q.b[i];
        }
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        if (threadIdx.x == 0) {
            bcast[0] = s0;
            bcast[1] = s1;
        }
    }
    __syncthreads();
    a = bcast[0];
    b = bcast[1];
    __syncthreads();
}

}  // namespace redve
