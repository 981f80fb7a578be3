// Deterministic FP64 reductions for wave64 (gfx950) without atomics or fences.
//
// A grid-wide sum is split across a kernel boundary: the producing kernel writes one FP64
// partial per workgroup (plain stores), and every workgroup of the consuming kernel re-sums
// those partials itself, in workgroup-index order. The kernel boundary makes the partials
// visible, so no device-scope atomic, fence or last-workgroup protocol is needed; every
// consumer workgroup computes the bitwise-identical total. The order of summation is fixed by
// the data-to-thread mapping, the butterfly inside a wavefront and the wave order inside a
// workgroup, so results are reproducible run to run.
#pragma once

#include "internal.h"

namespace redve {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums NV values across the workgroup; the result is valid in thread 0 only.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* scratch /* NV * kThreads/64 */) {
    constexpr int NW = kThreads / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) scratch[k * NW + w] = s;
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

}  // namespace redve
