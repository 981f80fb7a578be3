// Deterministic FP64 workgroup and grid reductions for wave64 (gfx950).
//
// Order of summation is fixed by the data-to-thread mapping, the butterfly order inside a
// wavefront and the wave order inside a workgroup; the grid stage sums per-workgroup partials
// in workgroup-index order. Results are therefore bitwise reproducible run to run.
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

// Publishes this workgroup's NV partials (held by thread 0) and returns true in every thread
// of the workgroup that completes the grid. In that workgroup, thread 0 then holds the grid
// totals in `tot` (summed over workgroups 0..nblk-1 in order) and the counter is re-armed.
template <int NV>
__device__ inline bool grid_sum(const double (&v)[NV], double (&tot)[NV], Reduction red,
                                int blk, int nblk, double* scratch) {
    __shared__ int s_last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red.partials[(size_t)k * red.capacity + blk] = v[k];
        unsigned prev = __hip_atomic_fetch_add(red.counter, 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (unsigned)(nblk - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nblk; i += kThreads)
            s += red.partials[(size_t)k * red.capacity + i];
        acc[k] = s;
    }
    block_sum<NV>(acc, scratch);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] = acc[k];
        __hip_atomic_store(red.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

}  // namespace redve
