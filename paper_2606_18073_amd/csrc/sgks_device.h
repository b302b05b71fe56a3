// Device helpers shared by the kernel sources (sgks_kernels.hip, sgks_gks.hip).
// Not part of the public ABI.
#pragma once

#include "sgks_internal.h"

namespace sgks {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum over a block of blockDim.x (multiple of 64) threads; every thread gets
// the same total (the per-wave sums are added in wave order).
__device__ inline double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Sum of p[0], p[stride], ..., p[(n-1) stride] in that order, sixteen
// independent loads in flight at a time (the small kernels are latency
// bound: a load-then-add loop would pay one memory latency per term).
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int64_t stride,
                                              int n) {
    // loads are unconditional from clamped (valid) addresses so that all
    // sixteen are issued before the first wait; the mask applies to values
    double acc = 0.0;
    for (int k = 0; k < n; k += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = p[(int64_t)min(k + u, n - 1) * stride];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (k + u < n) acc += v[u];
    }
    return acc;
}

// sum_k p[k stride] v[k], k < n, in order, sixteen loads in flight
// Thread-strided sum of p[i], i = threadIdx.x, threadIdx.x + T, ... < n,
// eight loads in flight (per-thread order fixed).
__device__ __forceinline__ double thread_strided_sum(const double* __restrict__ p, int n, int T) {
    const int tid = threadIdx.x;
    const int cnt = tid < n ? (n - tid + T - 1) / T : 0;
    return strided_sum(p + tid, T, cnt);
}

// ---------------------------------------------------------------------------
// batched launches: workgroup -> (problem, local workgroup)
// ---------------------------------------------------------------------------

struct Slot {
    int p;      // problem
    int blk;    // workgroup within the problem
    int nblk;   // workgroups of the problem
};

// One problem: the grid is the problem's.  Several: binary search of the
// prefix table in the kernel-argument segment (a few scalar loads).
__device__ __forceinline__ Slot find_slot(const BTab& t) {
    const int b = blockIdx.x;
    if (t.np == 1) return Slot{0, b, t.pref[1]};
    int lo = 0, hi = t.np;   // pref[lo] <= b < pref[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b >= t.pref[mid])
            lo = mid;
        else
            hi = mid;
    }
    return Slot{lo, b - t.pref[lo], t.pref[lo + 1] - t.pref[lo]};
}

// The States are read-only while any kernel runs, so they are read through the
// constant address space: the fields become scalar loads and every pointer
// loaded from them is known to address global memory (global, not flat,
// memory instructions in the loops that use it).
__device__ __forceinline__ State load_state(const State* SS, int p) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef __attribute__((address_space(4))) const State ConstState;
    return ((ConstState*)SS)[p];
#else
    return SS[p];   // the host pass never runs device functions
#endif
}

inline int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace sgks
