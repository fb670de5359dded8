// Deterministic reductions: 64-lane wavefront butterflies, a fixed-order
// sum over the waves of a block, and a grid-level finish in which the last
// block to arrive (integer ticket) sums the per-block partials in block
// order.  No floating-point atomics, so every result is bitwise
// reproducible for a given launch shape.
#pragma once
#include "common.hpp"

namespace jfnk {

constexpr int BLOCK = 256;
constexpr int MAX_WAVES = 1024 / 64;

struct Red {
    double *part;        // >= gridDim.x * NS partial sums
    unsigned *count;     // arrival ticket, 0 between launches
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;   // identical in every lane: IEEE addition is commutative
}

// Sum NS values over the block; the totals land in tot[0..NS) (shared).
template <int NS>
__device__ __forceinline__ void block_sum(double (&v)[NS], double *scratch, double *tot) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k) scratch[wid * NS + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += scratch[w * NS + threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ double load_l2(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide sums of v.  The last block calls fin(tot) on thread 0 with the
// totals, then resets the ticket.  Every block of the grid must call this.
template <int NS, class Fin>
__device__ __forceinline__ void grid_sum(double (&v)[NS], const Red &red, const Fin &fin) {
    __shared__ double scratch[MAX_WAVES * NS];
    __shared__ double tot[NS];
    __shared__ int last;
    block_sum<NS>(v, scratch, tot);
    if (threadIdx.x < NS) red.part[(size_t)blockIdx.x * NS + threadIdx.x] = tot[threadIdx.x];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(red.count, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NS; ++k) acc[k] += load_l2(red.part + (size_t)b * NS + k);
    }
    block_sum<NS>(acc, scratch, tot);
    if (threadIdx.x == 0) {
        fin(tot);
        *red.count = 0u;
    }
}

// Finalisers: write the totals (or derived scalars) to device slots.
struct FinNone {
    __device__ void operator()(const double *) const {}
};
template <int NS> struct FinStore {
    double *out;
    __device__ void operator()(const double *t) const {
#pragma unroll
        for (int k = 0; k < NS; ++k) out[k] = t[k];
    }
};

}  // namespace jfnk
