// Deterministic reductions: 64-lane wavefront butterflies, a fixed-order
// sum over the waves of a block, per-block partials, and a one-block
// finishing kernel that sums the partials in block order.  No
// floating-point atomics, so every result is bitwise reproducible for a
// given launch shape.
#pragma once
#include <map>

#include "common.hpp"

namespace jfnk {

constexpr int BLOCK = 256;
constexpr int MAX_WAVES = 1024 / 64;

struct Red {
    double *part;        // >= gridDim.x * NS partial sums
};

// host side: launch the finishing kernel of a reduction over nb blocks
template <int NS, class Fin>
inline void finish(hipStream_t st, const Red &red, int nb, const Fin &fin);

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

// Per-block partial sums: the block's totals go to part[blockIdx.x * NS + k].
// Every block of the grid must call this (it synchronises the block).
template <int NS>
__device__ __forceinline__ void block_partials(double (&v)[NS], const Red &red) {
    __shared__ double scratch[MAX_WAVES * NS];
    __shared__ double tot[NS];
    block_sum<NS>(v, scratch, tot);
    if (threadIdx.x < NS) red.part[(size_t)blockIdx.x * NS + threadIdx.x] = tot[threadIdx.x];
}

// Second kernel of a grid reduction: one block sums the nb partials in
// block order and hands the totals to fin on thread 0.  Launched on the same
// stream right after the producing kernel, whose completion makes the
// partials visible (no device-wide fence inside the producer, whose cost on
// gfx950 is an L2 write-back per block).
template <int NS, class Fin>
__global__ __launch_bounds__(256) void k_finish(Red red, int nb, Fin fin) {
    __shared__ double scratch[MAX_WAVES * NS];
    __shared__ double tot[NS];
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NS; ++k) acc[k] += red.part[(size_t)b * NS + k];
    }
    block_sum<NS>(acc, scratch, tot);
    if (threadIdx.x == 0) fin(tot);
}

// Step of the finite-difference quotient (Sec. 1): eps = num / ||v||, read
// from device slots at kernel start, or a fixed test step.  ||v||^2 is either
// a slot or, for a deferred reduction, the per-block partials of the kernel
// that produced v: then every block sums them itself in a fixed order.
struct FdStep {
    const double *num;             // numerator slot (nullptr: not an FD evaluation)
    const double *vn2;             // ||v||^2 slot
    double fixed;                  // > 0: use this step
    const double *part = nullptr;  // deferred ||v||^2: partials of nb blocks
    int nb = 0;
    // called by every thread of the block (a block-wide sum when deferred);
    // n2out, when given, receives ||v||^2 (also with a fixed step)
    __device__ double eps(double *n2out = nullptr) const {
        if (!n2out && fixed > 0.0) return fixed;
        if (!n2out && num == nullptr) return 0.0;
        double n2 = 0.0;
        if (part) {
            __shared__ double scratch[MAX_WAVES];
            __shared__ double tot[1];
            // eight independent loads in flight per trip
            const int bd = blockDim.x;
            double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int b = threadIdx.x;
            for (; b + 7 * bd < nb; b += 8 * bd) {
#pragma unroll
                for (int k = 0; k < 8; ++k) acc[k] += part[b + k * bd];
            }
            for (; b < nb; b += bd) acc[0] += part[b];
            double a[1] = {((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]))};
            block_sum<1>(a, scratch, tot);
            n2 = tot[0];
        } else if (vn2) {
            n2 = *vn2;
        }
        if (n2out) *n2out = n2;
        if (fixed > 0.0) return fixed;
        if (num == nullptr) return 0.0;
        return n2 > 0.0 ? *num / sqrt(n2) : 0.0;
    }
};

// Deferred reductions (host side).  A slot registered in buf gets the
// per-block partials of its producer in a buffer of its own and no
// finishing kernel; pend records them until the slot is produced again.
constexpr int LAZY_CAP = 8192;     // partials per deferred slot
struct Pending {
    const double *part;
    int nb;
};
struct LazyTable {
    std::map<const double *, double *> buf;
    std::map<const double *, Pending> pend;
};

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

namespace jfnk {
template <int NS, class Fin>
inline void finish(hipStream_t st, const Red &red, int nb, const Fin &fin) {
    k_finish<NS, Fin><<<1, 256, 0, st>>>(red, nb, fin);
}
}  // namespace jfnk
