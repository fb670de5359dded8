// Deterministic reductions: 64-lane wavefront sums by DPP, a fixed-order
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

// Lane data movement within 16-lane rows (DPP), one 32-bit half at a time.
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active), the same value in
// every lane.  Inside a 16-lane row each step adds the value of a partner
// lane whose partner is the lane itself (lane ^ 1, lane ^ 2, then the
// mirror images within 8 and 16 lanes), so both lanes of a pair form the
// same IEEE sum; the four row sums are then added in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);    // row_half_mirror
    v += dpp_mov<0x140>(v);    // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Sum NS values over the block; the totals land in tot[0..NS) (shared).
// blockDim.x must be a multiple of 64.
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

// One value summed over the block with a single barrier: every thread reads
// the wave totals (an LDS broadcast) and adds them in wave order.  scratch
// (MAX_WAVES entries) must not be written again until every thread of the
// block has passed a later barrier: callers that sum repeatedly alternate
// two scratch arrays.
__device__ __forceinline__ double block_sum1(double v, double *scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += scratch[w];
    return s;
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
            // eight independent loads in flight per trip
            const int bd = blockDim.x;
            double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int b = threadIdx.x;
            for (; b + 7 * bd < nb; b += 8 * bd) {
#pragma unroll
                for (int k = 0; k < 8; ++k) acc[k] += part[b + k * bd];
            }
            for (; b < nb; b += bd) acc[0] += part[b];
            n2 = block_sum1(((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])),
                            scratch);
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
