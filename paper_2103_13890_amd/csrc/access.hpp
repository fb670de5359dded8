// Node addressing for the stencil kernels and their epilogues.
//
// PtrAt addresses node i of an array through a 64-bit per-lane address.
// BufAt addresses a node of a grid row as (row start, column): the row
// start is the same for every lane of the block and goes into the scalar
// offset of a buffer instruction, the column is the lane's and is the same
// for every row.  A tiled kernel that walks rows then issues its loads and
// stores with no vector address arithmetic at all.  Buffer offsets are
// 32-bit byte offsets, so BufAt serves arrays below 2 GiB.
#pragma once
#include "common.hpp"

namespace jfnk {

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p) {
    // raw buffer (stride 0), every byte offset below 2^31 in range; dword 3
    // as the hardware's default for 32-bit data
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7fffffff, 0x00020000);
}

template <typename T> __device__ __forceinline__ T buf_ld(const T *p, unsigned voff, unsigned soff) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(buf_rsrc(p), (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(buf_rsrc(p), (int)voff, (int)soff, 0));
}
template <typename T> __device__ __forceinline__ void buf_st(T *p, unsigned voff, unsigned soff, T v) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), buf_rsrc(p), (int)voff, (int)soff, 0);
    } else {
        using U2 = unsigned __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), buf_rsrc(p), (int)voff, (int)soff, 0);
    }
}

struct PtrAt {
    long long i;
    // element c + i (c: component offset)
    template <typename T> __device__ __forceinline__ T ld(const T *p, long long c) const { return p[c + i]; }
    template <typename T> __device__ __forceinline__ void st(T *p, long long c, T v) const { p[c + i] = v; }
};

// row must be the same in every lane: it is read from the first active lane
// (a plain copy when the compiler already holds it in a scalar register;
// otherwise the read keeps it from looping over distinct lane values).
struct BufAt {
    unsigned row;   // index of the row's first node (block-uniform)
    unsigned col;   // the lane's column
    template <typename T> __device__ __forceinline__ unsigned soff(long long c) const {
        return __builtin_amdgcn_readfirstlane((row + (unsigned)c) * (unsigned)sizeof(T));
    }
    template <typename T> __device__ __forceinline__ T ld(const T *p, long long c) const {
        return buf_ld<T>(p, col * (unsigned)sizeof(T), soff<T>(c));
    }
    template <typename T> __device__ __forceinline__ void st(T *p, long long c, T v) const {
        buf_st<T>(p, col * (unsigned)sizeof(T), soff<T>(c), v);
    }
};

}  // namespace jfnk
