// Device helpers shared by the gfx950 kernels.
//
// Vector blocks are row-major N x ld (ld a multiple of 4): the ld values of one
// unknown are contiguous, so a neighbour gather in a sparse product is one
// contiguous segment.  A "row group" of TPR = ld / CPT lanes of a 64-wide
// wavefront owns one row; lane `sub` of the group owns columns
// [sub*CPT, sub*CPT + CPT).  A wavefront holds RPW = 64 / TPR row groups.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace amgeig {

constexpr int kWave = 64;
constexpr int kXcds = 8;

// Bijective block remap so that each XCD (blocks are dispatched round-robin
// over the 8 XCDs) works on one contiguous range of logical blocks, keeping
// neighbour rows of a sparse product in that XCD's L2.
__device__ __forceinline__ int64_t xcd_block() {
    const int64_t nb = gridDim.x, b = blockIdx.x;
    const int64_t per = nb / kXcds, rem = nb % kXcds;
    const int64_t x = b % kXcds, slot = b / kXcds;
    return x * per + (x < rem ? x : rem) + slot;
}

struct RowMap {
    int tpr, rpw, sub, grp;
    int64_t row;
    bool active;
    __device__ __forceinline__ RowMap(int ld, int cpt, int64_t nrows) {
        tpr = ld / cpt;
        rpw = kWave / tpr;
        const int lane = threadIdx.x & (kWave - 1);
        grp = lane / tpr;
        sub = lane - grp * tpr;
        const int64_t wave = xcd_block() * (blockDim.x / kWave) + threadIdx.x / kWave;
        row = wave * rpw + grp;
        active = grp < rpw && row < nrows;
    }
};

template <typename T, int N>
struct Vec {
    T v[N];
};

template <typename T, int N>
__device__ __forceinline__ Vec<T, N> ldv(const T *p) {
    Vec<T, N> r;
    if constexpr (sizeof(T) * N == 16) {
        const uint4 u = *reinterpret_cast<const uint4 *>(p);
        __builtin_memcpy(&r, &u, 16);
    } else if constexpr (sizeof(T) * N == 8) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        __builtin_memcpy(&r, &u, 8);
    } else if constexpr (sizeof(T) * N == 32) {
        const uint4 u0 = reinterpret_cast<const uint4 *>(p)[0];
        const uint4 u1 = reinterpret_cast<const uint4 *>(p)[1];
        __builtin_memcpy(&r, &u0, 16);
        __builtin_memcpy(reinterpret_cast<char *>(&r) + 16, &u1, 16);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) r.v[i] = p[i];
    }
    return r;
}

template <typename T, int N>
__device__ __forceinline__ void stv(T *p, const Vec<T, N> &r) {
    if constexpr (sizeof(T) * N == 16) {
        uint4 u;
        __builtin_memcpy(&u, &r, 16);
        *reinterpret_cast<uint4 *>(p) = u;
    } else if constexpr (sizeof(T) * N == 8) {
        uint2 u;
        __builtin_memcpy(&u, &r, 8);
        *reinterpret_cast<uint2 *>(p) = u;
    } else if constexpr (sizeof(T) * N == 32) {
        uint4 u0, u1;
        __builtin_memcpy(&u0, &r, 16);
        __builtin_memcpy(&u1, reinterpret_cast<const char *>(&r) + 16, 16);
        reinterpret_cast<uint4 *>(p)[0] = u0;
        reinterpret_cast<uint4 *>(p)[1] = u1;
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) p[i] = r.v[i];
    }
}

// Block-wide sum of `cnt` per-thread partials held in `val[]`, written to
// out[0..cnt) by thread 0's block (deterministic order).  `red` is LDS of at
// least blockDim.x doubles.
__device__ __forceinline__ double block_sum(double v, double *red) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += red[i];
    __syncthreads();
    if (threadIdx.x == 0) red[0] = s;
    __syncthreads();
    s = red[0];
    __syncthreads();
    return s;
}

// Last-block-done protocol: returns true in every thread of the one block
// that arrives last; the counter is reset to zero by that block, so the
// pattern needs no memset and replays inside a captured graph.
__device__ __forceinline__ bool last_block(unsigned *counter) {
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(counter, 1u);
        is_last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
    return is_last;
}

}  // namespace amgeig
