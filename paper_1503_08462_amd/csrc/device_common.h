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

// Lane -> (row, columns) map of the row kernels: the rows of a block of
// width ld are served by ld / cpt consecutive threads each (cpt consecutive
// columns per thread), numbered across the whole grid, so that every lane of
// every wavefront has work (a row may span two wavefronts: the row kernels
// exchange nothing between lanes).  Blocks are taken in XCD-aware order
// (xcd_block), so neighbouring rows run on the same XCD.
struct RowMap {
    int tpr, sub;
    int64_t row;
    bool active;
    __device__ __forceinline__ RowMap(int ld, int cpt, int64_t nrows) {
        tpr = ld / cpt;
        const uint32_t t = (uint32_t)xcd_block() * blockDim.x + threadIdx.x;  // < nrows * tpr + blockDim.x < 2^31
        const uint32_t r = t / (uint32_t)tpr;
        row = r;
        sub = (int)(t - r * (uint32_t)tpr);
        active = row < nrows;
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

typedef double dbl4 __attribute__((ext_vector_type(4)));

// One 16 x 16 tile of X^T Y over rows [0, K) on the FP64 matrix cores
// (v_mfma_f64_16x16x4: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
// D[i][j] in lane j + 16 (i mod 4), register i / 4).  X(i, c) and Y(i, c)
// return column c (0..15) of the tile operand in row i.  One wavefront, all
// lanes active.  Element (4u + (lane >> 4), lane & 15) of the result is in
// component u.
template <class FX, class FY>
__device__ __forceinline__ dbl4 mfma_tn16(const FX &X, const FY &Y, int K) {
    const int lane = threadIdx.x & (kWave - 1), kk = lane >> 4, c = lane & 15;
    dbl4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
    int base = 0;
    for (; base + 16 <= K; base += 16) {  // operands of four steps loaded ahead of the products
        const int i0 = base + kk;
        const double x0 = X(i0, c), y0 = Y(i0, c), x1 = X(i0 + 4, c), y1 = Y(i0 + 4, c);
        const double x2 = X(i0 + 8, c), y2 = Y(i0 + 8, c), x3 = X(i0 + 12, c), y3 = Y(i0 + 12, c);
        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, a1, 0, 0, 0);
        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x2, y2, a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x3, y3, a1, 0, 0, 0);
    }
    for (; base < K; base += 4) {
        const int i0 = base + kk;
        const int ic = i0 < K ? i0 : K - 1;  // clamped: never reads past row K - 1
        double x = X(ic, c), y = Y(ic, c);
        if (i0 >= K) x = y = 0.0;
        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a0, 0, 0, 0);
    }
    return a0 + a1;
}

// mfma_tn16 with the operands of eight steps (32 rows) loaded ahead of the
// products: for long K read from memory, where load latency dominates.
template <class FX, class FY>
__device__ __forceinline__ dbl4 mfma_tn16_deep(const FX &X, const FY &Y, int K) {
    const int lane = threadIdx.x & (kWave - 1), kk = lane >> 4, c = lane & 15;
    dbl4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
    int base = 0;
    for (; base + 32 <= K; base += 32) {
        double x[8], y[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            x[t] = X(base + kk + 4 * t, c);
            y[t] = Y(base + kk + 4 * t, c);
        }
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t], y[t], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t + 1], y[t + 1], a1, 0, 0, 0);
        }
    }
    for (; base < K; base += 4) {
        const int i0 = base + kk;
        const int ic = i0 < K ? i0 : K - 1;  // clamped: never reads past row K - 1
        double x = X(ic, c), y = Y(ic, c);
        if (i0 >= K) x = y = 0.0;
        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, a0, 0, 0, 0);
    }
    return a0 + a1;
}

// out(i, j, sum_k X(k, i) Y(k, j)) for i < mi, j < mj, k < K, in 16 x 16 tiles
// on the matrix cores.  X(k, a) and Y(k, b) must return zero for a >= mi
// (b >= mj); `out` receives each finished entry once.  With fewer tiles than
// wavefronts the K range is split over the wavefronts and the partial tiles
// summed in a fixed order, provided red (red_cap doubles) holds
// ntiles * wavefronts * 256 doubles.  Ends with a barrier.
template <class FX, class FY, class FO>
__device__ void block_tiles(const FX &X, const FY &Y, int K, int mi, int mj, const FO &out, double *red,
                            int red_cap) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int ti = (mi + 15) >> 4, tj = (mj + 15) >> 4, ntiles = ti * tj;
    if (K > 0 && (ntiles >= nw || nw == 1 || ntiles * nw * 256 > red_cap)) {
        for (int t = wv; t < ntiles; t += nw) {
            const int ta = t / tj, tb = t - ta * tj;
            const dbl4 acc = mfma_tn16([&](int k, int c) { return X(k, 16 * ta + c); },
                                       [&](int k, int c) { return Y(k, 16 * tb + c); }, K);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = 16 * ta + (lane >> 4) + 4 * u, j = 16 * tb + (lane & 15);
                if (i < mi && j < mj) out(i, j, acc[u]);
            }
        }
    } else if (K > 0) {
        const int chunk = ((K + nw - 1) / nw + 3) & ~3;
        const int k0 = wv * chunk, k1 = K < k0 + chunk ? K : k0 + chunk;
        for (int t = 0; t < ntiles; ++t) {
            const int ta = t / tj, tb = t - ta * tj;
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
            if (k1 > k0)
                acc = mfma_tn16([&](int k, int c) { return X(k0 + k, 16 * ta + c); },
                                [&](int k, int c) { return Y(k0 + k, 16 * tb + c); }, k1 - k0);
#pragma unroll
            for (int u = 0; u < 4; ++u) red[((t * nw + wv) * 4 + u) * kWave + lane] = acc[u];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ntiles * 256; e += blockDim.x) {
            const int t = e >> 8, u = (e >> 6) & 3, ln = e & 63;
            double s = 0.0;
            for (int v = 0; v < nw; ++v) s += red[((t * nw + v) * 4 + u) * kWave + ln];
            const int ta = t / tj, tb = t - ta * tj;
            const int i = 16 * ta + (ln >> 4) + 4 * u, j = 16 * tb + (ln & 15);
            if (i < mi && j < mj) out(i, j, s);
        }
    }
    __syncthreads();
}

// out = X^T Y (mi x mj, row stride ostr): block_tiles storing into an array.
template <class FX, class FY>
__device__ void block_xty(const FX &X, const FY &Y, int K, int mi, int mj, double *out, int ostr, double *red,
                          int red_cap) {
    block_tiles(X, Y, K, mi, mj, [&](int i, int j, double v) { out[i * ostr + j] = v; }, red, red_cap);
}

// Workgroup copy of n doubles (n even, both pointers 16-byte aligned) as
// double2, four loads in flight per thread.
__device__ __forceinline__ void block_copy(double *dst, const double *src, int n) {
    const int n2 = n / 2, nthr = blockDim.x;
    const double2 *s2 = reinterpret_cast<const double2 *>(src);
    double2 *d2 = reinterpret_cast<double2 *>(dst);
    int e = threadIdx.x;
    for (; e + 3 * nthr < n2; e += 4 * nthr) {
        const double2 a = s2[e], b = s2[e + nthr], c = s2[e + 2 * nthr], d = s2[e + 3 * nthr];
        d2[e] = a;
        d2[e + nthr] = b;
        d2[e + 2 * nthr] = c;
        d2[e + 3 * nthr] = d;
    }
    for (; e < n2; e += nthr) d2[e] = s2[e];
}

}  // namespace amgeig
