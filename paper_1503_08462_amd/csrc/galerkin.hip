// Galerkin coarse operators on the device, eq. (2.5): A_{k+1} = P^T A_k P and
// M_{k+1} = P^T M_k P with the same prolongation P (eqs. (2.2)-(2.4)), the two
// products on one pattern.  A sparse-sparse product in two stages, T = X P
// (n x n_c, for X = A_k and M_k together) and C = P^T T, each row by one lane.
//
// Every output row is accumulated in the order its contributions arise: the
// entries of the row of the left factor in storage order, and for each of them
// the entries of the matching row of the right factor in storage order.  A new
// column is appended where it first appears and later contributions are added
// to it, products and sums rounded separately (no fused multiply-add).  Rows of
// T keep that first-appearance order; rows of C are then sorted by column.  The
// host setup forms its Galerkin products in the same order, so both give the
// same bits.
//
// Each lane owns a stretch of a temporary array sized by the row's product
// count (an upper bound of its distinct columns), found by an exclusive scan.
// A lane looks up a column by a linear search of its row so far: rows of these
// operators hold tens to a few hundred entries, and the work is done once per
// level at setup.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "amg_eig.h"

namespace {

constexpr int kRowThreads = 256;
constexpr int kScanThreads = 1024;

// ub[r] = sum over the entries (r, j) of the left factor of len(j), where
// len(j) is the row length of the right factor: from its row pointers when
// rlen is null, else rlen[j].
__global__ __launch_bounds__(kRowThreads) void k_gal_bound(int64_t rows, const int64_t *lptr, const int32_t *lcol,
                                                           const int64_t *rptr, const int64_t *rlen, int64_t *ub) {
    const int64_t r = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (r >= rows) return;
    int64_t s = 0;
    for (int64_t p = lptr[r]; p < lptr[r + 1]; ++p) {
        const int64_t j = lcol[p];
        s += rlen ? rlen[j] : rptr[j + 1] - rptr[j];
    }
    ub[r] = s;
}

// out[0] = 0, out[i+1] = in[0] + ... + in[i] (i < m), in one workgroup: each
// thread sums a contiguous chunk, the chunk sums are scanned in LDS, then each
// thread writes its chunk's running sums.
__global__ __launch_bounds__(kScanThreads) void k_gal_scan(int64_t m, const int64_t *in, int64_t *out) {
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t chunk = (m + kScanThreads - 1) / kScanThreads;
    const int64_t b = t * chunk < m ? t * chunk : m;
    const int64_t e = b + chunk < m ? b + chunk : m;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    if (t == 0) out[0] = 0;
    for (int64_t i = b; i < e; ++i) {
        run += in[i];
        out[i + 1] = run;
    }
}

// Append (c, va, vm) to the row held in col/a/m[0, len) or add to the entry of
// column c.
__device__ __forceinline__ void gal_accumulate(int32_t c, double va, double vm, int32_t *col, double *a, double *m,
                                               int64_t &len) {
#pragma clang fp contract(off)
    for (int64_t s = 0; s < len; ++s)
        if (col[s] == c) {
            a[s] = a[s] + va;
            m[s] = m[s] + vm;
            return;
        }
    col[len] = c;
    a[len] = va;
    m[len] = vm;
    ++len;
}

// T = [A P | M P] row by row, row i into its stretch from toff[i]; tlen[i]
// receives its length.
__global__ __launch_bounds__(kRowThreads) void k_gal_xp(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                        const double *xa, const double *xm, const int64_t *pptr,
                                                        const int32_t *pcol, const double *pval, const int64_t *toff,
                                                        int32_t *tcol, double *ta, double *tm, int64_t *tlen) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t base = toff[i];
    int64_t len = 0;
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p) {
        const int64_t j = xcol[p];
        const double va = xa[p], vm = xm[p];
        for (int64_t r = pptr[j]; r < pptr[j + 1]; ++r) {
            const double w = pval[r];
            gal_accumulate(pcol[r], va * w, vm * w, tcol + base, ta + base, tm + base, len);
        }
    }
    tlen[i] = len;
}

// C = P^T T row by row, row c into its stretch from coff[c], then sorted by
// column (insertion sort); clen[c] receives its length.
__global__ __launch_bounds__(kRowThreads) void k_gal_ptt(int64_t nc, const int64_t *ptptr, const int32_t *ptcol,
                                                         const double *ptval, const int64_t *toff,
                                                         const int64_t *tlen, const int32_t *tcol, const double *ta,
                                                         const double *tm, const int64_t *coff, int32_t *ccol,
                                                         double *ca, double *cm, int64_t *clen) {
#pragma clang fp contract(off)
    const int64_t c = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (c >= nc) return;
    const int64_t base = coff[c];
    int32_t *col = ccol + base;
    double *a = ca + base, *m = cm + base;
    int64_t len = 0;
    for (int64_t p = ptptr[c]; p < ptptr[c + 1]; ++p) {
        const int64_t i = ptcol[p];
        const double w = ptval[p];
        for (int64_t r = toff[i]; r < toff[i] + tlen[i]; ++r) gal_accumulate(tcol[r], w * ta[r], w * tm[r], col, a, m, len);
    }
    for (int64_t s = 1; s < len; ++s) {
        const int32_t k = col[s];
        const double va = a[s], vm = m[s];
        int64_t t = s - 1;
        while (t >= 0 && col[t] > k) {
            col[t + 1] = col[t];
            a[t + 1] = a[t];
            m[t + 1] = m[t];
            --t;
        }
        col[t + 1] = k;
        a[t + 1] = va;
        m[t + 1] = vm;
    }
    clen[c] = len;
}

// Row c of C from its stretch to its place c_ptr[c] in the output.
__global__ __launch_bounds__(kRowThreads) void k_gal_compact(int64_t nc, const int64_t *coff, const int64_t *cptr,
                                                             const int32_t *scol, const double *sa, const double *sm,
                                                             int32_t *ocol, double *oa, double *om) {
    const int64_t c = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (c >= nc) return;
    const int64_t from = coff[c], to = cptr[c], len = cptr[c + 1] - cptr[c];
    for (int64_t s = 0; s < len; ++s) {
        ocol[to + s] = scol[from + s];
        oa[to + s] = sa[from + s];
        om[to + s] = sm[from + s];
    }
}

inline unsigned grid_of(int64_t rows) { return (unsigned)((rows + kRowThreads - 1) / kRowThreads); }

// Temporary device arrays, freed on every return path.
struct Temps {
    void *p[12] = {};
    int k = 0;
    ~Temps() {
        for (int i = 0; i < k; ++i) (void)hipFree(p[i]);
    }
    template <class T>
    bool get(T *&out, int64_t count) {
        out = nullptr;
        if (count <= 0) count = 1;
        if (hipMalloc(&p[k], (size_t)count * sizeof(T)) != hipSuccess) return false;
        out = (T *)p[k++];
        return true;
    }
};

}  // namespace

extern "C" int amg_eig_galerkin(int64_t n, int64_t nc, const int64_t *x_ptr, const int32_t *x_col, const double *x_a,
                                const double *x_m, const int64_t *p_ptr, const int32_t *p_col, const double *p_val,
                                const int64_t *pt_ptr, const int32_t *pt_col, const double *pt_val, int64_t *c_ptr,
                                int32_t *c_col, double *c_a, double *c_m, int64_t cap, int64_t *nnz,
                                void *hip_stream) {
    if (n < 0 || nc < 0 || cap < 0 || !nnz || !c_ptr) return AMG_EIG_EINVAL;
    // column and value arrays may be null when they hold no entries
    if (n > 0 && (!x_ptr || !p_ptr)) return AMG_EIG_EINVAL;
    if (nc > 0 && !pt_ptr) return AMG_EIG_EINVAL;
    if (cap > 0 && (!c_col || !c_a || !c_m)) return AMG_EIG_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    *nnz = 0;
    Temps tmp;
    int64_t *ub_t, *toff, *tlen, *ub_c, *coff, *clen;
    if (!tmp.get(ub_t, n) || !tmp.get(toff, n + 1) || !tmp.get(tlen, n) || !tmp.get(ub_c, nc) ||
        !tmp.get(coff, nc + 1) || !tmp.get(clen, nc))
        return AMG_EIG_EHIP;
    // T = X P: bounds, offsets, rows
    if (n > 0) k_gal_bound<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, p_ptr, nullptr, ub_t);
    k_gal_scan<<<1, kScanThreads, 0, st>>>(n, ub_t, toff);
    int64_t tcap = 0;
    if (hipMemcpyAsync(&tcap, toff + n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return AMG_EIG_EHIP;
    int32_t *tcol;
    double *ta, *tm;
    if (!tmp.get(tcol, tcap) || !tmp.get(ta, tcap) || !tmp.get(tm, tcap)) return AMG_EIG_EHIP;
    if (n > 0)
        k_gal_xp<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, x_a, x_m, p_ptr, p_col, p_val, toff, tcol, ta,
                                                     tm, tlen);
    // C = P^T T: bounds, offsets, rows, row pointers
    if (nc > 0) k_gal_bound<<<grid_of(nc), kRowThreads, 0, st>>>(nc, pt_ptr, pt_col, nullptr, tlen, ub_c);
    k_gal_scan<<<1, kScanThreads, 0, st>>>(nc, ub_c, coff);
    int64_t ccap = 0;
    if (hipMemcpyAsync(&ccap, coff + nc, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return AMG_EIG_EHIP;
    int32_t *scol;
    double *sa, *sm;
    if (!tmp.get(scol, ccap) || !tmp.get(sa, ccap) || !tmp.get(sm, ccap)) return AMG_EIG_EHIP;
    if (nc > 0)
        k_gal_ptt<<<grid_of(nc), kRowThreads, 0, st>>>(nc, pt_ptr, pt_col, pt_val, toff, tlen, tcol, ta, tm, coff,
                                                       scol, sa, sm, clen);
    k_gal_scan<<<1, kScanThreads, 0, st>>>(nc, clen, c_ptr);
    int64_t total = 0;
    if (hipMemcpyAsync(&total, c_ptr + nc, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return AMG_EIG_EHIP;
    *nnz = total;
    if (total > cap) return AMG_EIG_EWORKSPACE;
    if (nc > 0)
        k_gal_compact<<<grid_of(nc), kRowThreads, 0, st>>>(nc, coff, c_ptr, scol, sa, sm, c_col, c_a, c_m);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return AMG_EIG_EHIP;
    return AMG_EIG_OK;
}
