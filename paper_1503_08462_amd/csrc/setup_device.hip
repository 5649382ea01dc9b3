// The row-parallel parts of the AMG setup of Section 2 on the device: strong
// couplings (eq. (2.1)), direct interpolation from a C/F splitting (eqs.
// (2.2)-(2.4)), the transpose of P, and the Galerkin coarse operators (eq.
// (2.5)), and a parallel C/F splitting (PMIS: parallel modified independent
// set, De Sterck, Yang and Heys 2006) in place of the sequential Ruge-Stueben
// passes, which stay on the host.  The first four reproduce the host setup's
// arithmetic in its order, so both give the same bits.
//
// Galerkin products: A_{k+1} = P^T A_k P and M_{k+1} = P^T M_k P with the same
// prolongation P, the two products on one pattern.  A sparse-sparse product in
// two stages, T = X P (n x n_c, for X = A_k and M_k together) and C = P^T T,
// each row by one lane.  Every output row is accumulated in the order its
// contributions arise: the entries of the row of the left factor in storage
// order, and for each of them the entries of the matching row of the right
// factor in storage order.  A new column is appended where it first appears
// and later contributions are added to it, products and sums rounded
// separately (no fused multiply-add).  Rows of T keep that first-appearance
// order; rows of C are then sorted by column.
//
// Each lane owns a stretch of a temporary array sized by the row's product
// count (an upper bound of its distinct columns), found by an exclusive scan.
// A lane looks up a column by a linear search of its row so far: rows of these
// operators hold tens to a few hundred entries, and the work is done once per
// level at setup.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "amg_eig.h"
#include "internal.h"

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

// out[0] = 0, out[i+1] = x_0 + ... + x_i (i < m) with x_i = in[i], or
// x_i = (in[i] == 1) for kFlag, in one workgroup: each thread sums a
// contiguous chunk, the chunk sums are scanned in LDS, then each thread writes
// its chunk's running sums.
template <class T, bool kFlag = false>
__device__ __forceinline__ int64_t scan_term(T v) {
    return kFlag ? (int64_t)(v == 1) : (int64_t)v;
}
template <class T, bool kFlag = false>
__global__ __launch_bounds__(kScanThreads) void k_gal_scan(int64_t m, const T *in, int64_t *out) {
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int64_t chunk = (m + kScanThreads - 1) / kScanThreads;
    const int64_t b = t * chunk < m ? t * chunk : m;
    const int64_t e = b + chunk < m ? b + chunk : m;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += scan_term<T, kFlag>(in[i]);
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
        run += scan_term<T, kFlag>(in[i]);
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

// Strong couplings, eq. (2.1): entry (i, j), j != i, is strong when a_ij < 0
// and -a_ij >= theta max_{k != i, a_ik < 0} (-a_ik); a row without negative
// off-diagonal entries has none.
__global__ __launch_bounds__(kRowThreads) void k_strength(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                          const double *xa, double theta, uint8_t *strong) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n) return;
    double mx = 0.0;
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p)
        if (xcol[p] != i && xa[p] < 0.0) mx = fmax(mx, -xa[p]);
    const double thr = theta * mx;
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p)
        strong[p] = (uint8_t)(mx != 0.0 && xcol[p] != i && xa[p] < 0.0 && -xa[p] >= thr);
}

// Row sums of direct interpolation for F row i: the diagonal, the negative and
// positive off-diagonal entries, and the strong couplings to C points, each in
// storage order; returns the number of strong C couplings.
__device__ __forceinline__ int64_t interp_sums(int64_t i, const int64_t *xptr, const int32_t *xcol, const double *xa,
                                               const uint8_t *strong, const int32_t *cf, double &diag, double &sneg,
                                               double &spos, double &sP) {
#pragma clang fp contract(off)
    diag = sneg = spos = sP = 0.0;
    int64_t cnt = 0;
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p) {
        const double v = xa[p];
        if (xcol[p] == i) {
            diag = diag + v;
        } else if (v < 0.0) {
            sneg = sneg + v;
            if (strong[p] && cf[xcol[p]] == 1) {
                sP = sP + v;
                ++cnt;
            }
        } else if (v > 0.0) {
            spos = spos + v;
        }
    }
    return cnt;
}

// Row lengths of P: 1 for a C point; for an F point its strong C couplings,
// none if they sum to zero.
__global__ __launch_bounds__(kRowThreads) void k_interp_len(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                            const double *xa, const uint8_t *strong, const int32_t *cf,
                                                            int64_t *len) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n) return;
    if (cf[i] == 1) {
        len[i] = 1;
        return;
    }
    double diag, sneg, spos, sP;
    const int64_t cnt = interp_sums(i, xptr, xcol, xa, strong, cf, diag, sneg, spos, sP);
    len[i] = sP != 0.0 ? cnt : 0;
}

// Rows of P, eqs. (2.2)-(2.4): C points injected (coarse index cidx[i]); an F
// point i takes w_ij = -alpha_i a_ij / a~_ii over its strong C couplings, with
// alpha_i = (sum of negative off-diagonal a_ij) / (sum of strong C couplings)
// and a~_ii = a_ii + (sum of positive off-diagonal a_ij).
__global__ __launch_bounds__(kRowThreads) void k_interp_fill(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                             const double *xa, const uint8_t *strong,
                                                             const int32_t *cf, const int64_t *cidx,
                                                             const int64_t *pptr, int32_t *pcol, double *pval) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n) return;
    int64_t q = pptr[i];
    if (cf[i] == 1) {
        pcol[q] = (int32_t)cidx[i];
        pval[q] = 1.0;
        return;
    }
    if (pptr[i + 1] == q) return;
    double diag, sneg, spos, sP;
    (void)interp_sums(i, xptr, xcol, xa, strong, cf, diag, sneg, spos, sP);
    const double alpha = sneg / sP;
    const double ahat = diag + spos;
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p)
        if (strong[p] && cf[xcol[p]] == 1) {
            pcol[q] = (int32_t)cidx[xcol[p]];
            pval[q] = -alpha * xa[p] / ahat;
            ++q;
        }
}

// Transpose of P: entries counted per column, placed by atomic slots, then
// each row of P^T sorted by its column (the fine row), so the result does not
// depend on the order of the atomics.
__global__ __launch_bounds__(kRowThreads) void k_tr_count(int64_t nr, const int64_t *pptr, const int32_t *pcol,
                                                          unsigned long long *cnt) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= nr) return;
    for (int64_t p = pptr[i]; p < pptr[i + 1]; ++p) atomicAdd(cnt + pcol[p], 1ull);
}

__global__ __launch_bounds__(kRowThreads) void k_tr_fill(int64_t nr, const int64_t *pptr, const int32_t *pcol,
                                                         const double *pval, const int64_t *tptr,
                                                         unsigned long long *slot, int32_t *tcol, double *tval) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= nr) return;
    for (int64_t p = pptr[i]; p < pptr[i + 1]; ++p) {
        const int32_t c = pcol[p];
        const int64_t q = tptr[c] + (int64_t)atomicAdd(slot + c, 1ull);
        tcol[q] = (int32_t)i;
        tval[q] = pval[p];
    }
}

__global__ __launch_bounds__(kRowThreads) void k_tr_sort(int64_t nc, const int64_t *tptr, int32_t *tcol,
                                                         double *tval) {
    const int64_t c = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (c >= nc) return;
    const int64_t b = tptr[c], e = tptr[c + 1];
    for (int64_t s = b + 1; s < e; ++s) {
        const int32_t k = tcol[s];
        const double v = tval[s];
        int64_t t = s - 1;
        while (t >= b && tcol[t] > k) {
            tcol[t + 1] = tcol[t];
            tval[t + 1] = tval[t];
            --t;
        }
        tcol[t + 1] = k;
        tval[t + 1] = v;
    }
}

// PMIS.  Per entry p = (i, j) of a structurally symmetric pattern: bit 0 =
// i depends strongly on j, bit 1 = j depends strongly on i (the flag of the
// mirror entry (j, i), found by binary search in row j).  w_i = |S_i^T| + r_i;
// a point no point depends on starts F (0), the others undecided (-1).
__global__ __launch_bounds__(kRowThreads) void k_pmis_init(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                           const uint8_t *strong, const double *rnd, uint8_t *sflag,
                                                           double *w, int32_t *state, int32_t *isc) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n) return;
    int64_t nst = 0;
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p) {
        const int32_t j = xcol[p];
        int64_t lo = xptr[j], hi = xptr[j + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (xcol[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        const uint8_t back = (lo < xptr[j + 1] && xcol[lo] == i && j != i) ? strong[lo] : 0;
        sflag[p] = (uint8_t)((strong[p] ? 1 : 0) | (back ? 2 : 0));
        nst += back ? 1 : 0;
    }
    w[i] = (double)nst + rnd[i];
    state[i] = nst == 0 ? 0 : -1;
    isc[i] = 0;
}

// An undecided point heavier (weight, then index) than every undecided
// neighbour in the symmetrised strength graph is marked C.
__global__ __launch_bounds__(kRowThreads) void k_pmis_select(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                             const uint8_t *sflag, const double *w,
                                                             const int32_t *state, int32_t *isc) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n || state[i] != -1) return;
    const double wi = w[i];
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p) {
        const int32_t j = xcol[p];
        if (!sflag[p] || j == i || state[j] != -1) continue;
        if (w[j] > wi || (w[j] == wi && j > i)) return;
    }
    isc[i] = 1;
}

// Marked points become C; an undecided point that depends strongly on a C
// point becomes F; the points left undecided are counted.
__global__ __launch_bounds__(kRowThreads) void k_pmis_update(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                             const uint8_t *sflag, const int32_t *isc,
                                                             int32_t *state, unsigned long long *left) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n || state[i] != -1) return;
    if (isc[i]) {
        state[i] = 1;
        return;
    }
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p)
        if ((sflag[p] & 1) && isc[xcol[p]]) {
            state[i] = 0;
            return;
        }
    atomicAdd(left, 1ull);
}

// ---------------------------------------------------------------------
// Dense symmetric-definite eigen-decomposition A z = lambda M z of the
// coarsest level: Cholesky M = L L^T, C = L^-1 A L^-T, cyclic Jacobi on C in
// the round-robin (circle) ordering, whose m/2 rotations of a step act on
// disjoint index pairs and are applied together (rows, then columns), then
// Z = L^-T V.  Row-major n x n arrays; one launch per elimination or Jacobi
// phase, each over many workgroups.

// Cholesky pivot of column k: sqrt(L_kk), or a flag and 1 when not positive.
__global__ void k_chol_pivot(int64_t n, int64_t k, double *L, int *status) {
    const double d = L[k * n + k];
    if (!(d > 0.0)) {
        *status = 1;
        L[k * n + k] = 1.0;
    } else {
        L[k * n + k] = sqrt(d);
    }
}

// L_ik /= L_kk for i > k.
__global__ __launch_bounds__(kRowThreads) void k_chol_col(int64_t n, int64_t k, double *L) {
    const int64_t i = k + 1 + (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n) return;
    L[i * n + k] = L[i * n + k] / L[k * n + k];
}

// Trailing update of the lower triangle: L_ij -= L_ik L_jk for k < j <= i.
__global__ __launch_bounds__(kRowThreads) void k_chol_trail(int64_t n, int64_t k, double *L) {
    const int64_t m = n - k - 1;
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= m * m) return;
    const int64_t i = k + 1 + t / m, j = k + 1 + t % m;
    if (j > i) return;
    L[i * n + j] = L[i * n + j] - L[i * n + k] * L[j * n + k];
}

// Forward substitution step k of W = L^-1 W: W_k. /= L_kk.
__global__ __launch_bounds__(kRowThreads) void k_fwd_row(int64_t n, int64_t k, const double *L, double *W) {
    const int64_t j = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (j >= n) return;
    W[k * n + j] = W[k * n + j] / L[k * n + k];
}

// W_i. -= L_ik W_k. for i > k.
__global__ __launch_bounds__(kRowThreads) void k_fwd_elim(int64_t n, int64_t k, const double *L, double *W) {
    const int64_t m = n - k - 1;
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= m * n) return;
    const int64_t i = k + 1 + t / n, j = t % n;
    W[i * n + j] = W[i * n + j] - L[i * n + k] * W[k * n + j];
}

// Backward substitution step k of Z = L^-T Z: Z_k. /= L_kk, then
// Z_i. -= L_ki Z_k. for i < k (two launches).
__global__ __launch_bounds__(kRowThreads) void k_bwd_elim(int64_t n, int64_t k, const double *L, double *Z) {
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= k * n) return;
    const int64_t i = t / n, j = t % n;
    Z[i * n + j] = Z[i * n + j] - L[k * n + i] * Z[k * n + j];
}

// out_ij = X_ji.
__global__ __launch_bounds__(kRowThreads) void k_transpose_sq(int64_t n, const double *X, double *out) {
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= n * n) return;
    const int64_t i = t / n, j = t % n;
    out[i * n + j] = X[j * n + i];
}

// out = (X + X^T) / 2.
__global__ __launch_bounds__(kRowThreads) void k_symmetrise(int64_t n, const double *X, double *out) {
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= n * n) return;
    const int64_t i = t / n, j = t % n;
    out[i * n + j] = 0.5 * (X[i * n + j] + X[j * n + i]);
}

__global__ __launch_bounds__(kRowThreads) void k_identity(int64_t n, double *V) {
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= n * n) return;
    V[t] = (t / n == t % n) ? 1.0 : 0.0;
}

// Pair k of step s of the circle method over m (even) indices: index 0 stays,
// the others rotate; r_t = 1 + (t + s) mod (m - 1); pairs (0, r_0) and
// (r_t, r_{m-1-t}), t = 1 .. m/2 - 1.  Returns p < q.
__device__ __forceinline__ void jacobi_pair(int64_t m, int64_t s, int64_t k, int64_t &p, int64_t &q) {
    int64_t a, b;
    if (k == 0) {
        a = 0;
        b = 1 + s % (m - 1);
    } else {
        a = 1 + (k + s) % (m - 1);
        b = 1 + (m - 1 - k + s) % (m - 1);
    }
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// Rotation of each pair zeroing C_pq (symmetric Schur decomposition of the
// 2 x 2 block): tau = (C_qq - C_pp) / (2 C_pq), t = sign(tau) / (|tau| +
// sqrt(1 + tau^2)), c = 1 / sqrt(1 + t^2), s = t c.  Pairs with the padding
// index n, or C_pq = 0, get c = 1, s = 0.
__global__ __launch_bounds__(kRowThreads) void k_jac_angles(int64_t n, int64_t m, int64_t step, const double *C,
                                                            double *cs) {
    const int64_t k = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (k >= m / 2) return;
    int64_t p, q;
    jacobi_pair(m, step, k, p, q);
    double c = 1.0, sn = 0.0;
    if (q < n) {
        const double apq = C[p * n + q];
        if (apq != 0.0) {
            const double tau = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
        }
    }
    cs[2 * k] = c;
    cs[2 * k + 1] = sn;
}

// Rows p, q of C <- J^T C for every pair (disjoint rows).
__global__ __launch_bounds__(kRowThreads) void k_jac_rows(int64_t n, int64_t m, int64_t step, const double *cs,
                                                          double *C) {
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= (m / 2) * n) return;
    const int64_t k = t / n, j = t % n;
    int64_t p, q;
    jacobi_pair(m, step, k, p, q);
    if (q >= n) return;
    const double c = cs[2 * k], sn = cs[2 * k + 1];
    const double x = C[p * n + j], y = C[q * n + j];
    C[p * n + j] = c * x - sn * y;
    C[q * n + j] = sn * x + c * y;
}

// Columns p, q of C <- C J and V <- V J for every pair (disjoint columns).
__global__ __launch_bounds__(kRowThreads) void k_jac_cols(int64_t n, int64_t m, int64_t step, const double *cs,
                                                          double *C, double *V) {
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= (m / 2) * n) return;
    const int64_t k = t % (m / 2), i = t / (m / 2);
    int64_t p, q;
    jacobi_pair(m, step, k, p, q);
    if (q >= n) return;
    const double c = cs[2 * k], sn = cs[2 * k + 1];
    double x = C[i * n + p], y = C[i * n + q];
    C[i * n + p] = c * x - sn * y;
    C[i * n + q] = sn * x + c * y;
    x = V[i * n + p];
    y = V[i * n + q];
    V[i * n + p] = c * x - sn * y;
    V[i * n + q] = sn * x + c * y;
}

// Sums of squares of the off-diagonal entries and of all entries of C, in
// one workgroup.
__global__ __launch_bounds__(kScanThreads) void k_offnorm(int64_t n, const double *C, double *out) {
    __shared__ double so[kScanThreads], sa[kScanThreads];
    double o = 0.0, a = 0.0;
    for (int64_t t = threadIdx.x; t < n * n; t += kScanThreads) {
        const double v = C[t] * C[t];
        a += v;
        if (t / n != t % n) o += v;
    }
    so[threadIdx.x] = o;
    sa[threadIdx.x] = a;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            so[threadIdx.x] += so[threadIdx.x + w];
            sa[threadIdx.x] += sa[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = so[0];
        out[1] = sa[0];
    }
}

// Eigenvalues ascending (ties by index) and the matching columns of Z.
__global__ __launch_bounds__(kRowThreads) void k_eig_rank(int64_t n, const double *C, double *lam, int64_t *rank) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n) return;
    const double d = C[i * n + i];
    int64_t r = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double e = C[j * n + j];
        r += (e < d || (e == d && j < i)) ? 1 : 0;
    }
    rank[i] = r;
    lam[r] = d;
}

__global__ __launch_bounds__(kRowThreads) void k_eig_cols(int64_t n, const double *V, const int64_t *rank, double *Z) {
    const int64_t t = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (t >= n * n) return;
    const int64_t i = t / n, j = t % n;
    Z[i * n + rank[j]] = V[i * n + j];
}

// Second pass after PMIS: for each F point i and each F point j it depends
// on strongly, a conflict when no C point influences both strongly; the
// heavier point of each conflicting pair (weight, then index) is marked.
__device__ __forceinline__ bool strong_entry(const int64_t *xptr, const int32_t *xcol, const uint8_t *sflag,
                                             int64_t j, int32_t k) {
    int64_t lo = xptr[j], hi = xptr[j + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (xcol[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo < xptr[j + 1] && xcol[lo] == k && (sflag[lo] & 1);
}

__global__ __launch_bounds__(kRowThreads) void k_pmis2_mark(int64_t n, const int64_t *xptr, const int32_t *xcol,
                                                            const uint8_t *sflag, const double *w, const int32_t *cf,
                                                            int32_t *mark) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n || cf[i] != 0) return;
    for (int64_t p = xptr[i]; p < xptr[i + 1]; ++p) {
        const int32_t j = xcol[p];
        if (!(sflag[p] & 1) || j == i || cf[j] != 0) continue;
        bool shared = false;
        for (int64_t r = xptr[i]; r < xptr[i + 1] && !shared; ++r) {
            const int32_t k = xcol[r];
            if ((sflag[r] & 1) && cf[k] == 1 && strong_entry(xptr, xcol, sflag, j, k)) shared = true;
        }
        if (shared) continue;
        const bool i_heavier = w[i] > w[j] || (w[i] == w[j] && i > j);
        mark[i_heavier ? i : j] = 1;
    }
}

__global__ __launch_bounds__(kRowThreads) void k_pmis2_apply(int64_t n, int32_t *mark, int32_t *cf,
                                                             unsigned long long *moved) {
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (i >= n || !mark[i]) return;
    mark[i] = 0;
    cf[i] = 1;
    atomicAdd(moved, 1ull);
}

// Last entry of a device row-pointer array (its nonzero count), read with a
// wait on the stream; -1 if the copy fails.
int64_t device_nnz(const int64_t *ptr, int64_t rows, hipStream_t st) {
    int64_t v = 0;
    if (rows <= 0 || !ptr) return 0;
    if (hipMemcpyAsync(&v, ptr + rows, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return -1;
    return v;
}

inline unsigned grid_of(int64_t rows) { return (unsigned)((rows + kRowThreads - 1) / kRowThreads); }

// Temporary device arrays (at most kMaxTemps per call), stream-ordered on the
// call's stream, so that a setup call does not synchronise the device while
// other streams work; freed on every return path.
constexpr int kMaxTemps = 12;
struct Temps {
    hipStream_t st;
    void *p[kMaxTemps] = {};
    int k = 0;
    explicit Temps(hipStream_t s) : st(s) {}
    ~Temps() {
        for (int i = 0; i < k; ++i) (void)hipFreeAsync(p[i], st);
    }
    template <class T>
    bool get(T *&out, int64_t count) {
        out = nullptr;
        if (k == kMaxTemps) return false;
        if (count <= 0) count = 1;
        if (hipMallocAsync(&p[k], (size_t)count * sizeof(T), st) != hipSuccess) return false;
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
    {
        const int64_t xn = device_nnz(x_ptr, n, st), pn = device_nnz(p_ptr, n, st), tn = device_nnz(pt_ptr, nc, st);
        if (xn < 0 || pn < 0 || tn < 0) return AMG_EIG_EHIP;
        if ((xn > 0 && (!x_col || !x_a || !x_m)) || (pn > 0 && (!p_col || !p_val)) || (tn > 0 && (!pt_col || !pt_val)))
            return AMG_EIG_EINVAL;
    }
    Temps tmp(st);
    int64_t *ub_t, *toff, *tlen, *ub_c, *coff, *clen;
    if (!tmp.get(ub_t, n) || !tmp.get(toff, n + 1) || !tmp.get(tlen, n) || !tmp.get(ub_c, nc) ||
        !tmp.get(coff, nc + 1) || !tmp.get(clen, nc))
        return AMG_EIG_EHIP;
    // T = X P: bounds, offsets, rows
    if (n > 0) k_gal_bound<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, p_ptr, nullptr, ub_t);
    k_gal_scan<int64_t><<<1, kScanThreads, 0, st>>>(n, ub_t, toff);
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
    k_gal_scan<int64_t><<<1, kScanThreads, 0, st>>>(nc, ub_c, coff);
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
    k_gal_scan<int64_t><<<1, kScanThreads, 0, st>>>(nc, clen, c_ptr);
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

extern "C" int amg_eig_strength(int64_t n, const int64_t *x_ptr, const int32_t *x_col, const double *x_a,
                                double theta, uint8_t *strong, void *hip_stream) {
    if (n < 0 || !(theta >= 0.0 && theta <= 1.0)) return AMG_EIG_EINVAL;
    if (n == 0) return AMG_EIG_OK;
    if (!x_ptr || !x_col || !x_a || !strong) return AMG_EIG_EINVAL;
    k_strength<<<grid_of(n), kRowThreads, 0, (hipStream_t)hip_stream>>>(n, x_ptr, x_col, x_a, theta, strong);
    return hipGetLastError() == hipSuccess ? AMG_EIG_OK : AMG_EIG_EHIP;
}

extern "C" int amg_eig_interpolation(int64_t n, const int64_t *x_ptr, const int32_t *x_col, const double *x_a,
                                     const uint8_t *strong, const int32_t *cf, int64_t *p_ptr, int32_t *p_col,
                                     double *p_val, int64_t cap, int64_t *nnz, int64_t *nc, void *hip_stream) {
    if (n < 0 || cap < 0 || !nnz || !nc || !p_ptr) return AMG_EIG_EINVAL;
    if (n > 0 && (!x_ptr || !cf)) return AMG_EIG_EINVAL;
    if (cap > 0 && (!p_col || !p_val)) return AMG_EIG_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    *nnz = 0;
    *nc = 0;
    {
        const int64_t xn = device_nnz(x_ptr, n, st);
        if (xn < 0) return AMG_EIG_EHIP;
        if (xn > 0 && (!x_col || !x_a || !strong)) return AMG_EIG_EINVAL;
    }
    Temps tmp(st);
    int64_t *cidx, *len;
    if (!tmp.get(cidx, n + 1) || !tmp.get(len, n)) return AMG_EIG_EHIP;
    k_gal_scan<int32_t, true><<<1, kScanThreads, 0, st>>>(n, cf, cidx);
    if (n > 0) k_interp_len<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, x_a, strong, cf, len);
    k_gal_scan<int64_t><<<1, kScanThreads, 0, st>>>(n, len, p_ptr);
    int64_t h[2] = {0, 0};
    if (hipMemcpyAsync(&h[0], cidx + n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&h[1], p_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return AMG_EIG_EHIP;
    *nc = h[0];
    *nnz = h[1];
    if (h[1] > cap) return AMG_EIG_EWORKSPACE;
    if (n > 0)
        k_interp_fill<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, x_a, strong, cf, cidx, p_ptr, p_col, p_val);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return AMG_EIG_EHIP;
    return AMG_EIG_OK;
}

extern "C" int amg_eig_transpose(int64_t nr, int64_t nc, const int64_t *p_ptr, const int32_t *p_col,
                                 const double *p_val, int64_t *pt_ptr, int32_t *pt_col, double *pt_val,
                                 void *hip_stream) {
    if (nr < 0 || nc < 0 || !pt_ptr || (nr > 0 && !p_ptr)) return AMG_EIG_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    {
        const int64_t pn = device_nnz(p_ptr, nr, st);
        if (pn < 0) return AMG_EIG_EHIP;
        if (pn > 0 && (!p_col || !p_val || !pt_col || !pt_val)) return AMG_EIG_EINVAL;
    }
    Temps tmp(st);
    unsigned long long *cnt;
    if (!tmp.get(cnt, nc)) return AMG_EIG_EHIP;
    if (hipMemsetAsync(cnt, 0, (size_t)(nc > 0 ? nc : 1) * sizeof(unsigned long long), st) != hipSuccess)
        return AMG_EIG_EHIP;
    if (nr > 0) k_tr_count<<<grid_of(nr), kRowThreads, 0, st>>>(nr, p_ptr, p_col, cnt);
    k_gal_scan<unsigned long long><<<1, kScanThreads, 0, st>>>(nc, cnt, pt_ptr);
    if (hipMemsetAsync(cnt, 0, (size_t)(nc > 0 ? nc : 1) * sizeof(unsigned long long), st) != hipSuccess)
        return AMG_EIG_EHIP;
    if (nr > 0) k_tr_fill<<<grid_of(nr), kRowThreads, 0, st>>>(nr, p_ptr, p_col, p_val, pt_ptr, cnt, pt_col, pt_val);
    if (nc > 0) k_tr_sort<<<grid_of(nc), kRowThreads, 0, st>>>(nc, pt_ptr, pt_col, pt_val);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return AMG_EIG_EHIP;
    return AMG_EIG_OK;
}

extern "C" int amg_eig_pmis(int64_t n, const int64_t *x_ptr, const int32_t *x_col, const uint8_t *strong,
                            const double *rnd, int second_pass, int32_t *cf, int *rounds, void *hip_stream) {
    if (n < 0 || !rounds || (n > 0 && (!x_ptr || !rnd || !cf))) return AMG_EIG_EINVAL;
    *rounds = 0;
    if (n == 0) return AMG_EIG_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    int64_t nnz = 0;
    if (hipMemcpyAsync(&nnz, x_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return AMG_EIG_EHIP;
    if (nnz > 0 && (!x_col || !strong)) return AMG_EIG_EINVAL;
    Temps tmp(st);
    uint8_t *sflag;
    double *w;
    int32_t *isc;
    unsigned long long *left;
    if (!tmp.get(sflag, nnz) || !tmp.get(w, n) || !tmp.get(isc, n) || !tmp.get(left, 1)) return AMG_EIG_EHIP;
    k_pmis_init<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, strong, rnd, sflag, w, cf, isc);
    // every round makes at least the heaviest undecided point C, so n rounds
    // decide every point
    for (int64_t r = 0; r < n; ++r) {
        unsigned long long h = 0;
        if (hipMemsetAsync(left, 0, sizeof(unsigned long long), st) != hipSuccess) return AMG_EIG_EHIP;
        k_pmis_select<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, sflag, w, cf, isc);
        k_pmis_update<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, sflag, isc, cf, left);
        if (hipMemcpyAsync(&h, left, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return AMG_EIG_EHIP;
        *rounds = (int)(r + 1);
        if (h == 0) break;
    }
    if (!second_pass) return hipGetLastError() == hipSuccess ? AMG_EIG_OK : AMG_EIG_EHIP;
    // second pass: every round promotes at least one F point, so n rounds
    // leave no conflict (isc is free again and serves as the marks)
    if (hipMemsetAsync(isc, 0, (size_t)n * sizeof(int32_t), st) != hipSuccess) return AMG_EIG_EHIP;
    for (int64_t r = 0; r <= n; ++r) {
        unsigned long long h = 0;
        if (hipMemsetAsync(left, 0, sizeof(unsigned long long), st) != hipSuccess) return AMG_EIG_EHIP;
        k_pmis2_mark<<<grid_of(n), kRowThreads, 0, st>>>(n, x_ptr, x_col, sflag, w, cf, isc);
        k_pmis2_apply<<<grid_of(n), kRowThreads, 0, st>>>(n, isc, cf, left);
        if (hipMemcpyAsync(&h, left, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return AMG_EIG_EHIP;
        if (h == 0) return hipGetLastError() == hipSuccess ? AMG_EIG_OK : AMG_EIG_EHIP;
    }
    return AMG_EIG_EHIP;
}

extern "C" int amg_eig_dense_sygv(int64_t n, const double *A, const double *M, double *lam, double *Z, int *sweeps,
                                  void *hip_stream) {
    if (n < 1 || n > 4096 || !A || !M || !lam || !Z) return AMG_EIG_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    if (sweeps) *sweeps = 0;
    Temps tmp(st);
    double *L, *C, *W, *cs, *nrm;
    int64_t *rank;
    int *status;
    const int64_t m = n + (n & 1);
    if (!tmp.get(L, n * n) || !tmp.get(C, n * n) || !tmp.get(W, n * n) || !tmp.get(cs, m) || !tmp.get(nrm, 2) ||
        !tmp.get(rank, n) || !tmp.get(status, 1))
        return AMG_EIG_EHIP;
    const size_t bytes = (size_t)(n * n) * sizeof(double);
    if (hipMemsetAsync(status, 0, sizeof(int), st) != hipSuccess ||
        hipMemcpyAsync(L, M, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(W, A, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return AMG_EIG_EHIP;
    const unsigned gnn = grid_of(n * n);
    // M = L L^T (lower triangle of L)
    for (int64_t k = 0; k < n; ++k) {
        k_chol_pivot<<<1, 1, 0, st>>>(n, k, L, status);
        if (k + 1 < n) {
            k_chol_col<<<grid_of(n - k - 1), kRowThreads, 0, st>>>(n, k, L);
            k_chol_trail<<<grid_of((n - k - 1) * (n - k - 1)), kRowThreads, 0, st>>>(n, k, L);
        }
    }
    // C = L^-1 A L^-T: W = L^-1 A, then (L^-1 W^T)^T, symmetrised
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t k = 0; k < n; ++k) {
            k_fwd_row<<<grid_of(n), kRowThreads, 0, st>>>(n, k, L, W);
            if (k + 1 < n) k_fwd_elim<<<grid_of((n - k - 1) * n), kRowThreads, 0, st>>>(n, k, L, W);
        }
        k_transpose_sq<<<gnn, kRowThreads, 0, st>>>(n, W, C);
        if (pass == 0 && hipMemcpyAsync(W, C, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return AMG_EIG_EHIP;
    }
    k_symmetrise<<<gnn, kRowThreads, 0, st>>>(n, C, W);
    std::swap(C, W);
    k_identity<<<gnn, kRowThreads, 0, st>>>(n, W);  // W now holds V
    // cyclic Jacobi, at most 40 sweeps, until the off-diagonal part is below
    // n eps of the Frobenius norm
    constexpr int kMaxSweeps = 40;
    int done = 0, sw = 0;
    int hstatus = 0;
    for (sw = 0; sw < kMaxSweeps && n > 1; ++sw) {
        double h[2];
        k_offnorm<<<1, kScanThreads, 0, st>>>(n, C, nrm);
        if (hipMemcpyAsync(h, nrm, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&hstatus, status, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return AMG_EIG_EHIP;
        if (hstatus) return AMG_EIG_ENOTSPD;
        // rounding leaves off-diagonal entries of order eps |C|, so the bound
        // grows with n
        const double tolr = (double)n * 2.220446049250313e-16;
        if (!(h[0] > tolr * tolr * h[1])) {
            done = 1;
            break;
        }
        for (int64_t step = 0; step < m - 1; ++step) {
            k_jac_angles<<<grid_of(m / 2), kRowThreads, 0, st>>>(n, m, step, C, cs);
            k_jac_rows<<<grid_of((m / 2) * n), kRowThreads, 0, st>>>(n, m, step, cs, C);
            k_jac_cols<<<grid_of((m / 2) * n), kRowThreads, 0, st>>>(n, m, step, cs, C, W);
        }
    }
    if (n == 1) done = 1;
    if (sweeps) *sweeps = sw;
    if (!done) return AMG_EIG_EBREAKDOWN;
    // Z = L^-T V (in W), then eigenvalues ascending with their columns
    for (int64_t k = n - 1; k >= 0; --k) {
        k_fwd_row<<<grid_of(n), kRowThreads, 0, st>>>(n, k, L, W);
        if (k > 0) k_bwd_elim<<<grid_of(k * n), kRowThreads, 0, st>>>(n, k, L, W);
    }
    k_eig_rank<<<grid_of(n), kRowThreads, 0, st>>>(n, C, lam, rank);
    k_eig_cols<<<gnn, kRowThreads, 0, st>>>(n, W, rank, Z);
    if (hipMemcpyAsync(&hstatus, status, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return AMG_EIG_EHIP;
    return hstatus ? AMG_EIG_ENOTSPD : AMG_EIG_OK;
}

namespace amgeig {
namespace {

// Device copy of a host array, stream-ordered on the stream it was allocated
// on and freed with the object.
template <class T>
struct DevArr {
    T *p = nullptr;
    int64_t n = 0;
    hipStream_t st = nullptr;
    DevArr() = default;
    DevArr(const DevArr &) = delete;
    DevArr &operator=(const DevArr &) = delete;
    ~DevArr() { reset(); }
    void reset() {
        if (p) (void)hipFreeAsync(p, st);
        p = nullptr;
        n = 0;
    }
    bool alloc(int64_t count, hipStream_t s) {
        reset();
        st = s;
        n = count;
        return hipMallocAsync((void **)&p, (size_t)(count > 0 ? count : 1) * sizeof(T), s) == hipSuccess;
    }
    bool up(const std::vector<T> &v, hipStream_t s) {
        return alloc((int64_t)v.size(), s) &&
               (v.empty() ||
                (hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s) == hipSuccess &&
                 hipStreamSynchronize(s) == hipSuccess));
    }
    bool down(std::vector<T> &v, int64_t count) const {
        v.resize((size_t)count);
        return count == 0 ||
               (hipMemcpyAsync(v.data(), p, (size_t)count * sizeof(T), hipMemcpyDeviceToHost, st) == hipSuccess &&
                hipStreamSynchronize(st) == hipSuccess);
    }
    void swap(DevArr &o) {
        std::swap(p, o.p);
        std::swap(n, o.n);
        std::swap(st, o.st);
    }
};

// A non-blocking stream of default priority owned by one setup call: the
// arrays declared after it free themselves on it first, then it is drained
// and destroyed.
struct OwnStream {
    hipStream_t s = nullptr;
    bool create() { return hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess; }
    ~OwnStream() {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
};

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output k of the stream
// seeded with s is the MurmurHash3 variant-13 finaliser of s + (k+1) * gamma;
// a uniform double in [0, 1) from its top 53 bits.
double splitmix_uniform(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

int device_coarsen(Hierarchy &H, const amg_eig_opts &o, int64_t cmin, std::string &err) {
    auto hip_fail = [&](const char *what) {
        err = std::string("device coarsening: ") + what + " failed";
        (void)hipGetLastError();
        return AMG_EIG_EHIP;
    };
    OwnStream os;
    if (!os.create()) return hip_fail("stream creation");
    hipStream_t st = os.s;
    DevArr<int64_t> xp, pp, ptp, cp;
    DevArr<int32_t> xc, cf, pc, ptc, cc;
    DevArr<double> xa, xm, rnd, pv, ptv, ca, cm;
    DevArr<uint8_t> strong;
    {
        const Level &L = H.lv.back();
        if (!xp.up(L.ptr, st) || !xc.up(L.col, st) || !xa.up(L.a, st) || !xm.up(L.m, st)) return hip_fail("upload");
    }
    while ((int)H.lv.size() < o.max_levels && H.lv.back().n > o.coarse_max) {
        const size_t k = H.lv.size() - 1;
        const int64_t n = H.lv[k].n;
        int rc;
        if (!strong.alloc(xc.n, st)) return hip_fail("allocation");
        rc = amg_eig_strength(n, xp.p, xc.p, xa.p, o.theta, strong.p, st);
        if (rc) return rc == AMG_EIG_EHIP ? hip_fail("strength") : rc;
        std::vector<double> r((size_t)n);
        for (int64_t i = 0; i < n; ++i) r[(size_t)i] = splitmix_uniform(o.coarsen_seed + (uint64_t)k, (uint64_t)i);
        if (!rnd.up(r, st) || !cf.alloc(n, st)) return hip_fail("upload");
        int rounds = 0;
        rc = amg_eig_pmis(n, xp.p, xc.p, strong.p, rnd.p, 1, cf.p, &rounds, st);
        if (rc) return rc == AMG_EIG_EHIP ? hip_fail("PMIS") : rc;
        int64_t pnnz = 0, nc = 0;
        if (!pp.alloc(n + 1, st)) return hip_fail("allocation");
        rc = amg_eig_interpolation(n, xp.p, xc.p, xa.p, strong.p, cf.p, pp.p, nullptr, nullptr, 0, &pnnz, &nc,
                                   st);
        if (rc != AMG_EIG_OK && rc != AMG_EIG_EWORKSPACE) return rc == AMG_EIG_EHIP ? hip_fail("interpolation") : rc;
        if (nc < cmin || (double)nc > 0.9 * (double)n || nc == 0) break;
        if (!pc.alloc(pnnz, st) || !pv.alloc(pnnz, st)) return hip_fail("allocation");
        rc = amg_eig_interpolation(n, xp.p, xc.p, xa.p, strong.p, cf.p, pp.p, pc.p, pv.p, pnnz, &pnnz, &nc, st);
        if (rc) return rc == AMG_EIG_EHIP ? hip_fail("interpolation") : rc;
        if (!ptp.alloc(nc + 1, st) || !ptc.alloc(pnnz, st) || !ptv.alloc(pnnz, st)) return hip_fail("allocation");
        rc = amg_eig_transpose(n, nc, pp.p, pc.p, pv.p, ptp.p, ptc.p, ptv.p, st);
        if (rc) return rc == AMG_EIG_EHIP ? hip_fail("transpose") : rc;
        int64_t cnnz = 0;
        if (!cp.alloc(nc + 1, st)) return hip_fail("allocation");
        rc = amg_eig_galerkin(n, nc, xp.p, xc.p, xa.p, xm.p, pp.p, pc.p, pv.p, ptp.p, ptc.p, ptv.p, cp.p, nullptr,
                              nullptr, nullptr, 0, &cnnz, st);
        if (rc != AMG_EIG_OK && rc != AMG_EIG_EWORKSPACE) return rc == AMG_EIG_EHIP ? hip_fail("Galerkin") : rc;
        if (cnnz >= ((int64_t)1 << 31)) {
            err = "device coarsening: a coarse level has 2^31 or more entries";
            return AMG_EIG_EINVAL;
        }
        if (!cc.alloc(cnnz, st) || !ca.alloc(cnnz, st) || !cm.alloc(cnnz, st)) return hip_fail("allocation");
        rc = amg_eig_galerkin(n, nc, xp.p, xc.p, xa.p, xm.p, pp.p, pc.p, pv.p, ptp.p, ptc.p, ptv.p, cp.p, cc.p, ca.p,
                              cm.p, cnnz, &cnnz, st);
        if (rc) return rc == AMG_EIG_EHIP ? hip_fail("Galerkin") : rc;
        // copy the splitting, P, P^T and the new level back
        Level &L = H.lv[k];
        L.P.nr = n;
        L.P.nc = nc;
        L.Pt.nr = nc;
        L.Pt.nc = n;
        Level next;
        next.n = nc;
        if (!cf.down(L.cf, n) || !pp.down(L.P.ptr, n + 1) || !pc.down(L.P.col, pnnz) || !pv.down(L.P.val, pnnz) ||
            !ptp.down(L.Pt.ptr, nc + 1) || !ptc.down(L.Pt.col, pnnz) || !ptv.down(L.Pt.val, pnnz) ||
            !cp.down(next.ptr, nc + 1) || !cc.down(next.col, cnnz) || !ca.down(next.a, cnnz) ||
            !cm.down(next.m, cnnz))
            return hip_fail("download");
        H.lv.push_back(std::move(next));
        xp.swap(cp);
        xc.swap(cc);
        xa.swap(ca);
        xm.swap(cm);
    }
    return AMG_EIG_OK;
}

}  // namespace amgeig

namespace amgeig {

int device_sygv(int n, const std::vector<double> &A, const std::vector<double> &M, std::vector<double> &lam,
                std::vector<double> &Z, std::string &err) {
    OwnStream os;
    if (!os.create()) {
        err = "device eigen-decomposition: stream creation failed";
        return AMG_EIG_EHIP;
    }
    hipStream_t st = os.s;
    DevArr<double> da, dm, dl, dz;
    if (!da.up(A, st) || !dm.up(M, st) || !dl.alloc(n, st) || !dz.alloc((int64_t)n * n, st)) {
        err = "device eigen-decomposition: allocation or upload failed";
        return AMG_EIG_EHIP;
    }
    int sweeps = 0;
    const int rc = amg_eig_dense_sygv(n, da.p, dm.p, dl.p, dz.p, &sweeps, st);
    if (rc == AMG_EIG_ENOTSPD) {
        err = "coarsest mass matrix not positive definite";
        return rc;
    }
    if (rc) {
        err = "device eigen-decomposition of the coarsest level failed";
        return rc;
    }
    if (!dl.down(lam, n) || !dz.down(Z, (int64_t)n * n)) {
        err = "device eigen-decomposition: download failed";
        return AMG_EIG_EHIP;
    }
    return AMG_EIG_OK;
}

}  // namespace amgeig
