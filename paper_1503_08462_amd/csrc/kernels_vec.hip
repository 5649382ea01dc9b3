// Sparse and vector-block kernels of one correction step (Algorithm 3.1) on
// gfx950.  All blocks are row-major N x ld; a row group of ld/CPT lanes owns
// one row (see device_common.h).  Sparse matrices are CSR with int32 indices.
//
//   k_residual      R = M U diag(theta) - A U (shared pattern of A and M, FP64)
//                   and the column norms giving rho_j (eq. (3.1) residual)
//   k_smooth_pre    V-cycle pre-smoothing from a zero guess fused with the
//                   residual: r = b - A D^-1 b (l1-Jacobi, x1 = D^-1 b not stored)
//   k_spmm          y = X x for a CSR X: restriction (P^T), prolongation (P),
//                   FP64 transfer chains of the Rayleigh-Ritz step
//   k_prolong_add   y = D^-1 b + P x_c (coarse-grid correction of x1)
//   k_smooth_post   x = y + D^-1 (b - A y); on the correction level it writes
//                   the FP64 block V = U + x
//   k_gs_colour     one colour of a multicolour Gauss-Seidel sweep (forward from
//                   a zero guess, or backward; on the correction level it writes
//                   the FP64 block V = U + x as rows finish)
//   k_dual_spmm     W = [A V | M V] (FP64, shared pattern)
//   k_gram          [V^T A V | V^T M V] by a two-phase deterministic reduction
//   k_dual_gram     both of the above in one pass over the rows (wide blocks)
//   k_final         U = P Y + V X_v on the correction level (recombination)
#include <algorithm>

#include <hip/hip_ext.h>

#include "device_common.h"
#include "kernels.h"

namespace amgeig {

namespace {

template <typename T, int C>
__device__ __forceinline__ void fma_v(Vec<T, C> &acc, T w, const Vec<T, C> &x) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc.v[c] += w * x.v[c];
}

template <typename T, int C>
__device__ __forceinline__ Vec<T, C> zero_v() {
    Vec<T, C> z;
#pragma unroll
    for (int c = 0; c < C; ++c) z.v[c] = T(0);
    return z;
}

// Gathers x[col[p]] (CPT values from column c0) for p in [p0, p1) and hands
// each to consume(p, j, x_j) in ascending p; the loads of four neighbours are
// issued before the first of them is consumed, and the last one to three
// neighbours of a row are loaded together too, so a row of 5, 7 or 15
// neighbours costs two or four dependent round trips, not one per leftover
// neighbour.
template <typename T, int CPT, class F>
__device__ __forceinline__ void gather4(int32_t p0, int32_t p1, const int32_t *__restrict__ col,
                                        const T *__restrict__ x, int ld, int c0, const F &consume) {
    int32_t p = p0;
    for (; p + 4 <= p1; p += 4) {
        const int64_t j0 = col[p], j1 = col[p + 1], j2 = col[p + 2], j3 = col[p + 3];
        const Vec<T, CPT> x0 = ldv<T, CPT>(x + j0 * ld + c0);
        const Vec<T, CPT> x1 = ldv<T, CPT>(x + j1 * ld + c0);
        const Vec<T, CPT> x2 = ldv<T, CPT>(x + j2 * ld + c0);
        const Vec<T, CPT> x3 = ldv<T, CPT>(x + j3 * ld + c0);
        consume(p, j0, x0);
        consume(p + 1, j1, x1);
        consume(p + 2, j2, x2);
        consume(p + 3, j3, x3);
    }
    const int rem = p1 - p;  // 0 .. 3
    if (rem > 0) {
        const int64_t j0 = col[p], j1 = rem > 1 ? col[p + 1] : j0, j2 = rem > 2 ? col[p + 2] : j0;
        const Vec<T, CPT> x0 = ldv<T, CPT>(x + j0 * ld + c0);
        const Vec<T, CPT> x1 = rem > 1 ? ldv<T, CPT>(x + j1 * ld + c0) : zero_v<T, CPT>();
        const Vec<T, CPT> x2 = rem > 2 ? ldv<T, CPT>(x + j2 * ld + c0) : zero_v<T, CPT>();
        consume(p, j0, x0);
        if (rem > 1) consume(p + 1, j1, x1);
        if (rem > 2) consume(p + 2, j2, x2);
    }
}

// Gathers like gather4, with the CSR entries loaded once per wavefront: the
// rows a wavefront serves (row groups may straddle wavefronts) have their
// entries in [wp0, wp1); when these are at most 64, lane l loads entry wp0 + l
// and every lane takes the column indices and values of its own row's entries
// from the lanes holding them (cross-lane reads, no memory access), so a
// neighbour costs one vector-memory load (its row of x) instead of one per
// column index and value.  Wavefronts with more entries (the denser Galerkin
// rows of coarse levels) load them per lane as gather4 does.  load_vals(p)
// returns the values of entry p (a struct of doubles or floats, moved lane to
// lane as 32-bit words); consume(vals, j, x_j) sees the row's entries in
// ascending p either way.  Every lane of the wavefront must call it (lanes
// past the last row with active = false); the loop that moves values between
// lanes is uniform across the wavefront.
template <typename V>
__device__ __forceinline__ V lane_take(const V &v, int src) {
    static_assert(sizeof(V) % 4 == 0, "values move as 32-bit words");
    V r;
    const int *pv = reinterpret_cast<const int *>(&v);
    int *pr = reinterpret_cast<int *>(&r);
#pragma unroll
    for (int w = 0; w < (int)(sizeof(V) / 4); ++w) pr[w] = __shfl(pv[w], src, kWave);
    return r;
}

template <typename T, int CPT, class LV, class F>
__device__ __forceinline__ void gather_wave(int64_t row, int sub, int tpr, bool active, int64_t nrows,
                                            const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                            const T *__restrict__ x, int ld, int c0, const LV &load_vals,
                                            const F &consume) {
    const int lane = threadIdx.x & (kWave - 1);
    // flat index of lane 0 of this wavefront, and the rows its lanes serve
    const int64_t t0 = (int64_t)__builtin_amdgcn_readfirstlane((int)(row * tpr + sub - lane));
    const int64_t r_lo = t0 / tpr;
    int64_t r_hi = (t0 + kWave - 1) / tpr;
    r_hi = r_hi < nrows - 1 ? r_hi : nrows - 1;
    if (r_lo > r_hi) return;  // the whole wavefront is past the last row
    const int32_t wp0 = ptr[r_lo], wp1 = ptr[r_hi + 1];
    const int32_t p0 = active ? ptr[row] : 0, p1 = active ? ptr[row + 1] : 0;
    if (wp1 - wp0 > kWave) {  // uniform: per-lane loads
        if (active)
            gather4<T, CPT>(p0, p1, col, x, ld, c0,
                            [&](int32_t p, int64_t j, const Vec<T, CPT> &xj) { consume(load_vals(p), j, xj); });
        return;
    }
    {
        const int32_t base = wp0;
        const int32_t pe = base + lane < wp1 ? base + lane : base;
        const int32_t cl = col[pe];
        const auto vl = load_vals(pe);
        const int cnt = p1 - p0;
        int cmax = cnt;
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const int o = __shfl_xor(cmax, off, kWave);
            cmax = o > cmax ? o : cmax;
        }
        const int q0 = cnt > 0 ? p0 - base : 0;  // lane holding this lane's first entry
        for (int t = 0; t < cmax; t += 4) {
            int q[4];
            int64_t j[4];
            Vec<T, CPT> xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                q[u] = t + u < cnt ? q0 + t + u : q0;
                j[u] = __shfl(cl, q[u], kWave);
            }
            // only the entries a lane consumes are loaded (rows of a wavefront
            // differ in length, and x rows are wide)
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = t + u < cnt ? ldv<T, CPT>(x + j[u] * ld + c0) : zero_v<T, CPT>();
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const auto vu = lane_take(vl, q[u]);
                if (t + u < cnt) consume(vu, j[u], xv[u]);
            }
        }
    }
}

}  // namespace

// ------------------------------------------------------------------- a1
template <typename TO, int CPT>
__global__ __launch_bounds__(256) void k_residual(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ a,
                                                  const double *__restrict__ m, const double *__restrict__ U,
                                                  const double *__restrict__ theta, TO *__restrict__ R,
                                                  double *__restrict__ part, const int *status) {
    __shared__ double sm[256 * CPT * 2];
    if (status[ST_CONVERGED]) return;
    const int tpr = ld / CPT, rpw = kWave / tpr;
    const int lane = threadIdx.x & (kWave - 1), wib = threadIdx.x / kWave, wpb = blockDim.x / kWave;
    const int grp = lane / tpr, sub = lane - grp * tpr, c0 = sub * CPT;
    const int64_t nb = gridDim.x, lb = xcd_block();
    const int64_t waves = (n + rpw - 1) / rpw;
    const int64_t w0 = waves * lb / nb, w1 = waves * (lb + 1) / nb;
    double th[CPT], rr[CPT], mm[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        th[c] = grp < rpw ? theta[c0 + c] : 0.0;
        rr[c] = mm[c] = 0.0;
    }
    for (int64_t w = w0 + wib; w < w1; w += wpb) {  // the same trip count for every lane of a wavefront
        const int64_t row = w * rpw + grp;
        const bool active = grp < rpw && row < n;
        Vec<double, CPT> au = zero_v<double, CPT>(), mu = zero_v<double, CPT>();
        gather_wave<double, CPT>(row, sub, tpr, active, n, ptr, col, U, ld, c0,
                                 [&](int32_t p) { return double2{a[p], m[p]}; },
                                 [&](const double2 &am, int64_t, const Vec<double, CPT> &u) {
                                     fma_v(au, am.x, u);
                                     fma_v(mu, am.y, u);
                                 });
        if (!active) continue;
        Vec<TO, CPT> out;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const double r = th[c] * mu.v[c] - au.v[c];
            out.v[c] = (TO)r;
            rr[c] += r * r;
            mm[c] += mu.v[c] * mu.v[c];
        }
        stv<TO, CPT>(R + row * ld + c0, out);
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        sm[(threadIdx.x * CPT + c) * 2 + 0] = rr[c];
        sm[(threadIdx.x * CPT + c) * 2 + 1] = mm[c];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 2 * ld; idx += blockDim.x) {
        const int cidx = idx >> 1, kind = idx & 1, s = cidx / CPT, c = cidx - s * CPT;
        double acc = 0.0;
        for (int w = 0; w < wpb; ++w)
            for (int g = 0; g < rpw; ++g) acc += sm[(((w * kWave) + g * tpr + s) * CPT + c) * 2 + kind];
        part[lb * 2 * ld + idx] = acc;
    }
}

// Right-hand side of a further AMG cycle of the same correction (m > 1 in
// eq. (3.2)): R = (Theta - sigma) M U - (A - sigma M) V, the residual of the
// linear equation (3.1) (shifted by sigma, Remark 3.1) at the current iterate
// V, its right-hand side formed from the iterate U the correction started
// from.  Shared pattern of A and M, FP64 products, output in the working
// precision.
template <typename TO, int CPT>
__global__ __launch_bounds__(256) void k_residual_cycle(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ col, const double *__restrict__ a,
                                                        const double *__restrict__ m, const double *__restrict__ U,
                                                        const double *__restrict__ V, const double *__restrict__ theta,
                                                        double sigma, TO *__restrict__ R, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int c0 = rm.sub * CPT;
    Vec<double, CPT> mu = zero_v<double, CPT>(), av = zero_v<double, CPT>();
    gather_wave<double, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, U, ld, c0, [&](int32_t p) { return m[p]; },
                             [&](const double &w, int64_t, const Vec<double, CPT> &x) { fma_v(mu, w, x); });
    gather_wave<double, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, V, ld, c0,
                             [&](int32_t p) { return a[p] - sigma * m[p]; },
                             [&](const double &w, int64_t, const Vec<double, CPT> &x) { fma_v(av, w, x); });
    if (!rm.active) return;
    Vec<TO, CPT> out;
#pragma unroll
    for (int c = 0; c < CPT; ++c) out.v[c] = (TO)((theta[c0 + c] - sigma) * mu.v[c] - av.v[c]);
    stv<TO, CPT>(R + rm.row * ld + c0, out);
}

// Residual norms: one workgroup per sum fin[e] = sum over blocks of
// part[b][e] (threads strided over blocks, fixed-order tree), then the last
// workgroup to finish forms rho_j = sqrt(sum R_j^2) / (|theta_j| sqrt(sum (MU)_j^2))
// and the convergence test max_{j < q} rho_j <= tol.
__global__ __launch_bounds__(256) void k_residual_finish(int64_t nb, int ld, const double *__restrict__ part,
                                                         double *__restrict__ fin, unsigned *counter,
                                                         const double *__restrict__ theta, double *__restrict__ rho,
                                                         int q, double tol, int *status, int check) {
    __shared__ double red[256 / kWave];
    if (status[ST_CONVERGED]) return;
    const int e = blockIdx.x, w2 = 2 * ld;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t b = threadIdx.x;
    for (; b + 3 * 256 < nb; b += 4 * 256) {
        s0 += part[b * w2 + e];
        s1 += part[(b + 256) * w2 + e];
        s2 += part[(b + 512) * w2 + e];
        s3 += part[(b + 768) * w2 + e];
    }
    for (; b < nb; b += 256) s0 += part[b * w2 + e];
    double v = (s0 + s1) + (s2 + s3);
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += red[i];
        fin[e] = t;
    }
    if (!last_block(counter)) return;
    if ((int)threadIdx.x < ld) {
        const int j = threadIdx.x;
        rho[j] = sqrt(fin[2 * j]) / (fabs(theta[j]) * sqrt(fin[2 * j + 1]));
    }
    __syncthreads();
    if (threadIdx.x == 0 && check) {
        double mx = 0.0;
        for (int j = 0; j < q; ++j) mx = fmax(mx, rho[j]);
        if (mx <= tol) status[ST_CONVERGED] = 1;
    }
}

// ------------------------------------------------------------------- a2
// vs = a_ij / d_j on the pattern of the V-cycle operator (column-scaled
// values, formed once at bind in the working precision)
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_smooth_pre(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ col, const T *__restrict__ vs,
                                                    const T *__restrict__ dinv, const T *__restrict__ b,
                                                    T *__restrict__ r, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = ldv<T, CPT>(b + row * ld + c0);
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, b, ld, c0, [&](int32_t p) { return vs[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &xj) { fma_v(acc, -v, xj); });
    if (!rm.active) return;
    stv<T, CPT>(r + rm.row * ld + c0, acc);
}

// ---------------------------------------------------------- a3, chains
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                              const int32_t *__restrict__ col, const T *__restrict__ val,
                                              const T *__restrict__ x, T *__restrict__ y, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = zero_v<T, CPT>();
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, x, ld, c0, [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &xj) { fma_v(acc, v, xj); });
    if (!rm.active) return;
    stv<T, CPT>(y + rm.row * ld + c0, acc);
}

// ------------------------------------------------------------------- a5
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_prolong_add(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ col, const T *__restrict__ val,
                                                     const T *__restrict__ xc, const T *__restrict__ dinv,
                                                     const T *__restrict__ b, T *__restrict__ y, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = ldv<T, CPT>(b + row * ld + c0);
    const T di = dinv[row];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc.v[c] *= di;
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, xc, ld, c0, [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &xj) { fma_v(acc, v, xj); });
    if (!rm.active) return;
    stv<T, CPT>(y + rm.row * ld + c0, acc);
}

// ------------------------------------------------------------------- a6
template <typename T, int CPT, bool FINAL>
__global__ __launch_bounds__(256) void k_smooth_post(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ col, const T *__restrict__ val,
                                                     const T *__restrict__ dinv, const T *__restrict__ b,
                                                     const T *__restrict__ y, T *__restrict__ x,
                                                     const double *__restrict__ U, double *__restrict__ V,
                                                     const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = ldv<T, CPT>(b + row * ld + c0);
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, y, ld, c0, [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &xj) { fma_v(acc, -v, xj); });
    if (!rm.active) return;
    const Vec<T, CPT> yi = ldv<T, CPT>(y + rm.row * ld + c0);
    const T di = dinv[rm.row];
    if constexpr (FINAL) {
        Vec<double, CPT> u = ldv<double, CPT>(U + rm.row * ld + c0);
#pragma unroll
        for (int c = 0; c < CPT; ++c) u.v[c] += (double)(yi.v[c] + di * acc.v[c]);
        stv<double, CPT>(V + rm.row * ld + c0, u);
    } else {
        Vec<T, CPT> o;
#pragma unroll
        for (int c = 0; c < CPT; ++c) o.v[c] = yi.v[c] + di * acc.v[c];
        stv<T, CPT>(x + rm.row * ld + c0, o);
    }
}

// ------------------------------------ multicolour Gauss-Seidel (a2, a6)
// One colour of a Gauss-Seidel sweep.  The colour's rows are positions
// [0, nrows) of a colour-ordered CSR (ptr, diag and rows start at the colour's
// first position; rows gives the row numbers): x_i = (b_i - sum a_ij x_j) / a_ii
// over the entries listed, which hold no diagonal (all off-diagonal entries,
// or, from a zero guess, those of smaller colours: the others multiply zeros).
// Rows of one colour are not neighbours, so they read rows of other colours
// only and update in parallel; x is read and written by the same launch at
// disjoint rows.  FINAL also writes V_i = U_i + x_i in FP64: in a sweep a row
// changes only in its own colour's step.
template <typename T, int CPT, bool FINAL>
__global__ __launch_bounds__(256) void k_gs_colour(int64_t nrows, int ld, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, const T *__restrict__ val,
                                                   const T *__restrict__ diag, const int32_t *__restrict__ rows,
                                                   const T *__restrict__ b, T *x, const double *__restrict__ U,
                                                   double *__restrict__ V, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, nrows);
    const int64_t pos = rm.active ? rm.row : nrows - 1;  // lanes past the last row read it and store nothing
    const int64_t row = rows[pos];
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = ldv<T, CPT>(b + row * ld + c0);
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, nrows, ptr, col, x, ld, c0,
                        [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &xj) { fma_v(acc, -v, xj); });
    if (!rm.active) return;
    const T di = diag[pos];
    Vec<T, CPT> o;
#pragma unroll
    for (int c = 0; c < CPT; ++c) o.v[c] = acc.v[c] / di;
    stv<T, CPT>(x + row * ld + c0, o);
    if constexpr (FINAL) {
        Vec<double, CPT> u = ldv<double, CPT>(U + row * ld + c0);
#pragma unroll
        for (int c = 0; c < CPT; ++c) u.v[c] += (double)o.v[c];
        stv<double, CPT>(V + row * ld + c0, u);
    }
}

// ---------------------------------------------- Chebyshev smoothing (a2, a6)
// Degree-2 Chebyshev smoothing on D^-1 A over [lo, 1] (D the l1 diagonal):
// with theta = (1 + lo) / 2, delta = (1 - lo) / 2, sigma = theta / delta,
// rho0 = 1 / sigma, rho1 = 1 / (2 sigma - rho0), c1 = rho1 rho0, c2 = 2 rho1 / delta,
//   r0 = D^-1 (b - A x0), d0 = r0 / theta, r1 = r0 - D^-1 A d0,
//   d1 = c1 d0 + c2 r1, x = x0 + d0 + d1.
struct ChebCoef {
    float itheta, theta, c1, c2;     // FP32 copies for the mixed-precision V-cycle
    double ditheta, dtheta, dc1, dc2;
};

template <typename T>
__device__ __forceinline__ void cheb_coef(const ChebCoef &k, T &itheta, T &theta, T &c1, T &c2) {
    if constexpr (sizeof(T) == 4) {
        itheta = k.itheta;
        theta = k.theta;
        c1 = k.c1;
        c2 = k.c2;
    } else {
        itheta = k.ditheta;
        theta = k.dtheta;
        c1 = k.dc1;
        c2 = k.dc2;
    }
}

// Pre-smoothing from x0 = 0: r0 = D^-1 b, so one product A (D^-1 b) gives x;
// vs = a_ij / d_j, the column-scaled values (no gather of d_j per neighbour).
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_cheb_pre(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col, const T *__restrict__ vs,
                                                  const T *__restrict__ dinv, const T *__restrict__ b,
                                                  T *__restrict__ x, ChebCoef kc, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    T itheta, theta, c1, c2;
    cheb_coef(kc, itheta, theta, c1, c2);
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> az = zero_v<T, CPT>();  // A D^-1 b
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, b, ld, c0, [&](int32_t p) { return vs[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &bj) { fma_v(az, v, bj); });
    if (!rm.active) return;
    const Vec<T, CPT> bi = ldv<T, CPT>(b + rm.row * ld + c0);
    const T di = dinv[rm.row];
    Vec<T, CPT> o;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const T r0 = di * bi.v[c];
        const T d0 = r0 * itheta;
        const T r1 = r0 - di * (az.v[c] * itheta);
        const T d1 = c1 * d0 + c2 * r1;
        o.v[c] = d0 + d1;
    }
    stv<T, CPT>(x + rm.row * ld + c0, o);
}

// r = b - A x on one level
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_level_residual(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ col, const T *__restrict__ val,
                                                        const T *__restrict__ b, const T *__restrict__ x,
                                                        T *__restrict__ r, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = ldv<T, CPT>(b + row * ld + c0);
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, x, ld, c0, [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &xj) { fma_v(acc, -v, xj); });
    if (!rm.active) return;
    stv<T, CPT>(r + rm.row * ld + c0, acc);
}

// y = x + P xc (prolongation onto the stored pre-smoothed iterate)
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_prolong_x(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, const T *__restrict__ val,
                                                   const T *__restrict__ xc, const T *__restrict__ x,
                                                   T *__restrict__ y, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = ldv<T, CPT>(x + row * ld + c0);
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, xc, ld, c0, [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &xj) { fma_v(acc, v, xj); });
    if (!rm.active) return;
    stv<T, CPT>(y + rm.row * ld + c0, acc);
}

// Post-smoothing, first product: d0 = D^-1 (b - A y) / theta
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_cheb_post1(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ col, const T *__restrict__ val,
                                                    const T *__restrict__ dinv, const T *__restrict__ b,
                                                    const T *__restrict__ y, T *__restrict__ d0, ChebCoef kc,
                                                    const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    T itheta, theta, c1, c2;
    cheb_coef(kc, itheta, theta, c1, c2);
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> acc = ldv<T, CPT>(b + row * ld + c0);
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, y, ld, c0, [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &yj) { fma_v(acc, -v, yj); });
    if (!rm.active) return;
    const T di = dinv[rm.row];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc.v[c] = (di * acc.v[c]) * itheta;
    stv<T, CPT>(d0 + rm.row * ld + c0, acc);
}

// Post-smoothing, second product: r1 = theta d0 - D^-1 A d0, d1 = c1 d0 + c2 r1,
// x = y + d0 + d1; on the correction level V = U + x in FP64 instead.
template <typename T, int CPT, bool FINAL>
__global__ __launch_bounds__(256) void k_cheb_post2(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ col, const T *__restrict__ val,
                                                    const T *__restrict__ dinv, const T *__restrict__ y,
                                                    const T *__restrict__ d0, T *__restrict__ x,
                                                    const double *__restrict__ U, double *__restrict__ V,
                                                    ChebCoef kc, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int64_t row = rm.active ? rm.row : n - 1;  // lanes past the last row read it and store nothing
    T itheta, theta, c1, c2;
    cheb_coef(kc, itheta, theta, c1, c2);
    const int c0 = rm.sub * CPT;
    Vec<T, CPT> ad = zero_v<T, CPT>();
    gather_wave<T, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, d0, ld, c0, [&](int32_t p) { return val[p]; },
                        [&](const T &v, int64_t, const Vec<T, CPT> &dj) { fma_v(ad, v, dj); });
    if (!rm.active) return;
    const Vec<T, CPT> di0 = ldv<T, CPT>(d0 + rm.row * ld + c0);
    const Vec<T, CPT> yi = ldv<T, CPT>(y + rm.row * ld + c0);
    const T di = dinv[rm.row];
    Vec<T, CPT> o;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const T r1 = theta * di0.v[c] - di * ad.v[c];
        const T d1 = c1 * di0.v[c] + c2 * r1;
        o.v[c] = yi.v[c] + di0.v[c] + d1;
    }
    if constexpr (FINAL) {
        Vec<double, CPT> u = ldv<double, CPT>(U + rm.row * ld + c0);
#pragma unroll
        for (int c = 0; c < CPT; ++c) u.v[c] += (double)o.v[c];
        stv<double, CPT>(V + rm.row * ld + c0, u);
    } else {
        stv<T, CPT>(x + rm.row * ld + c0, o);
    }
}

// ------------------------------------------------------------ small GEMM
// C (m x n) = A^T B with A (K x m, row-major, lda) and B (K x n, ldb) of
// element type T, accumulated on the FP64 matrix cores.  One workgroup per
// 16 x 16 tile of C; its four wavefronts take a quarter of K each and the
// partial tiles are summed in a fixed order.
template <typename T>
__device__ __forceinline__ void gemm_tn_tile(int m, int n, int K, const T *__restrict__ A, int lda,
                                             const T *__restrict__ B, int ldb, T *__restrict__ C, int ldc, int ta,
                                             int tb) {
    __shared__ double part[4 * 256];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int chunk = ((K + 3) / 4 + 3) & ~3;
    const int k0 = wv * chunk, k1 = K < k0 + chunk ? K : k0 + chunk;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    if (k1 > k0)
        acc = mfma_tn16_deep(
            [&](int i, int c) -> double {
                const int col = 16 * ta + c;
                return col < m ? (double)A[(int64_t)(k0 + i) * lda + col] : 0.0;
            },
            [&](int i, int c) -> double {
                const int col = 16 * tb + c;
                return col < n ? (double)B[(int64_t)(k0 + i) * ldb + col] : 0.0;
            },
            k1 - k0);
#pragma unroll
    for (int u = 0; u < 4; ++u) part[(wv * 4 + u) * kWave + lane] = acc[u];
    __syncthreads();
    const int u = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const double v = (part[(0 * 4 + u) * kWave + ln] + part[(1 * 4 + u) * kWave + ln]) +
                     (part[(2 * 4 + u) * kWave + ln] + part[(3 * 4 + u) * kWave + ln]);
    const int i = 16 * ta + (ln >> 4) + 4 * u, j = 16 * tb + (ln & 15);
    if (i < m && j < n) C[(int64_t)i * ldc + j] = (T)v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_tn(int m, int n, int K, const T *__restrict__ A, int lda,
                                                 const T *__restrict__ B, int ldb, T *__restrict__ C, int ldc,
                                                 const int *status) {
    if (status[ST_CONVERGED]) return;
    gemm_tn_tile<T>(m, n, K, A, lda, B, ldb, C, ldc, blockIdx.x, blockIdx.y);
}

// C (m x n) = A^T B as k_gemm_tn for long K: one workgroup of 16 wavefronts
// per 16 x 16 tile of C, each wavefront a sixteenth of K, the partial tiles
// summed in a fixed order in LDS.
template <typename T>
__device__ __forceinline__ void gemm_tn_long_tile(int m, int n, int K, const T *__restrict__ A, int lda,
                                                  const T *__restrict__ B, int ldb, T *__restrict__ C, int ldc,
                                                  int ta, int tb) {
    __shared__ double red[16 * 256];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int chunk = ((K + nw - 1) / nw + 3) & ~3;
    const int k0 = wv * chunk, k1 = K < k0 + chunk ? K : k0 + chunk;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    if (k1 > k0)
        acc = mfma_tn16_deep(
            [&](int i, int c) -> double {
                const int col = 16 * ta + c;
                return col < m ? (double)A[(int64_t)(k0 + i) * lda + col] : 0.0;
            },
            [&](int i, int c) -> double {
                const int col = 16 * tb + c;
                return col < n ? (double)B[(int64_t)(k0 + i) * ldb + col] : 0.0;
            },
            k1 - k0);
#pragma unroll
    for (int u = 0; u < 4; ++u) red[(wv * 4 + u) * kWave + lane] = acc[u];
    __syncthreads();
    if (threadIdx.x < 256) {
        const int u = threadIdx.x >> 6, ln = threadIdx.x & 63;
        double v = 0.0;
        for (int w = 0; w < nw; ++w) v += red[(w * 4 + u) * kWave + ln];
        const int i = 16 * ta + (ln >> 4) + 4 * u, j = 16 * tb + (ln & 15);
        if (i < m && j < n) C[(int64_t)i * ldc + j] = (T)v;
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_gemm_tn_long(int m, int n, int K, const T *__restrict__ A, int lda,
                                                       const T *__restrict__ B, int ldb, T *__restrict__ C, int ldc,
                                                       const int *status) {
    if (status[ST_CONVERGED]) return;
    gemm_tn_long_tile<T>(m, n, K, A, lda, B, ldb, C, ldc, blockIdx.x, blockIdx.y);
}

// The coarse-space products of several requests in one launch: workgroup b
// computes tile b - first[r] of request r's product (the descriptors live in
// the requests' device memory), with the same tile code as the single launch.
template <bool LONG>
__device__ __forceinline__ void gemm_batch_body(const GemmTable &t) {
    int r = 0;
    while (r + 1 < t.n && t.first[r + 1] <= (int)blockIdx.x) ++r;
    const SmallItem *it = t.item[r];
    if (it->w.status[ST_CONVERGED]) return;
    const GemmDesc g = t.which ? it->yg : it->fg;
    const int local = (int)blockIdx.x - t.first[r], tm = (g.m + 15) / 16;
    const int ta = local % tm, tb = local / tm;
    if constexpr (LONG)
        gemm_tn_long_tile<double>(g.m, g.n, g.K, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, ta, tb);
    else
        gemm_tn_tile<double>(g.m, g.n, g.K, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, ta, tb);
}
__global__ __launch_bounds__(256) void k_gemm_tn_batch(GemmTable t) { gemm_batch_body<false>(t); }
__global__ __launch_bounds__(1024) void k_gemm_tn_long_batch(GemmTable t) { gemm_batch_body<true>(t); }

// b (n x ld) = columns j0 .. j0 + ld - 1 of the identity
template <typename T>
__global__ void k_identity_block(int64_t n, int ld, int64_t j0, T *__restrict__ b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ld) return;
    const int64_t i = e / ld, c = e - i * ld;
    b[e] = i == j0 + c ? T(1) : T(0);
}

// rows j0 .. j0 + ld - 1 of Bt (n x n) = the columns of x (n x ld)
template <typename T>
__global__ void k_rows_from_block(int64_t n, int ld, int64_t j0, const T *__restrict__ x, T *__restrict__ Bt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ld) return;
    const int64_t c = e / n, i = e - c * n;  // consecutive threads: consecutive i of one column
    if (j0 + c < n) Bt[(j0 + c) * n + i] = x[i * ld + c];
}

// ------------------------------------------------------------------- a7
template <int CPT>
__global__ __launch_bounds__(256) void k_dual_spmm(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ a,
                                                   const double *__restrict__ m, const double *__restrict__ V,
                                                   double *__restrict__ W, const int *status) {
    if (status[ST_CONVERGED]) return;
    RowMap rm(ld, CPT, n);
    const int c0 = rm.sub * CPT;
    Vec<double, CPT> wa = zero_v<double, CPT>(), wm = zero_v<double, CPT>();
    gather_wave<double, CPT>(rm.row, rm.sub, rm.tpr, rm.active, n, ptr, col, V, ld, c0,
                             [&](int32_t p) { return double2{a[p], m[p]}; },
                             [&](const double2 &am, int64_t, const Vec<double, CPT> &v) {
                                 fma_v(wa, am.x, v);
                                 fma_v(wm, am.y, v);
                             });
    if (!rm.active) return;
    stv<double, CPT>(W + rm.row * 2 * ld + c0, wa);
    stv<double, CPT>(W + rm.row * 2 * ld + ld + c0, wm);
}

// Phase 1 of [V^T A V | V^T M V] = V^T W on the FP64 matrix cores: workgroup
// b takes the contiguous rows [n b / nb, n (b+1) / nb), each wavefront a
// quarter of them; per 16 x 16 tile of the ld x 2ld result the four partial
// tiles are summed in a fixed order and written to part[b].  The rows of a
// wavefront (a few KB) are re-read from cache for the later tiles.
__global__ __launch_bounds__(256) void k_gram(int64_t n, int ld, const double *__restrict__ V,
                                              const double *__restrict__ W, double *__restrict__ part,
                                              const int *status) {
    __shared__ double red[4 * 256];
    if (status[ST_CONVERGED]) return;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t nb = gridDim.x, lb = xcd_block();
    const int64_t r0 = n * lb / nb, r1 = n * (lb + 1) / nb;
    const int64_t per = (r1 - r0 + 3) / 4;
    const int64_t w0 = r0 + wv * per < r1 ? r0 + wv * per : r1;
    const int64_t w1 = w0 + per < r1 ? w0 + per : r1;
    const int K = (int)(w1 - w0);
    const int l2 = 2 * ld, ti = (ld + 15) / 16, tj = (l2 + 15) / 16;
    const int outsz = ld * l2;
    for (int t = 0; t < ti * tj; ++t) {
        const int ta = t / tj, tb = t - ta * tj;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        if (K > 0)
            acc = mfma_tn16(
                [&](int k, int c) -> double {
                    const int col = 16 * ta + c;
                    return col < ld ? V[(w0 + k) * ld + col] : 0.0;
                },
                [&](int k, int c) -> double {
                    const int col = 16 * tb + c;
                    return col < l2 ? W[(w0 + k) * l2 + col] : 0.0;
                },
                K);
#pragma unroll
        for (int u = 0; u < 4; ++u) red[(wv * 4 + u) * kWave + lane] = acc[u];
        __syncthreads();
        {
            const int u = threadIdx.x >> 6, ln = threadIdx.x & 63;
            const double v = (red[(0 * 4 + u) * kWave + ln] + red[(1 * 4 + u) * kWave + ln]) +
                             (red[(2 * 4 + u) * kWave + ln] + red[(3 * 4 + u) * kWave + ln]);
            const int i = 16 * ta + (ln >> 4) + 4 * u, j = 16 * tb + (ln & 15);
            if (i < ld && j < l2) part[lb * outsz + i * l2 + j] = v;
        }
        __syncthreads();
    }
}

// W = [A V | M V] and phase 1 of [V^T A V | V^T M V] = V^T W for wide blocks
// in one pass over the rows, so that V and W leave memory once for both
// products.  Workgroup b (eight wavefronts) walks the contiguous rows
// [n b / nb, n (b+1) / nb) in passes of R = 8 rpw rows: each wavefront gathers
// rpw rows of W as k_dual_spmm does (ld / CPT lanes per row, the lanes left
// over idle) and writes them out; the pass's rows of W and of V are staged in
// LDS (at most 98 KB for ld <= 80), and the 16 x 16 tiles on and above the
// diagonals of V^T A V and V^T M V are accumulated from there on the FP64
// matrix cores, at most four per wavefront, and written to part[b] (k_gram_reduce
// fills the entries below the diagonals from their mirror images).  Eight
// wavefronts per workgroup, four per SIMD, keep enough rows' gathers in flight
// between the barriers of a pass.
constexpr int kDualGramWaves = 8;
constexpr int kDualGramTiles = (30 + kDualGramWaves - 1) / kDualGramWaves;  // tiles per wavefront, ld <= 80
template <int CPT>
__global__ __launch_bounds__(kDualGramWaves * kWave) __attribute__((amdgpu_waves_per_eu(CPT == 8 ? 2 : 4)))
void k_dual_gram(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ a,
                                                   const double *__restrict__ m, const double *__restrict__ V,
                                                   double *__restrict__ W, double *__restrict__ part,
                                                   const int *status) {
    extern __shared__ double stage[];  // R rows of V (ld each), then the same rows of W (2 ld each)
    if (status[ST_CONVERGED]) return;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int tpr = ld / CPT, rpw = kWave / tpr, R = nw * rpw;
    const int grp = lane / tpr, sub = lane - grp * tpr, c0 = sub * CPT;
    const int64_t nb = gridDim.x, lb = xcd_block();
    const int64_t r0 = n * lb / nb, r1 = n * (lb + 1) / nb;
    const int l2 = 2 * ld, ti = (ld + 15) / 16, tu = ti * (ti + 1) / 2, ntiles = 2 * tu;
    const int outsz = ld * l2;
    const int kk = lane >> 4, c = lane & 15;
    // tile t of the upper triangles: grid half (A or M part), row tile, column
    // tile >= row tile (recomputed where used: wave-uniform scalar work)
    auto tile = [&](int t, int &off, int &ta, int &tb) {
        const int h = t < tu ? 0 : 1;
        int u = t - h * tu;
        ta = 0;
        while (ta < ti && u >= ti - ta) {
            u -= ti - ta;
            ++ta;
        }
        off = h * ld;
        tb = ta + u;
    };
    dbl4 acc[kDualGramTiles];
#pragma unroll
    for (int s2 = 0; s2 < kDualGramTiles; ++s2) acc[s2] = dbl4{0.0, 0.0, 0.0, 0.0};
    double *sv = stage, *sw = stage + R * ld;
    for (int64_t base = r0; base < r1; base += R) {  // uniform across the workgroup
        const int rows = r1 - base < R ? (int)(r1 - base) : R;
        const int lr = wv * rpw + grp;  // this lane's row within the pass
        const int64_t row = base + lr;
        const bool active = grp < rpw && lr < rows;
        Vec<double, CPT> wa = zero_v<double, CPT>(), wm = zero_v<double, CPT>();
        gather_wave<double, CPT>(row, sub, tpr, active, n, ptr, col, V, ld, c0,
                                 [&](int32_t p) { return double2{a[p], m[p]}; },
                                 [&](const double2 &am, int64_t, const Vec<double, CPT> &v) {
                                     fma_v(wa, am.x, v);
                                     fma_v(wm, am.y, v);
                                 });
        Vec<double, CPT> vi = zero_v<double, CPT>();
        if (active) {
            stv<double, CPT>(W + row * l2 + c0, wa);
            stv<double, CPT>(W + row * l2 + ld + c0, wm);
            vi = ldv<double, CPT>(V + row * ld + c0);
        }
        __syncthreads();  // the previous pass's products are done with the stage
        if (active) {
            stv<double, CPT>(sv + lr * ld + c0, vi);
            stv<double, CPT>(sw + lr * l2 + c0, wa);
            stv<double, CPT>(sw + lr * l2 + ld + c0, wm);
        }
        __syncthreads();
#pragma unroll
        for (int s2 = 0; s2 < kDualGramTiles; ++s2) {
            if (wv + s2 * nw < ntiles) {  // wave-uniform
                int off, ta, tb;
                tile(wv + s2 * nw, off, ta, tb);
                const int ca = 16 * ta + c, cb = 16 * tb + c;
                for (int k0 = 0; k0 < R; k0 += 4) {
                    const int rr = k0 + kk;
                    const double x = (ca < ld && rr < rows) ? sv[rr * ld + ca] : 0.0;
                    const double y = (cb < ld && rr < rows) ? sw[rr * l2 + off + cb] : 0.0;
                    acc[s2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[s2], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int s2 = 0; s2 < kDualGramTiles; ++s2) {
        if (wv + s2 * nw < ntiles) {
            int off, ta, tb;
            tile(wv + s2 * nw, off, ta, tb);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = 16 * ta + (lane >> 4) + 4 * u, j = 16 * tb + (lane & 15);
                if (i < ld && j < ld) part[lb * outsz + i * l2 + off + j] = acc[s2][u];
            }
        }
    }
}

// Phase 2: G[e] = sum over blocks of part[b][e]; one wavefront per element,
// lane l sums blocks l, l+64, ..., then a fixed butterfly over the lanes.
__global__ __launch_bounds__(256) void k_gram_reduce(int64_t nb, int outsz, int ld, int sym,
                                                     const double *__restrict__ part, double *__restrict__ G,
                                                     const int *status) {
    if (status[ST_CONVERGED]) return;
    const int e = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (e >= outsz) return;
    int src = e;  // with sym, an entry below the diagonal of V^T A V or V^T M V is its mirror's sum
    if (sym) {
        const int l2 = 2 * ld, i = e / l2, j = e - i * l2, h = j < ld ? 0 : ld, jl = j - h;
        if (jl < i) src = jl * l2 + h + i;
    }
    double sum = 0.0;
    for (int64_t b = lane; b < nb; b += kWave) sum += part[b * outsz + src];
    for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, kWave);
    if (lane == 0) G[e] = sum;
}

// ------------------------------------------------------------------- a11
// Narrow blocks (ld <= 32): one row group per row, X_v in LDS, the
// prolongation gathered four neighbours at a time.
template <int CPT>
__global__ __launch_bounds__(256) void k_final_rows(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                               const int32_t *__restrict__ col, const double *__restrict__ val,
                                               const double *__restrict__ Y, const double *__restrict__ V,
                                               const double *__restrict__ Xv, double *__restrict__ U,
                                               const int *status) {
    extern __shared__ double xv[];
    if (status[ST_CONVERGED]) return;
    for (int e = threadIdx.x; e < ld * ld; e += blockDim.x) xv[e] = Xv[e];
    __syncthreads();
    RowMap rm(ld, CPT, n);
    if (!rm.active) return;
    const int c0 = rm.sub * CPT;
    Vec<double, CPT> acc = zero_v<double, CPT>();
    gather4<double, CPT>(ptr[rm.row], ptr[rm.row + 1], col, Y, ld, c0,
                         [&](int32_t p, int64_t, const Vec<double, CPT> &yj) { fma_v(acc, val[p], yj); });
    const double *vr = V + rm.row * ld;
    for (int a = 0; a < ld; a += 4) {
        const Vec<double, 4> v4 = ldv<double, 4>(vr + a);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int c = 0; c < CPT; ++c) acc.v[c] += v4.v[t] * xv[(a + t) * ld + c0 + c];
    }
    stv<double, CPT>(U + rm.row * ld + c0, acc);
}

// Wide blocks: U = P Y + V X_v on the correction level.  Each wavefront owns
// 16 consecutive rows at a time and holds their V rows in registers, already
// in the matrix cores' operand layout (lane l: row l mod 16, columns 4s + l / 16),
// so V is read once whatever the number of column tiles; X_v is staged once
// per workgroup in LDS (ld x ld) and supplies the other operand.  Per 16 x 16
// column tile each lane then adds P Y for its four (row, column) entries: the
// first kPRow entries of its four rows of P are held in registers across the
// tiles, so a tile's gathers of Y are independent loads issued together.  No
// barrier after the staging of X_v; LDS of 51 KB at ld = 80 leaves room for
// three workgroups per CU.
constexpr int kPRow = 4;
constexpr int kFinalWaves = 4;
__global__ __launch_bounds__(kFinalWaves * kWave) void k_final(int64_t n, int ld, const int32_t *__restrict__ ptr,
                                               const int32_t *__restrict__ col, const double *__restrict__ val,
                                               const double *__restrict__ Y, const double *__restrict__ V,
                                               const double *__restrict__ Xv, double *__restrict__ U,
                                               const int *status) {
    extern __shared__ double xv[];  // ld x ld
    if (status[ST_CONVERGED]) return;
    for (int e = threadIdx.x; e < ld * ld; e += blockDim.x) xv[e] = Xv[e];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int c = lane & 15, kk = lane >> 4;
    const int tj = (ld + 15) / 16, ks = ld / 4;  // ld is a multiple of 4
    // the wavefronts of workgroup b take the row tiles [T b / nb, T (b+1) / nb)
    // in turn: neighbouring fine rows, whose prolongation reads the same coarse
    // rows of Y, run on the same CU close together in time
    const int64_t tiles = (n + 15) / 16, nbk = gridDim.x, lb = xcd_block();
    const int64_t t0 = tiles * lb / nbk, t1 = tiles * (lb + 1) / nbk;
    for (int64_t t = t0 + wv; t < t1; t += kFinalWaves) {
        const int64_t r0 = t * 16;
        // V rows of the tile, operand layout; rows past n read as zeros
        double a[kMaxWidth / 4];
        {
            const int64_t rr = r0 + c;
            const bool ok = rr < n;
            const double *vr = V + (ok ? rr : 0) * ld + kk;
#pragma unroll
            for (int s2 = 0; s2 < kMaxWidth / 4; ++s2) a[s2] = (ok && s2 < ks) ? vr[4 * s2] : 0.0;
        }
        int32_t pb[4], pe[4], pc[4][kPRow];
        double pv[4][kPRow];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = r0 + kk + 4 * u;
            pb[u] = row < n ? ptr[row] : 0;
            pe[u] = row < n ? ptr[row + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < kPRow; ++q) {
                const bool ok = pb[u] + q < pe[u];
                pc[u][q] = ok ? col[pb[u] + q] : 0;  // padding reads row 0 of Y with weight 0
                pv[u][q] = ok ? val[pb[u] + q] : 0.0;
            }
        for (int tb = 0; tb < tj; ++tb) {
            const int j = 16 * tb + c;
            const int jc = j < ld ? j : ld - 1;  // clamped column for the gathers
            double yv[4][kPRow];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < kPRow; ++q) yv[u][q] = Y[(int64_t)pc[u][q] * ld + jc];
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < kMaxWidth / 4; ++s2) {
                if (s2 < ks) {
                    const double b = j < ld ? xv[(4 * s2 + kk) * ld + j] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s2], b, acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t row = r0 + kk + 4 * u;
                if (row < n && j < ld) {
                    double v = acc[u];
#pragma unroll
                    for (int q = 0; q < kPRow; ++q)
                        if (pb[u] + q < pe[u]) v += pv[u][q] * yv[u][q];
                    for (int32_t pp = pb[u] + kPRow; pp < pe[u]; ++pp) v += val[pp] * Y[(int64_t)col[pp] * ld + j];
                    U[row * ld + j] = v;
                }
            }
        }
    }
}

// ------------------------------------------------------------- init fills
// SplitMix64 (Steele, Lea, Flood 2014): output k of the stream seeded with s is
// mix(s + (k+1) * 0x9E3779B97F4A7C15); element (i, j) uses k = j * n + i.
__device__ __forceinline__ uint64_t splitmix_out(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_fill_random(int64_t n, int ld, int qe, uint64_t seed, double *U) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ld) return;
    const int64_t i = e / ld;
    const int j = (int)(e - i * ld);
    double v = 0.0;
    if (j < qe) {
        const uint64_t z = splitmix_out(seed, (uint64_t)j * (uint64_t)n + (uint64_t)i);
        v = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
    }
    U[e] = v;
}

// dst (rows x dcols, leading dim ldd) <- columns [0, cols) of src (leading dim
// lds); columns [cols, dcols) are zeroed.
__global__ void k_copy_cols(int64_t rows, int dcols, int64_t ldd, int cols, const double *src, int64_t lds,
                            double *dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * dcols) return;
    const int64_t i = e / dcols;
    const int j = (int)(e - i * dcols);
    dst[i * ldd + j] = j < cols ? src[i * lds + j] : 0.0;
}

__global__ void k_copy_f64(int64_t count, const double *src, double *dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) dst[e] = src[e];
}

__global__ void k_fill_i32(int count, int value, int *dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) dst[e] = value;
}

// ------------------------------------------------------------ launchers
namespace {
constexpr int kBlock = 256;

// workgroups of the row kernels (RowMap): n rows of ld / cpt threads each
inline int64_t row_blocks(int64_t n, int ld, int cpt) {
    const int64_t threads = n * (ld / cpt);
    return (threads + kBlock - 1) / kBlock;
}
}  // namespace

// Columns per lane for a row-major block of the given width when no tuned
// value is set: 4 (16-byte FP32 and 32-byte FP64 accesses per lane) when the
// width allows it, else 2, else 8.  With RowMap's flat numbering every lane
// has work whatever the choice; the autotuner times the others.
int cpt_for(int width) {
    for (int c : {4, 2, 8})
        if (width % c == 0 && width / c <= kWave) return c;
    return 8;
}

bool cpt_valid(int width, int cpt) {
    return (cpt == 2 || cpt == 4 || cpt == 8) && width % cpt == 0 && width / cpt <= kWave;
}

// `hint` when it is a valid choice for the width (a tuned value), else cpt_for.
int pick_cpt(int width, int hint) { return cpt_valid(width, hint) ? hint : cpt_for(width); }

// Events handed to the next launch of a single-kernel timing site: recorded by
// the dispatch itself at the kernel's start and end (hipExtLaunchKernelGGL),
// so their elapsed time is the kernel's own duration.
namespace {
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;
}
void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_ev_start = start;
    t_ev_stop = stop;
}
bool launch_events_pending() { return t_ev_start != nullptr; }
void clear_launch_events() { t_ev_start = t_ev_stop = nullptr; }

#define KLAUNCH(K, G, B, SH, S, ...)                                                  \
    do {                                                                              \
        if (t_ev_start) {                                                             \
            hipEvent_t e0_ = t_ev_start, e1_ = t_ev_stop;                             \
            t_ev_start = t_ev_stop = nullptr;                                         \
            hipExtLaunchKernelGGL(K, G, B, (std::uint32_t)(SH), S, e0_, e1_, 0, __VA_ARGS__); \
        } else {                                                                      \
            hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                          \
        }                                                                             \
    } while (0)

#define DISPATCH_CPT(width, hint, ...)             \
    do {                                           \
        const int cpt_sel = pick_cpt(width, hint); \
        if (cpt_sel == 2) {                  \
            constexpr int CPT = 2;           \
            __VA_ARGS__;                     \
        } else if (cpt_sel == 4) {           \
            constexpr int CPT = 4;           \
            __VA_ARGS__;                     \
        } else {                             \
            constexpr int CPT = 8;           \
            __VA_ARGS__;                     \
        }                                    \
    } while (0)

int64_t residual_blocks(int64_t n, int ld, int cpt) {
    const int64_t need = row_blocks(n, ld, pick_cpt(ld, cpt));
    return need < 2048 ? need : 2048;
}

int64_t residual_blocks_max(int64_t n, int ld) {  // over every columns-per-lane choice
    int64_t best = residual_blocks(n, ld, 0);
    for (int c = 2; c <= 8; c *= 2)
        if (cpt_valid(ld, c)) best = std::max(best, residual_blocks(n, ld, c));
    return best;
}

template <typename TO>
void launch_residual(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                     const double *m, const double *U, const double *theta, TO *R, double *part, const int *status,
                     int cpt) {
    // part: 2 ld final sums, then nb x 2 ld per-block partials
    const int64_t nb = residual_blocks(n, ld, cpt);
    double *blocks = part + 2 * ld;
    DISPATCH_CPT(ld, cpt, KLAUNCH((k_residual<TO, CPT>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, ld,
                                             ptr, col, a, m, U, theta, R, blocks, status));
}

template <typename TO>
void launch_residual_cycle(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                           const double *m, const double *U, const double *V, const double *theta, double sigma, TO *R,
                           const int *status, int cpt) {
    DISPATCH_CPT(ld, cpt, KLAUNCH((k_residual_cycle<TO, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)), dim3(kBlock),
                                  0, s, n, ld, ptr, col, a, m, U, V, theta, sigma, R, status));
}

void launch_residual_finish(hipStream_t s, int64_t n, int ld, double *part, unsigned *counter, const double *theta,
                            double *rho, int q, double tol, int *status, int check, int cpt) {
    const int64_t nb = residual_blocks(n, ld, cpt);
    hipLaunchKernelGGL(k_residual_finish, dim3(2 * ld), dim3(kBlock), 0, s, nb, ld, part + 2 * ld, part, counter,
                       theta, rho, q, tol, status, check);
}

template <typename T>
void launch_smooth_pre(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *vs,
                       const T *dinv, const T *b, T *r, const int *status, int cpt) {
    DISPATCH_CPT(ld, cpt, KLAUNCH((k_smooth_pre<T, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)), dim3(kBlock),
                                        0, s, n, ld, ptr, col, vs, dinv, b, r, status));
}

template <typename T>
void launch_spmm(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                 const T *x, T *y, const int *status, int cpt) {
    DISPATCH_CPT(ld, cpt, KLAUNCH((k_spmm<T, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)), dim3(kBlock), 0, s,
                                        n, ld, ptr, col, val, x, y, status));
}

template <typename T>
void launch_prolong_add(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                        const T *xc, const T *dinv, const T *b, T *y, const int *status, int cpt) {
    DISPATCH_CPT(ld, cpt, hipLaunchKernelGGL((k_prolong_add<T, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)),
                                        dim3(kBlock), 0, s, n, ld, ptr, col, val, xc, dinv, b, y, status));
}

template <typename T>
void launch_smooth_post(hipStream_t s, bool final, int64_t n, int ld, const int32_t *ptr, const int32_t *col,
                        const T *val, const T *dinv, const T *b, const T *y, T *x, const double *U, double *V,
                        const int *status, int cpt) {
    if (final)
        DISPATCH_CPT(ld, cpt, KLAUNCH((k_smooth_post<T, CPT, true>), dim3((unsigned)row_blocks(n, ld, CPT)),
                                            dim3(kBlock), 0, s, n, ld, ptr, col, val, dinv, b, y, x, U, V, status));
    else
        DISPATCH_CPT(ld, cpt, KLAUNCH((k_smooth_post<T, CPT, false>), dim3((unsigned)row_blocks(n, ld, CPT)),
                                            dim3(kBlock), 0, s, n, ld, ptr, col, val, dinv, b, y, x, U, V, status));
}

template <typename T>
void launch_gs_colour(hipStream_t s, bool final, int64_t nrows, int ld, const int32_t *ptr, const int32_t *col,
                      const T *val, const T *diag, const int32_t *rows, const T *b, T *x, const double *U, double *V,
                      const int *status, int cpt) {
    if (nrows <= 0) return;
    if (final)
        DISPATCH_CPT(ld, cpt, KLAUNCH((k_gs_colour<T, CPT, true>), dim3((unsigned)row_blocks(nrows, ld, CPT)),
                                            dim3(kBlock), 0, s, nrows, ld, ptr, col, val, diag, rows, b, x, U, V,
                                            status));
    else
        DISPATCH_CPT(ld, cpt, KLAUNCH((k_gs_colour<T, CPT, false>), dim3((unsigned)row_blocks(nrows, ld, CPT)),
                                            dim3(kBlock), 0, s, nrows, ld, ptr, col, val, diag, rows, b, x, U, V,
                                            status));
}

void launch_dual_spmm(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                      const double *m, const double *V, double *W, const int *status, int cpt) {
    DISPATCH_CPT(ld, cpt, KLAUNCH((k_dual_spmm<CPT>), dim3((unsigned)row_blocks(n, ld, CPT)), dim3(kBlock), 0,
                                        s, n, ld, ptr, col, a, m, V, W, status));
}

int64_t gram_blocks(int64_t n, int ld) {  // about 64 rows per wavefront, at most 1024 workgroups
    (void)ld;
    int64_t nb = (n + 255) / 256;
    return nb < 1024 ? (nb < 1 ? 1 : nb) : 1024;
}

// narrow blocks (ld <= 32); wider ones take launch_dual_gram
void launch_gram(hipStream_t s, int64_t n, int ld, const double *V, const double *W, double *part, double *G,
                 const int *status) {
    const int64_t nb = gram_blocks(n, ld);
    const int outsz = 2 * ld * ld;
    hipLaunchKernelGGL(k_gram, dim3((unsigned)nb), dim3(kBlock), 0, s, n, ld, V, W, part, status);
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((outsz + 3) / 4)), dim3(256), 0, s, nb, outsz, ld, 0, part, G,
                       status);
}

bool dual_gram_fused(int ld) { return (ld + 15) / 16 * ((2 * ld + 15) / 16) > 8; }  // the wide Gram layout

void launch_dual_gram(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                      const double *m, const double *V, double *W, double *part, const int *status, int cpt) {
    const int64_t nb = gram_blocks(n, ld);
    DISPATCH_CPT(ld, cpt, {
        const int rows = kDualGramWaves * (kWave / (ld / CPT));
        KLAUNCH((k_dual_gram<CPT>), dim3((unsigned)nb), dim3(kDualGramWaves * kWave),
                (size_t)rows * 3 * ld * sizeof(double), s,
                n, ld, ptr, col, a, m, V, W, part, status);
    });
}

void launch_gram_reduce(hipStream_t s, int64_t n, int ld, const double *part, double *G, const int *status) {
    const int64_t nb = gram_blocks(n, ld);
    const int outsz = 2 * ld * ld;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((outsz + 3) / 4)), dim3(256), 0, s, nb, outsz, ld,
                       dual_gram_fused(ld) ? 1 : 0, part, G, status);
}

void launch_final(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *val,
                  const double *Y, const double *V, const double *Xv, double *U, const int *status, int cpt) {
    if (ld <= 32) {
        DISPATCH_CPT(ld, cpt, KLAUNCH((k_final_rows<CPT>), dim3((unsigned)row_blocks(n, ld, CPT)),
                                            dim3(kBlock), (size_t)ld * ld * sizeof(double), s, n, ld, ptr, col, val,
                                            Y, V, Xv, U, status));
        return;
    }
    // workgroups of four wavefronts, each owning a contiguous range of 16-row
    // tiles; LDS holds X_v only
    const int64_t tiles = (n + 15) / 16;
    const int64_t want = (tiles + kFinalWaves * 32 - 1) / (kFinalWaves * 32);  // about 32 tiles per wavefront
    const int64_t nb = want < 1 ? 1 : (want > 2048 ? 2048 : want);
    KLAUNCH(k_final, dim3((unsigned)nb), dim3(kFinalWaves * kWave), (size_t)ld * ld * sizeof(double), s, n, ld, ptr,
            col, val, Y, V, Xv, U, status);
}

template <typename T>
void launch_gemm_tn(hipStream_t s, int m, int n, int K, const T *A, int lda, const T *B, int ldb, T *C, int ldc,
                    const int *status) {
    const dim3 g((m + 15) / 16, (n + 15) / 16);
    hipLaunchKernelGGL(k_gemm_tn<T>, g, dim3(256), 0, s, m, n, K, A, lda, B, ldb, C, ldc, status);
}
template void launch_gemm_tn<float>(hipStream_t, int, int, int, const float *, int, const float *, int, float *, int,
                                    const int *);
template void launch_gemm_tn<double>(hipStream_t, int, int, int, const double *, int, const double *, int, double *,
                                     int, const int *);

ChebCoef cheb_coefficients(double lo) {
    const double theta = 0.5 * (1.0 + lo), delta = 0.5 * (1.0 - lo);
    const double sigma = theta / delta, rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
    ChebCoef k;
    k.ditheta = 1.0 / theta;
    k.dtheta = theta;
    k.dc1 = rho1 * rho0;
    k.dc2 = 2.0 * rho1 / delta;
    k.itheta = (float)k.ditheta;
    k.theta = (float)k.dtheta;
    k.c1 = (float)k.dc1;
    k.c2 = (float)k.dc2;
    return k;
}

template <typename T>
void launch_cheb_pre(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *vs,
                     const T *dinv, const T *b, T *x, double lo, const int *status, int cpt) {
    const ChebCoef kc = cheb_coefficients(lo);
    DISPATCH_CPT(ld, cpt, KLAUNCH((k_cheb_pre<T, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)), dim3(kBlock),
                                        0, s, n, ld, ptr, col, vs, dinv, b, x, kc, status));
}

template <typename T>
void launch_level_residual(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                           const T *b, const T *x, T *r, const int *status, int cpt) {
    DISPATCH_CPT(ld, cpt, hipLaunchKernelGGL((k_level_residual<T, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)),
                                        dim3(kBlock), 0, s, n, ld, ptr, col, val, b, x, r, status));
}

template <typename T>
void launch_prolong_x(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                      const T *xc, const T *x, T *y, const int *status, int cpt) {
    DISPATCH_CPT(ld, cpt, hipLaunchKernelGGL((k_prolong_x<T, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)), dim3(kBlock),
                                        0, s, n, ld, ptr, col, val, xc, x, y, status));
}

template <typename T>
void launch_cheb_post1(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                       const T *dinv, const T *b, const T *y, T *d0, double lo, const int *status, int cpt) {
    const ChebCoef kc = cheb_coefficients(lo);
    DISPATCH_CPT(ld, cpt, hipLaunchKernelGGL((k_cheb_post1<T, CPT>), dim3((unsigned)row_blocks(n, ld, CPT)), dim3(kBlock),
                                        0, s, n, ld, ptr, col, val, dinv, b, y, d0, kc, status));
}

template <typename T>
void launch_cheb_post2(hipStream_t s, bool final, int64_t n, int ld, const int32_t *ptr, const int32_t *col,
                       const T *val, const T *dinv, const T *y, const T *d0, T *x, const double *U, double *V,
                       double lo, const int *status, int cpt) {
    const ChebCoef kc = cheb_coefficients(lo);
    if (final)
        DISPATCH_CPT(ld, cpt, KLAUNCH((k_cheb_post2<T, CPT, true>), dim3((unsigned)row_blocks(n, ld, CPT)),
                                            dim3(kBlock), 0, s, n, ld, ptr, col, val, dinv, y, d0, x, U, V, kc,
                                            status));
    else
        DISPATCH_CPT(ld, cpt, KLAUNCH((k_cheb_post2<T, CPT, false>), dim3((unsigned)row_blocks(n, ld, CPT)),
                                            dim3(kBlock), 0, s, n, ld, ptr, col, val, dinv, y, d0, x, U, V, kc,
                                            status));
}

template <typename T>
void launch_gemm_tn_long(hipStream_t s, int m, int n, int K, const T *A, int lda, const T *B, int ldb, T *C, int ldc,
                         const int *status) {
    const dim3 g((m + 15) / 16, (n + 15) / 16);
    hipLaunchKernelGGL(k_gemm_tn_long<T>, g, dim3(1024), 0, s, m, n, K, A, lda, B, ldb, C, ldc, status);
}
template void launch_gemm_tn_long<float>(hipStream_t, int, int, int, const float *, int, const float *, int, float *,
                                         int, const int *);

void launch_gemm_batch(hipStream_t s, const GemmTable &t, bool long_k) {
    if (t.n <= 0 || t.first[t.n] <= 0) return;
    if (long_k)
        hipLaunchKernelGGL(k_gemm_tn_long_batch, dim3((unsigned)t.first[t.n]), dim3(1024), 0, s, t);
    else
        hipLaunchKernelGGL(k_gemm_tn_batch, dim3((unsigned)t.first[t.n]), dim3(256), 0, s, t);
}
template void launch_gemm_tn_long<double>(hipStream_t, int, int, int, const double *, int, const double *, int,
                                          double *, int, const int *);

template <typename T>
void launch_identity_block(hipStream_t s, int64_t n, int ld, int64_t j0, T *b) {
    const int64_t tot = n * ld;
    hipLaunchKernelGGL(k_identity_block<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, ld, j0, b);
}
template void launch_identity_block<float>(hipStream_t, int64_t, int, int64_t, float *);
template void launch_identity_block<double>(hipStream_t, int64_t, int, int64_t, double *);

template <typename T>
void launch_rows_from_block(hipStream_t s, int64_t n, int ld, int64_t j0, const T *x, T *Bt) {
    const int64_t tot = n * ld;
    hipLaunchKernelGGL(k_rows_from_block<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, ld, j0, x,
                       Bt);
}
template void launch_rows_from_block<float>(hipStream_t, int64_t, int, int64_t, const float *, float *);
template void launch_rows_from_block<double>(hipStream_t, int64_t, int, int64_t, const double *, double *);

void launch_fill_random(hipStream_t s, int64_t n, int ld, int qe, uint64_t seed, double *U) {
    const int64_t tot = n * ld;
    hipLaunchKernelGGL(k_fill_random, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, ld, qe, seed, U);
}

void launch_copy_cols(hipStream_t s, int64_t rows, int dcols, int64_t ldd, int cols, const double *src,
                      int64_t lds, double *dst) {
    const int64_t tot = rows * dcols;
    if (tot == 0) return;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rows, dcols, ldd, cols, src,
                       lds, dst);
}

void launch_copy_f64(hipStream_t s, int64_t count, const double *src, double *dst) {
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, src, dst);
}

void launch_fill_i32(hipStream_t s, int count, int value, int *dst) {
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, value, dst);
}

#define INST(T)                                                                                                      \
    template void launch_smooth_pre<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const T *,       \
                                       const T *, const T *, T *, const int *, int);                                      \
    template void launch_spmm<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const T *, const T *,  \
                                 T *, const int *, int);                                                                  \
    template void launch_prolong_add<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const T *,      \
                                        const T *, const T *, const T *, T *, const int *, int);                          \
    template void launch_smooth_post<T>(hipStream_t, bool, int64_t, int, const int32_t *, const int32_t *,           \
                                        const T *, const T *, const T *, const T *, T *, const double *, double *,   \
                                        const int *, int);                                                                \
    template void launch_gs_colour<T>(hipStream_t, bool, int64_t, int, const int32_t *, const int32_t *, const T *,   \
                                      const T *, const int32_t *, const T *, T *, const double *, double *,          \
                                      const int *, int);                                                             \
    template void launch_residual_cycle<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *,              \
                                           const double *, const double *, const double *, const double *,            \
                                           const double *, double, T *, const int *, int);                            \
    template void launch_residual<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const double *,    \
                                     const double *, const double *, const double *, T *, double *, const int *,      \
                                     int);                                                                            \
    template void launch_cheb_pre<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const T *,         \
                                     const T *, const T *, T *, double, const int *, int);                                \
    template void launch_level_residual<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const T *,   \
                                           const T *, const T *, T *, const int *, int);                                  \
    template void launch_prolong_x<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const T *,        \
                                      const T *, const T *, T *, const int *, int);                                       \
    template void launch_cheb_post1<T>(hipStream_t, int64_t, int, const int32_t *, const int32_t *, const T *,       \
                                       const T *, const T *, const T *, T *, double, const int *, int);                   \
    template void launch_cheb_post2<T>(hipStream_t, bool, int64_t, int, const int32_t *, const int32_t *, const T *, \
                                       const T *, const T *, const T *, T *, const double *, double *, double,       \
                                       const int *, int);
INST(float)
INST(double)
#undef INST

}  // namespace amgeig
