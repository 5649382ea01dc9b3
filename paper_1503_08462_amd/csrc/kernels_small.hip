// Small dense kernels of the Rayleigh-Ritz step (Algorithm 3.1, step 2), FP64.
//
// The coarse basis Q_c = I_n^k Z (Z: coarsest eigenvectors, Z^T M_n Z = I,
// Z^T A_n Z = Lambda) is augmented with the new block V.  With
//   B = I_k^n [A V | M V],  F = Z^T B_A,  G = Z^T B_M,
// the part of V that is M-orthogonal to the coarse space, V_perp = V - Q_c G,
// has Gram matrices
//   D_M = V^T M V - G^T G,
//   D_A = V^T A V - G^T F - F^T G + G^T Lambda G,
// and couples to the coarse basis by C = F - Lambda G.  A pivoted Cholesky
// D_M(perm, perm) = L L^T keeps the r numerically independent columns, so the
// projected pencil of eq. (3.3) becomes the standard symmetric matrix
//   H = [[Lambda, C~], [C~^T, D~]],  C~ = C(:, perm_r) L^-T,  D~ = L^-1 D_A(perm_r, perm_r) L^-T,
// the same Ritz pairs as the paper's (A_{n,k}, M_{n,k}) written in an
// M-orthonormal basis.  Its q_e smallest eigenpairs are found by
//   - Sylvester inertia counts nu(s) = #{lambda_i < s} + #neg(S(s)),
//     S(s) = D~ - s I - C~^T (Lambda - s)^-1 C~ (Bunch-Kaufman LDL^T), in a
//     bisection per eigenvalue (one workgroup each),
//   - inverse iteration with the same Schur-complement factorisation,
//   - Cholesky-QR orthonormalisation and a final Rayleigh-Ritz (cyclic Jacobi)
//     on the span of the computed vectors.
#include "device_common.h"
#include "kernels.h"

namespace amgeig {

namespace {

constexpr int kB = 256;  // threads per block of the small kernels
// The single-workgroup pencil and Rayleigh-Ritz kernels of wide blocks
// (ld > 32, operands beyond LDS in global memory) run sixteen wavefronts:
// their products deal 16 x 16 tiles to the wavefronts, each tile summed by one
// wavefront in a fixed order, so more wavefronts hide more load latency and
// leave the results unchanged.
constexpr int kBWide = 1024;
inline int small_threads(int ld) { return ld > 32 ? kBWide : kB; }
// The eigenvalue workgroups of wide blocks run eight wavefronts: the register
// budget of sixteen would not hold the deep product pipeline.
constexpr int kBisectWide = 512;
inline int bisect_threads(int ld) { return ld > 32 ? kBisectWide : kB; }

// Solver statistics (inertia counts per eigenvalue, fallbacks, Jacobi sweeps
// and phase clocks, added into w.diag) are compiled in only with
// -DAMG_EIG_SMALL_STATS=1.  Otherwise no clock is read and w.diag is null, so
// every statistics branch is skipped.
#ifndef AMG_EIG_SMALL_STATS
#define AMG_EIG_SMALL_STATS 0
#endif
__device__ __forceinline__ uint64_t stat_clock() {
#if AMG_EIG_SMALL_STATS
    return wall_clock64();
#else
    return 0;
#endif
}
// Rayleigh-quotient iteration stops at ||H x - rho x|| <= kRqiTol |rho|.  The
// Rayleigh-Ritz polish over the span of all accepted vectors then leaves the
// Ritz values with errors of the order of the squared residual over the gap.
constexpr double kRqiTol = 1e-8;

// ---------------------------------------------------------------------
// Value of v in lane `src` of the wavefront (src must be wave-uniform).
__device__ __forceinline__ double lane_bcast(double v, int src) {
    src = __builtin_amdgcn_readfirstlane(src);
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the wavefront; the xor butterfly leaves the same bits in every lane.
__device__ __forceinline__ double wave_allsum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Largest v over the wavefront and the lowest index holding it; every lane
// ends with the same pair.  Applied to per-lane scans that keep the first of
// equal values (strict >), it selects what one scan in index order selects.
__device__ __forceinline__ void wave_argmax(double &v, int &idx) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, kWave);
        const int oi = __shfl_xor(idx, off, kWave);
        const bool take = ov > v || (ov == v && oi < idx);
        v = take ? ov : v;
        idx = take ? oi : idx;
    }
}

__device__ __forceinline__ double wave_allmax(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// X = L^-1 for the lower triangular r x r matrix whose entries L(i, k), i >= k,
// the accessor returns, into X (row stride xs, zero above the diagonal).  Right-looking: step k subtracts L_ik times row
// k of the inverse from the rows i > k, where row k is X(k, :) / L_kk, the
// division of a forward substitution; the stored row k receives that quotient
// one step later, once nobody reads it.  Every entry thus sees the subtractions
// in increasing k and one division, as in a column-by-column substitution, with
// one barrier per step.
template <class LF>
__device__ void tri_inverse(LF L, double *X, int xs, int r) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int e = tid; e < r * r; e += nthr) {
        const int a = e / r, b = e - a * r;
        X[a * xs + b] = a == b ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        const double lkk = L(k, k);
        const int rows = r - 1 - k, cols = k + 1;
        for (int e = tid; e < rows * cols; e += nthr) {
            const int i = k + 1 + e / cols, c = e - (i - k - 1) * cols;
            X[i * xs + c] -= L(i, k) * (X[k * xs + c] / lkk);
        }
        if (k > 0) {  // row k - 1 is no longer read: store its quotient
            const double lpp = L(k - 1, k - 1);
            for (int c = tid; c < k; c += nthr) X[(k - 1) * xs + c] /= lpp;
        }
        __syncthreads();
    }
    if (r > 0)
        for (int c = tid; c < r; c += nthr) X[(r - 1) * xs + c] /= L(r - 1, r - 1);
    __syncthreads();
}

// Bunch-Kaufman symmetric indefinite LDL^T of S (r x r, LDS, row stride ls).
// D (1x1 and 2x2 diagonal blocks) stays on the diagonal of S, the multipliers
// go to the strict lower part of Lm (same stride).
// ipiv[p] = kp >= 0: 1x1 pivot, rows p and kp interchanged;
// ipiv[p] = ipiv[p+1] = -(kp+1): 2x2 pivot, rows p+1 and kp interchanged.
// Returns the number of negative eigenvalues of S (Sylvester's law).  Every
// wavefront evaluates the pivot choice itself from the shared column (a scan
// split over its lanes and a butterfly reduction), so a pivot step costs one
// barrier, two with an interchange.  The trailing update evaluates the same
// product for (i, j) and (j, i): the active part stays exactly symmetric.
__device__ int bk_factor(double *S, double *Lm, int r, int ls, int *ipiv) {
    const double alpha = 0.6403882032022076;  // (1 + sqrt(17)) / 8
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & (kWave - 1);
    const int tx = tid & 15, ty = tid >> 4, nty = nthr >> 4;
    int neg = 0;
    int p = 0;
    while (p < r) {
        double colmax = 0.0;  // largest |S[i][p]|, i > p, lowest index on ties
        int imax = p;
        for (int i = p + 1 + lane; i < r; i += kWave) {
            const double v = fabs(S[i * ls + p]);
            imax = v > colmax ? i : imax;
            colmax = v > colmax ? v : colmax;
        }
        wave_argmax(colmax, imax);
        const double absakk = fabs(S[p * ls + p]);
        int kp = p, size = 1;
        const bool read_row = colmax > 0.0 && absakk < alpha * colmax;  // the same in every thread
        if (read_row) {
            double rowmax = 0.0;
            for (int j = p + lane; j < r; j += kWave)
                if (j != imax) rowmax = fmax(rowmax, fabs(S[imax * ls + j]));
            rowmax = wave_allmax(rowmax);
            if (absakk * rowmax >= alpha * colmax * colmax) {
                kp = p;
            } else if (fabs(S[imax * ls + imax]) >= alpha * rowmax) {
                kp = imax;
            } else {
                kp = imax;
                size = 2;
            }
        }
        const int tgt = size == 1 ? p : p + 1;
        if (read_row && kp == tgt) __syncthreads();  // row imax is read before the update writes it
        if (kp != tgt) {  // symmetric interchange of tgt and kp, with the multipliers found so far
            __syncthreads();  // every thread has read the pivot column
            for (int j = tid; j < r; j += nthr) {
                if (j == tgt || j == kp) continue;
                double t = S[tgt * ls + j];
                S[tgt * ls + j] = S[kp * ls + j];
                S[kp * ls + j] = t;
                t = S[j * ls + tgt];
                S[j * ls + tgt] = S[j * ls + kp];
                S[j * ls + kp] = t;
                if (j < p) {
                    t = Lm[tgt * ls + j];
                    Lm[tgt * ls + j] = Lm[kp * ls + j];
                    Lm[kp * ls + j] = t;
                }
            }
            if (tid == 0) {
                const double t = S[tgt * ls + tgt];
                S[tgt * ls + tgt] = S[kp * ls + kp];
                S[kp * ls + kp] = t;
            }
            __syncthreads();
        }
        if (size == 1) {
            const double d = S[p * ls + p];
            const double dinv = d != 0.0 ? 1.0 / d : 0.0;
            neg += d < 0.0 ? 1 : 0;
            if (tid == 0) ipiv[p] = kp;
            for (int i = p + 1 + ty; i < r; i += nty) {
                const double ci = S[i * ls + p], li = ci * dinv;
                for (int j = p + 1 + tx; j < r; j += 16) {
                    const double cj = S[j * ls + p];
                    S[i * ls + j] -= i >= j ? li * cj : (cj * dinv) * ci;
                }
                if (tx == 0) Lm[i * ls + p] = li;
            }
            __syncthreads();
            p += 1;
        } else {
            const double a = S[p * ls + p], b = S[(p + 1) * ls + p], c = S[(p + 1) * ls + p + 1];
            const double det = a * c - b * b;
            neg += det < 0.0 ? 1 : (a + c < 0.0 ? 2 : 0);
            if (tid == 0) ipiv[p] = ipiv[p + 1] = -(kp + 1);
            const double id = 1.0 / det;
            for (int i = p + 2 + ty; i < r; i += nty) {
                const double c1i = S[i * ls + p], c2i = S[i * ls + p + 1];
                const double l1 = (c1i * c - c2i * b) * id, l2 = (c2i * a - c1i * b) * id;
                for (int j = p + 2 + tx; j < r; j += 16) {
                    const double c1j = S[j * ls + p], c2j = S[j * ls + p + 1];
                    double t;
                    if (i >= j) {
                        t = l1 * c1j + l2 * c2j;
                    } else {
                        const double m1 = (c1j * c - c2j * b) * id, m2 = (c2j * a - c1j * b) * id;
                        t = m1 * c1i + m2 * c2i;
                    }
                    S[i * ls + j] -= t;
                }
                if (tx == 0) {
                    Lm[i * ls + p] = l1;
                    Lm[i * ls + p + 1] = l2;
                }
            }
            __syncthreads();
            p += 2;
        }
    }
    return neg;
}

// Solve S z = f with the factors of bk_factor (D in S, L in Lm; f in LDS,
// overwritten by z).
// Wavefront 0 keeps f in registers (entry i in lane i mod 64, slot i / 64,
// r <= 128) and exchanges values by lane reads; the other wavefronts wait at
// the closing barrier.
__device__ void bk_solve(const double *S, const double *Lm, int r, int ls, const int *ipiv, double *f) {
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        double f0 = lane < r ? f[lane] : 0.0;
        double f1 = lane + kWave < r ? f[lane + kWave] : 0.0;
        auto get = [&](int i) __attribute__((always_inline)) -> double {
            const double src = i < kWave ? f0 : f1;  // value select: f0, f1 stay in registers
            return lane_bcast(src, i & (kWave - 1));
        };
        auto put = [&](int i, double v) __attribute__((always_inline)) {
            const bool mine = lane == (i & (kWave - 1));
            f0 = (mine && i < kWave) ? v : f0;
            f1 = (mine && i >= kWave) ? v : f1;
        };
        auto swap = [&](int a, int b) __attribute__((always_inline)) {
            if (a == b) return;
            const double va = get(a), vb = get(b);
            put(a, vb);
            put(b, va);
        };
        // axpy on the entries i in [lo, hi): f_i -= col(i) * s, col read from S
        auto axpy_col = [&](int lo, int hi, int c, double s) __attribute__((always_inline)) {
            if (lane >= lo && lane < hi) f0 -= Lm[lane * ls + c] * s;
            if (lane + kWave >= lo && lane + kWave < hi) f1 -= Lm[(lane + kWave) * ls + c] * s;
        };
        auto axpy_row = [&](int hi, int rw, double s) __attribute__((always_inline)) {  // f_i -= L[rw][i] s, i < hi
            if (lane < hi) f0 -= Lm[rw * ls + lane] * s;
            if (lane + kWave < hi) f1 -= Lm[rw * ls + lane + kWave] * s;
        };
        // the pivot record and the diagonal blocks in registers (entry p in lane
        // p mod 64), read by lane reads instead of one shared-memory load per step
        const int iv0 = lane < r ? ipiv[lane] : 0, iv1 = lane + kWave < r ? ipiv[lane + kWave] : 0;
        const double dg0 = lane < r ? S[lane * ls + lane] : 0.0;
        const double dg1 = lane + kWave < r ? S[(lane + kWave) * ls + lane + kWave] : 0.0;
        const double sb0 = lane + 1 < r ? S[(lane + 1) * ls + lane] : 0.0;
        const double sb1 = lane + kWave + 1 < r ? S[(lane + kWave + 1) * ls + lane + kWave] : 0.0;
        auto piv = [&](int p) __attribute__((always_inline)) -> int {
            return __builtin_amdgcn_readlane(p < kWave ? iv0 : iv1, p & (kWave - 1));
        };
        auto diag = [&](int p) __attribute__((always_inline)) -> double {  // S[p][p]
            return lane_bcast(p < kWave ? dg0 : dg1, p & (kWave - 1));
        };
        auto subd = [&](int p) __attribute__((always_inline)) -> double {  // S[p + 1][p]
            return lane_bcast(p < kWave ? sb0 : sb1, p & (kWave - 1));
        };
        for (int p = 0; p < r;) {  // interchanges in order
            const int ip = piv(p);
            if (ip >= 0) {
                swap(p, ip);
                p += 1;
            } else {
                swap(p + 1, -ip - 1);
                p += 2;
            }
        }
        for (int p = 0; p < r;) {  // L y = f
            if (piv(p) >= 0) {
                axpy_col(p + 1, r, p, get(p));
                p += 1;
            } else {
                const double y0 = get(p), y1 = get(p + 1);
                axpy_col(p + 2, r, p, y0);
                axpy_col(p + 2, r, p + 1, y1);
                p += 2;
            }
        }
        for (int p = 0; p < r;) {  // D solve; singular pivots are replaced by a tiny value
            if (piv(p) >= 0) {
                double d = diag(p);
                if (d == 0.0) d = 1e-300;
                put(p, get(p) / d);
                p += 1;
            } else {
                const double a = diag(p), b = subd(p), c = diag(p + 1);
                const double det = a * c - b * b;
                const double y0 = get(p), y1 = get(p + 1);
                put(p, (c * y0 - b * y1) / det);
                put(p + 1, (a * y1 - b * y0) / det);
                p += 2;
            }
        }
        for (int p = r - 1; p >= 0;) {  // L^T w = y, last block first
            if (piv(p) < 0) {
                const int p0 = p - 1;
                const double w0 = get(p0), w1 = get(p);
                axpy_row(p0, p0, w0);
                axpy_row(p0, p, w1);
                p -= 2;
            } else {
                axpy_row(p, p, get(p));
                p -= 1;
            }
        }
        for (int p = r - 1; p >= 0;) {  // undo the interchanges in reverse order
            const int ip = piv(p);
            if (ip < 0) {
                swap(p, -ip - 1);
                p -= 2;
            } else {
                swap(p, ip);
                p -= 1;
            }
        }
        if (lane < r) f[lane] = f0;
        if (lane + kWave < r) f[lane + kWave] = f1;
    }
    __syncthreads();
}

// Pseudo-random start vector entry in (-1, 1) for eigenvalue k, row i.
__device__ __forceinline__ double start_entry(int k, int i) {
    uint64_t z = (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull + (uint64_t)(i + 1) * 0xD1B54A32D192ED03ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

}  // namespace

// ------------------------------------------------------------- pencil (a9)
// One workgroup.  P3 = G^T [F | G | Lambda G] on the matrix cores, the Gram
// blocks D_M, D_A of the part of V outside the coarse space, a pivoted
// Cholesky D_M(perm, perm) = L L^T stopped at rank r (pivot below
// rank_tol * max diag(V^T M V)), D~ = L^-1 D_A(perm_r, perm_r) L^-T and
// C~ = (F - Lambda G)(:, perm_r) L^-T.  The pivot choice is evaluated by every
// thread from the shared diagonal (no broadcast through shared memory).
constexpr int kRedSmall = 3 * 4 * 256;

__device__ __forceinline__ void pencil_body(SmallWork w, double rank_tol, int fg_in_lds) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn, tid = threadIdx.x, nthr = blockDim.x, lane = tid & (kWave - 1);
    const int tx = tid & 15, ty = tid >> 4, nty = nthr >> 4;
    // ld <= 32: everything in LDS; wider: D_M, D_A, L^-1 in LDS, P3 and
    // [V^T A V | V^T M V] in global memory.  The ld x ld matrices in LDS have
    // row stride ls = ld + 1, so that a column walk spreads over the banks.
    const bool small = ld <= 32;
    const int ls = ld + 1, msz = ld * ls;  // msz is even (ld is a multiple of 4)
    double *DM = sm;               // ld x ls: D_M, then L^T in its strict upper triangle, then L^-1 D_A
    double *DA = DM + msz;         // ld x ls
    double *Li = DA + msz;         // ld x ls: L^-1
    double *ext = Li + msz;        // small: P3, gag, partial tiles, lambda, FG
    double *P3 = small ? ext : w.P3;                           // ld x 3 ld
    double *gagl = ext + 3 * ld * ld;                          // ld x 2 ld when small
    double *red = small ? ext + 5 * ld * ld : ext;             // kRedSmall (small only)
    double *lam = red + kRedSmall;                             // dn (small only)
    double *fg = lam + ((dn + 1) & ~1);  // dn x 2 ld when fg_in_lds (small only; 16-byte aligned)
    const double *gag = small ? gagl : w.GAGM;
    __shared__ int perm[kMaxWidth];
    __shared__ double ldg[kMaxWidth];  // diagonal of L
    uint64_t tk[8];  // solver statistics: phase clocks (thread 0)
    tk[0] = stat_clock();
    if (small) {
        for (int i = tid; i < dn; i += nthr) lam[i] = w.lam[i];
        if (fg_in_lds) block_copy(fg, w.FG, dn * 2 * ld);
        block_copy(gagl, w.GAGM, 2 * ld * ld);
    }
    if (tid < ld) perm[tid] = tid;
    __syncthreads();
    const int l2 = 2 * ld;
    auto fgv = [&](int i, int a) -> double { return fg_in_lds ? fg[i * l2 + a] : w.FG[(int64_t)i * l2 + a]; };
    tk[1] = stat_clock();
    // P3 = G^T [F | G | Lambda G]   (G = FG(:, ld:2ld), F = FG(:, 0:ld)); for
    // wide blocks k_pencil_p3 has formed it over many workgroups
    if (small)
        block_xty([&](int i, int a) -> double { return a < ld ? fgv(i, ld + a) : 0.0; },
                  [&](int i, int b) -> double {
                      if (b < l2) return fgv(i, b);
                      return b < 3 * ld ? lam[i] * fgv(i, b - ld) : 0.0;
                  },
                  dn, ld, 3 * ld, P3, 3 * ld, red, kRedSmall);
    for (int e = tid; e < ld * ld; e += nthr) {
        const int a = e / ld, b = e - a * ld;
        const double gm_ab = gag[a * l2 + ld + b], gm_ba = gag[b * l2 + ld + a];
        const double ga_ab = gag[a * l2 + b], ga_ba = gag[b * l2 + a];
        const double gg = 0.5 * (P3[a * 3 * ld + ld + b] + P3[b * 3 * ld + ld + a]);
        const double gf = P3[a * 3 * ld + b], fgt = P3[b * 3 * ld + a];
        const double glg = 0.5 * (P3[a * 3 * ld + 2 * ld + b] + P3[b * 3 * ld + 2 * ld + a]);
        DM[a * ls + b] = 0.5 * (gm_ab + gm_ba) - gg;
        DA[a * ls + b] = 0.5 * (ga_ab + ga_ba) - gf - fgt + glg;
    }
    double scale = 0.0;
    for (int a = lane; a < ld; a += kWave) scale = fmax(scale, gag[a * l2 + ld + a]);
    scale = wave_allmax(scale);
    for (int e = tid; e < msz; e += nthr) Li[e] = 0.0;
    __syncthreads();
    tk[2] = stat_clock();
    // pivoted Cholesky of D_M, the same symmetric permutation applied to D_A.
    // Step p writes column p of L, transposed, into row p of D_M right of the
    // diagonal (no thread reads that row during the step) and L_pp into ldg.
    // The symmetric interchange of a later step then swaps these stored
    // columns exactly as it swaps rows of L.
    int r = 0;
    for (int p = 0; p < ld; ++p) {
        int best = p;  // largest remaining diagonal entry, lowest index on ties
        double bv = DM[p * ls + p];
        for (int a = p + 1 + lane; a < ld; a += kWave) {
            const double v = DM[a * ls + a];
            best = v > bv ? a : best;
            bv = v > bv ? v : bv;
        }
        wave_argmax(bv, best);
        if (!(bv > rank_tol * scale)) break;  // the same decision in every thread
        __syncthreads();  // every thread has read the diagonal before the update below rewrites it
        if (best != p) {
            for (int j = tid; j < ld; j += nthr) {
                if (j == p || j == best) continue;
                double t = DM[p * ls + j];
                DM[p * ls + j] = DM[best * ls + j];
                DM[best * ls + j] = t;
                t = DM[j * ls + p];
                DM[j * ls + p] = DM[j * ls + best];
                DM[j * ls + best] = t;
                t = DA[p * ls + j];
                DA[p * ls + j] = DA[best * ls + j];
                DA[best * ls + j] = t;
                t = DA[j * ls + p];
                DA[j * ls + p] = DA[j * ls + best];
                DA[j * ls + best] = t;
            }
            if (tid == 0) {
                double t = DM[p * ls + p];
                DM[p * ls + p] = DM[best * ls + best];
                DM[best * ls + best] = t;
                t = DA[p * ls + p];
                DA[p * ls + p] = DA[best * ls + best];
                DA[best * ls + best] = t;
                const int ti = perm[p];
                perm[p] = perm[best];
                perm[best] = ti;
            }
            __syncthreads();
        }
        const double dpp = DM[p * ls + p], lpp = sqrt(dpp), ipp = 1.0 / lpp;
        // trailing update with the scaled column computed on the fly; column p itself is not written
        for (int i = p + 1 + ty; i < ld; i += nty) {
            const double li = DM[i * ls + p] * ipp;
            for (int j = p + 1 + tx; j <= i; j += 16) {
                const double t = li * (DM[j * ls + p] * ipp);
                DM[i * ls + j] -= t;
                DM[j * ls + i] = DM[i * ls + j];
            }
            if (tx == 0) DM[p * ls + i] = li;
        }
        if (tid == 0) ldg[p] = lpp;
        r = p + 1;
        __syncthreads();
    }
    tk[3] = stat_clock();
    auto lval = [&](int i, int k) -> double { return i == k ? ldg[k] : DM[k * ls + i]; };  // L_ik, i >= k
    tri_inverse(lval, Li, ls, r);
    for (int e = tid; e < ld * ld; e += nthr) {
        const int a = e / ld, b = e - a * ld;
        w.L1[e] = (a < r && b <= a) ? lval(a, b) : 0.0;
    }
    __syncthreads();  // L is read: D_M's buffer takes L^-1 D_A
    double *Yb = DM;
    for (int e = tid; e < r * r; e += nthr) {  // Yb = L^-1 D_A
        const int a = e / r, b = e - a * r;
        double v = 0.0;
        for (int k = 0; k <= a; ++k) v += Li[a * ls + k] * DA[k * ls + b];
        Yb[a * ls + b] = v;
    }
    __syncthreads();
    for (int e = tid; e < ld * ld; e += nthr) {
        const int a = e / ld, b = e - a * ld;
        double v = 0.0;
        if (a < r && b < r) {  // D~ = Yb L^-T, symmetrised
            double s1 = 0.0, s2 = 0.0;
            for (int k = 0; k <= b; ++k) s1 += Yb[a * ls + k] * Li[b * ls + k];
            for (int k = 0; k <= a; ++k) s2 += Yb[b * ls + k] * Li[a * ls + k];
            v = 0.5 * (s1 + s2);
        }
        w.Dt[e] = v;
        w.Li[e] = Li[a * ls + b];
    }
    if (tid < ld) w.perm[tid] = perm[tid];
    if (tid == 0) w.status[ST_RANK] = r;
    tk[4] = stat_clock();
    // C~ = (F - Lambda G)(:, perm_r) L^-T on the matrix cores (for wide blocks
    // k_pencil_ct forms it over many workgroups after this kernel)
    if (small)
    block_tiles(
        [&](int k, int i) -> double {
            if (i >= dn || k >= r) return 0.0;
            const int pk = perm[k];
            return fgv(i, pk) - lam[i] * fgv(i, ld + pk);
        },
        [&](int k, int a) -> double { return a < r ? Li[a * ls + k] : 0.0; }, r, dn, ld,
        [&](int i, int a, double v) { w.Ct[(int64_t)i * ld + a] = v; }, red, kRedSmall);
    if (tid == 0 && w.diag) {
        tk[5] = stat_clock();
        for (int j = 0; j < 5; ++j) atomicAdd(&w.diag[330 + j], (int)(tk[j + 1] - tk[j]));
    }
}

// --------------------------------------------------- eigenvalues (a10)
// One workgroup per wanted eigenvalue k (0-based: the (k+1)-th smallest).
// nu(s) = #{lambda_i < s} + #neg(S(s)) counts the eigenvalues of H below s
// (Sylvester); S(s) is formed on the FP64 matrix cores and factored by
// Bunch-Kaufman.  After the first correction the corrected vector V e_k,
// expressed in the basis of H, is a close approximation of the wanted
// eigenvector: one Rayleigh-quotient step from it and one more count around
// the result usually isolate the eigenvalue and deliver its vector.
// Otherwise the eigenvalue is bracketed (Gershgorin and the interlacing bound
// mu_k <= lambda_k fill in the missing ends), isolated by bisection (or
// narrowed to a cluster of relative width kRqiTol that holds it), and
// Rayleigh-quotient iteration with the exact Schur-complement solve
// (H - s)^-1 runs inside the bracket: every factorisation is also a count and
// narrows the bracket.  An iterate is accepted once its Rayleigh quotient rho
// lies in the bracket with ||H x - rho x|| <= kRqiTol |rho| and more than
// that residual away from both ends, which pins it to the bracketed
// eigenvalue (or cluster).
__device__ __forceinline__ void arrow_bisect_body(SmallWork w, const double *__restrict__ theta_prev, int ct_in_lds,
                                                  int k, int nk) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn;
    const int r = w.status[ST_RANK];
    const int ldp = (ld + 15) & ~15;
    const int ls = ld + 1;
    const bool dt_in_lds = ld <= 32;  // wider D~ is read from global memory (L2)
    const int dts = dt_in_lds ? ldp : ld;
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave, nw = nthr / kWave;
    double *S = sm;                                    // ld x ls
    double *ctl = S + ld * ls;                         // dn x ldp, zero beyond column r
    double *wdn = ctl + (ct_in_lds ? dn * ldp : 0);    // dn weights 1 / (lambda_i - sigma)
    double *vec = wdn + dn;                            // dn + ldp: current vector
    double *hx = vec + dn + ldp;                       // dn + ldp: H x
    double *fz = hx + dn + ldp;                        // ldp
    double *lam = fz + ldp;                            // dn
    double *dtl = lam + dn;                            // ldp x ldp when dt_in_lds
    double *Lm = dtl + (dt_in_lds ? ldp * ldp : 0);    // ld x ls: multipliers of the factorisation
    double *red = Lm + ld * ls;                        // 4 x 256 partial tiles + 64 cross-wavefront sums
    double *vec0 = red + 1024 + 64;                    // dn + ldp: the starting vector
    const double *dt = dt_in_lds ? dtl : w.Dt;
    __shared__ int ipiv[kMaxWidth];
    __shared__ unsigned long long tim[8];  // solver statistics: phase clocks
    if (tid < 8) tim[tid] = 0;
    const uint64_t t_begin = stat_clock();
    if (ct_in_lds) {  // rows of ld doubles (ld a multiple of 4) as double2 pairs
        const int hp = ldp / 2, hl = ld / 2;
        for (int e = tid; e < dn * hp; e += nthr) {
            const int i = e / hp, a2 = e - i * hp;
            double2 v = make_double2(0.0, 0.0);
            if (a2 < hl) v = reinterpret_cast<const double2 *>(w.Ct + (int64_t)i * ld)[a2];
            if (2 * a2 >= r) v.x = 0.0;
            if (2 * a2 + 1 >= r) v.y = 0.0;
            reinterpret_cast<double2 *>(ctl + i * ldp)[a2] = v;
        }
    }
    for (int i = tid; i < dn; i += nthr) lam[i] = w.lam[i];
    if (dt_in_lds)
        for (int e = tid; e < ldp * ldp; e += nthr) {
            const int a = e / ldp, b = e - a * ldp;
            dtl[e] = (a < r && b < r) ? w.Dt[a * ld + b] : 0.0;
        }
    __syncthreads();
    if (tid == 0) tim[0] += stat_clock() - t_begin;
    auto ct = [&](int i, int a) -> double {
        if (ct_in_lds) return ctl[i * ldp + a];
        return a < ld ? w.Ct[(int64_t)i * ld + a] : 0.0;  // columns r..ld-1 hold zeros
    };
    auto bsum = [&](double v) -> double {
        v = wave_allsum(v);
        if (nw == 1) return v;
        __syncthreads();
        if (lane == 0) red[wv] = v;
        __syncthreads();
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += red[i];
        return s;
    };

    int ncount = 0;
    // ---- factorisation of H - sigma through S(sigma); returns nu(sigma)
    auto factor = [&](double sigma) -> int {
        ++ncount;
        const uint64_t f0 = stat_clock();
        int lo_i = 0, hi_i = dn;  // #{lambda_i < sigma}, lam ascending
        while (lo_i < hi_i) {
            const int mid = (lo_i + hi_i) / 2;
            if (lam[mid] < sigma) lo_i = mid + 1; else hi_i = mid;
        }
        const int nlow = lo_i;
        __syncthreads();
        for (int i = tid; i < dn; i += nthr) {
            double den = lam[i] - sigma;
            if (den == 0.0) den = 1e-300;
            wdn[i] = 1.0 / den;
        }
        __syncthreads();
        const int nt = (r + 15) >> 4, ntiles = nt * (nt + 1) / 2;
        // row chunks per tile; their partial tiles (ntiles * ksplit * 256) fit in red
        const int kcap = 4 / ntiles > 1 ? 4 / ntiles : 1;
        const int ksplit = ntiles >= nw ? 1 : (nw / ntiles < kcap ? nw / ntiles : kcap);
        const int chunk = ((dn + ksplit - 1) / ksplit + 3) & ~3;
        for (int item = wv; item < ntiles * ksplit; item += nw) {  // lower tiles of C~^T W C~
            const int t = item % ntiles, kc = item / ntiles;
            int ta = 0;
            while ((ta + 1) * (ta + 2) / 2 <= t) ++ta;
            const int tb = t - ta * (ta + 1) / 2;
            const int k0 = kc * chunk, k1 = dn < k0 + chunk ? dn : k0 + chunk;
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
            if (k1 > k0) {
                if (ct_in_lds)
                    acc = mfma_tn16([&](int i, int c) { return wdn[k0 + i] * ct(k0 + i, 16 * ta + c); },
                                    [&](int i, int c) { return ct(k0 + i, 16 * tb + c); }, k1 - k0);
                else  // C~ from global memory (L2): eight steps of operands in flight
                    acc = mfma_tn16_deep([&](int i, int c) { return wdn[k0 + i] * ct(k0 + i, 16 * ta + c); },
                                         [&](int i, int c) { return ct(k0 + i, 16 * tb + c); }, k1 - k0);
            }
            if (ksplit == 1) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = 16 * ta + (lane >> 4) + 4 * u, j = 16 * tb + (lane & 15);
                    if (i < r && j < r && (ta != tb || i >= j)) {
                        const double v = dt[i * dts + j] - (i == j ? sigma : 0.0) - acc[u];
                        S[i * ls + j] = v;
                        S[j * ls + i] = v;
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) red[(item * 4 + u) * kWave + lane] = acc[u];
            }
        }
        if (ksplit > 1) {
            __syncthreads();
            for (int e = tid; e < ntiles * 256; e += nthr) {
                const int t = e >> 8, u = (e >> 6) & 3, ln = e & 63;
                double v = 0.0;
                for (int kc = 0; kc < ksplit; ++kc) v += red[((kc * ntiles + t) * 4 + u) * kWave + ln];
                int ta = 0;
                while ((ta + 1) * (ta + 2) / 2 <= t) ++ta;
                const int tb = t - ta * (ta + 1) / 2;
                const int i = 16 * ta + (ln >> 4) + 4 * u, j = 16 * tb + (ln & 15);
                if (i < r && j < r && (ta != tb || i >= j)) {
                    v = dt[i * dts + j] - (i == j ? sigma : 0.0) - v;
                    S[i * ls + j] = v;
                    S[j * ls + i] = v;
                }
            }
        }
        __syncthreads();
        const uint64_t f1 = stat_clock();
        const int neg = bk_factor(S, Lm, r, ls, ipiv);
        if (tid == 0) {
            tim[1] += f1 - f0;
            tim[2] += stat_clock() - f1;
        }
        return nlow + neg;
    };

    // ---- out[a] = sum over the dn coarse rows of C~_{i a} u_i (matrix cores)
    auto ct_t_times = [&](const double *u, double *out) {
        const int nt = (r + 15) >> 4;
        const int ksplit = nt >= nw ? 1 : nw / nt;
        const int chunk = ((dn + ksplit - 1) / ksplit + 3) & ~3;
        for (int item = wv; item < nt * ksplit; item += nw) {
            const int ta = item % nt, kc = item / nt;
            const int k0 = kc * chunk, k1 = dn < k0 + chunk ? dn : k0 + chunk;
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
            if (k1 > k0)
                acc = mfma_tn16([&](int i, int c) { return ct(k0 + i, 16 * ta + c); },
                                [&](int i, int c) { return c == 0 ? u[k0 + i] : 0.0; }, k1 - k0);
            if ((lane & 15) == 0) {
#pragma unroll
                for (int uu = 0; uu < 4; ++uu) red[(item * 4 + uu) * 4 + (lane >> 4)] = acc[uu];
            }
        }
        __syncthreads();
        for (int a = tid; a < r; a += nthr) {  // a = 16 ta + 4 uu + (lane >> 4)
            const int ta = a >> 4, rem = a & 15, uu = rem >> 2, q4 = rem & 3;
            double v = 0.0;
            for (int kc = 0; kc < ksplit; ++kc) v += red[(((kc * nt + ta) * 4 + uu) * 4) + q4];
            out[a] = v;
        }
        __syncthreads();
    };

    // ---- x <- (H - sigma)^-1 x for the factorisation in S, ipiv, wdn
    auto solve = [&](double *x) {
        const uint64_t s0 = stat_clock();
        for (int i = tid; i < dn; i += nthr) x[i] *= wdn[i];  // t = (Lambda - sigma)^-1 x_y
        __syncthreads();
        ct_t_times(x, fz);
        for (int a = tid; a < r; a += nthr) fz[a] = x[dn + a] - fz[a];
        __syncthreads();
        bk_solve(S, Lm, r, ls, ipiv, fz);
        for (int i = tid; i < dn; i += nthr) {
            double s2 = 0.0;
            for (int a = 0; a < r; ++a) s2 += ct(i, a) * fz[a];
            x[i] -= s2 * wdn[i];
        }
        for (int a = tid; a < r; a += nthr) x[dn + a] = fz[a];
        __syncthreads();
        if (tid == 0) tim[3] += stat_clock() - s0;
    };
    auto normalise = [&](double *x) {
        double s2 = 0.0;
        for (int i = tid; i < dn + r; i += nthr) s2 += x[i] * x[i];
        s2 = bsum(s2);
        const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
        __syncthreads();
        for (int i = tid; i < dn + r; i += nthr) x[i] *= inv;
        __syncthreads();
    };
    // rho = x^T H x (x normalised) and ||H x - rho x||
    auto rayleigh = [&](const double *x, double &rho, double &res) {
        const uint64_t q0 = stat_clock();
        ct_t_times(x, fz);  // C~^T y
        for (int i = tid; i < dn; i += nthr) {
            double s2 = lam[i] * x[i];
            for (int a = 0; a < r; ++a) s2 += ct(i, a) * x[dn + a];
            hx[i] = s2;
        }
        for (int a = tid; a < r; a += nthr) {
            double s2 = fz[a];
            for (int b = 0; b < r; ++b) s2 += dt[a * dts + b] * x[dn + b];
            hx[dn + a] = s2;
        }
        __syncthreads();
        double q = 0.0;
        for (int i = tid; i < dn + r; i += nthr) q += x[i] * hx[i];
        rho = bsum(q);
        double e2 = 0.0;
        for (int i = tid; i < dn + r; i += nthr) {
            const double d = hx[i] - rho * x[i];
            e2 += d * d;
        }
        res = sqrt(bsum(e2));
        if (tid == 0) tim[4] += stat_clock() - q0;
    };

    // ---- warm start.  The corrected vector V e_k has the coordinates
    // y = G e_k, z = L^T Pi^T e_k in the basis of H (its part outside span Z is
    // (V - Z G) e_k = W L^T Pi^T e_k with W the M-orthonormalised columns).
    // Up to three Rayleigh-quotient steps from it; every factorisation on the
    // way is a count that tightens the bracket.
    double lo = 0.0, hi = 0.0;
    int nulo = 0, nuhi = 1 << 30;
    bool have_lo = false, have_hi = false;
    bool done = false;
    // the previous Ritz values are meaningful only after a first Rayleigh-Ritz
    // step (or from the coarsest eigenvalues in the nested start)
    const bool warm = w.status[ST_WARM] != 0;
    const double tp = warm ? theta_prev[k] : 0.0;
    const double cap = lam[k] * (1.0 + 1e-14) + 1e-300;  // interlacing: mu_k <= lambda_k
    double rho = 0.0, res = 0.0;
    // bracket updates are value selects (a branch on which end to write would
    // turn the ends into addressable stack slots)
    auto note = [&](double sg, int c) __attribute__((always_inline)) {
        const bool is_lo = c <= k;
        const bool up_lo = is_lo && (!have_lo || sg > lo);
        const bool up_hi = !is_lo && (!have_hi || sg < hi);
        lo = up_lo ? sg : lo;
        nulo = up_lo ? c : nulo;
        have_lo = have_lo || up_lo;
        hi = up_hi ? sg : hi;
        nuhi = up_hi ? c : nuhi;
        have_hi = have_hi || up_hi;
    };
    auto force = [&](double sg, int c) __attribute__((always_inline)) {  // replace the end on c's side
        const bool is_lo = c <= k;
        lo = is_lo ? sg : lo;
        nulo = is_lo ? c : nulo;
        have_lo = have_lo || is_lo;
        hi = is_lo ? hi : sg;
        nuhi = is_lo ? nuhi : c;
        have_hi = have_hi || !is_lo;
    };
    __shared__ int s_pos;
    if (warm) {
        if (tid == 0) {
            s_pos = -1;
            for (int a = 0; a < r; ++a)
                if (w.perm[a] == k) s_pos = a;
        }
        __syncthreads();
        const int pos = s_pos;
        for (int i = tid; i < dn + r; i += nthr) {
            double v;
            if (i < dn)
                v = w.FG[(int64_t)i * 2 * ld + ld + k];
            else if (pos >= 0)
                v = (i - dn) <= pos ? w.L1[pos * ld + (i - dn)] : 0.0;
            else
                v = start_entry(k, i);
            vec[i] = v;
        }
        __syncthreads();
        normalise(vec);
        for (int i = tid; i < dn + r; i += nthr) vec0[i] = vec[i];
        // up to two attempts: the second from the starting vector with the
        // eigenvector found by the first projected out, when the first settled
        // on a neighbouring eigenvalue (a close pair whose starting vector
        // mixed both)
        for (int attempt = 0; attempt < 2 && !done; ++attempt) {
            rayleigh(vec, rho, res);
            for (int it = 0; it < 3; ++it) {
                if (res <= kRqiTol * fabs(rho) || !(rho > 0.0 && rho < cap)) break;
                note(rho, factor(rho));
                solve(vec);
                normalise(vec);
                rayleigh(vec, rho, res);
            }
            if (!(res <= kRqiTol * fabs(rho) && rho > 0.0 && rho < cap)) break;
            // ends more than the residual away from rho, counted if not yet known
            const double span = fmax(4.0 * res, 1e-12 * fabs(rho));
            // (an end that would not isolate eigenvalue k only tightens the bracket)
            const double l0 = rho - span, h0 = fmin(rho + span, cap);
            int cl = -1, ch = -1;  // counts at l0 and h0, where taken
            if (!(have_lo && nulo == k && rho - lo > res)) {
                cl = factor(l0);
                if (cl == k) force(l0, cl); else note(l0, cl);
            }
            if (!(have_hi && nuhi == k + 1 && hi - rho > res)) {
                ch = factor(h0);
                if (ch == k + 1) force(h0, ch); else note(h0, ch);
            }
            done = have_lo && have_hi && nulo == k && nuhi == k + 1 && rho > lo && rho < hi && rho - lo > res &&
                   hi - rho > res;
            // a cluster: eigenvalue k lies in [l0, h0) together with others that
            // no count can separate from it at this residual.  Then rho is within
            // span of eigenvalue k, and x lies in the cluster's invariant subspace
            // up to the residual over the gap to the rest of the spectrum; the
            // cluster members start from different corrected vectors, and the
            // Ritz polish that follows resolves the subspace they span
            if (!done && (cl >= 0) != (ch >= 0)) {  // count the end not taken in this attempt
                if (cl < 0) {
                    cl = factor(l0);
                    note(l0, cl);
                } else {
                    ch = factor(h0);
                    note(h0, ch);
                }
            }
            done = done || (cl >= 0 && ch >= 0 && cl <= k && k < ch);
            if (done || attempt == 1 || !((have_hi && hi < rho) || (have_lo && lo > rho))) break;
            double d = 0.0;
            for (int i = tid; i < dn + r; i += nthr) d += vec[i] * vec0[i];
            d = bsum(d);
            __syncthreads();
            double s2 = 0.0;
            for (int i = tid; i < dn + r; i += nthr) {
                const double v = vec0[i] - d * vec[i];
                vec[i] = v;
                s2 += v * v;
            }
            s2 = bsum(s2);
            if (!(s2 > 1e-12)) {  // nothing left: a pseudo-random start instead
                __syncthreads();
                for (int i = tid; i < dn + r; i += nthr) vec[i] = start_entry(k, i);
            }
            __syncthreads();
            normalise(vec);
        }
    } else {
        for (int i = tid; i < dn + r; i += nthr) vec[i] = start_entry(k, i);
        __syncthreads();
    }
    const int c_warm = ncount;  // solver statistics: counts per phase
    // ---- the previous Ritz value theta_prev[k] is close to eigenvalue k once
    // the iteration has settled: counts at widening windows around it give a
    // narrow bracket in a few factorisations (any count is a valid bracket
    // end, so a poor guess only costs the counts)
    if (!done && warm && tp > 0.0 && tp < cap) {
        double d = 1e-7 * tp;
        for (int t = 0; t < 3; ++t, d *= 100.0) {
            const double a = tp - d, b = fmin(tp + d, cap);
            if (!(have_lo && lo >= a) && !(have_hi && hi <= a)) note(a, factor(a));
            if (!(have_hi && hi <= b) && !(have_lo && lo >= b)) note(b, factor(b));
            if (have_lo && have_hi && hi - lo <= 2.0 * d) break;
        }
    }
    const int c_win = ncount;
    if (!(have_lo && have_hi)) {
        // Gershgorin lower bound of H; the upper end is the interlacing bound
        double g = 1e300;
        for (int i = tid; i < dn; i += nthr) {
            double s2 = 0.0;
            for (int a = 0; a < r; ++a) s2 += fabs(ct(i, a));
            g = fmin(g, lam[i] - s2);
        }
        for (int a = tid; a < r; a += nthr) {
            double s2 = 0.0;
            for (int b = 0; b < r; ++b)
                if (b != a) s2 += fabs(dt[a * dts + b]);
            for (int i = 0; i < dn; ++i) s2 += fabs(ct(i, a));
            g = fmin(g, dt[a * dts + a] - s2);
        }
        for (int off = kWave / 2; off > 0; off >>= 1) g = fmin(g, __shfl_xor(g, off, kWave));
        __syncthreads();
        if (lane == 0) red[wv] = g;
        __syncthreads();
        double glo = red[0];
        for (int i = 1; i < nw; ++i) glo = fmin(glo, red[i]);
        __syncthreads();
        hi = have_hi ? hi : cap;                // not counted yet: at least k + 1 by interlacing
        nuhi = have_hi ? nuhi : (1 << 30);
        // no eigenvalue below a Gershgorin bound, nor below 0: H is the
        // projection of the positive definite A in an M-orthonormal basis
        const double g0 = glo - fabs(glo) * 1e-14 - 1e-300;
        lo = have_lo ? lo : (g0 > 0.0 ? g0 : 0.0);
        nulo = have_lo ? nulo : 0;
    }
    // ---- isolate by bisection, or narrow to a cluster no wider than the
    // acceptance residual: then every eigenvalue in the bracket is within
    // kRqiTol |rho| of eigenvalue k, and the iteration below settles on one
    // of them with its vector in the cluster's invariant subspace
    for (int it = 0; it < 200 && !done; ++it) {
        if (nulo == k && nuhi == k + 1) break;
        if (hi - lo <= kRqiTol * fmax(fabs(lo), fabs(hi))) break;
        const double mid = 0.5 * (lo + hi);
        force(mid, factor(mid));
    }
    const int c_bis = ncount;
    // ---- Rayleigh-quotient iteration inside the bracket, from the corrected
    // vector when there is one (the warm attempts may have left a neighbour's
    // eigenvector in vec)
    if (!done && warm) {
        for (int i = tid; i < dn + r; i += nthr) vec[i] = vec0[i];
        __syncthreads();
    }
    double sigma = (rho > lo && rho < hi) ? rho : ((tp > lo && tp < hi) ? tp : 0.5 * (lo + hi));
    for (int it = 0; it < 12 && !done; ++it) {
        const int c = factor(sigma);
        const bool up = c >= k + 1;
        hi = up ? fmin(hi, sigma) : hi;
        lo = up ? lo : fmax(lo, sigma);
        solve(vec);
        normalise(vec);
        rayleigh(vec, rho, res);
        const bool inside = rho > lo && rho < hi;
        if (inside && res <= kRqiTol * fabs(rho) && rho - lo > res && hi - rho > res) break;
        sigma = inside ? rho : 0.5 * (lo + hi);
        if (hi - lo <= 1e-13 * fmax(fabs(lo), fabs(hi))) break;
    }
    if (tid == 0 && w.diag && (k == 0 || k == nk - 1)) {
        tim[5] = stat_clock() - t_begin;
        int *slot = w.diag + (k == 0 ? 5 * kMaxWidth - 8 : 3 * kMaxWidth);
        for (int j = 0; j < 6; ++j) atomicAdd(&slot[j], (int)tim[j]);
    }
    if (tid == 0 && w.diag) {
        atomicAdd(&w.diag[340], c_warm);
        atomicAdd(&w.diag[341], c_win - c_warm);
        atomicAdd(&w.diag[342], c_bis - c_win);
        atomicAdd(&w.diag[343], ncount - c_bis);
        atomicAdd(&w.diag[344], c_bis > c_win ? 1 : 0);
        atomicMax(&w.diag[345], ncount);
        atomicAdd(&w.diag[k], ncount);
        atomicAdd(&w.diag[kMaxWidth + k], done ? 1 : 0);
        atomicAdd(&w.diag[2 * kMaxWidth + k], 1);
    }
    for (int i = tid; i < dn + ld; i += nthr) w.X[(int64_t)i * ld + k] = i < dn + r ? vec[i] : 0.0;
}

// ------------------------------------------- Rayleigh-Ritz polish (a10)
// One workgroup: X <- orthonormal basis of span X (two Cholesky-QR passes),
// T = X^T H X, T = Q diag(theta) Q^T by cyclic Jacobi, Xr = X Q sorted.
// When they fit, X, H X and C~ are copied to LDS (use_lds); otherwise the same
// code works on the global buffers.
constexpr int kRed = kRedSmall;

__device__ __forceinline__ void arrow_rr_body(SmallWork w, int qe, int use_lds, double *theta_out, int final_level) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn, r = w.status[ST_RANK];
    const int nh = dn + r, m = qe;
    // row stride of the ld x ld matrices below, odd so that a column walk
    // spreads over the LDS banks
    const int ldp = ld + 1, msz = ld * ldp;  // msz is even (ld is a multiple of 4)
    const bool small = ld <= 32;          // wider: D~ and lambda from global memory, no split-K partials
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave, nw = nthr / kWave;
    uint64_t tk[9];  // solver statistics: phase clocks (thread 0)
    tk[0] = stat_clock();
    double *T = sm;                 // ld x ldp
    double *Q = T + msz;            // ld x ldp
    double *G = Q + msz;            // ld x ldp
    double *red = G + msz;          // kRed (small) or 64
    double *lamv = red + (small ? kRed : 64);              // dn when small
    double *dtl = lamv + (small ? ((dn + 1) & ~1) : 0);    // ld x ldp when small (keeps the copies below 16-byte aligned)
    if (small) {
        for (int i = tid; i < dn; i += nthr) lamv[i] = w.lam[i];
        for (int e = tid; e < msz; e += nthr) {
            const int a = e / ldp, b = e - a * ldp;
            dtl[e] = (a < r && b < r) ? w.Dt[a * ld + b] : 0.0;
        }
    }
    const double *lamp = small ? lamv : w.lam;
    const double *dtv = small ? dtl : w.Dt;
    const int dts = small ? ldp : ld;  // row stride of D~: the LDS copy's or the global array's
    const int rcap = small ? kRed : 64;
    double *Xp = w.X, *HXp = w.HX;
    const double *Ctp = w.Ct;
    if (use_lds) {
        double *Xl = dtl + (small ? msz : 0);
        double *HXl = Xl + (dn + ld) * ld;
        double *Ctl = HXl + (dn + ld) * ld;
        block_copy(Xl, w.X, nh * ld);
        block_copy(Ctl, w.Ct, dn * ld);
        Xp = Xl;
        HXp = HXl;
        Ctp = Ctl;
    }
    __syncthreads();
    auto xa = [&](int i, int c) -> double { return c < m ? Xp[(int64_t)i * ld + c] : 0.0; };
    auto hxa = [&](int i, int c) -> double { return c < m ? HXp[(int64_t)i * ld + c] : 0.0; };
    auto cta = [&](int i, int a) -> double { return a < r ? Ctp[(int64_t)i * ld + a] : 0.0; };
    __shared__ double cs[kMaxWidth];
    __shared__ double sn[kMaxWidth];
    __shared__ int pairs[kMaxWidth];
    __shared__ double s_off;
    __shared__ int order[kMaxWidth];
    __shared__ double s_theta[kMaxWidth];
    tk[1] = stat_clock();
    // ---- Cholesky-QR on X (nh x m); a second pass unless every pivot of the
    // first was within 10% of 1 (then X was already orthonormal to a few
    // units of rounding and one pass leaves it so).  A column whose pivot
    // falls below 1e-10 (columns have unit norm) repeats a direction of the
    // columns before it, as two vectors of a multiple eigenvalue can: it is
    // replaced by the coordinates of the corrected vector V e_p (then, if
    // that fails too, by a pseudo-random vector) and the pass restarts.
    __shared__ int tries[kMaxWidth];
    __shared__ double ldq[kMaxWidth];  // diagonal of the Cholesky factor
    const int tx = tid & 15, ty = tid >> 4, nty = nthr >> 4;
    if (tid < m) tries[tid] = 0;
    int passes = 0;
    for (int it = 0; it < 2 + 2 * m && passes < 2; ++it) {
        bool near_identity = true;  // the same in every thread
        int bad = -1;
        block_xty(xa, xa, nh, m, m, G, ldp, red, rcap);
        // G = L L^T, one barrier per step: the update of the lower triangle
        // right of column p scales column p on the fly, and the scaled column
        // goes to row p right of the diagonal (no thread reads it during the
        // step), L_pp to ldq
        for (int p = 0; p < m; ++p) {
            const double d = G[p * ldp + p];
            near_identity = near_identity && d > 0.9 && d < 1.1;
            if (!(d > 1e-10)) {
                bad = p;
                break;
            }
            const double lpp = sqrt(d);
            for (int i = p + 1 + ty; i < m; i += nty) {
                const double li = G[i * ldp + p] / lpp;
                for (int j = p + 1 + tx; j <= i; j += 16) G[i * ldp + j] -= li * (G[j * ldp + p] / lpp);
                if (tx == 0) G[p * ldp + i] = li;
            }
            if (tid == 0) ldq[p] = lpp;
            __syncthreads();
        }
        if (bad >= 0) {
            const int tr = tries[bad];
            __syncthreads();
            if (tr >= 2) {  // no independent direction found
                if (tid == 0) w.status[ST_BREAKDOWN] = 1;
                break;
            }
            __shared__ int s_pos;
            if (tid == 0) {
                s_pos = -1;
                for (int a2 = 0; a2 < r; ++a2)
                    if (w.perm[a2] == bad) s_pos = a2;
                tries[bad] = tr + 1;
            }
            __syncthreads();
            const int pos = tr == 0 ? s_pos : -1;
            double s2 = 0.0;
            for (int i = tid; i < nh; i += nthr) {
                double v;
                if (i < dn && tr == 0)
                    v = w.FG[(int64_t)i * 2 * ld + ld + bad];
                else if (i >= dn && pos >= 0)
                    v = (i - dn) <= pos ? w.L1[pos * ld + (i - dn)] : 0.0;
                else
                    v = start_entry(bad + 7 * (tr + 1), i);
                Xp[(int64_t)i * ld + bad] = v;
                s2 += v * v;
            }
            for (int o = kWave / 2; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, kWave);
            if (lane == 0) red[wv] = s2;
            __syncthreads();
            double nrm = 0.0;
            for (int i = 0; i < nw; ++i) nrm += red[i];
            const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
            for (int i = tid; i < nh; i += nthr) Xp[(int64_t)i * ld + bad] *= inv;
            __syncthreads();
            continue;
        }
        tri_inverse([&](int i, int k) -> double { return i == k ? ldq[k] : G[k * ldp + i]; }, Q, ldp, m);  // L^-1 into Q
        // X L^-T on the matrix cores into the other buffer, then swap
        block_tiles([&](int a, int i) -> double { return (i < nh && a < m) ? Xp[(int64_t)i * ld + a] : 0.0; },
                    [&](int a, int c) -> double { return c < m ? Q[c * ldp + a] : 0.0; }, m, nh, m,
                    [&](int i, int c, double v) { HXp[(int64_t)i * ld + c] = v; }, red, rcap);
        double *t = Xp;
        Xp = HXp;
        HXp = t;
        ++passes;
        if (near_identity) break;
    }
    tk[2] = stat_clock();
    // ---- HX (nh x m): rows i < dn: lam_i x_i + C~_i z ; rows dn+a: C~^T y + D~ z
    block_tiles([&](int a, int i) -> double { return (i < dn && a < r) ? Ctp[(int64_t)i * ld + a] : 0.0; },
                [&](int a, int c) -> double { return c < m ? Xp[(int64_t)(dn + a) * ld + c] : 0.0; }, r, dn, m,
                [&](int i, int c, double v) { HXp[(int64_t)i * ld + c] = lamp[i] * Xp[(int64_t)i * ld + c] + v; },
                red, rcap);
    block_xty(cta, xa, dn, r, m, HXp + (int64_t)dn * ld, ld, red, rcap);
    block_tiles([&](int b, int a) -> double { return (a < r && b < r) ? dtv[b * dts + a] : 0.0; },  // D~ symmetric
                [&](int b, int c) -> double { return c < m ? Xp[(int64_t)(dn + b) * ld + c] : 0.0; }, r, r, m,
                [&](int a, int c, double v) { HXp[(int64_t)(dn + a) * ld + c] += v; }, red, rcap);
    tk[3] = stat_clock();
    // ---- T = X^T HX, symmetrised
    block_xty(xa, hxa, nh, m, m, Q, ldp, red, rcap);
    for (int e = tid; e < m * m; e += nthr) {
        const int a = e / m, b = e - a * m;
        T[a * ldp + b] = 0.5 * (Q[a * ldp + b] + Q[b * ldp + a]);
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += nthr) {
        const int a = e / m, b = e - a * m;
        Q[a * ldp + b] = a == b ? 1.0 : 0.0;
    }
    __syncthreads();
    tk[4] = stat_clock();
    // ---- cyclic Jacobi with the round-robin ordering (m even)
    for (int sweep = 0; sweep < 30; ++sweep) {
        for (int round = 0; round < m - 1; ++round) {
            if (tid < m / 2) {
                const int k2 = tid;
                auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (m - 1)) + 1; };
                int p = player(k2), q = player(m - 1 - k2);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                pairs[2 * k2] = p;
                pairs[2 * k2 + 1] = q;
                const double apq = T[p * ldp + q], app = T[p * ldp + p], aqq = T[q * ldp + q];
                double c = 1.0, sv = 0.0;
                if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    sv = t * c;
                }
                cs[k2] = c;
                sn[k2] = sv;
            }
            __syncthreads();
            // J^T T J and Q J in one phase: the pairs split the indices, so the
            // 2 x 2 block of T at rows (p, q) of pair k2 and columns (p3, q3) of
            // pair k3 is one thread's: rotated by k2 over its rows, then by k3
            // over its columns; a row of Q's column pair k3 likewise
            const int h = m / 2;
            for (int e = tid; e < h * h + h * m; e += nthr) {
                if (e < h * h) {
                    const int k2 = e / h, k3 = e - k2 * h;
                    const int p = pairs[2 * k2], q = pairs[2 * k2 + 1], p3 = pairs[2 * k3], q3 = pairs[2 * k3 + 1];
                    const double c = cs[k2], sv = sn[k2], c3 = cs[k3], s3 = sn[k3];
                    const double tpp = T[p * ldp + p3], tqp = T[q * ldp + p3];
                    const double tpq = T[p * ldp + q3], tqq = T[q * ldp + q3];
                    const double rpp = c * tpp - sv * tqp, rqp = sv * tpp + c * tqp;  // rows of column p3
                    const double rpq = c * tpq - sv * tqq, rqq = sv * tpq + c * tqq;  // rows of column q3
                    T[p * ldp + p3] = c3 * rpp - s3 * rpq;
                    T[p * ldp + q3] = s3 * rpp + c3 * rpq;
                    T[q * ldp + p3] = c3 * rqp - s3 * rqq;
                    T[q * ldp + q3] = s3 * rqp + c3 * rqq;
                } else {
                    const int e2 = e - h * h, k3 = e2 / m, i = e2 - k3 * m;
                    const int p = pairs[2 * k3], q = pairs[2 * k3 + 1];
                    const double c = cs[k3], sv = sn[k3];
                    const double qp = Q[i * ldp + p], qq = Q[i * ldp + q];
                    Q[i * ldp + p] = c * qp - sv * qq;
                    Q[i * ldp + q] = sv * qp + c * qq;
                }
            }
            __syncthreads();
        }
        double off = 0.0;  // largest scaled off-diagonal entry
        for (int e = tid; e < m * m; e += nthr) {
            const int a = e / m, b = e - a * m;
            if (a != b)
                off = fmax(off, fabs(T[a * ldp + b]) / sqrt(fabs(T[a * ldp + a] * T[b * ldp + b]) + 1e-300));
        }
        for (int o = kWave / 2; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o, kWave));
        if (lane == 0) red[wv] = off;
        __syncthreads();
        if (tid == 0) {
            double mx = red[0];
            for (int i = 1; i < nw; ++i) mx = fmax(mx, red[i]);
            s_off = mx;
            if (w.diag) atomicAdd(&w.diag[4 * kMaxWidth], 1);
        }
        __syncthreads();
        if (s_off < 1e-15) break;
    }
    tk[5] = stat_clock();
    // ---- sort Ritz values ascending and write Xr = X Q(:, order), theta
    if (tid == 0) {
        for (int a = 0; a < m; ++a) {
            order[a] = a;
            s_theta[a] = T[a * ldp + a];
        }
        for (int a = 1; a < m; ++a) {  // insertion sort, stable
            const int oa = order[a];
            int b = a - 1;
            while (b >= 0 && s_theta[order[b]] > s_theta[oa]) {
                order[b + 1] = order[b];
                --b;
            }
            order[b + 1] = oa;
        }
    }
    __syncthreads();
    for (int c = tid; c < m; c += nthr) {
        const double th = s_theta[order[c]];
        w.theta[c] = th;
        theta_out[c] = th;
    }
    tk[6] = stat_clock();
    // ---- Ritz vectors of H: Xr = X Q(:, order)   (H X is no longer needed)
    double *Xr = use_lds ? HXp : w.Xr;
    block_tiles([&](int a, int i) -> double { return (i < nh && a < m) ? Xp[(int64_t)i * ld + a] : 0.0; },
                [&](int a, int c) -> double { return c < m ? Q[a * ldp + order[c]] : 0.0; }, m, nh, ld,
                [&](int i, int c, double v) { Xr[(int64_t)i * ld + c] = v; }, red, rcap);
    tk[7] = stat_clock();
    // ---- recombination coefficients X_v = Pi_r L^-T z, X_c = y - G X_v
    double *Li = G;   // r x r, stride ldp (only the lower triangle is read)
    double *Xv = T;   // ld x ld, stride ldp
    for (int e = tid; e < r * r; e += nthr) {  // L^-1 from the pencil kernel
        const int a = e / r, b = e - a * r;
        Li[a * ldp + b] = w.Li[a * ld + b];
    }
    for (int e = tid; e < msz; e += nthr) Xv[e] = 0.0;
    __syncthreads();
    for (int e = tid; e < r * ld; e += nthr) {
        const int a = e / ld, c = e - a * ld;
        double v = 0.0;
        for (int b = a; b < r; ++b) v += Li[b * ldp + a] * Xr[(int64_t)(dn + b) * ld + c];
        Xv[w.perm[a] * ldp + c] = v;
    }
    __syncthreads();
    for (int e = tid; e < ld * ld; e += nthr) {
        const int a = e / ld, c = e - a * ld;
        w.Xv[e] = Xv[a * ldp + c];
    }
    block_tiles([&](int a, int i) -> double { return (i < dn && a < ld) ? w.FG[(int64_t)i * 2 * ld + ld + a] : 0.0; },
                [&](int a, int c) -> double { return c < ld ? Xv[a * ldp + c] : 0.0; }, ld, dn, ld,
                [&](int i, int c, double v) { w.Xc[(int64_t)i * ld + c] = Xr[(int64_t)i * ld + c] - v; }, red, rcap);
    if (tid == 0) {
        w.status[ST_WARM] = 1;
        if (final_level) w.status[ST_STEPS] += 1;
        if (w.diag) {
            tk[8] = stat_clock();
            for (int j = 0; j < 8; ++j) atomicAdd(&w.diag[321 + j], (int)(tk[j + 1] - tk[j]));
        }
    }
}

// ------------------------------------------- wide pencil products (a9)
// For wide blocks (ld > 32) the two plain products of the pencil step run
// over many workgroups, before and after the single-workgroup part:
//   P3 = G^T [F | G | Lambda G]          (ld x 3 ld, sum over the d_n coarse rows)
//   C~ = (F - Lambda G)(:, perm_r) L^-T   (d_n x ld, sum over the r kept columns)
// P3: one 16 x 16 tile per workgroup, whose four wavefronts take a quarter of
// the rows each (partial tiles summed in a fixed order); C~: one tile per
// wavefront.  The same device functions serve the single and the batched
// launches, so a joint step computes what a separate one does.
__device__ __forceinline__ int p3_tiles(int ld) { return ((ld + 15) / 16) * ((3 * ld + 15) / 16); }
__device__ __forceinline__ int ct_tiles(int ld, int dn) { return ((dn + 15) / 16) * ((ld + 15) / 16); }

__device__ void pencil_p3_tile(const SmallWork &w, int tile) {
    __shared__ double part[4 * 4 * kWave];
    const int ld = w.ld, dn = w.dn, l2 = 2 * ld, l3 = 3 * ld, tj = (l3 + 15) / 16;
    const int ta = tile / tj, tb = tile - ta * tj;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int chunk = ((dn + nw - 1) / nw + 3) & ~3;
    const int k0 = wv * chunk, k1 = dn < k0 + chunk ? dn : k0 + chunk;
    const double *FG = w.FG;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    if (k1 > k0)
        acc = mfma_tn16_deep(
            [&](int i, int c) -> double {
                const int a = 16 * ta + c;
                return a < ld ? FG[(int64_t)(k0 + i) * l2 + ld + a] : 0.0;
            },
            [&](int i, int c) -> double {
                const int b = 16 * tb + c;
                const int64_t row = (int64_t)(k0 + i) * l2;
                if (b < l2) return FG[row + b];
                return b < l3 ? w.lam[k0 + i] * FG[row + b - ld] : 0.0;
            },
            k1 - k0);
#pragma unroll
    for (int u = 0; u < 4; ++u) part[(wv * 4 + u) * kWave + lane] = acc[u];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double v = 0.0;
            for (int x = 0; x < nw; ++x) v += part[(x * 4 + u) * kWave + lane];
            const int i = 16 * ta + (lane >> 4) + 4 * u, j = 16 * tb + (lane & 15);
            if (i < ld && j < l3) w.P3[i * l3 + j] = v;
        }
    }
}

__device__ void pencil_ct_tile(const SmallWork &w, int tile) {  // one wavefront
    const int ld = w.ld, dn = w.dn, l2 = 2 * ld, r = w.status[ST_RANK], tj = (ld + 15) / 16;
    const int ti = tile / tj, tb = tile - ti * tj, lane = threadIdx.x & (kWave - 1);
    const double *FG = w.FG;
    const dbl4 acc = mfma_tn16(
        [&](int k, int c) -> double {
            const int i = 16 * ti + c;
            if (i >= dn || k >= r) return 0.0;
            const int pk = w.perm[k];
            return FG[(int64_t)i * l2 + pk] - w.lam[i] * FG[(int64_t)i * l2 + ld + pk];
        },
        [&](int k, int c) -> double {
            const int a = 16 * tb + c;
            return (a < r && k < r) ? w.Li[a * ld + k] : 0.0;
        },
        r);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = 16 * ti + (lane >> 4) + 4 * u, a = 16 * tb + (lane & 15);
        if (i < dn && a < ld) w.Ct[(int64_t)i * ld + a] = acc[u];
    }
}

__global__ __launch_bounds__(256) void k_pencil_p3(SmallWork w) {
    if (w.status[ST_CONVERGED]) return;
    pencil_p3_tile(w, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_pencil_ct(SmallWork w) {
    const int t = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (w.status[ST_CONVERGED] || t >= ct_tiles(w.ld, w.dn)) return;  // wave-uniform
    pencil_ct_tile(w, t);
}

// ------------------------------------------------------------ kernels
__global__ __launch_bounds__(1024) void k_pencil(SmallWork w, double rank_tol, int fg_in_lds) {
    pencil_body(w, rank_tol, fg_in_lds);
}

__global__ __launch_bounds__(kBisectWide) void k_arrow_bisect(SmallWork w, const double *__restrict__ theta_prev,
                                                      int ct_in_lds) {
    arrow_bisect_body(w, theta_prev, ct_in_lds, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(1024) void k_arrow_rr(SmallWork w, int qe, int use_lds, double *theta_out, int final_level) {
    arrow_rr_body(w, qe, use_lds, theta_out, final_level);
}

// The same three steps for several requests in one launch each: workgroup b of
// the pencil and Rayleigh-Ritz kernels serves member b of the table, and the
// eigenvalue workgroups of member m are blocks first[m] .. first[m + 1] - 1.
// Every member's descriptor (pointers into its own workspace, widths, LDS
// layout flags) lives in device memory; the launch takes the largest LDS size
// any member needs.
__global__ __launch_bounds__(1024) void k_pencil_batch(SmallTable t, double rank_tol) {
    const SmallItem *it = t.item[blockIdx.x];
    pencil_body(it->w, rank_tol, it->fg_in_lds);
}

// the wide pencil products of the members with ld > 32: P3 tiles (workgroups)
// of member m are p3first[m] .. p3first[m + 1] - 1, C~ tiles (wavefronts)
// ctfirst[m] .. ctfirst[m + 1] - 1
__global__ __launch_bounds__(256) void k_pencil_p3_batch(SmallTable t) {
    int m = 0;
    while (m + 1 < t.n && t.p3first[m + 1] <= (int)blockIdx.x) ++m;
    const SmallItem *it = t.item[m];
    if (it->w.status[ST_CONVERGED]) return;
    pencil_p3_tile(it->w, (int)blockIdx.x - t.p3first[m]);
}

__global__ __launch_bounds__(256) void k_pencil_ct_batch(SmallTable t) {
    const int g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (g >= t.ctfirst[t.n]) return;
    int m = 0;
    while (m + 1 < t.n && t.ctfirst[m + 1] <= g) ++m;
    const SmallItem *it = t.item[m];
    if (it->w.status[ST_CONVERGED]) return;
    pencil_ct_tile(it->w, g - t.ctfirst[m]);
}

__global__ __launch_bounds__(kBisectWide) void k_arrow_bisect_batch(SmallTable t) {
    int m = 0;
    while (m + 1 < t.n && t.first[m + 1] <= (int)blockIdx.x) ++m;
    const SmallItem *it = t.item[m];
    arrow_bisect_body(it->w, it->theta, it->ct_in_lds, (int)blockIdx.x - t.first[m], it->qe);
}

__global__ __launch_bounds__(1024) void k_arrow_rr_batch(SmallTable t) {
    const SmallItem *it = t.item[blockIdx.x];
    arrow_rr_body(it->w, it->qe, it->use_lds, it->theta, t.final_level);
}

// ------------------------------------------------------------ launchers
// Dynamic LDS a small kernel may take for its optional copies: the 160 KB of a
// gfx950 workgroup less 4 KB for the kernels' static shared arrays (at most
// 2.9 KB).
constexpr size_t kLdsBudget = 160 * 1024 - 4096;

void small_layout(const SmallWork &w, int qe, double *theta, SmallItem *it, SmallLds *lds) {
    const size_t ld = w.ld, dn = w.dn, msz = ld * (ld + 1);  // the ld x (ld + 1) matrices of the pencil and Rayleigh-Ritz kernels
    const size_t pbase = ld <= 32 ? 3 * msz + 5 * ld * ld + kRedSmall + dn + 1 : 3 * msz + 64;
    const int fg_in_lds = ld <= 32 && (pbase + dn * 2 * ld) * sizeof(double) <= kLdsBudget ? 1 : 0;
    // the rank r <= ld is only known on the device: size for r = ld
    const size_t ldp = (ld + 15) & ~(size_t)15, dtl = ld <= 32 ? ldp * ldp : 0;  // the kernel's layout
    const size_t bbase = 2 * ld * (ld + 1) + dn + 2 * (dn + ldp) + ldp + dn + dtl + 1024 + 64 + dn + ldp;
    const int ct_in_lds = (bbase + dn * ldp) * sizeof(double) <= kLdsBudget ? 1 : 0;
    const size_t rsmall = ld <= 32;
    const size_t rbase = 3 * msz + (rsmall ? kRed + dn + 1 + msz : 64);
    const size_t full = rbase + 2 * (dn + ld) * ld + dn * ld;
    const int use_lds = full * sizeof(double) <= kLdsBudget ? 1 : 0;
    it->w = w;
    it->theta = theta;
    it->qe = qe;
    it->fg_in_lds = fg_in_lds;
    it->ct_in_lds = ct_in_lds;
    it->use_lds = use_lds;
    lds->pencil = (pbase + (fg_in_lds ? dn * 2 * ld : 0)) * sizeof(double);
    lds->bisect = (bbase + (ct_in_lds ? dn * ldp : 0)) * sizeof(double);
    lds->rr = (use_lds ? full : rbase) * sizeof(double);
}

int pencil_p3_blocks(int ld) { return ld > 32 ? ((ld + 15) / 16) * ((3 * ld + 15) / 16) : 0; }
int pencil_ct_waves(int ld, int dn) { return ld > 32 ? ((dn + 15) / 16) * ((ld + 15) / 16) : 0; }

void launch_pencil(hipStream_t s, const SmallWork &w, double rank_tol) {
    SmallItem it;
    SmallLds lds;
    small_layout(w, 1, nullptr, &it, &lds);
    const int np3 = pencil_p3_blocks(w.ld), nct = pencil_ct_waves(w.ld, w.dn);
    if (np3) hipLaunchKernelGGL(k_pencil_p3, dim3(np3), dim3(kB), 0, s, w);
    hipLaunchKernelGGL(k_pencil, dim3(1), dim3(small_threads(w.ld)), lds.pencil, s, w, rank_tol, it.fg_in_lds);
    if (nct) hipLaunchKernelGGL(k_pencil_ct, dim3((nct + kB / kWave - 1) / (kB / kWave)), dim3(kB), 0, s, w);
}

void launch_arrow_eig(hipStream_t s, const SmallWork &w, int qe, double *theta, int final_level) {
    SmallItem it;
    SmallLds lds;
    small_layout(w, qe, theta, &it, &lds);
    hipLaunchKernelGGL(k_arrow_bisect, dim3(qe), dim3(bisect_threads(w.ld)), lds.bisect, s, w, theta, it.ct_in_lds);
    hipLaunchKernelGGL(k_arrow_rr, dim3(1), dim3(small_threads(w.ld)), lds.rr, s, w, qe, it.use_lds, theta, final_level);
}

void launch_small_batch(hipStream_t s, const SmallTable &t, const SmallLds &lds, double rank_tol, bool wide) {
    const int nt = wide ? kBWide : kB;
    if (t.n <= 0) return;
    if (t.p3first[t.n] > 0) hipLaunchKernelGGL(k_pencil_p3_batch, dim3(t.p3first[t.n]), dim3(kB), 0, s, t);
    hipLaunchKernelGGL(k_pencil_batch, dim3(t.n), dim3(nt), lds.pencil, s, t, rank_tol);
    if (t.ctfirst[t.n] > 0)
        hipLaunchKernelGGL(k_pencil_ct_batch, dim3((t.ctfirst[t.n] + kB / kWave - 1) / (kB / kWave)), dim3(kB), 0, s,
                           t);
    hipLaunchKernelGGL(k_arrow_bisect_batch, dim3(t.first[t.n]), dim3(wide ? kBisectWide : kB), lds.bisect, s, t);
    hipLaunchKernelGGL(k_arrow_rr_batch, dim3(t.n), dim3(nt), lds.rr, s, t);
}

}  // namespace amgeig
