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

// ---------------------------------------------------------------------
// Bunch-Kaufman symmetric indefinite LDL^T of S (r x r, LDS, row stride ls),
// in place: multipliers below the diagonal, D on the (block) diagonal.
// ipiv[p] = kp >= 0: 1x1 pivot, rows p and kp interchanged;
// ipiv[p] = ipiv[p+1] = -(kp+1): 2x2 pivot, rows p+1 and kp interchanged.
// Returns the number of negative eigenvalues of S (Sylvester's law).
__device__ int bk_factor(double *S, int r, int ls, int *ipiv, double *logabs) {
    __shared__ int s_kp, s_size, s_neg;
    __shared__ double s_log;
    const double alpha = 0.6403882032022076;  // (1 + sqrt(17)) / 8
    if (threadIdx.x == 0) {
        s_neg = 0;
        s_log = 0.0;
    }
    __syncthreads();
    int p = 0;
    while (p < r) {
        if (threadIdx.x < kWave) {
            const int lane = threadIdx.x;
            double best = -1.0;
            int bi = r;
            for (int i = p + 1 + lane; i < r; i += kWave) {
                const double v = fabs(S[i * ls + p]);
                if (v > best) {
                    best = v;
                    bi = i;
                }
            }
            for (int off = kWave / 2; off > 0; off >>= 1) {
                const double ov = __shfl_xor(best, off, kWave);
                const int oi = __shfl_xor(bi, off, kWave);
                if (ov > best || (ov == best && oi < bi)) {
                    best = ov;
                    bi = oi;
                }
            }
            const double colmax = best > 0.0 ? best : 0.0;
            const int imax = bi;
            const double absakk = fabs(S[p * ls + p]);
            int kp = p, size = 1;
            if (colmax > 0.0 && absakk < alpha * colmax) {
                double rb = 0.0;
                for (int j = p + lane; j < r; j += kWave)
                    if (j != imax) rb = fmax(rb, fabs(S[imax * ls + j]));
                for (int off = kWave / 2; off > 0; off >>= 1) rb = fmax(rb, __shfl_xor(rb, off, kWave));
                const double rowmax = rb;
                if (absakk * rowmax >= alpha * colmax * colmax) {
                    kp = p;
                } else if (fabs(S[imax * ls + imax]) >= alpha * rowmax) {
                    kp = imax;
                } else {
                    kp = imax;
                    size = 2;
                }
            }
            if (lane == 0) {
                s_kp = kp;
                s_size = size;
            }
        }
        __syncthreads();
        const int kp = s_kp, size = s_size;
        const int tgt = size == 1 ? p : p + 1;
        if (kp != tgt) {
            for (int j = threadIdx.x; j < r; j += blockDim.x) {
                const double t = S[tgt * ls + j];
                S[tgt * ls + j] = S[kp * ls + j];
                S[kp * ls + j] = t;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < r; i += blockDim.x) {
                const double t = S[i * ls + tgt];
                S[i * ls + tgt] = S[i * ls + kp];
                S[i * ls + kp] = t;
            }
            __syncthreads();
        }
        if (size == 1) {
            const double d = S[p * ls + p];
            const double dinv = d != 0.0 ? 1.0 / d : 0.0;
            if (threadIdx.x == 0) {
                ipiv[p] = kp;
                if (d < 0.0) s_neg += 1;
                s_log += log(fabs(d) + 1e-300);
            }
            const int m = r - p - 1;
            for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
                const int i = p + 1 + e / m, j = p + 1 + e % m;
                S[i * ls + j] -= S[i * ls + p] * S[j * ls + p] * dinv;
            }
            __syncthreads();
            for (int i = p + 1 + threadIdx.x; i < r; i += blockDim.x) S[i * ls + p] *= dinv;
            __syncthreads();
            p += 1;
        } else {
            const double a = S[p * ls + p], b = S[(p + 1) * ls + p], c = S[(p + 1) * ls + p + 1];
            const double det = a * c - b * b;
            if (threadIdx.x == 0) {
                ipiv[p] = ipiv[p + 1] = -(kp + 1);
                s_neg += det < 0.0 ? 1 : (a + c < 0.0 ? 2 : 0);
                s_log += log(fabs(det) + 1e-300);
            }
            const double id = 1.0 / det;
            const int m = r - p - 2;
            for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
                const int i = p + 2 + e / m, j = p + 2 + e % m;
                const double c1 = S[i * ls + p], c2 = S[i * ls + p + 1];
                const double l1 = (c1 * c - c2 * b) * id, l2 = (c2 * a - c1 * b) * id;
                S[i * ls + j] -= l1 * S[j * ls + p] + l2 * S[j * ls + p + 1];
            }
            __syncthreads();
            for (int i = p + 2 + threadIdx.x; i < r; i += blockDim.x) {
                const double c1 = S[i * ls + p], c2 = S[i * ls + p + 1];
                S[i * ls + p] = (c1 * c - c2 * b) * id;
                S[i * ls + p + 1] = (c2 * a - c1 * b) * id;
            }
            __syncthreads();
            p += 2;
        }
    }
    __syncthreads();
    if (logabs) *logabs = s_log;
    return s_neg;
}

// Solve S z = f with the factors of bk_factor (f overwritten by z, LDS).
__device__ void bk_solve(const double *S, int r, int ls, const int *ipiv, double *f) {
    if (threadIdx.x == 0) {
        for (int p = 0; p < r;) {
            if (ipiv[p] >= 0) {
                const int kp = ipiv[p];
                const double t = f[p];
                f[p] = f[kp];
                f[kp] = t;
                p += 1;
            } else {
                const int kp = -ipiv[p] - 1;
                const double t = f[p + 1];
                f[p + 1] = f[kp];
                f[kp] = t;
                p += 2;
            }
        }
    }
    __syncthreads();
    for (int p = 0; p < r;) {  // L y = f
        if (ipiv[p] >= 0) {
            const double fp = f[p];
            for (int i = p + 1 + threadIdx.x; i < r; i += blockDim.x) f[i] -= S[i * ls + p] * fp;
            __syncthreads();
            p += 1;
        } else {
            const double f0 = f[p], f1 = f[p + 1];
            for (int i = p + 2 + threadIdx.x; i < r; i += blockDim.x) f[i] -= S[i * ls + p] * f0 + S[i * ls + p + 1] * f1;
            __syncthreads();
            p += 2;
        }
    }
    if (threadIdx.x == 0) {  // D solve; singular pivots are replaced by a tiny value
        for (int p = 0; p < r;) {
            if (ipiv[p] >= 0) {
                double d = S[p * ls + p];
                if (d == 0.0) d = 1e-300;
                f[p] /= d;
                p += 1;
            } else {
                const double a = S[p * ls + p], b = S[(p + 1) * ls + p], c = S[(p + 1) * ls + p + 1];
                const double det = a * c - b * b;
                const double y0 = f[p], y1 = f[p + 1];
                f[p] = (c * y0 - b * y1) / det;
                f[p + 1] = (a * y1 - b * y0) / det;
                p += 2;
            }
        }
    }
    __syncthreads();
    // L^T w = y, blocks from the last one backwards: once w of a block is known,
    // remove its contribution from the rows above.
    int starts[kMaxWidth];
    int nblk = 0;
    for (int p = 0; p < r;) {
        starts[nblk++] = p;
        p += ipiv[p] >= 0 ? 1 : 2;
    }
    for (int bidx = nblk - 1; bidx >= 0; --bidx) {
        const int p = starts[bidx];
        if (ipiv[p] >= 0) {
            const double wp = f[p];
            for (int i = threadIdx.x; i < p; i += blockDim.x) f[i] -= S[p * ls + i] * wp;
        } else {
            const double w0 = f[p], w1 = f[p + 1];
            for (int i = threadIdx.x; i < p; i += blockDim.x) f[i] -= S[p * ls + i] * w0 + S[(p + 1) * ls + i] * w1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int bidx = nblk - 1; bidx >= 0; --bidx) {
            const int p = starts[bidx];
            if (ipiv[p] >= 0) {
                const int kp = ipiv[p];
                const double t = f[p];
                f[p] = f[kp];
                f[kp] = t;
            } else {
                const int kp = -ipiv[p] - 1;
                const double t = f[p + 1];
                f[p + 1] = f[kp];
                f[kp] = t;
            }
        }
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

// ------------------------------------------------------------- products
// P3 = G^T [F | G | Lambda G] (ld x 3ld) over the dn coarse rows.
__global__ __launch_bounds__(256) void k_small_products(int dn, int ld, const double *__restrict__ lam,
                                                        const double *__restrict__ FG, double *__restrict__ P3,
                                                        const int *status) {
    __shared__ double xs[64][17];
    __shared__ double ys[64][17];
    if (status[ST_CONVERGED]) return;
    const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
    const int ta = threadIdx.x / 16, tb = threadIdx.x % 16;
    double acc = 0.0;
    for (int i0 = 0; i0 < dn; i0 += 64) {
        for (int e = threadIdx.x; e < 64 * 16; e += blockDim.x) {
            const int ii = e / 16, cc = e % 16, i = i0 + ii;
            double xv = 0.0, yv = 0.0;
            if (i < dn) {
                const int a = a0 + cc, b = b0 + cc;
                if (a < ld) xv = FG[(int64_t)i * 2 * ld + ld + a];
                if (b < ld)
                    yv = FG[(int64_t)i * 2 * ld + b];
                else if (b < 2 * ld)
                    yv = FG[(int64_t)i * 2 * ld + ld + (b - ld)];
                else if (b < 3 * ld)
                    yv = lam[i] * FG[(int64_t)i * 2 * ld + ld + (b - 2 * ld)];
            }
            xs[ii][cc] = xv;
            ys[ii][cc] = yv;
        }
        __syncthreads();
        const int lim = dn - i0 < 64 ? dn - i0 : 64;
        for (int ii = 0; ii < lim; ++ii) acc += xs[ii][ta] * ys[ii][tb];
        __syncthreads();
    }
    const int a = a0 + ta, b = b0 + tb;
    if (a < ld && b < 3 * ld) P3[a * 3 * ld + b] = acc;
}

// ------------------------------------------------------------- pencil (a9)
__global__ __launch_bounds__(256) void k_pencil(SmallWork w, double rank_tol) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn;
    double *DM = sm;             // ld x ld, becomes L
    double *DA = sm + ld * ld;   // ld x ld
    double *Y = DA + ld * ld;    // ld x ld scratch
    __shared__ int perm[kMaxWidth];
    __shared__ int s_r, s_piv;
    __shared__ double s_scale;
    for (int e = threadIdx.x; e < ld * ld; e += blockDim.x) {
        const int a = e / ld, b = e % ld;
        const double gm_ab = w.GAGM[a * 2 * ld + ld + b], gm_ba = w.GAGM[b * 2 * ld + ld + a];
        const double ga_ab = w.GAGM[a * 2 * ld + b], ga_ba = w.GAGM[b * 2 * ld + a];
        const double gg = 0.5 * (w.P3[a * 3 * ld + ld + b] + w.P3[b * 3 * ld + ld + a]);
        const double gf = w.P3[a * 3 * ld + b], fg = w.P3[b * 3 * ld + a];
        const double glg = 0.5 * (w.P3[a * 3 * ld + 2 * ld + b] + w.P3[b * 3 * ld + 2 * ld + a]);
        DM[e] = 0.5 * (gm_ab + gm_ba) - gg;
        DA[e] = 0.5 * (ga_ab + ga_ba) - gf - fg + glg;
    }
    if (threadIdx.x < ld) perm[threadIdx.x] = threadIdx.x;
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int a = 0; a < ld; ++a) mx = fmax(mx, w.GAGM[a * 2 * ld + ld + a]);
        s_scale = mx;
        s_r = 0;
    }
    __syncthreads();
    // pivoted Cholesky of D_M, same symmetric permutation applied to D_A
    for (int p = 0; p < ld; ++p) {
        if (threadIdx.x == 0) {
            int best = p;
            for (int a = p + 1; a < ld; ++a)
                if (DM[a * ld + a] > DM[best * ld + best]) best = a;
            s_piv = DM[best * ld + best] > rank_tol * s_scale ? best : -1;
        }
        __syncthreads();
        const int piv = s_piv;
        if (piv < 0) break;
        if (piv != p) {
            for (int j = threadIdx.x; j < ld; j += blockDim.x) {
                double t = DM[p * ld + j];
                DM[p * ld + j] = DM[piv * ld + j];
                DM[piv * ld + j] = t;
                t = DA[p * ld + j];
                DA[p * ld + j] = DA[piv * ld + j];
                DA[piv * ld + j] = t;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < ld; i += blockDim.x) {
                double t = DM[i * ld + p];
                DM[i * ld + p] = DM[i * ld + piv];
                DM[i * ld + piv] = t;
                t = DA[i * ld + p];
                DA[i * ld + p] = DA[i * ld + piv];
                DA[i * ld + piv] = t;
            }
            if (threadIdx.x == 0) {
                const int t = perm[p];
                perm[p] = perm[piv];
                perm[piv] = t;
            }
            __syncthreads();
        }
        const double lpp = sqrt(DM[p * ld + p]);
        __syncthreads();
        for (int i = p + 1 + threadIdx.x; i < ld; i += blockDim.x) DM[i * ld + p] /= lpp;
        if (threadIdx.x == 0) DM[p * ld + p] = lpp;
        __syncthreads();
        const int m = ld - p - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int i = p + 1 + e / m, j = p + 1 + e % m;
            DM[i * ld + j] -= DM[i * ld + p] * DM[j * ld + p];
        }
        if (threadIdx.x == 0) s_r = p + 1;
        __syncthreads();
    }
    const int r = s_r;
    // Y = L^-1 D_A(perm_r, perm_r)  (column c by thread c)
    if ((int)threadIdx.x < r) {
        const int c = threadIdx.x;
        for (int i = 0; i < r; ++i) {
            double s = DA[i * ld + c];
            for (int k = 0; k < i; ++k) s -= DM[i * ld + k] * Y[k * ld + c];
            Y[i * ld + c] = s / DM[i * ld + i];
        }
    }
    __syncthreads();
    // D~ = L^-1 Y^T (column c by thread c), symmetrised afterwards
    if ((int)threadIdx.x < r) {
        const int c = threadIdx.x;
        for (int i = 0; i < r; ++i) {
            double s = Y[c * ld + i];
            for (int k = 0; k < i; ++k) s -= DM[i * ld + k] * DA[k * ld + c];
            DA[i * ld + c] = s / DM[i * ld + i];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ld * ld; e += blockDim.x) {
        const int a = e / ld, b = e % ld;
        w.Dt[e] = (a < r && b < r) ? 0.5 * (DA[a * ld + b] + DA[b * ld + a]) : 0.0;
        w.L1[e] = (a < r && b <= a) ? DM[a * ld + b] : 0.0;
    }
    if ((int)threadIdx.x < ld) w.perm[threadIdx.x] = perm[threadIdx.x];
    if (threadIdx.x == 0) w.status[ST_RANK] = r;
    // C~ rows: c = F_i - lambda_i G_i (permuted), then L^-1 c
    double t[kMaxWidth];
    for (int i = threadIdx.x; i < dn; i += blockDim.x) {
        const double li = w.lam[i];
        const double *row = w.FG + (int64_t)i * 2 * ld;
        for (int a = 0; a < r; ++a) {
            const int pa = perm[a];
            double s = row[pa] - li * row[ld + pa];
            for (int k = 0; k < a; ++k) s -= DM[a * ld + k] * t[k];
            t[a] = s / DM[a * ld + a];
        }
        for (int a = 0; a < ld; ++a) w.Ct[(int64_t)i * ld + a] = a < r ? t[a] : 0.0;
    }
}

// --------------------------------------------------- eigenvalues (a10)
// One workgroup per wanted eigenvalue k (0-based: the (k+1)-th smallest).
// nu(s) = #{lambda_i < s} + #neg(S(s)) counts the eigenvalues of H below s
// (Sylvester), and sign det(H - s) = (-1)^nu(s) with
// log|det(H - s)| = sum_i log|lambda_i - s| + log|det S(s)|.
// The eigenvalue is bracketed (warm bracket around the previous step's Ritz
// value when it validates, else Gershgorin and the interlacing bound
// mu_{k+1} <= lambda_{k+1}), isolated by bisection, then refined by
// regula falsi with the Illinois modification on det(H - s).  Two steps of
// inverse iteration at the final shift give column k of X.
struct CountOut {
    int nu;
    double logdet;
};

__global__ __launch_bounds__(256) void k_arrow_bisect(SmallWork w, const double *__restrict__ theta_prev,
                                                      int ct_in_lds) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn, k = blockIdx.x;
    const int r = w.status[ST_RANK];
    const int ls = r + 1;
    double *S = sm;                      // r x ls
    double *cch = S + r * ls;            // C~ in LDS (dn x r) or a 64-row chunk
    const int chunk_rows = ct_in_lds ? dn : 64;
    double *wdn = cch + chunk_rows * r;  // dn weights 1 / (lambda_i - sigma)
    double *vec = wdn + dn;              // dn + r
    double *fz = vec + dn + r;           // r
    __shared__ int ipiv[kMaxWidth];
    __shared__ double red[kB];
    __shared__ double s_log;
    const int npairs = r * (r + 1) / 2;
    const int nthr = blockDim.x;
    if (ct_in_lds) {
        for (int e = threadIdx.x; e < dn * r; e += nthr) cch[e] = w.Ct[(int64_t)(e / r) * ld + e % r];
        __syncthreads();
    }

    auto count = [&](double sigma) -> CountOut {
        // #{lambda_i < sigma} (lam ascending), per thread
        int lo_i = 0, hi_i = dn;
        while (lo_i < hi_i) {
            const int mid = (lo_i + hi_i) / 2;
            if (w.lam[mid] < sigma) lo_i = mid + 1; else hi_i = mid;
        }
        const int nlow = lo_i;
        double lsum = 0.0;
        __syncthreads();
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double den = w.lam[i] - sigma;
            if (den == 0.0) den = 1e-300;
            lsum += log(fabs(den));
            wdn[i] = 1.0 / den;
        }
        __syncthreads();
        double acc[(kMaxWidth * (kMaxWidth + 1) / 2 + 63) / 64];
        const int per = (npairs + nthr - 1) / nthr;
        for (int t = 0; t < per; ++t) acc[t] = 0.0;
        for (int i0 = 0; i0 < dn; i0 += chunk_rows) {
            const int lim = dn - i0 < chunk_rows ? dn - i0 : chunk_rows;
            const double *ct = ct_in_lds ? cch + (int64_t)i0 * r : cch;
            if (!ct_in_lds) {
                __syncthreads();
                for (int e = threadIdx.x; e < lim * r; e += nthr) cch[e] = w.Ct[(int64_t)(i0 + e / r) * ld + e % r];
                __syncthreads();
            }
            for (int t = 0; t < per; ++t) {
                const int pr = threadIdx.x + t * nthr;
                if (pr >= npairs) break;
                int a = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
                while (a * (a + 1) / 2 > pr) --a;
                while ((a + 1) * (a + 2) / 2 <= pr) ++a;
                const int b = pr - a * (a + 1) / 2;
                double sacc = 0.0;
                const double *wi = wdn + i0;
                for (int ii = 0; ii < lim; ++ii) sacc += ct[ii * r + a] * ct[ii * r + b] * wi[ii];
                acc[t] += sacc;
            }
        }
        __syncthreads();
        for (int t = 0; t < per; ++t) {
            const int pr = threadIdx.x + t * nthr;
            if (pr >= npairs) break;
            int a = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
            while (a * (a + 1) / 2 > pr) --a;
            while ((a + 1) * (a + 2) / 2 <= pr) ++a;
            const int b = pr - a * (a + 1) / 2;
            const double v = w.Dt[a * ld + b] - (a == b ? sigma : 0.0) - acc[t];
            S[a * ls + b] = v;
            S[b * ls + a] = v;
        }
        lsum = block_sum(lsum, red);
        const int neg = bk_factor(S, r, ls, ipiv, &s_log);
        CountOut o;
        o.nu = nlow + neg;
        o.logdet = lsum + s_log;
        __syncthreads();
        return o;
    };

    // ---- bracket
    double lo, hi;
    CountOut clo, chi;
    bool have = false;
    const double tp = theta_prev[k];
    if (w.status[ST_WARM] && tp > 0.0) {
        for (double delta = 1e-4; delta < 0.2 && !have; delta *= 100.0) {
            const double l0 = tp * (1.0 - delta), h0 = fmin(tp * (1.0 + delta), w.lam[k] * (1.0 + 1e-14) + 1e-300);
            if (!(l0 < h0)) break;
            CountOut a0 = count(l0);
            if (a0.nu > k) continue;
            CountOut b0 = count(h0);
            if (b0.nu < k + 1) continue;
            lo = l0; hi = h0; clo = a0; chi = b0;
            have = true;
        }
    }
    if (!have) {
        double g = 1e300;
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double s2 = 0.0;
            for (int a = 0; a < r; ++a) s2 += fabs(w.Ct[(int64_t)i * ld + a]);
            g = fmin(g, w.lam[i] - s2);
        }
        for (int a = threadIdx.x; a < r; a += nthr) {
            double s2 = 0.0;
            for (int b = 0; b < r; ++b)
                if (b != a) s2 += fabs(w.Dt[a * ld + b]);
            for (int i = 0; i < dn; ++i) s2 += fabs(w.Ct[(int64_t)i * ld + a]);
            g = fmin(g, w.Dt[a * ld + a] - s2);
        }
        red[threadIdx.x] = g;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mn = red[0];
            for (int t = 1; t < nthr; ++t) mn = fmin(mn, red[t]);
            red[0] = mn;
        }
        __syncthreads();
        lo = red[0];
        __syncthreads();
        hi = w.lam[k];
        hi = hi + fabs(hi) * 1e-14 + 1e-300;
        lo = lo - fabs(lo) * 1e-14 - 1e-300;
        clo = count(lo);
        chi = count(hi);
    }
    // ---- isolate, then regula falsi (Illinois) on det(H - s)
    double flo = clo.logdet, fhi = chi.logdet;  // log-magnitudes; signs from the counts
    int side = 0;
    for (int it = 0; it < 200; ++it) {
        const double width = hi - lo;
        if (width <= 1e-10 * fmax(fabs(lo), fabs(hi))) break;
        double c;
        const bool isolated = (clo.nu == k) && (chi.nu == k + 1);
        if (!isolated) {
            c = 0.5 * (lo + hi);
        } else {
            // f(lo) f(hi) < 0 because nu differs by one: c = hi - (hi - lo) / (1 + |f(lo)| / |f(hi)|)
            const double q = exp(fmin(700.0, flo - fhi));
            c = hi - width / (1.0 + q);
            const double guard = 1e-3 * width;
            if (!(c > lo + guard)) c = lo + guard;
            if (!(c < hi - guard)) c = hi - guard;
        }
        if (c <= lo || c >= hi) break;
        const CountOut cc = count(c);
        if (cc.nu >= k + 1) {
            hi = c; chi = cc; fhi = cc.logdet;
            if (side == 1) flo += -0.69314718055994531;  // Illinois: halve the stale end
            side = 1;
        } else {
            lo = c; clo = cc; flo = cc.logdet;
            if (side == -1) fhi += -0.69314718055994531;
            side = -1;
        }
    }
    const double sigma = 0.5 * (lo + hi);
    (void)count(sigma);  // factorisation at sigma kept in S, ipiv
    const int nh = dn + r;
    for (int i = threadIdx.x; i < nh; i += nthr) vec[i] = start_entry(k, i);
    __syncthreads();
    for (int step = 0; step < 2; ++step) {
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double den = w.lam[i] - sigma;
            if (den == 0.0) den = 1e-300;
            vec[i] = vec[i] / den;
        }
        __syncthreads();
        // f = b_z - C~^T t : thread a (or a slice) per column
        for (int a = threadIdx.x; a < r; a += nthr) {
            double s2 = 0.0;
            if (ct_in_lds)
                for (int i = 0; i < dn; ++i) s2 += cch[(int64_t)i * r + a] * vec[i];
            else
                for (int i = 0; i < dn; ++i) s2 += w.Ct[(int64_t)i * ld + a] * vec[i];
            fz[a] = vec[dn + a] - s2;
        }
        __syncthreads();
        bk_solve(S, r, ls, ipiv, fz);
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double s2 = 0.0;
            if (ct_in_lds)
                for (int a = 0; a < r; ++a) s2 += cch[(int64_t)i * r + a] * fz[a];
            else
                for (int a = 0; a < r; ++a) s2 += w.Ct[(int64_t)i * ld + a] * fz[a];
            double den = w.lam[i] - sigma;
            if (den == 0.0) den = 1e-300;
            vec[i] -= s2 / den;
        }
        for (int a = threadIdx.x; a < r; a += nthr) vec[dn + a] = fz[a];
        __syncthreads();
        double s2 = 0.0;
        for (int i = threadIdx.x; i < nh; i += nthr) s2 += vec[i] * vec[i];
        s2 = block_sum(s2, red);
        const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
        for (int i = threadIdx.x; i < nh; i += nthr) vec[i] *= inv;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < dn + ld; i += nthr) w.X[(int64_t)i * ld + k] = i < nh ? vec[i] : 0.0;
}

// ------------------------------------------- Rayleigh-Ritz polish (a10)
// One workgroup: X <- orthonormal basis of span X (two Cholesky-QR passes),
// T = X^T H X, T = Q diag(theta) Q^T by cyclic Jacobi, Xr = X Q sorted.
// When they fit, X, H X and C~ are copied to LDS (use_lds); otherwise the same
// code works on the global buffers.
__global__ __launch_bounds__(256) void k_arrow_rr(SmallWork w, int qe, int use_lds) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn, r = w.status[ST_RANK];
    const int nh = dn + r, m = qe;
    double *T = sm;          // m x m
    double *Q = T + m * m;   // m x m
    double *xs = Q + m * m;  // 32 x m staging
    double *Xp = w.X, *HXp = w.HX;
    const double *Ctp = w.Ct;
    int xst = ld, cst = ld;
    if (use_lds) {
        double *Xl = xs + 32 * m;
        double *HXl = Xl + nh * m;
        double *Ctl = HXl + nh * m;
        for (int e = threadIdx.x; e < nh * m; e += blockDim.x) Xl[e] = w.X[(int64_t)(e / m) * ld + e % m];
        for (int e = threadIdx.x; e < dn * r; e += blockDim.x) Ctl[e] = w.Ct[(int64_t)(e / r) * ld + e % r];
        Xp = Xl;
        HXp = HXl;
        Ctp = Ctl;
        xst = m;
        cst = r;
        __syncthreads();
    }
    __shared__ double cs[kMaxWidth];
    __shared__ double sn[kMaxWidth];
    __shared__ int pairs[kMaxWidth];
    __shared__ double s_off;
    __shared__ int order[kMaxWidth];
    __shared__ double s_theta[kMaxWidth];
    // ---- two Cholesky-QR passes on X (nh x m)
    for (int pass = 0; pass < 2; ++pass) {
        double acc[(kMaxWidth * kMaxWidth + kB - 1) / kB];
        const int per = (m * m + kB - 1) / kB;
        for (int t = 0; t < per; ++t) acc[t] = 0.0;
        for (int i0 = 0; i0 < nh; i0 += 32) {
            const int lim = nh - i0 < 32 ? nh - i0 : 32;
            __syncthreads();
            for (int e = threadIdx.x; e < lim * m; e += blockDim.x) xs[e] = Xp[(int64_t)(i0 + e / m) * xst + e % m];
            __syncthreads();
            for (int t = 0; t < per; ++t) {
                const int e = threadIdx.x + t * kB;
                if (e >= m * m) break;
                const int a = e / m, b = e % m;
                double s2 = 0.0;
                for (int ii = 0; ii < lim; ++ii) s2 += xs[ii * m + a] * xs[ii * m + b];
                acc[t] += s2;
            }
        }
        __syncthreads();
        for (int t = 0; t < per; ++t) {
            const int e = threadIdx.x + t * kB;
            if (e < m * m) T[e] = acc[t];
        }
        __syncthreads();
        for (int p = 0; p < m; ++p) {  // T = L L^T in place (lower)
            double d = T[p * m + p];
            if (!(d > 0.0)) {
                if (threadIdx.x == 0) w.status[ST_BREAKDOWN] = 1;
                d = 1e-300;
            }
            const double lpp = sqrt(d);
            __syncthreads();
            for (int i = p + 1 + threadIdx.x; i < m; i += blockDim.x) T[i * m + p] /= lpp;
            if (threadIdx.x == 0) T[p * m + p] = lpp;
            __syncthreads();
            const int mm = m - p - 1;
            for (int e = threadIdx.x; e < mm * mm; e += blockDim.x) {
                const int i = p + 1 + e / mm, j = p + 1 + e % mm;
                if (j <= i) T[i * m + j] -= T[i * m + p] * T[j * m + p];
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < nh; i += blockDim.x) {  // x <- x L^-T
            double z[kMaxWidth];
            double *xr = Xp + (int64_t)i * xst;
            for (int c = 0; c < m; ++c) {
                double s2 = xr[c];
                for (int a2 = 0; a2 < c; ++a2) s2 -= z[a2] * T[c * m + a2];
                z[c] = s2 / T[c * m + c];
            }
            for (int c = 0; c < m; ++c) xr[c] = z[c];
        }
        __syncthreads();
    }
    // ---- HX (nh x m): rows i < dn: lam_i x_i + C~_i z ; rows dn+a: C~^T y + D~ z
    for (int e = threadIdx.x; e < dn * m; e += blockDim.x) {
        const int i = e / m, c = e % m;
        double s2 = w.lam[i] * Xp[(int64_t)i * xst + c];
        for (int a2 = 0; a2 < r; ++a2) s2 += Ctp[(int64_t)i * cst + a2] * Xp[(int64_t)(dn + a2) * xst + c];
        HXp[(int64_t)i * xst + c] = s2;
    }
    for (int e = threadIdx.x; e < r * m; e += blockDim.x) {
        const int a2 = e / m, c = e % m;
        double s2 = 0.0;
        for (int i = 0; i < dn; ++i) s2 += Ctp[(int64_t)i * cst + a2] * Xp[(int64_t)i * xst + c];
        for (int b2 = 0; b2 < r; ++b2) s2 += w.Dt[a2 * ld + b2] * Xp[(int64_t)(dn + b2) * xst + c];
        HXp[(int64_t)(dn + a2) * xst + c] = s2;
    }
    __syncthreads();
    // ---- T = X^T HX, symmetrised
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int a2 = e / m, b2 = e % m;
        double s2 = 0.0;
        for (int i = 0; i < nh; ++i) s2 += Xp[(int64_t)i * xst + a2] * HXp[(int64_t)i * xst + b2];
        Q[e] = s2;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int a2 = e / m, b2 = e % m;
        T[e] = 0.5 * (Q[a2 * m + b2] + Q[b2 * m + a2]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) Q[e] = (e / m == e % m) ? 1.0 : 0.0;
    __syncthreads();
    // ---- cyclic Jacobi with the round-robin ordering (m even)
    for (int sweep = 0; sweep < 30; ++sweep) {
        for (int round = 0; round < m - 1; ++round) {
            if ((int)threadIdx.x < m / 2) {
                const int k2 = threadIdx.x;
                auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (m - 1)) + 1; };
                int p = player(k2), q = player(m - 1 - k2);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                pairs[2 * k2] = p;
                pairs[2 * k2 + 1] = q;
                const double apq = T[p * m + q], app = T[p * m + p], aqq = T[q * m + q];
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
            for (int e = threadIdx.x; e < (m / 2) * m; e += blockDim.x) {  // rows: J^T T
                const int k2 = e / m, j = e % m, p = pairs[2 * k2], q = pairs[2 * k2 + 1];
                const double c = cs[k2], sv = sn[k2];
                const double tp = T[p * m + j], tq = T[q * m + j];
                T[p * m + j] = c * tp - sv * tq;
                T[q * m + j] = sv * tp + c * tq;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < (m / 2) * m; e += blockDim.x) {  // columns: T J, Q J
                const int k2 = e / m, i = e % m, p = pairs[2 * k2], q = pairs[2 * k2 + 1];
                const double c = cs[k2], sv = sn[k2];
                const double tp = T[i * m + p], tq = T[i * m + q];
                T[i * m + p] = c * tp - sv * tq;
                T[i * m + q] = sv * tp + c * tq;
                const double qp = Q[i * m + p], qq = Q[i * m + q];
                Q[i * m + p] = c * qp - sv * qq;
                Q[i * m + q] = sv * qp + c * qq;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double off = 0.0;
            for (int a2 = 0; a2 < m; ++a2)
                for (int b2 = 0; b2 < m; ++b2)
                    if (a2 != b2) off = fmax(off, fabs(T[a2 * m + b2]) / sqrt(fabs(T[a2 * m + a2] * T[b2 * m + b2]) + 1e-300));
            s_off = off;
        }
        __syncthreads();
        if (s_off < 1e-15) break;
        __syncthreads();
    }
    // ---- sort Ritz values ascending and write Xr = X Q(:, order), theta
    if (threadIdx.x == 0) {
        for (int a2 = 0; a2 < m; ++a2) {
            order[a2] = a2;
            s_theta[a2] = T[a2 * m + a2];
        }
        for (int a2 = 1; a2 < m; ++a2) {  // insertion sort, stable
            const int oa = order[a2];
            int b2 = a2 - 1;
            while (b2 >= 0 && s_theta[order[b2]] > s_theta[oa]) {
                order[b2 + 1] = order[b2];
                --b2;
            }
            order[b2 + 1] = oa;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < m; c += blockDim.x) w.theta[c] = s_theta[order[c]];
    for (int e = threadIdx.x; e < (dn + ld) * ld; e += blockDim.x) {
        const int i = e / ld, c = e % ld;
        double v = 0.0;
        if (i < nh && c < m) {
            const int oc = order[c];
            for (int a2 = 0; a2 < m; ++a2) v += Xp[(int64_t)i * xst + a2] * Q[a2 * m + oc];
        }
        w.Xr[(int64_t)i * ld + c] = v;
    }
}

// ---------------------------------------------- recombination coefficients
// X_v = Pi_r L^-T z (ld x ld), X_c = y - G X_v (dn x ld).
__global__ __launch_bounds__(256) void k_recombine_coeffs(SmallWork w) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn, r = w.status[ST_RANK];
    double *Xv = sm;  // ld x ld
    for (int e = threadIdx.x; e < ld * ld; e += blockDim.x) Xv[e] = 0.0;
    __syncthreads();
    if ((int)threadIdx.x < ld) {
        const int c = threadIdx.x;
        double t[kMaxWidth];
        for (int a = r - 1; a >= 0; --a) {
            double s = w.Xr[(int64_t)(dn + a) * ld + c];
            for (int b = a + 1; b < r; ++b) s -= w.L1[b * ld + a] * t[b];
            t[a] = s / w.L1[a * ld + a];
        }
        for (int a = 0; a < r; ++a) Xv[w.perm[a] * ld + c] = t[a];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ld * ld; e += blockDim.x) w.Xv[e] = Xv[e];
    for (int e = threadIdx.x; e < dn * ld; e += blockDim.x) {
        const int i = e / ld, c = e % ld;
        const double *gi = w.FG + (int64_t)i * 2 * ld + ld;
        double s = w.Xr[(int64_t)i * ld + c];
        for (int a = 0; a < ld; ++a) s -= gi[a] * Xv[a * ld + c];
        w.Xc[e] = s;
    }
}

__global__ void k_theta_update(SmallWork w, double *theta_out, int final_level) {
    if (w.status[ST_CONVERGED]) return;
    const int c = threadIdx.x;
    if (c < w.ld) theta_out[c] = w.theta[c];
    if (c == 0) {
        w.status[ST_WARM] = 1;
        if (final_level) w.status[ST_STEPS] += 1;
    }
}

// ------------------------------------------------------------ launchers
void launch_small_products(hipStream_t s, const SmallWork &w) {
    dim3 grid((w.ld + 15) / 16, (3 * w.ld + 15) / 16);
    hipLaunchKernelGGL(k_small_products, grid, dim3(256), 0, s, w.dn, w.ld, w.lam, w.FG, w.P3, w.status);
}

void launch_pencil(hipStream_t s, const SmallWork &w, double rank_tol) {
    const size_t lds = 3 * (size_t)w.ld * w.ld * sizeof(double);
    hipLaunchKernelGGL(k_pencil, dim3(1), dim3(kB), lds, s, w, rank_tol);
}

void launch_arrow_eig(hipStream_t s, const SmallWork &w, int qe, const double *theta_prev) {
    const int r = w.ld;  // upper bound of the rank
    const int ct_in_lds = (int64_t)w.dn * r <= 8192 ? 1 : 0;
    const size_t rows = ct_in_lds ? (size_t)w.dn : 64;
    const size_t lds = ((size_t)r * (r + 1) + rows * r + (size_t)w.dn + (size_t)w.dn + r + r) * sizeof(double);
    const int threads = r <= 32 ? 64 : 256;
    hipLaunchKernelGGL(k_arrow_bisect, dim3(qe), dim3(threads), lds, s, w, theta_prev, ct_in_lds);
    // the rank is only known on the device: size the LDS path for r = ld
    const size_t base = 2 * (size_t)qe * qe + 32 * (size_t)qe;
    const size_t nh = (size_t)w.dn + w.ld;
    const size_t full = base + 2 * nh * qe + (size_t)w.dn * w.ld;
    const int use_lds = full * sizeof(double) <= 150 * 1024 ? 1 : 0;
    hipLaunchKernelGGL(k_arrow_rr, dim3(1), dim3(kB), (use_lds ? full : base) * sizeof(double), s, w, qe, use_lds);
}

void launch_recombine_coeffs(hipStream_t s, const SmallWork &w) {
    hipLaunchKernelGGL(k_recombine_coeffs, dim3(1), dim3(kB), (size_t)w.ld * w.ld * sizeof(double), s, w);
}

void launch_theta_update(hipStream_t s, const SmallWork &w, double *theta_out, int final_level) {
    hipLaunchKernelGGL(k_theta_update, dim3(1), dim3(128), 0, s, w, theta_out, final_level);
}

}  // namespace amgeig
