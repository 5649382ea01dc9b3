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
__device__ int bk_factor(double *S, int r, int ls, int *ipiv, double *mult) {
    __shared__ int s_kp, s_size, s_neg;
    const double alpha = 0.6403882032022076;  // (1 + sqrt(17)) / 8
    if (threadIdx.x == 0) s_neg = 0;
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
            // column p and its multipliers l_i = S[i][p] / d are staged in
            // mult[] so that the trailing update and the store of the
            // multipliers into column p share one pass
            const double d = S[p * ls + p];
            const double dinv = d != 0.0 ? 1.0 / d : 0.0;
            if (threadIdx.x == 0) {
                ipiv[p] = kp;
                if (d < 0.0) s_neg += 1;
            }
            for (int i = p + 1 + threadIdx.x; i < r; i += blockDim.x) {
                const double c1 = S[i * ls + p];
                mult[4 * i] = c1 * dinv;
                mult[4 * i + 2] = c1;
            }
            __syncthreads();
            const int m = r - p - 1;
            for (int e = threadIdx.x; e < m * (m + 1); e += blockDim.x) {
                const int i = p + 1 + e / (m + 1), jj = e % (m + 1);
                if (jj == m) {
                    S[i * ls + p] = mult[4 * i];
                } else {
                    const int j = p + 1 + jj;
                    S[i * ls + j] -= mult[4 * i] * mult[4 * j + 2];
                }
            }
            __syncthreads();
            p += 1;
        } else {
            const double a = S[p * ls + p], b = S[(p + 1) * ls + p], c = S[(p + 1) * ls + p + 1];
            const double det = a * c - b * b;
            if (threadIdx.x == 0) {
                ipiv[p] = ipiv[p + 1] = -(kp + 1);
                s_neg += det < 0.0 ? 1 : (a + c < 0.0 ? 2 : 0);
            }
            const double id = 1.0 / det;
            // l_i = [S[i][p], S[i][p+1]] D^-1 and the two column entries
            // themselves, staged in mult[4i .. 4i+3]
            for (int i = p + 2 + threadIdx.x; i < r; i += blockDim.x) {
                const double c1 = S[i * ls + p], c2 = S[i * ls + p + 1];
                mult[4 * i] = (c1 * c - c2 * b) * id;
                mult[4 * i + 1] = (c2 * a - c1 * b) * id;
                mult[4 * i + 2] = c1;
                mult[4 * i + 3] = c2;
            }
            __syncthreads();
            const int m = r - p - 2;
            for (int e = threadIdx.x; e < m * (m + 1); e += blockDim.x) {
                const int i = p + 2 + e / (m + 1), jj = e % (m + 1);
                const double l1 = mult[4 * i], l2 = mult[4 * i + 1];
                if (jj == m) {
                    S[i * ls + p] = l1;
                    S[i * ls + p + 1] = l2;
                } else {
                    const int j = p + 2 + jj;
                    S[i * ls + j] -= l1 * mult[4 * j + 2] + l2 * mult[4 * j + 3];
                }
            }
            __syncthreads();
            p += 2;
        }
    }
    __syncthreads();
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
    // L^T w = y, blocks from the last one backwards (a 2x2 block has both
    // ipiv entries negative): once w of a block is known, remove its
    // contribution from the rows above.
    for (int p = r - 1; p >= 0;) {
        if (ipiv[p] < 0) {
            const int p0 = p - 1;
            const double w0 = f[p0], w1 = f[p];
            for (int i = threadIdx.x; i < p0; i += blockDim.x) f[i] -= S[p0 * ls + i] * w0 + S[p * ls + i] * w1;
            p -= 2;
        } else {
            const double wp = f[p];
            for (int i = threadIdx.x; i < p; i += blockDim.x) f[i] -= S[p * ls + i] * wp;
            p -= 1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {  // undo the interchanges in reverse order
        for (int p = r - 1; p >= 0;) {
            if (ipiv[p] < 0) {
                const int kp = -ipiv[p] - 1;
                const double t = f[p];
                f[p] = f[kp];
                f[kp] = t;
                p -= 2;
            } else {
                const int kp = ipiv[p];
                const double t = f[p];
                f[p] = f[kp];
                f[kp] = t;
                p -= 1;
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
// (Sylvester).  The eigenvalue is bracketed (a warm bracket around the
// previous step's Ritz value when two counts validate it, else Gershgorin and
// the interlacing bound mu_{k+1} <= lambda_{k+1}) and isolated by bisection.
// Inside the isolating bracket, Rayleigh-quotient iteration with the exact
// Schur-complement solve (H - s)^-1 refines the eigenvector: every
// factorisation is also a count and narrows the bracket, and an iterate is
// accepted once its Rayleigh quotient rho lies in the bracket with
// ||H x - rho x|| <= 1e-10 |rho|, which pins it to the bracketed eigenvalue.
// A shift leaving the bracket falls back to the bracket midpoint.

constexpr int kPairGroup = 8;  // pairs of S accumulated per work item
constexpr int kMaxItems = 4;   // work items per thread (npairs <= 4 * 256 * 8)

__global__ __launch_bounds__(256) void k_arrow_bisect(SmallWork w, const double *__restrict__ theta_prev,
                                                      int ct_in_lds) {
    extern __shared__ double sm[];
    if (w.status[ST_CONVERGED]) return;
    const int ld = w.ld, dn = w.dn, k = blockIdx.x;
    const int r = w.status[ST_RANK];
    const int ls = r + 1;
    const int nthr = blockDim.x;
    const int npairs = r * (r + 1) / 2;
    const int ngroups = (npairs + kPairGroup - 1) / kPairGroup;
    const int slices = ngroups >= nthr ? 1 : nthr / (ngroups > 0 ? ngroups : 1);
    double *S = sm;                      // r x ls
    double *cch = S + r * ls;            // C~ (dn x r) in LDS, or a 64-row chunk
    const int chunk_rows = ct_in_lds ? dn : 64;
    double *wdn = cch + chunk_rows * r;  // dn weights 1 / (lambda_i - sigma)
    double *vec = wdn + dn;              // dn + r : current vector
    double *hx = vec + dn + r;           // dn + r : H x
    double *fz = hx + dn + r;            // r
    double *lam = fz + r;                // dn
    double *dt = lam + dn;               // r x r
    double *mult = dt + r * r;           // 4 r: multipliers and pivot columns of the factorisation
    double *part = mult + 4 * r;         // slices x npairs partial sums (also reused for reductions)
    __shared__ int ipiv[kMaxWidth];
    __shared__ double red[kB];
    const uint64_t t_start_g = wall_clock64();
    if (ct_in_lds)
        for (int e = threadIdx.x; e < dn * r; e += nthr) cch[e] = w.Ct[(int64_t)(e / r) * ld + e % r];
    for (int i = threadIdx.x; i < dn; i += nthr) lam[i] = w.lam[i];
    for (int e = threadIdx.x; e < r * r; e += nthr) dt[e] = w.Dt[(e / r) * ld + e % r];
    __syncthreads();

    int ncount = 0;
    __shared__ unsigned long long tim[4];  // S formation, BK, solve, Rayleigh (thread 0)
    if (threadIdx.x == 0) tim[0] = tim[1] = tim[2] = tim[3] = 0;
    // ---- factorisation of H - sigma through S(sigma); returns nu(sigma)
    auto factor = [&](double sigma) -> int {
        ++ncount;
        const uint64_t f0 = wall_clock64();
        int lo_i = 0, hi_i = dn;  // #{lambda_i < sigma}, lam ascending
        while (lo_i < hi_i) {
            const int mid = (lo_i + hi_i) / 2;
            if (lam[mid] < sigma) lo_i = mid + 1; else hi_i = mid;
        }
        const int nlow = lo_i;
        __syncthreads();
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double den = lam[i] - sigma;
            if (den == 0.0) den = 1e-300;
            wdn[i] = 1.0 / den;
        }
        // S partial sums: work item = (pair group g, row slice sl); a thread owns
        // at most kMaxItems items, kept in registers across the row chunks
        double acc[kMaxItems][kPairGroup];
        int pa[kMaxItems][kPairGroup], pb[kMaxItems][kPairGroup];
        const int nitems = ngroups * slices;
#pragma unroll
        for (int j = 0; j < kMaxItems; ++j) {
            const int item = threadIdx.x + j * nthr;
            const int g = item < nitems ? item % ngroups : 0;
#pragma unroll
            for (int t = 0; t < kPairGroup; ++t) {
                int pr = g * kPairGroup + t;
                acc[j][t] = 0.0;
                if (pr >= npairs) pr = npairs > 0 ? npairs - 1 : 0;  // padded pairs: computed, never stored
                int aa = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
                while (aa * (aa + 1) / 2 > pr) --aa;
                while ((aa + 1) * (aa + 2) / 2 <= pr) ++aa;
                pa[j][t] = aa;
                pb[j][t] = pr - aa * (aa + 1) / 2;
            }
        }
        __syncthreads();  // wdn ready
        for (int i0 = 0; i0 < dn; i0 += chunk_rows) {
            const int lim = dn - i0 < chunk_rows ? dn - i0 : chunk_rows;
            if (!ct_in_lds) {
                __syncthreads();
                for (int e = threadIdx.x; e < lim * r; e += nthr) cch[e] = w.Ct[(int64_t)(i0 + e / r) * ld + e % r];
                __syncthreads();
            }
            const double *ct = ct_in_lds ? cch + (int64_t)i0 * r : cch;
#pragma unroll
            for (int j = 0; j < kMaxItems; ++j) {
                const int item = threadIdx.x + j * nthr;
                if (item >= nitems) continue;
                const int sl = item / ngroups;
                for (int ii = sl; ii < lim; ii += slices) {
                    const double wi = wdn[i0 + ii];
                    const double *row = ct + ii * r;
#pragma unroll
                    for (int t = 0; t < kPairGroup; ++t) acc[j][t] += row[pa[j][t]] * row[pb[j][t]] * wi;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kMaxItems; ++j) {
            const int item = threadIdx.x + j * nthr;
            if (item >= nitems) continue;
            const int g = item % ngroups, sl = item / ngroups;
            for (int t = 0; t < kPairGroup; ++t) {
                const int pr = g * kPairGroup + t;
                if (pr < npairs) part[sl * npairs + pr] = acc[j][t];
            }
        }
        __syncthreads();
        for (int pr = threadIdx.x; pr < npairs; pr += nthr) {
            double v = 0.0;
            for (int sl = 0; sl < slices; ++sl) v += part[sl * npairs + pr];
            int aa = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
            while (aa * (aa + 1) / 2 > pr) --aa;
            while ((aa + 1) * (aa + 2) / 2 <= pr) ++aa;
            const int bb = pr - aa * (aa + 1) / 2;
            v = dt[aa * r + bb] - (aa == bb ? sigma : 0.0) - v;
            S[aa * ls + bb] = v;
            S[bb * ls + aa] = v;
        }
        __syncthreads();
        const uint64_t f1 = wall_clock64();
        const int neg = bk_factor(S, r, ls, ipiv, mult);
        if (threadIdx.x == 0) {
            const uint64_t f2 = wall_clock64();
            tim[0] += f1 - f0;
            tim[1] += f2 - f1;
        }
        return nlow + neg;
    };

    // ---- sum over the dn coarse rows of C~_{i a} u_i, for all a (slices + LDS)
    auto ct_t_times = [&](const double *u, double *out) {
        const int sl2 = nthr / (r > 0 ? r : 1) > 0 ? nthr / (r > 0 ? r : 1) : 1;
        for (int item = threadIdx.x; item < r * sl2; item += nthr) {
            const int a2 = item % r, sl = item / r;
            double s0 = 0.0, s1 = 0.0;
            int i = sl;
            for (; i + sl2 < dn; i += 2 * sl2) {
                const double *c0 = ct_in_lds ? cch + (int64_t)i * r : w.Ct + (int64_t)i * ld;
                const double *c1 = ct_in_lds ? cch + (int64_t)(i + sl2) * r : w.Ct + (int64_t)(i + sl2) * ld;
                s0 += c0[a2] * u[i];
                s1 += c1[a2] * u[i + sl2];
            }
            if (i < dn) s0 += (ct_in_lds ? cch[(int64_t)i * r + a2] : w.Ct[(int64_t)i * ld + a2]) * u[i];
            part[sl * r + a2] = s0 + s1;
        }
        __syncthreads();
        for (int a2 = threadIdx.x; a2 < r; a2 += nthr) {
            double v = 0.0;
            for (int sl = 0; sl < sl2; ++sl) v += part[sl * r + a2];
            out[a2] = v;
        }
        __syncthreads();
    };
    auto ct_row = [&](int i, int a2) -> double { return ct_in_lds ? cch[(int64_t)i * r + a2] : w.Ct[(int64_t)i * ld + a2]; };

    // ---- x <- (H - sigma)^-1 x for the factorisation in S, ipiv, wdn
    auto solve = [&](double *x) {
        for (int i = threadIdx.x; i < dn; i += nthr) x[i] *= wdn[i];  // t = (Lambda - sigma)^-1 b_y
        __syncthreads();
        ct_t_times(x, fz);
        for (int a2 = threadIdx.x; a2 < r; a2 += nthr) fz[a2] = x[dn + a2] - fz[a2];
        __syncthreads();
        bk_solve(S, r, ls, ipiv, fz);
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double s2 = 0.0;
            for (int a2 = 0; a2 < r; ++a2) s2 += ct_row(i, a2) * fz[a2];
            x[i] -= s2 * wdn[i];
        }
        for (int a2 = threadIdx.x; a2 < r; a2 += nthr) x[dn + a2] = fz[a2];
        __syncthreads();
    };
    auto normalise = [&](double *x) {
        double s2 = 0.0;
        for (int i = threadIdx.x; i < dn + r; i += nthr) s2 += x[i] * x[i];
        s2 = block_sum(s2, red);
        const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
        for (int i = threadIdx.x; i < dn + r; i += nthr) x[i] *= inv;
        __syncthreads();
    };
    // rho = x^T H x (x normalised) and ||H x - rho x||
    auto rayleigh = [&](const double *x, double &rho, double &res) {
        ct_t_times(x, fz);  // C~^T y
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double s2 = lam[i] * x[i];
            for (int a2 = 0; a2 < r; ++a2) s2 += ct_row(i, a2) * x[dn + a2];
            hx[i] = s2;
        }
        for (int a2 = threadIdx.x; a2 < r; a2 += nthr) {
            double s2 = fz[a2];
            for (int b2 = 0; b2 < r; ++b2) s2 += dt[a2 * r + b2] * x[dn + b2];
            hx[dn + a2] = s2;
        }
        __syncthreads();
        double q = 0.0;
        for (int i = threadIdx.x; i < dn + r; i += nthr) q += x[i] * hx[i];
        rho = block_sum(q, red);
        double e2 = 0.0;
        for (int i = threadIdx.x; i < dn + r; i += nthr) {
            const double d = hx[i] - rho * x[i];
            e2 += d * d;
        }
        res = sqrt(block_sum(e2, red));
    };

    // ---- warm start.  The corrected vector V e_k has the coordinates
    // y = G e_k, z = L^T Pi^T e_k in the basis of H (its part outside span Z is
    // (V - Z G) e_k = W L^T Pi^T e_k); after the first correction it is close
    // to the wanted eigenvector, so its Rayleigh quotient is a good shift.
    double lo = 0.0, hi = 0.0;
    int nulo = 0, nuhi = 1 << 30;
    bool have_lo = false, have_hi = false;
    bool done = false;
    const double tp = theta_prev[k];
    const double cap = lam[k] * (1.0 + 1e-14) + 1e-300;  // interlacing: mu_k <= lambda_k
    double rho = 0.0, res = 0.0;
    __shared__ int s_pos;
    const bool warm = w.status[ST_WARM] != 0;
    if (warm) {
        if (threadIdx.x == 0) {
            s_pos = -1;
            for (int a2 = 0; a2 < r; ++a2)
                if (w.perm[a2] == k) s_pos = a2;
        }
        __syncthreads();
        const int pos = s_pos;
        for (int i = threadIdx.x; i < dn + r; i += nthr) {
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
        rayleigh(vec, rho, res);
        const bool ok0 = rho > 0.0 && rho < cap;
        if (ok0 && res <= 1e-10 * fabs(rho)) {
            // already accurate: two counts around rho decide
            const double span = fmax(4.0 * res, 1e-12 * fabs(rho));
            const int cl = factor(rho - span);
            if (cl <= k) { lo = rho - span; nulo = cl; have_lo = true; }
            const double h0 = fmin(rho + span, cap);
            const int ch = factor(h0);
            if (ch >= k + 1) { hi = h0; nuhi = ch; have_hi = true; }
            done = have_lo && have_hi && nulo == k && nuhi == k + 1;
        } else {
            const double s0 = ok0 ? rho : (tp > 0.0 && tp < cap ? tp : -1.0);
            if (s0 > 0.0) {
                const double rho0 = rho;
                const int c0 = factor(s0);
                if (c0 <= k) { lo = s0; nulo = c0; have_lo = true; } else { hi = s0; nuhi = c0; have_hi = true; }
                solve(vec);
                normalise(vec);
                rayleigh(vec, rho, res);
                const double span = fmax(4.0 * res, 1e-12 * fabs(rho));
                if (have_lo && !(fabs(rho - s0) > res)) {
                    // the shift is too close to rho to serve as the bracket end
                    have_lo = false;
                }
                if (have_hi && !(fabs(rho - s0) > res)) have_hi = false;
                if (!have_lo) {
                    const double l0 = fmin(rho, rho0 > 0.0 ? rho0 : rho) - span;
                    const int c1 = factor(l0);
                    if (c1 <= k) { lo = l0; nulo = c1; have_lo = true; }
                }
                if (!have_hi) {
                    const double h0 = fmin(rho + span, cap);
                    const int c1 = factor(h0);
                    if (c1 >= k + 1) { hi = h0; nuhi = c1; have_hi = true; }
                }
                if (have_lo && have_hi && nulo == k && nuhi == k + 1) {
                    const bool inside = rho > lo && rho < hi;
                    done = inside && res <= 1e-10 * fabs(rho) && rho - lo > res && hi - rho > res;
                }
            }
        }
    } else {
        for (int i = threadIdx.x; i < dn + r; i += nthr) vec[i] = start_entry(k, i);
        __syncthreads();
    }
    const bool have = have_lo && have_hi;
    if (!have) {
        double g = 1e300;
        for (int i = threadIdx.x; i < dn; i += nthr) {
            double s2 = 0.0;
            for (int a2 = 0; a2 < r; ++a2) s2 += fabs(ct_row(i, a2));
            g = fmin(g, lam[i] - s2);
        }
        for (int a2 = threadIdx.x; a2 < r; a2 += nthr) {
            double s2 = 0.0;
            for (int b2 = 0; b2 < r; ++b2)
                if (b2 != a2) s2 += fabs(dt[a2 * r + b2]);
            for (int i = 0; i < dn; ++i) s2 += fabs(ct_row(i, a2));
            g = fmin(g, dt[a2 * r + a2] - s2);
        }
        red[threadIdx.x] = g;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mn = red[0];
            for (int t = 1; t < nthr; ++t) mn = fmin(mn, red[t]);
            red[0] = mn;
        }
        __syncthreads();
        const double glo = red[0];
        __syncthreads();
        if (!have_hi) {
            hi = cap;
            nuhi = 1 << 30;  // not counted yet (at least k + 1 by interlacing)
        }
        if (!have_lo) {
            lo = glo - fabs(glo) * 1e-14 - 1e-300;
            nulo = 0;        // Gershgorin: no eigenvalue below lo
        }
    }
    // ---- isolate by bisection
    for (int it = 0; it < 200 && !done; ++it) {
        if (nulo == k && nuhi == k + 1) break;
        if (hi - lo <= 1e-13 * fmax(fabs(lo), fabs(hi))) break;  // a cluster closer than rounding
        const double mid = 0.5 * (lo + hi);
        const int c = factor(mid);
        if (c >= k + 1) { hi = mid; nuhi = c; } else { lo = mid; nulo = c; }
    }
    const uint64_t t_bracket = wall_clock64();
    // ---- Rayleigh-quotient iteration inside the bracket
    double sigma = (rho > lo && rho < hi) ? rho : ((tp > lo && tp < hi) ? tp : 0.5 * (lo + hi));
    for (int it = 0; it < 12 && !done; ++it) {
        const int c = factor(sigma);
        if (c >= k + 1) { hi = fmin(hi, sigma); } else { lo = fmax(lo, sigma); }
        const uint64_t q0 = wall_clock64();
        solve(vec);
        normalise(vec);
        const uint64_t q1 = wall_clock64();
        rayleigh(vec, rho, res);
        if (threadIdx.x == 0) {
            tim[2] += q1 - q0;
            tim[3] += wall_clock64() - q1;
        }
        const bool inside = rho > lo && rho < hi;
        if (inside && res <= 1e-10 * fabs(rho) && rho - lo > res && hi - rho > res) break;
        sigma = inside ? rho : 0.5 * (lo + hi);
        if (hi - lo <= 1e-13 * fmax(fabs(lo), fabs(hi))) break;
    }
    const uint64_t t_refine = wall_clock64();
    if (threadIdx.x == 0 && w.diag) {
        atomicAdd(&w.diag[k], ncount);
        atomicAdd(&w.diag[kMaxWidth + k], done ? 1 : 0);
        atomicAdd(&w.diag[2 * kMaxWidth + k], 1);
    }
    for (int i = threadIdx.x; i < dn + ld; i += nthr) w.X[(int64_t)i * ld + k] = i < dn + r ? vec[i] : 0.0;
    const uint64_t t_end = wall_clock64();
    if (threadIdx.x == 0 && w.diag && k == 0) {
        atomicAdd(&w.diag[5 * kMaxWidth - 8], (int)(t_bracket - t_start_g));
        atomicAdd(&w.diag[5 * kMaxWidth - 7], (int)(t_refine - t_bracket));
        atomicAdd(&w.diag[5 * kMaxWidth - 6], (int)(t_end - t_refine));
        atomicAdd(&w.diag[5 * kMaxWidth - 5], (int)tim[0]);
        atomicAdd(&w.diag[5 * kMaxWidth - 4], (int)tim[1]);
        atomicAdd(&w.diag[5 * kMaxWidth - 3], (int)tim[2]);
        atomicAdd(&w.diag[5 * kMaxWidth - 2], (int)tim[3]);
    }
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
    double *lamv = xs + 32 * m;  // dn
    double *dtv = lamv + dn;     // ld x ld
    for (int i = threadIdx.x; i < dn; i += blockDim.x) lamv[i] = w.lam[i];
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) dtv[e] = w.Dt[(e / r) * ld + e % r];
    double *Xp = w.X, *HXp = w.HX;
    const double *Ctp = w.Ct;
    int xst = ld, cst = ld;
    if (use_lds) {
        double *Xl = dtv + ld * ld;
        double *HXl = Xl + nh * m;
        double *Ctl = HXl + nh * m;
        for (int e = threadIdx.x; e < nh * m; e += blockDim.x) Xl[e] = w.X[(int64_t)(e / m) * ld + e % m];
        for (int e = threadIdx.x; e < dn * r; e += blockDim.x) Ctl[e] = w.Ct[(int64_t)(e / r) * ld + e % r];
        Xp = Xl;
        HXp = HXl;
        Ctp = Ctl;
        xst = m;
        cst = r;
    }
    __syncthreads();
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
        double s2 = lamv[i] * Xp[(int64_t)i * xst + c];
        for (int a2 = 0; a2 < r; ++a2) s2 += Ctp[(int64_t)i * cst + a2] * Xp[(int64_t)(dn + a2) * xst + c];
        HXp[(int64_t)i * xst + c] = s2;
    }
    for (int e = threadIdx.x; e < r * m; e += blockDim.x) {
        const int a2 = e / m, c = e % m;
        double s2 = 0.0;
        for (int i = 0; i < dn; ++i) s2 += Ctp[(int64_t)i * cst + a2] * Xp[(int64_t)i * xst + c];
        for (int b2 = 0; b2 < r; ++b2) s2 += dtv[a2 * r + b2] * Xp[(int64_t)(dn + b2) * xst + c];
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
        if (threadIdx.x == 0 && w.diag) atomicAdd(&w.diag[4 * kMaxWidth], 1);
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
    double *Xv = sm;             // ld x ld
    double *L1 = Xv + ld * ld;   // ld x ld
    double *z = L1 + ld * ld;    // r x ld
    for (int e = threadIdx.x; e < ld * ld; e += blockDim.x) {
        Xv[e] = 0.0;
        L1[e] = w.L1[e];
    }
    for (int e = threadIdx.x; e < r * ld; e += blockDim.x) z[e] = w.Xr[(int64_t)(dn + e / ld) * ld + e % ld];
    __syncthreads();
    if ((int)threadIdx.x < ld) {
        const int c = threadIdx.x;
        double t[kMaxWidth];
        for (int a = r - 1; a >= 0; --a) {
            double s = z[a * ld + c];
            for (int b = a + 1; b < r; ++b) s -= L1[b * ld + a] * t[b];
            t[a] = s / L1[a * ld + a];
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
    const int threads = r <= 32 ? 64 : 256;
    const size_t npairs = (size_t)r * (r + 1) / 2;
    const size_t ngroups = (npairs + 7) / 8;
    const size_t slices = ngroups >= (size_t)threads ? 1 : threads / ngroups;
    size_t partsz = slices * npairs;
    if (partsz < (size_t)threads) partsz = threads;  // also holds the C~^T u partials
    const size_t lds = ((size_t)r * (r + 1) + rows * r + (size_t)w.dn + 2 * ((size_t)w.dn + r) + r + (size_t)w.dn +
                        (size_t)r * r + 4 * (size_t)r + partsz) * sizeof(double);
    hipLaunchKernelGGL(k_arrow_bisect, dim3(qe), dim3(threads), lds, s, w, theta_prev, ct_in_lds);
    // the rank is only known on the device: size the LDS path for r = ld
    const size_t base = 2 * (size_t)qe * qe + 32 * (size_t)qe + (size_t)w.dn + (size_t)w.ld * w.ld;
    const size_t nh = (size_t)w.dn + w.ld;
    const size_t full = base + 2 * nh * qe + (size_t)w.dn * w.ld;
    const int use_lds = full * sizeof(double) <= 150 * 1024 ? 1 : 0;
    hipLaunchKernelGGL(k_arrow_rr, dim3(1), dim3(kB), (use_lds ? full : base) * sizeof(double), s, w, qe, use_lds);
}

void launch_recombine_coeffs(hipStream_t s, const SmallWork &w) {
    hipLaunchKernelGGL(k_recombine_coeffs, dim3(1), dim3(kB), 3 * (size_t)w.ld * w.ld * sizeof(double), s, w);
}

void launch_theta_update(hipStream_t s, const SmallWork &w, double *theta_out, int final_level) {
    hipLaunchKernelGGL(k_theta_update, dim3(1), dim3(128), 0, s, w, theta_out, final_level);
}

}  // namespace amgeig
