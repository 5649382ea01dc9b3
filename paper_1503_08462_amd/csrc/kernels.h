// Host-side launchers of the gfx950 kernels (all enqueue on the given stream).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace amgeig {

// status words (int32, device)
enum : int {
    ST_CONVERGED = 0,  // residual test of the finest level holds: later steps skip
    ST_STEPS = 1,      // finest-level corrections done
    ST_RANK = 2,       // columns of the new block kept after M-orthogonalisation
    ST_BREAKDOWN = 3,  // set when the projected problem lost definiteness
    ST_WARM = 4,       // the previous Ritz values may seed the eigenvalue brackets
    ST_COUNT = 8
};

constexpr int kMaxWidth = 80;  // block width limit (LDS budget of the small kernels)

// ---------------------------------------------------------- kernels_vec.hip
int64_t residual_blocks(int64_t n, int ld, int cpt);
int64_t residual_blocks_max(int64_t n, int ld);  // the most over the columns-per-lane choices
int64_t gram_blocks(int64_t n, int ld);
template <typename TO>
void launch_residual(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                     const double *m, const double *U, const double *theta, TO *R, double *part, const int *status,
                     int cpt = 0);
// right-hand side of a further cycle of one correction:
// R = (Theta - sigma) M U - (A - sigma M) V (working precision T)
template <typename T>
void launch_residual_cycle(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                           const double *m, const double *U, const double *V, const double *theta, double sigma, T *R,
                           const int *status, int cpt);
// the norms rho_j and the convergence flag from the partial sums of launch_residual
void launch_residual_finish(hipStream_t s, int64_t n, int ld, double *part, unsigned *counter, const double *theta,
                            double *rho, int q, double tol, int *status, int check, int cpt = 0);
template <typename T>
void launch_smooth_pre(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *vs,
                       const T *dinv, const T *b, T *r, const int *status, int cpt = 0);
template <typename T>
void launch_spmm(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                 const T *x, T *y, const int *status, int cpt = 0);
template <typename T>
void launch_prolong_add(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                        const T *xc, const T *dinv, const T *b, T *y, const int *status, int cpt = 0);
template <typename T>
void launch_smooth_post(hipStream_t s, bool final, int64_t n, int ld, const int32_t *ptr, const int32_t *col,
                        const T *val, const T *dinv, const T *b, const T *y, T *x, const double *U, double *V,
                        const int *status, int cpt = 0);
// One colour of a multicolour Gauss-Seidel sweep: rows[0, nrows) of a
// colour-ordered CSR without diagonal (ptr, diag and rows offset to the
// colour's first position), x_i = (b_i - sum a_ij x_j) / a_ii in place; with
// final also V_i = U_i + x_i (FP64).
template <typename T>
void launch_gs_colour(hipStream_t s, bool final, int64_t nrows, int ld, const int32_t *ptr, const int32_t *col,
                      const T *val, const T *diag, const int32_t *rows, const T *b, T *x, const double *U, double *V,
                      const int *status, int cpt = 0);
// Degree-2 Chebyshev smoothing on D^-1 A over [lo, 1] (D the l1 diagonal):
// pre-smoothing from a zero guess (x), the level residual r = b - A x, the
// prolongation y = x + P xc, and post-smoothing of y (scratch d0; x, or on
// the correction level V = U + x in FP64).
template <typename T>
void launch_cheb_pre(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *vs,
                     const T *dinv, const T *b, T *x, double lo, const int *status, int cpt = 0);
template <typename T>
void launch_level_residual(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                           const T *b, const T *x, T *r, const int *status, int cpt = 0);
template <typename T>
void launch_prolong_x(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                      const T *xc, const T *x, T *y, const int *status, int cpt = 0);
template <typename T>
void launch_cheb_post1(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const T *val,
                       const T *dinv, const T *b, const T *y, T *d0, double lo, const int *status, int cpt = 0);
template <typename T>
void launch_cheb_post2(hipStream_t s, bool final, int64_t n, int ld, const int32_t *ptr, const int32_t *col,
                       const T *val, const T *dinv, const T *y, const T *d0, T *x, const double *U, double *V,
                       double lo, const int *status, int cpt = 0);
// C (m x n) = A^T B, A K x m, B K x n (row-major), FP64 matrix-core accumulation
template <typename T>
void launch_gemm_tn(hipStream_t s, int m, int n, int K, const T *A, int lda, const T *B, int ldb, T *C, int ldc,
                    const int *status);
void launch_dual_spmm(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                      const double *m, const double *V, double *W, const int *status, int cpt = 0);
// Wide blocks (ld > 32): W = [A V | M V] and the partials of the Gram products
// in one kernel; launch_gram_reduce then forms G from the partials.
bool dual_gram_fused(int ld);
void launch_dual_gram(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *a,
                      const double *m, const double *V, double *W, double *part, const int *status, int cpt = 0);
void launch_gram_reduce(hipStream_t s, int64_t n, int ld, const double *part, double *G, const int *status);
void launch_gram(hipStream_t s, int64_t n, int ld, const double *V, const double *W, double *part, double *G,
                 const int *status);
void launch_final(hipStream_t s, int64_t n, int ld, const int32_t *ptr, const int32_t *col, const double *val,
                  const double *Y, const double *V, const double *Xv, double *U, const int *status, int cpt = 0);
// columns-per-lane choice of the row kernels: `hint` when valid for the width, else the built-in rule
bool cpt_valid(int width, int cpt);
int pick_cpt(int width, int hint);
// launch_gemm_tn for long K: sixteen wavefronts per tile of C
template <typename T>
void launch_gemm_tn_long(hipStream_t s, int m, int n, int K, const T *A, int lda, const T *B, int ldb, T *C, int ldc,
                         const int *status);
// columns j0 .. j0 + ld - 1 of the n x n identity as an n x ld block
template <typename T>
void launch_identity_block(hipStream_t s, int64_t n, int ld, int64_t j0, T *b);
// rows j0 .. of the n x n matrix Bt from the columns of the n x ld block x
template <typename T>
void launch_rows_from_block(hipStream_t s, int64_t n, int ld, int64_t j0, const T *x, T *Bt);
void launch_fill_random(hipStream_t s, int64_t n, int ld, int qe, uint64_t seed, double *U);
void launch_copy_cols(hipStream_t s, int64_t rows, int dcols, int64_t ldd, int cols, const double *src,
                      int64_t lds, double *dst);
void launch_copy_f64(hipStream_t s, int64_t count, const double *src, double *dst);
void launch_fill_i32(hipStream_t s, int count, int value, int *dst);

// -------------------------------------------------------- kernels_small.hip
// Scratch of the small kernels (device, FP64 unless noted), sizes in elements:
struct SmallWork {
    int dn = 0, ld = 0;
    const double *lam = nullptr;  // dn, ascending
    double *FG = nullptr;         // dn x 2ld: row i = [(Z^T B_A)_i | (Z^T B_M)_i] = [F_i | G_i]
    double *GAGM = nullptr;       // ld x 2ld: [V^T A V | V^T M V]
    double *P3 = nullptr;         // ld x 3ld: G^T [F | G | Lambda G]
    double *Ct = nullptr;         // dn x ld: coupling block of H
    double *Dt = nullptr;         // ld x ld: trailing block of H
    double *L1 = nullptr;         // ld x ld: Cholesky factor of the kept columns
    double *Li = nullptr;         // ld x ld: its inverse (lower)
    int *perm = nullptr;          // ld: pivot order of the M-orthogonalisation
    double *X = nullptr;          // (dn + ld) x ld: eigenvectors of H (inverse iteration)
    double *HX = nullptr;         // (dn + ld) x ld scratch
    double *Xr = nullptr;         // (dn + ld) x ld: Ritz vectors of H
    double *theta = nullptr;      // ld: Ritz values
    double *Xc = nullptr;         // dn x ld: coarse coefficients
    double *Xv = nullptr;         // ld x ld: coefficients of V
    int *status = nullptr;
    int *diag = nullptr;          // 5 * kMaxWidth + 8 counters (solver statistics; null unless
                                  // built with AMG_EIG_SMALL_STATS)
};
// Start/stop events for the next launch of a single-kernel launcher (the
// residual, smoothing, SpMM, dual SpMM and final-update launchers): recorded
// by the dispatch at the kernel's own start and end, then cleared.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_pending();
void clear_launch_events();

void launch_pencil(hipStream_t s, const SmallWork &w, double rank_tol);
// one request's small-eigensolver launch parameters, kept in device memory for
// the batched launches
// C (m x n, row stride ldc) = A^T B, A K x m and B K x n row-major (FP64);
// long_k selects the sixteen-wavefront tile code
struct GemmDesc {
    const double *A = nullptr, *B = nullptr;
    double *C = nullptr;
    int m = 0, n = 0, K = 0, lda = 0, ldb = 0, ldc = 0, long_k = 0;
};
struct SmallItem {
    SmallWork w;
    double *theta = nullptr;  // Ritz values: previous on entry, new on exit
    int qe = 0;
    int fg_in_lds = 0, ct_in_lds = 0, use_lds = 0;
    GemmDesc fg, yg;  // finest-level steps: Z^T B into FG, and Y = Z X_c
};
struct SmallLds {
    size_t pencil = 0, bisect = 0, rr = 0;  // dynamic LDS bytes per kernel
};
void small_layout(const SmallWork &w, int qe, double *theta, SmallItem *it, SmallLds *lds);
constexpr int kMaxBatch = 64;
struct SmallTable {
    const SmallItem *item[kMaxBatch];  // device addresses
    int first[kMaxBatch + 1];          // eigenvalue workgroups of member m: first[m] .. first[m+1]-1
    int p3first[kMaxBatch + 1];        // wide pencil products: P3 workgroups of member m
    int ctfirst[kMaxBatch + 1];        // and its C~ wavefronts (prefix sums; 0 for ld <= 32)
    int n;
    int final_level;                   // finest-level step (counted) or a step of the nested start
};
// P3 workgroups and C~ wavefronts of the wide pencil products of one member
// (zero for ld <= 32, where the pencil kernel forms both in LDS)
int pencil_p3_blocks(int ld);
int pencil_ct_waves(int ld, int dn);
// pencil, eigenpairs and Ritz polish of every member of the table, three
// launches in all; lds holds the largest size over the members
// wide: every member has ld > 32 (the pencil and Rayleigh-Ritz kernels then
// run sixteen wavefronts, as in a member's separate launch), else none has
void launch_small_batch(hipStream_t s, const SmallTable &t, const SmallLds &lds, double rank_tol, bool wide);
struct GemmTable {
    const SmallItem *item[kMaxBatch];  // device addresses
    int first[kMaxBatch + 1];          // tiles of member m: first[m] .. first[m+1]-1
    int n;
    int which;                         // 0: the fg product, 1: the yg product
};
// the fg or yg products of the members of the table (all with the same long_k)
void launch_gemm_batch(hipStream_t s, const GemmTable &t, bool long_k);
// eigenpairs of H, Ritz polish and recombination coefficients; theta holds the
// previous Ritz values on entry and the new ones on exit
void launch_arrow_eig(hipStream_t s, const SmallWork &w, int qe, double *theta, int final_level);

}  // namespace amgeig
