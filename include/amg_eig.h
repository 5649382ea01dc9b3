/*
 * amg_eig: AMG multilevel-correction eigensolver for A u = lambda M u on one
 * MI355X (gfx950) GPU.
 *
 * Method: Zhang, Han, He, Xie, You, "An Algebraic Multigrid Method for
 * Eigenvalue Problems in Some Different Cases" (arXiv 1503.08462).
 *   - problem (1.1): the q smallest eigenpairs of the symmetric pencil (A, M),
 *     A symmetric positive definite, M symmetric positive (semi)definite,
 *     with U^T M U = I;
 *   - hierarchy (Section 2): strength (2.1), classical Ruge-Stueben C/F
 *     splitting, direct interpolation (2.2)-(2.4), Galerkin operators (2.5);
 *   - correction step (Algorithm 3.1): one block V-cycle on A_k u = lambda M_k u
 *     from the current iterate (3.1)-(3.2), then Rayleigh-Ritz on the coarsest
 *     space augmented with the new block, eigenproblem (3.3);
 *   - driver (Algorithm 3.2): coarsest eigen-solve, prolongation and one
 *     correction per level, then corrections on the finest level.
 *
 * Conventions for every entry point:
 *   - return 0 on success, > 0 for a warning, < 0 for an error (codes below);
 *     amg_eig_strerror() names a code, amg_eig_last_error() gives the message
 *     of the last failure on a context;
 *   - no C++ exception crosses this interface;
 *   - host arrays passed in are borrowed for the duration of the call only;
 *   - device memory is owned by the caller: the solver never allocates or
 *     frees device memory; it carves everything from the workspace given to
 *     amg_eig_bind() (the exceptions are the standalone device setup routines
 *     amg_eig_galerkin(), amg_eig_pmis(), amg_eig_interpolation(),
 *     amg_eig_transpose() and amg_eig_dense_sygv(), which allocate and free
 *     their own temporaries);
 *   - all device work of a context is enqueued on the stream given to
 *     amg_eig_bind(); only amg_eig_progress() and amg_eig_solve() wait on it;
 *   - one host thread at a time per context; contexts are independent.
 * Vector blocks on the device are row-major N x ld double arrays (the values of
 * one unknown are contiguous), ld >= the number of columns.
 */
#ifndef AMG_EIG_H
#define AMG_EIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- codes */
#define AMG_EIG_OK 0
#define AMG_EIG_NOT_CONVERGED 1   /* warning: best-so-far results returned */
#define AMG_EIG_WIDENED 2         /* warning: automatic block width raised (see
                                     amg_eig_progress); the iterate is discarded */
#define AMG_EIG_EINVAL (-1)       /* malformed input or option */
#define AMG_EIG_ENOTSPD (-2)      /* a_ii <= 0 or m_ii < 0 */
#define AMG_EIG_EBREAKDOWN (-3)   /* projected problem lost definiteness */
#define AMG_EIG_ENOMEM (-4)       /* host allocation failed */
#define AMG_EIG_EWORKSPACE (-5)   /* device workspace missing or too small */
#define AMG_EIG_EHIP (-6)         /* a HIP runtime call failed */
#define AMG_EIG_ECANCELLED (-7)   /* cancelled by the caller */
#define AMG_EIG_ESTATE (-8)       /* call out of order (e.g. correct before init) */

/* --------------------------------------------------------------- options */
#define AMG_EIG_SMOOTH_L1JACOBI 0  /* x += D^-1 (b - A x), d_i = sum_j |a_ij| */
#define AMG_EIG_SMOOTH_CHEBYSHEV 1 /* degree-2 Chebyshev polynomial in D^-1 A on [cheb_lo, 1] (cheb_degree must be 2) */
#define AMG_EIG_SMOOTH_GAUSS_SEIDEL 2 /* multicolour Gauss-Seidel, the smoother of the paper's Section 4.1
                                        settings with each level's rows visited colour by colour (first-fit
                                        colouring of the graph of A_k in natural row order): a forward sweep
                                        before the coarse correction, a backward sweep after it */

#define AMG_EIG_PREC_FP64 0  /* everything in FP64 */
#define AMG_EIG_PREC_MIXED 1 /* V-cycle (smoothing, transfers) in FP32 with FP32
                                accumulation; residual, Rayleigh-Ritz and the
                                eigenvector block in FP64 */

#define AMG_EIG_COARSEN_RS 0   /* host setup: Ruge-Stueben first and second pass (Section 2) */
#define AMG_EIG_COARSEN_PMIS 1 /* device setup on the current device: strength, PMIS splitting
                                  with the parallel second pass,
                                  direct interpolation, transpose and Galerkin products per level
                                  (amg_eig_strength .. amg_eig_galerkin), levels copied back, and
                                  the coarsest eigen-decomposition by amg_eig_dense_sygv */

#define AMG_EIG_INIT_NESTED 0 /* Algorithm 3.2 start from the coarsest level */
#define AMG_EIG_INIT_RANDOM 1 /* seeded U(-1,1) block, then Rayleigh-Ritz */
#define AMG_EIG_INIT_USER 2   /* caller's device block, then Rayleigh-Ritz */

typedef struct {
    double theta;       /* strength threshold of (2.1); paper default 0.25 */
    int coarse_max;     /* stop coarsening once d_k <= coarse_max */
    int coarse_min;     /* never create a level smaller than this (0: auto) */
    int max_levels;     /* hierarchy depth limit */
    int qe;             /* block width (wanted + extra pairs); 0: guard rule
                           on the coarsest eigenvalues, rounded up to a
                           multiple of 4, then the width control of
                           amg_eig_progress() */
    double guard_gap;   /* guard rule: block may not end inside a cluster of
                           relative width < guard_gap */
    int smoother;       /* AMG_EIG_SMOOTH_* */
    int cheb_degree;    /* Chebyshev degree per smoothing step */
    double cheb_lo;     /* lower end of the Chebyshev interval in D^-1 A */
    int nu_pre, nu_post;/* smoothing steps before / after coarse correction */
    int precision;      /* AMG_EIG_PREC_* */
    double tol;         /* convergence: max_{j<=q} rho_j <= tol */
    int max_steps;      /* finest-level corrections in amg_eig_solve */
    int use_graph;      /* capture one correction step as a hipGraph (captured on the bound
                           stream at the first step after a bind, thread-local capture mode;
                           another thread that synchronises the device meanwhile, e.g. through
                           hipFree, invalidates the capture and the step returns AMG_EIG_EHIP) */
    int qe_max;         /* widest block the automatic width control may choose
                           (0: min(80, d_n, N - d_n)) */
    double shift;       /* Remark 3.1 shift sigma of the linear equation of Algorithm 3.1:
                           (A_k - sigma M_k) u~ = (lambda - sigma) M_k u, solved by the V-cycle
                           of A_k - sigma M_k on every level (coarsest: A_n - sigma M_n).  Must
                           lie below the smallest eigenvalue lambda_1, e.g. a lower bound the
                           continuous problem gives.  The library cannot verify that: setup
                           rejects (EINVAL) only a shift not below the coarsest level's smallest
                           eigenvalue, an upper bound of lambda_1 that can exceed it by a large
                           factor, or one that leaves a level's diagonal a_ii - sigma m_ii <= 0 */
    int coarsening;     /* AMG_EIG_COARSEN_*: how setup splits each level into C and F points */
    uint64_t coarsen_seed; /* PMIS only: seed of the random parts of the point weights (level k
                           draws SplitMix64 stream coarsen_seed + k, one uniform [0,1) per point) */
    int vcycles;        /* m of Algorithm 3.1, eq. (3.2): AMG cycles on the linear equation per
                           correction, each from the previous iterate (1 .. 16; paper default 1) */
} amg_eig_opts;

/* Paper defaults (Section 4.1: theta = 0.25, one V-cycle (m = 1) with one
 * pre- and one post-smoothing step, n_1 = n, p_k = 1 on coarse levels) plus the GPU
 * options: degree-2 Chebyshev smoothing on [0.25, 1] in D^-1 A (D the l1
 * diagonal), FP64, coarse_max 512, tol 1e-8, Ruge-Stueben coarsening on the
 * host. */
void amg_eig_opts_default(amg_eig_opts *o);

/* Host CSR, borrowed for the call: rowptr[n+1] (int64, rowptr[0] = 0,
 * non-decreasing), col[rowptr[n]] (int32, sorted, unique per row, in [0,n)),
 * val[rowptr[n]]. */
typedef struct {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
} amg_eig_csr;

typedef struct amg_eig_ctx amg_eig_ctx;

/* Build the AMG hierarchy on the host (Section 2) for the q smallest
 * eigenpairs of (A, M), plus the coarsest eigen-decomposition Z, Lambda_n with
 * Z^T M_n Z = I, Z^T A_n Z = Lambda_n.  No device call is made, except with
 * coarsening = AMG_EIG_COARSEN_PMIS: then the levels are formed on the current
 * device (on a non-blocking stream of its own with stream-ordered arrays, so
 * other streams are not synchronised) and copied back, and a HIP failure
 * there returns EHIP.
 * Errors: EINVAL (shapes, unsorted/duplicate/out-of-range columns, q < 1,
 * qe + d_n > n, nnz >= 2^31), ENOTSPD (a_ii <= 0, m_ii < 0, coarsest M_n or
 * A_n not positive definite), ENOMEM.  *out is NULL on error. */
int amg_eig_setup(const amg_eig_csr *A, const amg_eig_csr *M, int q, const amg_eig_opts *o,
                  amg_eig_ctx **out);

/* Galerkin coarse operators on the device (Section 2, eq. (2.5)):
 * C_A = P^T A P and C_M = P^T M P for one prolongation P (n x nc, eqs.
 * (2.2)-(2.4)), A and M given on one pattern.  Standalone: no context.
 * Inputs, all device memory, borrowed for the call:
 *   x_ptr[n+1] (int64), x_col[x_ptr[n]] (int32, in [0,n)), x_a, x_m: A and M
 *     on their shared CSR pattern;
 *   p_ptr[n+1], p_col (in [0,nc)), p_val: P in CSR;
 *   pt_ptr[nc+1], pt_col (in [0,n)), pt_val: P^T in CSR, each row's columns
 *     ascending.
 * Outputs, device memory owned by the caller: c_ptr[nc+1] (int64) always; when
 * the result fits (nnz <= cap), c_col[cap] (int32, ascending within a row)
 * and c_a[cap], c_m[cap] (FP64).  *nnz (host) receives the result's nonzero
 * count, so a call with cap = 0 and null c_col/c_a/c_m sizes the outputs.
 * Each output entry is accumulated in the order its contributions arise (left
 * factor's entries in storage order, then the right factor's), products and
 * sums rounded separately: the same bits as the host setup's coarse levels.
 * Column indices are not range-checked on the device.  Allocates and frees
 * temporary device memory (about 20 bytes per product of T = A P and of
 * P^T T) stream-ordered on the given stream (hipMallocAsync / hipFreeAsync,
 * so other streams are not synchronised) and waits for that stream
 * (hipStream_t, NULL for the null stream).  The same holds for the
 * temporaries of amg_eig_pmis, amg_eig_interpolation, amg_eig_transpose and
 * amg_eig_dense_sygv.
 * Column and value arrays may be null where they hold no entries (the
 * nonzero counts are read from the row pointers first).
 * Errors: EINVAL (negative sizes, a null row-pointer or c_ptr array, a null
 * array that holds entries, cap > 0 with null outputs),
 * EWORKSPACE (nnz > cap: c_ptr and *nnz written, nothing else), EHIP. */
int amg_eig_galerkin(int64_t n, int64_t nc, const int64_t *x_ptr, const int32_t *x_col, const double *x_a,
                     const double *x_m, const int64_t *p_ptr, const int32_t *p_col, const double *p_val,
                     const int64_t *pt_ptr, const int32_t *pt_col, const double *pt_val, int64_t *c_ptr,
                     int32_t *c_col, double *c_a, double *c_m, int64_t cap, int64_t *nnz, void *hip_stream);

/* Strong couplings on the device (Section 2, eq. (2.1)): strong[p] = 1 for an
 * entry p = (i, j) of A with j != i, a_ij < 0 and
 * -a_ij >= theta max_{k != i, a_ik < 0} (-a_ik), else 0 (a row without
 * negative off-diagonal entries has none).  Device arrays: x_ptr[n+1],
 * x_col, x_a as in amg_eig_galerkin; strong[x_ptr[n]] (out, caller-owned).
 * The same flags as the host setup's.  Asynchronous on the stream; allocates
 * nothing.  Errors: EINVAL (n < 0, theta outside [0, 1], a null array for
 * n > 0), EHIP. */
int amg_eig_strength(int64_t n, const int64_t *x_ptr, const int32_t *x_col, const double *x_a, double theta,
                     uint8_t *strong, void *hip_stream);

/* Parallel C/F splitting on the device, for the coarsening step of Section 2
 * (which the host setup does with the sequential Ruge-Stueben passes): PMIS,
 * the parallel modified independent set of De Sterck, Yang and Heys (2006), on
 * the strength graph of eq. (2.1).  Point i weighs |S_i^T| + rnd[i] (the
 * number of points depending strongly on it plus a caller-drawn number in
 * [0, 1)); points that no point depends on are F.  Each round every undecided
 * point heavier (weight, then larger index) than all its undecided neighbours
 * in the symmetrised strength graph becomes C, then every undecided point
 * depending strongly on a C point becomes F, until none is undecided.
 * With second_pass != 0 a parallel form of the Ruge-Stueben second pass
 * follows: while two F points i, j (j in S_i) share no C point that
 * influences both strongly, the heavier of each such pair becomes C.
 * Device inputs: x_ptr[n+1], x_col (a structurally symmetric pattern, columns
 * ascending within a row), strong[] from amg_eig_strength, rnd[n].  Output:
 * cf[n] (device, caller-owned; 1 = C, 0 = F); *rounds (host) the rounds
 * taken by the first pass (at most n).  Allocates and frees temporaries (1 byte
 * per entry, 12 per row), waits for the stream after each round.
 * Errors: EINVAL (n < 0, null arrays for n > 0; x_col and strong may be null
 * only when the pattern has no entries), EHIP. */
int amg_eig_pmis(int64_t n, const int64_t *x_ptr, const int32_t *x_col, const uint8_t *strong, const double *rnd,
                 int second_pass, int32_t *cf, int *rounds, void *hip_stream);

/* Direct interpolation on the device (Section 2, eqs. (2.2)-(2.4)) from a C/F
 * splitting: P (n x nc) injects the C points (coarse index = number of C
 * points before it) and gives an F point i the weights
 * w_ij = -alpha_i a_ij / a~_ii over its strong couplings to C points, with
 * alpha_i = (sum of negative off-diagonal a_ij) / (sum over those couplings)
 * and a~_ii = a_ii + (sum of positive off-diagonal a_ij); an F point whose
 * couplings sum to zero gets an empty row.  Device inputs: A as in
 * amg_eig_galerkin, strong[] from amg_eig_strength, cf[n] (1 = C, 0 = F).
 * Device outputs (caller-owned): p_ptr[n+1] always; p_col[cap] (int32,
 * ascending within a row), p_val[cap] when nnz <= cap.  *nnz and *nc (host)
 * receive P's nonzero count and column count.  The same bits as the host
 * setup's P.  Allocates and frees temporaries (16 bytes per row), waits for
 * the stream.  Errors: EINVAL (negative sizes, null required arrays; x_col,
 * x_a and strong may be null only when A has no entries),
 * EWORKSPACE (nnz > cap: p_ptr, *nnz and *nc written), EHIP. */
int amg_eig_interpolation(int64_t n, const int64_t *x_ptr, const int32_t *x_col, const double *x_a,
                          const uint8_t *strong, const int32_t *cf, int64_t *p_ptr, int32_t *p_col, double *p_val,
                          int64_t cap, int64_t *nnz, int64_t *nc, void *hip_stream);

/* Transpose of an nr x nc CSR matrix on the device (P^T for the restriction
 * and the Galerkin products of eq. (2.5)): pt_ptr[nc+1], pt_col[p_ptr[nr]]
 * and pt_val[p_ptr[nr]] (caller-owned), each row's columns ascending.  Columns
 * of P must lie in [0, nc) and be unique within a row.  Allocates and frees a
 * counter array (8 bytes per column), waits for the stream.
 * Errors: EINVAL (negative sizes, null row pointers, a null column or value
 * array while P has entries), EHIP. */
int amg_eig_transpose(int64_t nr, int64_t nc, const int64_t *p_ptr, const int32_t *p_col, const double *p_val,
                      int64_t *pt_ptr, int32_t *pt_col, double *pt_val, void *hip_stream);

/* Dense symmetric-definite eigen-decomposition on the device, for the
 * coarsest level of the hierarchy (the coarsest eigen-solve that starts
 * Algorithm 3.2 and gives the exact coarsest solve): A z = lambda M z with
 * Z^T M Z = I, eigenvalues ascending.  Cholesky M = L L^T, cyclic Jacobi on
 * L^-1 A L^-T in the parallel round-robin ordering until the off-diagonal
 * Frobenius norm is below n * 2^-52 of the whole (at most 40 sweeps), then
 * Z = L^-T V.  Device arrays, row-major: A[n*n] and M[n*n] symmetric (read
 * only), lam[n] and Z[n*n] (column j = eigenvector j) written.  *sweeps (host,
 * may be NULL) receives the Jacobi sweeps.  Allocates and frees three n x n
 * temporaries, waits for the stream; thousands of small launches (for setup,
 * not for a solve loop).  Errors: EINVAL (n < 1 or n > 4096, null arrays),
 * ENOTSPD (a Cholesky pivot of M not positive), EBREAKDOWN (no convergence in
 * 40 sweeps), EHIP. */
int amg_eig_dense_sygv(int64_t n, const double *A, const double *M, double *lam, double *Z, int *sweeps,
                       void *hip_stream);

/* Device bytes needed by amg_eig_bind(). */
int amg_eig_footprint(const amg_eig_ctx *c, size_t *device_bytes);

/* Hand the context a caller-owned device workspace (>= footprint bytes,
 * 256-byte aligned) and a HIP stream (hipStream_t, may be NULL for the null
 * stream), then upload the hierarchy with asynchronous copies on that stream.
 * The workspace must stay valid until amg_eig_destroy() or the next bind.
 * Errors: EWORKSPACE, EHIP. */
int amg_eig_bind(amg_eig_ctx *c, void *dev_workspace, size_t bytes, void *hip_stream);

/* amg_eig_bind without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops or harnesses that
 * forbid hipMalloc): the workspace is a static device array inside the library,
 * 64 MiB per device (*static_bytes, when non-NULL, receives the size), held by
 * each device the library runs on until the process ends.  Otherwise as
 * amg_eig_bind on the current device and the given stream; no device memory is
 * allocated or freed.  One context per device holds the array at a time:
 * binding another context to it waits for the previous holder's stream and
 * leaves that context unbound (its later calls fail with ESTATE until it is
 * bound again).  Work of two contexts on the array must not overlap: calls
 * that overlap on one device race.  A widening of the block (see
 * amg_eig_progress) stays inside the array when it fits.
 * Errors: EWORKSPACE (footprint above the array's size), EHIP. */
int amg_eig_bind_static(amg_eig_ctx *c, void *hip_stream, size_t *static_bytes);

/* Start the iteration on the finest level (asynchronous).
 * NESTED: Algorithm 3.2 (coarsest eigenvectors, prolongation, one correction
 *         per intermediate level).
 * RANDOM: U = seeded U(-1,1) block (SplitMix64: element (i, j) is output
 *         j*N + i of the stream seeded with `seed`), then Rayleigh-Ritz on the
 *         coarsest space augmented with span U.
 * USER:   U_dev (device, N x ldu row-major doubles, first qe columns used),
 *         then Rayleigh-Ritz as for RANDOM.
 * Errors: ESTATE (not bound), EINVAL. */
int amg_eig_init(amg_eig_ctx *c, int mode, uint64_t seed, const double *U_dev, int64_t ldu);

/* Enqueue `steps` correction steps (Algorithm 3.1 on the finest level).
 * Each step first evaluates the residuals of the current iterate; once the
 * convergence test holds, later steps do no work (device-side flag).
 * Asynchronous. Errors: ESTATE. */
int amg_eig_correct(amg_eig_ctx *c, int steps);

/* Wait for the bound stream and report the current Ritz values theta[qe],
 * relative residuals rho[qe] (of the iterate before the last step's update),
 * the number of corrections done and whether the test holds.  Any output
 * pointer may be NULL.  rho_j = ||A u_j - theta_j M u_j||_2 / (theta_j ||M u_j||_2),
 * the stopping test of the driver (Algorithm 3.2 with the residual of (3.1)).
 *
 * Block width control (contexts set up with opts.qe = 0, whose width comes
 * from the guard rule on the coarsest eigenvalues): the coarsest level may
 * not resolve a cluster of eigenvalues, and a block that ends inside one
 * stalls.  When, after at least 16 corrections since the start, the smallest
 * max_{j<=q} rho_j reported over the last 10 corrections is not below half
 * the smallest reported before them, while the Ritz values past the q-th show no relative gap >=
 * guard_gap inside the block, the width is doubled (at most qe_max) - the
 * paper's remedy of computing extra eigenpairs (Section 4.5) - and WIDENED is
 * returned: the iterate is discarded, and amg_eig_init() must follow, after a
 * bind of a workspace of amg_eig_footprint() bytes if the new width does not
 * fit the bound one (the context is then unbound).  Once a widened block has
 * converged, the next start takes the narrowest multiple of 4, w >= q, with
 * theta_{w+1} >= 1.25 theta_q (so the wanted pairs keep contracting by about
 * (theta_q / theta_{w+1})^2 <= 0.64 per correction), if the wide block holds
 * one; otherwise the wide width stays.  amg_eig_info() reports the width in
 * effect.
 * Errors: ESTATE (not bound), EBREAKDOWN, EHIP. */
int amg_eig_progress(amg_eig_ctx *c, double *theta, double *rho, int *steps, int *converged);

/* Driver of Algorithm 3.2: init(NESTED) unless already initialised, then
 * correction steps (Algorithm 3.1) until max_{j<=q} rho_j <= tol or max_steps
 * corrections; copies the q wanted eigenvalues to lambda_host[q] and
 * eigenvectors to U_dev (device, N x ldu row-major, ldu >= q) when non-NULL.
 * A solve of an iterate that an earlier call left converged re-tests it
 * against this tol.  When the block width control widens the block inside the
 * bound workspace, the solve restarts with the wider block by itself; when
 * the wider block needs a larger workspace it returns WIDENED (bind, then call
 * again).  Returns NOT_CONVERGED (with the best-so-far pairs) if the step
 * limit is reached. */
int amg_eig_solve(amg_eig_ctx *c, double tol, int max_steps, double *lambda_host, double *U_dev,
                  int64_t ldu);

/* Batching form of the correction step (Algorithm 3.1): enqueue `steps`
 * correction steps for each of n initialised contexts (requests of uneven N;
 * each context keeps its own hierarchy and block), step by step across the
 * members.  hip_stream NULL: each member on its own bound stream, so the
 * kernels of different members overlap; else every member must be bound to
 * that stream.  Errors: EINVAL, ESTATE, EHIP. */
int amg_eig_correct_batch(amg_eig_ctx *const *cs, int n, int steps, void *hip_stream);

/* Batching form of the correction (Algorithm 3.1, steps of eq (3.3)): enqueue
 * `steps` correction steps for each of n initialised contexts, with the small
 * eigenproblem of every member solved jointly.  Per step, each member's
 * residual, V-cycle, dual SpMM, Gram product and restriction chain run on its
 * own stream; the lead stream (that of cs[0]) then waits for all of them and,
 * over a device-side table of per-request descriptors (members of different
 * N, d_n and qe side by side, up to 64 per launch), forms the coarse products
 * Z^T B (a work list of 16 x 16 tiles over all members), solves the n small
 * pencils in three launches (one workgroup per member for the pencil and the
 * Ritz polish, qe workgroups per member for the eigenvalues) and forms
 * Y = Z X_c; the members' streams wait for that and recombine.  Results are bitwise those of amg_eig_correct on each member.
 * A member whose options ask for graphs (and whose site timing is off)
 * replays its two own parts from graphs captured on its first joint step; the
 * joint launches are eager.  Members may share streams.  A context may appear
 * once.  Errors: EINVAL (NULL, duplicate), ESTATE (not initialised),
 * EHIP. */
int amg_eig_correct_batch_joint(amg_eig_ctx *const *cs, int n, int steps);

/* Nested start (Algorithm 3.2) of n bound contexts together: every member's
 * coarse-level corrections run on its own stream with their small
 * eigenproblems (eq (3.3)) solved jointly per level, as in
 * amg_eig_correct_batch_joint; a member with fewer levels joins at the later
 * rounds, so all reach the finest level together.  Results are bitwise those
 * of amg_eig_init(NESTED) on each member.  Eager launches.  Errors: EINVAL
 * (NULL, duplicate), ESTATE (not bound), EHIP. */
int amg_eig_init_batch_joint(amg_eig_ctx *const *cs, int n);

/* Sizes: block width qe, number of levels, and the dimension of each level
 * (dims[nlev], may be NULL). */
int amg_eig_info(const amg_eig_ctx *c, int *qe, int *nlevels, int64_t *dims);

/* Host copies of the hierarchy, for inspection and tests: the C/F splitting
 * of level k (cf[d_k], 1 = C), the level's A and M on the shared pattern
 * (rowptr[d_k+1], col[nnz], a[nnz], m[nnz]; pass NULL to query nnz), the
 * prolongation P_k (d_k x d_{k+1}), and the coarsest eigenvalues lam[d_n]. */
int amg_eig_level_matrix(const amg_eig_ctx *c, int level, int64_t *nnz, int64_t *rowptr, int32_t *col,
                         double *a, double *m);
int amg_eig_level_prolongation(const amg_eig_ctx *c, int level, int64_t *nnz, int64_t *rowptr,
                               int32_t *col, double *p);
int amg_eig_level_splitting(const amg_eig_ctx *c, int level, int32_t *cf);
/* Multicolour Gauss-Seidel only: the colour of each row of level k < nlevels-1
 * (colour[d_k], may be NULL) and the number of colours.  EINVAL for another
 * smoother or the coarsest level. */
int amg_eig_level_colouring(const amg_eig_ctx *c, int level, int32_t *colour, int *ncolours);
int amg_eig_coarse_eigenvalues(const amg_eig_ctx *c, double *lam);

/* Device pointer to the current FP64 iterate (N x ld row-major) and its ld. */
int amg_eig_iterate(const amg_eig_ctx *c, const double **U_dev, int64_t *ld);

/* Kernel sites on the finest level, for per-kernel timing. */
#define AMG_EIG_SITE_RESIDUAL 0   /* outer residual R = M U Theta - A U (FP64 dual SpMM) */
#define AMG_EIG_SITE_PRESMOOTH 1  /* zero-guess pre-smoothing (l1-Jacobi: fused with the residual) */
#define AMG_EIG_SITE_POSTSMOOTH 2 /* last post-smoothing product, fused with V = U + delta */
#define AMG_EIG_SITE_DUALSPMM 3   /* W = [A V | M V] */
#define AMG_EIG_SITE_GRAM 4       /* V^T [A V | M V] (counted in flops) */
#define AMG_EIG_SITE_RESTRICT 5   /* FP64 restriction of W, level 1 -> 2 */
#define AMG_EIG_SITE_FINAL 6      /* U = P Y + V X_v */
#define AMG_EIG_SITE_SMALL 7      /* coarse-space Rayleigh-Ritz kernels (all) */
#define AMG_EIG_SITE_COUNT 8

/* Enable (1) or stop (0) HIP-event timing of the finest-level kernel sites
 * for eagerly launched steps (steps replayed from a captured graph are not
 * timed; with use_graph and timing on, the second step of every enqueued
 * chunk of three or more steps runs eagerly and is timed).  A site of one
 * kernel (all but GRAM and SMALL) passes its events to that kernel's launch,
 * which records them at the kernel's own start and end; GRAM and SMALL are
 * bracketed by events recorded on the stream.  Enabling resets the
 * counters. */
int amg_eig_timing(amg_eig_ctx *c, int enable);

/* Waits for the bound stream, then reports for one site: the algorithmic
 * bytes of one launch (each operand read once, each result written once;
 * flops for the Gram site), the summed event time in ms and the number of
 * timed launches. */
int amg_eig_site_stats(amg_eig_ctx *c, int site, double *alg_bytes, double *ms_total, int64_t *launches);

/* Launch shape of the row kernels (batching form: per-level choice by a
 * timing autotuner).  A row kernel gives each row of its block width / cpt
 * lanes, every lane cpt consecutive columns; cpt is 2, 4 or 8, must divide the
 * width and leave at most 64 lanes per row, and 0 selects the built-in rule
 * (fewest idle lanes, then fewest columns per lane).  Each vector entry is the
 * same ordered sum for every cpt, so the iterates do not depend on the choice;
 * only the residual norms rho_j, summed over rows in an order that follows the
 * launch shape, can differ in the last bits.
 * Kinds, by the rows a kernel produces on `level`:
 *   VCYCLE     smoothing, level residual and transfers of the V-cycle, in the
 *              working precision, width q_e (levels 0 .. nlev-2);
 *   FP64       outer residual, dual SpMM [A V | M V], prolongation of the
 *              coarse part of the Ritz vectors and the final update, width q_e
 *              (0 .. nlev-2);
 *   FP64_WIDE  restriction of [A V | M V], width 2 q_e (1 .. nlev-2).
 * set_cpt: EINVAL for an invalid kind, level or cpt; drops a captured step.
 * get_cpt: the cpt in effect (the built-in rule's when none is set). */
#define AMG_EIG_TUNE_VCYCLE 0
#define AMG_EIG_TUNE_FP64 1
#define AMG_EIG_TUNE_FP64_WIDE 2
int amg_eig_set_cpt(amg_eig_ctx *c, int kind, int level, int cpt);
int amg_eig_get_cpt(const amg_eig_ctx *c, int kind, int level, int *cpt);

/* Time the row kernels of one kind on one level with the given cpt (0: the
 * built-in rule): one untimed pass, then `reps` passes between two HIP events
 * on the bound stream; waits for them and returns the microseconds per pass.
 * The kernels work on the context's scratch (never on the iterate U) and the
 * solve state is cleared, so init() must follow before the next correction.
 * Errors: EINVAL (kind, level, cpt, reps < 1), ESTATE (not bound), EHIP. */
int amg_eig_tune_time(amg_eig_ctx *c, int kind, int level, int cpt, int reps, double *us_per_rep);

void amg_eig_destroy(amg_eig_ctx *c);
const char *amg_eig_strerror(int code);
const char *amg_eig_last_error(const amg_eig_ctx *c);

#ifdef __cplusplus
}
#endif
#endif
