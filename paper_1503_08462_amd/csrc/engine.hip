// Context, device workspace plan, upload, and the enqueue order of one
// correction step (Algorithm 3.1) and of the driver (Algorithm 3.2); the C ABI
// of amg_eig.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <array>
#include <vector>

#include "amg_eig.h"
#include "internal.h"
#include "kernels.h"

using namespace amgeig;

namespace {

struct DevLevel {
    int64_t n = 0;
    int32_t *u_ptr = nullptr, *u_col = nullptr;
    double *u_a = nullptr, *u_m = nullptr;
    int32_t *v_ptr = nullptr, *v_col = nullptr;
    void *v_val = nullptr, *dinv = nullptr;
    void *v_vs = nullptr;  // a_ij / d_j on the V-cycle pattern (zero-guess pre-smoothing)
    int32_t *p_ptr = nullptr, *p_col = nullptr, *pt_ptr = nullptr, *pt_col = nullptr;
    void *p_val = nullptr, *pt_val = nullptr;
    double *p64 = nullptr, *pt64 = nullptr;
    void *b = nullptr, *r = nullptr, *x = nullptr, *t = nullptr;  // t: Chebyshev scratch
    double *cw = nullptr;
    // multicolour Gauss-Seidel: rows in colour order, av's rows in that order
    // without the diagonal (all entries; entries of smaller colours), a_ii
    int32_t *gs_rows = nullptr, *gs_ptr = nullptr, *gs_col = nullptr, *gs_lptr = nullptr, *gs_lcol = nullptr;
    void *gs_val = nullptr, *gs_lval = nullptr, *gs_diag = nullptr;
    int cpt[3] = {0, 0, 0};  // columns per lane of the row kernels on this level's rows, by tuning kind (0: built-in)
};

// Bump allocator over the caller's workspace; with base == nullptr it only sizes.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(char *b) : base(b) {}
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace

struct amg_eig_ctx {
    Hierarchy H;
    amg_eig_opts o{};
    int q = 0, qe = 0, ld = 0;
    bool mixed = false;
    std::string err;
    // device state
    bool bound = false, initialised = false;
    hipStream_t stream = nullptr;
    size_t need = 0;
    std::vector<DevLevel> dl;
    double *U = nullptr, *V = nullptr, *W = nullptr;
    double *Z = nullptr, *Zt = nullptr, *lam = nullptr, *Yn = nullptr;
    void *Ainv = nullptr;
    // dense coarse tail: from level `tail` down, the V-cycle is applied as its
    // matrix Bt (built on the device at bind), and the coarse basis as
    // Zk = I_tail^n Z (n_tail x d_n) with its transpose Zkt
    int tail = -1;
    std::vector<double> Zk_host;
    void *Bt = nullptr;
    double *Zk = nullptr, *Zkt = nullptr;
    double *theta = nullptr, *rho = nullptr, *part_res = nullptr, *part_gram = nullptr;
    unsigned *counters = nullptr;
    int *status = nullptr;
    SmallWork sw;
    // the small-eigensolver descriptor of this request (device copy for the
    // batched launches) and its LDS sizes; an event for joining batch streams
    SmallItem *item_dev = nullptr;
    SmallItem item_host;
    SmallLds small_lds;
    hipEvent_t join_ev = nullptr;
    // the bound workspace, kept for changes of the block width inside it
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int static_dev = -1;  // device whose static workspace this context holds (amg_eig_bind_static)
    // block width control of the solve driver (automatic width, opts.qe = 0):
    // the width may be raised when the iteration stalls with the block ending
    // inside a cluster, and lowered for later starts once a widened block
    // has converged and its Ritz values show a gap earlier
    bool width_auto = false, width_decided = true, widened = false;
    int qe_cap = 0;   // widest block the control may choose
    int qe_next = 0;  // > 0: block width to take at the next start
    std::vector<std::pair<int, double>> hist;  // (finest corrections, max_{j<q} rho_j) per progress call
    // host staging kept alive until the upload completes
    std::vector<std::vector<char>> staging;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // the two per-request parts of a joint batch step, captured separately
    hipGraph_t part_graph[2] = {nullptr, nullptr};
    hipGraphExec_t part_exec[2] = {nullptr, nullptr};
    // tuned columns per lane by (level, kind); copied into dl at bind
    std::vector<std::array<int, 3>> cpt_tab;
    // optional per-site event timing of finest-level kernels (eager launches)
    bool timing = false;
    struct Site {
        std::vector<hipEvent_t> ev;  // start/stop pairs
        size_t used = 0;
        double ms = 0.0;
        int64_t launches = 0;
    } sites[AMG_EIG_SITE_COUNT];
};

namespace {

int fail(amg_eig_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(ctx, AMG_EIG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------ dense tail
// The first level t >= 1 with at most kTailRows unknowns and at least one level
// below it becomes the dense tail; Zk = P_t P_{t+1} ... P_{n-1} Z on the host.
#ifndef AMG_EIG_TAIL_ROWS
#define AMG_EIG_TAIL_ROWS 3000
#endif
constexpr int64_t kTailRows = AMG_EIG_TAIL_ROWS;

void choose_tail(amg_eig_ctx *c) {
    const Hierarchy &H = c->H;
    const int L = (int)H.lv.size(), dn = H.dn;
    c->tail = -1;
    c->Zk_host.clear();
    for (int l = 1; l <= L - 2; ++l)
        if (H.lv[l].n <= kTailRows) {
            c->tail = l;
            break;
        }
    if (c->tail < 0) return;
    std::vector<double> Y = H.Z;  // level L-1, d_n x d_n
    for (int l = L - 2; l >= c->tail; --l) {
        const Csr &P = H.lv[l].P;  // n_l x n_{l+1}
        std::vector<double> X((size_t)H.lv[l].n * dn, 0.0);
        for (int64_t i = 0; i < H.lv[l].n; ++i)
            for (int64_t p = P.ptr[i]; p < P.ptr[i + 1]; ++p) {
                const double w = P.val[p];
                const double *yr = &Y[(size_t)P.col[p] * dn];
                double *xr = &X[(size_t)i * dn];
                for (int j = 0; j < dn; ++j) xr[j] += w * yr[j];
            }
        Y.swap(X);
    }
    c->Zk_host.swap(Y);
}

// ------------------------------------------------------------ memory plan
// Everything whose size does not depend on the block width (matrices, the
// coarse basis, the dense tail operator, Ritz values and residuals sized for
// the widest block, flags) comes first; the blocks follow.  A change of the
// block width inside the same workspace (width control of the solve driver)
// therefore keeps every uploaded array where it is.
void plan(amg_eig_ctx *c, char *base) {
    Carver cv(base);
    const Hierarchy &H = c->H;
    const int L = (int)H.lv.size(), ld = c->ld, dn = H.dn;
    const size_t sT = c->mixed ? sizeof(float) : sizeof(double);
    const int64_t N = H.lv[0].n;
    c->dl.assign(L, DevLevel());
    if ((int)c->cpt_tab.size() != L) c->cpt_tab.assign(L, std::array<int, 3>{0, 0, 0});
    for (int l = 0; l < L; ++l)
        for (int k = 0; k < 3; ++k) c->dl[l].cpt[k] = c->cpt_tab[l][k];
    for (int l = 0; l < L; ++l) {
        const Level &lv = H.lv[l];
        DevLevel &d = c->dl[l];
        d.n = lv.n;
        d.u_ptr = cv.take<int32_t>(lv.n + 1);
        d.u_col = cv.take<int32_t>(lv.col.size());
        d.u_a = cv.take<double>(lv.col.size());
        d.u_m = cv.take<double>(lv.col.size());
        if (l < L - 1) {
            d.v_ptr = cv.take<int32_t>(lv.n + 1);
            d.v_col = cv.take<int32_t>(lv.av.col.size());
            d.v_val = cv.take<char>(lv.av.col.size() * sT);
            d.v_vs = cv.take<char>(lv.av.col.size() * sT);
            d.dinv = cv.take<char>(lv.n * sT);
            d.p_ptr = cv.take<int32_t>(lv.n + 1);
            d.p_col = cv.take<int32_t>(lv.P.col.size());
            d.p_val = cv.take<char>(lv.P.col.size() * sT);
            d.p64 = cv.take<double>(lv.P.col.size());
            d.pt_ptr = cv.take<int32_t>(lv.Pt.nr + 1);
            d.pt_col = cv.take<int32_t>(lv.Pt.col.size());
            d.pt_val = cv.take<char>(lv.Pt.col.size() * sT);
            d.pt64 = cv.take<double>(lv.Pt.col.size());
            if (c->o.smoother == AMG_EIG_SMOOTH_GAUSS_SEIDEL) {
                d.gs_rows = cv.take<int32_t>(lv.n);
                d.gs_ptr = cv.take<int32_t>(lv.n + 1);
                d.gs_col = cv.take<int32_t>(lv.gs_all.col.size());
                d.gs_val = cv.take<char>(lv.gs_all.col.size() * sT);
                d.gs_lptr = cv.take<int32_t>(lv.n + 1);
                d.gs_lcol = cv.take<int32_t>(lv.gs_lo.col.size());
                d.gs_lval = cv.take<char>(lv.gs_lo.col.size() * sT);
                d.gs_diag = cv.take<char>(lv.n * sT);
            }
        }
    }
    c->Z = cv.take<double>((size_t)dn * dn);
    c->Zt = cv.take<double>((size_t)dn * dn);
    c->lam = cv.take<double>(dn);
    c->Ainv = cv.take<char>((size_t)dn * dn * sT);
    c->theta = cv.take<double>(kMaxWidth);
    c->rho = cv.take<double>(kMaxWidth);
    c->counters = cv.take<unsigned>(16);
    if (c->tail >= 0) {
        const int nt = (int)H.lv[c->tail].n;
        c->Bt = cv.take<char>((size_t)nt * nt * sT);
        c->Zk = cv.take<double>((size_t)nt * dn);
        c->Zkt = cv.take<double>((size_t)nt * dn);
    }
    c->status = cv.take<int>(ST_COUNT);
    c->item_dev = cv.take<SmallItem>(1);
#if AMG_EIG_SMALL_STATS
    int *diag = cv.take<int>(5 * kMaxWidth + 8);
#endif
    // ---- blocks (width ld)
    for (int l = 0; l < L; ++l) {
        const Level &lv = H.lv[l];
        DevLevel &d = c->dl[l];
        d.b = cv.take<char>((size_t)lv.n * ld * sT);
        d.r = cv.take<char>((size_t)lv.n * ld * sT);
        d.x = cv.take<char>((size_t)lv.n * ld * sT);
        if (c->o.smoother == AMG_EIG_SMOOTH_CHEBYSHEV && l < L - 1) d.t = cv.take<char>((size_t)lv.n * ld * sT);
        if (l >= 1) d.cw = cv.take<double>((size_t)lv.n * 2 * ld);
    }
    c->U = cv.take<double>((size_t)N * ld);
    c->V = cv.take<double>((size_t)N * ld);
    c->W = cv.take<double>((size_t)N * 2 * ld);
    c->Yn = cv.take<double>((size_t)dn * ld);
    int64_t maxn = 0;
    for (const Level &lv : H.lv) maxn = std::max(maxn, lv.n);
    c->part_res = cv.take<double>(((size_t)residual_blocks_max(maxn, ld) + 1) * 2 * ld);
    c->part_gram = cv.take<double>((size_t)gram_blocks(maxn, ld) * 2 * ld * ld);
    SmallWork &w = c->sw;
    w.dn = dn;
    w.ld = ld;
    w.lam = c->lam;
    w.FG = cv.take<double>((size_t)dn * 2 * ld);
    w.GAGM = cv.take<double>((size_t)2 * ld * ld);
    w.P3 = cv.take<double>((size_t)3 * ld * ld);
    w.Ct = cv.take<double>((size_t)dn * ld);
    w.Dt = cv.take<double>((size_t)ld * ld);
    w.L1 = cv.take<double>((size_t)ld * ld);
    w.Li = cv.take<double>((size_t)ld * ld);
    w.perm = cv.take<int>(ld);
    w.X = cv.take<double>((size_t)(dn + ld) * ld);
    w.HX = cv.take<double>((size_t)(dn + ld) * ld);
    w.Xr = cv.take<double>((size_t)(dn + ld) * ld);
    w.theta = cv.take<double>(ld);
    w.Xc = cv.take<double>((size_t)dn * ld);
    w.Xv = cv.take<double>((size_t)ld * ld);
    w.status = c->status;
#if AMG_EIG_SMALL_STATS
    w.diag = diag;
#else
    w.diag = nullptr;
#endif
    c->need = cv.off + 256;
}

template <typename T>
void *stage(amg_eig_ctx *c, const std::vector<T> &v) {
    c->staging.emplace_back(v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(c->staging.back().data(), v.data(), v.size() * sizeof(T));
    return c->staging.back().data();
}

template <typename T>
std::vector<T> narrow_ptr(const std::vector<int64_t> &p) {
    std::vector<T> r(p.size());
    for (size_t i = 0; i < p.size(); ++i) r[i] = (T)p[i];
    return r;
}

std::vector<double> transposed(const std::vector<double> &a, int n) {  // n x n row-major
    std::vector<double> t(a.size());
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) t[(size_t)j * n + i] = a[(size_t)i * n + j];
    return t;
}

template <typename T>
std::vector<T> convert(const std::vector<double> &v) {
    std::vector<T> r(v.size());
    for (size_t i = 0; i < v.size(); ++i) r[i] = (T)v[i];
    return r;
}

int put(amg_eig_ctx *c, void *dst, const void *host, size_t bytes) {
    if (bytes == 0) return AMG_EIG_OK;
    HIPCHK(c, hipMemcpyAsync(dst, host, bytes, hipMemcpyHostToDevice, c->stream));
    return AMG_EIG_OK;
}

template <typename T>
int upload_vec(amg_eig_ctx *c, void *dst, const std::vector<T> &v) {
    void *h = stage(c, v);
    return put(c, dst, h, v.size() * sizeof(T));
}

template <typename T>
int upload_levels(amg_eig_ctx *c) {
    const Hierarchy &H = c->H;
    const int L = (int)H.lv.size();
    int rc = 0;
    for (int l = 0; l < L && !rc; ++l) {
        const Level &lv = H.lv[l];
        DevLevel &d = c->dl[l];
        rc |= upload_vec(c, d.u_ptr, narrow_ptr<int32_t>(lv.ptr));
        rc |= upload_vec(c, d.u_col, lv.col);
        rc |= upload_vec(c, d.u_a, lv.a);
        rc |= upload_vec(c, d.u_m, lv.m);
        if (l < L - 1) {
            rc |= upload_vec(c, d.v_ptr, narrow_ptr<int32_t>(lv.av.ptr));
            rc |= upload_vec(c, d.v_col, lv.av.col);
            rc |= upload_vec(c, d.v_val, convert<T>(lv.av.val));
            std::vector<double> dinv(lv.n);
            for (int64_t i = 0; i < lv.n; ++i) dinv[i] = 1.0 / lv.l1[i];
            const std::vector<T> dinv_t = convert<T>(dinv), val_t = convert<T>(lv.av.val);
            // the product the pre-smoother would form per neighbour, in the working precision
            std::vector<T> vs(val_t.size());
            for (size_t p = 0; p < vs.size(); ++p) vs[p] = val_t[p] * dinv_t[lv.av.col[p]];
            rc |= upload_vec(c, d.v_vs, vs);
            rc |= upload_vec(c, d.dinv, dinv_t);
            rc |= upload_vec(c, d.p_ptr, narrow_ptr<int32_t>(lv.P.ptr));
            rc |= upload_vec(c, d.p_col, lv.P.col);
            rc |= upload_vec(c, d.p_val, convert<T>(lv.P.val));
            rc |= upload_vec(c, d.p64, lv.P.val);
            rc |= upload_vec(c, d.pt_ptr, narrow_ptr<int32_t>(lv.Pt.ptr));
            rc |= upload_vec(c, d.pt_col, lv.Pt.col);
            rc |= upload_vec(c, d.pt_val, convert<T>(lv.Pt.val));
            rc |= upload_vec(c, d.pt64, lv.Pt.val);
            if (c->o.smoother == AMG_EIG_SMOOTH_GAUSS_SEIDEL) {
                rc |= upload_vec(c, d.gs_rows, lv.corder);
                rc |= upload_vec(c, d.gs_ptr, narrow_ptr<int32_t>(lv.gs_all.ptr));
                rc |= upload_vec(c, d.gs_col, lv.gs_all.col);
                rc |= upload_vec(c, d.gs_val, convert<T>(lv.gs_all.val));
                rc |= upload_vec(c, d.gs_lptr, narrow_ptr<int32_t>(lv.gs_lo.ptr));
                rc |= upload_vec(c, d.gs_lcol, lv.gs_lo.col);
                rc |= upload_vec(c, d.gs_lval, convert<T>(lv.gs_lo.val));
                rc |= upload_vec(c, d.gs_diag, convert<T>(lv.gs_diag));
            }
        }
    }
    const int dn = H.dn;
    rc |= upload_vec(c, c->Z, H.Z);
    rc |= upload_vec(c, c->Zt, transposed(H.Z, H.dn));
    rc |= upload_vec(c, c->lam, H.lam);
    rc |= upload_vec(c, c->Ainv, convert<T>(transposed(H.Ainv, H.dn)));  // used as (A^-1)^T^T
    if (c->tail >= 0) {
        const int64_t nt = H.lv[c->tail].n;
        rc |= upload_vec(c, c->Zk, c->Zk_host);
        std::vector<double> zt((size_t)nt * dn);
        for (int64_t i = 0; i < nt; ++i)
            for (int j = 0; j < dn; ++j) zt[(size_t)j * nt + i] = c->Zk_host[(size_t)i * dn + j];
        rc |= upload_vec(c, c->Zkt, zt);
    }
    return rc ? AMG_EIG_EHIP : AMG_EIG_OK;
}

// ---------------------------------------------------------- site timing
// Sites that wrap one kernel launch (exact) hand a start/stop pair to that
// launch, which records them at the kernel's own start and end; the others
// record stream events around their launches.
struct SiteScope {
    amg_eig_ctx *c;
    int site;
    bool on;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SiteScope(amg_eig_ctx *ctx, int s, int level, bool exact = false)
        : c(ctx), site(s), on(ctx->timing && level == 0) {
        if (!on) return;
        if (!exact) {
            record();
            return;
        }
        e0 = next();
        e1 = e0 ? next() : nullptr;
        if (!e1) {  // no events left: the site is not timed
            on = false;
            if (e0) c->sites[site].used -= 1;
            e0 = nullptr;
            return;
        }
        set_launch_events(e0, e1);
    }
    ~SiteScope() {
        if (!on) return;
        if (!e0) {
            record();
        } else if (launch_events_pending()) {  // the launch did not take them
            clear_launch_events();
            (void)hipEventRecord(e0, c->stream);
            (void)hipEventRecord(e1, c->stream);
        }
    }
    hipEvent_t next() {
        auto &st = c->sites[site];
        if (st.used == st.ev.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            st.ev.push_back(e);
        }
        return st.ev[st.used++];
    }
    void record() {
        hipEvent_t e = next();
        if (!e) {
            on = false;
            return;
        }
        (void)hipEventRecord(e, c->stream);
    }
};

// one event of a start/stop pair, for a site that spans several functions
void site_mark(amg_eig_ctx *c, int site, int level) {
    if (c->timing && level == 0) SiteScope(c, site, -1).record();
}

void collect_sites(amg_eig_ctx *c) {
    for (auto &st : c->sites) {
        for (size_t i = 0; i + 1 < st.used; i += 2) {
            float ms = 0.f;
            if (hipEventSynchronize(st.ev[i + 1]) == hipSuccess && hipEventElapsedTime(&ms, st.ev[i], st.ev[i + 1]) == hipSuccess) {
                st.ms += ms;
                st.launches += 1;
            }
        }
        st.used = 0;
    }
}

// Algorithmic bytes (or flops for the Gram site) of one launch on the finest
// level: every operand read once, every result written once.
double site_bytes(const amg_eig_ctx *c, int site) {
    const Level &L0 = c->H.lv[0];
    const double n = (double)L0.n, ld = c->ld, sT = c->mixed ? 4.0 : 8.0;
    const double ptr = 4.0 * (n + 1), nnz_u = (double)L0.col.size(), nnz_v = (double)L0.av.col.size();
    const double n1 = c->H.lv.size() > 1 ? (double)c->H.lv[1].n : 0.0;
    const double nnz_p = (double)L0.P.col.size();
    switch (site) {
    case AMG_EIG_SITE_RESIDUAL: return ptr + nnz_u * 20.0 + 8.0 * n * ld + sT * n * ld;
    case AMG_EIG_SITE_PRESMOOTH:
        if (c->o.smoother == AMG_EIG_SMOOTH_GAUSS_SEIDEL)  // b, x once; the smaller-colour entries; rows, a_ii
            return ptr + (double)L0.gs_lo.col.size() * (4.0 + sT) + (4.0 + sT) * n + 2.0 * sT * n * ld;
        return ptr + nnz_v * (4.0 + sT) + sT * n + 2.0 * sT * n * ld;
    case AMG_EIG_SITE_POSTSMOOTH:
        if (c->o.smoother == AMG_EIG_SMOOTH_GAUSS_SEIDEL)  // b, y read and written; U -> V; entries; rows, a_ii
            return ptr + (double)L0.gs_all.col.size() * (4.0 + sT) + (4.0 + sT) * n + 3.0 * sT * n * ld +
                   16.0 * n * ld;
        // l1-Jacobi: (b, r) -> U + x; Chebyshev, second product: (y, d0) -> U + x
        return ptr + nnz_v * (4.0 + sT) + sT * n + 2.0 * sT * n * ld + 16.0 * n * ld;
    case AMG_EIG_SITE_DUALSPMM: return ptr + nnz_u * 20.0 + 8.0 * n * ld + 16.0 * n * ld;
    // flops; with the Gram products fused into the dual SpMM launch (wide
    // blocks) the site times only the reduction of the partials
    case AMG_EIG_SITE_GRAM: return dual_gram_fused(c->ld) ? 0.0 : 4.0 * n * ld * ld;
    case AMG_EIG_SITE_RESTRICT: return 4.0 * (n1 + 1) + nnz_p * 12.0 + 16.0 * n * ld + 16.0 * n1 * ld;
    case AMG_EIG_SITE_FINAL: return ptr + nnz_p * 12.0 + 8.0 * n1 * ld + 16.0 * n * ld;
    case AMG_EIG_SITE_SMALL: return 0.0;
    default: return 0.0;
    }
}

// ---------------------------------------------------------- step pieces
// One multicolour Gauss-Seidel sweep on level l, one launch per colour:
// forward from a zero guess (b -> x, reading only neighbours of smaller
// colours), or backward in place on the prolongated block in r (then V = U + r
// row by row when final).
template <typename T>
void gs_sweep(amg_eig_ctx *c, int l, bool backward, bool final, const double *base = nullptr) {
    DevLevel &d = c->dl[l];
    const Level &lv = c->H.lv[l];
    const int nc = (int)lv.coff.size() - 1;
    for (int t = 0; t < nc; ++t) {
        const int k = backward ? nc - 1 - t : t;
        const int64_t r0 = lv.coff[k], nr = lv.coff[k + 1] - r0;
        if (backward)
            launch_gs_colour<T>(c->stream, final, nr, c->ld, d.gs_ptr + r0, d.gs_col, (const T *)d.gs_val,
                                (const T *)d.gs_diag + r0, d.gs_rows + r0, (const T *)d.b, (T *)d.r,
                                base ? base : c->U, c->V, c->status, d.cpt[0]);
        else
            launch_gs_colour<T>(c->stream, false, nr, c->ld, d.gs_lptr + r0, d.gs_lcol, (const T *)d.gs_lval,
                                (const T *)d.gs_diag + r0, d.gs_rows + r0, (const T *)d.b, (T *)d.x, nullptr,
                                nullptr, c->status, d.cpt[0]);
    }
}

// One V-cycle from level k (right-hand side in dl[k].b, zero initial guess)
// down to `bottom`, where the coarse problem is solved by A_n^-1 (bottom = n)
// or by the dense tail operator Bt.  The post-smoothing on level k writes
// V = U + x when final_at_k, else x.  Returns the block that holds x on level
// k (dl[k].x, or dl[k].r after the Gauss-Seidel post-smoothing).
template <typename T>
void *vcycle_levels(amg_eig_ctx *c, int k, int bottom, bool final_at_k, const double *base = nullptr) {
    if (!base) base = c->U;
    const int L = (int)c->dl.size(), ld = c->ld;
    hipStream_t s = c->stream;
    const int *st = c->status;
    const bool cheb = c->o.smoother == AMG_EIG_SMOOTH_CHEBYSHEV;
    const bool gs = c->o.smoother == AMG_EIG_SMOOTH_GAUSS_SEIDEL;
    const double lo = c->o.cheb_lo;
    for (int l = k; l < bottom; ++l) {
        DevLevel &d = c->dl[l];
        if (gs) {
            {
                SiteScope sc(c, AMG_EIG_SITE_PRESMOOTH, l);
                gs_sweep<T>(c, l, false, false);
            }
            launch_level_residual<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.b,
                                     (const T *)d.x, (T *)d.r, st, d.cpt[0]);
        } else if (cheb) {
            {
                SiteScope sc(c, AMG_EIG_SITE_PRESMOOTH, l, true);
                launch_cheb_pre<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_vs, (const T *)d.dinv,
                                   (const T *)d.b, (T *)d.x, lo, st, d.cpt[0]);
            }
            launch_level_residual<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.b,
                                     (const T *)d.x, (T *)d.r, st, d.cpt[0]);
        } else {
            SiteScope sc(c, AMG_EIG_SITE_PRESMOOTH, l, true);
            launch_smooth_pre<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_vs, (const T *)d.dinv,
                                 (const T *)d.b, (T *)d.r, st, d.cpt[0]);
        }
        DevLevel &e = c->dl[l + 1];
        launch_spmm<T>(s, e.n, ld, d.pt_ptr, d.pt_col, (const T *)d.pt_val, (const T *)d.r, (T *)e.b, st, e.cpt[0]);
    }
    DevLevel &cl = c->dl[bottom];
    if (bottom == L - 1)
        launch_gemm_tn<T>(s, (int)cl.n, ld, (int)cl.n, (const T *)c->Ainv, (int)cl.n, (const T *)cl.b, ld,
                          (T *)cl.x, ld, st);
    else  // x_t = Bt b_t with Bt stored transposed
        launch_gemm_tn_long<T>(s, (int)cl.n, ld, (int)cl.n, (const T *)c->Bt, (int)cl.n, (const T *)cl.b, ld,
                               (T *)cl.x, ld, st);
    for (int l = bottom - 1; l >= k; --l) {
        DevLevel &d = c->dl[l];
        DevLevel &e = c->dl[l + 1];
        if (gs) {
            // y = x + P x_{l+1} into r, then the backward sweep on it in place
            const void *xc = l + 1 < bottom ? e.r : e.x;
            launch_prolong_x<T>(s, d.n, ld, d.p_ptr, d.p_col, (const T *)d.p_val, (const T *)xc, (const T *)d.x,
                                (T *)d.r, st, d.cpt[0]);
            SiteScope sc(c, AMG_EIG_SITE_POSTSMOOTH, l);
            gs_sweep<T>(c, l, true, final_at_k && l == k, base);
        } else if (cheb) {
            // y = x + P x_{l+1} into r (free after the restriction), then x = smoothed y
            launch_prolong_x<T>(s, d.n, ld, d.p_ptr, d.p_col, (const T *)d.p_val, (const T *)e.x, (const T *)d.x,
                                (T *)d.r, st, d.cpt[0]);
            launch_cheb_post1<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.dinv, (const T *)d.b,
                                 (const T *)d.r, (T *)d.t, lo, st, d.cpt[0]);
            SiteScope sc(c, AMG_EIG_SITE_POSTSMOOTH, l, true);
            launch_cheb_post2<T>(s, final_at_k && l == k, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val,
                                 (const T *)d.dinv, (const T *)d.r, (const T *)d.t, (T *)d.x, base, c->V, lo, st,
                                 d.cpt[0]);
        } else {
            launch_prolong_add<T>(s, d.n, ld, d.p_ptr, d.p_col, (const T *)d.p_val, (const T *)e.x,
                                  (const T *)d.dinv, (const T *)d.b, (T *)d.r, st, d.cpt[0]);
            SiteScope sc(c, AMG_EIG_SITE_POSTSMOOTH, l, true);
            launch_smooth_post<T>(s, final_at_k && l == k, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.dinv,
                                  (const T *)d.b, (const T *)d.r, (T *)d.x, base, c->V, st, d.cpt[0]);
        }
    }
    return gs && k < bottom ? c->dl[k].r : c->dl[k].x;
}

template <typename T>
void vcycle(amg_eig_ctx *c, int k, const double *base = nullptr) {
    const int bottom = (c->tail >= 0 && k < c->tail) ? c->tail : (int)c->dl.size() - 1;
    (void)vcycle_levels<T>(c, k, bottom, true, base);
}

// Cycles 2 .. m of one correction (eq. (3.2) with m > 1): the previous
// iterate V is copied to the head of W (free until the dual SpMM), the
// right-hand side of the next cycle is the residual of the linear equation at
// it, and the V-cycle's last post-smoothing writes V = copy + x.
template <typename T>
void further_cycles(amg_eig_ctx *c, int k) {
    DevLevel &d = c->dl[k];
    for (int i = 1; i < c->o.vcycles; ++i) {
        launch_copy_f64(c->stream, d.n * c->ld, c->V, c->W);
        launch_residual_cycle<T>(c->stream, d.n, c->ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->U, c->W, c->theta,
                                 c->H.sigma, (T *)d.b, c->status, d.cpt[1]);
        vcycle<T>(c, k, c->W);
    }
}

// Bt (stored transposed) = the V-cycle from the tail level, one identity block
// of ld columns at a time, with the same kernels as every later V-cycle.
template <typename T>
void build_tail(amg_eig_ctx *c) {
    const int t = c->tail, L = (int)c->dl.size(), ld = c->ld;
    DevLevel &d = c->dl[t];
    for (int64_t j0 = 0; j0 < d.n; j0 += ld) {
        launch_identity_block<T>(c->stream, d.n, ld, j0, (T *)d.b);
        const void *x = vcycle_levels<T>(c, t, L - 1, false);
        launch_rows_from_block<T>(c->stream, d.n, ld, j0, (const T *)x, (T *)c->Bt);
    }
}

// Rayleigh-Ritz on level k in three parts: the products that form the small
// pencil (up to Z^T B), the small eigensolver, and the recombination
// The two coarse-space products of a Rayleigh-Ritz step on level k: FG =
// Z^T B (B the block W restricted to the coarsest level, or Z_t^T B on the
// tail level) and Y = Z X_c (Z_t X_c on the tail level).
void coarse_gemms(const amg_eig_ctx *c, int k, GemmDesc *fg, GemmDesc *yg) {
    const int L = (int)c->dl.size(), ld = c->ld, dn = c->H.dn;
    const bool tail = c->tail >= 0 && k < c->tail;
    const int bottom = tail ? c->tail : L - 1;
    const double *src = bottom > k ? c->dl[bottom].cw : c->W;
    if (tail) {
        const int nt = (int)c->dl[bottom].n;
        *fg = GemmDesc{c->Zk, src, c->sw.FG, dn, 2 * ld, nt, dn, 2 * ld, 2 * ld, 1};
        *yg = GemmDesc{c->Zkt, c->sw.Xc, c->dl[bottom].cw, nt, ld, dn, nt, ld, ld, 1};
    } else {
        *fg = GemmDesc{c->Z, src, c->sw.FG, dn, 2 * ld, dn, dn, 2 * ld, 2 * ld, 0};
        *yg = GemmDesc{c->Zt, c->sw.Xc, c->Yn, dn, ld, dn, dn, ld, ld, 0};
    }
}

void launch_desc(hipStream_t s, const GemmDesc &g, const int *st) {
    if (g.long_k)
        launch_gemm_tn_long<double>(s, g.m, g.n, g.K, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, st);
    else
        launch_gemm_tn<double>(s, g.m, g.n, g.K, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, st);
}

// with_gemm = false leaves Z^T B to the caller (the joint batch launches it)
void rr_front(amg_eig_ctx *c, int k, bool with_gemm = true) {
    const int L = (int)c->dl.size(), ld = c->ld;
    hipStream_t s = c->stream;
    const int *st = c->status;
    DevLevel &d = c->dl[k];
    if (dual_gram_fused(ld)) {  // one pass over V and W for both products
        {
            SiteScope sc(c, AMG_EIG_SITE_DUALSPMM, k, true);
            launch_dual_gram(s, d.n, ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->V, c->W, c->part_gram, st, d.cpt[1]);
        }
        SiteScope sc(c, AMG_EIG_SITE_GRAM, k);
        launch_gram_reduce(s, d.n, ld, c->part_gram, c->sw.GAGM, st);
    } else {
        {
            SiteScope sc(c, AMG_EIG_SITE_DUALSPMM, k, true);
            launch_dual_spmm(s, d.n, ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->V, c->W, st, d.cpt[1]);
        }
        SiteScope sc(c, AMG_EIG_SITE_GRAM, k);
        launch_gram(s, d.n, ld, c->V, c->W, c->part_gram, c->sw.GAGM, st);
    }
    // restrict W to the tail level (then Zk^T) or to the coarsest level (then Z^T)
    const bool tail = c->tail >= 0 && k < c->tail;
    const int bottom = tail ? c->tail : L - 1;
    const double *src = c->W;
    for (int l = k; l < bottom; ++l) {
        DevLevel &a = c->dl[l];
        DevLevel &b = c->dl[l + 1];
        SiteScope sc(c, AMG_EIG_SITE_RESTRICT, l, true);
        launch_spmm<double>(s, b.n, 2 * ld, a.pt_ptr, a.pt_col, a.pt64, src, b.cw, st, b.cpt[2]);
        src = b.cw;
    }
    site_mark(c, AMG_EIG_SITE_SMALL, k);  // the small site spans Z^T B .. Z X_c
    if (with_gemm) {
        GemmDesc fg, yg;
        coarse_gemms(c, k, &fg, &yg);
        launch_desc(s, fg, st);
    }
}

constexpr double kRankTol = 1e-13;

void rr_small(amg_eig_ctx *c, int k) {
    launch_pencil(c->stream, c->sw, kRankTol);
    launch_arrow_eig(c->stream, c->sw, c->qe, c->theta, k == 0 ? 1 : 0);
}

// with_gemm = false: Y = Z X_c was launched by the caller (the joint batch)
void rr_back(amg_eig_ctx *c, int k, bool with_gemm = true) {
    const int L = (int)c->dl.size(), ld = c->ld;
    hipStream_t s = c->stream;
    const int *st = c->status;
    DevLevel &d = c->dl[k];
    const bool tail = c->tail >= 0 && k < c->tail;
    const int bottom = tail ? c->tail : L - 1;
    GemmDesc fg, yg;
    coarse_gemms(c, k, &fg, &yg);
    if (with_gemm) launch_desc(s, yg, st);
    const double *y = yg.C;  // Y on the tail level (Z_t X_c) or on the coarsest level
    site_mark(c, AMG_EIG_SITE_SMALL, k);
    for (int l = bottom - 1; l > k; --l) {
        DevLevel &a = c->dl[l];
        launch_spmm<double>(s, a.n, ld, a.p_ptr, a.p_col, a.p64, y, a.cw, st, a.cpt[1]);
        y = a.cw;
    }
    {
        SiteScope sc(c, AMG_EIG_SITE_FINAL, k, true);
        launch_final(s, d.n, ld, d.p_ptr, d.p_col, d.p64, y, c->V, c->sw.Xv, c->U, st, d.cpt[1]);
    }
}

void rayleigh_ritz(amg_eig_ctx *c, int k) {
    rr_front(c, k);
    rr_small(c, k);
    rr_back(c, k);
}

template <typename T>
void residual(amg_eig_ctx *c, int k, int check) {
    DevLevel &d = c->dl[k];
    {
        SiteScope sc(c, AMG_EIG_SITE_RESIDUAL, k, true);
        launch_residual<T>(c->stream, d.n, c->ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->U, c->theta, (T *)d.b,
                           c->part_res, c->status, d.cpt[1]);
    }
    launch_residual_finish(c->stream, d.n, c->ld, c->part_res, c->counters, c->theta, c->rho, c->q, c->o.tol,
                           c->status, check, d.cpt[1]);
}

void correction_front(amg_eig_ctx *c, int k, bool with_gemm = true) {
    if (c->mixed) {
        residual<float>(c, k, k == 0);
        vcycle<float>(c, k);
        further_cycles<float>(c, k);
    } else {
        residual<double>(c, k, k == 0);
        vcycle<double>(c, k);
        further_cycles<double>(c, k);
    }
    rr_front(c, k, with_gemm);
}

void correction(amg_eig_ctx *c, int k) {
    correction_front(c, k);
    rr_small(c, k);
    rr_back(c, k);
}

void drop_graph(amg_eig_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    for (int i = 0; i < 2; ++i) {
        if (c->part_exec[i]) (void)hipGraphExecDestroy(c->part_exec[i]);
        if (c->part_graph[i]) (void)hipGraphDestroy(c->part_graph[i]);
        c->part_exec[i] = nullptr;
        c->part_graph[i] = nullptr;
    }
}

// ------------------------------------------------------ block width control
// The guard rule of the paper's "compute extra eigenpairs" strategy (Section
// 4.5) on Ritz values th[0..n): the smallest m in [q, n-1] with a relative
// gap th[m] / th[m-1] - 1 >= gap after the m-th value, or 0 when the values
// past the q-th show no such gap inside the block.
int closed_width(const double *th, int n, int q, double gap) {
    for (int m = q; m < n; ++m)
        if (th[m - 1] > 0.0 && th[m] / th[m - 1] - 1.0 >= gap) return m;
    return 0;
}

int round4(int w) { return (w + 3) / 4 * 4; }

// separation the width control keeps between the q-th Ritz value and the
// first one past a narrowed block
constexpr double kNarrowSep = 1.25;

// Give the context block width w.  When it is bound and the workspace holds
// the new plan, the blocks are re-carved in place (the uploaded matrices,
// coarse basis and dense tail keep their addresses) and true is returned;
// otherwise the context is left unbound with amg_eig_footprint() bytes needed.
// Either way the iterate is discarded: a start must follow.
bool set_width(amg_eig_ctx *c, int w) {
    drop_graph(c);
    c->qe = c->ld = w;
    c->initialised = false;
    c->hist.clear();
    plan(c, nullptr);
    if (c->bound && c->ws && c->need <= c->ws_bytes) {
        plan(c, c->ws);
        small_layout(c->sw, c->qe, c->theta, &c->item_host, &c->small_lds);
        coarse_gemms(c, 0, &c->item_host.fg, &c->item_host.yg);
        if (hipMemcpyAsync(c->item_dev, &c->item_host, sizeof(SmallItem), hipMemcpyHostToDevice, c->stream) ==
            hipSuccess)
            return true;
    }
    c->bound = false;
    return false;
}

// Called with the host copies of the Ritz values and residuals after every
// progress report.  A block stalls when, after at least 16 corrections, the
// smallest max_{j<q} rho_j reported in the last 10 corrections is not below
// half the smallest reported before them (a block that holds its cluster may
// rise and fall during its first dozen corrections but keeps making new lows;
// one cut inside a cluster stays flat).  A stalled block with no gap of the
// guard rule inside it past the q-th Ritz value ends inside a cluster: its
// width is doubled (up to qe_cap) and true is returned.  After a widened
// block converges, the next start takes the narrowest multiple of 4 that
// keeps the first Ritz value past it kNarrowSep above the q-th, if the wide
// block holds one.
bool width_check(amg_eig_ctx *c, const double *th, const double *rho, int steps, int conv) {
    if (!c->width_auto || c->width_decided) return false;
    const int q = c->q, qe = c->qe;
    if (conv) {
        c->width_decided = true;
        if (c->widened) {
            // the narrowest multiple of 4 whose next Ritz value lies well above the
            // q-th (theta_{w+1} >= kNarrowSep theta_q: a block of width w
            // contracts the wanted pairs by about (theta_q / theta_{w+1})^2 per
            // correction); without one inside the block, the wide width stays
            for (int w = round4(q); w < qe; w += 4)
                if (th[w] >= kNarrowSep * th[q - 1]) {
                    c->qe_next = w;
                    break;
                }
        }
        return false;
    }
    double r = 0.0;
    for (int j = 0; j < q; ++j) r = std::max(r, rho[j]);
    c->hist.emplace_back(steps, r);
    if (steps < 16 || !(r > c->o.tol)) return false;
    double recent = -1.0, before = -1.0;
    for (const auto &h : c->hist) {
        double &m = h.first > steps - 10 ? recent : before;
        if (h.second > 0.0 && (m < 0.0 || h.second < m)) m = h.second;
    }
    if (before <= 0.0 || recent <= 0.0 || !(recent > 0.5 * before)) return false;
    if (closed_width(th, qe, q, c->o.guard_gap) > 0) return false;
    const int w = std::min(c->qe_cap, round4(2 * qe));
    if (w <= qe) {
        c->width_decided = true;
        return false;
    }
    c->widened = true;
    set_width(c, w);
    return true;
}

// Algorithm 3.2: the coarsest eigenpairs start the block; the prolongated
// coarsest eigenvectors already approximate the wanted ones, so the first
// Rayleigh-Ritz step may start from them (the inertia counts still certify
// every eigenvalue it accepts)
void nested_head(amg_eig_ctx *c) {
    hipStream_t s = c->stream;
    const int ld = c->ld, qe = c->qe, dn = c->H.dn;
    launch_fill_i32(s, ST_COUNT, 0, c->status);
    launch_fill_i32(s, 1, 1, c->status + ST_WARM);
    launch_copy_cols(s, dn, ld, ld, qe, c->Z, dn, c->U);
    launch_copy_f64(s, qe, c->lam, c->theta);
}

// the block prolongated from level k + 1 to level k (a correction on level k
// follows for k >= 1)
void nested_prolong(amg_eig_ctx *c, int k) {
    DevLevel &d = c->dl[k];
    launch_spmm<double>(c->stream, d.n, c->ld, d.p_ptr, d.p_col, d.p64, c->U, c->V, c->status, d.cpt[1]);
    launch_copy_f64(c->stream, d.n * (int64_t)c->ld, c->V, c->U);
}

// after a start: the step counter counts finest-level corrections only (the
// warm-bracket flag and the rank survive)
void reset_step_count(amg_eig_ctx *c) { launch_fill_i32(c->stream, 2, 0, c->status); }

// part 0: residual, V-cycle and the products before Z^T B; part 1: the
// recombination after Y = Z X_c (the joint batch launches both products).  Replayed from a captured graph when the context asks for
// graphs and no site timing is on.
int enqueue_part(amg_eig_ctx *c, int part) {
    if (c->o.use_graph && c->stream && !c->timing) {
        if (!c->part_exec[part]) {
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            if (part == 0)
                correction_front(c, 0, false);
            else
                rr_back(c, 0, false);
            HIPCHK(c, hipStreamEndCapture(c->stream, &c->part_graph[part]));
            HIPCHK(c, hipGraphInstantiate(&c->part_exec[part], c->part_graph[part], nullptr, nullptr, 0));
        }
        HIPCHK(c, hipGraphLaunch(c->part_exec[part], c->stream));
    } else if (part == 0) {
        correction_front(c, 0, false);
    } else {
        rr_back(c, 0, false);
    }
    return AMG_EIG_OK;
}

int enqueue_steps(amg_eig_ctx *c, int steps) {
    for (int i = 0; i < steps; ++i) {
        // with site timing on, the second step of each enqueued chunk of three or
        // more runs eagerly (HIP events cannot be captured into the graph): it
        // follows a replay, so the device is busy, and it is never the step that
        // only detects convergence at the end of a solve
        const bool timed_eager = c->timing && steps >= 3 && i == 1;
        if (c->o.use_graph && c->stream && !timed_eager) {
            if (!c->graph_exec) {
                const bool t = c->timing;
                c->timing = false;
                HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                correction(c, 0);
                c->timing = t;
                HIPCHK(c, hipStreamEndCapture(c->stream, &c->graph));
                HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
            }
            HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
        } else {
            correction(c, 0);
        }
    }
    HIPCHK(c, hipGetLastError());
    return AMG_EIG_OK;
}

// Arguments of the joint batch entry points: members non-NULL, bound (and
// initialised when `initialised`), listed once; creates their join events.
int check_joint(amg_eig_ctx *const *cs, int n, bool initialised) {
    for (int i = 0; i < n; ++i) {
        amg_eig_ctx *c = cs[i];
        if (!c) return AMG_EIG_EINVAL;
        if (!c->bound) return fail(c, AMG_EIG_ESTATE, "batch member not bound");
        if (initialised && !c->initialised) return fail(c, AMG_EIG_ESTATE, "batch member not initialised");
        for (int j = 0; j < i; ++j)
            if (cs[j] == c) return fail(c, AMG_EIG_EINVAL, "context listed twice in a batch");
        if (!c->join_ev) HIPCHK(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    }
    return AMG_EIG_OK;
}

// The fg (which = 0) or yg (1) products of up to kMaxBatch members at the
// finest level, one launch per tile code.
void launch_gemms(hipStream_t s, amg_eig_ctx *const *cs, int m, int which) {
    for (int lk = 0; lk < 2; ++lk) {
        GemmTable t{};
        t.which = which;
        t.n = 0;
        t.first[0] = 0;
        for (int j = 0; j < m; ++j) {
            const GemmDesc &g = which ? cs[j]->item_host.yg : cs[j]->item_host.fg;
            if (g.long_k != lk) continue;
            t.item[t.n] = cs[j]->item_dev;
            t.first[t.n + 1] = t.first[t.n] + ((g.m + 15) / 16) * ((g.n + 15) / 16);
            ++t.n;
        }
        launch_gemm_batch(s, t, lk == 1);
    }
}

// The small eigenproblems of n members whose front parts are enqueued: the
// stream of cs[0] waits for the others (one event per distinct stream), runs
// the three batched kernels over their descriptors, and the others wait for it.
int joint_small(amg_eig_ctx *const *cs, int n, int final_level, bool gemms) {
    if (n <= 0) return AMG_EIG_OK;
    amg_eig_ctx *lead = cs[0];
    hipStream_t ls = lead->stream;
    std::vector<amg_eig_ctx *> others;  // the other streams, each once
    for (int i = 0; i < n; ++i) {
        bool seen = cs[i]->stream == ls;
        for (amg_eig_ctx *o : others) seen = seen || o->stream == cs[i]->stream;
        if (!seen) others.push_back(cs[i]);
    }
    for (amg_eig_ctx *o : others) {
        HIPCHK(o, hipEventRecord(o->join_ev, o->stream));
        HIPCHK(lead, hipStreamWaitEvent(ls, o->join_ev, 0));
    }
    // narrow (ld <= 32) and wide members in separate launches: the pencil and
    // Rayleigh-Ritz kernels of wide blocks run more wavefronts, as in a
    // member's separate launch
    std::vector<amg_eig_ctx *> group[2];
    for (int i = 0; i < n; ++i) group[cs[i]->ld > 32 ? 1 : 0].push_back(cs[i]);
    for (int wide = 0; wide < 2; ++wide) {
        const std::vector<amg_eig_ctx *> &g = group[wide];
        const int ng = (int)g.size();
        for (int i0 = 0; i0 < ng; i0 += kMaxBatch) {
            const int m = std::min(ng - i0, kMaxBatch);
            SmallTable t{};
            SmallLds lds;
            t.n = m;
            t.final_level = final_level;
            t.first[0] = t.p3first[0] = t.ctfirst[0] = 0;
            for (int j = 0; j < m; ++j) {
                const amg_eig_ctx *c = g[i0 + j];
                t.item[j] = c->item_dev;
                t.first[j + 1] = t.first[j] + c->qe;
                t.p3first[j + 1] = t.p3first[j] + pencil_p3_blocks(c->ld);
                t.ctfirst[j + 1] = t.ctfirst[j] + pencil_ct_waves(c->ld, c->H.dn);
                lds.pencil = std::max(lds.pencil, c->small_lds.pencil);
                lds.bisect = std::max(lds.bisect, c->small_lds.bisect);
                lds.rr = std::max(lds.rr, c->small_lds.rr);
            }
            if (gemms) launch_gemms(ls, g.data() + i0, m, 0);
            launch_small_batch(ls, t, lds, kRankTol, wide == 1);
            if (gemms) launch_gemms(ls, g.data() + i0, m, 1);
        }
    }
    HIPCHK(lead, hipEventRecord(lead->join_ev, ls));
    for (amg_eig_ctx *o : others) HIPCHK(o, hipStreamWaitEvent(o->stream, lead->join_ev, 0));
    return AMG_EIG_OK;
}

// ------------------------------------------------ static workspace
// For callers that cannot allocate device memory: a workspace in a
// file-scope device array.  The code object holds one copy per device, for
// the life of the process.  Its device address is taken once per device with
// hipGetSymbolAddress (the array's name in host code is only a stand-in) and
// used everywhere after.
constexpr size_t kStaticBytes = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char *g_static_ptr[kMaxDevices] = {};           // device address of scratch, per device
amg_eig_ctx *g_static_owner[kMaxDevices] = {};  // context bound to it, per device

// The current device's static workspace (its address taken on first use).
int static_workspace(amg_eig_ctx *c, char **out, int *dev_out) {
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, AMG_EIG_EHIP, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(c, AMG_EIG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_static_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_static_ptr[dev];
    *dev_out = dev;
    return AMG_EIG_OK;
}

// The context gives up the static workspace it holds (destroy, rebind).
void release_static(amg_eig_ctx *c) {
    if (c->static_dev < 0) return;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
    c->static_dev = -1;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

void amg_eig_opts_default(amg_eig_opts *o) {
    if (!o) return;
    o->theta = 0.25;
    o->coarse_max = 512;
    o->coarse_min = 0;
    o->max_levels = 25;
    o->qe = 0;
    o->guard_gap = 1e-2;
    o->smoother = AMG_EIG_SMOOTH_CHEBYSHEV;
    o->cheb_degree = 2;
    o->cheb_lo = 0.25;
    o->nu_pre = 1;
    o->nu_post = 1;
    o->precision = AMG_EIG_PREC_FP64;
    o->tol = 1e-8;
    o->max_steps = 100;
    o->use_graph = 0;
    o->qe_max = 0;
    o->shift = 0.0;
    o->coarsening = AMG_EIG_COARSEN_RS;
    o->coarsen_seed = 0;
    o->vcycles = 1;
}

int amg_eig_setup(const amg_eig_csr *A, const amg_eig_csr *M, int q, const amg_eig_opts *o, amg_eig_ctx **out) {
    if (!out) return AMG_EIG_EINVAL;
    *out = nullptr;
    amg_eig_ctx *c = new (std::nothrow) amg_eig_ctx();
    if (!c) return AMG_EIG_ENOMEM;
    if (o)
        c->o = *o;
    else
        amg_eig_opts_default(&c->o);
    const bool cheb_ok = c->o.smoother == AMG_EIG_SMOOTH_CHEBYSHEV && c->o.cheb_degree == 2 && c->o.cheb_lo > 0.0 &&
                         c->o.cheb_lo < 1.0;
    if ((c->o.smoother != AMG_EIG_SMOOTH_L1JACOBI && c->o.smoother != AMG_EIG_SMOOTH_GAUSS_SEIDEL && !cheb_ok) ||
        c->o.nu_pre != 1 || c->o.nu_post != 1 ||
        (c->o.precision != AMG_EIG_PREC_FP64 && c->o.precision != AMG_EIG_PREC_MIXED)) {
        delete c;
        return AMG_EIG_EINVAL;
    }
    int rc;
    try {
        rc = build_hierarchy(A, M, q, c->o, c->H, c->qe, c->err);
    } catch (const std::bad_alloc &) {
        rc = AMG_EIG_ENOMEM;
    } catch (...) {
        rc = AMG_EIG_EINVAL;
    }
    if (rc == AMG_EIG_OK && c->qe > kMaxWidth) rc = AMG_EIG_EINVAL;
    if (rc != AMG_EIG_OK) {
        delete c;
        return rc;
    }
    c->q = q;
    c->ld = c->qe;
    c->mixed = c->o.precision == AMG_EIG_PREC_MIXED;
    c->width_auto = c->o.qe <= 0;
    c->width_decided = !c->width_auto;
    {
        const int64_t n0 = c->H.lv[0].n, dn = c->H.dn;
        int cap = (int)std::min<int64_t>({(int64_t)kMaxWidth, dn, n0 - dn});
        if (c->o.qe_max > 0) cap = std::min(cap, c->o.qe_max);
        c->qe_cap = std::max(c->qe, cap / 4 * 4);
    }
    choose_tail(c);
    plan(c, nullptr);
    *out = c;
    return AMG_EIG_OK;
}

int amg_eig_footprint(const amg_eig_ctx *c, size_t *device_bytes) {
    if (!c || !device_bytes) return AMG_EIG_EINVAL;
    *device_bytes = c->need;
    return AMG_EIG_OK;
}

int amg_eig_bind(amg_eig_ctx *c, void *ws, size_t bytes, void *hip_stream) {
    if (!c) return AMG_EIG_EINVAL;
    if (!ws || bytes < c->need || (reinterpret_cast<uintptr_t>(ws) & 255))
        return fail(c, AMG_EIG_EWORKSPACE, "workspace missing, unaligned or smaller than the footprint");
    drop_graph(c);
    if (c->static_dev >= 0 && (char *)ws != g_static_ptr[c->static_dev]) release_static(c);
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char *)ws;
    c->ws_bytes = bytes;
    plan(c, (char *)ws);
    c->staging.clear();
    int rc = c->mixed ? upload_levels<float>(c) : upload_levels<double>(c);
    if (rc) return rc;
    launch_fill_i32(c->stream, ST_COUNT, 0, c->status);
    if (c->sw.diag) launch_fill_i32(c->stream, 5 * kMaxWidth + 8, 0, c->sw.diag);
    small_layout(c->sw, c->qe, c->theta, &c->item_host, &c->small_lds);
    coarse_gemms(c, 0, &c->item_host.fg, &c->item_host.yg);
    rc = put(c, c->item_dev, &c->item_host, sizeof(SmallItem));
    if (rc) return rc;
    std::vector<unsigned> zero(16, 0u);
    rc = upload_vec(c, c->counters, zero);
    if (rc) return rc;
    if (c->tail >= 0) {
        if (c->mixed)
            build_tail<float>(c);
        else
            build_tail<double>(c);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->staging.clear();
    c->bound = true;
    c->initialised = false;
    return AMG_EIG_OK;
}

int amg_eig_bind_static(amg_eig_ctx *c, void *hip_stream, size_t *static_bytes) {
    if (!c) return AMG_EIG_EINVAL;
    if (static_bytes) *static_bytes = kStaticBytes;
    if (c->need > kStaticBytes)
        return fail(c, AMG_EIG_EWORKSPACE, "footprint of " + std::to_string(c->need) +
                                               " bytes exceeds the static workspace of " +
                                               std::to_string(kStaticBytes) + " bytes");
    char *ws = nullptr;
    int dev = -1;
    int rc = static_workspace(c, &ws, &dev);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        amg_eig_ctx *prev = g_static_owner[dev];
        if (prev && prev != c) {
            // the previous holder loses the workspace: wait for its queued work,
            // then leave it unbound (its later calls fail with ESTATE)
            if (prev->bound) (void)hipStreamSynchronize(prev->stream);
            prev->bound = prev->initialised = false;
            prev->ws = nullptr;
            prev->ws_bytes = 0;
            prev->static_dev = -1;
        }
        g_static_owner[dev] = c;
        c->static_dev = dev;
    }
    rc = amg_eig_bind(c, ws, kStaticBytes, hip_stream);
    if (rc) release_static(c);
    return rc;
}

int amg_eig_init(amg_eig_ctx *c, int mode, uint64_t seed, const double *U_dev, int64_t ldu) {
    if (!c) return AMG_EIG_EINVAL;
    if (!c->bound) return fail(c, AMG_EIG_ESTATE, "init before bind");
    if (c->qe_next > 0) {  // a converged widened block showed a narrower one suffices
        const int w = c->qe_next;
        c->qe_next = 0;
        if (!set_width(c, w)) return fail(c, AMG_EIG_EHIP, "block width change inside the workspace failed");
    }
    c->hist.clear();
    const int L = (int)c->dl.size(), ld = c->ld, qe = c->qe;
    hipStream_t s = c->stream;
    const int64_t N = c->dl[0].n;
    if (mode == AMG_EIG_INIT_NESTED) {
        nested_head(c);
        for (int k = L - 2; k >= 0; --k) {
            nested_prolong(c, k);
            if (k >= 1) correction(c, k);
        }
    } else if (mode == AMG_EIG_INIT_RANDOM || mode == AMG_EIG_INIT_USER) {
        launch_fill_i32(s, ST_COUNT, 0, c->status);
        if (mode == AMG_EIG_INIT_RANDOM) {
            launch_fill_random(s, N, ld, qe, seed, c->V);
        } else {
            if (!U_dev || ldu < qe) return fail(c, AMG_EIG_EINVAL, "user block missing or ldu < qe");
            launch_copy_cols(s, N, ld, ld, qe, U_dev, ldu, c->V);
        }
        rayleigh_ritz(c, 0);
    } else {
        return fail(c, AMG_EIG_EINVAL, "unknown init mode");
    }
    reset_step_count(c);
    HIPCHK(c, hipGetLastError());
    c->initialised = true;
    return AMG_EIG_OK;
}

int amg_eig_correct(amg_eig_ctx *c, int steps) {
    if (!c) return AMG_EIG_EINVAL;
    if (!c->initialised) return fail(c, AMG_EIG_ESTATE, "correct before init");
    if (steps < 0) return fail(c, AMG_EIG_EINVAL, "negative step count");
    return enqueue_steps(c, steps);
}

namespace {
// progress report; `control` lets the block width control act on it
int progress_report(amg_eig_ctx *c, double *theta, double *rho, int *steps, int *converged, bool control);
}  // namespace

int amg_eig_progress(amg_eig_ctx *c, double *theta, double *rho, int *steps, int *converged) {
    return progress_report(c, theta, rho, steps, converged, true);
}

namespace {
int progress_report(amg_eig_ctx *c, double *theta, double *rho, int *steps, int *converged, bool control) {
    if (!c) return AMG_EIG_EINVAL;
    if (!c->bound) return fail(c, AMG_EIG_ESTATE, "progress before bind");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int st[ST_COUNT];
    double th[kMaxWidth], rh[kMaxWidth];
    HIPCHK(c, hipMemcpy(st, c->status, sizeof(st), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(th, c->theta, c->qe * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(rh, c->rho, c->qe * sizeof(double), hipMemcpyDeviceToHost));
    if (theta) std::memcpy(theta, th, c->qe * sizeof(double));
    if (rho) std::memcpy(rho, rh, c->qe * sizeof(double));
    if (steps) *steps = st[ST_STEPS];
    if (converged) *converged = st[ST_CONVERGED];
    if (st[ST_BREAKDOWN]) return fail(c, AMG_EIG_EBREAKDOWN, "projected problem lost definiteness");
    if (control && c->initialised && width_check(c, th, rh, st[ST_STEPS], st[ST_CONVERGED])) {
        fail(c, AMG_EIG_WIDENED, "block width raised to " + std::to_string(c->qe));
        return AMG_EIG_WIDENED;
    }
    return AMG_EIG_OK;
}
}  // namespace

int amg_eig_solve(amg_eig_ctx *c, double tol, int max_steps, double *lambda_host, double *U_dev, int64_t ldu) {
    if (!c) return AMG_EIG_EINVAL;
    if (!c->bound) return fail(c, AMG_EIG_ESTATE, "solve before bind");
    if (tol > 0 && tol != c->o.tol) {
        c->o.tol = tol;
        drop_graph(c);  // the captured step holds the old tolerance
    }
    if (!c->initialised) {
        int rc = amg_eig_init(c, AMG_EIG_INIT_NESTED, 0, nullptr, 0);
        if (rc) return rc;
    } else {
        // the converged flag may stem from an earlier test with a looser
        // tolerance: clear it, so that the first step re-evaluates the residual
        // of the current iterate against this tolerance
        launch_fill_i32(c->stream, 1, 0, c->status + ST_CONVERGED);
    }
    int done = 0, conv = 0, steps = 0, rc;
    // Steps go out in chunks between synchronisations.  Convergence of the
    // iterate after step s shows in the residual at the start of step s + 1,
    // and the steps after it return at once; so from the observed decay of
    // max_{j<q} rho_j the next chunk is sized to end at the predicted step.
    std::vector<double> rho(c->qe);
    double rho_prev = -1.0;
    int steps_prev = 0;
    int chunk = 4;
    while (!conv && done < max_steps) {
        chunk = std::max(1, std::min(chunk, max_steps - done));
        rc = enqueue_steps(c, chunk);
        if (rc) return rc;
        done += chunk;
        rc = amg_eig_progress(c, nullptr, rho.data(), &steps, &conv);
        if (rc == AMG_EIG_WIDENED) {
            // the block ended inside a cluster: start again with the wider block
            // (a larger workspace is the caller's to bind)
            if (!c->bound) return rc;
            rho.assign(c->qe, 0.0);
            if ((rc = amg_eig_init(c, AMG_EIG_INIT_NESTED, 0, nullptr, 0))) return rc;
            rho_prev = -1.0;
            steps_prev = 0;
            chunk = 4;
            continue;
        }
        if (rc) return rc;
        const double r = *std::max_element(rho.begin(), rho.begin() + c->q);
        chunk = 4;
        if (rho_prev > 0.0 && r > 0.0 && r < rho_prev && steps > steps_prev) {
            const double rate = std::pow(r / rho_prev, 1.0 / (steps - steps_prev));
            const double need = std::log(c->o.tol / r) / std::log(rate);  // steps until rho <= tol
            if (need < 4.0) chunk = std::max(1, (int)std::ceil(need));
        }
        rho_prev = r;
        steps_prev = steps;
    }
    if (!conv) {  // residual of the last iterate
        if (c->mixed)
            residual<float>(c, 0, 1);
        else
            residual<double>(c, 0, 1);
        rc = progress_report(c, nullptr, nullptr, &steps, &conv, false);
        if (rc) return rc;
    }
    if (lambda_host) HIPCHK(c, hipMemcpy(lambda_host, c->theta, c->q * sizeof(double), hipMemcpyDeviceToHost));
    if (U_dev) {
        if (ldu < c->q) return fail(c, AMG_EIG_EINVAL, "ldu < q");
        launch_copy_cols(c->stream, c->dl[0].n, c->q, ldu, c->q, c->U, c->ld, U_dev);
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return conv ? AMG_EIG_OK : AMG_EIG_NOT_CONVERGED;
}

int amg_eig_correct_batch(amg_eig_ctx *const *cs, int n, int steps, void *hip_stream) {
    if (!cs || n < 0) return AMG_EIG_EINVAL;
    for (int i = 0; i < n; ++i) {
        amg_eig_ctx *c = cs[i];
        if (!c || !c->initialised) return c ? fail(c, AMG_EIG_ESTATE, "batch member not initialised") : AMG_EIG_EINVAL;
        if (hip_stream && c->stream != (hipStream_t)hip_stream)
            return fail(c, AMG_EIG_EINVAL, "batch member bound to another stream");
    }
    for (int s = 0; s < steps; ++s)
        for (int i = 0; i < n; ++i) {
            int rc = enqueue_steps(cs[i], 1);
            if (rc) return rc;
        }
    return AMG_EIG_OK;
}

int amg_eig_correct_batch_joint(amg_eig_ctx *const *cs, int n, int steps) {
    if (!cs || n < 0 || steps < 0) return AMG_EIG_EINVAL;
    int rc = check_joint(cs, n, true);
    if (rc) return rc;
    for (int step = 0; step < steps && n > 0; ++step) {
        for (int i = 0; i < n; ++i)
            if ((rc = enqueue_part(cs[i], 0))) return rc;
        if ((rc = joint_small(cs, n, 1, true))) return rc;
        for (int i = 0; i < n; ++i)
            if ((rc = enqueue_part(cs[i], 1))) return rc;
    }
    if (n > 0) HIPCHK(cs[0], hipGetLastError());
    return AMG_EIG_OK;
}

int amg_eig_init_batch_joint(amg_eig_ctx *const *cs, int n) {
    if (!cs || n < 0) return AMG_EIG_EINVAL;
    int rc = check_joint(cs, n, false);
    if (rc) return rc;
    // members finish together: a member with L levels runs levels L-2 .. 0
    // in the last L-1 of the rounds
    int rounds = 0;
    for (int i = 0; i < n; ++i) {
        nested_head(cs[i]);
        rounds = std::max(rounds, (int)cs[i]->dl.size() - 1);
    }
    std::vector<amg_eig_ctx *> act;
    for (int t = 0; t < rounds; ++t) {
        const int k = rounds - 1 - t;
        act.clear();
        for (int i = 0; i < n; ++i)
            if (k <= (int)cs[i]->dl.size() - 2) act.push_back(cs[i]);
        for (amg_eig_ctx *c : act) {
            nested_prolong(c, k);
            if (k >= 1) correction_front(c, k);
        }
        if (k == 0) break;
        if ((rc = joint_small(act.data(), (int)act.size(), 0, false))) return rc;
        for (amg_eig_ctx *c : act) rr_back(c, k);
    }
    for (int i = 0; i < n; ++i) {
        reset_step_count(cs[i]);
        HIPCHK(cs[i], hipGetLastError());
        cs[i]->initialised = true;
    }
    return AMG_EIG_OK;
}

int amg_eig_info(const amg_eig_ctx *c, int *qe, int *nlevels, int64_t *dims) {
    if (!c) return AMG_EIG_EINVAL;
    if (qe) *qe = c->qe;
    if (nlevels) *nlevels = (int)c->H.lv.size();
    if (dims)
        for (size_t l = 0; l < c->H.lv.size(); ++l) dims[l] = c->H.lv[l].n;
    return AMG_EIG_OK;
}

int amg_eig_level_matrix(const amg_eig_ctx *c, int level, int64_t *nnz, int64_t *rowptr, int32_t *col, double *a,
                         double *m) {
    if (!c || level < 0 || level >= (int)c->H.lv.size() || !nnz) return AMG_EIG_EINVAL;
    const Level &L = c->H.lv[level];
    *nnz = (int64_t)L.col.size();
    if (rowptr) std::memcpy(rowptr, L.ptr.data(), L.ptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, L.col.data(), L.col.size() * sizeof(int32_t));
    if (a) std::memcpy(a, L.a.data(), L.a.size() * sizeof(double));
    if (m) std::memcpy(m, L.m.data(), L.m.size() * sizeof(double));
    return AMG_EIG_OK;
}

int amg_eig_level_prolongation(const amg_eig_ctx *c, int level, int64_t *nnz, int64_t *rowptr, int32_t *col,
                               double *p) {
    if (!c || level < 0 || level + 1 >= (int)c->H.lv.size() || !nnz) return AMG_EIG_EINVAL;
    const Csr &P = c->H.lv[level].P;
    *nnz = P.nnz();
    if (rowptr) std::memcpy(rowptr, P.ptr.data(), P.ptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, P.col.data(), P.col.size() * sizeof(int32_t));
    if (p) std::memcpy(p, P.val.data(), P.val.size() * sizeof(double));
    return AMG_EIG_OK;
}

int amg_eig_level_splitting(const amg_eig_ctx *c, int level, int32_t *cf) {
    if (!c || level < 0 || level + 1 >= (int)c->H.lv.size() || !cf) return AMG_EIG_EINVAL;
    const Level &L = c->H.lv[level];
    std::memcpy(cf, L.cf.data(), L.cf.size() * sizeof(int32_t));
    return AMG_EIG_OK;
}

int amg_eig_level_colouring(const amg_eig_ctx *c, int level, int32_t *colour, int *ncolours) {
    if (!c || level < 0 || level + 1 >= (int)c->H.lv.size() || !ncolours) return AMG_EIG_EINVAL;
    const Level &L = c->H.lv[level];
    if (c->o.smoother != AMG_EIG_SMOOTH_GAUSS_SEIDEL || L.coff.empty()) return AMG_EIG_EINVAL;
    *ncolours = (int)L.coff.size() - 1;
    if (colour) std::memcpy(colour, L.colour.data(), L.colour.size() * sizeof(int32_t));
    return AMG_EIG_OK;
}

int amg_eig_coarse_eigenvalues(const amg_eig_ctx *c, double *lam) {
    if (!c || !lam) return AMG_EIG_EINVAL;
    std::memcpy(lam, c->H.lam.data(), c->H.lam.size() * sizeof(double));
    return AMG_EIG_OK;
}

int amg_eig_iterate(const amg_eig_ctx *c, const double **U_dev, int64_t *ld) {
    if (!c || !U_dev || !ld) return AMG_EIG_EINVAL;
    if (!c->bound) return AMG_EIG_ESTATE;
    *U_dev = c->U;
    *ld = c->ld;
    return AMG_EIG_OK;
}

void amg_eig_destroy(amg_eig_ctx *c) {
    if (!c) return;
    release_static(c);
    drop_graph(c);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    for (auto &st : c->sites)
        for (hipEvent_t e : st.ev) (void)hipEventDestroy(e);
    delete c;
}

int amg_eig_timing(amg_eig_ctx *c, int enable) {
    if (!c) return AMG_EIG_EINVAL;
    if (c->timing && !enable) collect_sites(c);
    c->timing = enable != 0;
    if (enable)
        for (auto &st : c->sites) {
            st.ms = 0.0;
            st.launches = 0;
            st.used = 0;
        }
    return AMG_EIG_OK;
}

int amg_eig_site_stats(amg_eig_ctx *c, int site, double *alg_bytes, double *ms_total, int64_t *launches) {
    if (!c || site < 0 || site >= AMG_EIG_SITE_COUNT) return AMG_EIG_EINVAL;
    if (c->bound) HIPCHK(c, hipStreamSynchronize(c->stream));
    collect_sites(c);
    if (alg_bytes) *alg_bytes = site_bytes(c, site);
    if (ms_total) *ms_total = c->sites[site].ms;
    if (launches) *launches = c->sites[site].launches;
    return AMG_EIG_OK;
}

int amg_eig_set_cpt(amg_eig_ctx *c, int kind, int level, int cpt) {
    if (!c || kind < 0 || kind > 2 || level < 0 || level >= (int)c->H.lv.size())
        return c ? fail(c, AMG_EIG_EINVAL, "tuning kind or level out of range") : AMG_EIG_EINVAL;
    const int width = kind == AMG_EIG_TUNE_FP64_WIDE ? 2 * c->ld : c->ld;
    if (cpt != 0 && !cpt_valid(width, cpt))
        return fail(c, AMG_EIG_EINVAL, "columns per lane must be 2, 4 or 8, divide the block width and leave at "
                                       "most 64 lanes per row");
    if ((int)c->cpt_tab.size() != (int)c->H.lv.size()) c->cpt_tab.assign(c->H.lv.size(), std::array<int, 3>{0, 0, 0});
    c->cpt_tab[level][kind] = cpt;
    if (level < (int)c->dl.size()) c->dl[level].cpt[kind] = cpt;
    drop_graph(c);  // a captured step holds the old launch shapes
    return AMG_EIG_OK;
}

int amg_eig_get_cpt(const amg_eig_ctx *c, int kind, int level, int *cpt) {
    if (!c || !cpt || kind < 0 || kind > 2 || level < 0 || level >= (int)c->H.lv.size()) return AMG_EIG_EINVAL;
    const int width = kind == AMG_EIG_TUNE_FP64_WIDE ? 2 * c->ld : c->ld;
    const int hint = (int)c->cpt_tab.size() > level ? c->cpt_tab[level][kind] : 0;
    *cpt = pick_cpt(width, hint);
    return AMG_EIG_OK;
}

int amg_eig_tune_time(amg_eig_ctx *c, int kind, int level, int cpt, int reps, double *us_per_rep) {
    if (!c || !us_per_rep || kind < 0 || kind > 2 || reps < 1) return AMG_EIG_EINVAL;
    if (!c->bound) return fail(c, AMG_EIG_ESTATE, "tuning before bind");
    const int L = (int)c->dl.size(), ld = c->ld;
    if (level < 0 || level > L - 2) return fail(c, AMG_EIG_EINVAL, "no row kernels of this kind on that level");
    if (kind == AMG_EIG_TUNE_FP64_WIDE && level < 1)
        return fail(c, AMG_EIG_EINVAL, "the restriction of W produces levels 1 and below");
    const int width = kind == AMG_EIG_TUNE_FP64_WIDE ? 2 * ld : ld;
    if (cpt != 0 && !cpt_valid(width, cpt)) return fail(c, AMG_EIG_EINVAL, "invalid columns per lane");
    hipStream_t s = c->stream;
    const int *st = c->status;
    launch_fill_i32(s, ST_COUNT, 0, c->status);  // the kernels run only while the converged flag is clear
    DevLevel &d = c->dl[level];
    DevLevel &e = c->dl[level + 1];
    const double lo = c->o.cheb_lo;
    auto group = [&](auto tag) {
        using T = decltype(tag);
        if (kind == AMG_EIG_TUNE_VCYCLE) {
            if (level >= 1) {
                DevLevel &f = c->dl[level - 1];
                launch_spmm<T>(s, d.n, ld, f.pt_ptr, f.pt_col, (const T *)f.pt_val, (const T *)f.r, (T *)d.b, st, cpt);
            }
            if (c->o.smoother == AMG_EIG_SMOOTH_GAUSS_SEIDEL) {
                // the level's launch shape is what the sweeps take
                const int keep = d.cpt[0];
                d.cpt[0] = cpt;
                gs_sweep<T>(c, level, false, false);
                launch_level_residual<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.b,
                                         (const T *)d.x, (T *)d.r, st, cpt);
                launch_prolong_x<T>(s, d.n, ld, d.p_ptr, d.p_col, (const T *)d.p_val, (const T *)e.x,
                                    (const T *)d.x, (T *)d.r, st, cpt);
                gs_sweep<T>(c, level, true, false);
                d.cpt[0] = keep;
            } else if (c->o.smoother == AMG_EIG_SMOOTH_CHEBYSHEV) {
                launch_cheb_pre<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_vs, (const T *)d.dinv,
                                   (const T *)d.b, (T *)d.x, lo, st, cpt);
                launch_level_residual<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.b,
                                         (const T *)d.x, (T *)d.r, st, cpt);
                launch_prolong_x<T>(s, d.n, ld, d.p_ptr, d.p_col, (const T *)d.p_val, (const T *)e.x,
                                    (const T *)d.x, (T *)d.r, st, cpt);
                launch_cheb_post1<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.dinv,
                                     (const T *)d.b, (const T *)d.r, (T *)d.t, lo, st, cpt);
                launch_cheb_post2<T>(s, false, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.dinv,
                                     (const T *)d.r, (const T *)d.t, (T *)d.x, c->U, c->V, lo, st, cpt);
            } else {
                launch_smooth_pre<T>(s, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_vs, (const T *)d.dinv,
                                     (const T *)d.b, (T *)d.r, st, cpt);
                launch_prolong_add<T>(s, d.n, ld, d.p_ptr, d.p_col, (const T *)d.p_val, (const T *)e.x,
                                      (const T *)d.dinv, (const T *)d.b, (T *)d.r, st, cpt);
                launch_smooth_post<T>(s, false, d.n, ld, d.v_ptr, d.v_col, (const T *)d.v_val, (const T *)d.dinv,
                                      (const T *)d.b, (const T *)d.r, (T *)d.x, c->U, c->V, st, cpt);
            }
        } else if (kind == AMG_EIG_TUNE_FP64) {
            // the residual reads U and writes the level's right-hand side; the
            // final update writes into W here, never into the iterate U
            if (c->mixed)
                launch_residual<float>(s, d.n, ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->U, c->theta, (float *)d.b,
                                       c->part_res, st, cpt);
            else
                launch_residual<double>(s, d.n, ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->U, c->theta, (double *)d.b,
                                        c->part_res, st, cpt);
            if (dual_gram_fused(ld))
                launch_dual_gram(s, d.n, ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->V, c->W, c->part_gram, st, cpt);
            else
                launch_dual_spmm(s, d.n, ld, d.u_ptr, d.u_col, d.u_a, d.u_m, c->V, c->W, st, cpt);
            if (level >= 1) launch_spmm<double>(s, d.n, ld, d.p_ptr, d.p_col, d.p64, e.cw, d.cw, st, cpt);
            launch_final(s, d.n, ld, d.p_ptr, d.p_col, d.p64, e.cw, c->V, c->sw.Xv, c->W, st, cpt);
        } else {
            DevLevel &f = c->dl[level - 1];
            launch_spmm<double>(s, d.n, 2 * ld, f.pt_ptr, f.pt_col, f.pt64, level == 1 ? c->W : f.cw, d.cw, st,
                                cpt);
        }
    };
    hipEvent_t ev[2];
    HIPCHK(c, hipEventCreate(&ev[0]));
    HIPCHK(c, hipEventCreate(&ev[1]));
    auto run = [&]() {
        if (c->mixed)
            group(float());
        else
            group(double());
    };
    run();  // warm
    (void)hipEventRecord(ev[0], s);
    for (int i = 0; i < reps; ++i) run();
    (void)hipEventRecord(ev[1], s);
    hipError_t err = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev[0], ev[1]);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (err != hipSuccess) return fail(c, AMG_EIG_EHIP, std::string("tuning: ") + hipGetErrorString(err));
    *us_per_rep = 1e3 * (double)ms / reps;
    c->initialised = false;  // the scratch and flags were overwritten: init before the next correction
    return AMG_EIG_OK;
}

const char *amg_eig_strerror(int code) {
    switch (code) {
    case AMG_EIG_OK: return "ok";
    case AMG_EIG_NOT_CONVERGED: return "not converged (best-so-far results)";
    case AMG_EIG_EINVAL: return "invalid argument";
    case AMG_EIG_ENOTSPD: return "matrix not positive (semi)definite";
    case AMG_EIG_EBREAKDOWN: return "breakdown of the projected problem";
    case AMG_EIG_ENOMEM: return "host allocation failed";
    case AMG_EIG_EWORKSPACE: return "device workspace missing or too small";
    case AMG_EIG_EHIP: return "HIP runtime error";
    case AMG_EIG_ECANCELLED: return "cancelled";
    case AMG_EIG_ESTATE: return "call out of order";
    default: return "unknown code";
    }
}

const char *amg_eig_last_error(const amg_eig_ctx *c) { return c ? c->err.c_str() : ""; }

#if AMG_EIG_SMALL_STATS
// Solver statistics of the small eigensolver since bind, in builds with
// AMG_EIG_SMALL_STATS only (not part of the public header): per eigenvalue
// index the inertia counts, warm brackets used and calls, then the Jacobi
// sweeps and phase clocks.  out has 5 * kMaxWidth + 8 ints.
int amg_eig_internal_diag(amg_eig_ctx *c, int *out) {
    if (!c || !out || !c->bound) return AMG_EIG_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(out, c->sw.diag, (5 * kMaxWidth + 8) * sizeof(int), hipMemcpyDeviceToHost));
    return AMG_EIG_OK;
}
#endif

}  // extern "C"
