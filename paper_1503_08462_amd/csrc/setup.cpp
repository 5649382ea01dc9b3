// Host AMG setup (Section 2 of the paper): strength of dependence (2.1),
// classical Ruge-Stueben C/F splitting (first and second pass), direct interpolation
// (2.2)-(2.4), Galerkin coarse operators (2.5) for A and M with the same P,
// and the coarsest-level eigen-decomposition used by the V-cycle's exact
// coarse solve, the Rayleigh-Ritz step and the nested start.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "internal.h"

namespace amgeig {

namespace {

int validate(const amg_eig_csr *X, const char *name, std::string &err) {
    if (!X || X->n < 1 || !X->rowptr || !X->col || !X->val) {
        err = std::string(name) + ": missing arrays or n < 1";
        return AMG_EIG_EINVAL;
    }
    const int64_t n = X->n;
    if (X->rowptr[0] != 0) {
        err = std::string(name) + ": rowptr[0] != 0";
        return AMG_EIG_EINVAL;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (X->rowptr[i + 1] < X->rowptr[i]) {
            err = std::string(name) + ": rowptr decreasing at row " + std::to_string(i);
            return AMG_EIG_EINVAL;
        }
        for (int64_t a = X->rowptr[i]; a < X->rowptr[i + 1]; ++a) {
            int64_t c = X->col[a];
            if (c < 0 || c >= n) {
                err = std::string(name) + ": column out of range in row " + std::to_string(i);
                return AMG_EIG_EINVAL;
            }
            if (a > X->rowptr[i] && X->col[a - 1] >= c) {
                err = std::string(name) + ": columns not sorted/unique in row " + std::to_string(i);
                return AMG_EIG_EINVAL;
            }
            if (!std::isfinite(X->val[a])) {
                err = std::string(name) + ": non-finite value in row " + std::to_string(i);
                return AMG_EIG_EINVAL;
            }
        }
    }
    if (X->rowptr[n] >= (int64_t)std::numeric_limits<int32_t>::max()) {
        err = std::string(name) + ": nnz >= 2^31 is not supported";
        return AMG_EIG_EINVAL;
    }
    return AMG_EIG_OK;
}

// Shared pattern of A and M (sorted merge per row), with both value arrays.
void merge_patterns(const amg_eig_csr *A, const amg_eig_csr *M, Level &L) {
    const int64_t n = A->n;
    L.n = n;
    L.ptr.assign(n + 1, 0);
    L.col.clear();
    L.a.clear();
    L.m.clear();
    L.col.reserve(A->rowptr[n]);
    for (int64_t i = 0; i < n; ++i) {
        int64_t pa = A->rowptr[i], ea = A->rowptr[i + 1], pm = M->rowptr[i], em = M->rowptr[i + 1];
        while (pa < ea || pm < em) {
            int32_t ca = pa < ea ? A->col[pa] : std::numeric_limits<int32_t>::max();
            int32_t cm = pm < em ? M->col[pm] : std::numeric_limits<int32_t>::max();
            int32_t c = std::min(ca, cm);
            L.col.push_back(c);
            L.a.push_back(ca == c ? A->val[pa++] : 0.0);
            L.m.push_back(cm == c ? M->val[pm++] : 0.0);
        }
        L.ptr[i + 1] = (int64_t)L.col.size();
    }
}

// Strong flags per entry, eq. (2.1): j in S_i iff j != i, a_ij < 0 and
// -a_ij >= theta * max_{l != i, a_il < 0} |a_il|.
void strong_flags(const Level &L, double theta, std::vector<uint8_t> &strong) {
    strong.assign(L.col.size(), 0);
    for (int64_t i = 0; i < L.n; ++i) {
        double mx = 0.0;
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
            if (L.col[p] != i && L.a[p] < 0.0) mx = std::max(mx, -L.a[p]);
        if (mx == 0.0) continue;
        const double thr = theta * mx;
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
            if (L.col[p] != i && L.a[p] < 0.0 && -L.a[p] >= thr) strong[p] = 1;
    }
}

// Max segment tree over points: leaf = measure of an undecided point, -1 once
// decided; the root gives the largest measure and, among equals, the lowest index.
struct MaxTree {
    int64_t size = 1;
    std::vector<int64_t> val;
    std::vector<int32_t> idx;
    explicit MaxTree(int64_t n) {
        while (size < n) size <<= 1;
        val.assign(2 * size, -1);
        idx.assign(2 * size, std::numeric_limits<int32_t>::max());
        for (int64_t i = 0; i < size; ++i) idx[size + i] = (int32_t)std::min<int64_t>(i, INT32_MAX);
    }
    void pull(int64_t v) {
        int64_t l = 2 * v, r = l + 1;
        bool left = val[l] >= val[r];  // ties go to the left child: lower index
        val[v] = left ? val[l] : val[r];
        idx[v] = left ? idx[l] : idx[r];
    }
    void build() {
        for (int64_t v = size - 1; v >= 1; --v) pull(v);
    }
    void set(int64_t i, int64_t x) {
        int64_t v = size + i;
        val[v] = x;
        for (v >>= 1; v >= 1; v >>= 1) pull(v);
    }
};

// Ruge-Stueben first pass.  cf: 1 = C, 0 = F.
void rs_first_pass(const Level &L, const std::vector<uint8_t> &strong, std::vector<int32_t> &cf) {
    const int64_t n = L.n;
    // S (dependencies) and S^T (influences) as CSR
    std::vector<int64_t> sp(n + 1, 0), tp(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
            if (strong[p]) {
                sp[i + 1]++;
                tp[L.col[p] + 1]++;
            }
    for (int64_t i = 0; i < n; ++i) {
        sp[i + 1] += sp[i];
        tp[i + 1] += tp[i];
    }
    std::vector<int32_t> sc(sp[n]), tc(tp[n]);
    std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0, k = 0; i < n; ++i)
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
            if (strong[p]) {
                sc[k++] = L.col[p];
                tc[fill[L.col[p]]++] = (int32_t)i;  // rows increase, so each S^T row stays sorted
            }
    enum : int32_t { UND = -1, F = 0, C = 1 };
    cf.assign(n, UND);
    std::vector<int64_t> lam(n);
    MaxTree tree(n);
    for (int64_t i = 0; i < n; ++i) {
        lam[i] = tp[i + 1] - tp[i];
        if (lam[i] == 0 && sp[i + 1] == sp[i]) {
            cf[i] = F;  // no strong couplings at all
        } else {
            tree.val[tree.size + i] = lam[i];
        }
    }
    tree.build();
    while (tree.val[1] >= 0) {
        const int64_t i = tree.idx[1];
        cf[i] = C;
        tree.set(i, -1);
        for (int64_t a = tp[i]; a < tp[i + 1]; ++a) {  // new F points: those depending on i
            const int64_t j = tc[a];
            if (cf[j] != UND) continue;
            cf[j] = F;
            tree.set(j, -1);
            for (int64_t b = sp[j]; b < sp[j + 1]; ++b) {
                const int64_t l = sc[b];
                if (cf[l] != UND) continue;
                tree.set(l, ++lam[l]);
            }
        }
        for (int64_t a = sp[i]; a < sp[i + 1]; ++a) {  // points i depends on lose value
            const int64_t j = sc[a];
            if (cf[j] != UND) continue;
            tree.set(j, --lam[j]);
        }
    }
}

// Ruge-Stueben second pass: an F point i and each strongly coupled F point j
// must share a strong C point.  Scanning the F points in increasing order, the
// first offending j becomes a tentative C point of i; a second one turns i
// itself into a C point (and the tentative one is dropped); a tentative point
// still standing after i's scan becomes a C point.
void rs_second_pass(const Level &L, const std::vector<uint8_t> &strong, std::vector<int32_t> &cf) {
    const int64_t n = L.n;
    std::vector<int64_t> owner(n, -1);  // owner[k] == i  <=>  k is in C_i for the current i
    auto strong_of = [&](int64_t i, auto &&fn) {
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
            if (strong[p] && fn(L.col[p])) return true;
        return false;
    };
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i] != 0) continue;
        strong_of(i, [&](int64_t k) {
            if (cf[k] == 1) owner[k] = i;
            return false;
        });
        int64_t pending = -1;
        bool promote_i = false;
        strong_of(i, [&](int64_t j) {
            if (cf[j] != 0) return false;
            const bool shares = strong_of(j, [&](int64_t k) { return owner[k] == i; });
            if (shares) return false;
            if (pending >= 0) {
                promote_i = true;
                return true;  // stop scanning
            }
            pending = j;
            owner[j] = i;
            return false;
        });
        if (promote_i)
            cf[i] = 1;
        else if (pending >= 0)
            cf[pending] = 1;
    }
}

// Direct interpolation (2.2)-(2.4).  For F point i with P_i = S_i cap C:
// w_ij = -alpha_i a_ij / a~_ii, alpha_i = sum_{N_i, a<0} a_ij / sum_{P_i} a_ij,
// a~_ii = a_ii + sum_{N_i, a>0} a_ij (positive couplings cannot be
// interpolated from P_i, which holds negative couplings only, and are lumped
// into the diagonal).  C points are injected.
void direct_interpolation(const Level &L, const std::vector<uint8_t> &strong, const std::vector<int32_t> &cf,
                          Csr &P) {
    const int64_t n = L.n;
    std::vector<int32_t> cidx(n, -1);
    int32_t nc = 0;
    for (int64_t i = 0; i < n; ++i)
        if (cf[i] == 1) cidx[i] = nc++;
    P.nr = n;
    P.nc = nc;
    P.ptr.assign(n + 1, 0);
    P.col.clear();
    P.val.clear();
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i] == 1) {
            P.col.push_back(cidx[i]);
            P.val.push_back(1.0);
        } else {
            double diag = 0.0, sneg = 0.0, spos = 0.0, sP = 0.0;
            for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p) {
                const double v = L.a[p];
                if (L.col[p] == i) {
                    diag += v;
                } else if (v < 0.0) {
                    sneg += v;
                    if (strong[p] && cf[L.col[p]] == 1) sP += v;
                } else if (v > 0.0) {
                    spos += v;
                }
            }
            if (sP != 0.0) {
                const double alpha = sneg / sP;
                const double ahat = diag + spos;
                for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
                    if (strong[p] && cf[L.col[p]] == 1) {
                        P.col.push_back(cidx[L.col[p]]);
                        P.val.push_back(-alpha * L.a[p] / ahat);
                    }
            }
        }
        P.ptr[i + 1] = (int64_t)P.col.size();
    }
}

void transpose(const Csr &P, Csr &T) {
    T.nr = P.nc;
    T.nc = P.nr;
    T.ptr.assign(P.nc + 1, 0);
    for (int64_t p = 0; p < P.nnz(); ++p) T.ptr[P.col[p] + 1]++;
    for (int64_t c = 0; c < P.nc; ++c) T.ptr[c + 1] += T.ptr[c];
    T.col.resize(P.nnz());
    T.val.resize(P.nnz());
    std::vector<int64_t> fill(T.ptr.begin(), T.ptr.end() - 1);
    for (int64_t i = 0; i < P.nr; ++i)
        for (int64_t p = P.ptr[i]; p < P.ptr[i + 1]; ++p) {
            int64_t q = fill[P.col[p]]++;
            T.col[q] = (int32_t)i;
            T.val[q] = P.val[p];
        }
}

// Galerkin products P^T A P and P^T M P on one pattern (two value arrays),
// with a dense accumulator; columns of each output row sorted.
void galerkin(const Level &L, const Csr &P, const Csr &Pt, Level &out) {
    const int64_t n = L.n, nc = P.nc;
    // T = X P (n x nc) for X = A and M
    std::vector<int64_t> tptr(n + 1, 0);
    std::vector<int32_t> tcol;
    std::vector<double> ta, tm;
    std::vector<int64_t> pos(nc, -1);
    tcol.reserve(L.col.size() * 2);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t start = (int64_t)tcol.size();
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p) {
            const int64_t j = L.col[p];
            const double va = L.a[p], vm = L.m[p];
            for (int64_t r = P.ptr[j]; r < P.ptr[j + 1]; ++r) {
                const int32_t c = P.col[r];
                if (pos[c] < start) {
                    pos[c] = (int64_t)tcol.size();
                    tcol.push_back(c);
                    ta.push_back(va * P.val[r]);
                    tm.push_back(vm * P.val[r]);
                } else {
                    ta[pos[c]] += va * P.val[r];
                    tm[pos[c]] += vm * P.val[r];
                }
            }
        }
        tptr[i + 1] = (int64_t)tcol.size();
    }
    // out = P^T T (nc x nc)
    out.n = nc;
    out.ptr.assign(nc + 1, 0);
    out.col.clear();
    out.a.clear();
    out.m.clear();
    std::fill(pos.begin(), pos.end(), -1);
    std::vector<int32_t> rowc;
    std::vector<double> rowa, rowm;
    std::vector<int32_t> order;
    for (int64_t c = 0; c < nc; ++c) {
        rowc.clear();
        rowa.clear();
        rowm.clear();
        for (int64_t p = Pt.ptr[c]; p < Pt.ptr[c + 1]; ++p) {
            const int64_t i = Pt.col[p];
            const double w = Pt.val[p];
            for (int64_t r = tptr[i]; r < tptr[i + 1]; ++r) {
                const int32_t k = tcol[r];
                if (pos[k] < 0) {
                    pos[k] = (int64_t)rowc.size();
                    rowc.push_back(k);
                    rowa.push_back(w * ta[r]);
                    rowm.push_back(w * tm[r]);
                } else {
                    rowa[pos[k]] += w * ta[r];
                    rowm[pos[k]] += w * tm[r];
                }
            }
        }
        order.resize(rowc.size());
        for (size_t t = 0; t < rowc.size(); ++t) order[t] = (int32_t)t;
        std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return rowc[x] < rowc[y]; });
        for (int32_t t : order) {
            out.col.push_back(rowc[t]);
            out.a.push_back(rowa[t]);
            out.m.push_back(rowm[t]);
            pos[rowc[t]] = -1;
        }
        out.ptr[c + 1] = (int64_t)out.col.size();
    }
}

// V-cycle operator: A_k - sigma M_k (the operator of the shifted linear
// equation of Remark 3.1; A_k when sigma = 0) without explicit off-diagonal
// zeros, and its l1 diagonal.  Returns false if a diagonal entry is not positive.
bool vcycle_operator(Level &L, double sigma) {
    Csr &V = L.av;
    V.nr = V.nc = L.n;
    V.ptr.assign(L.n + 1, 0);
    V.col.clear();
    V.val.clear();
    L.l1.assign(L.n, 0.0);
    bool ok = true;
    for (int64_t i = 0; i < L.n; ++i) {
        for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p) {
            const double v = L.a[p] - sigma * L.m[p];
            if (L.col[p] == i) ok = ok && v > 0.0;
            if (v == 0.0 && L.col[p] != i) continue;
            V.col.push_back(L.col[p]);
            V.val.push_back(v);
            L.l1[i] += std::fabs(v);
        }
        V.ptr[i + 1] = (int64_t)V.col.size();
    }
    return ok;
}

// Multicolour ordering of the V-cycle operator: i and j are neighbours when
// a_ij != 0 or a_ji != 0 (i != j); rows 0, 1, ... take the smallest colour no
// already coloured neighbour holds (first fit).  A Gauss-Seidel sweep that
// visits the rows colour by colour updates the rows of one colour from values
// of other colours only, so each colour is one parallel step.
void colour_level(Level &L) {
    const Csr &V = L.av;
    const int64_t n = L.n;
    // symmetric neighbour lists: row i's off-diagonal columns plus the rows
    // that hold column i
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = V.ptr[i]; p < V.ptr[i + 1]; ++p)
            if (V.col[p] != i) {
                ++deg[i + 1];
                ++deg[V.col[p] + 1];
            }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    std::vector<int32_t> nb(deg[n]);
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = V.ptr[i]; p < V.ptr[i + 1]; ++p) {
            const int32_t j = V.col[p];
            if (j == i) continue;
            nb[fill[i]++] = j;
            nb[fill[j]++] = (int32_t)i;
        }
    L.colour.assign(n, -1);
    std::vector<int64_t> mark;  // mark[c] == i: colour c is held next to row i
    int32_t ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = deg[i]; p < deg[i + 1]; ++p) {
            const int32_t c = L.colour[nb[p]];
            if (c >= 0) mark[c] = i;
        }
        int32_t c = 0;
        while (c < ncol && mark[c] == i) ++c;
        L.colour[i] = c;
        if (c == ncol) {
            ++ncol;
            mark.push_back(-1);
        }
    }
    L.coff.assign(ncol + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++L.coff[L.colour[i] + 1];
    for (int32_t c = 0; c < ncol; ++c) L.coff[c + 1] += L.coff[c];
    L.corder.assign(n, 0);
    {
        std::vector<int64_t> at(L.coff.begin(), L.coff.end() - 1);
        for (int64_t i = 0; i < n; ++i) L.corder[at[L.colour[i]]++] = (int32_t)i;
    }
    for (Csr *g : {&L.gs_all, &L.gs_lo}) {
        g->nr = g->nc = n;
        g->ptr.assign(n + 1, 0);
        g->col.clear();
        g->val.clear();
    }
    L.gs_diag.assign(n, 0.0);
    for (int64_t s = 0; s < n; ++s) {
        const int64_t i = L.corder[s];
        for (int64_t p = V.ptr[i]; p < V.ptr[i + 1]; ++p) {
            const int32_t j = V.col[p];
            if (j == i) {
                L.gs_diag[s] += V.val[p];
                continue;
            }
            L.gs_all.col.push_back(j);
            L.gs_all.val.push_back(V.val[p]);
            if (L.colour[j] < L.colour[i]) {
                L.gs_lo.col.push_back(j);
                L.gs_lo.val.push_back(V.val[p]);
            }
        }
        L.gs_all.ptr[s + 1] = (int64_t)L.gs_all.col.size();
        L.gs_lo.ptr[s + 1] = (int64_t)L.gs_lo.col.size();
    }
}

}  // namespace

int build_hierarchy(const amg_eig_csr *A, const amg_eig_csr *M, int q, const amg_eig_opts &o, Hierarchy &H,
                    int &qe, std::string &err) {
    int rc = validate(A, "A", err);
    if (rc) return rc;
    rc = validate(M, "M", err);
    if (rc) return rc;
    if (A->n != M->n) {
        err = "A and M differ in size";
        return AMG_EIG_EINVAL;
    }
    if (q < 1 || !(o.theta > 0.0 && o.theta < 1.0) || o.coarse_max < 1 || o.max_levels < 2) {
        err = "invalid q or options";
        return AMG_EIG_EINVAL;
    }
    H.lv.clear();
    H.lv.emplace_back();
    merge_patterns(A, M, H.lv[0]);
    {
        const Level &L = H.lv[0];
        for (int64_t i = 0; i < L.n; ++i) {
            double aii = 0.0, mii = 0.0;
            for (int64_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p)
                if (L.col[p] == i) {
                    aii = L.a[p];
                    mii = L.m[p];
                }
            if (!(aii > 0.0) || mii < 0.0) {
                err = "non-positive a_ii or negative m_ii at row " + std::to_string(i);
                return AMG_EIG_ENOTSPD;
            }
        }
    }
    const int qcap = o.qe > 0 ? o.qe : 2 * q + 8;
    const int64_t cmin = o.coarse_min > 0 ? o.coarse_min : std::max<int64_t>(2 * qcap + 2, 16);
    if (o.vcycles < 1 || o.vcycles > 16) {
        err = "vcycles must lie in 1 .. 16";
        return AMG_EIG_EINVAL;
    }
    if (o.coarsening != AMG_EIG_COARSEN_RS && o.coarsening != AMG_EIG_COARSEN_PMIS) {
        err = "invalid coarsening";
        return AMG_EIG_EINVAL;
    }
    if (o.coarsening == AMG_EIG_COARSEN_PMIS) {
        rc = device_coarsen(H, o, cmin, err);
        if (rc) return rc;
    }
    std::vector<uint8_t> strong;
    while (o.coarsening == AMG_EIG_COARSEN_RS && (int)H.lv.size() < o.max_levels && H.lv.back().n > o.coarse_max) {
        Level &L = H.lv.back();
        strong_flags(L, o.theta, strong);
        std::vector<int32_t> cf;
        rs_first_pass(L, strong, cf);
        rs_second_pass(L, strong, cf);
        int64_t nc = 0;
        for (int32_t v : cf) nc += v == 1;
        if (nc < cmin || (double)nc > 0.9 * (double)L.n || nc == 0) break;
        L.cf.swap(cf);
        direct_interpolation(L, strong, L.cf, L.P);
        transpose(L.P, L.Pt);
        Level next;
        galerkin(L, L.P, L.Pt, next);
        H.lv.push_back(std::move(next));
    }
    if (H.lv.size() < 2) {
        err = "the hierarchy needs at least two levels (n <= coarse_max or coarsening stalled)";
        return AMG_EIG_EINVAL;
    }
    // coarsest eigen-decomposition
    const Level &Lc = H.lv.back();
    const int dn = (int)Lc.n;
    std::vector<double> Ad((size_t)dn * dn, 0.0), Md((size_t)dn * dn, 0.0);
    for (int i = 0; i < dn; ++i)
        for (int64_t p = Lc.ptr[i]; p < Lc.ptr[i + 1]; ++p) {
            Ad[(size_t)i * dn + Lc.col[p]] = Lc.a[p];
            Md[(size_t)i * dn + Lc.col[p]] = Lc.m[p];
        }
    for (int i = 0; i < dn; ++i)
        for (int j = 0; j < i; ++j) {
            double sa = 0.5 * (Ad[(size_t)i * dn + j] + Ad[(size_t)j * dn + i]);
            double sm = 0.5 * (Md[(size_t)i * dn + j] + Md[(size_t)j * dn + i]);
            Ad[(size_t)i * dn + j] = Ad[(size_t)j * dn + i] = sa;
            Md[(size_t)i * dn + j] = Md[(size_t)j * dn + i] = sm;
        }
    if (o.coarsening == AMG_EIG_COARSEN_PMIS) {
        rc = device_sygv(dn, Ad, Md, H.lam, H.Z, err);
        if (rc) return rc;
    } else if (!dense_sygv(dn, Ad, Md, H.lam, H.Z)) {
        err = "coarsest mass matrix not positive definite";
        return AMG_EIG_ENOTSPD;
    }
    if (!(H.lam[0] > 0.0)) {
        err = "coarsest stiffness matrix not positive definite";
        return AMG_EIG_ENOTSPD;
    }
    H.dn = dn;
    // shift of the linear equation (Remark 3.1): below the smallest coarsest
    // eigenvalue, an upper bound of the smallest eigenvalue of every level
    if (!std::isfinite(o.shift)) {
        err = "shift must be finite";
        return AMG_EIG_EINVAL;
    }
    H.sigma = o.shift;
    if (!(H.sigma < H.lam[0])) {
        err = "shift not below the smallest eigenvalue of the coarsest level";
        return AMG_EIG_EINVAL;
    }
    for (size_t l = 0; l < H.lv.size(); ++l)
        if (!vcycle_operator(H.lv[l], H.sigma) && H.sigma != 0.0) {
            err = "a_ii - sigma m_ii <= 0 on level " + std::to_string(l) + ": shift too large";
            return AMG_EIG_EINVAL;
        }
    if (o.smoother == AMG_EIG_SMOOTH_GAUSS_SEIDEL)
        for (size_t l = 0; l + 1 < H.lv.size(); ++l) colour_level(H.lv[l]);
    H.Ainv.assign((size_t)dn * dn, 0.0);
    for (int i = 0; i < dn; ++i)
        for (int k = 0; k < dn; ++k) {
            const double zik = H.Z[(size_t)i * dn + k] / (H.lam[k] - H.sigma);
            if (zik == 0.0) continue;
            for (int j = 0; j < dn; ++j) H.Ainv[(size_t)i * dn + j] += zik * H.Z[(size_t)j * dn + k];
        }
    // block width: explicit, or the guard rule on the coarsest eigenvalues;
    // rounded up to a multiple of 4 (the extra columns are extra eigenpairs)
    int w = o.qe > 0 ? o.qe : guard_width(H.lam, q, o.guard_gap, 2 * q + 8);
    w = std::max(w, q);
    w = (w + 3) / 4 * 4;
    if (w > dn || (int64_t)w + dn > A->n) {
        err = "block width " + std::to_string(w) + " does not fit the coarsest space (" + std::to_string(dn) +
              ") or N - d_n";
        return AMG_EIG_EINVAL;
    }
    qe = w;
    return AMG_EIG_OK;
}

}  // namespace amgeig
