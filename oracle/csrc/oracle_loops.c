/*
 * Oracle loops that are inherently sequential, in plain C (test infrastructure
 * only: the eigensolver library never links or calls this file).
 *
 *  rs_first_pass  classical Ruge-Stueben C/F splitting, first pass
 *                 (Section 2.1: measure |S_i^T|, greedy choice of C points).
 *  rs_second_pass classical second pass: strongly coupled F points must share
 *                 a strong C point (the coarsening the paper refers to).
 *  gs_sweep       one Gauss-Seidel sweep on a block of right-hand sides
 *                 (the smoother of the paper's default settings, Section 4.1),
 *                 in the natural row order or in a given one.
 *  greedy_colour  first-fit colouring of a graph in the natural vertex order
 *                 (the ordering of the multicolour Gauss-Seidel smoother).
 */
#include <stdint.h>
#include <stdlib.h>

/* ---- binary heap of (-measure, index): pops max measure, lowest index ---- */
typedef struct { int64_t key; int32_t idx; } item;

static int less(item a, item b) { return a.key < b.key || (a.key == b.key && a.idx < b.idx); }

static void push(item *h, int64_t *n, item it) {
    int64_t i = (*n)++;
    h[i] = it;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!less(h[i], h[p])) break;
        item t = h[i]; h[i] = h[p]; h[p] = t; i = p;
    }
}

static item pop(item *h, int64_t *n) {
    item top = h[0];
    h[0] = h[--(*n)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && less(h[l], h[m])) m = l;
        if (r < *n && less(h[r], h[m])) m = r;
        if (m == i) break;
        item t = h[i]; h[i] = h[m]; h[m] = t; i = m;
    }
    return top;
}

/*
 * S (strong dependencies, row i lists S_i) and ST (row i lists S_i^T), both CSR.
 * Output cf[i] = 1 for C, 0 for F.  Returns the number of C points, or -1 on
 * allocation failure.
 *
 * Rule: points with S_i and S_i^T both empty are F.  Repeatedly take the
 * undecided point with the largest measure (ties: lowest index) as C; its
 * undecided strong influencees (S_i^T) become F, and each undecided point that
 * such a new F point strongly depends on gains one unit of measure; undecided
 * points that the new C point strongly depends on lose one unit.
 */
int64_t rs_first_pass(int64_t n, const int64_t *s_ptr, const int32_t *s_col,
                      const int64_t *st_ptr, const int32_t *st_col, int32_t *cf) {
    enum { UND = -1, F = 0, C = 1 };
    int64_t *lam = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t cap = n + 8;
    for (int64_t i = 0; i < n; ++i) cap += st_ptr[i + 1] - st_ptr[i] + s_ptr[i + 1] - s_ptr[i];
    item *heap = (item *)malloc(sizeof(item) * (size_t)cap);
    if (!lam || !heap) { free(lam); free(heap); return -1; }
    int64_t hn = 0, nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        lam[i] = st_ptr[i + 1] - st_ptr[i];
        if (lam[i] == 0 && s_ptr[i + 1] == s_ptr[i]) { cf[i] = F; continue; }
        cf[i] = UND;
        push(heap, &hn, (item){-lam[i], (int32_t)i});
    }
    while (hn > 0) {
        item it = pop(heap, &hn);
        int64_t i = it.idx;
        if (cf[i] != UND || -it.key != lam[i]) continue; /* stale entry */
        cf[i] = C; ++nc;
        for (int64_t a = st_ptr[i]; a < st_ptr[i + 1]; ++a) {
            int64_t j = st_col[a];
            if (cf[j] != UND) continue;
            cf[j] = F;
            for (int64_t b = s_ptr[j]; b < s_ptr[j + 1]; ++b) {
                int64_t l = s_col[b];
                if (cf[l] != UND) continue;
                lam[l] += 1;
                push(heap, &hn, (item){-lam[l], (int32_t)l});
            }
        }
        for (int64_t a = s_ptr[i]; a < s_ptr[i + 1]; ++a) {
            int64_t j = s_col[a];
            if (cf[j] != UND) continue;
            lam[j] -= 1;
            push(heap, &hn, (item){-lam[j], (int32_t)j});
        }
        if (hn + n + 8 > cap) { /* grow: bounded by total pushes, never expected */
            cap *= 2;
            item *nh = (item *)realloc(heap, sizeof(item) * (size_t)cap);
            if (!nh) { free(lam); free(heap); return -1; }
            heap = nh;
        }
    }
    free(lam);
    free(heap);
    return nc;
}

/*
 * Second pass over the F points in increasing order.  For F point i with
 * strong C points C_i = S_i cap C, every strong F neighbour j must strongly
 * depend on some point of C_i; the first j that does not is added to C_i
 * tentatively, and a second such j makes i itself a C point instead.  A
 * tentative point that survives the scan of i becomes a C point.
 */
int64_t rs_second_pass(int64_t n, const int64_t *s_ptr, const int32_t *s_col, int32_t *cf) {
    int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!stamp) return -1;
    for (int64_t k = 0; k < n; ++k) stamp[k] = -1;
    int64_t added = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (cf[i] != 0) continue;
        for (int64_t a = s_ptr[i]; a < s_ptr[i + 1]; ++a)
            if (cf[s_col[a]] == 1) stamp[s_col[a]] = i;
        int64_t tentative = -1;
        int became_c = 0;
        for (int64_t a = s_ptr[i]; a < s_ptr[i + 1]; ++a) {
            int64_t j = s_col[a];
            if (cf[j] != 0) continue;
            int common = 0;
            for (int64_t b = s_ptr[j]; b < s_ptr[j + 1]; ++b)
                if (stamp[s_col[b]] == i) { common = 1; break; }
            if (common) continue;
            if (tentative >= 0) { cf[i] = 1; became_c = 1; ++added; break; }
            tentative = j;
            stamp[j] = i;
        }
        if (!became_c && tentative >= 0) { cf[tentative] = 1; ++added; }
    }
    free(stamp);
    return added;
}

/*
 * One Gauss-Seidel sweep for A x = b, q right-hand sides stored row-major
 * (x[i*q + c]).  Rows are visited in the order order[0], order[1], ...
 * (natural order when order is NULL); backward != 0 runs that sequence from
 * its end.
 */
void gs_sweep(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              int q, const double *b, double *x, int backward, const int64_t *order) {
    double *acc = (double *)malloc(sizeof(double) * (size_t)q);
    for (int64_t t = 0; t < n; ++t) {
        int64_t s = backward ? n - 1 - t : t;
        int64_t i = order ? order[s] : s;
        double diag = 0.0;
        for (int c = 0; c < q; ++c) acc[c] = b[i * q + c];
        for (int64_t a = rowptr[i]; a < rowptr[i + 1]; ++a) {
            int64_t j = col[a];
            if (j == i) { diag += val[a]; continue; }
            for (int c = 0; c < q; ++c) acc[c] -= val[a] * x[j * q + c];
        }
        for (int c = 0; c < q; ++c) x[i * q + c] = acc[c] / diag;
    }
    free(acc);
}

/*
 * First-fit colouring: vertices 0, 1, ..., n-1 in turn take the smallest
 * colour that no already coloured neighbour holds.  adj is a symmetric
 * adjacency list in CSR form without self loops.  Returns the number of
 * colours, or -1 if memory runs out.
 */
int64_t greedy_colour(int64_t n, const int64_t *rowptr, const int32_t *adj, int32_t *colour) {
    int64_t ncol = 0;
    int64_t *seen = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!seen) return -1;
    for (int64_t c = 0; c <= n; ++c) seen[c] = -1;
    for (int64_t i = 0; i < n; ++i) colour[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t a = rowptr[i]; a < rowptr[i + 1]; ++a) {
            int32_t c = colour[adj[a]];
            if (c >= 0) seen[c] = i;  /* colour c is taken next to vertex i */
        }
        int32_t c = 0;
        while (seen[c] == i) ++c;
        colour[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(seen);
    return ncol;
}
