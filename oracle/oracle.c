/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, single-threaded reference implementations used to check the
 * HIP solver.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library; the solver never calls it and shares no
 * code with it.
 *
 * Paper: Zhang, Azad, Hu, "FastSV: A Distributed-Memory Connected Component
 * Algorithm with Fast Convergence" (arXiv 1910.05971).
 *
 * Input everywhere: an undirected graph as a symmetric CSR (row_ptr[n+1],
 * col[nnz]); the stored entries (u,v) with v in row u are the edge set E with
 * both orientations of every undirected edge (Sec. 2.1 notation; Alg. 3 works
 * on the symmetric adjacency matrix).  Self loops and duplicates are allowed.
 *
 * Contents
 *   oracle_uf_labels      union-find; plain definition of the result
 *   oracle_bfs_labels     BFS from each smallest unlabelled vertex (brute force)
 *   oracle_fastsv_alg2    FastSV (Algorithm 2), Jacobi f / f_next
 *   oracle_fastsv_alg3    FastSV in the linear-algebra form of Algorithm 3
 *   oracle_sv_alg1        Algorithm 1 (simplified SV)
 *   oracle_sv_variant     Alg. 1 plus any subset of the Sec. 3 optimisations
 *   oracle_fastsv_async   Algorithm 2 with one vector read and written in place
 *
 * Trace arguments (all optional, may be NULL): after iteration k (1-based),
 * f_trace[(k-1)*n ...] receives f and changed[k-1] the termination count of
 * that iteration, for k <= trace_cap.
 *
 * Return value of the iterative routines: number of iterations executed
 * (>= 1 for n >= 1, 0 for n == 0), or -1 if max_iters > 0 iterations ran
 * without meeting the termination test (f then holds the last iterate), or
 * -2 on allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int32_t min32(int32_t a, int32_t b) { return a < b ? a : b; }

static void record(int32_t n, int32_t k, const int32_t *f, int64_t changed,
                   int32_t *f_trace, int64_t *changed_trace, int32_t trace_cap) {
    if (k > trace_cap) return;
    if (f_trace) memcpy(f_trace + (int64_t)(k - 1) * n, f, (size_t)n * sizeof(int32_t));
    if (changed_trace) changed_trace[k - 1] = changed;
}

/* ------------------------------------------------------------------------
 * O1: union-find.  For every stored edge (u,v) find both roots (path halving)
 * and link the larger root below the smaller one, so every root is the
 * smallest vertex of its set.  Result: labels[u] = min{w : w connected to u},
 * the final state the paper states for FastSV (Sec. 3.4; Appendix A).
 * ------------------------------------------------------------------------ */
static int32_t uf_find(int32_t *p, int32_t x) {
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

int32_t oracle_uf_labels(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *labels) {
    for (int32_t u = 0; u < n; ++u) labels[u] = u;
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t a = uf_find(labels, u), b = uf_find(labels, col[e]);
            if (a < b) labels[b] = a;
            else if (b < a) labels[a] = b;
        }
    }
    for (int32_t u = 0; u < n; ++u) labels[u] = uf_find(labels, u);
    return 0;
}

/* Union-find over an edge list (both endpoints given once per edge). */
int32_t oracle_uf_labels_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               int32_t *labels) {
    for (int32_t u = 0; u < n; ++u) labels[u] = u;
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = uf_find(labels, src[i]), b = uf_find(labels, dst[i]);
        if (a < b) labels[b] = a;
        else if (b < a) labels[a] = b;
    }
    for (int32_t u = 0; u < n; ++u) labels[u] = uf_find(labels, u);
    return 0;
}

/* ------------------------------------------------------------------------
 * O2: breadth-first search.  Vertices are visited in increasing order; an
 * unlabelled vertex s starts a BFS that labels its whole component with s,
 * which is then the component's smallest vertex.
 * ------------------------------------------------------------------------ */
int32_t oracle_bfs_labels(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t *labels) {
    int32_t *queue = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!queue) return -2;
    for (int32_t u = 0; u < n; ++u) labels[u] = -1;
    for (int32_t s = 0; s < n; ++s) {
        if (labels[s] >= 0) continue;
        int32_t head = 0, tail = 0;
        labels[s] = s;
        queue[tail++] = s;
        while (head < tail) {
            int32_t x = queue[head++];
            for (int32_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e) {
                int32_t y = col[e];
                if (labels[y] < 0) { labels[y] = s; queue[tail++] = y; }
            }
        }
    }
    free(queue);
    return 0;
}

/* ------------------------------------------------------------------------
 * O3: FastSV as Algorithm 2 states it (Sec. 3).
 * Start from n single-vertex trees, f = iota, and a write vector f_next that
 * holds the same values.  An iteration reads only the f it started with and
 * lowers entries of f_next by min-updates (Sec. 2.4: separate read and write
 * vectors make every iterate deterministic), in the paper's order:
 *   - for each stored entry (u,v), the parent f[u] of u is offered v's
 *     grandparent f[f[v]]: the tree containing u, or a part of it, hooks
 *     onto v's tree without any root test (Sec. 3.1 and 3.2);
 *   - for each stored entry (u,v), u itself is offered f[f[v]] (Sec. 3.3);
 *   - every vertex is offered its own grandparent f[f[u]] (shortcutting).
 * f then takes the values of f_next.  The loop ends after the first
 * iteration that leaves the grandparent vector f[f] unchanged (Sec. 3.4,
 * justified in Appendix A); the grandparent vector before the first
 * iteration is that of the initial f, i.e. iota.
 * ------------------------------------------------------------------------ */
int32_t oracle_fastsv_alg2(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t max_iters,
                           int32_t *f_out, int32_t *f_trace, int64_t *changed_trace, int32_t trace_cap) {
    if (n == 0) return 0;
    int32_t *f = f_out;
    int32_t *fn = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *gprev = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!fn || !gprev) { free(fn); free(gprev); return -2; }
    for (int32_t u = 0; u < n; ++u) { f[u] = u; fn[u] = u; }
    for (int32_t u = 0; u < n; ++u) gprev[u] = f[f[u]];
    int32_t it = 0;
    for (;;) {
        /* hooking of f[u] onto v's grandparent (stochastic, Sec. 3.2) */
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                fn[f[u]] = min32(fn[f[u]], f[f[v]]);
            }
        /* hooking of u itself onto v's grandparent (aggressive, Sec. 3.3) */
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                fn[u] = min32(fn[u], f[f[v]]);
            }
        /* shortcutting onto the own grandparent */
        for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);
        /* the next iteration reads what was written */
        memcpy(f, fn, (size_t)n * sizeof(int32_t));
        ++it;
        /* did any grandparent change? (Sec. 3.4) */
        int64_t changed = 0;
        for (int32_t u = 0; u < n; ++u) {
            int32_t g = f[f[u]];
            changed += (g != gprev[u]);
            gprev[u] = g;
        }
        record(n, it, f, changed, f_trace, changed_trace, trace_cap);
        if (changed == 0) break;
        if (max_iters > 0 && it >= max_iters) { it = -1; break; }
    }
    free(fn);
    free(gprev);
    return it;
}

/* ------------------------------------------------------------------------
 * O4: FastSV in the linear-algebra form of Sec. 4.1 (Algorithm 3), on dense
 * vectors.  State: the parent vector f (the input f_init, or iota), the
 * grandparent vector gf, its copy from the previous iteration (dup), the
 * neighbour minimum mngf and value, the parents as they were when gf was
 * last formed.  The algorithm initialises gf, dup and mngf with f itself.
 * One iteration:
 *   - mngf[i] is lowered to the smallest gf[j] over the stored entries (i,j)
 *     of row i: the matrix-vector product over the (select2nd, min)
 *     semiring, accumulated with MIN into the mngf kept from before; an
 *     empty row leaves mngf[i] as it is;
 *   - f[value[i]] is lowered to mngf[i] (stochastic hooking as an assign
 *     with a MIN accumulator; the target is the parent of i from the start
 *     of the iteration);
 *   - f[i] is lowered to mngf[i] (aggressive hooking) and to gf[i]
 *     (shortcutting), both element-wise minima;
 *   - value takes the new f, and gf[i] = f[value[i]] is the new grandparent;
 *   - the number of entries in which gf differs from dup is the termination
 *     count; dup then takes gf (the whole vector).
 * The loop ends when that count is zero.
 * ------------------------------------------------------------------------ */
int32_t oracle_fastsv_alg3(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t max_iters,
                           const int32_t *f_init, int32_t *f_out, int32_t *f_trace,
                           int64_t *changed_trace, int32_t trace_cap) {
    if (n == 0) return 0;
    int32_t *f = f_out;
    int32_t *gf = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *dup = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *mngf = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *value = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!gf || !dup || !mngf || !value) { free(gf); free(dup); free(mngf); free(value); return -2; }
    for (int32_t i = 0; i < n; ++i) f[i] = f_init ? f_init[i] : i;
    memcpy(gf, f, (size_t)n * sizeof(int32_t));
    memcpy(dup, gf, (size_t)n * sizeof(int32_t));
    memcpy(mngf, gf, (size_t)n * sizeof(int32_t));
    memcpy(value, f, (size_t)n * sizeof(int32_t));
    int32_t it = 0;
    for (;;) {
        /* neighbour minimum of the grandparents, then the hook of each parent */
        for (int32_t i = 0; i < n; ++i) {
            if (row_ptr[i + 1] == row_ptr[i]) continue;
            int32_t t = gf[col[row_ptr[i]]];
            for (int32_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e) t = min32(t, gf[col[e]]);
            mngf[i] = min32(mngf[i], t);
        }
        for (int32_t i = 0; i < n; ++i) f[value[i]] = min32(f[value[i]], mngf[i]);
        /* each vertex onto its neighbour minimum */
        for (int32_t i = 0; i < n; ++i) f[i] = min32(f[i], mngf[i]);
        /* each vertex onto its grandparent */
        for (int32_t i = 0; i < n; ++i) f[i] = min32(f[i], gf[i]);
        /* the new grandparents */
        memcpy(value, f, (size_t)n * sizeof(int32_t));
        for (int32_t i = 0; i < n; ++i) gf[i] = f[value[i]];
        /* count the grandparents that changed, and remember them */
        int64_t sum = 0;
        for (int32_t i = 0; i < n; ++i) sum += (dup[i] != gf[i]);
        memcpy(dup, gf, (size_t)n * sizeof(int32_t));
        ++it;
        record(n, it, f, sum, f_trace, changed_trace, trace_cap);
        if (sum == 0) break;
        if (max_iters > 0 && it >= max_iters) { it = -1; break; }
    }
    free(gf); free(dup); free(mngf); free(value);
    return it;
}

/* ------------------------------------------------------------------------
 * Algorithm 1 (simplified SV, Sec. 2.4) and the Sec. 3 optimisations.
 *
 * flags (bit set = optimisation on):
 *   1  grandparent hooking (Sec. 3.1): hook onto f[f[v]] instead of f[v]
 *   2  stochastic hooking  (Sec. 3.2): drop the root test f[u] == f[f[u]];
 *      hooking, shortcutting and the copy then happen in one Jacobi pass as
 *      in Alg. 2, with every update a min-assign
 *   4  aggressive hooking  (Sec. 3.3): f_next[u] <-min f[f[v]] (or f[v]
 *      without bit 1) for every (u,v)
 *   8  early termination   (Sec. 3.4): stop when f[f] is unchanged instead
 *      of when f is unchanged
 * flags = 0 is Alg. 1; flags = 15 is Alg. 2.
 *
 * Without bit 2 the iteration is Alg. 1's two phases.  First, conditional
 * hooking into f_next: for a stored entry (u,v), if f[u] is a root
 * (f[u] == f[f[u]]) and v's parent is smaller than it (f[v] < f[u]), f[u] is
 * hooked onto v's parent, or with bit 1 onto v's grandparent f[f[v]].
 * Sec. 3.1 changes only the vertex hooked onto and keeps the condition on
 * f[v]; since f[f[v]] <= f[v], the hook still lowers f[u].  Several edges
 * may hook the same root in one phase; the writes are resolved by taking the
 * minimum, which keeps the iterates deterministic (Sec. 2.4 and the MIN
 * accumulator of Sec. 4.1).  With bit 4 every u is also lowered to the
 * smallest such value over all of its entries, unconditionally (Sec. 3.3).
 * f <- f_next.  Second, shortcutting: f_next[u] <- f[f[u]] where f[u] is not
 * a root; f <- f_next.
 * With bit 2 the root test goes (Sec. 3.2), and the updates are Alg. 2's
 * min-assignments: removing the root test turns the hook into Alg. 2's
 * stochastic hook, and sv4 then differs from Alg. 2 only in its termination
 * test (Sec. 5.2 reports that early termination removes one iteration).
 * Termination without bit 8: f after the iteration equals f before it.
 * ------------------------------------------------------------------------ */
int32_t oracle_sv_variant(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t flags,
                          int32_t max_iters, int32_t *f_out, int32_t *f_trace,
                          int64_t *changed_trace, int32_t trace_cap) {
    if (n == 0) return 0;
    const int grand = flags & 1, stoch = flags & 2, aggr = flags & 4, early = flags & 8;
    int32_t *f = f_out;
    int32_t *fn = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *prev = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!fn || !prev) { free(fn); free(prev); return -2; }
    for (int32_t u = 0; u < n; ++u) { f[u] = u; fn[u] = u; }
    for (int32_t u = 0; u < n; ++u) prev[u] = early ? f[f[u]] : f[u];
    int32_t it = 0;
    for (;;) {
        if (stoch) {
            /* one Jacobi pass: hooking (no root test), aggressive, shortcut */
            for (int32_t u = 0; u < n; ++u)
                for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                    int32_t v = col[e];
                    int32_t h = grand ? f[f[v]] : f[v];
                    fn[f[u]] = min32(fn[f[u]], h);
                }
            if (aggr)
                for (int32_t u = 0; u < n; ++u)
                    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                        int32_t v = col[e];
                        int32_t h = grand ? f[f[v]] : f[v];
                        fn[u] = min32(fn[u], h);
                    }
            for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);
            memcpy(f, fn, (size_t)n * sizeof(int32_t));
        } else {
            /* phase 1: conditional hooking of roots */
            for (int32_t u = 0; u < n; ++u)
                for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                    int32_t v = col[e];
                    int32_t h = grand ? f[f[v]] : f[v];
                    if (f[u] == f[f[u]] && f[v] < f[u]) fn[f[u]] = min32(fn[f[u]], h);
                }
            if (aggr)
                for (int32_t u = 0; u < n; ++u)
                    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                        int32_t v = col[e];
                        int32_t h = grand ? f[f[v]] : f[v];
                        fn[u] = min32(fn[u], h);
                    }
            memcpy(f, fn, (size_t)n * sizeof(int32_t));
            /* phase 2: shortcutting */
            for (int32_t u = 0; u < n; ++u)
                if (f[u] != f[f[u]]) fn[u] = f[f[u]];
            memcpy(f, fn, (size_t)n * sizeof(int32_t));
        }
        ++it;
        int64_t changed = 0;
        for (int32_t u = 0; u < n; ++u) {
            int32_t x = early ? f[f[u]] : f[u];
            changed += (x != prev[u]);
            prev[u] = x;
        }
        record(n, it, f, changed, f_trace, changed_trace, trace_cap);
        if (changed == 0) break;
        if (max_iters > 0 && it >= max_iters) { it = -1; break; }
    }
    free(fn);
    free(prev);
    return it;
}

int32_t oracle_sv_alg1(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t max_iters,
                       int32_t *f_out, int32_t *f_trace, int64_t *changed_trace, int32_t trace_cap) {
    return oracle_sv_variant(n, row_ptr, col, 0, max_iters, f_out, f_trace, changed_trace, trace_cap);
}

/* ------------------------------------------------------------------------
 * Algorithm 2 with a single vector read and written in place (the
 * concurrent form mentioned in Sec. 2.4).  Sequential order here: for each
 * vertex u in increasing order, its edges in row order; then shortcutting in
 * vertex order.  The iterates depend on the order; the final labels do not.
 * Termination: a whole pass leaves f unchanged.  Then every vertex points to
 * a root (f[u] <= f[f[u]] <= f[u]) and f[u] <= f[f[v]] = f[v] on every edge,
 * so adjacent vertices share a root and each component is one star.
 * ------------------------------------------------------------------------ */
int32_t oracle_fastsv_async(int32_t n, const int32_t *row_ptr, const int32_t *col, int32_t max_iters,
                            int32_t *f_out) {
    if (n == 0) return 0;
    int32_t *f = f_out;
    for (int32_t u = 0; u < n; ++u) f[u] = u;
    int32_t it = 0;
    for (;;) {
        int64_t changed = 0;
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                int32_t h = f[f[v]];
                int32_t x = f[u];
                if (h < f[x]) { f[x] = h; ++changed; }
                if (h < f[u]) { f[u] = h; ++changed; }
            }
        for (int32_t u = 0; u < n; ++u)
            if (f[f[u]] < f[u]) { f[u] = f[f[u]]; ++changed; }
        ++it;
        if (changed == 0) break;
        if (max_iters > 0 && it >= max_iters) { it = -1; break; }
    }
    return it;
}
