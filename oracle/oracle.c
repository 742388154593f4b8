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
 *   oracle_fastsv_alg2    Algorithm 2 (FastSV) step by step, Jacobi f / f_next
 *   oracle_fastsv_alg3    Algorithm 3 (FastSV in GraphBLAS) call by call
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
 * O3: Algorithm 2 (FastSV), Sec. 3.
 *   init:   f[u] = f_next[u] = u                                  (Alg. 2 init)
 *   step 1: stochastic hooking  f_next[f[u]] <-min f[f[v]]  for (u,v) in E  (Sec. 3.2)
 *   step 2: aggressive hooking  f_next[u]    <-min f[f[v]]  for (u,v) in E  (Sec. 3.3)
 *   step 3: shortcutting        f_next[u]    <-min f[f[u]]  for u in V
 *   f <- f_next (a copy: both vectors hold the same values afterwards)
 *   until f[f] is unchanged (early termination, Sec. 3.4): the grandparent
 *   vector after the iteration is compared with the one before it, the first
 *   "before" being f[f] of the initial f, i.e. iota.
 * All reads in steps 1-3 see f as it was at the start of the iteration; all
 * writes go to f_next (Sec. 2.4, deterministic Jacobi form).
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
        /* step 1: stochastic hooking */
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                fn[f[u]] = min32(fn[f[u]], f[f[v]]);
            }
        /* step 2: aggressive hooking */
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t v = col[e];
                fn[u] = min32(fn[u], f[f[v]]);
            }
        /* step 3: shortcutting */
        for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);
        /* f <- f_next */
        memcpy(f, fn, (size_t)n * sizeof(int32_t));
        ++it;
        /* termination test on the grandparent vector */
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
 * O4: Algorithm 3 (FastSV expressed with GraphBLAS calls), Sec. 4.1.
 * Each call is written out on dense vectors:
 *   gf = dup(f); dup = dup(gf); mngf = dup(gf); value = f (extractTuples)
 *   repeat
 *     mxv(mngf, MIN, (select2nd,min), A, gf):
 *         t[i] = min over stored A(i,j) of gf[j]  (absent for an empty row);
 *         mngf[i] = min(mngf[i], t[i])
 *     assign(f, MIN, mngf, value):      f[value[i]] = min(f[value[i]], mngf[i])
 *     eWiseMult(f, MIN, f, mngf):       f[i] = min(f[i], mngf[i])
 *     eWiseMult(f, MIN, f, gf):         f[i] = min(f[i], gf[i])
 *     extractTuples(value, f):          value = f
 *     extract(gf, f, value):            gf[i] = f[value[i]]
 *     eWiseMult(diff, ISNE, dup, gf); reduce(sum, +, diff)
 *     assign(dup, gf)   (the listing prints "gp"; it is the vector gf)
 *   until sum == 0
 * `f_init` (may be NULL for iota) is the input parent vector of Alg. 3.
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
        /* Step 1: stochastic hooking = mxv then assign */
        for (int32_t i = 0; i < n; ++i) {
            if (row_ptr[i + 1] == row_ptr[i]) continue;
            int32_t t = gf[col[row_ptr[i]]];
            for (int32_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e) t = min32(t, gf[col[e]]);
            mngf[i] = min32(mngf[i], t);
        }
        for (int32_t i = 0; i < n; ++i) f[value[i]] = min32(f[value[i]], mngf[i]);
        /* Step 2: aggressive hooking */
        for (int32_t i = 0; i < n; ++i) f[i] = min32(f[i], mngf[i]);
        /* Step 3: shortcutting */
        for (int32_t i = 0; i < n; ++i) f[i] = min32(f[i], gf[i]);
        /* Step 4: grandparents */
        memcpy(value, f, (size_t)n * sizeof(int32_t));
        for (int32_t i = 0; i < n; ++i) gf[i] = f[value[i]];
        /* Step 5: termination */
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
 * Without bit 2 the iteration is Alg. 1's two phases: conditional hooking
 * (only when f[u] is a root and the hook value is smaller than f[u]) into
 * f_next, f <- f_next, then shortcutting f_next[u] <- f[f[u]] where f[u] is
 * not a root, f <- f_next.  Several edges may hook the same root in one
 * phase; the writes are resolved by taking the minimum, which keeps the
 * iterates deterministic (Sec. 2.4 and the MIN accumulator of Sec. 4.1).
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
                    if (f[u] == f[f[u]] && h < f[u]) fn[f[u]] = min32(fn[f[u]], h);
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
