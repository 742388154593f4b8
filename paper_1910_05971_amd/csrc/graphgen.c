/*
 * Seeded synthetic graph generators and COO -> symmetric CSR conversion.
 *
 * This module is shared input plumbing: it produces the graphs that both the
 * HIP solver and the CPU oracle consume.  It holds none of the connected-
 * components arithmetic.  Every random number comes from a counter-based
 * generator, so any edge can be produced independently of the others and the
 * output is byte-identical for any thread count.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  The n-th output of a
 * SplitMix64 stream started at state s is mix(s + (n+1)*GAMMA), which makes
 * it counter-based by construction.  Integers are mapped to [0, n) with
 * Lemire's multiply-shift ((r32 * n) >> 32); probabilities are compared as
 * 32-bit integer thresholds floor(p * 2^32).
 *
 * Workload shapes stand in for the paper's datasets (Table 1): R-MAT for the
 * skewed web/social graphs, a percolated lattice for the high-diameter graphs
 * with many components, Erdos-Renyi for generic sparse graphs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Start state of stream `stream` under seed `seed`. */
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(mix64(seed + GAMMA) + (stream + 1) * GAMMA);
}

/* Output number `ctr` (0-based) of the stream. */
static inline uint64_t rng_at(uint64_t key, uint64_t ctr) {
    return mix64(key + (ctr + 1) * GAMMA);
}

static inline uint32_t lemire32(uint32_t r, uint32_t n) {
    return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

static inline double unit53(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* ---- exported raw RNG (tests check the stream against its definition) ---- */
uint64_t gg_rng_at(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return rng_at(stream_key(seed, stream), ctr);
}

/* ---- stable compaction of (src,dst) pairs with src != dst ----
 * Counts are taken in parallel per block; the copy runs block by block in
 * increasing order, which is safe in place because block t's output range
 * starts at or before its input range. */
static int64_t compact_loops(int32_t *src, int32_t *dst, int64_t m) {
    int nt = omp_get_max_threads();
    int64_t *cnt = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
    if (!cnt) return -1;
    int64_t chunk = (m + nt - 1) / nt;
#pragma omp parallel for num_threads(nt) schedule(static, 1)
    for (int t = 0; t < nt; ++t) {
        int64_t lo = (int64_t)t * chunk, hi = lo + chunk < m ? lo + chunk : m;
        int64_t c = 0;
        for (int64_t i = lo; i < hi; ++i) c += (src[i] != dst[i]);
        cnt[t + 1] = c;
    }
    for (int t = 0; t < nt; ++t) cnt[t + 1] += cnt[t];
    for (int t = 0; t < nt; ++t) {
        int64_t lo = (int64_t)t * chunk, hi = lo + chunk < m ? lo + chunk : m;
        int64_t w = cnt[t];
        for (int64_t i = lo; i < hi; ++i)
            if (src[i] != dst[i]) { src[w] = src[i]; dst[w] = dst[i]; ++w; }
    }
    int64_t total = cnt[nt];
    free(cnt);
    return total;
}

/*
 * Erdos-Renyi multigraph: draw `m` endpoint pairs uniform in [0,n); draw i
 * uses output i of the stream (high 32 bits -> u, low 32 bits -> v).  Self
 * loops are dropped without redrawing; duplicates are kept.  Returns the
 * number of kept edges (written to the front of src/dst, in draw order).
 */
int64_t gg_er_edges(uint64_t seed, uint64_t stream, int32_t n, int64_t m,
                    int32_t *src, int32_t *dst) {
    if (n <= 0 || m < 0) return 0;
    uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        uint64_t r = rng_at(key, (uint64_t)i);
        src[i] = (int32_t)lemire32((uint32_t)(r >> 32), (uint32_t)n);
        dst[i] = (int32_t)lemire32((uint32_t)r, (uint32_t)n);
    }
    return compact_loops(src, dst, m);
}

/*
 * Fisher-Yates shuffle of iota(n): for i = n-1 .. 1, swap perm[i] with
 * perm[j], j uniform in [0, i], drawn from output (n-1-i) of the stream.
 */
void gg_permutation(uint64_t seed, uint64_t stream, int32_t n, int32_t *perm) {
    uint64_t key = stream_key(seed, stream);
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int32_t i = n - 1; i >= 1; --i) {
        uint64_t r = rng_at(key, (uint64_t)(n - 1 - i));
        int32_t j = (int32_t)lemire32((uint32_t)(r >> 32), (uint32_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) without noise: edge i descends
 * `scale` levels, most significant bit first; at each level the quadrant
 * (0,0),(0,1),(1,0),(1,1) is chosen with 32-bit thresholds ta < tb < tc
 * (cumulative a, a+b, a+b+c).  Level pair (2k, 2k+1) of edge i uses output
 * i*ceil(scale/2)+k of stream 0 (high half for level 2k, low half for 2k+1).
 * Ids are then relabelled through a Fisher-Yates permutation (stream 1), and
 * self loops are dropped; duplicates are kept.
 */
int64_t gg_rmat_edges(uint64_t seed, int32_t scale, int64_t m, uint32_t ta, uint32_t tb,
                      uint32_t tc, int32_t permute, int32_t *src, int32_t *dst) {
    if (scale <= 0 || scale > 30 || m < 0) return 0;
    int32_t n = (int32_t)1 << scale;
    uint64_t key = stream_key(seed, 0);
    int64_t per = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        uint32_t u = 0, v = 0;
        for (int32_t lv = 0; lv < scale; ++lv) {
            uint64_t r64 = rng_at(key, (uint64_t)(i * per + lv / 2));
            uint32_t r = (lv & 1) ? (uint32_t)r64 : (uint32_t)(r64 >> 32);
            uint32_t bu, bv;
            if (r < ta) { bu = 0; bv = 0; }
            else if (r < tb) { bu = 0; bv = 1; }
            else if (r < tc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
    if (permute) {
        int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        if (!perm) return -1;
        gg_permutation(seed, 1, n, perm);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) { src[i] = perm[src[i]]; dst[i] = perm[dst[i]]; }
        free(perm);
    }
    return compact_loops(src, dst, m);
}

/*
 * Bond-percolated rows x cols 4-neighbour lattice.  Vertex (r,c) has
 * row-major id r*cols+c.  Bond b enumerates right bonds first
 * ((r,c)-(r,c+1), b = r*(cols-1)+c) and then down bonds
 * ((r,c)-(r+1,c), b = R + r*cols + c with R = rows*(cols-1)); bond b is kept
 * when the high 32 bits of output b of stream 0 are below `tp`.  If `permute`,
 * ids are relabelled through a Fisher-Yates permutation (stream 1).
 * Returns the number of kept bonds; src/dst need rows*(cols-1)+(rows-1)*cols
 * slots.
 */
int64_t gg_grid_edges(uint64_t seed, int32_t rows, int32_t cols, uint32_t tp, int32_t permute,
                      int32_t *src, int32_t *dst) {
    if (rows <= 0 || cols <= 0) return 0;
    uint64_t key = stream_key(seed, 0);
    int64_t R = (int64_t)rows * (cols - 1);
    int64_t D = (int64_t)(rows - 1) * cols;
    int64_t nb = R + D;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        int64_t a, c;
        if (b < R) { int64_t r = b / (cols - 1), cc = b % (cols - 1); a = r * cols + cc; c = a + 1; }
        else { int64_t q = b - R; a = q; c = q + cols; }
        uint32_t rv = (uint32_t)(rng_at(key, (uint64_t)b) >> 32);
        if (rv < tp) { src[b] = (int32_t)a; dst[b] = (int32_t)c; }
        else { src[b] = -1; dst[b] = -1; }
    }
    if (permute) {
        int32_t n = rows * cols;
        int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        if (!perm) return -1;
        gg_permutation(seed, 1, n, perm);
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < nb; ++b)
            if (src[b] >= 0) { src[b] = perm[src[b]]; dst[b] = perm[dst[b]]; }
        free(perm);
    }
    return compact_loops(src, dst, nb); /* removed bonds have src == dst == -1 */
}

/* ---- in-place row sort (median-of-three quicksort + insertion sort) ---- */
static void isort(int32_t *a, int64_t n) {
    for (int64_t i = 1; i < n; ++i) {
        int32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
        a[j + 1] = x;
    }
}

static void qsort_i32(int32_t *a, int64_t n) {
    while (n > 24) {
        int32_t x = a[0], y = a[n / 2], z = a[n - 1];
        int32_t p = (x < y) ? ((y < z) ? y : (x < z ? z : x)) : ((x < z) ? x : (y < z ? z : y));
        int64_t i = 0, j = n - 1;
        for (;;) {
            while (a[i] < p) ++i;
            while (a[j] > p) --j;
            if (i >= j) break;
            int32_t t = a[i]; a[i] = a[j]; a[j] = t;
            ++i; --j;
        }
        /* [0, j] <= p <= [j+1, n) ; recurse on the smaller part */
        int64_t left = j + 1, right = n - (j + 1);
        if (left < right) { qsort_i32(a, left); a += left; n = right; }
        else { qsort_i32(a + left, right); n = left; }
    }
    isort(a, n);
}

/*
 * Symmetric CSR from an undirected edge list: edge (u,v) stores v in row u and
 * u in row v (a self loop (u,u) is stored twice in row u).  Rows are sorted
 * ascending, so the result does not depend on thread scheduling.
 * row_ptr has n+1 entries; col has 2*m entries.  Returns 0, or -1 when an id
 * is outside [0,n) or the entry count does not fit int32.
 */
int32_t gg_csr_from_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                          int32_t *row_ptr, int32_t *col) {
    if (2 * m > 2147483647LL) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < m; ++i)
        bad |= (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n);
    if (bad) return -1;
    int32_t *deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!deg) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
#pragma omp atomic
        deg[src[i]]++;
#pragma omp atomic
        deg[dst[i]]++;
    }
    row_ptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) row_ptr[v + 1] = row_ptr[v] + deg[v];
    /* deg becomes the per-row write cursor */
#pragma omp parallel for schedule(static)
    for (int32_t v = 0; v < n; ++v) deg[v] = row_ptr[v];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = src[i], v = dst[i], pu, pv;
#pragma omp atomic capture
        pu = deg[u]++;
#pragma omp atomic capture
        pv = deg[v]++;
        col[pu] = v;
        col[pv] = u;
    }
    free(deg);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t v = 0; v < n; ++v) qsort_i32(col + row_ptr[v], (int64_t)row_ptr[v + 1] - row_ptr[v]);
    return 0;
}

/*
 * Sizes for a batch of `g` Erdos-Renyi graphs (stream g of `seed` for graph g):
 * n_g = floor(64 * 1024^U1), so log n_g is uniform over [64, 65536);
 * average degree d_g = 2 + 30*U2 (uniform in [2,32]); edge draws
 * m_g = round(n_g * d_g / 2).  U1, U2 are outputs 0 and 1 of the graph's size
 * stream (stream 2*g of seed+1000003); the edges use stream g of `seed`.
 */
void gg_batch_sizes(uint64_t seed, int32_t g, int32_t *n_out, int64_t *m_out) {
    for (int32_t i = 0; i < g; ++i) {
        uint64_t key = stream_key(seed + 1000003ULL, 2 * (uint64_t)i);
        double u1 = unit53(rng_at(key, 0)), u2 = unit53(rng_at(key, 1));
        int32_t n = (int32_t)floor(64.0 * exp2(10.0 * u1));
        if (n < 64) n = 64;
        if (n > 65535) n = 65535;
        double d = 2.0 + 30.0 * u2;
        n_out[i] = n;
        m_out[i] = llround((double)n * d / 2.0);
    }
}

/* Uniform double in [0,1) from output `ctr` of stream `stream`. */
double gg_uniform(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return unit53(rng_at(stream_key(seed, stream), ctr));
}

int32_t gg_num_threads(void) { return omp_get_max_threads(); }
