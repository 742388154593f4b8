/*
 * fastsv.h -- connected components of undirected graphs on MI355X (gfx950)
 * with the FastSV method (Zhang, Azad, Hu, "FastSV: A Distributed-Memory
 * Connected Component Algorithm with Fast Convergence", arXiv 1910.05971).
 *
 * Problem (Sec. 1, Sec. 2.1): an undirected graph G(V,E) with vertices
 * 0..n-1.  Result: the parent vector f of Algorithm 2 at termination, in
 * which every vertex points to the smallest vertex of its connected
 * component (Sec. 3.4 and Appendix A); isolated vertices point to
 * themselves.
 *
 * Method per iteration (Algorithm 3, Sec. 4.1), all on the GPU:
 *   mngf = A (select2nd,min) gf, MIN-accumulated      -- SpMV (Sec. 4.1)
 *   f[f_start[u]] <-min mngf[u]                       -- stochastic hooking (Sec. 3.2)
 *   f[u] <-min mngf[u]                                -- aggressive hooking (Sec. 3.3)
 *   f[u] <-min gf[u]                                  -- shortcutting
 *   gf = f[f]; stop when gf is unchanged              -- early termination (Sec. 3.4)
 * with the SpMV replaced by a push over the changed entries of gf when they
 * are few (sparse frontier, Sec. 4.2 "Taking advantage of the sparsity").
 * The default mode keeps separate read and write vectors (Sec. 2.4), so the
 * iterates and the iteration count are deterministic and equal those of
 * Algorithm 2.
 *
 * Conventions for every entry point
 *   - Device pointers are plain hipMalloc'd (or torch-allocated) memory of
 *     the current device of the context.  The caller owns all buffers; the
 *     library keeps no pointer after a call returns.
 *   - Return value: FASTSV_OK or a negative fastsv_status.  Argument errors
 *     are detected before any launch; the output buffers are then untouched.
 *     On FASTSV_EHIP the outputs are unspecified.
 *   - A context is not thread-safe: use one per host thread.
 */
#ifndef FASTSV_H
#define FASTSV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FASTSV_OK = 0,
    FASTSV_EINVAL = -1,        /* bad argument (null pointer, n < 0, bad options, workspace too small) */
    FASTSV_ERANGE = -2,        /* validation found a column id outside [0,n) or a bad row_ptr */
    FASTSV_EOVERFLOW = -3,     /* sizes do not fit the int32 layout */
    FASTSV_ENOMEM = -4,        /* device or pinned host allocation failed */
    FASTSV_EHIP = -5,          /* a HIP runtime call failed */
    FASTSV_ENOTCONVERGED = -6, /* max_iters iterations ran without meeting the termination test */
    FASTSV_EBUSY = -7,         /* resource in use (serving: a request's admission copies are still
                                  in flight, see fastsv_server_cancel) */
    FASTSV_ESCRATCH = -8       /* the call needs more workspace than the library's fixed scratch
                                  memory holds (fastsv_cc_csr_noalloc) */
} fastsv_status;

typedef struct fastsv_ctx fastsv_ctx;

/* Solver options.  Zero-initialised options are NOT the defaults; start from
 * fastsv_default_opts(). */
typedef struct {
    int32_t max_iters;      /* > 0: stop after this many iterations with FASTSV_ENOTCONVERGED and
                               labels = f after that iteration; <= 0: no cap (the paper gives no
                               iteration bound, Sec. 2.4) */
    float frontier_tau;     /* sparse-frontier switch (Sec. 4.2): iteration k+1 pushes from the
                               changed grandparents of iteration k when their total degree is
                               below frontier_tau * nnz.  The degree sum is only taken when the
                               changed count c allows it (c <= frontier_tau * nnz and
                               c * nnz / n <= 2 * frontier_tau * nnz); otherwise the next pass
                               is dense.  0: always dense SpMV; >= 1: sparse whenever possible
                               (from iteration 2 on).  The labels and iterates do not depend on
                               it. */
    int32_t validate;       /* 1: check row_ptr (monotone, row_ptr[0] = 0, row_ptr[n] = nnz) and
                               every column id on the device before solving (FASTSV_ERANGE) */
    int32_t timing;         /* 1: time every kernel with HIP events on the call's stream
                               (fills fastsv_stats.ms_hook / ms_gp) */
    int32_t binned;         /* binned dense SpMV: the stored entries are regrouped once per call
                               by bins of consecutive vertices of their column (a 4-byte record per
                               entry, plus at most ((n-1) >> 16) + 1 per bin for the high bits of
                               the sources), and each dense iteration from the second on reduces
                               a bin in LDS while gathering gf in ascending order.  1 use it, 0
                               never, -1 automatic (the default: graphs with more than 2^22
                               vertices whose entries are at least 4 times those extra records).
                               Same iterates either way; not used when the graph needs more than
                               2048 bins. */
    int32_t bin_shift;      /* bin width 2^bin_shift vertices, 8..15; 0 = automatic: the fewest
                               bins that are a multiple of 256 (the CU count) with at most 40960
                               vertices each (the dense pass's 160 KB LDS window) */
    int32_t sv_flags;       /* convergence ablation (Sec. 5.2): which of the four changes of Sec. 3
                               that turn Algorithm 1 into Algorithm 2 are applied.  Bit 1 grandparent
                               hooking (Sec. 3.1), 2 stochastic hooking (3.2), 4 aggressive hooking
                               (3.3), 8 early termination on gf (3.4).  15 (the default) is FastSV;
                               0 is Algorithm 1; the paper's sv1..sv5 add them in this order
                               (0, 1, 3, 7, 15).  Other than 15: dense pull passes only, no batch
                               entry point (FASTSV_EINVAL there), the server ignores it. */
    int32_t mode;           /* 0 (default): Jacobi, f read and f_next written (Sec. 2.4): the
                               iterates and the iteration count are deterministic.  1: one parent
                               vector read and written concurrently (the form Sec. 2.4 notes is
                               also correct): passes of hooking with live grandparents and
                               shortcutting until a pass changes nothing; final labels exact,
                               iterates and pass count not reproducible.  Mode 1 needs
                               sv_flags = 15, runs dense pull passes only, and is refused by the
                               batch entry point.  stats.changed counts the values each pass
                               lowered. */
    int32_t trace;          /* 1: count on the device the global atomics that hooking issues
                               (fastsv_stats.atomics_issued and atomics[k]); every wave of a hooking
                               kernel then issues one more atomic of its own, so traced runs are
                               for measurement, not for timing.  Counted for sv_flags = 15 in
                               mode 0 (fastsv_cc_csr, _warm, _noalloc, _edges and the batch).
                               0 (default): not counted, atomics_issued = -1.
                               There is no option that records the iterates themselves: the
                               iterate f_k of any k is the result of a call with max_iters = k
                               (FASTSV_ENOTCONVERGED), and the statistics below record the
                               per-iteration figures. */
    int32_t bin_span;       /* records per lane and step of the binned dense pass: 8, 16 or 32;
                               0 = automatic (16 for bins of at least 2^17 records, else 8).
                               Same iterates either way. */
    int32_t admit_mb;       /* serving only: megabytes of graph data a server step admits once one
                               graph is in (1..4096; 0 = 128) */
} fastsv_opts;

#define FASTSV_TRACE_ITERS 64

/* Per-call statistics (host memory, filled when the call returns). */
typedef struct {
    int32_t iterations;            /* iterations executed, including the confirming one */
    int32_t dense_iterations;      /* iterations whose SpMV step was the dense pull */
    int32_t sparse_iterations;     /* iterations that pushed from the changed grandparents */
    int32_t num_tiles;             /* edge tiles of the dense kernel */
    int32_t binned_iterations;     /* dense iterations that ran the binned passes */
    int32_t num_bins;              /* bins of the binned layout (0 when it was not built) */
    int32_t bin_fused_first;       /* 1 if the layout's fill pass also performed the first
                                      iteration (that pass is then ms_hook[0]) */
    int32_t bin_span;              /* records per lane and step of the binned dense pass that
                                      ran (8, 16 or 32, as opts.bin_span; 0 if none) */
    float ms_bin_prepare;          /* time to build the binned layout; with bin_fused_first only
                                      its count and scan before the fill (opts.timing) */
    int64_t frontier_edges;        /* sum over sparse iterations of the pushed edge slots */
    int64_t alg_bytes;             /* algorithmic bytes of all executed iterations (4 B per int32
                                      read or written, each gather counted; with opts.trace also
                                      8 B per atomic, a read-modify-write) */
    int64_t atomics_issued;        /* global atomics issued by hooking over all iterations
                                      (opts.trace = 1), else -1 */
    double ms_total;               /* host wall time of the call */
    int64_t changed[FASTSV_TRACE_ITERS];  /* entries of gf changed in iteration k (k < 64) */
    int32_t sparse[FASTSV_TRACE_ITERS];   /* 1 if iteration k used the sparse push */
    int64_t pushed[FASTSV_TRACE_ITERS];   /* edge slots pushed in iteration k (sparse iterations; 0 if dense) */
    int64_t atomics[FASTSV_TRACE_ITERS];  /* global atomics of iteration k's hooking (opts.trace), else -1 */
    int64_t alg_hook[FASTSV_TRACE_ITERS]; /* algorithmic bytes of iteration k's hooking pass (the
                                             SpMV and the hooks, as in alg_bytes; without the
                                             grandparent pass and the layout build) */
    float ms_hook[FASTSV_TRACE_ITERS];    /* hooking kernel time of iteration k (opts.timing) */
    float ms_gp[FASTSV_TRACE_ITERS];      /* grandparent/termination kernel time, with the frontier list
                                             build when one follows (opts.timing) */
} fastsv_stats;

/* Default options: no iteration cap, frontier_tau = 0.05, no validation, no timing,
 * automatic binned layout, FastSV (sv_flags = 15), mode 0, no atomics count. */
fastsv_opts fastsv_default_opts(void);

/* Create a context on HIP device `device` (allocates pinned host counters).
 * *out is NULL on failure. */
int fastsv_create(fastsv_ctx **out, int device);
void fastsv_destroy(fastsv_ctx *ctx);

const char *fastsv_strerror(int status);

/*
 * Workspace bytes needed by fastsv_cc_csr for a graph with n vertices and nnz
 * stored entries: five int32[n] vectors (two parent buffers of the Jacobi
 * pair, the MIN-accumulated mngf, the frontier list and its edge offsets),
 * the dense kernel's tile table and counters, and for graphs with more than
 * 2^22 vertices the binned layout (about 4 B per stored entry; see
 * fastsv_opts.binned).  Returns 0 for invalid sizes.
 */
size_t fastsv_workspace_bytes(int32_t n, int64_t nnz);

/* Workspace bytes for the given options (binned and bin_shift change the
 * layout); returns 0 for invalid sizes or options. */
size_t fastsv_workspace_bytes_opts(int32_t n, int64_t nnz, const fastsv_opts *opts);

/*
 * Connected components of a graph in symmetric CSR form.
 *
 *   n          vertices (>= 0); n == 0 is a no-op
 *   nnz        stored entries = row_ptr[n] (0 <= nnz < 2^31)
 *   d_row_ptr  int32[n+1], nondecreasing, row_ptr[0] = 0, row_ptr[n] = nnz
 *   d_col_idx  int32[nnz], ids in [0,n).  The matrix must be symmetric: the
 *              method hooks only along stored entries (Alg. 3 multiplies by
 *              the symmetric adjacency matrix); an entry stored in one
 *              direction only does not connect its endpoints in both.
 *              Self loops and duplicate entries are allowed.
 *   d_labels   int32[n] output: labels[u] = min{w : w connected to u}
 *              (on FASTSV_ENOTCONVERGED: f after max_iters iterations)
 *   d_ws       workspace of at least fastsv_workspace_bytes_opts(n, nnz, opts) bytes,
 *              256-byte aligned; NULL lets the context allocate and keep one
 *   stream     HIP stream for all work; the call synchronises it once per
 *              iteration (it reads the termination count) and returns after
 *              the last kernel has finished
 *   opts       NULL for defaults
 *   stats      may be NULL
 */
int fastsv_cc_csr(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *d_row_ptr,
                  const int32_t *d_col_idx, int32_t *d_labels, void *d_ws, size_t ws_bytes,
                  hipStream_t stream, const fastsv_opts *opts, fastsv_stats *stats);

/*
 * The same from a given parent vector instead of the identity (Alg. 3 takes
 * the parent vector f as input and duplicates it into gf): restart after
 * edges were added, from the labels of the graph before.
 *
 *   d_f_init   int32[n], each f_init[u] a vertex of u's component in the graph
 *              with 0 <= f_init[u] <= u (labels or any iterate of an earlier
 *              solve of a subgraph qualify).  With opts.validate the bounds are
 *              checked (FASTSV_ERANGE); membership in u's component cannot be
 *              checked, and without it the labels are unspecified.  May alias
 *              d_labels (in-place restart).
 *   other arguments as fastsv_cc_csr; opts.sv_flags must be 15 (FASTSV_EINVAL).
 * From f_init the iterates follow Alg. 3 with that input; the first iteration
 * gathers gf like every later one.
 */
int fastsv_cc_csr_warm(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                       const int32_t *d_f_init, int32_t *d_labels, void *d_ws, size_t ws_bytes, hipStream_t stream,
                       const fastsv_opts *opts, fastsv_stats *stats);

/*
 * fastsv_cc_csr for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it).
 * The call allocates nothing: its workspace is a fixed array of
 * FASTSV_NOALLOC_SCRATCH_BYTES bytes that the library holds in device
 * memory, one per GPU, for as long as the process runs (its address on a
 * device is resolved once, when the first context on that device is
 * created).  Arguments, options, statistics and results are those of
 * fastsv_cc_csr with d_ws = NULL, and the same kernels run.
 *   FASTSV_ESCRATCH  fastsv_workspace_bytes_opts(n, nnz, opts) exceeds
 *                    FASTSV_NOALLOC_SCRATCH_BYTES (about 3 million vertices
 *                    with the plain passes; graphs that take the binned
 *                    layout need about 4 more bytes per stored entry); the
 *                    labels are then untouched.
 * Every call on a device uses that device's one array, and a call leaves its
 * contents behind (each call initialises what it reads).  Calls that overlap
 * in time on one device (from several host threads or contexts) race on it;
 * calls made one after another from one thread do not, since a call returns
 * after its last kernel has finished.
 */
#define FASTSV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fastsv_cc_csr_noalloc(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *d_row_ptr,
                          const int32_t *d_col_idx, int32_t *d_labels, hipStream_t stream,
                          const fastsv_opts *opts, fastsv_stats *stats);

/*
 * Edge-list entry (the problem statement of Sec. 1 and the edge form of
 * Algorithm 2): n vertices, m undirected edges given once each as
 * (d_src[i], d_dst[i]) in either orientation; self loops and repeats are
 * allowed.  The library builds the symmetric CSR on the device (edge (u,v)
 * stored in both rows) and then runs fastsv_cc_csr's loop on it, so labels,
 * iterates and iteration count equal those of the CSR entry on that matrix.
 *   m          0 <= 2m < 2^31
 *   d_ws       at least fastsv_edges_workspace_bytes(n, m) bytes (or NULL)
 */
size_t fastsv_edges_workspace_bytes(int32_t n, int64_t m);
int fastsv_cc_edges(fastsv_ctx *ctx, int32_t n, int64_t m, const int32_t *d_src, const int32_t *d_dst,
                    int32_t *d_labels, void *d_ws, size_t ws_bytes, hipStream_t stream,
                    const fastsv_opts *opts, fastsv_stats *stats);

/*
 * Batch of independent graphs solved in one pass of launches.  Graph g owns
 * the vertices [vtx_off[g], vtx_off[g+1]) of the concatenation and the entries
 * [edge_off[g], edge_off[g+1]); row_ptr is global over the concatenation
 * (row_ptr[vtx_off[g]] = edge_off[g]) and column ids are LOCAL to the graph
 * (0 .. n_g-1).  Each graph is solved exactly as alone: the batch runs
 * Algorithm 3 on the block-diagonal union with every vertex keeping a global
 * id, so no hook ever crosses graphs and every graph's iterates are those of
 * its solo run, shifted by vtx_off[g].
 *   num_graphs  G >= 0; total_n = vtx_off[G] < 2^31; total_nnz = edge_off[G] < 2^31
 *   d_vtx_off, d_edge_off  int32[G+1] device arrays, nondecreasing, starting at 0
 *   d_labels    int32[total_n] output, LOCAL ids: labels[vtx_off[g] + u] =
 *               smallest local vertex of u's component in graph g
 *   d_iters     int32[G] output: iterations graph g needs alone (-1 if it had
 *               not converged when max_iters stopped the batch; 0 for a graph
 *               without vertices)
 *   d_ws        at least fastsv_batch_workspace_bytes(total_n, total_nnz) bytes (or NULL)
 *   opts.validate also checks the offsets against row_ptr and the local ids.
 * The call returns after the last kernel has finished.
 */
size_t fastsv_batch_workspace_bytes(int32_t total_n, int64_t total_nnz);
int fastsv_cc_batch_csr(fastsv_ctx *ctx, int32_t num_graphs, int32_t total_n, int64_t total_nnz,
                        const int32_t *d_vtx_off, const int32_t *d_edge_off, const int32_t *d_row_ptr,
                        const int32_t *d_col_idx, int32_t *d_labels, int32_t *d_iters, void *d_ws,
                        size_t ws_bytes, hipStream_t stream, const fastsv_opts *opts, fastsv_stats *stats);

/*
 * Serving: continuous batching of connected-components requests.
 *
 * The server owns a device pool of max_vertices vertices and max_entries
 * stored entries.  A request (host CSR, copied at submit) is admitted first
 * come first served as soon as a slot, n+1 pool vertices and nnz pool
 * entries are free.  Each fastsv_server_step runs one iteration of the method
 * (Algorithm 3, dense or sparse-frontier SpMV as for fastsv_cc_csr) for ALL
 * resident graphs at once.  An admitted graph starts its first iteration in
 * the step that admits it when its copy is small and no request waits behind
 * it, otherwise in the first step after its copy has completed (a long copy
 * never holds up the resident graphs).  A graph leaves in the first step in
 * which none of its grandparents changed (termination test of Sec. 3.4 for
 * that graph): when that step returns, its local labels are in h_labels_out,
 * its iteration count in *h_iters_out, and its ticket is available from
 * fastsv_server_poll.  Graphs never exchange values, so every request gets
 * exactly the labels and the iteration count it would get alone.
 *
 * Threading: a server is driven from one host thread; it uses `stream` for
 * all device work and synchronises it inside fastsv_server_step.
 */
typedef struct fastsv_server fastsv_server;

typedef struct {
    int64_t submitted, admitted, completed, steps, dense_steps, sparse_steps, cancelled;
} fastsv_server_stats;

/* Device bytes the pool of a server with these limits occupies. */
size_t fastsv_server_pool_bytes(int32_t max_vertices, int64_t max_entries, int32_t max_slots);

/* max_vertices >= 1, 0 <= max_entries < 2^31, max_slots >= 1 resident graphs.
 * opts (NULL: defaults): frontier_tau picks dense or sparse per graph and
 * step; validate = 1 makes submit check every row pointer and column id on
 * the host (otherwise only row_ptr[0] and row_ptr[n], and the caller
 * guarantees a valid symmetric CSR).  FASTSV_ENOMEM if the pool cannot be
 * allocated. */
int fastsv_server_create(fastsv_ctx *ctx, int32_t max_vertices, int64_t max_entries, int32_t max_slots,
                         hipStream_t stream, const fastsv_opts *opts, fastsv_server **out);
void fastsv_server_destroy(fastsv_server *srv);

/* Queue a request: n vertices, nnz entries of a symmetric CSR in HOST memory
 * (page-locked memory makes the admission copy a plain DMA).  The arrays are
 * copied to the device at admission, so
 * h_row_ptr, h_col, h_labels_out (n ints) and h_iters_out (may be NULL) must
 * stay valid until the ticket is reported done.
 * FASTSV_ERANGE for a malformed CSR (see opts.validate); FASTSV_ENOMEM if the
 * graph can never fit the pool. */
int fastsv_server_submit(fastsv_server *srv, int32_t n, int64_t nnz, const int32_t *h_row_ptr,
                         const int32_t *h_col_idx, int32_t *h_labels_out, int32_t *h_iters_out,
                         uint64_t *ticket);

/* The same for a caller whose h_row_ptr and h_col_idx are page-locked host
 * memory mapped into the device address space at the same address (memory
 * from hipHostMalloc on ROCm): the per-request query of the pointers'
 * attributes is skipped.  Passing other memory here is undefined. */
int fastsv_server_submit_mapped(fastsv_server *srv, int32_t n, int64_t nnz, const int32_t *h_row_ptr,
                                const int32_t *h_col_idx, int32_t *h_labels_out, int32_t *h_iters_out,
                                uint64_t *ticket);

/* count requests in one call, as count calls of fastsv_server_submit (mapped
 * = 0) or fastsv_server_submit_mapped (mapped = 1); request i is (n[i],
 * nnz[i], h_row_ptr[i], h_col_idx[i], h_labels_out[i], &h_iters_out[i]) and
 * gets tickets[i] (h_iters_out and tickets may be NULL).  Stops at the first
 * request that is refused and returns its status; *n_accepted says how many
 * were queued. */
int fastsv_server_submit_batch(fastsv_server *srv, int32_t count, const int32_t *n, const int64_t *nnz,
                               const int32_t *const *h_row_ptr, const int32_t *const *h_col_idx,
                               int32_t *const *h_labels_out, int32_t *h_iters_out, uint64_t *tickets,
                               int32_t mapped, int32_t *n_accepted);

/* Admit what fits (at most opts.admit_mb megabytes of graph data per step
 * once one graph is in, so that admission copies overlap the iterations), run one iteration
 * for all running graphs, and deliver the ones that converged in it.  Reports
 * how many graphs are resident (admitted and not yet delivered, including
 * those whose copies are still in flight) and queued after it. */
int fastsv_server_step(fastsv_server *srv, int32_t *n_resident, int32_t *n_queued);

/* Cancel a request: a queued one is dropped at once; an admitted one leaves
 * at the next step, which frees its slot and pool ranges.  Its labels and
 * iteration count are not written and its ticket is never reported.
 * FASTSV_EBUSY: the request was admitted but its copies to the device are
 * still in flight; call again after a step.  FASTSV_EINVAL: no such request
 * (unknown, or already delivered). */
int fastsv_server_cancel(fastsv_server *srv, uint64_t ticket);

/* Up to cap tickets completed since the last poll, oldest first. */
int fastsv_server_poll(fastsv_server *srv, uint64_t *done, int32_t cap, int32_t *n_done);

int fastsv_server_get_stats(const fastsv_server *srv, fastsv_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* FASTSV_H */
