// FastSV connected components: gfx950 kernels and the C ABI of fastsv.h.
//
// Method: Algorithm 3 of Zhang, Azad, Hu (arXiv 1910.05971), executed with
// separate read/write parent vectors (Sec. 2.4).  State entering iteration k:
//   F  = f_{k-1}            parent vector (read only during the iteration)
//   G  = f_{k-1}[f_{k-1}]   grandparents (also the caller's label buffer)
//   M  = mngf, MIN-accumulated across iterations (Alg. 3 keeps it)
//   Fn = write buffer, seeded with G by the previous grandparent pass
// One iteration is two kernels:
//   hook (dense k_hook_dense or sparse k_hook_sparse):
//       m[u] = min_{v in N(u)} G[v]; M[u] <-min m[u]        SpMV, (select2nd,min)
//       if m[u] < G[u]:  Fn[u] <-min m[u]                    aggressive hooking
//                        Fn[F[u]] <-min m[u]                 stochastic hooking
//   k_grandparent:  G_k[u] = Fn[Fn[u]], count and list the u with
//       G_k[u] != G_{k-1}[u] (termination test of Sec. 3.4), and seed the next
//       write buffer (the old F buffer) with G_k.
// Shortcutting (Fn[u] <-min G[u]) is the seed of Fn: G[u] <= F[u], so the
// seed already equals min(F[u], G[u]).  The filter m[u] < G[u] is exact:
// Fn[u] <= G[u] and Fn[F[u]] <= G[F[u]] <= F[F[u]] = G[u] hold before any hook
// (f[x] <= x, Appendix A), so a hook with m[u] >= G[u] changes nothing.
// Values of M accumulated in earlier iterations never beat the current hook
// targets (f only decreases and f_{k-1}[u] <= M[u] after the aggressive hook
// of the previous iteration), so the hooks use the fresh m[u].
//
// Sparse frontier (Sec. 4.2): let D = {v : G_{k-1}[v] != G_{k-2}[v]}.  Every
// other neighbour value is already folded into M, and G never increases, so
// min(M[u], min_{v in N(u) & D} G[v]) equals the dense M update.  A vertex whose
// M did not drop has m[u] >= M_{k-1}[u] >= F[u] >= G[u], i.e. only no-op hooks.
// Hence pushing G[v] from v in D along its row and hooking where M dropped
// gives exactly the dense iterate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "fastsv.h"
#include "engine.h"
#include "kernels.h"
#include "binned.h"

namespace fsv {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    int64_t n, nnz, ntiles;
    bool bin;        // binned dense pass arrays present
    BinDiv bdiv;  // bin width W and the divisor for u / W
    int nbins, nchunks, chunk_tiles;
    int64_t bin_scan_len;
    int bin_cap;     // records the binned layout can hold (entries plus markers)
    size_t off_F0, off_F1, off_M, off_frontier, off_eoff, off_fmask, off_tiles, off_ctr;
    size_t off_brec, off_bck, off_bcnt, off_bsums;
    size_t total;
};

// Dense-pass choices that change the workspace layout.
struct LayoutOpts {
    int bin_mode = -1;   // binned: -1 automatic, 0 off, 1 forced
    int bin_shift = 0;   // 0 = automatic bin width
};

// the batch entry point uses the plain passes (column ids are graph-local)
LayoutOpts batch_layout_opts() {
    LayoutOpts lo;
    lo.bin_mode = 0;
    return lo;
}

LayoutOpts layout_opts(const fastsv_opts &o) {
    LayoutOpts lo;
    lo.bin_mode = o.binned;
    lo.bin_shift = o.bin_shift;
    if (o.sv_flags != kSvFastSV || o.mode == kModeAsync) lo.bin_mode = 0;  // ablation variants and async: plain passes only
    return lo;
}

Layout layout_for(int64_t n, int64_t nnz, const LayoutOpts &lo = LayoutOpts()) {
    Layout L{};
    L.n = n;
    L.nnz = nnz;
    L.ntiles = (nnz + kTileEntries - 1) / kTileEntries;
    size_t p = 0;
    auto take = [&](size_t bytes) { size_t o = p; p += align256(bytes > 0 ? bytes : 1); return o; };
    const size_t vec = sizeof(int) * (size_t)(n > 0 ? n : 1);
    L.off_F0 = take(vec);
    L.off_F1 = take(vec);
    L.off_M = take(vec);
    L.off_frontier = take(vec);
    L.off_eoff = take(vec);
    L.off_fmask = take(sizeof(unsigned long long) * (size_t)((n + kWave - 1) / kWave));
    L.off_tiles = take(sizeof(Tile) * (size_t)L.ntiles);
    L.off_ctr = take(sizeof(Counters));
    // binned dense passes: one 32-bit record per stored entry and per marker
    // (see engine.h), the checkpoints of the high source bits, the
    // (bin, chunk) counts and their scan
    // automatic width: the fewest bins that are a multiple of the CU count
    // (the dense pass then runs whole rounds of one workgroup per CU) with at
    // most kBinRowsMax rows each
    const int64_t nb_auto =
        (int64_t)kNumCUs * std::max<int64_t>(1, (n + (int64_t)kNumCUs * kBinRowsMax - 1) / ((int64_t)kNumCUs * kBinRowsMax));
    const int W = lo.bin_shift > 0 ? 1 << lo.bin_shift : (int)std::max<int64_t>(1, (n + nb_auto - 1) / nb_auto);
    const int64_t nb = (n + W - 1) / W;
    L.bin = nnz > 0 && nb <= kMaxBins && (lo.bin_mode == 1 || (lo.bin_mode == -1 && n > kBinAutoMinN));
    if (L.bin) {
        L.bdiv = make_bindiv(W);
        L.nbins = (int)nb;
        // chunks of whole rounds of tiles: at least kBinChunkTilesMin tiles, so that a
        // (chunk, bin) run spans whole cache lines, and few enough for the counter budget
        const int64_t rounds = (L.ntiles + kFillThreads / kWave - 1) / (kFillThreads / kWave);
        int64_t ct = (kFillThreads / kWave) * ((nb * rounds + kBinMaxCounts - 1) / kBinMaxCounts);
        if (ct < kBinChunkTilesMin) ct = kBinChunkTilesMin;
        L.chunk_tiles = (int)ct;
        L.nchunks = (int)((L.ntiles + ct - 1) / ct);
        L.bin_scan_len = nb * L.nchunks + 1;
        // markers: per bin, one per value of the high source bits, at most
        // ((n - 1) >> kSrcLoBits) + 1 (a malformed row_ptr may ask for more;
        // the fill drops writes beyond the capacity)
        const int64_t markers = nb * (((n - 1) >> kSrcLoBits) + 1);
        const int64_t cap = nnz + markers;
        // positions are int; the automatic mode also skips graphs so sparse
        // that markers would be more than a quarter of the records
        if (cap + (int64_t)kBinSpanWide * 1024 >= INT32_MAX || (lo.bin_mode == -1 && 4 * markers > nnz)) {
            L.bin = false;
            L.nbins = L.nchunks = 0;
        } else {
            L.bin_cap = (int)cap;
            L.off_brec = take(sizeof(unsigned) * (size_t)cap);
            L.off_bck = take(sizeof(int) * (size_t)((cap >> kBinCkShift) + 1));
            L.off_bcnt = take(sizeof(int) * (size_t)L.bin_scan_len);
            L.off_bsums = take(sizeof(int) * (size_t)(grid_for(L.bin_scan_len, kScanBlock) + 1));
        }
    }
    L.total = p;
    return L;
}

struct Workspace {
    int *F[2];
    int *M;
    int *frontier;
    int *eoff;
    unsigned long long *fmask;  // changed vertices of the last grandparent pass, one bit each
    Tile *tiles;
    Counters *ctr;
    unsigned *brec;
    int *bck;
    int *bcnt, *bsums;
};

Workspace carve(void *base, const Layout &L) {
    char *p = static_cast<char *>(base);
    Workspace w{};
    w.F[0] = reinterpret_cast<int *>(p + L.off_F0);
    w.F[1] = reinterpret_cast<int *>(p + L.off_F1);
    w.M = reinterpret_cast<int *>(p + L.off_M);
    w.frontier = reinterpret_cast<int *>(p + L.off_frontier);
    w.eoff = reinterpret_cast<int *>(p + L.off_eoff);
    w.fmask = reinterpret_cast<unsigned long long *>(p + L.off_fmask);
    w.tiles = reinterpret_cast<Tile *>(p + L.off_tiles);
    w.ctr = reinterpret_cast<Counters *>(p + L.off_ctr);
    if (L.bin) {
        w.brec = reinterpret_cast<unsigned *>(p + L.off_brec);
        w.bck = reinterpret_cast<int *>(p + L.off_bck);
        w.bcnt = reinterpret_cast<int *>(p + L.off_bcnt);
        w.bsums = reinterpret_cast<int *>(p + L.off_bsums);
    }
    return w;
}

// Exclusive scan of x[0..len) in place; the total lands in sums[m], m = number
// of scan blocks.
void scan_inplace(int *x, int64_t len, int *sums, hipStream_t stream) {
    const int m = grid_for(len, kScanBlock);
    hipLaunchKernelGGL(k_scan_reduce, dim3(m), dim3(kScanThreads), 0, stream, x, len, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, stream, sums, m);
    hipLaunchKernelGGL(k_scan_down, dim3(m), dim3(kScanThreads), 0, stream, x, len, sums, x);
}

// Build the binned layout (count, scan, fill).  With M and Fn given, the fill
// also performs the first iteration's hooking (the grandparent vector is then
// still the identity).
void bin_prepare(const Layout &L, const Workspace &w, int n, const int *rp, const int *col, hipStream_t stream,
                 int *M = nullptr, int *Fn = nullptr, hipEvent_t before_fill = nullptr,
                 unsigned long long *atom = nullptr) {
    hipLaunchKernelGGL(k_bin_count, dim3(L.nchunks), dim3(kBinThreads), 0, stream, L.nnz, n, col, w.tiles,
                       (int)L.ntiles, L.bdiv, L.nbins, L.nchunks, L.chunk_tiles, w.bcnt);
    scan_inplace(w.bcnt, L.bin_scan_len, w.bsums, stream);
    if (before_fill) (void)hipEventRecord(before_fill, stream);
    const size_t lds = 3 * sizeof(int) * (size_t)L.nbins;
    if (M)
        hipLaunchKernelGGL(k_bin_fill<true>, dim3(L.nchunks), dim3(kFillThreads), lds, stream, w.tiles, (int)L.ntiles,
                           n, rp, col, L.bdiv, L.nbins, L.nchunks, L.chunk_tiles, w.bcnt, L.bin_cap, w.brec, w.bck,
                           M, Fn, atom);
    else
        hipLaunchKernelGGL(k_bin_fill<false>, dim3(L.nchunks), dim3(kFillThreads), lds, stream, w.tiles, (int)L.ntiles,
                           n, rp, col, L.bdiv, L.nbins, L.nchunks, L.chunk_tiles, w.bcnt, L.bin_cap, w.brec, w.bck,
                           nullptr, nullptr, nullptr);
}

// ---- launch wrappers ----
// The iteration counters to the host's mapped mirror (read after the
// stream's synchronisation): one small kernel instead of a copy command.
void launch_publish(hipStream_t s, const IterCounters *src, IterCounters *dst) {
    hipLaunchKernelGGL(k_publish_counters, dim3(1), dim3(64), 0, s, src, dst);
}

void launch_init(hipStream_t s, int n, int *F, int *Fn, int *G, int *M, int base) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_init, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, F, Fn, G, M, base);
}

void launch_build_tiles(hipStream_t s, int nrows, int r_begin, int e_begin, int e_end, const int *rp, Tile *tiles) {
    if (nrows <= 0 || e_end <= e_begin) return;
    hipLaunchKernelGGL(k_build_tiles, dim3(grid_for(nrows, 256)), dim3(256), 0, s, nrows, r_begin, e_begin, e_end, rp,
                       tiles);
}

void launch_dense(hipStream_t s, int mode, const Tile *tiles, int ntiles, const int *rp, const int *col,
                  const int *vbase, const int *F, int *Fn, const int *G, int *M, unsigned long long *atom) {
    if (ntiles <= 0) return;
    const dim3 grid(grid_for(ntiles, kHookWaves)), block(kWave * kHookWaves);
    switch (mode) {
        case kDenseIota:
            hipLaunchKernelGGL((k_tile_reduce<kIota>), grid, block, 0, s, tiles, ntiles, rp, col, vbase, F, Fn, G, M, 0,
                               atom, SrvTiles{});
            break;
        case kDenseGather:
            hipLaunchKernelGGL((k_tile_reduce<kGather>), grid, block, 0, s, tiles, ntiles, rp, col, vbase, F, Fn, G, M,
                               0, atom, SrvTiles{});
            break;
        case kDenseBaseIota:
            hipLaunchKernelGGL((k_tile_reduce<kBaseIota>), grid, block, 0, s, tiles, ntiles, rp, col, vbase, F, Fn, G,
                               M, 0, atom, SrvTiles{});
            break;
        default:
            hipLaunchKernelGGL((k_tile_reduce<kBaseGather>), grid, block, 0, s, tiles, ntiles, rp, col, vbase, F, Fn,
                               G, M, 0, atom, SrvTiles{});
            break;
    }
}

void launch_sparse(hipStream_t s, const int *frontier, const int *eoff, int fcnt, int edges, const int *rp,
                   const int *col, const int *vbase, const int *F, int *Fn, const int *G, int *M,
                   unsigned long long *atom) {
    if (edges <= 0) return;
    const dim3 grid(grid_for(edges, kPushSlots)), block(kPushThreads);
    const IterCounters *none = nullptr;
    const int *no_skip = nullptr;
    if (vbase)
        hipLaunchKernelGGL(k_hook_sparse<true>, grid, block, 0, s, frontier, eoff, fcnt, edges, none, rp, col, vbase,
                           F, Fn, G, M, no_skip, 0, atom);
    else
        hipLaunchKernelGGL(k_hook_sparse<false>, grid, block, 0, s, frontier, eoff, fcnt, edges, none, rp, col, vbase,
                           F, Fn, G, M, no_skip, 0, atom);
}

void launch_sparse_dev(hipStream_t s, const IterCounters *counts, int max_blocks, const int *frontier,
                       const int *eoff, const int *rp, const int *col, const int *vbase, const int *F, int *Fn,
                       const int *G, int *M, const int *skip_mark, int skip_val) {
    const dim3 grid(max_blocks > 0 ? max_blocks : 1), block(kPushThreads);
    unsigned long long *no_count = nullptr;
    if (vbase)
        hipLaunchKernelGGL(k_hook_sparse<true>, grid, block, 0, s, frontier, eoff, 0, 0, counts, rp, col, vbase, F,
                           Fn, G, M, skip_mark, skip_val, no_count);
    else
        hipLaunchKernelGGL(k_hook_sparse<false>, grid, block, 0, s, frontier, eoff, 0, 0, counts, rp, col, vbase, F,
                           Fn, G, M, skip_mark, skip_val, no_count);
}

void launch_zero_iter(hipStream_t s, IterCounters *ic) {
    hipLaunchKernelGGL(k_zero_iter_counters, dim3(1), dim3(64), 0, s, ic);
}

void launch_grandparent(hipStream_t s, int n, const int *Fn, int *G, int *next_fn, const int *rp, int *frontier,
                        int *eoff, IterCounters *ic, int write_frontier, int *lastk, int iter, const int *vbase,
                        int *gedge, unsigned long long *fmask, int u_begin) {
    u_begin -= u_begin % kGpBlockVerts;
    if (n <= u_begin) return;
    hipLaunchKernelGGL(k_grandparent, dim3(grid_for(n - u_begin, kGpBlockVerts)), dim3(kGpThreads), 0, s, u_begin, n,
                       Fn, G, next_fn, rp, frontier, eoff, ic, write_frontier, lastk, iter, vbase, gedge, fmask);
}

void launch_frontier_from_mask(hipStream_t s, int n, const unsigned long long *fmask, const int *rp, int *frontier,
                               int *eoff, IterCounters *fb) {
    if (n <= 0) return;
    launch_zero_iter(s, fb);
    hipLaunchKernelGGL(k_frontier_from_mask, dim3(grid_for(n, kGpBlockVerts)), dim3(kGpThreads), 0, s, n, fmask, rp,
                       frontier, eoff, fb);
}

void launch_fill_iota(hipStream_t s, int n, int *x) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, x);
}

void launch_fill(hipStream_t s, int n, int *x, int v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, n, x, v);
}

void launch_srv_settle(hipStream_t s, int nrun, int blocks, const SrvRun *run, const int *blk_off, int step,
                       int *lastk, int *gedge, int *h_flag, int *h_edges, int *h_out, int *F0, int *F1, int *G,
                       int *M, int *vbase, IterCounters *next_ic) {
    if (nrun <= 0 || blocks <= 0) return;
    hipLaunchKernelGGL(k_srv_settle, dim3(blocks), dim3(256), 0, s, nrun, run, blk_off, step, lastk, gedge, h_flag,
                       h_edges, h_out, F0, F1, G, M, vbase, next_ic);
}

void launch_srv_dense(hipStream_t s, int ndense, int total_tiles, const SrvNew *desc, const int *tile_off,
                      const Tile *pool_tiles, int *mark, int step, const int *rp, const int *col, const int *vbase,
                      const int *F, int *Fn, const int *G, int *M) {
    if (ndense <= 0 || total_tiles <= 0) return;
    const dim3 grid(grid_for(total_tiles, kHookWaves)), block(kWave * kHookWaves);
    hipLaunchKernelGGL((k_tile_reduce<kSrvGather>), grid, block, 0, s, pool_tiles, total_tiles, rp, col, vbase, F, Fn,
                       G, M, 0, (unsigned long long *)nullptr, SrvTiles{ndense, desc, tile_off, mark, step});
}

void launch_srv_place(hipStream_t s, int nchunks, const PlaceChunk *chunks, const SrvNew *desc,
                      const int *const *srcs, int *rp, int *col, int *F0, int *F1, int *G, int *M, int *vbase,
                      int *lastk, Tile *tiles) {
    if (nchunks <= 0) return;
    hipLaunchKernelGGL(k_srv_place, dim3(nchunks), dim3(256), 0, s, chunks, desc, srcs, rp, col, F0, F1, G, M, vbase,
                       lastk, tiles);
}


}  // namespace fsv

using namespace fsv;

struct fastsv_ctx {
    int device = 0;
    Counters *host_ctr = nullptr;  // pinned, mapped: the kernels' counters are published here
    Counters *dev_ctr = nullptr;   // host_ctr as the device addresses it
    void *ws = nullptr;
    size_t ws_size = 0;
    hipEvent_t ev[6] = {};  // iteration phases; [4], [5] bracket the frontier list build
    // the main loop's iteration phases, one set per traced iteration (read
    // after the loop, so that timing adds no host work between iterations):
    // start, hooking done, grandparent pass done, frontier list start and end
    hipEvent_t tev[FASTSV_TRACE_ITERS][5] = {};
    bool events = false;
};

#define HIP_TRY(expr)                                              \
    do {                                                           \
        hipError_t _e = (expr);                                    \
        if (_e != hipSuccess) {                                    \
            if (getenv("FASTSV_DEBUG"))                            \
                fprintf(stderr, "fastsv: %s failed: %s\n", #expr,   \
                        hipGetErrorString(_e));                    \
            return FASTSV_EHIP;                                    \
        }                                                          \
    } while (0)

int fsv::ctx_device(const fastsv_ctx *ctx) { return ctx->device; }

// Workspace of fastsv_cc_csr_noalloc: a fixed array that every device holding
// this code object keeps for the life of the process.  In host code its name
// only stands in for the symbol; the device address of each GPU's copy is
// taken once per device with hipGetSymbolAddress (with that device current)
// and used wherever host code passes the array on.
static __device__ __align__(256) unsigned char scratch[FASTSV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on `device`, which must be current.
int resolve_scratch(int device) {
    if (device < 0 || device >= kScratchDevices) return FASTSV_OK;  // noalloc calls refuse such devices
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return FASTSV_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        if (getenv("FASTSV_DEBUG")) fprintf(stderr, "fastsv: hipGetSymbolAddress(scratch): %s\n", hipGetErrorString(e));
        return FASTSV_EHIP;
    }
    g_scratch_ptr[device] = p;
    return FASTSV_OK;
}

void *scratch_ptr(int device) {
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

namespace {

bool opts_ok(const fastsv_opts &o, int64_t n) {
    if (!(o.frontier_tau >= 0.0f)) return false;  // also rejects NaN
    if (o.binned < -1 || o.binned > 1) return false;
    if (o.sv_flags < 0 || o.sv_flags > kSvFastSV) return false;
    if (o.mode != kModeJacobi && o.mode != kModeAsync) return false;
    if (o.mode == kModeAsync && o.sv_flags != kSvFastSV) return false;
    if (o.bin_shift != 0 && (o.bin_shift < kBinShiftMin || o.bin_shift > kBinShiftMax)) return false;
    if (o.trace != 0 && o.trace != 1) return false;
    if (o.bin_span != 0 && o.bin_span != kBinSpanNarrow && o.bin_span != kBinSpan && o.bin_span != kBinSpanWide)
        return false;
    if (o.admit_mb < 0 || o.admit_mb > 4096) return false;
    return true;
}

// Statistics before a call: zero, with the atomics marked as not counted.
void clear_stats(fastsv_stats *stats) {
    if (!stats) return;
    memset(stats, 0, sizeof(*stats));
    stats->atomics_issued = -1;
    for (auto &a : stats->atomics) a = -1;
}

// Caller-provided workspace, or the context's own (grown on demand).
int get_workspace(fastsv_ctx *ctx, void *&d_ws, size_t ws_bytes, size_t need) {
    if (d_ws) {
        if (ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return FASTSV_EINVAL;
        return FASTSV_OK;
    }
    if (ctx->ws_size < need) {
        if (ctx->ws) HIP_TRY(hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_size = 0;
        if (hipMalloc(&ctx->ws, need) != hipSuccess) return FASTSV_ENOMEM;
        ctx->ws_size = need;
    }
    d_ws = ctx->ws;
    return FASTSV_OK;
}

// Run the optional device check whose kernel sets ctr->status (already
// launched on the stream); FASTSV_ERANGE when it fired.
int read_status(fastsv_ctx *ctx, Counters *ctr, hipStream_t stream) {
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ctx->host_ctr, ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return ctx->host_ctr->status ? FASTSV_ERANGE : FASTSV_OK;
}

struct Problem {
    int n;
    int64_t nnz;
    const int *rp;     // absolute row pointers, monotone over all n rows
    const int *col;    // column ids: global, or local to the row's graph when vbase is set
    const int *vbase;  // nullable: global id of the first vertex of each row's graph
    int *lastk;        // nullable: per-vertex iteration of the last grandparent change
    int *G;            // grandparent vector, final labels in global ids
    const int *f_init = nullptr;  // nullable: initial parent vector (Alg. 3's input f)
};

// Iteration loop of a convergence-ablation variant (opts.sv_flags other than
// 15; Sec. 5.2 builds Algorithm 2 from Algorithm 1 by adding the four changes
// of Sec. 3 in turn): dense pull passes only, the write buffer seeded as the
// variant requires, Alg. 1's shortcut phase when stochastic hooking is off,
// and the termination test on f or on gf.
int solve_variant(fastsv_ctx *ctx, const Problem &P, const Layout &L, const Workspace &w, hipStream_t stream,
                  const fastsv_opts &opts, fastsv_stats *stats, int &it, int *&fk) {
    const int n = P.n;
    const int64_t ntiles = L.ntiles;
    const int fl = opts.sv_flags;
    const bool grand = fl & 1, stoch = fl & 2, early = fl & 8;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, w.ctr);
    launch_init(stream, n, w.F[0], w.F[1], P.G, w.M, 0);
    launch_build_tiles(stream, n, 0, 0, (int)P.nnz, P.rp, w.tiles);
    HIP_TRY(hipGetLastError());
    int *G = P.G;
    int *T = w.frontier;  // the shortcut phase's output
    int status = FASTSV_OK;
    it = 0;
    const dim3 grid(grid_for(ntiles, kHookWaves)), block(kWave * kHookWaves);
    const dim3 vgrid(grid_for(n, 256, 65536)), vblock(256);
    const dim3 rgrid(grid_for(n, 256 / kWave, 8192));  // k_var_root_hook: one wave per row
    for (;;) {
        ++it;
        int *F = w.F[(it + 1) & 1];
        int *Fn = w.F[it & 1];
        fk = Fn;
        IterCounters *ic = &w.ctr->it[it & 1];
        IterCounters *hc = &ctx->host_ctr->it[it & 1];
        const int ti = it - 1;
        const bool timed = opts.timing && ti < FASTSV_TRACE_ITERS;
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[0], stream));
        if (ntiles > 0) {
            if (grand && !stoch)
                hipLaunchKernelGGL(k_var_root_hook, rgrid, dim3(256), 0, stream, n, P.rp, P.col, F, G, Fn,
                                   (fl & 4) ? 1 : 0);
            else
                hipLaunchKernelGGL((k_tile_reduce<kVariant>), grid, block, 0, stream, w.tiles, (int)ntiles, P.rp,
                                   P.col, grand ? G : F, F, Fn, G, w.M, fl, (unsigned long long *)nullptr, SrvTiles{});
        }
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[1], stream));
        launch_zero_iter(stream, ic);
        if (!stoch) hipLaunchKernelGGL(k_var_shortcut, vgrid, vblock, 0, stream, n, Fn, T);
        hipLaunchKernelGGL(k_var_finish, vgrid, vblock, 0, stream, n, stoch ? Fn : T, Fn, F, G, ic, stoch ? 1 : 0,
                           early ? 1 : 0);
        HIP_TRY(hipGetLastError());
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[2], stream));
        launch_publish(stream, ic, &ctx->dev_ctr->it[it & 1]);
        HIP_TRY(hipStreamSynchronize(stream));
        const int64_t changed = (int64_t)(hc->packed >> 32);
        if (stats) {
            stats->dense_iterations++;
            if (ti < FASTSV_TRACE_ITERS) {
                stats->changed[ti] = changed;
                if (timed) {
                    float a = 0, b = 0;
                    HIP_TRY(hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
                    HIP_TRY(hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
                    stats->ms_hook[ti] = a;
                    stats->ms_gp[ti] = b;
                }
            }
        }
        if (changed == 0) break;
        if (opts.max_iters > 0 && it >= opts.max_iters) {
            status = FASTSV_ENOTCONVERGED;
            break;
        }
    }
    if (stats) {
        stats->iterations = it;
        stats->num_tiles = (int32_t)ntiles;
    }
    return status;
}

// Asynchronous mode (opts.mode = 1): the caller's label buffer is the single
// parent vector f; every pass hooks with live grandparents and shortcuts in
// place, and the loop ends after a pass that changed nothing.  Then every
// read of that pass saw the final f, so f[u] = f[f[u]] for every u and
// f[u] <= f[f[v]] = f[v] along every stored entry (both directions): each
// component is one star whose root, the component minimum (f[w] <= w and f
// stays in the component), labels it.
int solve_async(fastsv_ctx *ctx, const Problem &P, const Layout &L, const Workspace &w, hipStream_t stream,
                const fastsv_opts &opts, fastsv_stats *stats, int &it) {
    const int n = P.n;
    const int64_t ntiles = L.ntiles;
    int *f = P.G;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, w.ctr);
    if (P.f_init) {
        if (P.f_init != f)
            HIP_TRY(hipMemcpyAsync(f, P.f_init, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, stream));
    } else {
        launch_fill_iota(stream, n, f);
    }
    launch_build_tiles(stream, n, 0, 0, (int)P.nnz, P.rp, w.tiles);
    HIP_TRY(hipGetLastError());
    int status = FASTSV_OK;
    it = 0;
    for (;;) {
        ++it;
        IterCounters *ic = &w.ctr->it[it & 1];
        IterCounters *hc = &ctx->host_ctr->it[it & 1];
        const int ti = it - 1;
        const bool timed = opts.timing && ti < FASTSV_TRACE_ITERS;
        launch_zero_iter(stream, ic);
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[0], stream));
        if (ntiles > 0)
            hipLaunchKernelGGL(k_async_hook, dim3(grid_for(ntiles, kHookWaves)), dim3(kWave * kHookWaves), 0, stream,
                               w.tiles, (int)ntiles, P.rp, P.col, f, ic);
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[1], stream));
        hipLaunchKernelGGL(k_async_shortcut, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, n, f, ic);
        HIP_TRY(hipGetLastError());
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[2], stream));
        launch_publish(stream, ic, &ctx->dev_ctr->it[it & 1]);
        HIP_TRY(hipStreamSynchronize(stream));
        const int64_t changed = (int64_t)(hc->packed >> 32);
        if (stats) {
            stats->dense_iterations++;
            if (ti < FASTSV_TRACE_ITERS) {
                stats->changed[ti] = changed;
                if (timed) {
                    float a = 0, b = 0;
                    HIP_TRY(hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
                    HIP_TRY(hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
                    stats->ms_hook[ti] = a;
                    stats->ms_gp[ti] = b;
                }
            }
        }
        if (changed == 0) break;
        if (opts.max_iters > 0 && it >= opts.max_iters) {
            status = FASTSV_ENOTCONVERGED;
            break;
        }
    }
    if (stats) {
        stats->iterations = it;
        stats->num_tiles = (int32_t)ntiles;
    }
    return status;
}

// The iteration loop shared by the entry points (Algorithm 3 with the
// sparse-frontier switch).  On return `it` holds the iterations executed and
// `fk` the buffer that holds f after the last iteration.
int solve(fastsv_ctx *ctx, const Problem &P, const Layout &L, const Workspace &w, hipStream_t stream,
          const fastsv_opts &opts, fastsv_stats *stats, int &it, int *&fk) {
    if (opts.sv_flags != kSvFastSV) return solve_variant(ctx, P, L, w, stream, opts, stats, it, fk);
    if (opts.mode == kModeAsync) {
        fk = P.G;  // f itself, also when capped
        return solve_async(ctx, P, L, w, stream, opts, stats, it);
    }
    const int n = P.n;
    const int64_t nnz = P.nnz;
    const int64_t ntiles = L.ntiles;
    const bool base = P.vbase != nullptr;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, w.ctr);
    // iteration 1 reads F from F[0] and writes Fn = F[1]; F = gf = mngf = Fn =
    // iota, or all equal to the given initial parent vector (Alg. 3 duplicates
    // its input f into gf)
    const bool warm = P.f_init != nullptr;
    if (warm)
        hipLaunchKernelGGL(k_init_from, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, n, P.f_init, w.F[0],
                           w.F[1], P.G, w.M);
    else
        launch_init(stream, n, w.F[0], w.F[1], P.G, w.M, 0);
    launch_build_tiles(stream, n, 0, 0, (int)nnz, P.rp, w.tiles);
    // binned layout: built before the first dense iteration that gathers
    int bin_state = (L.bin && !base) ? 0 : -1;  // 0 not built, 1 ready, -1 unused
    // when later iterations will run dense, the layout build also performs the
    // first iteration (it streams the same column ids)
    const bool fuse_first = bin_state == 0 && opts.frontier_tau < 1.0f && !warm;
    HIP_TRY(hipGetLastError());

    int *G = P.G;
    int status = FASTSV_OK;
    it = 0;
    int64_t prev_fcnt = 0, prev_edges = nnz;
    bool frontier_ready = false;
    const double tau_edges = (double)opts.frontier_tau * (double)nnz;
    int64_t alg = 0;
    bool listed[FASTSV_TRACE_ITERS] = {};  // traced iterations that built the frontier list
    for (;;) {
        ++it;
        int *F = w.F[(it + 1) & 1];
        int *Fn = w.F[it & 1];
        fk = Fn;
        IterCounters *ic = &w.ctr->it[it & 1];
        IterCounters *hc = &ctx->host_ctr->it[it & 1];
        // (the slot was last read by the host after iteration it - 2)
        launch_zero_iter(stream, ic);
        unsigned long long *atom = opts.trace ? &ic->atomics : nullptr;
        const bool sparse = it > 1 && frontier_ready && opts.frontier_tau > 0.0f &&
                            (opts.frontier_tau >= 1.0f || (double)prev_edges < tau_edges);
        const int ti = it - 1;
        const bool timed = opts.timing && ti < FASTSV_TRACE_ITERS;
        const int64_t alg_before = alg;  // the iteration's bytes start here
        // iteration 1 gathers too when it starts from a given f
        const bool gathers = it > 1 || warm;
        if (!sparse && gathers && bin_state == 0) {
            if (opts.timing) HIP_TRY(hipEventRecord(ctx->ev[0], stream));
            bin_prepare(L, w, n, P.rp, P.col, stream);
            HIP_TRY(hipGetLastError());
            if (opts.timing) {
                HIP_TRY(hipEventRecord(ctx->ev[1], stream));
                HIP_TRY(hipEventSynchronize(ctx->ev[1]));
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
                if (stats) stats->ms_bin_prepare = ms;
            }
            bin_state = 1;
            if (stats) stats->num_bins = L.nbins;
        }
        hipEvent_t *tv = timed ? ctx->tev[ti] : nullptr;
        if (timed) HIP_TRY(hipEventRecord(tv[0], stream));
        if (sparse) {
            launch_sparse(stream, w.frontier, w.eoff, (int)prev_fcnt, (int)prev_edges, P.rp, P.col, P.vbase, F, Fn, G,
                          w.M, atom);
            // frontier ids, offsets, row starts and values; per slot col and an M read-modify-write
            alg += 16 * prev_fcnt + 12 * prev_edges;
        } else {
            if (it == 1 && fuse_first) {
                bin_prepare(L, w, n, P.rp, P.col, stream, w.M, Fn, timed ? ctx->ev[3] : nullptr, atom);
                bin_state = 1;
                if (stats) {
                    stats->num_bins = L.nbins;
                    stats->bin_fused_first = 1;
                }
            } else if (!gathers) {
                launch_dense(stream, base ? kDenseBaseIota : kDenseIota, w.tiles, (int)ntiles, P.rp, P.col, P.vbase,
                             F, Fn, G, w.M, atom);
            } else if (bin_state == 1) {
                // narrow steps where bins are short (their rows get few
                // records), the filtered middle span otherwise
                const int64_t per_bin = L.bin_cap / L.nbins;
                const int span = opts.bin_span ? opts.bin_span : per_bin >= kBinMidMin ? kBinSpan : kBinSpanNarrow;
                if (span == kBinSpanWide)
                    hipLaunchKernelGGL(k_bin_pull<kBinSpanWide>, dim3(L.nbins), dim3(1024), 0, stream, n, L.bdiv.rows,
                                       L.nchunks, L.bin_cap, w.bcnt, w.brec, w.bck, F, Fn, G, w.M, atom);
                else if (span == kBinSpan)
                    hipLaunchKernelGGL(k_bin_pull<kBinSpan>, dim3(L.nbins), dim3(1024), 0, stream, n, L.bdiv.rows,
                                       L.nchunks, L.bin_cap, w.bcnt, w.brec, w.bck, F, Fn, G, w.M, atom);
                else
                    hipLaunchKernelGGL(k_bin_pull<kBinSpanNarrow>, dim3(L.nbins), dim3(1024), 0, stream, n,
                                       L.bdiv.rows, L.nchunks, L.bin_cap, w.bcnt, w.brec, w.bck, F, Fn, G, w.M, atom);
                if (stats) {
                    stats->binned_iterations++;
                    stats->bin_span = span;
                }
            } else {
                launch_dense(stream, base ? kDenseBaseGather : kDenseGather, w.tiles, (int)ntiles, P.rp, P.col,
                             P.vbase, F, Fn, G, w.M, atom);
            }
            // row_ptr, col, gathers of G[col] (none while G is the identity), then G[u], F[u], M[u] per row
            alg += 4 * ((int64_t)n + 1) + (gathers ? 8 : 4) * nnz + 12 * (int64_t)n + (base ? 4 * (int64_t)n : 0);
        }
        if (timed) HIP_TRY(hipEventRecord(tv[1], stream));
        int64_t alg_hook = alg - alg_before;  // the hooking pass's bytes (completed below)
        const bool want_frontier = opts.frontier_tau > 0.0f;
        launch_grandparent(stream, n, Fn, G, F, P.rp, w.frontier, w.eoff, ic, want_frontier ? 2 : 0, P.lastk, it,
                           P.vbase, nullptr, w.fmask);
        HIP_TRY(hipGetLastError());
        if (timed) HIP_TRY(hipEventRecord(tv[2], stream));
        launch_publish(stream, ic, &ctx->dev_ctr->it[it & 1]);
        HIP_TRY(hipStreamSynchronize(stream));
        const int64_t changed = (int64_t)(hc->packed >> 32);
        const int64_t atomics = opts.trace ? (int64_t)hc->atomics : -1;
        if (atomics > 0) alg_hook += 8 * atomics;
        // read Fn[u], gather Fn[Fn[u]], read G[u], write G[u] and the next seed
        // (with the frontier wanted: a mask bit per vertex); each counted
        // atomic is a read-modify-write of 4 bytes
        alg += 20 * (int64_t)n + (want_frontier ? ((int64_t)n + 7) / 8 : 0) + (atomics > 0 ? 8 * atomics : 0);
        // the frontier list, and its total degree which decides the next
        // iteration's pass, are built from the mask only while a sparse pass is
        // still possible: every changed vertex has at least one entry, and at
        // the average degree the volume must not exceed twice the threshold
        // (a larger volume, or no list, means a dense pass, whose iterate is
        // the same)
        int64_t edges = nnz + 1;
        bool list_ready = false;
        if (want_frontier && changed > 0 &&
            (opts.frontier_tau >= 1.0f ||
             ((double)changed <= tau_edges && (double)changed * (double)nnz <= 2.0 * tau_edges * (double)n))) {
            if (timed) HIP_TRY(hipEventRecord(tv[3], stream));
            launch_frontier_from_mask(stream, n, w.fmask, P.rp, w.frontier, w.eoff, &w.ctr->fb);
            HIP_TRY(hipGetLastError());
            if (timed) HIP_TRY(hipEventRecord(tv[4], stream));
            launch_publish(stream, &w.ctr->fb, &ctx->dev_ctr->fb);
            HIP_TRY(hipStreamSynchronize(stream));
            edges = (int64_t)(ctx->host_ctr->fb.packed & 0xffffffffull);
            list_ready = true;
            // mask, the marked rows' starts, ids and offsets written
            alg += ((int64_t)n + 7) / 8 + 16 * changed;
        }
        if (stats && ti < FASTSV_TRACE_ITERS) {
            stats->changed[ti] = changed;
            stats->sparse[ti] = sparse ? 1 : 0;
            stats->pushed[ti] = sparse ? prev_edges : 0;
            stats->atomics[ti] = atomics;
            stats->alg_hook[ti] = alg_hook;
        }
        if (timed) listed[ti] = list_ready;
        if (stats) {
            if (sparse) {
                stats->sparse_iterations++;
                stats->frontier_edges += prev_edges;
            } else {
                stats->dense_iterations++;
            }
            if (atomics >= 0) stats->atomics_issued = std::max<int64_t>(stats->atomics_issued, 0) + atomics;
        }
        frontier_ready = list_ready;
        prev_fcnt = changed;
        prev_edges = edges;
        if (changed == 0) break;
        if (opts.max_iters > 0 && it >= opts.max_iters) {
            status = FASTSV_ENOTCONVERGED;
            break;
        }
    }
    if (stats && opts.timing) {
        // the phases of every traced iteration, from its events
        for (int ti = 0; ti < std::min(it, FASTSV_TRACE_ITERS); ++ti) {
            hipEvent_t *tv = ctx->tev[ti];
            float a = 0, b = 0;
            HIP_TRY(hipEventElapsedTime(&a, tv[0], tv[1]));
            HIP_TRY(hipEventElapsedTime(&b, tv[1], tv[2]));
            if (ti == 0 && fuse_first) {
                // the count and scan before the fill, and the fill itself
                float c = 0;
                HIP_TRY(hipEventElapsedTime(&c, tv[0], ctx->ev[3]));
                stats->ms_bin_prepare = c;
                a -= c;
            }
            if (listed[ti]) {
                // the frontier list build counts with the grandparent pass
                float l = 0;
                HIP_TRY(hipEventElapsedTime(&l, tv[3], tv[4]));
                b += l;
            }
            stats->ms_hook[ti] = a;
            stats->ms_gp[ti] = b;
        }
    }
    if (stats) {
        stats->iterations = it;
        stats->num_tiles = (int32_t)ntiles;
        stats->alg_bytes = alg;
    }
    return status;
}

// Extra arrays of the edge-list and batch entry points, placed after the
// solver workspace.
struct ExtraLayout {
    size_t off_rp, off_col, off_cursor, off_sums;  // edge list -> CSR
    size_t off_vbase, off_lastk, off_G;            // batch
    size_t total;
};

ExtraLayout edge_extra(size_t start, int64_t n, int64_t m) {
    ExtraLayout X{};
    size_t p = start;
    auto take = [&](size_t bytes) { size_t o = p; p += align256(bytes > 0 ? bytes : 1); return o; };
    X.off_rp = take(sizeof(int) * (size_t)(n + 1));
    X.off_col = take(sizeof(int) * (size_t)(2 * m));
    X.off_cursor = take(sizeof(int) * (size_t)(n > 0 ? n : 1));
    X.off_sums = take(sizeof(int) * (size_t)(grid_for(n > 0 ? n : 1, kScanBlock) + 1));
    X.total = p;
    return X;
}

ExtraLayout batch_extra(size_t start, int64_t n) {
    ExtraLayout X{};
    size_t p = start;
    auto take = [&](size_t bytes) { size_t o = p; p += align256(bytes > 0 ? bytes : 1); return o; };
    X.off_vbase = take(sizeof(int) * (size_t)(n > 0 ? n : 1));
    X.off_lastk = take(sizeof(int) * (size_t)(n > 0 ? n : 1));
    X.off_G = take(sizeof(int) * (size_t)(n > 0 ? n : 1));
    X.total = p;
    return X;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

fastsv_opts fastsv_default_opts(void) {
    fastsv_opts o;
    memset(&o, 0, sizeof(o));
    o.max_iters = 0;
    o.frontier_tau = 0.05f;
    o.validate = 0;
    o.timing = 0;
    o.binned = -1;
    o.bin_shift = 0;
    o.sv_flags = kSvFastSV;
    o.mode = kModeJacobi;
    o.trace = 0;
    o.bin_span = 0;
    o.admit_mb = 0;
    return o;
}

const char *fastsv_strerror(int s) {
    switch (s) {
        case FASTSV_OK: return "ok";
        case FASTSV_EINVAL: return "invalid argument";
        case FASTSV_ERANGE: return "graph validation failed (row_ptr, offsets or an id out of range)";
        case FASTSV_EOVERFLOW: return "size does not fit the int32 layout";
        case FASTSV_ENOMEM: return "out of memory";
        case FASTSV_EHIP: return "HIP runtime error";
        case FASTSV_ENOTCONVERGED: return "not converged within max_iters";
        case FASTSV_EBUSY: return "busy";
        case FASTSV_ESCRATCH: return "workspace exceeds the library's fixed scratch memory";
        default: return "unknown status";
    }
}

int fastsv_create(fastsv_ctx **out, int device) {
    if (!out) return FASTSV_EINVAL;
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return FASTSV_EINVAL;
    HIP_TRY(hipSetDevice(device));
    fastsv_ctx *c = new (std::nothrow) fastsv_ctx();
    if (!c) return FASTSV_ENOMEM;
    c->device = device;
    if (hipHostMalloc(reinterpret_cast<void **>(&c->host_ctr), sizeof(Counters),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        delete c;
        return FASTSV_ENOMEM;
    }
    if (hipHostGetDevicePointer(reinterpret_cast<void **>(&c->dev_ctr), c->host_ctr, 0) != hipSuccess || !c->dev_ctr) {
        fastsv_destroy(c);
        return FASTSV_EHIP;
    }
    memset(c->host_ctr, 0, sizeof(Counters));
    // timing events are made here, so that no solve call creates runtime objects
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            fastsv_destroy(c);
            return FASTSV_EHIP;
        }
        c->events = true;
    }
    for (auto &set : c->tev)
        for (auto &e : set)
            if (hipEventCreate(&e) != hipSuccess) {
                fastsv_destroy(c);
                return FASTSV_EHIP;
            }
    const int rs = resolve_scratch(device);
    if (rs != FASTSV_OK) {
        fastsv_destroy(c);
        return rs;
    }
    *out = c;
    return FASTSV_OK;
}

void fastsv_destroy(fastsv_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->events)
        for (auto &e : c->ev)
            if (e) (void)hipEventDestroy(e);
    for (auto &set : c->tev)
        for (auto &e : set)
            if (e) (void)hipEventDestroy(e);
    if (c->ws) (void)hipFree(c->ws);
    if (c->host_ctr) (void)hipHostFree(c->host_ctr);
    delete c;
}

size_t fastsv_workspace_bytes(int32_t n, int64_t nnz) {
    if (n < 0 || nnz < 0 || nnz > INT_MAX - kTileEntries) return 0;
    return layout_for(n, nnz).total;
}

size_t fastsv_workspace_bytes_opts(int32_t n, int64_t nnz, const fastsv_opts *opts) {
    if (n < 0 || nnz < 0 || nnz > INT_MAX - kTileEntries) return 0;
    fastsv_opts o = opts ? *opts : fastsv_default_opts();
    if (!opts_ok(o, n)) return 0;
    return layout_for(n, nnz, layout_opts(o)).total;
}

}  // extern "C"

namespace {

// noalloc: the workspace is the device's copy of `scratch` (d_ws and
// ws_bytes are ignored), and a layout that does not fit it is refused.
int cc_csr_impl(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col, const int32_t *f_init,
                int32_t *labels, void *d_ws, size_t ws_bytes, hipStream_t stream, const fastsv_opts *opts_in,
                fastsv_stats *stats, bool noalloc = false) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return FASTSV_EINVAL;
    if (n < 0 || nnz < 0) return FASTSV_EINVAL;
    if (nnz > INT_MAX - kTileEntries) return FASTSV_EOVERFLOW;
    fastsv_opts opts = opts_in ? *opts_in : fastsv_default_opts();
    if (!opts_ok(opts, n)) return FASTSV_EINVAL;
    clear_stats(stats);
    if (n == 0) return FASTSV_OK;
    if (!rp || !labels || (nnz > 0 && !col)) return FASTSV_EINVAL;
    if (f_init && opts.sv_flags != kSvFastSV) return FASTSV_EINVAL;  // the variants start from the identity
    const Layout L = layout_for(n, nnz, layout_opts(opts));
    if (noalloc) {
        if (L.total > FASTSV_NOALLOC_SCRATCH_BYTES) return FASTSV_ESCRATCH;
        d_ws = scratch_ptr(ctx->device);
        if (!d_ws) return FASTSV_EINVAL;  // a device the scratch table does not cover
        ws_bytes = FASTSV_NOALLOC_SCRATCH_BYTES;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    int st = get_workspace(ctx, d_ws, ws_bytes, L.total);
    if (st != FASTSV_OK) return st;
    const Workspace w = carve(d_ws, L);
    if (opts.validate) {
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, w.ctr);
        hipLaunchKernelGGL(k_validate, dim3(grid_for((int64_t)n + nnz, 256, 4096)), dim3(256), 0, stream, n, (int)nnz,
                           rp, col, w.ctr);
        if (f_init)
            hipLaunchKernelGGL(k_validate_parents, dim3(grid_for(n, 256, 4096)), dim3(256), 0, stream, n, f_init,
                               w.ctr);
        st = read_status(ctx, w.ctr, stream);
        if (st != FASTSV_OK) return st;
    }
    Problem P{n, nnz, rp, col, nullptr, nullptr, labels};
    P.f_init = f_init;
    int it = 0;
    int *fk = nullptr;
    st = solve(ctx, P, L, w, stream, opts, stats, it, fk);
    if (st == FASTSV_ENOTCONVERGED && fk != labels) {
        // labels hold G_k; report the iterate f_k instead (the asynchronous
        // mode's f is the label buffer itself)
        HIP_TRY(hipMemcpyAsync(labels, fk, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }
    if (stats) stats->ms_total = ms_since(t0);
    return st;
}

}  // namespace

extern "C" {

int fastsv_cc_csr(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                  int32_t *labels, void *d_ws, size_t ws_bytes, hipStream_t stream,
                  const fastsv_opts *opts, fastsv_stats *stats) {
    return cc_csr_impl(ctx, n, nnz, rp, col, nullptr, labels, d_ws, ws_bytes, stream, opts, stats);
}

int fastsv_cc_csr_noalloc(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                          int32_t *labels, hipStream_t stream, const fastsv_opts *opts, fastsv_stats *stats) {
    return cc_csr_impl(ctx, n, nnz, rp, col, nullptr, labels, nullptr, 0, stream, opts, stats, true);
}

int fastsv_cc_csr_warm(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                       const int32_t *f_init, int32_t *labels, void *d_ws, size_t ws_bytes, hipStream_t stream,
                       const fastsv_opts *opts, fastsv_stats *stats) {
    if (!f_init) return FASTSV_EINVAL;
    return cc_csr_impl(ctx, n, nnz, rp, col, f_init, labels, d_ws, ws_bytes, stream, opts, stats);
}

size_t fastsv_edges_workspace_bytes(int32_t n, int64_t m) {
    if (n < 0 || m < 0 || 2 * m > INT_MAX - kTileEntries) return 0;
    const Layout L = layout_for(n, 2 * m);
    return edge_extra(L.total, n, m).total;
}

int fastsv_cc_edges(fastsv_ctx *ctx, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                    int32_t *labels, void *d_ws, size_t ws_bytes, hipStream_t stream, const fastsv_opts *opts_in,
                    fastsv_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return FASTSV_EINVAL;
    if (n < 0 || m < 0) return FASTSV_EINVAL;
    if (2 * m > INT_MAX - kTileEntries) return FASTSV_EOVERFLOW;
    fastsv_opts opts = opts_in ? *opts_in : fastsv_default_opts();
    if (!opts_ok(opts, n)) return FASTSV_EINVAL;
    clear_stats(stats);
    if (n == 0) return FASTSV_OK;
    if (!labels || (m > 0 && (!src || !dst))) return FASTSV_EINVAL;
    const int64_t nnz = 2 * m;
    const Layout L = layout_for(n, nnz, layout_opts(opts));
    const ExtraLayout X = edge_extra(L.total, n, m);
    HIP_TRY(hipSetDevice(ctx->device));
    int st = get_workspace(ctx, d_ws, ws_bytes, X.total);
    if (st != FASTSV_OK) return st;
    const Workspace w = carve(d_ws, L);
    char *base = static_cast<char *>(d_ws);
    int *rp = reinterpret_cast<int *>(base + X.off_rp);
    int *col = reinterpret_cast<int *>(base + X.off_col);
    int *cursor = reinterpret_cast<int *>(base + X.off_cursor);
    int *sums = reinterpret_cast<int *>(base + X.off_sums);
    if (opts.validate && m > 0) {
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, w.ctr);
        hipLaunchKernelGGL(k_validate_edges, dim3(grid_for(m, 256, 4096)), dim3(256), 0, stream, m, n, src, dst, w.ctr);
        st = read_status(ctx, w.ctr, stream);
        if (st != FASTSV_OK) return st;
    }
    // symmetric CSR: degrees, exclusive scan, scatter through atomic cursors
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, n, rp, 0);
    if (m > 0)
        hipLaunchKernelGGL(k_edge_degrees, dim3(grid_for(m, 256, 65536)), dim3(256), 0, stream, m, src, dst, rp);
    scan_inplace(rp, n, sums, stream);
    hipLaunchKernelGGL(k_edge_rowptr_tail, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, n, rp,
                       sums + grid_for(n, kScanBlock), cursor);
    if (m > 0)
        hipLaunchKernelGGL(k_edge_scatter, dim3(grid_for(m, 256, 65536)), dim3(256), 0, stream, m, src, dst, cursor,
                           col);
    HIP_TRY(hipGetLastError());
    Problem P{n, nnz, rp, col, nullptr, nullptr, labels};
    int it = 0;
    int *fk = nullptr;
    st = solve(ctx, P, L, w, stream, opts, stats, it, fk);
    if (st == FASTSV_ENOTCONVERGED && fk != labels) {
        HIP_TRY(hipMemcpyAsync(labels, fk, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }
    if (stats) stats->ms_total = ms_since(t0);
    return st;
}

size_t fastsv_batch_workspace_bytes(int32_t total_n, int64_t total_nnz) {
    if (total_n < 0 || total_nnz < 0 || total_nnz > INT_MAX - kTileEntries) return 0;
    const Layout L = layout_for(total_n, total_nnz, batch_layout_opts());
    return batch_extra(L.total, total_n).total;
}

int fastsv_cc_batch_csr(fastsv_ctx *ctx, int32_t num_graphs, int32_t total_n, int64_t total_nnz,
                        const int32_t *vtx_off, const int32_t *edge_off, const int32_t *rp, const int32_t *col,
                        int32_t *labels, int32_t *iters, void *d_ws, size_t ws_bytes, hipStream_t stream,
                        const fastsv_opts *opts_in, fastsv_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!ctx) return FASTSV_EINVAL;
    if (num_graphs < 0 || total_n < 0 || total_nnz < 0) return FASTSV_EINVAL;
    if (total_nnz > INT_MAX - kTileEntries) return FASTSV_EOVERFLOW;
    fastsv_opts opts = opts_in ? *opts_in : fastsv_default_opts();
    if (!opts_ok(opts, total_n)) return FASTSV_EINVAL;
    // per-graph termination is FastSV's Jacobi one
    if (opts.sv_flags != kSvFastSV || opts.mode != kModeJacobi) return FASTSV_EINVAL;
    clear_stats(stats);
    if (num_graphs == 0) return total_n == 0 && total_nnz == 0 ? FASTSV_OK : FASTSV_EINVAL;
    if (!vtx_off || !edge_off || !rp || !iters || (total_n > 0 && !labels) || (total_nnz > 0 && !col))
        return FASTSV_EINVAL;
    const Layout L = layout_for(total_n, total_nnz, batch_layout_opts());
    const ExtraLayout X = batch_extra(L.total, total_n);
    HIP_TRY(hipSetDevice(ctx->device));
    int st = get_workspace(ctx, d_ws, ws_bytes, X.total);
    if (st != FASTSV_OK) return st;
    const Workspace w = carve(d_ws, L);
    char *base = static_cast<char *>(d_ws);
    int *vbase = reinterpret_cast<int *>(base + X.off_vbase);
    int *lastk = reinterpret_cast<int *>(base + X.off_lastk);
    int *G = reinterpret_cast<int *>(base + X.off_G);
    if (opts.validate) {
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, w.ctr);
        hipLaunchKernelGGL(k_batch_validate, dim3(num_graphs), dim3(256), 0, stream, num_graphs, total_n,
                           (int)total_nnz, vtx_off, edge_off, rp, col, w.ctr);
        st = read_status(ctx, w.ctr, stream);
        if (st != FASTSV_OK) return st;
    }
    hipLaunchKernelGGL(k_batch_bases, dim3(num_graphs), dim3(256), 0, stream, num_graphs, vtx_off, vbase, lastk);
    HIP_TRY(hipGetLastError());
    int it = 0;
    int *fk = nullptr;
    if (total_n > 0) {
        Problem P{total_n, total_nnz, rp, col, vbase, lastk, G};
        st = solve(ctx, P, L, w, stream, opts, stats, it, fk);
        if (st != FASTSV_OK && st != FASTSV_ENOTCONVERGED) return st;
    }
    const bool capped = st == FASTSV_ENOTCONVERGED;
    hipLaunchKernelGGL(k_batch_finish, dim3(num_graphs), dim3(256), 0, stream, num_graphs, vtx_off,
                       capped ? fk : G, lastk, labels, iters, it, capped ? 1 : 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(stream));
    if (stats) stats->ms_total = ms_since(t0);
    return st;
}

}  // extern "C"
