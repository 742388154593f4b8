// Internal interface of the FastSV library (not part of the public C ABI):
// shared layout types, kernel geometry and host-side launch wrappers used by
// the solver entry points and by the serving scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fsv {

constexpr int kWave = 64;

// ---- dense hook kernel geometry ----
constexpr int kPerLane = 16;                  // consecutive entries per lane
constexpr int kTileEntries = kWave * kPerLane; // entries per wave tile
constexpr int kHookWaves = 4;                 // waves per workgroup
constexpr int kRowWin = 512;                  // row_ptr window held in LDS per wave

// ---- grandparent kernel geometry ----
constexpr int kGpThreads = 1024;
constexpr int kGpPerThread = 4;
constexpr int kGpBlockVerts = kGpThreads * kGpPerThread;

// ---- sparse push kernel geometry ----
constexpr int kPushThreads = 256;
constexpr int kPushSlots = 2048;              // edge slots per workgroup

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

struct Tile {
    int e0, e1;      // entry range [e0, e1)
    int r_lo, r_hi;  // rows containing entries e0 and e1-1
};

// Bin of a vertex id for a bin width W that need not be a power of two:
// floor(u / W) = (u * m) >> s with s = 31 + ceil(log2 W) and m = ceil(2^s / W).
// With m = (2^s + e) / W, 0 <= e < W, the product overshoots u / W by
// u * e / (W * 2^s) < 2^31 / 2^s <= 1 / W, which never reaches the next
// integer, so the quotient is exact for every 0 <= u < 2^31.
struct BinDiv {
    int rows;              // W
    int s;
    unsigned long long m;
};

inline BinDiv make_bindiv(int W) {
    int l = 0;
    while ((1LL << l) < W) ++l;
    BinDiv d;
    d.rows = W;
    d.s = 31 + l;
    d.m = (unsigned long long)((((unsigned __int128)1 << d.s) + (unsigned)W - 1) / (unsigned)W);
    return d;
}

__device__ __forceinline__ int bin_of(int u, const BinDiv &d) {
    return (int)(((unsigned long long)(unsigned)u * d.m) >> d.s);
}

// Per-iteration counters written by the grandparent pass (two slots, used
// alternately by consecutive iterations).
struct IterCounters {
    // high 32 bits: entries of gf that changed (termination test; they form the
    // frontier list), low 32 bits: their total degree
    unsigned long long packed;
    // global atomics issued by the iteration's hooking (counted when the
    // kernels are given this counter)
    unsigned long long atomics;
};

struct Counters {
    IterCounters it[2];
    IterCounters fb;  // frontier list built from the changed-vertex mask
    int status;
    int pad[7];
};

constexpr int kSvFastSV = 15;  // all four changes of Sec. 3: Algorithm 2
constexpr int kModeJacobi = 0;  // read f, write f_next (Sec. 2.4)
constexpr int kModeAsync = 1;   // one f read and written concurrently

// ---- binned dense pass geometry ----
constexpr int kMaxBins = 2048;          // bins per graph (scatter histogram in LDS)
constexpr int kBinShiftMax = 15;        // largest power-of-two bin width that may be asked for
constexpr int kBinShiftMin = 8;
constexpr int kBinRowsMax = 40960;      // widest bin: a 160 KB LDS window in the dense pass
constexpr int kNumCUs = 256;            // MI355X compute units: one dense-pass workgroup each at a time
// entries per lane and step of the binned dense pass, by the bin's length in
// records: a shorter step keeps the workgroups of an XCD gathering from a
// narrower slice of G at a time (bins whose sources spread over all of G:
// short bins); the spans from kBinSpan on read a row's minimum before its
// atomic, which pays where rows get many records (long bins).  The wide span
// is taken only when asked for.
constexpr int kBinSpanNarrow = 8;       // bins of fewer than kBinMidMin records
constexpr int kBinSpan = 16;            // bins of at least kBinMidMin records
constexpr int kBinSpanWide = 32;
constexpr int64_t kBinMidMin = 1 << 17;
constexpr int kFinishBatch = 8;         // rows per thread whose loads the dense pass's row finish batches
constexpr int kBinThreads = 256;        // layout count pass
constexpr int kFillThreads = 512;       // layout fill: one tile per wave and round
constexpr int64_t kBinMaxCounts = 1 << 27;  // (bin, chunk) counters of the layout build
constexpr int kBinChunkTilesMin = 32;   // tiles per chunk of the layout build (whole fill rounds)
constexpr int kNumXcd = 8;              // workgroups are dealt round-robin to the XCDs

// Workgroup index -> work index such that the workgroups on one XCD (index
// congruent mod kNumXcd) take consecutive work items: their writes to
// neighbouring runs meet in one L2.
__host__ __device__ inline int xcd_major(int bid, int nblocks) {
    const int per = nblocks / kNumXcd, rem = nblocks % kNumXcd;
    const int x = bid % kNumXcd, i = bid / kNumXcd;
    // XCD x gets per (+1 for the first rem XCDs) consecutive items
    return x * per + (x < rem ? x : rem) + i;
}
constexpr int kBinAutoMinN = 1 << 22;   // automatic mode: graphs with more vertices (G well beyond L2)

// One 32-bit record per layout entry: the low kSrcLoBits bits of the source
// above the row offset inside the bin.  The high bits of the source are
// carried by marker records (row offset kBinMarker, high bits above it) that
// precede the first record of every new value of the high bits along a bin
// (a bin opens with the marker of 0); a bin's sources ascend, so a record
// takes the high bits of the last marker before it.  kBinCkShift: the high bits in force at every position that is a
// multiple of 2^kBinCkShift are also stored in a checkpoint array, where a
// wave of the dense pass starts.
constexpr int kSrcLoBits = 16;
constexpr unsigned kBinMarker = 0xFFFFu;
constexpr int kBinCkShift = 9;
static_assert(kBinRowsMax < (int)kBinMarker, "a row offset never equals the marker tag");

// A graph entering or leaving the serving pool (see server.hip).
struct SrvNew {
    int vb, eb, n, nnz;  // pool vertex base, pool entry base, vertices, entries
    int s_rp, s_col;     // offsets of its row_ptr / col in the staging buffer
    int tile_base;       // first tile of its dense first iteration
    int pad;
};

// A graph resident in the serving pool during one step.
struct SrvRun {
    int vb, n;   // pool vertex base, vertices
    int cancel;  // 1: cancelled, leaves in this step without output
    int pad;
};
constexpr int kSettleChunk = 4096;  // vertices per workgroup of the step's settle pass

// One workgroup's share of the placement of newly admitted graphs.
struct PlaceChunk {
    int k;      // graph of the step's admission list
    int part;   // 0: vertex slots 0..n (row pointers, init); 1: column ids
    int start, count;
};
constexpr int kPlaceChunk = 1 << 14;  // items per placement workgroup
constexpr int kPlaceUnroll = 8;

// Exclusive-scan geometry.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;

inline int grid_for(int64_t items, int per_block, int cap = 1 << 30) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace fsv

struct fastsv_ctx;

namespace fsv {

// device of a library context (defined in fastsv.hip)
int ctx_device(const fastsv_ctx *ctx);

// ---- launch wrappers (defined in fastsv.hip) ----
enum DenseMode : int { kDenseIota = 0, kDenseGather = 1, kDenseBaseIota = 2, kDenseBaseGather = 3 };

// F = Fn = G = M = base + i for i in [0, n)
void launch_init(hipStream_t s, int n, int *F, int *Fn, int *G, int *M, int base = 0);
// tiles of one CSR graph whose entries are [e_begin, e_end) of col and whose
// rows are [r_begin, r_begin + nrows) with absolute row_ptr values
void launch_build_tiles(hipStream_t s, int nrows, int r_begin, int e_begin, int e_end, const int *rp, Tile *tiles);
// atom (nullable): where the hooking kernels add the global atomics they issue
void launch_dense(hipStream_t s, int mode, const Tile *tiles, int ntiles, const int *rp, const int *col,
                  const int *vbase, const int *F, int *Fn, const int *G, int *M, unsigned long long *atom = nullptr);
void launch_sparse(hipStream_t s, const int *frontier, const int *eoff, int fcnt, int edges, const int *rp,
                   const int *col, const int *vbase, const int *F, int *Fn, const int *G, int *M,
                   unsigned long long *atom = nullptr);
// the same with the frontier size read on the device from `counts`; frontier
// vertices v with skip_mark[vbase[v]] == skip_val are not pushed
void launch_sparse_dev(hipStream_t s, const IterCounters *counts, int max_blocks, const int *frontier,
                       const int *eoff, const int *rp, const int *col, const int *vbase, const int *F, int *Fn,
                       const int *G, int *M, const int *skip_mark, int skip_val);
void launch_zero_iter(hipStream_t s, IterCounters *ic);
// lastk (nullable): iteration of the last change per vertex, or per graph at
// index vbase[u] when vbase is given; gedge (nullable, needs vbase): frontier
// degree sum per graph at index vbase[u]
// the pass covers [u_begin rounded down to a block, n)
void launch_grandparent(hipStream_t s, int n, const int *Fn, int *G, int *next_fn, const int *rp, int *frontier,
                        int *eoff, IterCounters *ic, int write_frontier, int *lastk, int iter,
                        const int *vbase = nullptr, int *gedge = nullptr, unsigned long long *fmask = nullptr,
                        int u_begin = 0);
// The frontier list of the vertices marked in fmask (see k_frontier_from_mask);
// fb ends as (count << 32 | degree sum).
void launch_frontier_from_mask(hipStream_t s, int n, const unsigned long long *fmask, const int *rp, int *frontier,
                               int *eoff, IterCounters *fb);
void launch_fill(hipStream_t s, int n, int *x, int v);
void launch_fill_iota(hipStream_t s, int n, int *x);

// serving pool helpers
// blocks = blk_off[nrun] (see k_srv_settle); h_flag, h_edges and h_out are
// device addresses of page-locked host memory
void launch_srv_settle(hipStream_t s, int nrun, int blocks, const SrvRun *run, const int *blk_off, int step,
                       int *lastk, int *gedge, int *h_flag, int *h_edges, int *h_out, int *F0, int *F1, int *G,
                       int *M, int *vbase, IterCounters *next_ic);
// the dense pull over the resident tiles of ndense graphs (desc[k]: tile_base
// = first resident tile, vb = graph base; tile_off = exclusive prefix of their
// tile counts), marking each in mark[] with the step
void launch_srv_dense(hipStream_t s, int ndense, int total_tiles, const SrvNew *desc, const int *tile_off,
                      const Tile *pool_tiles, int *mark, int step, const int *rp, const int *col, const int *vbase,
                      const int *F, int *Fn, const int *G, int *M);
// placement of admitted graphs, with the tiles of their dense first iteration
void launch_srv_place(hipStream_t s, int nchunks, const PlaceChunk *chunks, const SrvNew *desc,
                      const int *const *srcs, int *rp, int *col, int *F0, int *F1, int *G, int *M, int *vbase,
                      int *lastk, Tile *tiles);

}  // namespace fsv
