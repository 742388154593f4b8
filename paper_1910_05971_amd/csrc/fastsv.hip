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

#include <chrono>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "fastsv.h"

namespace {

constexpr int kWave = 64;

// ---- dense hook kernel geometry ----
constexpr int kPerLane = 16;                  // consecutive entries per lane
constexpr int kTileEntries = kWave * kPerLane; // entries per wave tile
constexpr int kHookWaves = 4;                 // waves per workgroup
constexpr int kRowWin = 1024;                 // row_ptr window held in LDS per wave

// ---- grandparent kernel geometry ----
constexpr int kGpThreads = 1024;
constexpr int kGpPerThread = 4;
constexpr int kGpBlockVerts = kGpThreads * kGpPerThread;

// ---- sparse push kernel geometry ----
constexpr int kPushThreads = 256;
constexpr int kPushSlots = 2048;              // edge slots per workgroup

typedef int v4i __attribute__((ext_vector_type(4)));

struct Tile {
    int e0, e1;      // entry range [e0, e1)
    int r_lo, r_hi;  // rows containing entries e0 and e1-1
};

// Per-iteration counters written by the grandparent pass (two slots, used
// alternately by consecutive iterations).
struct IterCounters {
    // high 32 bits: entries of gf that changed (termination test; they form the
    // frontier list), low 32 bits: their total degree
    unsigned long long packed;
    unsigned long long pad;
};

struct Counters {
    IterCounters it[2];
    int status;
    int pad[7];
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Inclusive min-scan over the lanes of a wave, restricted to runs of equal
// keys; keys must be nondecreasing across lanes.
__device__ __forceinline__ int seg_min_scan(int key, int val) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int ov = __shfl_up(val, d, kWave);
        int ok = __shfl_up(key, d, kWave);
        if (lane >= d && ok == key) val = min(val, ov);
    }
    return val;
}

__device__ __forceinline__ int wave_incl_sum(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

// Apply the result m of row u: M update, then the two hooks if they can
// change anything.  `shared_row` is set when other tiles also hold entries of
// row u (its M slot then needs an atomic).
// kIota (first iteration): F = G = M = iota, so m < u is the whole filter, and
// both hooks target u itself; a row owned by one tile is then the only writer
// of M[u] and Fn[u] and stores them directly.
template <bool kIota>
__device__ __forceinline__ void finish_row(int u, int m, bool shared_row, const int *__restrict__ F,
                                           int *__restrict__ Fn, const int *__restrict__ G,
                                           int *__restrict__ M) {
    if (kIota) {
        if (m < u) {
            if (shared_row) {
                atomicMin(M + u, m);
                atomicMin(Fn + u, m);
            } else {
                M[u] = m;
                Fn[u] = m;
            }
        }
        return;
    }
    int mu = M[u];
    if (m < mu) {
        if (shared_row) atomicMin(M + u, m);
        else M[u] = m;
    }
    int gu = G[u];
    if (m < gu) {
        atomicMin(Fn + u, m);
        int x = F[u];
        if (x != u) atomicMin(Fn + x, m);
    }
}

// ---------------------------------------------------------------------------
// Tile table for a CSR graph: tile t covers entries [t*T, min((t+1)*T, nnz)).
// The row holding entry t*T writes r_lo, the row holding the tile's last
// entry writes r_hi; every tile gets exactly one writer of each.
// ---------------------------------------------------------------------------
__global__ void k_build_tiles(int n, int nnz, const int *__restrict__ rp, Tile *__restrict__ tiles) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int s = rp[r], e = rp[r + 1];
    if (s >= e) return;
    for (int t = s / kTileEntries; t <= (e - 1) / kTileEntries; ++t) {
        int t0 = t * kTileEntries;
        int last = min(t0 + kTileEntries, nnz) - 1;
        if (t0 >= s && t0 < e) {
            tiles[t].e0 = t0;
            tiles[t].e1 = last + 1;
            tiles[t].r_lo = r;
        }
        if (last >= s && last < e) tiles[t].r_hi = r;
    }
}

// Optional argument check on the device: row_ptr monotone with the stated
// ends, every column id in [0,n).
__global__ void k_validate(int n, int nnz, const int *__restrict__ rp, const int *__restrict__ col,
                           Counters *ctr) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    bool bad = false;
    for (int r = i; r < n; r += stride) bad |= rp[r] > rp[r + 1];
    if (i == 0) bad |= (rp[0] != 0) || (rp[n] != nnz);
    for (int e = i; e < nnz; e += stride) {
        int c = col[e];
        bad |= (c < 0) || (c >= n);
    }
    if (bad) atomicOr(&ctr->status, 1);
}

__global__ void k_init(int n, int *__restrict__ F, int *__restrict__ Fn, int *__restrict__ G,
                       int *__restrict__ M) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) {
        F[u] = u;
        Fn[u] = u;
        G[u] = u;
        M[u] = u;
    }
}

__global__ void k_zero_counters(Counters *ctr) {
    if (threadIdx.x == 0) {
        for (int i = 0; i < 2; ++i) ctr->it[i].packed = 0ull;
        ctr->status = 0;
    }
}

// ---------------------------------------------------------------------------
// Tile reduction: the pull SpMV over (select2nd, min), row by row.
// One wave per tile of 1024 consecutive entries of a CSR; lane l owns entries
// [e0 + 16 l, e0 + 16 l + 16).  Rows of the tile are located through a copy of
// row_ptr[r_lo .. r_hi+1] in LDS (global memory when the window is larger).
// Each lane reduces its rows sequentially; rows crossing lanes are combined
// with a segmented min-scan; rows crossing tiles are flagged `shared`.
//
// Modes
//   kIota       first iteration: G is the identity, so the gathered value is
//               the column id itself
//   kGather     m = min G[col]; finish = M update + hooks
//   kBaseIota / kBaseGather
//               the same for a batch of graphs with local column ids: the
//               global id is col + base[row]
//   kPhase      column-blocked pass: the CSR's rows are segments (row, column
//               block); finish = M update of the segment's row only (the
//               hooks run afterwards from M, see k_hook_rows)
// ---------------------------------------------------------------------------
enum Mode : int { kIota = 0, kGather = 1, kBaseIota = 2, kBaseGather = 3, kPhase = 4 };

template <int kMode>
__device__ __forceinline__ void finish_tile_row(int r, int m, bool shared_row, const int *__restrict__ aux,
                                                const int *__restrict__ F, int *__restrict__ Fn,
                                                const int *__restrict__ G, int *__restrict__ M) {
    if (kMode == kPhase) {
        int sr = aux[r];
        int u = sr & 0x7fffffff;
        bool sh = shared_row || sr < 0;
        if (m < M[u]) {
            if (sh) atomicMin(M + u, m);
            else M[u] = m;
        }
    } else {
        finish_row<kMode == kIota || kMode == kBaseIota>(r, m, shared_row, F, Fn, G, M);
    }
}

template <int kMode>
__global__ __launch_bounds__(kWave *kHookWaves) void k_tile_reduce(
    const Tile *__restrict__ tiles, int ntiles, const int *__restrict__ rp, const int *__restrict__ col,
    const int *__restrict__ aux, const int *__restrict__ F, int *__restrict__ Fn, const int *__restrict__ G,
    int *__restrict__ M) {
    constexpr bool kBase = kMode == kBaseIota || kMode == kBaseGather;
    constexpr bool kNoGather = kMode == kIota || kMode == kBaseIota;
    __shared__ int win[kHookWaves][kRowWin];
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int t = blockIdx.x * kHookWaves + wave;
    const bool tile_ok = t < ntiles;
    Tile T = tile_ok ? tiles[t] : Tile{0, 0, 0, -1};
    const int a = T.e0 + lane * kPerLane;
    const int cnt = tile_ok ? max(0, min(kPerLane, T.e1 - a)) : 0;

    // column ids first (streamed, kept out of the caches' way), then the gathers,
    // so both are in flight while the row window is staged
    int c[kPerLane];
    if (cnt == kPerLane && ((reinterpret_cast<uintptr_t>(col + a) & 15) == 0)) {
        const v4i *p = reinterpret_cast<const v4i *>(col + a);
#pragma unroll
        for (int q = 0; q < kPerLane / 4; ++q) {
            v4i v = __builtin_nontemporal_load(p + q);
            c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) c[j] = j < cnt ? __builtin_nontemporal_load(col + a + j) : 0;
    }
    int g[kPerLane];
    if (!kBase) {
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) g[j] = j < cnt ? (kNoGather ? c[j] : G[c[j]]) : INT_MAX;
    }

    const int nwin = T.r_hi - T.r_lo + 2;  // row_ptr[r_lo .. r_hi+1]
    const bool in_lds = nwin <= kRowWin;
    if (tile_ok && in_lds)
        for (int i = lane; i < nwin; i += kWave) win[wave][i] = rp[T.r_lo + i];
    __syncthreads();
    if (!tile_ok) return;
    const int *wrow = &win[wave][0];
    auto rpw = [&](int r) -> int { return in_lds ? wrow[r - T.r_lo] : rp[r]; };

    int row0 = 0, nxt = 0;
    if (cnt > 0) {
        // row containing entry a: the last row r in [r_lo, r_hi] with row_ptr[r] <= a
        int lo = T.r_lo, hi = T.r_hi;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (rpw(mid) <= a) lo = mid;
            else hi = mid - 1;
        }
        row0 = lo;
        nxt = rpw(row0 + 1);
    }
    if (kBase) {
        // batched graphs: local column ids, shifted by the base of the row's graph
        int r = row0, nx = nxt, b = cnt > 0 ? aux[row0] : 0;
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            if (j < cnt) {
                int e = a + j;
                if (e >= nx) {
                    do { ++r; nx = rpw(r + 1); } while (e >= nx);
                    b = aux[r];
                }
                g[j] = kNoGather ? c[j] + b : G[c[j] + b];
            } else {
                g[j] = INT_MAX;
            }
        }
    }

    // sequential per-lane reduction over the lane's rows
    int row = row0, cur = INT_MAX, first_min = INT_MAX;
    bool first_closed = false;
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) {
        if (j < cnt) {
            int e = a + j;
            if (e >= nxt) {
                if (!first_closed) {
                    first_min = cur;
                    first_closed = true;
                } else {
                    finish_tile_row<kMode>(row, cur, false, aux, F, Fn, G, M);  // row inside this lane
                }
                do { ++row; nxt = rpw(row + 1); } while (e >= nxt);
                cur = INT_MAX;
            }
            cur = min(cur, g[j]);
        }
    }
    const bool first_is_head = cnt > 0 && rpw(row0) == a;
    const int key = cnt > 0 ? row : INT_MAX;
    const int S = seg_min_scan(key, cnt > 0 ? cur : INT_MAX);
    const int prevS = __shfl_up(S, 1, kWave);
    const int next_head = __shfl_down(first_is_head ? 1 : 0, 1, kWave);
    const int next_cnt = __shfl_down(cnt, 1, kWave);
    if (cnt == 0) return;
    if (first_closed) {
        int m = first_min;
        if (lane > 0 && !first_is_head) m = min(m, prevS);
        finish_tile_row<kMode>(row0, m, rpw(row0) < T.e0, aux, F, Fn, G, M);
    }
    const bool ends_here = lane == kWave - 1 || next_cnt == 0 || next_head;
    if (ends_here) {
        bool shared_row = rpw(row) < T.e0 || rpw(row + 1) > T.e1;
        finish_tile_row<kMode>(row, S, shared_row, aux, F, Fn, G, M);
    }
}

// Hooks from the accumulated M after the column-blocked passes:
//   if M[u] < G[u]:  Fn[u] <-min M[u],  Fn[F[u]] <-min M[u].
// M[u] = min(M_{k-1}[u], m[u]); the older part never beats G[u] (it is at
// least f_{k-1}[u] >= G[u]), so this is the same filter and value as hooking
// with the fresh m[u].
__global__ void k_hook_rows(int n, const int *__restrict__ M, const int *__restrict__ G,
                            const int *__restrict__ F, int *__restrict__ Fn) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) {
        int m = M[u];
        if (m < G[u]) {
            atomicMin(Fn + u, m);
            int x = F[u];
            if (x != u) atomicMin(Fn + x, m);
        }
    }
}

// ---------------------------------------------------------------------------
// Column-blocked layout (built once per solve for large graphs with sorted
// rows).  Column block b holds the vertices [b W, (b+1) W).  The entries are
// regrouped, stably, by block: block-major, then source tile, then row.  A
// segment is the run of one row's entries inside one source tile and one
// block; block b's segments form a CSR over its region of cb_col.  A dense
// iteration then runs one pass per block, whose gathers stay inside a
// W-vertex slice of G that fits in L2, and combines the per-segment minima in
// M.  A segment whose row also has entries in another source tile is flagged
// (sign bit of seg_row): its M update is atomic.
// ---------------------------------------------------------------------------
constexpr int kMaxBlocks = 64;

// Row walk shared by the two preparation passes: for lane entries
// [a, a+cnt), the row of each entry, its block, and whether it starts a segment.
struct PrepLane {
    int row[kPerLane];
    int blk[kPerLane];
    bool head[kPerLane];
};

__device__ __forceinline__ void prep_lane(const Tile &T, const int *__restrict__ rp, const int *__restrict__ col,
                                          const int *wrow, bool in_lds, int a, int cnt, int wshift, PrepLane &P,
                                          int &unsorted) {
    auto rpw = [&](int r) -> int { return in_lds ? wrow[r - T.r_lo] : rp[r]; };
    const int lane = lane_id();
    int c[kPerLane];
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) c[j] = j < cnt ? col[a + j] : 0;
    // column id of the entry before a (previous lane's last entry)
    int prev_c = __shfl_up(c[kPerLane - 1], 1, kWave);
    int row = 0, nxt = 0;
    if (cnt > 0) {
        int lo = T.r_lo, hi = T.r_hi;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (rpw(mid) <= a) lo = mid;
            else hi = mid - 1;
        }
        row = lo;
        nxt = rpw(row + 1);
    }
    int pc = prev_c;
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) {
        P.head[j] = false;
        P.blk[j] = 0;
        P.row[j] = row;
        if (j < cnt) {
            int e = a + j;
            while (e >= nxt) { ++row; nxt = rpw(row + 1); }
            int b = c[j] >> wshift;
            b = b < 0 ? 0 : (b >= kMaxBlocks ? kMaxBlocks - 1 : b);  // only out-of-range ids get clamped
            bool row_start = e == rpw(row);
            bool tile_start = (lane == 0 && j == 0);
            P.head[j] = tile_start || row_start || (pc >> wshift) != b;
            if (!tile_start && !row_start && pc > c[j]) unsorted = 1;
            P.row[j] = row;
            P.blk[j] = b;
            pc = c[j];
        }
    }
}

// Pass 1: per (block, source tile) counts of entries and segments, block-major.
__global__ __launch_bounds__(kWave) void k_cb_count(const Tile *__restrict__ tiles, int ntiles,
                                                    const int *__restrict__ rp, const int *__restrict__ col,
                                                    int wshift, int nblk, int *__restrict__ cnt_e,
                                                    int *__restrict__ cnt_s, int *__restrict__ flags) {
    __shared__ int win[kRowWin];
    __shared__ int h_e[kMaxBlocks], h_s[kMaxBlocks];
    const int t = blockIdx.x;
    const int lane = lane_id();
    const Tile T = tiles[t];
    const int nwin = T.r_hi - T.r_lo + 2;
    const bool in_lds = nwin <= kRowWin;
    if (in_lds)
        for (int i = lane; i < nwin; i += kWave) win[i] = rp[T.r_lo + i];
    for (int b = lane; b < nblk; b += kWave) { h_e[b] = 0; h_s[b] = 0; }
    __syncthreads();
    const int a = T.e0 + lane * kPerLane;
    const int cnt = max(0, min(kPerLane, T.e1 - a));
    PrepLane P;
    int unsorted = 0;
    prep_lane(T, rp, col, win, in_lds, a, cnt, wshift, P, unsorted);
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) {
        if (j < cnt) {
            atomicAdd(&h_e[P.blk[j]], 1);
            if (P.head[j]) atomicAdd(&h_s[P.blk[j]], 1);
        }
    }
    if (unsorted) atomicOr(flags, 1);
    __syncthreads();
    for (int b = lane; b < nblk; b += kWave) {
        cnt_e[(int64_t)b * ntiles + t] = h_e[b];
        cnt_s[(int64_t)b * ntiles + t] = h_s[b];
    }
}

// Exclusive scan of int32 (totals below 2^31): block-local scans of 4096
// items, a single-block scan of the block sums, then the add-back.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ int block_excl_scan(int v, int *s_tmp, int &total) {
    // s_tmp: kScanThreads / kWave ints
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    int incl = wave_incl_sum(v);
    if (lane == kWave - 1) s_tmp[wave] = incl;
    __syncthreads();
    int wpre = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
        int x = s_tmp[w];
        if (w < wave) wpre += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return wpre + incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int *__restrict__ x, int64_t len,
                                                              int *__restrict__ sums) {
    __shared__ int s_tmp[kScanThreads / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanBlock;
    int v = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t k = base + (int64_t)i * kScanThreads + threadIdx.x;
        if (k < len) v += x[k];
    }
    int total;
    block_excl_scan(v, s_tmp, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// single block: exclusive scan of sums[0..m) in place, total in sums[m]
__global__ __launch_bounds__(1024) void k_scan_top(int *__restrict__ sums, int m) {
    __shared__ int s_tmp[1024 / kWave];
    __shared__ int s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < m; base += 1024) {
        int k = base + threadIdx.x;
        int v = k < m ? sums[k] : 0;
        int total;
        int ex = block_excl_scan(v, s_tmp, total);
        int carry = s_carry;
        if (k < m) sums[k] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + total;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[m] = s_carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int *__restrict__ x, int64_t len,
                                                            const int *__restrict__ sums, int *__restrict__ y) {
    __shared__ int s_tmp[kScanThreads / kWave];
    // each thread owns kScanItems consecutive items of the block
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t k = base + i;
        v[i] = k < len ? x[k] : 0;
        sum += v[i];
    }
    int total;
    int ex = block_excl_scan(sum, s_tmp, total);
    int run = sums[blockIdx.x] + ex;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t k = base + i;
        if (k < len) y[k] = run;
        run += v[i];
    }
}

// Block bases: entries of block b start at cbb[b] (4-entry aligned), its
// segments at sbb[b]; tb[b] = first phase tile of block b.  Also writes the
// per-block sentinel of the segment pointer array.  Single thread.
struct CbInfo {
    int cbb[kMaxBlocks + 1];   // aligned entry base of each block; cbb[nblk] = padded total
    int len[kMaxBlocks];       // entries of each block
    int sbb[kMaxBlocks + 1];   // segment base of each block; sbb[nblk] = S
    int tb[kMaxBlocks + 1];    // phase tile base of each block; tb[nblk] = total phase tiles
    int flags;                 // bit 0: some row is not sorted
    int pad[3];
};

__global__ void k_cb_bases(const int *__restrict__ off_e, const int *__restrict__ off_s, int ntiles, int nblk,
                           int nnz, const int *__restrict__ total_s, CbInfo *__restrict__ info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int base = 0, tiles = 0;
    for (int b = 0; b < nblk; ++b) {
        int start = off_e[(int64_t)b * ntiles];
        int end = b + 1 < nblk ? off_e[(int64_t)(b + 1) * ntiles] : nnz;
        int len = end - start;
        info->cbb[b] = base;
        info->len[b] = len;
        info->sbb[b] = off_s[(int64_t)b * ntiles];
        info->tb[b] = tiles;
        tiles += (len + kTileEntries - 1) / kTileEntries;
        base += (len + 3) & ~3;
    }
    info->cbb[nblk] = base;
    info->sbb[nblk] = *total_s;
    info->tb[nblk] = tiles;
}

// Pass 2: stable scatter of entries into cb_col and of segment heads into
// seg_ptr / seg_row.
__global__ __launch_bounds__(kWave) void k_cb_scatter(const Tile *__restrict__ tiles, int ntiles,
                                                      const int *__restrict__ rp, const int *__restrict__ col,
                                                      int wshift, int nblk, const int *__restrict__ off_e,
                                                      const int *__restrict__ off_s, const CbInfo *__restrict__ info,
                                                      int *__restrict__ cb_col, int *__restrict__ seg_ptr,
                                                      int *__restrict__ seg_row) {
    __shared__ int win[kRowWin];
    __shared__ unsigned short pe[kWave][kMaxBlocks];  // per-lane entry counts -> exclusive prefix over lanes
    __shared__ unsigned short ps[kWave][kMaxBlocks];  // per-lane head counts  -> exclusive prefix over lanes
    const int t = blockIdx.x;
    const int lane = lane_id();
    const Tile T = tiles[t];
    const int nwin = T.r_hi - T.r_lo + 2;
    const bool in_lds = nwin <= kRowWin;
    if (in_lds)
        for (int i = lane; i < nwin; i += kWave) win[i] = rp[T.r_lo + i];
    for (int b = 0; b < nblk; ++b) { pe[lane][b] = 0; ps[lane][b] = 0; }
    __syncthreads();
    const int a = T.e0 + lane * kPerLane;
    const int cnt = max(0, min(kPerLane, T.e1 - a));
    PrepLane P;
    int unsorted = 0;
    prep_lane(T, rp, col, win, in_lds, a, cnt, wshift, P, unsorted);
    int lre[kPerLane], lrs[kPerLane];
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) {
        if (j < cnt) {
            lre[j] = pe[lane][P.blk[j]]++;
            lrs[j] = P.head[j] ? ps[lane][P.blk[j]]++ : 0;
        }
    }
    __syncthreads();
    // exclusive prefix over lanes, one block column per lane
    for (int b = lane; b < nblk; b += kWave) {
        int re = 0, rs = 0;
        for (int l = 0; l < kWave; ++l) {
            int xe = pe[l][b], xs = ps[l][b];
            pe[l][b] = (unsigned short)re;
            ps[l][b] = (unsigned short)rs;
            re += xe;
            rs += xs;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) {
        if (j < cnt) {
            const int b = P.blk[j];
            const int64_t k = (int64_t)b * ntiles + t;
            const int pos = off_e[k] - off_e[(int64_t)b * ntiles] + info->cbb[b] + pe[lane][b] + lre[j];
            cb_col[pos] = col[a + j];
            if (P.head[j]) {
                const int sp = off_s[k] + ps[lane][b] + lrs[j];
                const int u = P.row[j];
                const bool shared = rp[u] < T.e0 || rp[u + 1] > T.e1;
                seg_ptr[sp + b] = pos;
                seg_row[sp] = shared ? (u | (int)0x80000000) : u;
            }
        }
    }
}

__global__ void k_cb_sentinels(int nblk, const CbInfo *__restrict__ info, int *__restrict__ seg_ptr) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nblk) seg_ptr[info->sbb[b + 1] + b] = info->cbb[b] + info->len[b];
}

// Phase tile table: for segment s of block b (local index r), the tiles of
// block b whose first / last entry lies in the segment.
__global__ void k_cb_tiles(int nblk, const CbInfo *__restrict__ info, const int *__restrict__ seg_ptr,
                           Tile *__restrict__ tiles) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= info->sbb[nblk]) return;
    int lo = 0, hi = nblk - 1;  // block of s: last b with sbb[b] <= s
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (info->sbb[mid] <= s) lo = mid;
        else hi = mid - 1;
    }
    const int b = lo;
    const int r = s - info->sbb[b];
    const int *rpb = seg_ptr + info->sbb[b] + b;
    const int base = info->cbb[b], end = base + info->len[b];
    const int st = rpb[r], en = rpb[r + 1];
    Tile *tb = tiles + info->tb[b];
    for (int t = (st - base) / kTileEntries; t <= (en - 1 - base) / kTileEntries; ++t) {
        int t0 = base + t * kTileEntries;
        int last = min(t0 + kTileEntries, end) - 1;
        if (t0 >= st && t0 < en) {
            tb[t].e0 = t0;
            tb[t].e1 = last + 1;
            tb[t].r_lo = r;
        }
        if (last >= st && last < en) tb[t].r_hi = r;
    }
}

// ---------------------------------------------------------------------------
// Grandparent pass + termination test + frontier compaction.
//   G_k[u] = Fn[Fn[u]];  changed = G_k[u] != G_{k-1}[u];  NextFn[u] = G_k[u]
// The changed vertices are counted (termination test) and, when requested,
// appended to the frontier list together with the exclusive prefix of their
// degrees (the sparse push balances edge slots with it).  Count and degree sum
// share one 64-bit counter (count in the high half), updated once per block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kGpThreads) void k_grandparent(
    int n, const int *__restrict__ Fn, int *__restrict__ G, int *__restrict__ next_fn,
    const int *__restrict__ rp, int *__restrict__ frontier, int *__restrict__ eoff,
    IterCounters *__restrict__ ctr, int write_frontier, int *__restrict__ lastk, int iter) {
    constexpr int kW = kGpThreads / kWave;
    __shared__ int s_cnt[kGpPerThread][kW];
    __shared__ int s_deg[kGpPerThread][kW];
    __shared__ unsigned long long s_base;
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int base_u = blockIdx.x * kGpBlockVerts;
    bool ch[kGpPerThread];
    int deg[kGpPerThread];
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        int u = base_u + i * kGpThreads + threadIdx.x;
        ch[i] = false;
        deg[i] = 0;
        if (u < n) {
            int p = Fn[u];
            int g = Fn[p];
            int old = G[u];
            next_fn[u] = g;
            if (g != old) {
                G[u] = g;
                ch[i] = true;
                if (lastk) lastk[u] = iter;
                if (write_frontier) deg[i] = rp[u + 1] - rp[u];
            }
        }
    }
    int rank[kGpPerThread], dpre[kGpPerThread];
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        unsigned long long bal = __ballot(ch[i]);
        rank[i] = __popcll(bal & ((1ull << lane) - 1ull));
        int incl = wave_incl_sum(deg[i]);
        dpre[i] = incl - deg[i];
        if (lane == kWave - 1) {
            s_cnt[i][wave] = __popcll(bal);
            s_deg[i][wave] = incl;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long c = 0, d = 0;
        for (int i = 0; i < kGpPerThread; ++i)
            for (int w = 0; w < kW; ++w) {
                int cc = s_cnt[i][w], dd = s_deg[i][w];
                s_cnt[i][w] = (int)c;
                s_deg[i][w] = (int)d;
                c += cc;
                d += dd;
            }
        s_base = c ? atomicAdd(&ctr->packed, (c << 32) | d) : 0ull;
    }
    __syncthreads();
    if (!write_frontier) return;
    const unsigned long long b = s_base;
    const int bc = (int)(b >> 32), bd = (int)(b & 0xffffffffull);
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        if (ch[i]) {
            int u = base_u + i * kGpThreads + threadIdx.x;
            int pos = bc + s_cnt[i][wave] + rank[i];
            frontier[pos] = u;
            eoff[pos] = bd + s_deg[i][wave] + dpre[i];
        }
    }
}

__global__ void k_zero_iter_counters(IterCounters *c) {
    if (threadIdx.x == 0) c->packed = 0ull;
}

// ---------------------------------------------------------------------------
// Sparse push: for every frontier vertex v and neighbour u,
//   old = atomicMin(M[u], G[v]);  if G[v] < old and G[v] < G[u]: hooks on u.
// Edge slots are spread evenly over workgroups: workgroup b owns slots
// [b*S, (b+1)*S) of the concatenated frontier rows; the frontier range it
// touches is found with a 64-way search over the edge offsets.
// ---------------------------------------------------------------------------
__device__ int wave_upper_search(const int *__restrict__ eoff, int cnt, int s) {
    // largest i in [0, cnt) with eoff[i] <= s (eoff[0] = 0 <= s)
    const int lane = lane_id();
    int lo = 0, hi = cnt;  // answer in [lo, hi)
    while (hi - lo > kWave) {
        int step = (hi - lo + kWave - 1) / kWave;
        int p = lo + lane * step;
        bool ok = p < hi && eoff[p] <= s;
        unsigned long long bal = __ballot(ok);
        int last = kWave - 1 - __clzll(bal);  // bal != 0: lane 0 probes lo, eoff[lo] <= s
        lo = lo + last * step;
        hi = min(lo + step, hi);
    }
    int p = lo + lane;
    bool ok = p < hi && eoff[p] <= s;
    unsigned long long bal = __ballot(ok);
    return lo + (kWave - 1 - __clzll(bal));
}

template <bool kHasBase>
__global__ __launch_bounds__(kPushThreads) void k_hook_sparse(
    const int *__restrict__ frontier, const int *__restrict__ eoff, int fcnt, int total,
    const int *__restrict__ rp, const int *__restrict__ col, const int *__restrict__ vbase,
    const int *__restrict__ F, int *__restrict__ Fn, const int *__restrict__ G, int *__restrict__ M) {
    __shared__ int s_range[2];
    __shared__ int s_off[kPushSlots + 1];
    __shared__ int s_row[kPushSlots + 1];
    __shared__ int s_val[kPushSlots + 1];
    __shared__ int s_base[kHasBase ? kPushSlots + 1 : 1];
    const int s0 = blockIdx.x * kPushSlots;
    const int s1 = min(s0 + kPushSlots, total);
    if (threadIdx.x < kWave) {
        int i0 = wave_upper_search(eoff, fcnt, s0);
        int i1 = wave_upper_search(eoff, fcnt, s1 - 1);
        if (threadIdx.x == 0) { s_range[0] = i0; s_range[1] = i1; }
    }
    __syncthreads();
    const int i0 = s_range[0], i1 = s_range[1];
    // every frontier vertex with edges owns >= 1 slot, so a block's slots touch at
    // most kPushSlots of them; vertices without edges (possible only when the
    // matrix is not symmetric) can make the range longer, then the block
    // searches the offsets in global memory instead
    const int nv = i1 - i0 + 1;
    const bool in_lds = nv <= kPushSlots + 1;
    if (in_lds) {
        for (int i = threadIdx.x; i < nv; i += kPushThreads) {
            int v = frontier[i0 + i];
            s_off[i] = eoff[i0 + i];
            s_row[i] = rp[v];
            s_val[i] = G[v];
            if (kHasBase) s_base[i] = vbase[v];
        }
    }
    __syncthreads();
    for (int s = s0 + threadIdx.x; s < s1; s += kPushThreads) {
        // frontier entry owning slot s: the last i with eoff[i] <= s
        int lo = 0, hi = nv - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            int om = in_lds ? s_off[mid] : eoff[i0 + mid];
            if (om <= s) lo = mid;
            else hi = mid - 1;
        }
        int off, row, val, vb = 0;
        if (in_lds) {
            off = s_off[lo]; row = s_row[lo]; val = s_val[lo];
            if (kHasBase) vb = s_base[lo];
        } else {
            int v = frontier[i0 + lo];
            off = eoff[i0 + lo]; row = rp[v]; val = G[v];
            if (kHasBase) vb = vbase[v];
        }
        int u = col[row + (s - off)] + vb;
        int old = atomicMin(M + u, val);
        if (val < old) {
            int gu = G[u];
            if (val < gu) {
                atomicMin(Fn + u, val);
                int x = F[u];
                if (x != u) atomicMin(Fn + x, val);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kCbMinShift = 19;  // 2^19 vertices = 2 MB of G per block

inline int cb_shift_for(int64_t n) {
    int sh = kCbMinShift;
    while (((n + (int64_t(1) << sh) - 1) >> sh) > kMaxBlocks) ++sh;
    return sh;
}

struct Layout {
    int64_t n, nnz, ntiles;
    bool cb;         // column-blocked arrays present
    int cb_shift, nblk;
    int64_t scan_len, scan_sums;
    size_t off_F0, off_F1, off_M, off_frontier, off_eoff, off_tiles, off_ctr;
    size_t off_cbcol, off_segptr, off_segrow, off_cnte, off_cnts, off_sums_e, off_sums_s, off_cbtiles, off_info;
    size_t total;
};

// cb_mode: -1 automatic, 0 off, 1 forced; shift 0 = automatic block width.
Layout layout_for(int64_t n, int64_t nnz, int cb_mode = -1, int shift = 0) {
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
    L.off_tiles = take(sizeof(Tile) * (size_t)L.ntiles);
    L.off_ctr = take(sizeof(Counters));
    // automatic mode does not pick the blocked passes yet: on the measured
    // workloads their per-segment M traffic and one-time regrouping cost more
    // than the gathers they keep in L2 (see the design notes); blocked = 1
    // selects them explicitly
    L.cb = nnz > 0 && cb_mode == 1;
    if (L.cb) {
        L.cb_shift = shift > 0 ? shift : cb_shift_for(n);
        L.nblk = (int)((n + (int64_t(1) << L.cb_shift) - 1) >> L.cb_shift);
        L.scan_len = (int64_t)L.nblk * L.ntiles;
        L.scan_sums = (L.scan_len + kScanBlock - 1) / kScanBlock + 1;
        L.off_cbcol = take(sizeof(int) * (size_t)(nnz + 4 * kMaxBlocks));
        L.off_segptr = take(sizeof(int) * (size_t)(nnz + kMaxBlocks + 1));
        L.off_segrow = take(sizeof(int) * (size_t)nnz);
        L.off_cnte = take(sizeof(int) * (size_t)L.scan_len);
        L.off_cnts = take(sizeof(int) * (size_t)L.scan_len);
        L.off_sums_e = take(sizeof(int) * (size_t)L.scan_sums);
        L.off_sums_s = take(sizeof(int) * (size_t)L.scan_sums);
        L.off_cbtiles = take(sizeof(Tile) * (size_t)(L.ntiles + kMaxBlocks));
        L.off_info = take(sizeof(CbInfo));
    }
    L.total = p;
    return L;
}

struct Workspace {
    int *F[2];
    int *M;
    int *frontier;
    int *eoff;
    Tile *tiles;
    Counters *ctr;
    int *cb_col, *seg_ptr, *seg_row, *cnt_e, *cnt_s, *sums_e, *sums_s;
    Tile *cb_tiles;
    CbInfo *info;
};

Workspace carve(void *base, const Layout &L) {
    char *p = static_cast<char *>(base);
    Workspace w{};
    w.F[0] = reinterpret_cast<int *>(p + L.off_F0);
    w.F[1] = reinterpret_cast<int *>(p + L.off_F1);
    w.M = reinterpret_cast<int *>(p + L.off_M);
    w.frontier = reinterpret_cast<int *>(p + L.off_frontier);
    w.eoff = reinterpret_cast<int *>(p + L.off_eoff);
    w.tiles = reinterpret_cast<Tile *>(p + L.off_tiles);
    w.ctr = reinterpret_cast<Counters *>(p + L.off_ctr);
    if (L.cb) {
        w.cb_col = reinterpret_cast<int *>(p + L.off_cbcol);
        w.seg_ptr = reinterpret_cast<int *>(p + L.off_segptr);
        w.seg_row = reinterpret_cast<int *>(p + L.off_segrow);
        w.cnt_e = reinterpret_cast<int *>(p + L.off_cnte);
        w.cnt_s = reinterpret_cast<int *>(p + L.off_cnts);
        w.sums_e = reinterpret_cast<int *>(p + L.off_sums_e);
        w.sums_s = reinterpret_cast<int *>(p + L.off_sums_s);
        w.cb_tiles = reinterpret_cast<Tile *>(p + L.off_cbtiles);
        w.info = reinterpret_cast<CbInfo *>(p + L.off_info);
    }
    return w;
}

inline int grid_for(int64_t items, int per_block, int cap = 1 << 30) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// Exclusive scan of x[0..len) in place; the total lands in sums[m], m = number
// of scan blocks.
void scan_inplace(int *x, int64_t len, int *sums, hipStream_t stream) {
    const int m = grid_for(len, kScanBlock);
    hipLaunchKernelGGL(k_scan_reduce, dim3(m), dim3(kScanThreads), 0, stream, x, len, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, stream, sums, m);
    hipLaunchKernelGGL(k_scan_down, dim3(m), dim3(kScanThreads), 0, stream, x, len, sums, x);
}

__global__ void k_cb_info_init(CbInfo *info) {
    if (threadIdx.x == 0) info->flags = 0;
}

// Build the column-blocked layout (entries, segments, phase tiles).  The
// caller reads CbInfo back afterwards.
void cb_prepare(const Layout &L, const Workspace &w, const int *rp, const int *col, hipStream_t stream) {
    const int nt = (int)L.ntiles;
    hipLaunchKernelGGL(k_cb_info_init, dim3(1), dim3(64), 0, stream, w.info);
    hipLaunchKernelGGL(k_cb_count, dim3(nt), dim3(kWave), 0, stream, w.tiles, nt, rp, col, L.cb_shift, L.nblk,
                       w.cnt_e, w.cnt_s, &w.info->flags);
    scan_inplace(w.cnt_e, L.scan_len, w.sums_e, stream);
    scan_inplace(w.cnt_s, L.scan_len, w.sums_s, stream);
    const int m = grid_for(L.scan_len, kScanBlock);
    hipLaunchKernelGGL(k_cb_bases, dim3(1), dim3(64), 0, stream, w.cnt_e, w.cnt_s, nt, L.nblk, (int)L.nnz,
                       w.sums_s + m, w.info);
    hipLaunchKernelGGL(k_cb_scatter, dim3(nt), dim3(kWave), 0, stream, w.tiles, nt, rp, col, L.cb_shift, L.nblk,
                       w.cnt_e, w.cnt_s, w.info, w.cb_col, w.seg_ptr, w.seg_row);
    hipLaunchKernelGGL(k_cb_sentinels, dim3(1), dim3(kMaxBlocks), 0, stream, L.nblk, w.info, w.seg_ptr);
    hipLaunchKernelGGL(k_cb_tiles, dim3(grid_for(L.nnz, 256)), dim3(256), 0, stream, L.nblk, w.info, w.seg_ptr,
                       w.cb_tiles);
}

}  // namespace

struct fastsv_ctx {
    int device = 0;
    Counters *host_ctr = nullptr;  // pinned
    void *ws = nullptr;
    size_t ws_size = 0;
    hipEvent_t ev[2 * FASTSV_TRACE_ITERS + 2] = {};
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

extern "C" {

fastsv_opts fastsv_default_opts(void) {
    fastsv_opts o;
    memset(&o, 0, sizeof(o));
    o.max_iters = 0;
    o.frontier_tau = 0.05f;
    o.validate = 0;
    o.timing = 0;
    o.blocked = -1;
    o.block_shift = 0;
    return o;
}

const char *fastsv_strerror(int s) {
    switch (s) {
        case FASTSV_OK: return "ok";
        case FASTSV_EINVAL: return "invalid argument";
        case FASTSV_ERANGE: return "graph validation failed (row_ptr or column id out of range)";
        case FASTSV_EOVERFLOW: return "size does not fit the int32 layout";
        case FASTSV_ENOMEM: return "out of memory";
        case FASTSV_EHIP: return "HIP runtime error";
        case FASTSV_ENOTCONVERGED: return "not converged within max_iters";
        case FASTSV_EBUSY: return "busy";
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
    if (hipHostMalloc(reinterpret_cast<void **>(&c->host_ctr), sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return FASTSV_ENOMEM;
    }
    memset(c->host_ctr, 0, sizeof(Counters));
    *out = c;
    return FASTSV_OK;
}

void fastsv_destroy(fastsv_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->events)
        for (auto &e : c->ev) (void)hipEventDestroy(e);
    if (c->ws) (void)hipFree(c->ws);
    if (c->host_ctr) (void)hipHostFree(c->host_ctr);
    delete c;
}

size_t fastsv_workspace_bytes(int32_t n, int64_t nnz) {
    if (n < 0 || nnz < 0 || nnz > INT_MAX - kTileEntries) return 0;
    return layout_for(n, nnz).total;
}

static bool opts_ok(const fastsv_opts &o, int64_t n) {
    if (!(o.frontier_tau >= 0.0f)) return false;  // also rejects NaN
    if (o.blocked < -1 || o.blocked > 1) return false;
    if (o.block_shift != 0 && (o.block_shift < 4 || o.block_shift > 30)) return false;
    if (o.block_shift != 0 && n > 0 && ((n + (int64_t(1) << o.block_shift) - 1) >> o.block_shift) > kMaxBlocks)
        return false;
    return true;
}

size_t fastsv_workspace_bytes_opts(int32_t n, int64_t nnz, const fastsv_opts *opts) {
    if (n < 0 || nnz < 0 || nnz > INT_MAX - kTileEntries) return 0;
    fastsv_opts o = opts ? *opts : fastsv_default_opts();
    if (!opts_ok(o, n)) return 0;
    return layout_for(n, nnz, o.blocked, o.block_shift).total;
}

int fastsv_cc_csr(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                  int32_t *labels, void *d_ws, size_t ws_bytes, hipStream_t stream,
                  const fastsv_opts *opts_in, fastsv_stats *stats) {
    auto t_start = std::chrono::steady_clock::now();
    if (!ctx) return FASTSV_EINVAL;
    if (n < 0 || nnz < 0) return FASTSV_EINVAL;
    if (nnz > INT_MAX - kTileEntries) return FASTSV_EOVERFLOW;
    fastsv_opts opts = opts_in ? *opts_in : fastsv_default_opts();
    if (!opts_ok(opts, n)) return FASTSV_EINVAL;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (n == 0) return FASTSV_OK;
    if (!rp || !labels || (nnz > 0 && !col)) return FASTSV_EINVAL;
    const Layout L = layout_for(n, nnz, opts.blocked, opts.block_shift);
    const int64_t ntiles = L.ntiles;
    HIP_TRY(hipSetDevice(ctx->device));
    if (d_ws) {
        if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return FASTSV_EINVAL;
    } else {
        if (ctx->ws_size < L.total) {
            if (ctx->ws) HIP_TRY(hipFree(ctx->ws));
            ctx->ws = nullptr;
            ctx->ws_size = 0;
            if (hipMalloc(&ctx->ws, L.total) != hipSuccess) return FASTSV_ENOMEM;
            ctx->ws_size = L.total;
        }
        d_ws = ctx->ws;
    }
    if (opts.timing && !ctx->events) {
        for (auto &e : ctx->ev) HIP_TRY(hipEventCreate(&e));
        ctx->events = true;
    }
    const Workspace w = carve(d_ws, L);
    const int nn = (int)nnz;

    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, stream, w.ctr);
    if (opts.validate) {
        hipLaunchKernelGGL(k_validate, dim3(grid_for((int64_t)n + nnz, 256, 4096)), dim3(256), 0, stream, n, nn, rp,
                           col, w.ctr);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(ctx->host_ctr, w.ctr, sizeof(Counters), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (ctx->host_ctr->status) return FASTSV_ERANGE;
    }
    // iteration 1 reads F = iota from F[0] and writes Fn = F[1]; G lives in labels
    hipLaunchKernelGGL(k_init, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, n, w.F[0], w.F[1], labels, w.M);
    if (ntiles > 0)
        hipLaunchKernelGGL(k_build_tiles, dim3(grid_for(n, 256)), dim3(256), 0, stream, n, nn, rp, w.tiles);
    HIP_TRY(hipGetLastError());

    int *G = labels;
    int status = FASTSV_OK;
    int it = 0;
    int64_t prev_fcnt = 0, prev_edges = nnz;
    bool frontier_ready = false;
    const double tau_edges = (double)opts.frontier_tau * (double)nnz;
    int64_t alg = 0;
    // column-blocked dense passes: prepared lazily before the first dense
    // iteration that gathers
    int cb_state = (L.cb && opts.blocked != 0) ? 0 : -1;  // 0 not built, 1 ready, -1 unused
    CbInfo cbh{};
    for (;;) {
        ++it;
        int *F = w.F[(it + 1) & 1];
        int *Fn = w.F[it & 1];
        IterCounters *ic = &w.ctr->it[it & 1];
        IterCounters *hc = &ctx->host_ctr->it[it & 1];
        const bool sparse = it > 1 && frontier_ready && opts.frontier_tau > 0.0f &&
                            (opts.frontier_tau >= 1.0f || (double)prev_edges < tau_edges);
        const int ti = it - 1;
        const bool timed = opts.timing && ti < FASTSV_TRACE_ITERS;
        if (!sparse && it > 1 && cb_state == 0) {
            cb_prepare(L, w, rp, col, stream);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(&cbh, w.info, sizeof(CbInfo), hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            cb_state = (cbh.flags & 1) ? -1 : 1;  // rows not sorted: keep the plain pass
            if (stats) stats->blocked_prepared = 1;
        }
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[0], stream));
        if (sparse) {
            if (prev_edges > 0)
                hipLaunchKernelGGL(k_hook_sparse<false>, dim3(grid_for(prev_edges, kPushSlots)), dim3(kPushThreads), 0,
                                   stream, w.frontier, w.eoff, (int)prev_fcnt, (int)prev_edges, rp, col, nullptr, F,
                                   Fn, G, w.M);
            // frontier ids, offsets, row starts and values; per slot col and an M read-modify-write
            alg += 16 * prev_fcnt + 12 * prev_edges;
        } else {
            const dim3 hgrid(grid_for(ntiles, kHookWaves)), hblock(kWave * kHookWaves);
            if (ntiles > 0) {
                if (it == 1) {
                    hipLaunchKernelGGL((k_tile_reduce<kIota>), hgrid, hblock, 0, stream, w.tiles, (int)ntiles, rp, col,
                                       nullptr, F, Fn, G, w.M);
                } else if (cb_state == 1) {
                    for (int b = 0; b < L.nblk; ++b) {
                        const int nt_b = cbh.tb[b + 1] - cbh.tb[b];
                        if (nt_b <= 0) continue;
                        hipLaunchKernelGGL((k_tile_reduce<kPhase>), dim3(grid_for(nt_b, kHookWaves)), hblock, 0,
                                           stream, w.cb_tiles + cbh.tb[b], nt_b, w.seg_ptr + cbh.sbb[b] + b, w.cb_col,
                                           w.seg_row + cbh.sbb[b], F, Fn, G, w.M);
                    }
                    hipLaunchKernelGGL(k_hook_rows, dim3(grid_for(n, 256, 65536)), dim3(256), 0, stream, n, w.M, G,
                                       F, Fn);
                    if (stats) stats->blocked_iterations++;
                } else {
                    hipLaunchKernelGGL((k_tile_reduce<kGather>), hgrid, hblock, 0, stream, w.tiles, (int)ntiles, rp,
                                       col, nullptr, F, Fn, G, w.M);
                }
            }
            // row_ptr, col, gathers of G[col] (none while G is the identity), then G[u], F[u], M[u] per row
            alg += 4 * ((int64_t)n + 1) + (it == 1 ? 4 : 8) * nnz + 12 * (int64_t)n;
        }
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[1], stream));
        hipLaunchKernelGGL(k_zero_iter_counters, dim3(1), dim3(64), 0, stream, ic);
        const bool want_frontier = opts.frontier_tau > 0.0f;
        hipLaunchKernelGGL(k_grandparent, dim3(grid_for(n, kGpBlockVerts)), dim3(kGpThreads), 0, stream, n, Fn, G, F, rp,
                           w.frontier, w.eoff, ic, want_frontier ? 1 : 0, nullptr, it);
        HIP_TRY(hipGetLastError());
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[2], stream));
        HIP_TRY(hipMemcpyAsync(hc, ic, sizeof(IterCounters), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const int64_t changed = (int64_t)(hc->packed >> 32);
        const int64_t edges = (int64_t)(hc->packed & 0xffffffffull);
        // read Fn[u], gather Fn[Fn[u]], read G[u], write G[u] and the next seed
        alg += 20 * (int64_t)n + (want_frontier ? 16 * changed : 0);
        if (stats && ti < FASTSV_TRACE_ITERS) {
            stats->changed[ti] = changed;
            stats->sparse[ti] = sparse ? 1 : 0;
            if (timed) {
                float a = 0, b = 0;
                HIP_TRY(hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
                HIP_TRY(hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
                stats->ms_hook[ti] = a;
                stats->ms_gp[ti] = b;
            }
        }
        if (stats) {
            if (sparse) {
                stats->sparse_iterations++;
                stats->frontier_edges += prev_edges;
            } else {
                stats->dense_iterations++;
            }
        }
        frontier_ready = want_frontier;
        prev_fcnt = changed;
        prev_edges = edges;
        if (changed == 0) break;
        if (opts.max_iters > 0 && it >= opts.max_iters) {
            // labels hold G_k; the iterate f_k is in Fn
            HIP_TRY(hipMemcpyAsync(labels, Fn, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            status = FASTSV_ENOTCONVERGED;
            break;
        }
    }
    if (stats) {
        stats->iterations = it;
        stats->num_tiles = (int32_t)ntiles;
        stats->alg_bytes = alg;
        stats->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    return status;
}

}  // extern "C"
