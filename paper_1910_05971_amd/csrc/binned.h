// Binned dense SpMV pass for graphs whose grandparent vector does not fit in
// L2.  Included by fastsv.hip after kernels.h.
//
// The dense step needs m[u] = min_{v in N(u)} G[v] for every row u (Alg. 3,
// the (select2nd, min) SpMV).  The plain pull pass gathers G[v] in the CSR's
// order, which for a graph with scattered ids is random over all of G: each
// 4-byte value costs a whole cache line from the fabric.
//
// Here the stored entries are regrouped once per solve.  Rows are cut into
// bins of W consecutive vertices (at most 40960, the most whose minima fit
// the 160 KB of LDS).  Because the CSR is symmetric, the
// entries (u, v) with u in bin b are exactly the entries (v, u) of the CSR
// whose column u falls in bin b; listing those in the CSR's own storage order
// (rows v ascending) gives bin b's entries sorted by source v.  The layout
// stores one 32-bit record per entry of bin b, bin after bin: the low 16 bits
// of the source v above the row offset u - bW.  The high bits of v change
// rarely along a bin, and marker records carry them (engine.h has the
// format).  A dense iteration then runs one workgroup per
// bin: it streams the bin's entries, gathers G[v] in ascending order of v,
// and min-reduces into an LDS window of W rows.  The waves of a workgroup
// advance through the bin in step, so that they gather from the same narrow
// slice of G at the same time and share its lines in L1 and L2.  Rows are then
// finished as in the pull pass (M update, aggressive and stochastic hooks).
// The minimum is order-free, so the iterate is bit-identical to the pull
// pass's.
//
// Building the layout: a count pass (records per chunk of tiles and bin), an
// exclusive scan of the counts in bin-major order, which gives every
// (bin, chunk) run its first position, and a fill pass that sorts each round
// of tiles by bin in LDS and writes the runs.  Inside a run, records follow
// the marker of their high bits; their order is otherwise not fixed, and no
// result depends on it.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "engine.h"
#include "kernels.h"

namespace fsv {

// High bits of the sources of chunk k's rows: [lo, end] from the rows of its
// first and last entries, and prev, the value in force along every bin when
// the chunk's run starts: the last value of chunk k - 1 (every run carries
// the markers of all values of its chunk up to end), -1 before chunk 0.  A
// run therefore holds the markers of (prev, end].  end >= lo >= prev even
// for a malformed row_ptr, so that the count and the fill pass agree.
struct ChunkHi {
    int prev, lo, end;
};
__device__ __forceinline__ ChunkHi chunk_hi(const Tile *__restrict__ tiles, int ntiles, int k, int chunk_tiles) {
    const int t_begin = k * chunk_tiles, t_end = min(t_begin + chunk_tiles, ntiles);
    ChunkHi h;
    h.lo = tiles[t_begin].r_lo >> kSrcLoBits;
    h.end = max(tiles[t_end - 1].r_hi >> kSrcLoBits, h.lo);
    h.prev = k == 0 ? -1 : min(tiles[t_begin - 1].r_hi >> kSrcLoBits, h.lo);
    return h;
}

// Records per (chunk, bin) in bin-major order: cnt[b * nchunks + k].  Chunk
// k is the tiles [k * chunk_tiles, (k + 1) * chunk_tiles), i.e. the entries
// from k * chunk_tiles * kTileEntries on.  A run holds the chunk's entries of
// the bin and the markers of the values of the high source bits (prev, end]
// (see chunk_hi).  Entries with a column id outside [0, n) are not counted
// (and not placed by the fill pass).
__global__ __launch_bounds__(kBinThreads) void k_bin_count(int64_t nnz, int n, const int *__restrict__ col,
                                                           const Tile *__restrict__ tiles, int ntiles, BinDiv bd,
                                                           int nbins, int nchunks, int chunk_tiles,
                                                           int *__restrict__ cnt) {
    __shared__ int hist[kMaxBins];
    const int tid = threadIdx.x;
    const int k = xcd_major(blockIdx.x, gridDim.x);
    for (int b = tid; b < nbins; b += kBinThreads) hist[b] = 0;
    __syncthreads();
    const int64_t e0 = (int64_t)k * chunk_tiles * kTileEntries;
    const int64_t e1 = min(e0 + (int64_t)chunk_tiles * kTileEntries, nnz);
    const bool vec = (reinterpret_cast<uintptr_t>(col) & 15) == 0;
    // kCountLoads 16-byte loads per thread are issued before their entries are
    // counted, so that they are in flight together
    constexpr int kCountLoads = 8;
    constexpr int64_t kStride = 4 * kBinThreads;
    auto count = [&](int c) {
        if (c >= 0 && c < n) atomicAdd(&hist[bin_of(c, bd)], 1);
    };
    int64_t e = e0 + 4 * tid;
    if (vec) {
        for (; e + (kCountLoads - 1) * kStride + 4 <= e1; e += kCountLoads * kStride) {
            v4i c[kCountLoads];
#pragma unroll
            for (int q = 0; q < kCountLoads; ++q)
                c[q] = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(col + e + q * kStride));
#pragma unroll
            for (int q = 0; q < kCountLoads; ++q) {
                count(c[q].x); count(c[q].y); count(c[q].z); count(c[q].w);
            }
        }
    }
    for (; e < e1; e += kStride)
        for (int64_t f = e; f < min(e + 4, e1); ++f) count(col[f]);
    __syncthreads();
    const ChunkHi ch = chunk_hi(tiles, ntiles, k, chunk_tiles);
    const int markers = ch.end - ch.prev;
    for (int b = tid; b < nbins; b += kBinThreads) cnt[(int64_t)b * nchunks + k] = hist[b] + markers;
    if (k == 0 && tid == 0) cnt[(int64_t)nbins * nchunks] = 0;  // becomes the total after the scan
}

// Fill pass: one workgroup per chunk, processed kFillThreads / kWave tiles at
// a time (one tile per wave).  Each round sorts its entries by bin in LDS and
// writes every bin's run at the bin's cursor, which starts at the chunk's
// offset from the scan: a (chunk, bin) run belongs to this workgroup only.
// Before the first record with high source bits h, every bin's run gets the
// marker of h, and of every value between the last one and h (values without
// entries included, so that each run holds the count pass's number of
// records); the first one is the value after the previous chunk's last.  A round whose rows share one value of the high bits (all but a
// few rounds) is sorted once; one whose rows cross a boundary is processed
// once per value in its row range, in ascending order.  Writes at or beyond
// cap (only a malformed row_ptr gets there) are dropped.
// With kFirst the pass also performs the first iteration of the method, whose
// grandparent vector is the identity: m[u] = min N(u) (the column ids
// themselves), and where m[u] < u, M[u] = Fn[u] = m[u] (both hooks target u,
// since f is the identity too); it replaces the first pull pass.
// Dynamic LDS: 3 * nbins ints.
template <bool kFirst>
// (at most 128 VGPRs: two workgroups of 8 waves share a CU)
__global__ __launch_bounds__(kFillThreads) __attribute__((amdgpu_waves_per_eu(4))) void
k_bin_fill(const Tile *__restrict__ tiles, int ntiles, int n, const int *__restrict__ rp, const int *__restrict__ col,
           BinDiv bd, int nbins, int nchunks, int chunk_tiles, const int *__restrict__ off, int cap,
           unsigned *__restrict__ brec, int *__restrict__ bck, int *__restrict__ M, int *__restrict__ Fn,
           unsigned long long *__restrict__ atom) {
    constexpr int kWaves = kFillThreads / kWave;
    constexpr int kCkMask = (1 << kBinCkShift) - 1;
    static_assert(2 * kRowWin <= kTileEntries, "row windows, row minima and the regrouped loads share the staging arrays");
    extern __shared__ int s_dyn[];
    int *cur = s_dyn;               // next free position of the bin's run
    int *hist = s_dyn + nbins;      // round's count per bin
    int *loff = s_dyn + 2 * nbins;  // round's exclusive offset per bin in the stage
    // the round's stage: every entry's record and layout position, in bin
    // order; before the stage is written its two halves (su, sv) hold the
    // waves' row windows, row minima and regrouped tiles
    __shared__ __align__(16) int2 s_stage[kWaves * kTileEntries];
    int *su = reinterpret_cast<int *>(s_stage);
    int *sv = su + kWaves * kTileEntries;
    __shared__ int s_wsum[kWaves];
    // the descriptors of the next kTileWin tiles; a round reads its tiles'
    // bounds here instead of from global memory
    constexpr int kTileWin = kBinChunkTilesMin;
    static_assert(kTileWin % kWaves == 0, "a descriptor window holds whole rounds");
    __shared__ Tile s_tw[kTileWin];
    // the wave's window of row starts and (first iteration) its per-row minima
    // live from the round's start to its second barrier, the staged entries
    // after it, so they share memory (the windows and minima of all waves take
    // the first halves of su and sv; whole tiles are regrouped in the second)
    int *winw = su + (threadIdx.x / kWave) * kRowWin;
    int *rminw = sv + (threadIdx.x / kWave) * kRowWin;
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = lane_id();
    const int k = xcd_major(blockIdx.x, gridDim.x);
    const int t_end = min((k + 1) * chunk_tiles, ntiles);
    const ChunkHi ch = chunk_hi(tiles, ntiles, k, chunk_tiles);
    auto hi_of = [&](int row) { return min(max(row >> kSrcLoBits, ch.lo), ch.end); };
    for (int b = tid; b < nbins; b += kFillThreads) cur[b] = off[(int64_t)b * nchunks + k];
    const int per = (nbins + kFillThreads - 1) / kFillThreads;
    const int b0 = tid * per, b1 = min(b0 + per, nbins);
    for (int b = b0; b < b1; ++b) hist[b] = 0;
    int na = 0;  // atomics of the first iteration's hooks
    // markers are in place for every value up to hi_done (the same in every thread)
    int hi_done = ch.prev;
    // markers of (hi_done, h] at the cursors of this thread's bins
    auto put_markers = [&](int h) {
        for (int b = b0; b < b1; ++b) {
            int pos = cur[b];
            for (int x = hi_done + 1; x <= h; ++x, ++pos) {
                if (pos >= cap) continue;
                brec[pos] = ((unsigned)x << kSrcLoBits) | kBinMarker;
                if ((pos & kCkMask) == 0) bck[pos >> kBinCkShift] = x;
            }
            cur[b] = pos;
        }
        hi_done = h;
    };
    int tw_base = 0, tw_end = 0;
    for (int t0 = k * chunk_tiles; t0 < t_end; t0 += kWaves) {
      if (t0 >= tw_end) {
          // every wave has passed its last read of the previous window: the
          // previous pass ended with a barrier after them
          tw_base = t0;
          tw_end = min(t0 + kTileWin, t_end);
          if (tid < tw_end - tw_base) s_tw[tid] = tiles[tw_base + tid];
          __syncthreads();
      }
      // high source bits of the round's rows: one value unless they cross a
      // boundary; then the round is processed once per value, each pass
      // placing the entries of its value only
      const int h_first = hi_of(s_tw[t0 - tw_base].r_lo);
      const int h_last = max(hi_of(s_tw[min(t0 + kWaves, t_end) - 1 - tw_base].r_hi), h_first);
      for (int h = h_first; h <= h_last; ++h) {
        const bool one = h_first == h_last;
        const bool first_pass = h == h_first;
        const int t = t0 + wave;
        const bool tile_ok = t < t_end;
        const Tile T = tile_ok ? s_tw[t - tw_base] : Tile{0, 0, 0, -1};
        const int a = T.e0 + lane * kPerLane;
        const int cnt = tile_ok ? max(0, min(kPerLane, T.e1 - a)) : 0;
        int c[kPerLane];
        // a whole tile is read with loads of 1 KB each and regrouped through
        // LDS after the barrier below, so that every lane then holds 16
        // consecutive entries; other tiles are read entry by entry
        const bool whole = tile_ok && T.e1 - T.e0 == kTileEntries &&
                           ((reinterpret_cast<uintptr_t>(col + T.e0) & 15) == 0);
        if (whole) {
            const v4i *p = reinterpret_cast<const v4i *>(col + T.e0) + lane;
#pragma unroll
            for (int q = 0; q < kPerLane / 4; ++q) {
                const v4i v = __builtin_nontemporal_load(p + q * kWave);
                c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
            }
        } else {
            const int last = tile_ok ? T.e1 - 1 : 0;
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) c[j] = __builtin_nontemporal_load(col + min(a + j, last));
        }
        const int nwin = T.r_hi - T.r_lo + 2;
        const bool in_lds = tile_ok && nwin <= kRowWin;
        if (in_lds) {
            // a window of at most 64 row starts takes one load per lane; a wider
            // one has all of its loads issued before the first is stored
            if (nwin <= kWave) {
                if (lane < nwin) {
                    winw[lane] = rp[T.r_lo + lane];
                    if (kFirst) rminw[lane] = INT_MAX;
                }
            } else {
                constexpr int kWinLoads = kRowWin / kWave;
                int wv[kWinLoads];
#pragma unroll
                for (int q = 0; q < kWinLoads; ++q) {
                    const int j = lane + q * kWave;
                    wv[q] = j < nwin ? rp[T.r_lo + j] : 0;
                }
#pragma unroll
                for (int q = 0; q < kWinLoads; ++q) {
                    const int j = lane + q * kWave;
                    if (j < nwin) {
                        winw[j] = wv[q];
                        if (kFirst) rminw[j] = INT_MAX;
                    }
                }
            }
        }
        __syncthreads();
        if (whole) {
            // tile entries [0, 512) pass through su, [512, 1024) through sv,
            // past the row windows and row minima of all waves (the first
            // kWaves * kRowWin ints of each); nothing else is there before the
            // round's entries are staged
            constexpr int kHalf = kTileEntries / 2;
            int *lo_half = su + kWaves * kRowWin + wave * kHalf;
            int *hi_half = sv + kWaves * kRowWin + wave * kHalf;
#pragma unroll
            for (int q = 0; q < kPerLane / 4; ++q) {
                const int x = 4 * lane + 4 * kWave * q;
                *reinterpret_cast<v4i *>(x < kHalf ? lo_half + x : hi_half + (x - kHalf)) =
                    v4i{c[4 * q], c[4 * q + 1], c[4 * q + 2], c[4 * q + 3]};
            }
            // LDS operations of one wave take effect in order; this keeps the
            // compiler from moving the reads above the writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int x0 = kPerLane * lane;
            const v4i *mine = reinterpret_cast<const v4i *>(x0 < kHalf ? lo_half + x0 : hi_half + (x0 - kHalf));
#pragma unroll
            for (int q = 0; q < kPerLane / 4; ++q) {
                const v4i w = mine[q];
                c[4 * q] = w.x; c[4 * q + 1] = w.y; c[4 * q + 2] = w.z; c[4 * q + 3] = w.w;
            }
        }
        const int *wrow = winw;
        // source row of every entry and its rank inside its bin in this round
        int r[kPerLane], rank[kPerLane];
        if (in_lds) {
            // every non-empty row of the window writes its index at its first
            // entry in the tile, and a running maximum over the tile's entries
            // carries it on to the rest of the row; the words are the wave's
            // staging halves, free from the regroup's reads to the staging
            constexpr int kHalf = kTileEntries / 2;
            int *lo_half = su + kWaves * kRowWin + wave * kHalf;
            int *hi_half = sv + kWaves * kRowWin + wave * kHalf;
            const int x0 = kPerLane * lane;
            v4i *mine = reinterpret_cast<v4i *>(x0 < kHalf ? lo_half + x0 : hi_half + (x0 - kHalf));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int q = 0; q < kPerLane / 4; ++q) mine[q] = v4i{0, 0, 0, 0};
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int nrows = nwin - 1;
            for (int i = lane; i < nrows; i += kWave) {
                const int s0 = wrow[i] - T.e0, s1 = wrow[i + 1] - T.e0;
                if (s1 > s0 && s1 > 0 && s0 < kTileEntries) {
                    const int x = max(s0, 0);
                    *(x < kHalf ? lo_half + x : hi_half + (x - kHalf)) = i;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            int m = 0;
#pragma unroll
            for (int q = 0; q < kPerLane / 4; ++q) {
                const v4i w = mine[q];
                m = max(m, w.x); r[4 * q] = m;
                m = max(m, w.y); r[4 * q + 1] = m;
                m = max(m, w.z); r[4 * q + 2] = m;
                m = max(m, w.w); r[4 * q + 3] = m;
            }
            const int carry = wave_shift_up1(wave_incl_max_nonneg(m));
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) r[j] = T.r_lo + max(r[j], carry);
        } else {
            // rows too far apart for the window: a binary search in row_ptr
            // for the lane's first entry, then a walk
            int row = T.r_lo, nxt = 0;
            if (cnt > 0) {
                int lo = T.r_lo, hi = T.r_hi;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (rp[mid] <= a) lo = mid;
                    else hi = mid - 1;
                }
                row = lo;
                nxt = rp[row + 1];
            }
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) {
                if (j < cnt) {
                    const int e = a + j;
                    while (e >= nxt) { ++row; nxt = rp[row + 1]; }
                }
                r[j] = row;
            }
        }
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            const bool ok = j < cnt && c[j] >= 0 && c[j] < n && (one || hi_of(r[j]) == h);
            rank[j] = ok ? atomicAdd(&hist[bin_of(c[j], bd)], 1) : -1;
        }
        if (kFirst && first_pass && cnt > 0) {
            // minimum column of every row segment of the lane: into the tile's
            // LDS row array, or straight to M / Fn for a tile whose rows are too
            // far apart for the window
            int rowc = r[0], cur_min = INT_MAX;
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) {
                if (j < cnt) {
                    if (r[j] != rowc) {
                        if (in_lds) atomicMin(&rminw[rowc - T.r_lo], cur_min);
                        else na += finish_row<true>(rowc, cur_min, true, nullptr, Fn, nullptr, M);
                        rowc = r[j];
                        cur_min = INT_MAX;
                    }
                    cur_min = min(cur_min, c[j]);
                }
            }
            if (in_lds) atomicMin(&rminw[rowc - T.r_lo], cur_min);
            else na += finish_row<true>(rowc, cur_min, true, nullptr, Fn, nullptr, M);
        }
        __syncthreads();
        if (kFirst && first_pass && in_lds) {
            // rows of the tile; a row that continues in a neighbouring tile
            // needs atomics, the others are written by this wave alone
            const int nrows = nwin - 1;
            for (int i = lane; i < nrows; i += kWave) {
                const int m = rminw[i];
                if (m == INT_MAX) continue;
                const bool shared_row = (i == 0 && wrow[0] < T.e0) || (i == nrows - 1 && wrow[nrows] > T.e1);
                na += finish_row<true>(T.r_lo + i, m, shared_row, nullptr, Fn, nullptr, M);
            }
        }
        if (h > hi_done) put_markers(h);
        // exclusive offsets of the round's bins in the stage
        int local = 0;
        for (int b = b0; b < b1; ++b) local += hist[b];
        const int incl = wave_incl_sum(local);
        if (lane == kWave - 1) s_wsum[wave] = incl;
        __syncthreads();
        int o = incl - local, total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            o += w < wave ? s_wsum[w] : 0;
            total += s_wsum[w];
        }
        for (int b = b0; b < b1; ++b) {
            loff[b] = o;
            o += hist[b];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            if (rank[j] >= 0) {
                const int b = bin_of(c[j], bd);
                s_stage[loff[b] + rank[j]] =
                    int2{(int)(((unsigned)r[j] << kSrcLoBits) | (unsigned)(c[j] - b * bd.rows)), cur[b] + rank[j]};
            }
        }
        __syncthreads();
        constexpr int kOut = kWaves * kTileEntries / kFillThreads;
        unsigned rec[kOut];
        int pos[kOut];
#pragma unroll
        for (int q = 0; q < kOut; ++q) {
            const int sidx = tid + q * kFillThreads;
            const int2 e = s_stage[sidx];
            pos[q] = sidx < total ? e.y : cap;
            rec[q] = (unsigned)e.x;
        }
#pragma unroll
        for (int q = 0; q < kOut; ++q) {
            if (pos[q] < cap) {
                brec[pos[q]] = rec[q];
                if ((pos[q] & kCkMask) == 0) bck[pos[q] >> kBinCkShift] = h;
            }
        }
        __syncthreads();
        for (int b = b0; b < b1; ++b) {
            cur[b] += hist[b];
            hist[b] = 0;
        }
        // the next pass's first barrier orders these updates before any use
      }
    }
    if (ch.end > hi_done) put_markers(ch.end);
    if (kFirst) wave_add_atomics(atom, na);
}

// Dense pass over the binned layout: one workgroup per bin, the bin's W rows
// in LDS from the first entry to the last, then the rows are finished as in
// the pull pass (M update, aggressive and stochastic hooks).  The bin's
// entries are sorted by source, and the workgroup walks them in block-wide
// steps of kWaves * kSpan consecutive records with a barrier after each, so
// that its waves gather from the same narrow slice of G at the same time and
// share its lines in L1 and L2.  The steps are aligned to the checkpoints, and
// every wave rebuilds the full sources of its records from the checkpoint at
// its first record and the markers among them.  All bins are launched at
// once; the device starts later bins as earlier ones finish.
template <int kPerLaneSpan>
__global__ __launch_bounds__(1024) void k_bin_pull(int n, int W, int nchunks, int cap, const int *__restrict__ off,
                                                   const unsigned *__restrict__ brec, const int *__restrict__ bck,
                                                   const int *__restrict__ F, int *__restrict__ Fn,
                                                   const int *__restrict__ G, int *__restrict__ M,
                                                   unsigned long long *__restrict__ atom) {
    __shared__ int wmin[kBinRowsMax];
    constexpr int kSpan = kWave * kPerLaneSpan;
    static_assert(kSpan % (1 << kBinCkShift) == 0, "every wave starts at a checkpoint");
    constexpr int kWaves = 1024 / kWave;
    const int tid = threadIdx.x;
    const int lane = lane_id(), wave = tid / kWave;
    const int b = blockIdx.x;
    const int u0 = b * W;
    const int rows = min(W, n - u0);
    for (int i = tid; i < rows; i += 1024) wmin[i] = INT_MAX;
    const int p0 = off[(int64_t)b * nchunks], p1 = min(off[(int64_t)(b + 1) * nchunks], cap);
    const unsigned long long upto = ~0ull >> (kWave - 1 - lane);  // lanes 0..lane
    __syncthreads();
    // the trip count is the same for every wave: the barrier is reached by all
    for (int blk = p0 & ~(kSpan - 1); blk < p1; blk += kWaves * kSpan) {
        const int base = blk + wave * kSpan;
        if (base < p1) {
            unsigned rec[kPerLaneSpan];
            if (base >= p0 && base + kSpan <= p1) {
#pragma unroll
                for (int x = 0; x < kPerLaneSpan; ++x) rec[x] = __builtin_nontemporal_load(brec + base + x * kWave + lane);
            } else {
                // positions outside the bin read as markers; the bin's first
                // record is a marker, which replaces what they carry
#pragma unroll
                for (int x = 0; x < kPerLaneSpan; ++x) {
                    const int q = base + x * kWave + lane;
                    const unsigned r = __builtin_nontemporal_load(brec + min(max(q, p0), p1 - 1));
                    rec[x] = q >= p0 && q < p1 ? r : kBinMarker;
                }
            }
            // high bits in force before the wave's first record
            int carry = base >= p0 ? bck[base >> kBinCkShift] : 0;
            int v[kPerLaneSpan], d[kPerLaneSpan];
#pragma unroll
            for (int x = 0; x < kPerLaneSpan; ++x) {
                const unsigned r = rec[x];
                const bool mk = (r & 0xFFFFu) == kBinMarker;
                const unsigned long long mm = __ballot(mk);
                const int lo = (int)(r >> kSrcLoBits);
                // the last marker at or before this lane, else the carry
                int hi = carry;
                if (mm) {  // (uniform: most groups hold no marker)
                    const unsigned long long le = mm & upto;
                    const int from = le ? kWave - 1 - __clzll(le) : lane;
                    const int hb = __builtin_amdgcn_ds_bpermute(from << 2, lo);
                    hi = le ? hb : carry;
                    carry = __builtin_amdgcn_readlane(lo, kWave - 1 - __clzll(mm));
                }
                const int dd = (int)(r & 0xFFFFu);
                d[x] = mk || dd >= rows ? -1 : dd;  // (a row offset beyond the bin is never written)
                v[x] = mk ? 0 : (int)min(((unsigned)hi << kSrcLoBits) | (unsigned)lo, (unsigned)(n - 1));
            }
#pragma unroll
            for (int x = 0; x < kPerLaneSpan; ++x) v[x] = G[v[x]];
            if (kPerLaneSpan >= kBinSpan) {
                // a record whose value is not below its row's current minimum
                // changes nothing (the minima only decrease, so an older value
                // read here only lets an atomic through), and in bins that
                // give every row many records most are of this kind after the
                // row's first few: the rows' minima are read first (all reads
                // issued together, unconditionally) and only the records below
                // them take an atomic.  (An LDS atomic costs per active lane;
                // a row of k records in random order sees about ln k + 0.58
                // new minima.)
                int cur[kPerLaneSpan];
#pragma unroll
                for (int x = 0; x < kPerLaneSpan; ++x) cur[x] = wmin[max(d[x], 0)];
#pragma unroll
                for (int x = 0; x < kPerLaneSpan; ++x)
                    if (d[x] >= 0 && v[x] < cur[x]) atomicMin(&wmin[d[x]], v[x]);
            } else {
#pragma unroll
                for (int x = 0; x < kPerLaneSpan; ++x)
                    if (d[x] >= 0) atomicMin(&wmin[d[x]], v[x]);
            }
        }
        __syncthreads();
    }
    // finish the rows (as finish_row: M update, aggressive and stochastic
    // hooks) kFinishBatch rows per thread at a time, each stage's loads for
    // the batch issued together: the rows are independent, and a hook's
    // pre-check read that sees an older (larger) Fn only costs an atomic
    int na = 0;
    for (int i0 = tid; i0 < rows; i0 += 1024 * kFinishBatch) {
        int m[kFinishBatch], mu[kFinishBatch], gu[kFinishBatch], fnu[kFinishBatch], fu[kFinishBatch],
            fnx[kFinishBatch];
#pragma unroll
        for (int k = 0; k < kFinishBatch; ++k) {
            const int i = i0 + k * 1024;
            m[k] = i < rows ? wmin[i] : INT_MAX;
        }
#pragma unroll
        for (int k = 0; k < kFinishBatch; ++k) {
            const int u = u0 + i0 + k * 1024;
            mu[k] = m[k] != INT_MAX ? M[u] : INT_MAX;
            gu[k] = m[k] != INT_MAX ? G[u] : INT_MAX;
        }
#pragma unroll
        for (int k = 0; k < kFinishBatch; ++k) {
            const int u = u0 + i0 + k * 1024;
            if (m[k] < mu[k]) M[u] = m[k];
            const bool hook = m[k] < gu[k];  // (false for a row without entries)
            fnu[k] = hook ? Fn[u] : INT_MIN;
            fu[k] = hook ? F[u] : u;
        }
#pragma unroll
        for (int k = 0; k < kFinishBatch; ++k) {
            const int u = u0 + i0 + k * 1024;
            fnx[k] = fu[k] != u ? Fn[fu[k]] : INT_MIN;
        }
#pragma unroll
        for (int k = 0; k < kFinishBatch; ++k) {
            const int u = u0 + i0 + k * 1024;
            if (fnu[k] > m[k]) {
                atomicMin(Fn + u, m[k]);
                ++na;
            }
            if (fu[k] != u && fnx[k] > m[k]) {
                atomicMin(Fn + fu[k], m[k]);
                ++na;
            }
        }
    }
    wave_add_atomics(atom, na);
}

}  // namespace fsv
