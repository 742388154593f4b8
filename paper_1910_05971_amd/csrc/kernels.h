// Device kernels of the FastSV library (gfx950).  Included by fastsv.hip only.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "engine.h"

namespace fsv {

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

// Inclusive max-scan over the lanes of a wave for values >= 0, with DPP lane
// moves (0 stands in for the lanes a move has no source for): shifts by 1, 2,
// 4 and 8 within each row of 16 lanes, then lane 15 into row 1 and lane 47
// into row 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ int wave_incl_max_nonneg(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// The value of the previous lane (0 in lane 0).
__device__ __forceinline__ int wave_shift_up1(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}

// Aggressive hook Fn[u] <-min m and stochastic hook Fn[F[u]] <-min m of a
// row whose minimum m is below G[u].  Fn only decreases while hooks run, so a
// read that already shows a value <= m (possibly an older one) proves the
// atomic would change nothing: hot targets (shared roots) then cost a load
// instead of an atomic.
// Returns the number of atomics issued.
__device__ __forceinline__ int hook_row(int u, int m, const int *__restrict__ F, int *__restrict__ Fn) {
    int na = 0;
    if (Fn[u] > m) {
        atomicMin(Fn + u, m);
        ++na;
    }
    const int x = F[u];
    if (x != u && Fn[x] > m) {
        atomicMin(Fn + x, m);
        ++na;
    }
    return na;
}

// Adds the atomics counted by the lanes of a wave (all 64 lanes active) to
// *atom with one atomic of the wave's own; nothing when atom is null.
__device__ __forceinline__ void wave_add_atomics(unsigned long long *atom, int na) {
    if (!atom) return;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) na += __shfl_xor(na, d, kWave);
    if (lane_id() == 0 && na > 0) atomicAdd(atom, (unsigned long long)na);
}

// Apply the result m of row u: M update, then the two hooks if they can
// change anything.  `shared_row` is set when other tiles also hold entries of
// row u (its M slot then needs an atomic).
// kIota (first iteration): F = G = M = iota, so m < u is the whole filter, and
// both hooks target u itself; a row owned by one tile is then the only writer
// of M[u] and Fn[u] and stores them directly.
// Returns the number of atomics issued.
template <bool kIota>
__device__ __forceinline__ int finish_row(int u, int m, bool shared_row, const int *__restrict__ F,
                                          int *__restrict__ Fn, const int *__restrict__ G,
                                          int *__restrict__ M) {
    if (kIota) {
        if (m < u) {
            if (shared_row) {
                atomicMin(M + u, m);
                atomicMin(Fn + u, m);
                return 2;
            }
            M[u] = m;
            Fn[u] = m;
        }
        return 0;
    }
    int na = 0;
    int mu = M[u];
    if (m < mu) {
        if (shared_row) {
            atomicMin(M + u, m);
            ++na;
        } else {
            M[u] = m;
        }
    }
    if (m < G[u]) na += hook_row(u, m, F, Fn);
    return na;
}

// ---------------------------------------------------------------------------
// Tile table of one CSR graph whose rows are [r_begin, r_begin + nrows) (with
// absolute row_ptr values) and whose entries are [e_begin, e_end): tile t
// covers entries [e_begin + t*T, min(e_begin + (t+1)*T, e_end)).  The row
// holding a tile's first entry writes r_lo, the row holding its last entry
// writes r_hi; every tile gets exactly one writer of each.  A row over more
// than kTileLongRow tiles (a hub) is handed to the whole block, so that no
// thread loops over thousands of tiles.  Launched with 256 threads per block.
// ---------------------------------------------------------------------------
constexpr int kTileLongRow = 8;
__global__ __launch_bounds__(256) void k_build_tiles(int nrows, int r_begin, int e_begin, int e_end,
                                                     const int *__restrict__ rp, Tile *__restrict__ tiles) {
    __shared__ int s_n;
    __shared__ int s_row[256], s_s[256], s_e[256];
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const int len = e_end - e_begin;
    auto put = [&](int r, int s, int e, int t) {
        const int t0 = t * kTileEntries;
        const int last = min(t0 + kTileEntries, len) - 1;
        if (t0 >= s && t0 < e) {
            tiles[t].e0 = e_begin + t0;
            tiles[t].e1 = e_begin + last + 1;
            tiles[t].r_lo = r;
        }
        if (last >= s && last < e) tiles[t].r_hi = r;
    };
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrows) {
        const int r = r_begin + i;
        const int s = rp[r] - e_begin, e = rp[r + 1] - e_begin;
        if (s < e) {
            const int ta = s / kTileEntries, tb = (e - 1) / kTileEntries;
            if (tb - ta < kTileLongRow) {
                for (int t = ta; t <= tb; ++t) put(r, s, e, t);
            } else {
                const int k = atomicAdd(&s_n, 1);
                s_row[k] = r;
                s_s[k] = s;
                s_e[k] = e;
            }
        }
    }
    __syncthreads();
    const int nlong = s_n;
    for (int k = 0; k < nlong; ++k) {
        const int r = s_row[k], s = s_s[k], e = s_e[k];
        for (int t = s / kTileEntries + (int)threadIdx.x; t <= (e - 1) / kTileEntries; t += blockDim.x) put(r, s, e, t);
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

// F = Fn = G = M = iota over global ids base + i.
__global__ void k_init(int n, int *__restrict__ F, int *__restrict__ Fn, int *__restrict__ G,
                       int *__restrict__ M, int base) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) {
        int v = base + u;
        F[u] = v;
        Fn[u] = v;
        G[u] = v;
        M[u] = v;
    }
}

// F = Fn = G = M = f0 (a given initial parent vector; f0 may alias G).
__global__ void k_init_from(int n, const int *__restrict__ f0, int *__restrict__ F, int *__restrict__ Fn, int *G,
                            int *__restrict__ M) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) {
        const int v = f0[u];
        F[u] = v;
        Fn[u] = v;
        G[u] = v;
        M[u] = v;
    }
}

// Optional check of an initial parent vector: 0 <= f0[u] <= u.
__global__ void k_validate_parents(int n, const int *__restrict__ f0, Counters *ctr) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    bool bad = false;
    for (int u = i; u < n; u += stride) {
        const int v = f0[u];
        bad |= (v < 0) || (v > u);
    }
    if (bad) atomicOr(&ctr->status, 1);
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
//   kSrvGather  kBaseGather over the tiles of the serving pool's dense graphs
//               (see SrvTiles)
//   kBaseIota / kBaseGather
//               the same for a batch of graphs with local column ids: the
//               global id is col + base[row]
// ---------------------------------------------------------------------------
enum Mode : int { kIota = 0, kGather = 1, kBaseIota = 2, kBaseGather = 3, kVariant = 5, kSrvGather = 6 };

// Tiles of the serving pool's dense graphs: wave t of the launch takes tile
// t - off[k] of graph k = the last one with off[k] <= t (desc[k].tile_base is
// its first resident tile), and the graph's first wave marks it in mark[] so
// that the step's push skips its frontier.
struct SrvTiles {
    int ndense;
    const SrvNew *desc;
    const int *off;
    int *mark;
    int step;
};

// Hooking of one row in a convergence-ablation variant (the flags of
// fastsv_opts.sv_flags): m = min over N(u) of X[v], X = gf with grandparent
// hooking (Sec. 3.1), f without.
//   stochastic (Sec. 3.2): one Jacobi pass whose write buffer starts as gf
//     (the shortcut); Fn[f[u]] <-min m with no root test, plus, when
//     aggressive (Sec. 3.3), Fn[u] <-min m.  Both are no-ops unless m < gf[u]
//     (the write buffer starts at or below gf[u] at both targets).
//   otherwise, without grandparent hooking (Alg. 1's first phase, write
//     buffer = copy of f): a root f[u] (f[u] = gf[u]) is hooked onto the
//     smallest f[v] below it, which is m whenever m < f[u]; aggressive hooking
//     adds Fn[u] <-min m.  (With grandparent hooking the hook condition tests
//     f[v], not the value hooked onto: k_var_root_hook.)
__device__ __forceinline__ int find_owner(const int *__restrict__ off, int count, int64_t x);

__device__ __forceinline__ void finish_variant(int u, int m, int flags, const int *__restrict__ F,
                                               int *__restrict__ Fn, const int *__restrict__ G) {
    const bool stoch = flags & 2, aggr = flags & 4;
    if (stoch) {
        if (m < G[u]) {
            if (aggr && Fn[u] > m) atomicMin(Fn + u, m);
            const int x = F[u];
            if ((!aggr || x != u) && Fn[x] > m) atomicMin(Fn + x, m);
        }
    } else {
        const int fu = F[u];
        if (m < fu) {
            if (fu == G[u]) atomicMin(Fn + fu, m);
            if (aggr) atomicMin(Fn + u, m);
        }
    }
}

// Returns the number of atomics issued (the variants' are not counted).
template <int kMode>
__device__ __forceinline__ int finish_tile_row(int r, int m, bool shared_row,
                                               const int *__restrict__ F, int *__restrict__ Fn,
                                               const int *__restrict__ G, int *__restrict__ M, int vflags) {
    if (kMode == kVariant) {
        finish_variant(r, m, vflags, F, Fn, G);
        return 0;
    }
    return finish_row<kMode == kIota || kMode == kBaseIota>(r, m, shared_row, F, Fn, G, M);
}

// atom (nullable): the iteration's count of the atomics hooking issues.
template <int kMode>
__global__ __launch_bounds__(kWave *kHookWaves) void k_tile_reduce(
    const Tile *__restrict__ tiles, int ntiles, const int *__restrict__ rp, const int *__restrict__ col,
    const int *__restrict__ aux, const int *__restrict__ F, int *__restrict__ Fn, const int *__restrict__ G,
    int *__restrict__ M, int vflags, unsigned long long *__restrict__ atom, SrvTiles srv) {
    constexpr bool kBase = kMode == kBaseIota || kMode == kBaseGather || kMode == kSrvGather;
    // gathered vector: G, or for a variant the one passed in aux (f or gf)
    const int *__restrict__ X = kMode == kVariant ? aux : G;
    constexpr bool kNoGather = kMode == kIota || kMode == kBaseIota;
    __shared__ int win[kHookWaves][kRowWin];   // row_ptr[r_lo .. r_hi+1]
    __shared__ int rmin[kHookWaves][kRowWin];  // per-row minimum of this tile
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int t = blockIdx.x * kHookWaves + wave;
    const bool tile_ok = t < ntiles;
    Tile T = Tile{0, 0, 0, -1};
    if (kMode == kSrvGather) {
        if (tile_ok) {
            const int k = find_owner(srv.off, srv.ndense, t);
            const SrvNew d = srv.desc[k];
            const int i = t - srv.off[k];
            T = tiles[d.tile_base + i];
            if (i == 0 && lane == 0) srv.mark[d.vb] = srv.step;
        }
    } else if (tile_ok) {
        T = tiles[t];
    }
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
        // partial lane: addresses are clamped into the tile (or to entry 0 for
        // a wave past the last tile) so that no load sits under a branch
        const int last = tile_ok ? T.e1 - 1 : 0;
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) c[j] = __builtin_nontemporal_load(col + min(a + j, last));
    }
    // Gathers are issued unconditionally (index 0 for the lane's unused
    // slots) and masked afterwards: a gather under a per-slot branch makes the
    // compiler wait for every earlier load before issuing it.
    int g[kPerLane];
    if (!kBase) {
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            const int v = kNoGather ? c[j] : X[j < cnt ? c[j] : 0];
            g[j] = j < cnt ? v : INT_MAX;
        }
    }

    const int nwin = T.r_hi - T.r_lo + 2;
    const bool in_lds = tile_ok && nwin <= kRowWin;
    if (in_lds)
        for (int i = lane; i < nwin; i += kWave) {
            win[wave][i] = rp[T.r_lo + i];
            rmin[wave][i] = INT_MAX;
        }
    __syncthreads();
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
        int gi[kPerLane];
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            const int e = a + j;
            if (j < cnt && e >= nx) {
                do { ++r; nx = rpw(r + 1); } while (e >= nx);
                b = aux[r];
            }
            gi[j] = j < cnt ? c[j] + b : 0;
        }
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            const int v = kNoGather ? gi[j] : G[gi[j]];
            g[j] = j < cnt ? v : INT_MAX;
        }
    }

    if (in_lds) {
        // every row segment of the lane folds its minimum into the tile's LDS
        // row array; rows are then finished together with coalesced accesses
        int row = row0, cur = INT_MAX;
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            if (j < cnt) {
                int e = a + j;
                if (e >= nxt) {
                    atomicMin(&rmin[wave][row - T.r_lo], cur);
                    do { ++row; nxt = rpw(row + 1); } while (e >= nxt);
                    cur = INT_MAX;
                }
                cur = min(cur, g[j]);
            }
        }
        if (cnt > 0) atomicMin(&rmin[wave][row - T.r_lo], cur);
    }
    __syncthreads();
    if (!tile_ok) return;  // (uniform in the wave)
    int na = 0;
    if (in_lds) {  // (uniform in the wave)
        const int nrows = nwin - 1;
        for (int i = lane; i < nrows; i += kWave) {
            int m = rmin[wave][i];
            if (m == INT_MAX) continue;  // empty row
            bool shared_row = (i == 0 && wrow[0] < T.e0) || (i == nrows - 1 && wrow[nrows] > T.e1);
            na += finish_tile_row<kMode>(T.r_lo + i, m, shared_row, F, Fn, G, M, vflags);
        }
        wave_add_atomics(atom, na);
        return;
    }

    // wide window (rows far apart): per-lane finish, rows crossing lanes are
    // combined with a segmented min-scan
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
                    na += finish_tile_row<kMode>(row, cur, false, F, Fn, G, M, vflags);  // row inside this lane
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
    if (cnt > 0) {
        if (first_closed) {
            int m = first_min;
            if (lane > 0 && !first_is_head) m = min(m, prevS);
            na += finish_tile_row<kMode>(row0, m, rpw(row0) < T.e0, F, Fn, G, M, vflags);
        }
        const bool ends_here = lane == kWave - 1 || next_cnt == 0 || next_head;
        if (ends_here) {
            bool shared_row = rpw(row) < T.e0 || rpw(row + 1) > T.e1;
            na += finish_tile_row<kMode>(row, S, shared_row, F, Fn, G, M, vflags);
        }
    }
    wave_add_atomics(atom, na);
}

// Exclusive scan of int32 (totals below 2^31): block-local scans of 4096
// items, a single-block scan of the block sums, then the add-back.
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

// ---------------------------------------------------------------------------
// Grandparent pass + termination test + frontier compaction.
//   G_k[u] = Fn[Fn[u]];  changed = G_k[u] != G_{k-1}[u];  NextFn[u] = G_k[u]
// The changed vertices are counted (termination test).  write_frontier = 1
// also appends them to the frontier list together with the exclusive prefix
// of their degrees (the sparse push balances edge slots with it);
// write_frontier = 2 marks them in fmask instead (one bit per vertex, one word
// per wave; no degrees are read), and k_frontier_from_mask builds the list and
// its degree sum when a sparse iteration may follow.  Count and degree sum share one 64-bit
// counter (count in the high half), updated once per block.
// ---------------------------------------------------------------------------
// The pass covers the vertices [u_begin, n); u_begin is a multiple of
// kGpBlockVerts (the serving pool skips its unused low part).
__global__ __launch_bounds__(kGpThreads) void k_grandparent(
    int u_begin, int n, const int *__restrict__ Fn, int *__restrict__ G, int *__restrict__ next_fn,
    const int *__restrict__ rp, int *__restrict__ frontier, int *__restrict__ eoff,
    IterCounters *__restrict__ ctr, int write_frontier, int *__restrict__ lastk, int iter,
    const int *__restrict__ vbase, int *__restrict__ gedge, unsigned long long *__restrict__ fmask) {
    constexpr int kW = kGpThreads / kWave;
    __shared__ int s_cnt[kGpPerThread][kW];
    __shared__ int s_deg[kGpPerThread][kW];
    __shared__ unsigned long long s_base;
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int base_u = u_begin + blockIdx.x * kGpBlockVerts;
    bool ch[kGpPerThread];
    int deg[kGpPerThread];
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        int u = base_u + i * kGpThreads + threadIdx.x;
        ch[i] = false;
        deg[i] = 0;
        if (u < n) {
            int p = Fn[u];
            int g = p == u ? p : Fn[p];  // (a root is its own grandparent)
            int old = G[u];
            next_fn[u] = g;
            if (g != old) {
                G[u] = g;
                ch[i] = true;
                // lastk: iteration of the last change, per vertex, or per graph
                // (at the graph's first vertex) when the graph bases are given
                if (lastk) lastk[vbase ? vbase[u] : u] = iter;
                if (write_frontier == 1) deg[i] = rp[u + 1] - rp[u];
            }
        }
    }
    if (gedge) {
        // per-graph frontier degree sums (graph bases are nondecreasing over the
        // consecutive vertices of a wave): one atomic per run of equal bases
#pragma unroll
        for (int i = 0; i < kGpPerThread; ++i) {
            int u = base_u + i * kGpThreads + threadIdx.x;
            int key = u < n ? vbase[u] : INT_MAX;
            int v = deg[i];
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                int ov = __shfl_up(v, d, kWave);
                int ok = __shfl_up(key, d, kWave);
                if (lane >= d && ok == key) v += ov;
            }
            int next_key = __shfl_down(key, 1, kWave);
            bool tail = lane == kWave - 1 || next_key != key;
            if (tail && key != INT_MAX && v > 0) atomicAdd(gedge + key, v);
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
        // the wave's 64 consecutive vertices as one mask word; stored past the
        // caches (plain 8-byte stores from every wave leave partly written
        // lines in L2 that slowed the next dense step by ~8%)
        const int u0 = base_u + i * kGpThreads + wave * kWave;
        if (write_frontier == 2 && lane == 0 && u0 < n) __builtin_nontemporal_store(bal, fmask + u0 / kWave);
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
    if (write_frontier != 1) return;
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

// The frontier list (ids and degree offsets, as k_grandparent's
// write_frontier = 1 writes it) of the vertices marked in fmask, one bit per
// vertex; ctr->packed must be zero on entry and ends as (count << 32 | degree
// sum).  The list's order differs from that mode's, which nothing depends on.
__global__ __launch_bounds__(kGpThreads) void k_frontier_from_mask(int n, const unsigned long long *__restrict__ fmask,
                                                                   const int *__restrict__ rp,
                                                                   int *__restrict__ frontier,
                                                                   int *__restrict__ eoff,
                                                                   IterCounters *__restrict__ ctr) {
    constexpr int kW = kGpThreads / kWave;
    __shared__ int s_cnt[kGpPerThread][kW];
    __shared__ int s_deg[kGpPerThread][kW];
    __shared__ unsigned long long s_base;
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int base_u = blockIdx.x * kGpBlockVerts;
    bool ch[kGpPerThread];
    int rank[kGpPerThread], dpre[kGpPerThread];
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        const int u0 = base_u + i * kGpThreads + wave * kWave;
        const unsigned long long word = u0 < n ? fmask[u0 / kWave] : 0ull;
        const int u = u0 + lane;
        ch[i] = u < n && ((word >> lane) & 1ull);
        const int deg = ch[i] ? rp[u + 1] - rp[u] : 0;
        rank[i] = __popcll(word & ((1ull << lane) - 1ull));
        const int incl = wave_incl_sum(deg);
        dpre[i] = incl - deg;
        if (lane == kWave - 1) {
            s_cnt[i][wave] = __popcll(word);
            s_deg[i][wave] = incl;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long c = 0, d = 0;
        for (int i = 0; i < kGpPerThread; ++i)
            for (int w = 0; w < kW; ++w) {
                const int cc = s_cnt[i][w], dd = s_deg[i][w];
                s_cnt[i][w] = (int)c;
                s_deg[i][w] = (int)d;
                c += cc;
                d += dd;
            }
        s_base = c ? atomicAdd(&ctr->packed, (c << 32) | d) : 0ull;
    }
    __syncthreads();
    const unsigned long long b = s_base;
    const int bc = (int)(b >> 32), bd = (int)(b & 0xffffffffull);
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        if (ch[i]) {
            const int pos = bc + s_cnt[i][wave] + rank[i];
            frontier[pos] = base_u + i * kGpThreads + wave * kWave + lane;
            eoff[pos] = bd + s_deg[i][wave] + dpre[i];
        }
    }
}

// Copies iteration counters (to mapped host memory), one 64-bit word per lane.
__global__ void k_publish_counters(const IterCounters *__restrict__ src, IterCounters *__restrict__ dst) {
    constexpr int kWords = (int)(sizeof(IterCounters) / sizeof(unsigned long long));
    const int i = threadIdx.x;
    if (i < kWords)
        reinterpret_cast<unsigned long long *>(dst)[i] = reinterpret_cast<const unsigned long long *>(src)[i];
}

__global__ void k_zero_iter_counters(IterCounters *c) {
    if (threadIdx.x == 0) {
        c->packed = 0ull;
        c->atomics = 0ull;
    }
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
    const int *__restrict__ frontier, const int *__restrict__ eoff, int fcnt_arg, int total_arg,
    const IterCounters *__restrict__ counts, const int *__restrict__ rp, const int *__restrict__ col,
    const int *__restrict__ vbase, const int *__restrict__ F, int *__restrict__ Fn, const int *__restrict__ G,
    int *__restrict__ M, const int *__restrict__ skip_mark, int skip_val, unsigned long long *__restrict__ atom) {
    __shared__ int s_range[2];
    __shared__ int s_off[kPushSlots + 1];
    __shared__ int s_row[kPushSlots + 1];
    __shared__ int s_val[kPushSlots + 1];
    __shared__ int s_base[kHasBase ? kPushSlots + 1 : 1];
    // frontier size from the arguments, or from the counters the grandparent
    // pass left on the device (then the grid is a fixed size and loops)
    int fcnt = fcnt_arg, total = total_arg;
    if (counts) {
        const unsigned long long pk = counts->packed;
        fcnt = (int)(pk >> 32);
        total = (int)(pk & 0xffffffffull);
    }
    int na = 0;
    for (int chunk = blockIdx.x; (int64_t)chunk * kPushSlots < total; chunk += gridDim.x) {
        const int s0 = chunk * kPushSlots;
        const int s1 = min(s0 + kPushSlots, total);
        __syncthreads();  // LDS of the previous chunk no longer in use
        if (threadIdx.x < kWave) {
            int i0 = wave_upper_search(eoff, fcnt, s0);
            int i1 = wave_upper_search(eoff, fcnt, s1 - 1);
            if (threadIdx.x == 0) { s_range[0] = i0; s_range[1] = i1; }
        }
        __syncthreads();
        const int i0 = s_range[0], i1 = s_range[1];
        // every frontier vertex with edges owns >= 1 slot, so a chunk's slots touch at
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
                // a vertex whose graph runs the dense pass in this step pushes nothing
                s_val[i] = (kHasBase && skip_mark && skip_mark[vbase[v]] == skip_val) ? INT_MAX : G[v];
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
                if (kHasBase) {
                    vb = vbase[v];
                    if (skip_mark && skip_mark[vb] == skip_val) val = INT_MAX;
                }
            }
            if (val == INT_MAX) continue;
            int u = col[row + (s - off)] + vb;
            // M only decreases: a push that a plain read shows cannot lower
            // M[u] would change nothing (the atomic would return old <= val,
            // and no hook follows), so it stays a load
            if (val >= M[u]) continue;
            int old = atomicMin(M + u, val);
            ++na;
            if (val < old && val < G[u]) na += hook_row(u, val, F, Fn);
        }
    }
    wave_add_atomics(atom, na);
}


// ---------------------------------------------------------------------------
// Edge-list entry: symmetric CSR built on the device.  Edge (u,v) is stored as
// v in row u and u in row v (a self loop twice in its row), like the
// reference graphs.  Order inside a row follows the atomic cursor; the method
// does not depend on it.
// ---------------------------------------------------------------------------
__global__ void k_validate_edges(int64_t m, int n, const int *__restrict__ src, const int *__restrict__ dst,
                                 Counters *ctr) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t e = i; e < m; e += stride) {
        int a = src[e], b = dst[e];
        bad |= a < 0 || a >= n || b < 0 || b >= n;
    }
    if (bad) atomicOr(&ctr->status, 1);
}

// ---------------------------------------------------------------------------
// End of an iteration of a convergence-ablation variant.
// Without stochastic hooking the iteration has Alg. 1's second phase, the
// shortcut f_k[u] = f1[f1[u]] of the hooked vector f1 (k_var_shortcut, into T).
// k_var_finish then, with fk the new parent vector (Fn, or T after the
// shortcut): G_k = fk[fk]; counts the vertices whose G (early termination,
// Sec. 3.4) or f changed; stores fk in Fn when it was built in T; and seeds the
// next write buffer (the old F buffer) with G_k (stochastic variants, whose
// pass includes the shortcut) or with fk (Alg. 1's first phase starts from f).
// ---------------------------------------------------------------------------
__global__ void k_var_shortcut(int n, const int *__restrict__ Fn, int *__restrict__ T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) T[u] = Fn[Fn[u]];
}

// Alg. 1's hooking phase with grandparent hooking and no stochastic hooking
// (Sec. 3.1: the hook still requires f[u] to be a root and f[v] < f[u]; only
// the vertex hooked onto changes, from f[v] to f[f[v]]).  One wave per row,
// rows dealt grid-stride: the lanes stride over the row's entries and keep
//   mc = min gf[v] over the entries with f[v] < f[u]   (the root hook)
//   ma = min gf[v] over all entries                     (aggressive hooking)
// then Fn[f[u]] <-min mc if f[u] is a root, and Fn[u] <-min ma if aggressive.
// Fn starts as a copy of f; f[f[v]] <= f[v] < f[u], so a root hook always
// lowers its target.
__global__ __launch_bounds__(256) void k_var_root_hook(int n, const int *__restrict__ rp,
                                                       const int *__restrict__ col, const int *__restrict__ F,
                                                       const int *__restrict__ G, int *__restrict__ Fn, int aggr) {
    const int lane = lane_id();
    const int waves = gridDim.x * (blockDim.x / kWave);
    for (int u = blockIdx.x * (blockDim.x / kWave) + (int)threadIdx.x / kWave; u < n; u += waves) {
        const int fu = F[u];
        const int e1 = rp[u + 1];
        int mc = INT_MAX, ma = INT_MAX;
        for (int e = rp[u] + lane; e < e1; e += kWave) {
            const int v = col[e];
            const int gv = G[v];
            ma = min(ma, gv);
            if (F[v] < fu) mc = min(mc, gv);
        }
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) {
            mc = min(mc, __shfl_xor(mc, d, kWave));
            ma = min(ma, __shfl_xor(ma, d, kWave));
        }
        if (lane == 0) {
            if (mc < fu && fu == G[u]) atomicMin(Fn + fu, mc);
            if (aggr && ma < fu) atomicMin(Fn + u, ma);
        }
    }
}

__global__ void k_var_finish(int n, const int *__restrict__ fk, int *__restrict__ Fn, int *__restrict__ F,
                             int *__restrict__ G, IterCounters *__restrict__ ctr, int stoch, int early) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    int changed = 0;
    for (int u = i; u < n; u += stride) {
        const int a = fk[u];
        const int g = fk[a];
        changed += early ? (g != G[u]) : (a != F[u]);
        G[u] = g;
        if (!stoch) Fn[u] = a;
        F[u] = stoch ? g : a;
    }
    // one atomic per wave (every lane reaches this point)
    const int tot = wave_incl_sum(changed);
    if (lane_id() == kWave - 1 && tot) atomicAdd(&ctr->packed, (unsigned long long)tot << 32);
}

// ---------------------------------------------------------------------------
// Asynchronous mode (Sec. 2.4: one parent vector read and written
// concurrently).  f is deliberately not restrict-qualified: it is read and
// written by every thread of the pass.
// Hooking pass: one wave per tile; for each row segment of a lane,
// m = min over its entries v of the live grandparent f[f[v]]; then
// f[f[u]] <-min m and f[u] <-min m.  ctr->packed (high 32 bits) counts the
// atomics that lowered a value.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int async_hook_row(int u, int m, int *f) {
    int changed = 0;
    const int x = f[u];
    if (m < f[x] && atomicMin(f + x, m) > m) ++changed;
    if (m < f[u] && atomicMin(f + u, m) > m) ++changed;
    return changed;
}

__global__ __launch_bounds__(kWave *kHookWaves) void k_async_hook(const Tile *__restrict__ tiles, int ntiles,
                                                                  const int *__restrict__ rp,
                                                                  const int *__restrict__ col, int *f,
                                                                  IterCounters *ctr) {
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int t = blockIdx.x * kHookWaves + wave;
    if (t >= ntiles) return;  // whole waves leave together
    const Tile T = tiles[t];
    const int a = T.e0 + lane * kPerLane;
    const int cnt = max(0, min(kPerLane, T.e1 - a));
    int g[kPerLane];
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) g[j] = col[min(a + j, T.e1 - 1)];
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) g[j] = f[g[j]];
#pragma unroll
    for (int j = 0; j < kPerLane; ++j) g[j] = f[g[j]];
    int changed = 0;
    if (cnt > 0) {
        int lo = T.r_lo, hi = T.r_hi;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= a) lo = mid;
            else hi = mid - 1;
        }
        int row = lo, nxt = rp[lo + 1], cur = INT_MAX;
        for (int j = 0; j < cnt; ++j) {
            const int e = a + j;
            if (e >= nxt) {
                changed += async_hook_row(row, cur, f);
                do { ++row; nxt = rp[row + 1]; } while (e >= nxt);
                cur = INT_MAX;
            }
            cur = min(cur, g[j]);
        }
        changed += async_hook_row(row, cur, f);
    }
    const int tot = wave_incl_sum(changed);
    if (lane == kWave - 1 && tot) atomicAdd(&ctr->packed, (unsigned long long)tot << 32);
}

// Shortcut pass of the asynchronous mode: f[u] <- f[f[u]] where smaller (only
// thread u writes f[u]; others may read it meanwhile, which is the mode's
// concurrent reading).  Counts the changes like the hooking pass.
__global__ void k_async_shortcut(int n, int *f, IterCounters *ctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    int changed = 0;
    for (int u = i; u < n; u += stride) {
        const int p = f[u];
        const int g = f[p];
        if (g < p) {
            f[u] = g;
            ++changed;
        }
    }
    const int tot = wave_incl_sum(changed);
    if (lane_id() == kWave - 1 && tot) atomicAdd(&ctr->packed, (unsigned long long)tot << 32);
}

__global__ void k_iota(int n, int *__restrict__ x) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) x[u] = u;
}

__global__ void k_fill(int n, int *__restrict__ x, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) x[u] = v;
}

__global__ void k_edge_degrees(int64_t m, const int *__restrict__ src, const int *__restrict__ dst,
                               int *__restrict__ deg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = i; e < m; e += stride) {
        atomicAdd(deg + src[e], 1);
        atomicAdd(deg + dst[e], 1);
    }
}

// rp[0..n) holds the exclusive prefix of the degrees; set rp[n] and a copy of
// the row starts as write cursors.
__global__ void k_edge_rowptr_tail(int n, int *__restrict__ rp, const int *__restrict__ total,
                                   int *__restrict__ cursor) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int stride = gridDim.x * blockDim.x;
    for (int u = i; u < n; u += stride) cursor[u] = rp[u];
    if (i == 0) rp[n] = *total;
}

__global__ void k_edge_scatter(int64_t m, const int *__restrict__ src, const int *__restrict__ dst,
                               int *__restrict__ cursor, int *__restrict__ col) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = i; e < m; e += stride) {
        int a = src[e], b = dst[e];
        col[atomicAdd(cursor + a, 1)] = b;
        col[atomicAdd(cursor + b, 1)] = a;
    }
}

// ---------------------------------------------------------------------------
// Batch of graphs solved as one block-diagonal graph.  Graph g owns the global
// vertices [vtx_off[g], vtx_off[g+1]) and entries [edge_off[g], edge_off[g+1]);
// its column ids are local.  Values of f and gf are global ids, so graphs
// never exchange anything and each follows its own trajectory exactly.
// One workgroup per graph for the per-graph passes below.
// ---------------------------------------------------------------------------
__global__ void k_batch_validate(int ngraphs, int total_n, int total_nnz, const int *__restrict__ vtx_off,
                                 const int *__restrict__ edge_off, const int *__restrict__ rp,
                                 const int *__restrict__ col, Counters *ctr) {
    const int g = blockIdx.x;
    if (g >= ngraphs) return;
    const int v0 = vtx_off[g], v1 = vtx_off[g + 1], e0 = edge_off[g], e1 = edge_off[g + 1];
    bool bad = v0 < 0 || v1 < v0 || v1 > total_n || e0 < 0 || e1 < e0 || e1 > total_nnz;
    if (g == 0) bad |= v0 != 0 || e0 != 0;
    if (g == ngraphs - 1) bad |= v1 != total_n || e1 != total_nnz;
    if (!bad) {
        bad |= rp[v0] != e0 || rp[v1] != e1;
        const int nloc = v1 - v0;
        for (int r = v0 + (int)threadIdx.x; r < v1 && !bad; r += blockDim.x) bad |= rp[r] > rp[r + 1];
        if (!bad)
            for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
                int c = col[e];
                bad |= c < 0 || c >= nloc;
            }
    }
    if (bad) atomicOr(&ctr->status, 1);
}

__global__ void k_batch_bases(int ngraphs, const int *__restrict__ vtx_off, int *__restrict__ vbase,
                              int *__restrict__ lastk) {
    const int g = blockIdx.x;
    if (g >= ngraphs) return;
    const int v0 = vtx_off[g], v1 = vtx_off[g + 1];
    for (int u = v0 + (int)threadIdx.x; u < v1; u += blockDim.x) {
        vbase[u] = v0;
        lastk[u] = 0;
    }
}

// labels in local ids and per-graph iteration counts: 1 + the last iteration
// in which a grandparent of the graph changed (-1 if that is the final
// iteration of a capped run, i.e. the graph had not converged; 0 for a graph
// without vertices).
__global__ void k_batch_finish(int ngraphs, const int *__restrict__ vtx_off, const int *__restrict__ src,
                               const int *__restrict__ lastk, int *__restrict__ labels, int *__restrict__ iters,
                               int final_iter, int capped) {
    const int g = blockIdx.x;
    if (g >= ngraphs) return;
    const int v0 = vtx_off[g], v1 = vtx_off[g + 1];
    for (int u = v0 + (int)threadIdx.x; u < v1; u += blockDim.x) labels[u] = src[u] - v0;
    if (threadIdx.x == 0) {
        // lastk[v0] holds the last iteration in which a grandparent of graph g changed
        const int m = v1 > v0 ? lastk[v0] : 0;
        // an empty graph needs no iteration (the solo call returns at once)
        iters[g] = v1 == v0 ? 0 : ((capped && m == final_iter) ? -1 : m + 1);
    }
}

// ---------------------------------------------------------------------------
// Serving pool.  A resident graph owns the pool vertices [vb, vb+n] (the extra
// vertex n only carries row_ptr[vb+n] = the graph's entry end) and the pool
// entries [eb, eb+nnz); ids in f and gf are pool-global.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_owner(const int *__restrict__ off, int count, int64_t x) {
    int lo = 0, hi = count - 1;  // last k with off[k] <= x
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// End of a serving step for every resident graph k (run[k]): whether it
// changed in this step and the total degree of its next frontier go straight
// to the host (flag and edge buffers in page-locked memory), and a graph that
// converged in this step, or was cancelled, leaves: its local labels go to
// the page-locked out buffer at its pool positions (not for a cancelled one)
// and its n + 1 pool vertices return to the neutral state (f = gf = mngf =
// vbase = u, lastk = 0; vbase = u keeps every free vertex a run of its own
// for the grandparent pass's per-graph sums).  Block b works on graph
// find_owner(blk_off, nrun, b), vertices [c * kSettleChunk, (c + 1) *
// kSettleChunk) with c = b - blk_off[k].  The flag is read from lastk[vb],
// which the reset of vertex vb may set to 0 meanwhile; either value tells a
// graph that converged (its lastk[vb] is below the step) apart from one that
// changed.  It also clears next_ic, the counters the next step's
// grandparent pass accumulates into.
__global__ __launch_bounds__(256) void k_srv_settle(int nrun, const SrvRun *__restrict__ run,
                                                    const int *__restrict__ blk_off, int step,
                                                    int *__restrict__ lastk, int *__restrict__ gedge,
                                                    int *__restrict__ h_flag, int *__restrict__ h_edges,
                                                    int *__restrict__ h_out, int *__restrict__ F0,
                                                    int *__restrict__ F1, int *__restrict__ G, int *__restrict__ M,
                                                    int *__restrict__ vbase, IterCounters *__restrict__ next_ic) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the next step's counters (this step's push has read them already)
        next_ic->packed = 0ull;
        next_ic->atomics = 0ull;
    }
    const int k = find_owner(blk_off, nrun, blockIdx.x);
    const int c = blockIdx.x - blk_off[k];
    const SrvRun r = run[k];
    const bool changed = !r.cancel && lastk[r.vb] == step;
    if (c == 0 && threadIdx.x == 0) {
        h_flag[k] = changed ? 1 : 0;
        h_edges[k] = gedge[r.vb];
        gedge[r.vb] = 0;
    }
    if (changed) return;
    const int end = min((c + 1) * kSettleChunk, r.n + 1);
    for (int i = c * kSettleChunk + threadIdx.x; i < end; i += blockDim.x) {
        const int u = r.vb + i;
        if (i < r.n && !r.cancel) h_out[u] = G[u] - r.vb;
        F0[u] = u; F1[u] = u; G[u] = u; M[u] = u;
        vbase[u] = u;
        lastk[u] = 0;
    }
}

// Batched admission.  For new graph k (descriptor SrvNew), staged CSR in
// `stage` (row_ptr at s_rp, col at s_col, both local) goes to the pool:
// row_ptr rebased to the pool entry base, col copied, and the vertex state of
// [vb, vb+n] set to its neutral start (f = gf = mngf = global id).  Work items
// are numbered across the batch; item_off is the exclusive prefix of the
// per-graph item counts (2(n+1) + nnz).

// Placement of newly admitted graphs: one workgroup per chunk of the
// per-step chunk table.  Part 0 of graph k covers its vertex slots 0..n
// (row pointer rebased to the pool, neutral-state init); part 1 its column ids
// (only when they were not copied by DMA).  Sources are device-visible: the
// staging buffer, or page-locked host memory read in place.
__global__ __launch_bounds__(256) void k_srv_place(const PlaceChunk *__restrict__ chunks,
                                                   const SrvNew *__restrict__ desc,
                                                   const int *const *__restrict__ srcs, int *__restrict__ rp,
                                                   int *__restrict__ col, int *__restrict__ F0, int *__restrict__ F1,
                                                   int *__restrict__ G, int *__restrict__ M, int *__restrict__ vbase,
                                                   int *__restrict__ lastk, Tile *__restrict__ tiles) {
    const PlaceChunk c = chunks[blockIdx.x];
    const SrvNew d = desc[c.k];
    const int end = c.start + c.count;
    if (c.part == 0) {
        const int *__restrict__ srp = srcs[2 * c.k];
        Tile *tb = tiles + d.tile_base;
        for (int i = c.start + threadIdx.x; i < end; i += blockDim.x) {
            const int u = d.vb + i;
            const int s0 = srp[i];
            rp[u] = s0 + d.eb;
            F0[u] = u; F1[u] = u; G[u] = u; M[u] = u;
            vbase[u] = d.vb;
            lastk[u] = 0;
            if (i == d.n) continue;
            // the graph's tiles for its dense first iteration: the row holding
            // a tile's first entry writes its range and r_lo, the row holding
            // its last entry r_hi (each tile has one writer of each)
            const int e0 = srp[i + 1];
            for (int t = s0 / kTileEntries; s0 < e0 && t <= (e0 - 1) / kTileEntries; ++t) {
                const int t0 = t * kTileEntries;
                const int last = min(t0 + kTileEntries, d.nnz) - 1;
                if (t0 >= s0 && t0 < e0) {
                    tb[t].e0 = d.eb + t0;
                    tb[t].e1 = d.eb + last + 1;
                    tb[t].r_lo = u;
                }
                if (last >= s0 && last < e0) tb[t].r_hi = u;
            }
        }
        return;
    }
    // column ids: kPlaceUnroll independent loads in flight per thread
    const int *__restrict__ scol = srcs[2 * c.k + 1];
    int *__restrict__ dst = col + d.eb;
    for (int base = c.start + threadIdx.x; base < end; base += kPlaceUnroll * blockDim.x) {
        int v[kPlaceUnroll];
#pragma unroll
        for (int q = 0; q < kPlaceUnroll; ++q) {
            const int idx = base + q * blockDim.x;
            v[q] = scol[idx < end ? idx : c.start];
        }
#pragma unroll
        for (int q = 0; q < kPlaceUnroll; ++q) {
            const int idx = base + q * blockDim.x;
            if (idx < end) dst[idx] = v[q];
        }
    }
}


}  // namespace fsv
