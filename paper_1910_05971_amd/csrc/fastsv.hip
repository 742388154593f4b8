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
constexpr int kGpThreads = 256;
constexpr int kGpPerThread = 4;
constexpr int kGpBlockVerts = kGpThreads * kGpPerThread;

// ---- sparse push kernel geometry ----
constexpr int kPushThreads = 256;
constexpr int kPushSlots = 2048;              // edge slots per workgroup

struct Tile {
    int e0, e1;      // entry range [e0, e1)
    int r_lo, r_hi;  // rows containing entries e0 and e1-1
};

// Per-iteration counters written by the grandparent pass (two slots, used
// alternately by consecutive iterations).
struct IterCounters {
    unsigned long long changed;   // entries of gf that changed (termination test)
    unsigned long long frontier;  // high 32 bits: frontier vertices, low 32: their total degree
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
__device__ __forceinline__ void finish_row(int u, int m, bool shared_row, const int *__restrict__ F,
                                           int *__restrict__ Fn, const int *__restrict__ G,
                                           int *__restrict__ M) {
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
        for (int i = 0; i < 2; ++i) {
            ctr->it[i].changed = 0ull;
            ctr->it[i].frontier = 0ull;
        }
        ctr->status = 0;
    }
}

// ---------------------------------------------------------------------------
// Dense hooking: pull SpMV over (select2nd, min) fused with the hooks.
// One wave per tile of 1024 consecutive entries; lane l owns entries
// [e0 + 16 l, e0 + 16 l + 16).  Rows of the tile are located through a copy of
// row_ptr[r_lo .. r_hi+1] in LDS.  Each lane reduces its rows sequentially;
// rows crossing lanes are combined with a segmented min-scan, and rows
// crossing tiles update M atomically.
// ---------------------------------------------------------------------------
template <bool kHasBase>
__global__ __launch_bounds__(kWave *kHookWaves) void k_hook_dense(
    const Tile *__restrict__ tiles, int ntiles, const int *__restrict__ rp, const int *__restrict__ col,
    const int *__restrict__ vbase, const int *__restrict__ F, int *__restrict__ Fn,
    const int *__restrict__ G, int *__restrict__ M) {
    __shared__ int win[kHookWaves][kRowWin];
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int t = blockIdx.x * kHookWaves + wave;
    const bool tile_ok = t < ntiles;
    Tile T = tile_ok ? tiles[t] : Tile{0, 0, 0, -1};
    const int nwin = T.r_hi - T.r_lo + 2;  // row_ptr[r_lo .. r_hi+1]
    const bool in_lds = nwin <= kRowWin;
    if (tile_ok && in_lds)
        for (int i = lane; i < nwin; i += kWave) win[wave][i] = rp[T.r_lo + i];
    __syncthreads();
    if (!tile_ok) return;
    const int *wrow = &win[wave][0];
    auto rpw = [&](int r) -> int { return in_lds ? wrow[r - T.r_lo] : rp[r]; };

    const int a = T.e0 + lane * kPerLane;
    const int cnt = max(0, min(kPerLane, T.e1 - a));

    int g[kPerLane];
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
    if (!kHasBase) {
        int c[kPerLane];
        if (cnt == kPerLane && ((reinterpret_cast<uintptr_t>(col + a) & 15) == 0)) {
            const int4 *p = reinterpret_cast<const int4 *>(col + a);
#pragma unroll
            for (int q = 0; q < kPerLane / 4; ++q) {
                int4 v = p[q];
                c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kPerLane; ++j) c[j] = j < cnt ? col[a + j] : 0;
        }
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) g[j] = j < cnt ? G[c[j]] : INT_MAX;
    } else {
        // batched graphs: local column ids, shifted by the base of the row's graph
        int r = row0, nx = nxt, b = cnt > 0 ? vbase[row0] : 0;
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            if (j < cnt) {
                int e = a + j;
                if (e >= nx) {
                    do { ++r; nx = rpw(r + 1); } while (e >= nx);
                    b = vbase[r];
                }
                g[j] = G[col[e] + b];
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
                    finish_row(row, cur, false, F, Fn, G, M);  // row started and ended in this lane
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
        finish_row(row0, m, rpw(row0) < T.e0, F, Fn, G, M);
    }
    const bool ends_here = lane == kWave - 1 || next_cnt == 0 || next_head;
    if (ends_here) {
        bool shared_row = rpw(row) < T.e0 || rpw(row + 1) > T.e1;
        finish_row(row, S, shared_row, F, Fn, G, M);
    }
}

// ---------------------------------------------------------------------------
// Grandparent pass + termination test + frontier compaction.
//   G_k[u] = Fn[Fn[u]];  changed = G_k[u] != G_{k-1}[u];  NextFn[u] = G_k[u]
// Every changed vertex counts for the termination test.  When requested,
// changed vertices with at least one stored entry are also appended to the
// frontier list together with the exclusive prefix of their degrees (the
// sparse push balances edge slots with it).  One atomic per block and counter.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kGpThreads) void k_grandparent(
    int n, const int *__restrict__ Fn, int *__restrict__ G, int *__restrict__ next_fn,
    const int *__restrict__ rp, int *__restrict__ frontier, int *__restrict__ eoff,
    IterCounters *__restrict__ ctr, int write_frontier, int *__restrict__ lastk, int iter) {
    __shared__ int s_chg[kGpThreads / kWave];
    __shared__ int s_cnt[kGpPerThread][kGpThreads / kWave];
    __shared__ int s_deg[kGpPerThread][kGpThreads / kWave];
    __shared__ unsigned long long s_base;
    const int wave = threadIdx.x / kWave;
    const int lane = lane_id();
    const int base_u = blockIdx.x * kGpBlockVerts;
    bool ch[kGpPerThread], fr[kGpPerThread];
    int deg[kGpPerThread];
    int nchg = 0;
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        int u = base_u + i * kGpThreads + threadIdx.x;
        ch[i] = false;
        fr[i] = false;
        deg[i] = 0;
        if (u < n) {
            int p = Fn[u];
            int g = Fn[p];
            int old = G[u];
            next_fn[u] = g;
            if (g != old) {
                G[u] = g;
                ch[i] = true;
                ++nchg;
                if (lastk) lastk[u] = iter;
                if (write_frontier) {
                    deg[i] = rp[u + 1] - rp[u];
                    fr[i] = deg[i] > 0;
                }
            }
        }
    }
    int wchg = wave_incl_sum(nchg);
    if (lane == kWave - 1) s_chg[wave] = wchg;
    int rank[kGpPerThread], dpre[kGpPerThread];
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        unsigned long long bal = __ballot(fr[i]);
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
        unsigned long long c = 0, d = 0, tot = 0;
        for (int w = 0; w < kGpThreads / kWave; ++w) tot += (unsigned)s_chg[w];
        for (int i = 0; i < kGpPerThread; ++i)
            for (int w = 0; w < kGpThreads / kWave; ++w) {
                int cc = s_cnt[i][w], dd = s_deg[i][w];
                s_cnt[i][w] = (int)c;
                s_deg[i][w] = (int)d;
                c += cc;
                d += dd;
            }
        if (tot) atomicAdd(&ctr->changed, tot);
        s_base = c ? atomicAdd(&ctr->frontier, (c << 32) | d) : 0ull;
    }
    __syncthreads();
    if (!write_frontier) return;
    const unsigned long long b = s_base;
    const int bc = (int)(b >> 32), bd = (int)(b & 0xffffffffull);
#pragma unroll
    for (int i = 0; i < kGpPerThread; ++i) {
        if (fr[i]) {
            int u = base_u + i * kGpThreads + threadIdx.x;
            int pos = bc + s_cnt[i][wave] + rank[i];
            frontier[pos] = u;
            eoff[pos] = bd + s_deg[i][wave] + dpre[i];
        }
    }
}

__global__ void k_zero_iter_counters(IterCounters *c) {
    if (threadIdx.x == 0) {
        c->changed = 0ull;
        c->frontier = 0ull;
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
    const int nv = i1 - i0 + 1;  // <= kPushSlots: every frontier vertex has degree >= 1
    for (int i = threadIdx.x; i < nv; i += kPushThreads) {
        int v = frontier[i0 + i];
        s_off[i] = eoff[i0 + i];
        s_row[i] = rp[v];
        s_val[i] = G[v];
        if (kHasBase) s_base[i] = vbase[v];
    }
    __syncthreads();
    for (int s = s0 + threadIdx.x; s < s1; s += kPushThreads) {
        // frontier entry owning slot s
        int lo = 0, hi = nv - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= s) lo = mid;
            else hi = mid - 1;
        }
        int u = col[s_row[lo] + (s - s_off[lo])];
        if (kHasBase) u += s_base[lo];
        int val = s_val[lo];
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

struct Workspace {
    int *F[2];
    int *M;
    int *frontier;
    int *eoff;
    Tile *tiles;
    Counters *ctr;
};

size_t ws_bytes_for(int64_t n, int64_t nnz, int64_t *ntiles_out) {
    int64_t ntiles = (nnz + kTileEntries - 1) / kTileEntries;
    if (ntiles_out) *ntiles_out = ntiles;
    size_t vec = align256(sizeof(int) * (size_t)(n > 0 ? n : 1));
    return 5 * vec + align256(sizeof(Tile) * (size_t)(ntiles > 0 ? ntiles : 1)) + align256(sizeof(Counters));
}

Workspace carve(void *base, int64_t n, int64_t ntiles) {
    char *p = static_cast<char *>(base);
    size_t vec = align256(sizeof(int) * (size_t)(n > 0 ? n : 1));
    Workspace w;
    w.F[0] = reinterpret_cast<int *>(p); p += vec;
    w.F[1] = reinterpret_cast<int *>(p); p += vec;
    w.M = reinterpret_cast<int *>(p); p += vec;
    w.frontier = reinterpret_cast<int *>(p); p += vec;
    w.eoff = reinterpret_cast<int *>(p); p += vec;
    w.tiles = reinterpret_cast<Tile *>(p); p += align256(sizeof(Tile) * (size_t)(ntiles > 0 ? ntiles : 1));
    w.ctr = reinterpret_cast<Counters *>(p);
    return w;
}

inline int grid_for(int64_t items, int per_block, int cap = 1 << 30) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
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
    if (n < 0 || nnz < 0 || nnz > INT_MAX) return 0;
    return ws_bytes_for(n, nnz, nullptr);
}

int fastsv_cc_csr(fastsv_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                  int32_t *labels, void *d_ws, size_t ws_bytes, hipStream_t stream,
                  const fastsv_opts *opts_in, fastsv_stats *stats) {
    auto t_start = std::chrono::steady_clock::now();
    if (!ctx) return FASTSV_EINVAL;
    if (n < 0 || nnz < 0) return FASTSV_EINVAL;
    if (nnz > INT_MAX - kTileEntries) return FASTSV_EOVERFLOW;
    fastsv_opts opts = opts_in ? *opts_in : fastsv_default_opts();
    if (!(opts.frontier_tau >= 0.0f)) return FASTSV_EINVAL;  // also rejects NaN
    if (stats) memset(stats, 0, sizeof(*stats));
    if (n == 0) return FASTSV_OK;
    if (!rp || !labels || (nnz > 0 && !col)) return FASTSV_EINVAL;
    int64_t ntiles = 0;
    size_t need = ws_bytes_for(n, nnz, &ntiles);
    HIP_TRY(hipSetDevice(ctx->device));
    if (d_ws) {
        if (ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return FASTSV_EINVAL;
    } else {
        if (ctx->ws_size < need) {
            if (ctx->ws) HIP_TRY(hipFree(ctx->ws));
            ctx->ws = nullptr;
            ctx->ws_size = 0;
            if (hipMalloc(&ctx->ws, need) != hipSuccess) return FASTSV_ENOMEM;
            ctx->ws_size = need;
        }
        d_ws = ctx->ws;
    }
    if (opts.timing && !ctx->events) {
        for (auto &e : ctx->ev) HIP_TRY(hipEventCreate(&e));
        ctx->events = true;
    }
    Workspace w = carve(d_ws, n, ntiles);
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
    int64_t prev_changed = n, prev_fcnt = 0, prev_edges = nnz;
    bool frontier_ready = false;
    const double tau_edges = (double)opts.frontier_tau * (double)nnz;
    int64_t alg = 0;
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
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[0], stream));
        if (sparse) {
            if (prev_edges > 0)
                hipLaunchKernelGGL(k_hook_sparse<false>, dim3(grid_for(prev_edges, kPushSlots)), dim3(kPushThreads), 0,
                                   stream, w.frontier, w.eoff, (int)prev_fcnt, (int)prev_edges, rp, col, nullptr, F,
                                   Fn, G, w.M);
            // frontier ids, offsets, row starts and values; per slot col and an M read-modify-write
            alg += 16 * prev_fcnt + 12 * prev_edges;
        } else {
            if (ntiles > 0)
                hipLaunchKernelGGL(k_hook_dense<false>, dim3(grid_for(ntiles, kHookWaves)), dim3(kWave * kHookWaves), 0,
                                   stream, w.tiles, (int)ntiles, rp, col, nullptr, F, Fn, G, w.M);
            // row_ptr, col, gathers of G[col], then G[u], F[u], M[u] per row
            alg += 4 * ((int64_t)n + 1) + 8 * nnz + 12 * (int64_t)n;
        }
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[1], stream));
        hipLaunchKernelGGL(k_zero_iter_counters, dim3(1), dim3(64), 0, stream, ic);
        const bool want_frontier = opts.frontier_tau > 0.0f && prev_changed < (int64_t)n / 2 + 1;
        hipLaunchKernelGGL(k_grandparent, dim3(grid_for(n, kGpBlockVerts)), dim3(kGpThreads), 0, stream, n, Fn, G, F, rp,
                           w.frontier, w.eoff, ic, want_frontier ? 1 : 0, nullptr, it);
        HIP_TRY(hipGetLastError());
        if (timed) HIP_TRY(hipEventRecord(ctx->ev[2], stream));
        HIP_TRY(hipMemcpyAsync(hc, ic, sizeof(IterCounters), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const int64_t changed = (int64_t)hc->changed;
        const int64_t fcnt = (int64_t)(hc->frontier >> 32);
        const int64_t edges = (int64_t)(hc->frontier & 0xffffffffull);
        // read Fn[u], gather Fn[Fn[u]], read G[u], write G[u] and the next seed
        alg += 20 * (int64_t)n + (want_frontier ? 8 * fcnt : 0);
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
        prev_changed = changed;
        prev_fcnt = fcnt;
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
