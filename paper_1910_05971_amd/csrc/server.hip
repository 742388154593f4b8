// Continuous-batching server for connected-components requests.
//
// Resident graphs share one device pool and advance together: every step is
// one iteration of Algorithm 3 (dense pull over the resident graphs' tiles or
// sparse push over the frontier, then the grandparent pass) for all of them.
// A graph leaves at the end of the first step in which none of its
// grandparents changed (the termination test of Sec. 3.4 applied to that
// graph alone); its labels reach the caller when that step returns.  Ids in f
// and gf are pool-global, so resident graphs never exchange values and each
// one follows exactly the iterates it would follow when solved alone.
//
// Admission is first-come first-served and by footprint: a request waits
// until a slot, n+1 pool vertices and nnz pool entries are free.
//
// One step: the iteration runs on the server's stream with a single host
// synchronisation, and admission runs beside it on two copy streams:
//   0. graphs whose admission copies have completed (polled with events)
//      join the running set; vertex, entry and tile ranges freed by the
//      previous step return to their allocators
//   1. admission of up to about kSrvStepAdmitBytes of requests: one placement
//      launch on the copy stream reads the row pointers and small column
//      arrays in place from page-locked host memory (pageable ones are staged
//      by DMA first), large or pageable column arrays go by DMA on the second
//      copy stream, and the tiles are built.  Small admissions with nothing
//      waiting behind them run in this step already (the step's stream waits
//      for their placement); the others start at the first step after their
//      copies have completed, so that a long copy never holds up a step.
//   2. hooking, decided per graph: the dense pull over the graph's resident
//      tiles in its first iteration and whenever its frontier (total degree of
//      the grandparents that changed in the previous step) exceeds
//      frontier_tau * nnz; otherwise the sparse push from its frontier (the
//      push skips the graphs that run dense; frontier size read on the device)
//   3. grandparent pass over the pool, per graph: changed or not, and the
//      degree sum of its new frontier
//   4. settle pass: the per-graph flags and frontier sizes go straight to
//      page-locked host memory, and every graph that converged (or was
//      cancelled) writes its labels there too and returns its vertex range to
//      the neutral state, all in the same step; it also clears the next step's
//      counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "engine.h"
#include "fastsv.h"
#include "range_alloc.h"

using namespace fsv;

namespace {

struct Request {
    uint64_t ticket;
    int n;
    int64_t nnz;
    const int32_t *rp, *col;    // caller's host arrays, read at admission
    const int32_t *drp, *dcol;  // the same as device-visible addresses (page-locked memory), or null
    int32_t *labels_out;
    int32_t *iters_out;
};

// kStaged: placed (or being placed) on the copy streams; runs from the first
// step after its copies have completed
enum SlotState : int { kFree = 0, kRunning = 1, kStaged = 3 };

// pinned requests at least this large have their column ids copied by the DMA
// engine straight into the pool; smaller ones are read by the placement kernel
constexpr int64_t kSrvDmaMinEntries = 1 << 18;
// default bytes of graph data admitted per step (once at least one graph is
// admitted; opts.admit_mb): a step's transfers then take about as long as its
// compute, and the copy stream works on the next graphs while the resident
// ones iterate
constexpr int64_t kSrvStepAdmitBytes = int64_t(128) << 20;
// admissions of at most this many bytes, with no DMA and no request waiting
// behind them, run in the step that admits them
constexpr int64_t kSrvSameStepBytes = int64_t(4) << 20;
// admission generations (events and host buffers) in flight at once: a
// generation's buffers are reused kSrvGens steps later, after its placement
// stream work has completed
constexpr int kSrvGens = 8;

struct Slot {
    int state = kFree;
    uint64_t ticket = 0;
    int n = 0;
    int64_t nnz = 0;
    int vb = 0, eb = 0, tb = 0, ntiles = 0;
    int64_t fedge = 0;  // frontier degree sum after its last iteration
    int admit_step = 0;  // the step of its first iteration
    int gen = 0;         // admission generation while staged
    bool cancel = false;  // cancelled: leaves at the next step that settles it
    int32_t *labels_out = nullptr;
    int32_t *iters_out = nullptr;
};

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct PoolLayout {
    size_t rp, col, F0, F1, G, M, vbase, lastk, frontier, eoff, tiles, ctr, stage, adm, gmode, gedge, stepbuf, total;
};

// The per-step descriptor, copied to the device in one transfer: the resident
// graphs (SrvRun) and the settle pass's block offsets, the graphs running the
// dense pass (SrvNew as the kSrvGather pull reads it) and their tile offsets.
struct StepLayout {
    size_t run, blk_off, dense, off_dense, total;
};

inline StepLayout step_layout(int64_t S) {
    StepLayout L{};
    size_t p = 0;
    auto take = [&](size_t b) { size_t o = p; p += (b + 15) & ~size_t(15); return o; };
    L.run = take(sizeof(SrvRun) * (size_t)S);
    L.blk_off = take(sizeof(int) * (size_t)(S + 1));
    L.dense = take(sizeof(SrvNew) * (size_t)S);
    L.off_dense = take(sizeof(int) * (size_t)(S + 1));
    L.total = p;
    return L;
}

// Placement chunks one step can need: every admitted graph's vertex slots and
// column ids, cut into kPlaceChunk items (at most S graphs, V + S vertex slots
// and E entries in the pool).
inline int64_t max_place_chunks(int64_t V, int64_t E, int64_t S) {
    return (V + S + E) / kPlaceChunk + 2 * S + 2;
}

// One admission's arrays, packed for a single host-to-device copy (16-byte
// aligned): descriptors, source pointers, placement chunks.
struct AdmLayout {
    size_t desc, srcs, chunks, total;
};

inline AdmLayout adm_layout(int64_t nnew, int64_t nchunks) {
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    AdmLayout A;
    A.desc = 0;
    A.srcs = al(A.desc + sizeof(SrvNew) * (size_t)nnew);
    A.chunks = al(A.srcs + sizeof(void *) * 2 * (size_t)nnew);
    A.total = A.chunks + sizeof(PlaceChunk) * (size_t)nchunks;
    return A;
}

// the largest admission: every slot, every placement chunk the pool allows
inline size_t adm_bytes(int64_t V, int64_t E, int64_t S) { return adm_layout(S, max_place_chunks(V, E, S)).total; }

// T: tiles of one step's new graphs; the staging buffer holds the row_ptr and
// col of all graphs admitted in one step (at most V + E ints) and the labels
// of all graphs retired in one step (at most V ints).
PoolLayout pool_layout(int64_t V, int64_t E, int64_t T, int64_t S) {
    PoolLayout L{};
    size_t p = 0;
    auto take = [&](size_t b) { size_t o = p; p += a256(b > 0 ? b : 1); return o; };
    const size_t v4 = sizeof(int) * (size_t)V;
    L.rp = take(sizeof(int) * (size_t)(V + 1));
    L.col = take(sizeof(int) * (size_t)E);
    L.F0 = take(v4);
    L.F1 = take(v4);
    L.G = take(v4);
    L.M = take(v4);
    L.vbase = take(v4);
    L.lastk = take(v4);
    L.frontier = take(v4);
    L.eoff = take(v4);
    L.tiles = take(sizeof(Tile) * (size_t)T);
    L.ctr = take(sizeof(Counters));
    L.stage = take(sizeof(int) * (size_t)(V + 1 + E));
    L.adm = take(adm_bytes(V, E, S));
    L.gmode = take(v4);
    L.gedge = take(v4);
    L.stepbuf = take(step_layout(S).total);
    L.total = p;
    return L;
}

}  // namespace

struct fastsv_server {
    fastsv_ctx *ctx = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cs = nullptr;            // placement stream: admission overlaps the compute of a step
    hipStream_t ds = nullptr;            // DMA stream for large column arrays, beside the placement
    hipEvent_t ev_placed[kSrvGens] = {};  // on cs: the graphs admitted at a step are in the pool
    hipEvent_t ev_dma[kSrvGens] = {};     // on ds: their DMA'd column arrays are too
    fastsv_opts opts{};
    int64_t V = 0, E = 0, T = 0;
    int S = 0;
    int64_t admit_bytes = 0;  // graph bytes admitted per step once one graph is in
    char *pool = nullptr;
    PoolLayout L{};
    int *rp, *col, *F[2], *G, *M, *vbase, *lastk, *frontier, *eoff, *stage, *gmode, *gedge;
    PlaceChunk *chunks;
    SrvNew *desc;
    const int **srcs;
    Tile *tiles;
    Counters *ctr;
    char *stepbuf;  // device copy of the step descriptor
    StepLayout SL{};
    // page-locked host memory that the settle pass writes directly (device
    // addresses in the d_ copies): labels at pool positions, per-graph flags
    // and frontier sizes
    int *h_out = nullptr, *h_flags = nullptr, *h_edges = nullptr;
    int *d_out = nullptr, *d_flags = nullptr, *d_edges = nullptr;
    char *h_step = nullptr;  // the step descriptor
    // admission buffers, rotating over kSrvGens generations, since the copy
    // streams may still read earlier steps' while the host prepares the next
    PlaceChunk *h_chunks2[kSrvGens] = {};
    SrvNew *h_desc2[kSrvGens] = {};
    const int **h_srcs2[kSrvGens] = {};
    char *h_adm2[kSrvGens] = {};  // the four arrays above packed for one copy
    char *adm = nullptr;          // its device copy
    bool next_ic_clean = true;    // the next step's counters were cleared by a settle pass
    std::vector<char> step_last;  // the step descriptor bytes the device holds
    size_t step_held = 0;
    RangeAlloc va, ea, ta;
    // ranges of graphs that left in the current step: allocatable from the
    // next step on, after their reset (compute stream) has completed, so that
    // the copy streams never wait for the compute stream
    std::vector<std::pair<int64_t, int64_t>> rel_v, rel_e, rel_t;
    std::deque<Request> queue;
    std::vector<Slot> slots;
    std::vector<int> free_slots;  // stack of free slot indices
    // the slots in use (staged or running), in admission order: a step
    // visits these only, however many slots the server was created with
    std::vector<int> active;
    std::vector<int> run_slot;    // slot of each entry of the step's run list
    std::deque<uint64_t> done;
    int step = 0;
    uint64_t next_ticket = 1;
    fastsv_server_stats st{};
};

#define SRV_TRY(expr)                                              \
    do {                                                           \
        hipError_t _e = (expr);                                    \
        if (_e != hipSuccess) {                                    \
            if (getenv("FASTSV_DEBUG"))                            \
                fprintf(stderr, "fastsv server: %s failed: %s\n",   \
                        #expr, hipGetErrorString(_e));             \
            return FASTSV_EHIP;                                    \
        }                                                          \
    } while (0)

namespace {

// Device address of page-locked host memory, or null for pageable memory.
const int32_t *device_view(const int32_t *h) {
    if (!h) return nullptr;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, h) != hipSuccess) {
        (void)hipGetLastError();  // pageable memory: clear the error, copy instead
        return nullptr;
    }
    if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
    return static_cast<const int32_t *>(a.devicePointer);
}

template <typename T>
bool pinned(T **p, size_t count) {
    return hipHostMalloc(reinterpret_cast<void **>(p), sizeof(T) * (count > 0 ? count : 1), hipHostMallocDefault) ==
           hipSuccess;
}

// Page-locked host memory that kernels write directly and the host reads
// after a stream synchronisation: coherent (not cached on the device) and
// mapped; *dev receives its device address.
template <typename T>
bool pinned_mapped(T **p, T **dev, size_t count) {
    if (hipHostMalloc(reinterpret_cast<void **>(p), sizeof(T) * (count > 0 ? count : 1),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return false;
    return hipHostGetDevicePointer(reinterpret_cast<void **>(dev), *p, 0) == hipSuccess && *dev;
}

}  // namespace

extern "C" {

size_t fastsv_server_pool_bytes(int32_t max_vertices, int64_t max_entries, int32_t max_slots) {
    if (max_vertices <= 0 || max_entries < 0 || max_slots <= 0 || max_entries > INT32_MAX - kTileEntries ||
        (int64_t)max_vertices + 1 + max_entries > INT32_MAX)
        return 0;
    const int64_t T = max_entries / kTileEntries + max_slots;
    return pool_layout(max_vertices, max_entries, T, max_slots).total;
}

int fastsv_server_create(fastsv_ctx *ctx, int32_t max_vertices, int64_t max_entries, int32_t max_slots,
                         hipStream_t stream, const fastsv_opts *opts, fastsv_server **out) {
    if (!out) return FASTSV_EINVAL;
    *out = nullptr;
    if (!ctx || max_vertices <= 0 || max_entries < 0 || max_slots <= 0) return FASTSV_EINVAL;
    if (max_entries > INT32_MAX - kTileEntries || (int64_t)max_vertices + 1 + max_entries > INT32_MAX)
        return FASTSV_EOVERFLOW;
    fastsv_server *s = new (std::nothrow) fastsv_server();
    if (!s) return FASTSV_ENOMEM;
    s->ctx = ctx;
    s->device = ctx_device(ctx);
    s->stream = stream;
    s->opts = opts ? *opts : fastsv_default_opts();
    if (!(s->opts.frontier_tau >= 0.0f) || s->opts.admit_mb < 0 || s->opts.admit_mb > 4096) {
        delete s;
        return FASTSV_EINVAL;
    }
    s->admit_bytes = s->opts.admit_mb > 0 ? (int64_t)s->opts.admit_mb << 20 : kSrvStepAdmitBytes;
    s->V = max_vertices;
    s->E = max_entries;
    s->T = max_entries / kTileEntries + max_slots;
    s->S = max_slots;
    s->L = pool_layout(s->V, s->E, s->T, s->S);
    if (hipSetDevice(s->device) != hipSuccess) { delete s; return FASTSV_EHIP; }
    if (hipMalloc(reinterpret_cast<void **>(&s->pool), s->L.total) != hipSuccess) { delete s; return FASTSV_ENOMEM; }
    char *p = s->pool;
    s->rp = reinterpret_cast<int *>(p + s->L.rp);
    s->col = reinterpret_cast<int *>(p + s->L.col);
    s->F[0] = reinterpret_cast<int *>(p + s->L.F0);
    s->F[1] = reinterpret_cast<int *>(p + s->L.F1);
    s->G = reinterpret_cast<int *>(p + s->L.G);
    s->M = reinterpret_cast<int *>(p + s->L.M);
    s->vbase = reinterpret_cast<int *>(p + s->L.vbase);
    s->lastk = reinterpret_cast<int *>(p + s->L.lastk);
    s->frontier = reinterpret_cast<int *>(p + s->L.frontier);
    s->eoff = reinterpret_cast<int *>(p + s->L.eoff);
    s->tiles = reinterpret_cast<Tile *>(p + s->L.tiles);
    s->ctr = reinterpret_cast<Counters *>(p + s->L.ctr);
    s->stage = reinterpret_cast<int *>(p + s->L.stage);
    s->adm = p + s->L.adm;
    s->gmode = reinterpret_cast<int *>(p + s->L.gmode);
    s->gedge = reinterpret_cast<int *>(p + s->L.gedge);
    s->stepbuf = p + s->L.stepbuf;
    s->SL = step_layout(s->S);
    // every host buffer below is the source or target of an asynchronous copy
    // or of direct device writes, and is written at most once per step
    bool ok = pinned_mapped(&s->h_out, &s->d_out, (size_t)s->V) &&
              pinned_mapped(&s->h_flags, &s->d_flags, max_slots) &&
              pinned_mapped(&s->h_edges, &s->d_edges, max_slots) && pinned(&s->h_step, s->SL.total);
    for (int b = 0; b < kSrvGens && ok; ++b)
        ok = pinned(&s->h_srcs2[b], 2 * (size_t)max_slots) && pinned(&s->h_desc2[b], max_slots) &&
             pinned(&s->h_chunks2[b], (size_t)max_place_chunks(s->V, s->E, s->S)) &&
             pinned(&s->h_adm2[b], adm_bytes(s->V, s->E, s->S));
    if (!ok) { fastsv_server_destroy(s); return FASTSV_ENOMEM; }
    // copy stream at the default priority, and its events
    bool evs_ok = hipStreamCreateWithFlags(&s->cs, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&s->ds, hipStreamNonBlocking) == hipSuccess;
    for (int g = 0; g < kSrvGens && evs_ok; ++g)
        evs_ok = hipEventCreateWithFlags(&s->ev_placed[g], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&s->ev_dma[g], hipEventDisableTiming) == hipSuccess;
    if (!evs_ok) {
        fastsv_server_destroy(s);
        return FASTSV_EHIP;
    }
    s->va.reset(s->V);
    s->ea.reset(s->E);
    s->ta.reset(s->T);
    s->slots.assign(max_slots, Slot{});
    s->active.reserve(max_slots);
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    // neutral state everywhere: every pool vertex its own root, empty rows
    launch_fill(stream, (int)(s->V + 1), s->rp, 0);
    launch_init(stream, (int)s->V, s->F[0], s->F[1], s->G, s->M, 0);
    launch_fill(stream, (int)s->V, s->lastk, 0);
    launch_fill_iota(stream, (int)s->V, s->vbase);  // a free vertex is a run of its own
    launch_fill(stream, (int)s->V, s->gmode, 0);
    launch_fill(stream, (int)s->V, s->gedge, 0);
    launch_zero_iter(stream, &s->ctr->it[0]);
    launch_zero_iter(stream, &s->ctr->it[1]);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
        fastsv_server_destroy(s);
        return FASTSV_EHIP;
    }
    *out = s;
    return FASTSV_OK;
}

void fastsv_server_destroy(fastsv_server *s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->cs) (void)hipStreamSynchronize(s->cs);
    if (s->ds) (void)hipStreamSynchronize(s->ds);
    if (s->pool) (void)hipFree(s->pool);
    for (void *h : {(void *)s->h_flags, (void *)s->h_out, (void *)s->h_edges, (void *)s->h_step})
        if (h) (void)hipHostFree(h);
    for (int g = 0; g < kSrvGens; ++g) {
        for (void *h : {(void *)s->h_desc2[g], (void *)s->h_chunks2[g], (void *)s->h_srcs2[g], (void *)s->h_adm2[g]})
            if (h) (void)hipHostFree(h);
        if (s->ev_placed[g]) (void)hipEventDestroy(s->ev_placed[g]);
        if (s->ev_dma[g]) (void)hipEventDestroy(s->ev_dma[g]);
    }
    if (s->cs) (void)hipStreamDestroy(s->cs);
    if (s->ds) (void)hipStreamDestroy(s->ds);
    delete s;
}

}  // extern "C"

namespace {

int submit_impl(fastsv_server *s, int32_t n, int64_t nnz, const int32_t *h_row_ptr, const int32_t *h_col,
                int32_t *h_labels_out, int32_t *h_iters_out, uint64_t *ticket, bool mapped) {
    if (!s || n < 0 || nnz < 0 || !h_row_ptr || (nnz > 0 && !h_col) || (n > 0 && !h_labels_out)) return FASTSV_EINVAL;
    if ((int64_t)n + 1 > s->V || nnz > s->E || (nnz + kTileEntries - 1) / kTileEntries > s->T) return FASTSV_ENOMEM;
    // with opts.validate, a host-side check of the CSR before it is ever
    // copied to the device; without it the caller guarantees a valid CSR
    if (h_row_ptr[0] != 0 || h_row_ptr[n] != nnz) return FASTSV_ERANGE;
    if (s->opts.validate) {
        for (int32_t u = 0; u < n; ++u)
            if (h_row_ptr[u] > h_row_ptr[u + 1]) return FASTSV_ERANGE;
        for (int64_t e = 0; e < nnz; ++e)
            if ((uint32_t)h_col[e] >= (uint32_t)n) return FASTSV_ERANGE;
    }
    Request r;
    r.ticket = s->next_ticket++;
    r.n = n;
    r.nnz = nnz;
    r.labels_out = h_labels_out;
    r.iters_out = h_iters_out;
    if (ticket) *ticket = r.ticket;
    s->st.submitted++;
    if (n == 0) {  // nothing to solve
        if (h_iters_out) *h_iters_out = 0;
        s->done.push_back(r.ticket);
        s->st.completed++;
        return FASTSV_OK;
    }
    r.rp = h_row_ptr;
    r.col = h_col;
    r.drp = mapped ? h_row_ptr : device_view(h_row_ptr);
    r.dcol = nnz > 0 ? (mapped ? h_col : device_view(h_col)) : r.drp;
    s->queue.push_back(r);
    return FASTSV_OK;
}

}  // namespace

extern "C" {

int fastsv_server_submit(fastsv_server *s, int32_t n, int64_t nnz, const int32_t *h_row_ptr, const int32_t *h_col,
                         int32_t *h_labels_out, int32_t *h_iters_out, uint64_t *ticket) {
    return submit_impl(s, n, nnz, h_row_ptr, h_col, h_labels_out, h_iters_out, ticket, false);
}

int fastsv_server_submit_mapped(fastsv_server *s, int32_t n, int64_t nnz, const int32_t *h_row_ptr,
                                const int32_t *h_col, int32_t *h_labels_out, int32_t *h_iters_out, uint64_t *ticket) {
    return submit_impl(s, n, nnz, h_row_ptr, h_col, h_labels_out, h_iters_out, ticket, true);
}

int fastsv_server_submit_batch(fastsv_server *s, int32_t count, const int32_t *n, const int64_t *nnz,
                               const int32_t *const *h_row_ptr, const int32_t *const *h_col,
                               int32_t *const *h_labels_out, int32_t *h_iters_out, uint64_t *tickets,
                               int32_t mapped, int32_t *n_accepted) {
    if (!s || count < 0 || (count > 0 && (!n || !nnz || !h_row_ptr || !h_col || !h_labels_out)) || !n_accepted)
        return FASTSV_EINVAL;
    *n_accepted = 0;
    for (int32_t i = 0; i < count; ++i) {
        const int st = submit_impl(s, n[i], nnz[i], h_row_ptr[i], h_col[i], h_labels_out[i],
                                   h_iters_out ? h_iters_out + i : nullptr, tickets ? tickets + i : nullptr,
                                   mapped != 0);
        if (st != FASTSV_OK) return st;
        *n_accepted = i + 1;
    }
    return FASTSV_OK;
}

namespace {

// 1 when every copy of the admission generation has completed, 0 when some
// is still in flight, negative on a HIP error.
int generation_done(fastsv_server *s, int gen) {
    for (hipEvent_t e : {s->ev_placed[gen], s->ev_dma[gen]}) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipErrorNotReady) return 0;
        if (q != hipSuccess) return FASTSV_EHIP;
    }
    return 1;
}

}  // namespace

int fastsv_server_step(fastsv_server *s, int32_t *n_resident, int32_t *n_queued) {
    if (!s) return FASTSV_EINVAL;
    SRV_TRY(hipSetDevice(s->device));
    hipStream_t st = s->stream;
    hipStream_t cs = s->cs;
    const int step = ++s->step;
    const int gen = step % kSrvGens;
    IterCounters *ic_front = &s->ctr->it[(step + 1) & 1];  // frontier left by the previous step
    IterCounters *ic = &s->ctr->it[step & 1];

    // 0. ranges freed by the previous step (their reset finished before that
    //    step's synchronisation returned), then the staged graphs whose
    //    admission copies have completed join
    for (auto &r : s->rel_v) s->va.release(r.first, r.second);
    for (auto &r : s->rel_e) s->ea.release(r.first, r.second);
    for (auto &r : s->rel_t) s->ta.release(r.first, r.second);
    s->rel_v.clear();
    s->rel_e.clear();
    s->rel_t.clear();
    int gen_state[kSrvGens];
    for (int g = 0; g < kSrvGens; ++g) gen_state[g] = -2;  // not queried yet
    int nrunning = 0;
    for (const int i : s->active) {
        Slot &sl = s->slots[i];
        if (sl.state == kStaged) {
            int &gs = gen_state[sl.gen];
            if (gs == -2) gs = generation_done(s, sl.gen);
            if (gs < 0) return FASTSV_EHIP;
            if (gs == 1) {
                sl.state = kRunning;
                sl.admit_step = step;
            }
        }
        nrunning += sl.state == kRunning;
    }

    // 1. admission, placed on the copy streams while this step computes.  The
    //    new vertex ranges hold the same values as the neutral state the
    //    resident graphs' whole-range kernels may touch (f = gf = mngf = u,
    //    lastk = 0), so the placement and those kernels cannot disturb each
    //    other.  A generation's host buffers are reused once its placement
    //    stream work (which reads them) has completed.
    SrvNew *h_desc = s->h_desc2[gen];
    const int **h_srcs = s->h_srcs2[gen];
    PlaceChunk *h_chunks = s->h_chunks2[gen];
    int nnew = 0, nchunks = 0;
    int64_t staged = 0;
    std::vector<int> admitted;
    int64_t admit_bytes = 0;
    bool any_dma = false;
    if (!s->queue.empty()) SRV_TRY(hipEventSynchronize(s->ev_placed[gen]));
    while (!s->queue.empty() && (nnew == 0 || admit_bytes < s->admit_bytes)) {
        if (s->free_slots.empty()) break;
        const int k = s->free_slots.back();
        Request &r = s->queue.front();
        const int ntiles = (int)((r.nnz + kTileEntries - 1) / kTileEntries);
        const int64_t vb = s->va.alloc(r.n + 1);
        if (vb < 0) break;
        const int64_t eb = s->ea.alloc(r.nnz);
        if (eb < 0) { s->va.release(vb, r.n + 1); break; }
        const int64_t tb = s->ta.alloc(ntiles);
        if (tb < 0) { s->va.release(vb, r.n + 1); s->ea.release(eb, r.nnz); break; }
        s->free_slots.pop_back();
        s->active.push_back(k);
        Slot &sl = s->slots[k];
        sl = Slot{};
        sl.state = kStaged;
        sl.ticket = r.ticket;
        sl.n = r.n;
        sl.nnz = r.nnz;
        sl.vb = (int)vb;
        sl.eb = (int)eb;
        sl.tb = (int)tb;
        sl.ntiles = ntiles;
        sl.gen = gen;
        sl.labels_out = r.labels_out;
        sl.iters_out = r.iters_out;
        admitted.push_back(k);
        SrvNew d{(int)vb, (int)eb, r.n, (int)r.nnz, (int)staged, (int)(staged + r.n + 1), (int)tb, 0};
        // row pointers: read in place when page-locked and small, else staged
        // by DMA; column ids: by DMA straight into the pool when pageable or
        // large, else read in place by the placement kernel
        const bool col_dma = r.nnz > 0 && (!r.dcol || r.nnz >= kSrvDmaMinEntries);
        // (row pointers of large graphs go by DMA too: the placement kernel
        // then reads them from device memory)
        if (r.drp && (int64_t)r.n + 1 < kSrvDmaMinEntries) {
            h_srcs[2 * nnew] = r.drp;
        } else {
            SRV_TRY(hipMemcpyAsync(s->stage + d.s_rp, r.rp, sizeof(int) * (size_t)(r.n + 1), hipMemcpyHostToDevice,
                                   cs));
            h_srcs[2 * nnew] = s->stage + d.s_rp;
            staged += r.n + 1;
        }
        if (col_dma) {
            SRV_TRY(hipMemcpyAsync(s->col + eb, r.col, sizeof(int) * (size_t)r.nnz, hipMemcpyHostToDevice, s->ds));
            any_dma = true;
        }
        h_srcs[2 * nnew + 1] = col_dma ? nullptr : r.dcol;
        h_desc[nnew] = d;
        for (int c0 = 0; c0 <= r.n; c0 += kPlaceChunk)
            h_chunks[nchunks++] = PlaceChunk{nnew, 0, c0, std::min(kPlaceChunk, r.n + 1 - c0)};
        if (!col_dma)
            for (int64_t c0 = 0; c0 < r.nnz; c0 += kPlaceChunk)
                h_chunks[nchunks++] = PlaceChunk{nnew, 1, (int)c0, (int)std::min<int64_t>(kPlaceChunk, r.nnz - c0)};
        admit_bytes += sizeof(int) * ((int64_t)r.n + 1 + r.nnz);
        ++nnew;
        s->queue.pop_front();
        s->st.admitted++;
    }
    if (nnew > 0) {
        // the admission's descriptors, source pointers and placement
        // chunks, packed and copied at once
        const AdmLayout A = adm_layout(nnew, nchunks);
        char *ha = s->h_adm2[gen];
        memcpy(ha + A.desc, h_desc, sizeof(SrvNew) * nnew);
        memcpy(ha + A.srcs, h_srcs, sizeof(void *) * 2 * nnew);
        memcpy(ha + A.chunks, h_chunks, sizeof(PlaceChunk) * nchunks);
        SRV_TRY(hipMemcpyAsync(s->adm, ha, A.total, hipMemcpyHostToDevice, cs));
        const SrvNew *d_desc = reinterpret_cast<const SrvNew *>(s->adm + A.desc);
        const int *const *d_srcs = reinterpret_cast<const int *const *>(s->adm + A.srcs);
        const PlaceChunk *d_chunks = reinterpret_cast<const PlaceChunk *>(s->adm + A.chunks);
        launch_srv_place(cs, nchunks, d_chunks, d_desc, d_srcs, s->rp, s->col, s->F[0], s->F[1], s->G, s->M,
                         s->vbase, s->lastk, s->tiles);
        SRV_TRY(hipGetLastError());
        SRV_TRY(hipEventRecord(s->ev_placed[gen], cs));
        SRV_TRY(hipEventRecord(s->ev_dma[gen], s->ds));
        // small admissions with nothing waiting behind them (or with nothing
        // else to run) start now: the step waits for their placement
        const bool now = !any_dma && (nrunning == 0 || (s->queue.empty() && admit_bytes <= kSrvSameStepBytes));
        if (now) {
            SRV_TRY(hipStreamWaitEvent(st, s->ev_placed[gen], 0));
            for (int k : admitted) {
                s->slots[k].state = kRunning;
                s->slots[k].admit_step = step;
            }
        }
    }

    // 2.-4. one iteration for every running graph, then the settle pass over
    //    the running and the cancelled graphs
    const StepLayout &SL = s->SL;
    SrvRun *h_run = reinterpret_cast<SrvRun *>(s->h_step + SL.run);
    int *h_blk = reinterpret_cast<int *>(s->h_step + SL.blk_off);
    SrvNew *h_dense = reinterpret_cast<SrvNew *>(s->h_step + SL.dense);
    int *h_off_dense = reinterpret_cast<int *>(s->h_step + SL.off_dense);
    int nrun = 0, ns = 0, vlow = INT32_MAX, vhigh = 0, ndense = 0, dense_tiles = 0, blocks = 0;
    int64_t fedge_all = 0;
    bool any_sparse = false;
    s->run_slot.clear();
    for (const int i : s->active) {
        Slot &sl = s->slots[i];
        // a cancelled graph is settled once its admission copies are complete
        const bool staged_cancel = sl.state == kStaged && sl.cancel && gen_state[sl.gen] == 1;
        if (sl.state != kRunning && !staged_cancel) continue;
        h_run[nrun] = SrvRun{sl.vb, sl.n, sl.cancel ? 1 : 0, 0};
        h_blk[nrun] = blocks;
        blocks += (sl.n + 1 + kSettleChunk - 1) / kSettleChunk;
        s->run_slot.push_back(i);
        ++nrun;
        if (sl.cancel) continue;
        ++ns;
        vlow = std::min(vlow, sl.vb);
        vhigh = std::max(vhigh, sl.vb + sl.n + 1);
        fedge_all += sl.fedge;
        const bool dense = sl.admit_step == step || (double)sl.fedge > (double)s->opts.frontier_tau * (double)sl.nnz;
        if (dense && sl.ntiles > 0) {
            h_dense[ndense] = SrvNew{sl.vb, sl.eb, sl.n, (int)sl.nnz, sl.ntiles, dense_tiles, sl.tb, 0};
            h_off_dense[ndense] = dense_tiles;
            ++ndense;
            dense_tiles += sl.ntiles;
        } else if (!dense) {
            any_sparse = true;
        }
    }
    if (nrun > 0) {
        h_blk[nrun] = blocks;
        h_off_dense[ndense] = dense_tiles;
        // one copy of the used part of the descriptor, skipped when the
        // device already holds the same bytes (the running set and its dense
        // choices often stay the same from one step to the next)
        const size_t bytes = ndense > 0 ? SL.off_dense + sizeof(int) * (size_t)(ndense + 1)
                                        : SL.blk_off + sizeof(int) * (size_t)(nrun + 1);
        const bool same = bytes <= s->step_held && !memcmp(s->step_last.data(), s->h_step, bytes);
        if (!same) {
            SRV_TRY(hipMemcpyAsync(s->stepbuf, s->h_step, bytes, hipMemcpyHostToDevice, st));
            s->step_last.assign(s->h_step, s->h_step + bytes);
            s->step_held = bytes;
        }
        const SrvRun *d_run = reinterpret_cast<const SrvRun *>(s->stepbuf + SL.run);
        const int *d_blk = reinterpret_cast<const int *>(s->stepbuf + SL.blk_off);
        const SrvNew *d_dense = reinterpret_cast<const SrvNew *>(s->stepbuf + SL.dense);
        const int *d_off_dense = reinterpret_cast<const int *>(s->stepbuf + SL.off_dense);
        int *F = s->F[(step + 1) & 1], *Fn = s->F[step & 1];
        if (ns > 0) {
            // (a step with a settle pass cleared these for this one)
            if (!s->next_ic_clean) launch_zero_iter(st, ic);
            if (ndense > 0) {
                launch_srv_dense(st, ndense, dense_tiles, d_dense, d_off_dense, s->tiles, s->gmode, step, s->rp,
                                 s->col, s->vbase, F, Fn, s->G, s->M);
                s->st.dense_steps++;
            }
            if (any_sparse) {
                // the push loops over the frontier (of all resident graphs) with
                // this many workgroups
                const int64_t want = (fedge_all + kPushSlots - 1) / kPushSlots;
                const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
                launch_sparse_dev(st, ic_front, nb, s->frontier, s->eoff, s->rp, s->col, s->vbase, F, Fn, s->G, s->M,
                                  s->gmode, step);
                s->st.sparse_steps++;
            }
            // the running graphs lie in [vlow, vhigh); below and above it the
            // pool holds only free or staged (unchanging) vertices
            launch_grandparent(st, vhigh, Fn, s->G, F, s->rp, s->frontier, s->eoff, ic, 1, s->lastk, step, s->vbase,
                               s->gedge, nullptr, vlow);
        }
        launch_srv_settle(st, nrun, blocks, d_run, d_blk, step, s->lastk, s->gedge, s->d_flags, s->d_edges, s->d_out,
                          s->F[0], s->F[1], s->G, s->M, s->vbase, &s->ctr->it[(step + 1) & 1]);
        SRV_TRY(hipGetLastError());
    }
    s->next_ic_clean = nrun > 0;
    SRV_TRY(hipStreamSynchronize(st));
    int left = 0;  // graphs that left in this step
    for (int j = 0; j < nrun; ++j) {
        const int i = s->run_slot[j];
        Slot &sl = s->slots[i];
        if (!sl.cancel && s->h_flags[j]) {
            sl.fedge = s->h_edges[j];
            continue;
        }
        if (!sl.cancel) {
            // converged in this step: labels and iteration count to the caller
            memcpy(sl.labels_out, s->h_out + sl.vb, sizeof(int) * (size_t)sl.n);
            if (sl.iters_out) *sl.iters_out = step - sl.admit_step + 1;
            s->done.push_back(sl.ticket);
            s->st.completed++;
        } else {
            s->st.cancelled++;
        }
        s->rel_v.emplace_back(sl.vb, sl.n + 1);
        s->rel_e.emplace_back(sl.eb, sl.nnz);
        s->rel_t.emplace_back(sl.tb, sl.ntiles);
        sl = Slot{};
        s->free_slots.push_back(i);
        ++left;
    }
    if (left > 0)
        s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                       [s](int i) { return s->slots[i].state == kFree; }),
                        s->active.end());
    s->st.steps++;
    if (n_resident) *n_resident = (int32_t)s->active.size();  // admitted and not left: running or staged
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return FASTSV_OK;
}

int fastsv_server_cancel(fastsv_server *s, uint64_t ticket) {
    if (!s) return FASTSV_EINVAL;
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
        if (it->ticket == ticket) {
            s->queue.erase(it);
            s->st.cancelled++;
            return FASTSV_OK;
        }
    for (const int i : s->active) {
        Slot &sl = s->slots[i];
        if (sl.ticket != ticket) continue;
        if (sl.cancel) return FASTSV_OK;
        if (sl.state == kStaged) {
            const int g = generation_done(s, sl.gen);
            if (g < 0) return FASTSV_EHIP;
            if (g == 0) return FASTSV_EBUSY;  // its admission copies are still in flight
        }
        sl.cancel = true;
        return FASTSV_OK;
    }
    return FASTSV_EINVAL;
}

int fastsv_server_poll(fastsv_server *s, uint64_t *done, int32_t cap, int32_t *n_done) {
    if (!s || cap < 0 || (cap > 0 && !done) || !n_done) return FASTSV_EINVAL;
    int32_t k = 0;
    while (k < cap && !s->done.empty()) {
        done[k++] = s->done.front();
        s->done.pop_front();
    }
    *n_done = k;
    return FASTSV_OK;
}

int fastsv_server_get_stats(const fastsv_server *s, fastsv_server_stats *out) {
    if (!s || !out) return FASTSV_EINVAL;
    *out = s->st;
    return FASTSV_OK;
}

}  // extern "C"
