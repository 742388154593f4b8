"""Seeded synthetic graph inputs (shared by the solver's tests, the bench and the
oracle-side tests).

The arithmetic lives in ``csrc/graphgen.c`` (counter-based SplitMix64, Lemire
range mapping, integer probability thresholds, COO -> symmetric CSR with
sorted rows).  Nothing here computes connected components.

Workload recipes (stand-ins for the paper's Table 1 datasets, which are not
available):

* ``er(n, m, seed)``       -- Erdos-Renyi multigraph, m uniform endpoint draws,
                              self loops dropped, duplicates kept.
* ``rmat(scale, ef, seed)``-- R-MAT a=.57 b=c=.19 d=.05, ids permuted, loops
                              dropped, duplicates kept (skewed web/social graphs).
* ``grid(r, c, p, seed)``  -- bond-percolated 4-neighbour lattice, ids permuted
                              (high-diameter graphs with many components).
* ``batch(G, seed)``       -- G Erdos-Renyi graphs, n log-uniform in
                              [64, 65536), average degree uniform in [2, 32].
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfastsv_gen.so")

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"graph generator library missing: {LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        vp = ctypes.c_void_p
        lib.gg_rng_at.restype = u64
        lib.gg_rng_at.argtypes = [u64, u64, u64]
        lib.gg_er_edges.restype = i64
        lib.gg_er_edges.argtypes = [u64, u64, i32, i64, vp, vp]
        lib.gg_permutation.restype = None
        lib.gg_permutation.argtypes = [u64, u64, i32, vp]
        lib.gg_rmat_edges.restype = i64
        lib.gg_rmat_edges.argtypes = [u64, i32, i64, u32, u32, u32, i32, vp, vp]
        lib.gg_grid_edges.restype = i64
        lib.gg_grid_edges.argtypes = [u64, i32, i32, u32, i32, vp, vp]
        lib.gg_csr_from_edges.restype = i32
        lib.gg_csr_from_edges.argtypes = [i32, i64, vp, vp, vp, vp]
        lib.gg_batch_sizes.restype = None
        lib.gg_batch_sizes.argtypes = [u64, i32, vp, vp]
        lib.gg_uniform.restype = ctypes.c_double
        lib.gg_uniform.argtypes = [u64, u64, u64]
        lib.gg_num_threads.restype = i32
        lib.gg_num_threads.argtypes = []
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def threshold(p: float) -> int:
    """32-bit integer threshold floor(p * 2^32), clamped to [0, 2^32-1]."""
    t = int(np.floor(p * 4294967296.0))
    return max(0, min(t, 4294967295))


@dataclasses.dataclass
class Graph:
    """Undirected graph as symmetric int32 CSR (rows sorted)."""
    name: str
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    m_eff: int           # undirected edges kept (nnz = 2*m_eff)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def rng_at(seed: int, stream: int, ctr: int) -> int:
    return int(_load().gg_rng_at(seed, stream, ctr))


def uniform(seed: int, stream: int, ctr: int) -> float:
    return float(_load().gg_uniform(seed, stream, ctr))


def permutation(n: int, seed: int, stream: int = 1) -> np.ndarray:
    perm = np.empty(n, dtype=np.int32)
    _load().gg_permutation(seed, stream, n, _ptr(perm))
    return perm


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric CSR: edge (u,v) stores v in row u and u in row v; rows sorted."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = int(src.shape[0])
    if dst.shape[0] != m:
        raise ValueError("src/dst length mismatch")
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(2 * m, dtype=np.int32)
    rc = _load().gg_csr_from_edges(n, m, _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col))
    if rc != 0:
        raise ValueError("edge ids out of range or too many entries for int32 CSR")
    return row_ptr, col


def er_edges(n: int, m: int, seed: int, stream: int = 0) -> tuple[np.ndarray, np.ndarray]:
    src = np.empty(max(m, 0), dtype=np.int32)
    dst = np.empty(max(m, 0), dtype=np.int32)
    k = _load().gg_er_edges(seed, stream, n, m, _ptr(src), _ptr(dst))
    if k < 0:
        raise MemoryError("generator allocation failed")
    return src[:k].copy(), dst[:k].copy()


def er(n: int, m: int, seed: int, stream: int = 0, name: str | None = None) -> Graph:
    src, dst = er_edges(n, m, seed, stream)
    rp, col = csr_from_edges(n, src, dst)
    return Graph(name or f"er_n{n}_m{m}_s{seed}", n, rp, col, int(src.shape[0]))


def rmat_edges(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
               permute: bool = True) -> tuple[np.ndarray, np.ndarray]:
    m = edge_factor << scale
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    ta, tb, tc = threshold(a), threshold(a + b), threshold(a + b + c)
    k = _load().gg_rmat_edges(seed, scale, m, ta, tb, tc, int(permute), _ptr(src), _ptr(dst))
    if k < 0:
        raise MemoryError("generator allocation failed")
    return src[:k], dst[:k]


def rmat(scale: int, edge_factor: int, seed: int, **kw) -> Graph:
    src, dst = rmat_edges(scale, edge_factor, seed, **kw)
    n = 1 << scale
    rp, col = csr_from_edges(n, src, dst)
    m_eff = int(src.shape[0])
    del src, dst
    return Graph(f"rmat_s{scale}_ef{edge_factor}_s{seed}", n, rp, col, m_eff)


def grid_edges(rows: int, cols: int, p: float, seed: int, permute: bool = True):
    nb = rows * (cols - 1) + (rows - 1) * cols
    src = np.empty(max(nb, 0), dtype=np.int32)
    dst = np.empty(max(nb, 0), dtype=np.int32)
    k = _load().gg_grid_edges(seed, rows, cols, threshold(p), int(permute), _ptr(src), _ptr(dst))
    if k < 0:
        raise MemoryError("generator allocation failed")
    return src[:k].copy(), dst[:k].copy()


def grid(rows: int, cols: int, p: float, seed: int, permute: bool = True) -> Graph:
    src, dst = grid_edges(rows, cols, p, seed, permute)
    n = rows * cols
    rp, col = csr_from_edges(n, src, dst)
    return Graph(f"grid_{rows}x{cols}_p{p}_s{seed}", n, rp, col, int(src.shape[0]))


@dataclasses.dataclass
class Batch:
    """G graphs concatenated: vertex/entry offsets, global row_ptr, local col ids."""
    n: np.ndarray         # int32[G]
    m_eff: np.ndarray     # int64[G]
    vtx_off: np.ndarray   # int32[G+1]
    edge_off: np.ndarray  # int32[G+1] (entry offsets into col)
    row_ptr: np.ndarray   # int32[sum n + 1], global entry positions
    col: np.ndarray       # int32[sum nnz], local ids

    @property
    def num_graphs(self) -> int:
        return int(self.n.shape[0])

    def graph(self, g: int) -> Graph:
        v0, v1 = int(self.vtx_off[g]), int(self.vtx_off[g + 1])
        e0, e1 = int(self.edge_off[g]), int(self.edge_off[g + 1])
        rp = (self.row_ptr[v0:v1 + 1] - e0).astype(np.int32)
        return Graph(f"batch_g{g}", v1 - v0, rp, self.col[e0:e1], int(self.m_eff[g]))


def batch_sizes(num_graphs: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    n = np.empty(num_graphs, dtype=np.int32)
    m = np.empty(num_graphs, dtype=np.int64)
    _load().gg_batch_sizes(seed, num_graphs, _ptr(n), _ptr(m))
    return n, m


def batch(num_graphs: int, seed: int, max_n: int | None = None) -> Batch:
    """Graph g: n_g vertices, m_g Erdos-Renyi draws from stream g of `seed`.

    ``max_n`` (tests only) caps n_g, scaling m_g by the same factor."""
    ns, ms = batch_sizes(num_graphs, seed)
    if max_n is not None:
        scale = np.minimum(1.0, max_n / ns.astype(np.float64))
        ns = np.minimum(ns, max_n).astype(np.int32)
        ms = np.round(ms * scale).astype(np.int64)
    rps, cols, meff = [], [], []
    for g in range(num_graphs):
        src, dst = er_edges(int(ns[g]), int(ms[g]), seed, g)
        rp, col = csr_from_edges(int(ns[g]), src, dst)
        rps.append(rp)
        cols.append(col)
        meff.append(src.shape[0])
    vtx_off = np.zeros(num_graphs + 1, dtype=np.int64)
    vtx_off[1:] = np.cumsum(ns)
    nnzs = np.array([c.shape[0] for c in cols], dtype=np.int64)
    edge_off = np.zeros(num_graphs + 1, dtype=np.int64)
    edge_off[1:] = np.cumsum(nnzs)
    if edge_off[-1] >= 2**31 or vtx_off[-1] >= 2**31:
        raise ValueError("batch too large for int32 offsets")
    row_ptr = np.empty(int(vtx_off[-1]) + 1, dtype=np.int32)
    for g in range(num_graphs):
        row_ptr[vtx_off[g]:vtx_off[g + 1]] = rps[g][:-1] + edge_off[g]
    row_ptr[-1] = edge_off[-1]
    col = np.concatenate(cols) if cols else np.empty(0, dtype=np.int32)
    return Batch(ns, np.array(meff, dtype=np.int64), vtx_off.astype(np.int32),
                 edge_off.astype(np.int32), row_ptr, col.astype(np.int32, copy=False))


# ---- the five workloads (sizes as stated; seeds 1..5) ----

def c1_er() -> Graph:
    """Erdos-Renyi n=65,536, 262,144 draws (seed 1)."""
    return er(65536, 262144, seed=1, name="er_n65536_m262144")


def c2_rmat(scale: int = 24, edge_factor: int = 16) -> Graph:
    """R-MAT scale 24, edge factor 16, a=.57 b=c=.19 (seed 2), permuted ids."""
    return rmat(scale, edge_factor, seed=2)


def c3_grid(side: int = 4096, p: float = 0.55) -> Graph:
    """Percolated side x side lattice, bond probability p (seed 3), permuted ids."""
    return grid(side, side, p, seed=3)


def c4_batch(num_graphs: int = 4096, max_n: int | None = None) -> Batch:
    """Batch of Erdos-Renyi graphs (seed 4)."""
    return batch(num_graphs, seed=4, max_n=max_n)


def num_threads() -> int:
    return int(_load().gg_num_threads())


# ---- request streams (serving workload) ----

@dataclasses.dataclass
class RequestTrace:
    arrivals: np.ndarray   # seconds after the start, nondecreasing
    kinds: np.ndarray      # 0 = Erdos-Renyi from the batch distribution, 1 = R-MAT
    graphs: list           # Graph per request (shared objects from the pools)


def request_trace(num_requests: int, rate_per_s: float, seed: int = 5, er_pool: int = 256,
                  rmat_pool: int = 2, rmat_frac: float = 0.01, rmat_scale: int = 20,
                  rmat_edge_factor: int = 16) -> RequestTrace:
    """Poisson arrivals (exponential gaps, output 2i of stream 0) of requests
    that are R-MAT graphs with probability rmat_frac (output 2i+1 of stream 0)
    and otherwise Erdos-Renyi graphs from the batch size distribution.  The
    graphs come from fixed pools (er_pool ER graphs, rmat_pool R-MAT graphs);
    request i takes pool entry (output i of stream 1) mod the pool size."""
    ns, ms = batch_sizes(er_pool, seed)
    ers = []
    for g in range(er_pool):
        src, dst = er_edges(int(ns[g]), int(ms[g]), seed, 1000 + g)
        rp, col = csr_from_edges(int(ns[g]), src, dst)
        ers.append(Graph(f"req_er{g}", int(ns[g]), rp, col, int(src.shape[0])))
    rmats = [rmat(rmat_scale, rmat_edge_factor, seed=seed * 100 + k) for k in range(rmat_pool)] if rmat_pool else []
    arrivals = np.empty(num_requests)
    kinds = np.empty(num_requests, dtype=np.int32)
    graphs = []
    t = 0.0
    for i in range(num_requests):
        u = uniform(seed, 0, 2 * i)
        t += -np.log1p(-u) / rate_per_s
        arrivals[i] = t
        is_rmat = rmats and uniform(seed, 0, 2 * i + 1) < rmat_frac
        pick = rng_at(seed, 1, i)
        if is_rmat:
            kinds[i] = 1
            graphs.append(rmats[pick % len(rmats)])
        else:
            kinds[i] = 0
            graphs.append(ers[pick % len(ers)])
    return RequestTrace(arrivals, kinds, graphs)
