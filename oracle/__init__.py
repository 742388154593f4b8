"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference for the FastSV connected-components
method (Zhang, Azad, Hu, arXiv 1910.05971).  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import this package.  The HIP
solver never calls it, links it or shares code with it.

* ``uf_labels``     union-find; the plain definition of the result
                    (labels[u] = smallest vertex of u's component; Sec. 3.4,
                    Appendix A)
* ``bfs_labels``    brute-force BFS labelling
* ``fastsv_alg2``   Algorithm 2 (Sec. 3), Jacobi f / f_next, per-iteration trace
* ``fastsv_alg3``   Algorithm 3 (Sec. 4.1), GraphBLAS calls written out
* ``sv_variant``    Algorithm 1 (Sec. 2.4) plus any subset of the four Sec. 3
                    optimisations (sv1..sv5 of Sec. 5.2)
* ``fastsv_async``  Algorithm 2 in place on one vector (Sec. 2.4's concurrent form)
* invariant checkers from Appendix A (``check_invariants``, ``check_final``)

Everything iterative works on a symmetric int32 CSR.  The C library is built by
``__graft_entry__.build()`` into ``oracle/liboracle.so``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCE = os.path.join(_HERE, "oracle.c")

# flag bits of sv_variant (Sec. 3.1 - 3.4)
GRANDPARENT, STOCHASTIC, AGGRESSIVE, EARLY_TERM = 1, 2, 4, 8
SV_FLAGS = {"sv1": 0, "sv2": 1, "sv3": 3, "sv4": 7, "sv5": 15}

def _bind(lib):
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_uf_labels.restype = i32
    lib.oracle_uf_labels.argtypes = [i32, vp, vp, vp]
    lib.oracle_uf_labels_edges.restype = i32
    lib.oracle_uf_labels_edges.argtypes = [i32, i64, vp, vp, vp]
    lib.oracle_bfs_labels.restype = i32
    lib.oracle_bfs_labels.argtypes = [i32, vp, vp, vp]
    lib.oracle_fastsv_alg2.restype = i32
    lib.oracle_fastsv_alg2.argtypes = [i32, vp, vp, i32, vp, vp, vp, i32]
    lib.oracle_fastsv_alg3.restype = i32
    lib.oracle_fastsv_alg3.argtypes = [i32, vp, vp, i32, vp, vp, vp, vp, i32]
    lib.oracle_sv_variant.restype = i32
    lib.oracle_sv_variant.argtypes = [i32, vp, vp, i32, i32, vp, vp, vp, i32]
    lib.oracle_fastsv_async.restype = i32
    lib.oracle_fastsv_async.argtypes = [i32, vp, vp, i32, vp]
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _csr(row_ptr, col):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    return row_ptr, col


class Result:
    """f: final (or last) parent vector; iterations: count, -1 if capped;
    trace: int32[k, n] of f after each recorded iteration; changed: int64[k]
    termination counts (entries of f[f] that changed) of those iterations."""

    def __init__(self, f, iterations, trace, changed):
        self.f, self.iterations, self.trace, self.changed = f, iterations, trace, changed


class Oracle:
    """ctypes front end of one build of oracle.c (the default build, or a
    test-only copy compiled elsewhere)."""

    def __init__(self, lib_path: str = LIB_PATH):
        if not os.path.exists(lib_path):
            raise RuntimeError(f"oracle library missing: {lib_path} (run __graft_entry__.build())")
        self.lib = _bind(ctypes.CDLL(lib_path))

    def uf_labels(self, n, row_ptr, col) -> np.ndarray:
        row_ptr, col = _csr(row_ptr, col)
        out = np.empty(n, dtype=np.int32)
        self.lib.oracle_uf_labels(n, _p(row_ptr), _p(col), _p(out))
        return out

    def uf_labels_edges(self, n, src, dst) -> np.ndarray:
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        out = np.empty(n, dtype=np.int32)
        self.lib.oracle_uf_labels_edges(n, int(src.shape[0]), _p(src), _p(dst), _p(out))
        return out

    def bfs_labels(self, n, row_ptr, col) -> np.ndarray:
        row_ptr, col = _csr(row_ptr, col)
        out = np.empty(n, dtype=np.int32)
        if self.lib.oracle_bfs_labels(n, _p(row_ptr), _p(col), _p(out)) != 0:
            raise MemoryError("oracle allocation failed")
        return out

    def _run(self, fn, n, row_ptr, col, max_iters, trace_cap, before=(), after=(), record_f=True):
        row_ptr, col = _csr(row_ptr, col)
        f = np.empty(n, dtype=np.int32)
        cap = int(trace_cap)
        tr = np.empty((cap, n), dtype=np.int32) if cap > 0 and record_f else None
        ch = np.empty(max(cap, 1), dtype=np.int64)
        it = fn(n, _p(row_ptr), _p(col), *before, int(max_iters), *after, _p(f), _p(tr), _p(ch), cap)
        if it == -2:
            raise MemoryError("oracle allocation failed")
        k = min(cap, max_iters if it == -1 else it) if cap > 0 else 0
        return Result(f, int(it), tr[:k] if tr is not None else None, ch[:k] if cap > 0 else None)

    def fastsv_alg2(self, n, row_ptr, col, max_iters=0, trace_cap=0, record_f=True) -> Result:
        """record_f=False keeps only the per-iteration changed counts."""
        return self._run(self.lib.oracle_fastsv_alg2, n, row_ptr, col, max_iters, trace_cap, record_f=record_f)

    def fastsv_alg3(self, n, row_ptr, col, max_iters=0, trace_cap=0, f_init=None) -> Result:
        fi = None if f_init is None else np.ascontiguousarray(f_init, dtype=np.int32)
        return self._run(self.lib.oracle_fastsv_alg3, n, row_ptr, col, max_iters, trace_cap,
                         after=(_p(fi),))

    def sv_variant(self, n, row_ptr, col, flags, max_iters=0, trace_cap=0) -> Result:
        return self._run(self.lib.oracle_sv_variant, n, row_ptr, col, max_iters, trace_cap,
                         before=(int(flags),))

    def fastsv_async(self, n, row_ptr, col, max_iters=0):
        row_ptr, col = _csr(row_ptr, col)
        f = np.empty(n, dtype=np.int32)
        it = self.lib.oracle_fastsv_async(n, _p(row_ptr), _p(col), int(max_iters), _p(f))
        if it == -2:
            raise MemoryError("oracle allocation failed")
        return f, int(it)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def uf_labels(n, row_ptr, col):
    return default().uf_labels(n, row_ptr, col)


def uf_labels_edges(n, src, dst):
    return default().uf_labels_edges(n, src, dst)


def bfs_labels(n, row_ptr, col):
    return default().bfs_labels(n, row_ptr, col)


def fastsv_alg2(n, row_ptr, col, max_iters=0, trace_cap=0, record_f=True):
    return default().fastsv_alg2(n, row_ptr, col, max_iters, trace_cap, record_f)


def fastsv_alg3(n, row_ptr, col, max_iters=0, trace_cap=0, f_init=None):
    return default().fastsv_alg3(n, row_ptr, col, max_iters, trace_cap, f_init)


def sv_variant(n, row_ptr, col, flags, max_iters=0, trace_cap=0):
    return default().sv_variant(n, row_ptr, col, flags, max_iters, trace_cap)


def fastsv_async(n, row_ptr, col, max_iters=0):
    return default().fastsv_async(n, row_ptr, col, max_iters)


# ---------------------------------------------------------------------------
# Invariant checkers (Appendix A).  They take plain arrays and raise
# AssertionError naming the violated property.
# ---------------------------------------------------------------------------

def check_invariants(trace: np.ndarray, labels: np.ndarray):
    """Per-iteration properties of a Jacobi FastSV trajectory f_1, f_2, ...

    * f_k[u] <= u                          (Lemma "f[u] <= u", Appendix A)
    * f_k <= f_{k-1} pointwise, f_0 = iota (every update is a min-assign)
    * f_k[f_k] <= f_{k-1}[f_{k-1}]         (grandparents never increase)
    * labels[f_k[u]] == labels[u]          (a parent stays in u's component)
    """
    n = labels.shape[0]
    iota = np.arange(n, dtype=np.int32)
    prev_f, prev_g = iota, iota
    for k, f in enumerate(trace, start=1):
        assert np.all(f <= iota), f"iteration {k}: f[u] > u"
        assert np.all(f >= 0), f"iteration {k}: negative parent"
        assert np.all(f <= prev_f), f"iteration {k}: f increased"
        g = f[f]
        assert np.all(g <= prev_g), f"iteration {k}: grandparent increased"
        assert np.all(labels[f] == labels), f"iteration {k}: parent left the component"
        prev_f, prev_g = f, g


def check_final(f: np.ndarray, row_ptr: np.ndarray, col: np.ndarray):
    """At termination every tree is a star and adjacent vertices share a root
    (Lemma "every vertex points to a root"; the converged state of Sec. 3.4)."""
    assert np.array_equal(f[f], f), "not a star forest"
    rows = np.repeat(np.arange(f.shape[0], dtype=np.int64), np.diff(row_ptr.astype(np.int64)))
    assert np.array_equal(f[rows], f[col]), "an edge joins two different stars"
