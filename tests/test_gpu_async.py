"""Asynchronous mode (one parent vector read and written concurrently, Sec. 2.4).

Its iterates are not reproducible, so only what is unique is compared: the
final labels, bit for bit against union-find.  Capped runs are checked for the
invariants every valid parent vector keeps (f[u] <= u, f[u] in u's component).
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import oracle_pins as P
from paper_1910_05971_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _solve(rp, col, **kw):
    import paper_1910_05971_amd as fs
    labels, stats, st = fs.cc_csr(rp, col, check=False, mode="async", **kw)
    torch.cuda.synchronize()
    ok = (fs.FASTSV_OK, fs.FASTSV_ENOTCONVERGED) if kw.get("max_iters") else (fs.FASTSV_OK,)
    assert st in ok, f"status {st}"
    return labels.cpu().numpy(), stats


def _graphs():
    n = 2000
    path = P.csr_from_pairs(n, [(i, i + 1) for i in range(n - 1)])
    star = P.csr_from_pairs(5000, [(4999, i) for i in range(4999)])
    empty = (np.zeros(101, dtype=np.int32), np.zeros(0, dtype=np.int32))
    return [gg.Graph("path2000", n, *path, n - 1), gg.Graph("star_last5000", 5000, *star, 4999),
            gg.Graph("edgeless100", 100, *empty, 0), gg.c1_er(), gg.rmat(16, 16, seed=91),
            gg.grid(200, 300, 0.55, seed=92), gg.er(100000, 60000, seed=93)]


def test_async_labels_exact(gpu_ok):
    for g in _graphs():
        rp, col = _dev(g.row_ptr), _dev(g.col)
        want = O.uf_labels(g.n, g.row_ptr, g.col)
        for rep in range(2):
            got, st = _solve(rp, col, validate=True)
            assert np.array_equal(got, want), (g.name, rep)
        jac = O.fastsv_alg2(g.n, g.row_ptr, g.col)
        _say(f"[gpu] async {g.name}: {st.iterations} passes (Jacobi {jac.iterations} iterations), "
             f"changes {st.changed_list()[:12]}")


def test_async_capped_keeps_invariants(gpu_ok):
    g = gg.grid(120, 150, 0.6, seed=94)
    rp, col = _dev(g.row_ptr), _dev(g.col)
    want = O.uf_labels(g.n, g.row_ptr, g.col)
    for k in (1, 2, 3):
        f, _ = _solve(rp, col, max_iters=k)
        u = np.arange(g.n)
        assert np.all(f <= u) and np.all(f >= 0)
        assert np.array_equal(want[f], want), k  # every parent lies in the vertex's component


def test_async_warm_and_edges(gpu_ok):
    import paper_1910_05971_amd as fs
    g = gg.rmat(14, 8, seed=95)
    rp, col = _dev(g.row_ptr), _dev(g.col)
    want = O.uf_labels(g.n, g.row_ptr, g.col)
    mid = O.fastsv_alg2(g.n, g.row_ptr, g.col, max_iters=1).f
    got, _ = _solve(rp, col, f_init=_dev(mid))
    assert np.array_equal(got, want)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    m = rows < g.col
    lab, st = fs.cc_edges(g.n, _dev(rows[m]), _dev(g.col[m]), mode="async")
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy(), want)
