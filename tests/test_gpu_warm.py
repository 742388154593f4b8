"""Warm start (Alg. 3 takes the parent vector f as input) vs the oracle.

fastsv_cc_csr_warm starts from a given f0 with gf = mngf = f0 (Alg. 3
duplicates its input into gf); the iterates from there must equal
oracle_fastsv_alg3 run with the same input, and the labels the union-find
labels of the whole graph.  Typical use: edges were added to a graph whose
labels are known.
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
    labels, stats, st = fs.cc_csr(rp, col, check=False, **kw)
    torch.cuda.synchronize()
    ok = (fs.FASTSV_OK, fs.FASTSV_ENOTCONVERGED) if kw.get("max_iters") else (fs.FASTSV_OK,)
    assert st in ok, f"status {st}"
    return labels.cpu().numpy(), stats


def _pairs(g):
    """Undirected pairs (u < v) of a symmetric CSR, one per stored entry pair."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    m = rows < g.col
    return np.stack([rows[m], g.col[m]], 1)


def _check_warm(g2, f0, taus=(0.0, 0.05), trajectory=True, **kw):
    rp, col = _dev(g2.row_ptr), _dev(g2.col)
    want = O.uf_labels(g2.n, g2.row_ptr, g2.col)
    ref = O.fastsv_alg3(g2.n, g2.row_ptr, g2.col, f_init=f0, trace_cap=128)
    for tau in taus:
        got, st = _solve(rp, col, f_init=_dev(f0), frontier_tau=tau, validate=True, **kw)
        assert np.array_equal(got, want), (g2.name, tau)
        assert np.array_equal(got, ref.f)
        assert st.iterations == ref.iterations, (g2.name, tau, st.iterations, ref.iterations)
        k = min(ref.iterations, 64)
        assert st.changed_list()[:k] == ref.changed[:k].tolist(), (g2.name, tau)
        if trajectory:
            for it in range(1, min(ref.iterations, 16) + 1):
                got_k, _ = _solve(rp, col, f_init=_dev(f0), frontier_tau=tau, max_iters=it, **kw)
                assert np.array_equal(got_k, ref.trace[it - 1]), (g2.name, tau, it)
    return ref


@pytest.mark.parametrize("binned", [False, True])
def test_added_edges_restart_from_old_labels(gpu_ok, binned):
    rng = np.random.default_rng(31)
    for g2 in (gg.er(20000, 30000, seed=81), gg.rmat(14, 8, seed=82), gg.grid(60, 80, 0.5, seed=83)):
        pairs = _pairs(g2)
        keep = rng.random(len(pairs)) < 0.6
        rp1, col1 = P.csr_from_pairs(g2.n, pairs[keep])
        lab1, _ = _solve(_dev(rp1), _dev(col1))
        assert np.array_equal(lab1, O.uf_labels(g2.n, rp1, col1))
        kw = {"binned": True, "bin_shift": 8} if binned else {"binned": False}
        ref = _check_warm(g2, lab1, **kw)
        cold = O.fastsv_alg2(g2.n, g2.row_ptr, g2.col)
        _say(f"[gpu] {g2.name} binned={binned}: warm {ref.iterations} iterations, cold {cold.iterations}")


def test_restart_from_an_iterate_and_from_the_result(gpu_ok):
    g = gg.rmat(13, 16, seed=84)
    mid = O.fastsv_alg2(g.n, g.row_ptr, g.col, max_iters=2)
    _check_warm(g, mid.f)
    final = O.uf_labels(g.n, g.row_ptr, g.col)
    ref = _check_warm(g, final, trajectory=False)
    assert ref.iterations == 1


def test_in_place_restart_and_checks(gpu_ok):
    import paper_1910_05971_amd as fs
    g = gg.er(5000, 4000, seed=85)
    pairs = _pairs(g)
    rp1, col1 = P.csr_from_pairs(g.n, pairs[: len(pairs) // 2])
    lab = _dev(O.uf_labels(g.n, rp1, col1))
    rp, col = _dev(g.row_ptr), _dev(g.col)
    fs.cc_csr(rp, col, labels=lab, f_init=lab)  # labels overwritten in place
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy(), O.uf_labels(g.n, g.row_ptr, g.col))
    bad = _dev(np.arange(g.n)[::-1].copy())  # f0[u] > u for the lower half
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    _, _, st = fs.cc_csr(rp, col, labels=out, f_init=bad, validate=True, check=False)
    assert st == fs.FASTSV_ERANGE and int(out[0]) == -7
    _, _, st = fs.cc_csr(rp, col, f_init=lab, sv_flags=3, check=False)
    assert st == fs.FASTSV_EINVAL
