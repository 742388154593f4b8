"""Seeded input generators (no GPU): determinism, structure, expected sizes."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1910_05971_amd import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MASK = (1 << 64) - 1


def splitmix64_next(state):
    """SplitMix64 step as published (Steele, Lea, Flood 2014): state += gamma,
    then the variant-13 finaliser."""
    state = (state + 0x9E3779B97F4A7C15) & MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return state, z ^ (z >> 31)


def test_rng_is_a_splitmix64_stream():
    # output ctr of stream (seed, s) is the (ctr+1)-th SplitMix64 output from
    # the stream's start state, i.e. the generator is counter-based
    for seed, stream in ((0, 0), (2, 1), (12345, 77)):
        outs = [gg.rng_at(seed, stream, c) for c in range(6)]
        # recover the start state from the definition of the stream key
        _, k0 = splitmix64_next(seed)           # mix(seed + gamma)
        start = (k0 + (stream + 1) * 0x9E3779B97F4A7C15) & MASK
        _, key = splitmix64_next((start - 0x9E3779B97F4A7C15) & MASK)
        st = key
        want = []
        for _ in range(6):
            st, z = splitmix64_next(st)
            want.append(z)
        assert outs == want


def _check_csr(g: gg.Graph):
    rp, col = g.row_ptr.astype(np.int64), g.col
    assert rp[0] == 0 and rp[-1] == col.shape[0]
    assert np.all(np.diff(rp) >= 0)
    assert col.shape[0] == 2 * g.m_eff
    if col.shape[0]:
        assert col.min() >= 0 and col.max() < g.n
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert not np.any(rows == col), "self loop stored"
    # symmetric: the multiset of (u,v) equals the multiset of (v,u)
    a = np.sort(rows * g.n + col)
    b = np.sort(col.astype(np.int64) * g.n + rows)
    assert np.array_equal(a, b)
    # rows sorted
    for u in range(0, g.n, max(1, g.n // 200)):
        seg = col[rp[u]:rp[u + 1]]
        assert np.all(np.diff(seg) >= 0)


def test_er_structure_and_counts():
    g = gg.er(5000, 40000, seed=3)
    _check_csr(g)
    # expected loops dropped: m/n = 8, sd ~ sqrt(8)
    assert abs((40000 - g.m_eff) - 8) < 5 * np.sqrt(8) + 1


def test_c1_sizes():
    g = gg.c1_er()
    _check_csr(g)
    assert g.n == 65536 and 262144 - g.m_eff < 20


def test_rmat_structure():
    g = gg.rmat(12, 8, seed=5)
    _check_csr(g)
    deg = np.diff(g.row_ptr)
    assert deg.max() > 20 * deg.mean()  # skewed
    # unpermuted R-MAT: vertex 0 collects the (0,0) quadrant every level, so
    # it has the largest expected degree
    src, dst = gg.rmat_edges(10, 4, seed=5, permute=False)
    cnt = np.bincount(np.concatenate([src, dst]), minlength=1024)
    assert cnt.argmax() == 0


def test_grid_structure_and_extremes():
    g = gg.grid(30, 40, 0.5, seed=1)
    _check_csr(g)
    nb = 30 * 39 + 29 * 40
    assert abs(g.m_eff - 0.5 * nb) < 5 * np.sqrt(nb * 0.25)
    assert gg.grid(10, 10, 0.0, seed=1).m_eff == 0
    assert gg.grid(10, 10, 1.0, seed=1).m_eff == 10 * 9 * 2
    # unpermuted bonds join lattice neighbours only
    src, dst = gg.grid_edges(8, 9, 1.0, seed=1, permute=False)
    d = np.abs(src - dst)
    assert set(np.unique(d)) <= {1, 9}


def test_permutation_is_a_permutation():
    p = gg.permutation(10007, seed=9)
    assert np.array_equal(np.sort(p), np.arange(10007))
    assert not np.array_equal(p, np.arange(10007))


def test_batch_sizes_distribution():
    n, m = gg.batch_sizes(4096, seed=4)
    assert n.min() >= 64 and n.max() < 65536
    d = 2 * m / n
    assert d.min() >= 2 - 1e-6 and d.max() <= 32 + 1e-6
    # log-uniform: log2 n uniform over [6, 16)
    lg = np.log2(n)
    assert abs(lg.mean() - 11.0) < 0.15
    assert abs(d.mean() - 17.0) < 0.5


def test_batch_layout():
    b = gg.c4_batch(16, max_n=500)
    assert b.vtx_off[-1] == b.row_ptr.shape[0] - 1
    assert b.edge_off[-1] == b.col.shape[0]
    for g in range(b.num_graphs):
        sub = b.graph(g)
        _check_csr(sub)


def test_deterministic_across_thread_counts():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1910_05971_amd import graphgen as gg\n"
            "import hashlib\n"
            "g = gg.rmat(13, 8, seed=2); h = hashlib.sha256(g.row_ptr.tobytes() + g.col.tobytes())\n"
            "g = gg.grid(50, 60, 0.55, seed=3); h.update(g.row_ptr.tobytes() + g.col.tobytes())\n"
            "print(h.hexdigest())\n") % ROOT
    outs = []
    for t in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout.strip())
    assert len(set(outs)) == 1, outs


def test_request_trace_shape():
    tr = gg.request_trace(300, 2000.0, er_pool=16, rmat_pool=1, rmat_scale=10, rmat_edge_factor=4)
    assert np.all(np.diff(tr.arrivals) >= 0)
    assert abs(tr.arrivals[-1] - 300 / 2000.0) < 0.05
    assert tr.kinds.sum() < 15
