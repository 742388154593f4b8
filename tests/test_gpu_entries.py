"""Edge-list and batched entry points vs the oracle (needs an MI355X)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1910_05971_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_edge_list_entry(gpu_ok):
    import paper_1910_05971_amd as fs
    rng = np.random.default_rng(11)
    cases = [(1, np.zeros((0, 2), np.int64)), (7, np.array([[5, 2], [5, 6], [6, 0]])),
             (10, np.array([[3, 3], [1, 2], [2, 1], [1, 2], [9, 0]]))]
    for n, m in ((5000, 4000), (50000, 200000), (300000, 400000)):
        cases.append((n, rng.integers(0, n, size=(m, 2))))
    src_er, dst_er = gg.er_edges(65536, 262144, seed=1)
    cases.append((65536, np.stack([src_er, dst_er], 1)))
    for n, e in cases:
        _say(f"[gpu] edges n={n} m={len(e)}")
        src = np.ascontiguousarray(e[:, 0], dtype=np.int32)
        dst = np.ascontiguousarray(e[:, 1], dtype=np.int32)
        want = O.uf_labels_edges(n, src, dst)
        rp, col = gg.csr_from_edges(n, src, dst)
        ref = O.fastsv_alg2(n, rp, col, trace_cap=256, record_f=False)
        for tau in (0.0, 0.05):
            labels, st = fs.cc_edges(n, torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda(),
                                     frontier_tau=tau, validate=True)
            torch.cuda.synchronize()
            assert np.array_equal(labels.cpu().numpy(), want), (n, tau)
            assert st.iterations == ref.iterations
            assert st.changed_list() == ref.changed.tolist()[:64]


def test_edge_list_rejects_bad_ids(gpu_ok):
    import paper_1910_05971_amd as fs
    src = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    dst = torch.tensor([1, 9], dtype=torch.int32, device="cuda")
    labels = torch.full((4,), -3, dtype=torch.int32, device="cuda")
    _, _, st = fs.cc_edges(4, src, dst, labels=labels, validate=True, check=False)
    assert st == fs.FASTSV_ERANGE and labels.cpu().tolist() == [-3] * 4


def _batch_to_dev(b):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (b.vtx_off, b.edge_off, b.row_ptr, b.col)]


def _check_batch(b, sample=None, **kw):
    import paper_1910_05971_amd as fs
    vo, eo, rp, col = _batch_to_dev(b)
    labels, iters, st = fs.cc_batch_csr(vo, eo, rp, col, validate=True, **kw)
    torch.cuda.synchronize()
    lab = labels.cpu().numpy()
    its = iters.cpu().numpy()
    idx = range(b.num_graphs) if sample is None else sample
    for g in idx:
        sub = b.graph(g)
        v0, v1 = int(b.vtx_off[g]), int(b.vtx_off[g + 1])
        want = O.uf_labels(sub.n, sub.row_ptr, sub.col)
        assert np.array_equal(lab[v0:v1], want), f"graph {g}"
        ref = O.fastsv_alg2(sub.n, sub.row_ptr, sub.col)
        assert its[g] == ref.iterations, (g, its[g], ref.iterations)
    return lab, its, st


def test_batch_small(gpu_ok):
    b = gg.c4_batch(64, max_n=3000)
    _say(f"[gpu] batch G=64 n={b.row_ptr.shape[0] - 1} nnz={b.col.shape[0]}")
    for tau in (0.0, 0.05, 1.0):
        _check_batch(b, frontier_tau=tau)


def _batch_of(graphs):
    """A Batch holding the given graphs (local column ids, global row_ptr)."""
    ns = [g.n for g in graphs]
    nnzs = [g.col.shape[0] for g in graphs]
    vtx_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    edge_off = np.concatenate([[0], np.cumsum(nnzs)]).astype(np.int32)
    row_ptr = np.concatenate([g.row_ptr[:-1].astype(np.int64) + edge_off[i] for i, g in enumerate(graphs)] +
                             [[edge_off[-1]]]).astype(np.int32)
    col = np.concatenate([g.col for g in graphs]).astype(np.int32)
    m_eff = np.array([g.m_eff for g in graphs], dtype=np.int64)
    return gg.Batch(np.array(ns, dtype=np.int32), m_eff, vtx_off, edge_off, row_ptr, col)


def test_batch_mixed_sizes(gpu_ok):
    # graphs from 64 to 100000 vertices in one batch (tiles that cross graphs,
    # graphs over many tiles), stars whose hub rows span 16 and 98 tiles and a
    # path (many iterations), each against its solo oracle run; also capped
    # runs against the solo iterates
    import paper_1910_05971_amd as fs
    import oracle_pins as P
    graphs = []
    for i, n in enumerate((64, 4096, 4097, 16384, 16385, 65536, 65537, 100_000)):
        graphs.append(gg.er(n, 3 * n, seed=90 + i))
    for n in (16_384, 100_000):
        graphs.append(gg.Graph(f"star{n}", n, *P.csr_from_pairs(n, [(7, v) for v in range(n) if v != 7]), n - 1))
    n = 3000
    graphs.append(gg.Graph("path", n, *P.csr_from_pairs(n, [(v, v + 1) for v in range(n - 1)]), n - 1))
    b = _batch_of(graphs)
    _say(f"[gpu] batch mixed G={b.num_graphs} n={b.row_ptr.shape[0] - 1} nnz={b.col.shape[0]}")
    for tau in (0.0, 0.05):
        _check_batch(b, frontier_tau=tau)
    vo, eo, rp, col = _batch_to_dev(b)
    refs = [O.fastsv_alg2(g.n, g.row_ptr, g.col, trace_cap=64) for g in graphs]
    for k in (2, 3, 5):
        labels, iters, st, status = fs.cc_batch_csr(vo, eo, rp, col, max_iters=k, frontier_tau=0.0, check=False)
        lab = labels.cpu().numpy()
        for g, r in enumerate(refs):
            v0, v1 = int(b.vtx_off[g]), int(b.vtx_off[g + 1])
            assert np.array_equal(lab[v0:v1], r.trace[min(k, r.iterations) - 1]), (g, k)


def test_batch_matches_solo_trajectory(gpu_ok):
    # capped runs: graph g's labels after k iterations are its solo f_k
    import paper_1910_05971_amd as fs
    b = gg.c4_batch(12, max_n=2000)
    vo, eo, rp, col = _batch_to_dev(b)
    refs = [O.fastsv_alg2(b.graph(g).n, b.graph(g).row_ptr, b.graph(g).col, trace_cap=64) for g in range(12)]
    kmax = max(r.iterations for r in refs)
    for k in range(1, kmax + 1):
        labels, iters, st, status = fs.cc_batch_csr(vo, eo, rp, col, max_iters=k, check=False)
        assert status in (fs.FASTSV_OK, fs.FASTSV_ENOTCONVERGED)
        lab = labels.cpu().numpy()
        its = iters.cpu().numpy()
        for g, r in enumerate(refs):
            v0, v1 = int(b.vtx_off[g]), int(b.vtx_off[g + 1])
            fk = r.trace[min(k, r.iterations) - 1]
            assert np.array_equal(lab[v0:v1], fk), (g, k)
            assert its[g] == (r.iterations if r.iterations <= k else -1), (g, k, its[g])


def test_batch_edge_cases(gpu_ok):
    import paper_1910_05971_amd as fs
    # graphs with no vertices and graphs with no edges inside a batch
    ns = [0, 1, 3, 0, 5]
    rps, cols = [], []
    pairs = {2: [(0, 1)], 4: [(0, 4), (1, 2)]}
    for g, n in enumerate(ns):
        import oracle_pins as P
        rp, col = P.csr_from_pairs(n, pairs.get(g, []))
        rps.append(rp)
        cols.append(col)
    vtx_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    edge_off = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int32)
    row_ptr = np.concatenate([rps[g][:-1] + edge_off[g] for g in range(len(ns))] + [[edge_off[-1]]]).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32)
    labels, iters, st = fs.cc_batch_csr(*[torch.from_numpy(x).cuda() for x in (vtx_off, edge_off, row_ptr, col)],
                                        validate=True)
    assert labels.cpu().tolist() == [0, 0, 0, 2, 0, 1, 1, 3, 0]
    assert iters.cpu().tolist() == [0, 1, 2, 0, 2]


def test_batch_rejects_bad_offsets(gpu_ok):
    import paper_1910_05971_amd as fs
    b = gg.c4_batch(4, max_n=100)
    vo, eo, rp, col = _batch_to_dev(b)
    eo_bad = eo.clone()
    eo_bad[2] += 1
    labels = torch.full((rp.numel() - 1,), -7, dtype=torch.int32, device="cuda")
    _, _, _, st = fs.cc_batch_csr(vo, eo_bad, rp, col, labels=labels, validate=True, check=False)
    assert st == fs.FASTSV_ERANGE and bool((labels == -7).all())
    col_bad = col.clone()
    col_bad[5] = int(b.n[0]) + 1000
    _, _, _, st = fs.cc_batch_csr(vo, eo, rp, col_bad, validate=True, check=False)
    assert st == fs.FASTSV_ERANGE


@pytest.mark.slow
def test_config_c4_batch(gpu_ok):
    b = gg.c4_batch()
    _say(f"[gpu] C4 G=4096 n={b.row_ptr.shape[0] - 1} nnz={b.col.shape[0]}")
    rng = np.random.default_rng(0)
    sample = sorted(rng.choice(4096, 128, replace=False).tolist())
    lab, its, st = _check_batch(b, sample=sample)
    # every graph's labels against union-find
    for g in range(b.num_graphs):
        sub = b.graph(g)
        v0, v1 = int(b.vtx_off[g]), int(b.vtx_off[g + 1])
        assert np.array_equal(lab[v0:v1], O.uf_labels(sub.n, sub.row_ptr, sub.col)), g
    _say(f"[gpu] C4 iterations={st.iterations} max per-graph={its.max()}")


def test_trace_counts_atomics_without_changing_iterates(gpu_ok):
    """opts.trace: the hooks' atomics are counted per iteration (their sum is
    the total, and alg_bytes grows by 8 B per atomic); labels, iteration count
    and changed counts are those of the untraced call.  A graph without edges
    issues no atomic."""
    import paper_1910_05971_amd as fs
    cases = [(gg.rmat(15, 16, seed=61), {}), (gg.er(40000, 90000, seed=62), {"frontier_tau": 1.0}),
             (gg.grid(200, 300, 0.55, seed=63), {"frontier_tau": 0.0}), (gg.rmat(16, 8, seed=64), {"binned": True})]
    for g, kw in cases:
        _say(f"[gpu] trace {g.name} {kw}")
        rp, col = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
        plain, sp = fs.cc_csr(rp, col, **kw)
        traced, st = fs.cc_csr(rp, col, trace=True, **kw)
        torch.cuda.synchronize()
        assert torch.equal(plain, traced)
        assert st.iterations == sp.iterations and st.changed_list() == sp.changed_list()
        assert sp.atomics_issued == -1 and all(a == -1 for a in sp.atomics_list())
        per = st.atomics_list()
        assert all(a >= 0 for a in per) and sum(per) == st.atomics_issued > 0
        assert st.alg_bytes == sp.alg_bytes + 8 * st.atomics_issued
        assert sum(st.pushed_list()) == st.frontier_edges == sp.frontier_edges
        assert all(p == 0 for p, s in zip(st.pushed_list(), st.sparse_list()) if not s)
    # vertices without edges: one iteration, nothing hooked
    rp0 = torch.zeros(1001, dtype=torch.int32, device="cuda")
    col0 = torch.zeros(0, dtype=torch.int32, device="cuda")
    _, s0 = fs.cc_csr(rp0, col0, trace=True)
    assert s0.iterations == 1 and s0.atomics_issued == 0
    # the batch entry counts too
    b = gg.batch(64, seed=65, max_n=4096)
    vo, eo, rpb, colb = _batch_to_dev(b)
    lab1, it1, sb1 = fs.cc_batch_csr(vo, eo, rpb, colb)
    lab2, it2, sb2 = fs.cc_batch_csr(vo, eo, rpb, colb, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(lab1, lab2) and torch.equal(it1, it2)
    assert sb2.atomics_issued == sum(sb2.atomics_list()) > 0 and sb1.atomics_issued == -1


def test_timing_stats(gpu_ok):
    # opts.timing: every iteration's hooking and grandparent phases are timed
    # (read after the loop), the fused layout build is split off, and the
    # result and per-iteration counts are those of the untimed call
    import paper_1910_05971_amd as fs
    g = gg.er(300_000, 1_200_000, seed=77)
    rp, col = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
    for kw in ({"binned": True, "bin_shift": 12}, {"binned": False}, {"binned": True, "bin_shift": 12,
                                                                       "frontier_tau": 0.5}):
        plain, sp = fs.cc_csr(rp, col, **kw)
        timed, st = fs.cc_csr(rp, col, timing=True, **kw)
        assert torch.equal(plain, timed) and st.iterations == sp.iterations
        assert st.changed_list() == sp.changed_list() and st.sparse_list() == sp.sparse_list()
        k = min(st.iterations, 64)
        assert all(st.ms_hook[i] > 0 for i in range(k)) and all(st.ms_gp[i] > 0 for i in range(k)), kw
        assert all(sp.ms_hook[i] == 0 for i in range(k))
        if kw["binned"]:
            assert st.bin_fused_first == 1 and st.ms_bin_prepare > 0
