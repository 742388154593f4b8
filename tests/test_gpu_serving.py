"""Continuous-batching server vs the oracle (needs an MI355X).

Every request must get the labels AND the iteration count of its solo run,
whatever else is resident at the same time."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle_pins as P
from paper_1910_05971_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def _mix():
    # rmat(18, 16) has more than 2^22 entries: its column ids go by DMA
    gs = [gg.er(3000, 5000, seed=61), gg.er(20000, 100000, seed=62), gg.rmat(13, 8, seed=63),
          gg.grid(60, 70, 0.55, seed=64), gg.er(64, 100, seed=65), gg.rmat(18, 16, seed=66)]
    rp, col = P.csr_from_pairs(1, [])
    gs.append(gg.Graph("single", 1, rp, col, 0))
    rp, col = P.csr_from_pairs(50, [])
    gs.append(gg.Graph("edgeless", 50, rp, col, 0))
    rp, col = P.csr_from_pairs(7, [(5, 2), (5, 6), (6, 0)])
    gs.append(gg.Graph("golden7", 7, rp, col, 3))
    b = gg.c4_batch(24, max_n=5000)
    gs += [b.graph(i) for i in range(24)]
    return gs


def _expected(g):
    lab = O.uf_labels(g.n, g.row_ptr, g.col)
    its = O.fastsv_alg2(g.n, g.row_ptr, g.col).iterations
    return lab, its


@pytest.mark.parametrize("tau", [0.0, 0.05, 1.0])
def test_server_matches_solo(gpu_ok, tau):
    from paper_1910_05971_amd.serving import Server
    gs = _mix()
    want = [_expected(g) for g in gs]
    srv = Server(max_vertices=600_000, max_entries=12_000_000, max_slots=16, frontier_tau=tau)
    ticket_of = {}
    got = {}
    rng = np.random.default_rng(1)
    pending = list(range(len(gs)))
    # staggered arrivals: a few new requests before each step
    while pending or ticket_of:
        for _ in range(int(rng.integers(0, 4))):
            if pending:
                i = pending.pop(0)
                ticket_of[srv.submit(gs[i].row_ptr, gs[i].col)] = i
        srv.step()
        for t, lab, its in srv.poll():
            got[ticket_of.pop(t)] = (lab.copy(), its)
    srv.close()
    for i, g in enumerate(gs):
        lab, its = got[i]
        assert np.array_equal(lab, want[i][0]), g.name
        assert its == want[i][1], (g.name, its, want[i][1])


def test_server_small_pool_queues(gpu_ok):
    from paper_1910_05971_amd.serving import Server
    gs = [gg.er(5000, 15000, seed=70 + k) for k in range(10)]
    nnz_max = max(g.nnz for g in gs)
    srv = Server(max_vertices=2 * 5001 + 10, max_entries=2 * nnz_max + 10, max_slots=4)
    tickets = {srv.submit(g.row_ptr, g.col): i for i, g in enumerate(gs)}
    got = {}
    for _ in range(1000):
        r, q = srv.step()
        for t, lab, its in srv.poll():
            got[tickets[t]] = (lab.copy(), its)
        if r == 0 and q == 0:
            break
    st = srv.stats()
    srv.close()
    assert len(got) == 10 and st.admitted == 10 and st.completed == 10
    for i, g in enumerate(gs):
        lab, its = _expected(g)
        assert np.array_equal(got[i][0], lab) and got[i][1] == its


def test_server_rejects(gpu_ok):
    import paper_1910_05971_amd as fs
    from paper_1910_05971_amd.serving import Server
    srv = Server(max_vertices=100, max_entries=100, max_slots=2)
    big = gg.er(500, 600, seed=3)
    with pytest.raises(fs.FastSVError) as e:
        srv.submit(big.row_ptr, big.col)
    assert e.value.status == fs.FASTSV_ENOMEM
    rp = np.array([0, 1, 2], dtype=np.int32)
    with pytest.raises(fs.FastSVError) as e:
        srv.submit(rp, np.array([1, 5], dtype=np.int32))
    assert e.value.status == fs.FASTSV_ERANGE
    srv.close()




@pytest.mark.parametrize("mapped", [False, True])
def test_server_page_locked_requests(gpu_ok, mapped):
    # page-locked request arrays: small ones read by the placement kernel in
    # place, large ones copied by DMA; admissions after the first step are
    # placed on the copy stream while the resident graphs iterate
    from paper_1910_05971_amd.serving import Server, pin_graphs
    gs = pin_graphs(_mix())
    srv = Server(max_vertices=600_000, max_entries=12_000_000, max_slots=8, validate=False)
    tickets = {srv.submit(g.row_ptr, g.col, mapped=mapped): i for i, g in enumerate(gs)}
    got = {}
    for _ in range(10000):
        r, q = srv.step()
        for t, lab, its in srv.poll():
            got[tickets[t]] = (lab.copy(), its)
        if len(got) == len(gs):
            break
    srv.close()
    for i, g in enumerate(gs):
        lab, its = _expected(g)
        assert np.array_equal(got[i][0], lab), g.name
        assert got[i][1] == its, g.name


@pytest.mark.parametrize("mapped", [False, True])
def test_server_batch_submit(gpu_ok, mapped):
    # all requests in one call; a pool that holds only part of them at a time
    from paper_1910_05971_amd.serving import Server, pin_graphs
    gs = _mix()
    if mapped:
        gs = pin_graphs(gs)
    want = [_expected(g) for g in gs]
    srv = Server(max_vertices=300_000, max_entries=9_000_000, max_slots=6, validate=not mapped)
    tickets = srv.submit_many(gs, mapped=mapped)
    assert len(set(tickets)) == len(gs)
    of = {t: i for i, t in enumerate(tickets)}
    got = {}
    for _ in range(10000):
        srv.step()
        for t, lab, its in srv.poll():
            got[of[t]] = (lab.copy(), its)
        if len(got) == len(gs):
            break
    srv.close()
    for i, g in enumerate(gs):
        assert np.array_equal(got[i][0], want[i][0]), g.name
        assert got[i][1] == want[i][1], (g.name, got[i][1], want[i][1])


@pytest.mark.slow
def test_server_request_trace_with_rmat20(gpu_ok):
    """The serving workload's own mix, shortened: Poisson arrivals of Erdos-
    Renyi graphs from the batch distribution and R-MAT scale-20 edge-factor-16
    graphs (5% here instead of 1%, so that several overlap), page-locked, with
    the benchmark's pool sizes, replayed open loop; every request against its
    oracle labels and Algorithm 2 iteration count."""
    import sys
    from paper_1910_05971_amd import serving
    tr = gg.request_trace(400, 2000.0, seed=55, er_pool=48, rmat_pool=2, rmat_frac=0.05)
    assert tr.kinds.sum() >= 5
    graphs = serving.pin_graphs(tr.graphs)
    want = {}
    for g in graphs:
        if id(g) not in want:
            want[id(g)] = _expected(g)
    print(f"[gpu] serving trace: {len(graphs)} requests, {int(tr.kinds.sum())} R-MAT scale 20", flush=True)
    sys.stdout.flush()
    got = [None] * len(graphs)

    def keep(i, lab, its):
        got[i] = (lab.copy(), its)
    srv = serving.Server(max_vertices=16_000_000, max_entries=320_000_000, max_slots=2048, validate=False)
    serving.run_open_loop(srv, graphs, tr.arrivals, on_done=keep, mapped=True)
    srv.close()
    for i, g in enumerate(graphs):
        lab, its = want[id(g)]
        assert got[i] is not None, i
        assert np.array_equal(got[i][0], lab), (i, g.name)
        assert got[i][1] == its, (i, g.name, got[i][1], its)


def test_server_cancel(gpu_ok):
    """A queued request is dropped at once; an admitted one (here the largest,
    whose column ids go by DMA) leaves at the next step; neither is ever
    reported, and the pool ranges they held serve later requests correctly.
    EBUSY only while the admission copies are in flight; unknown or delivered
    tickets are refused."""
    import paper_1910_05971_amd as fs
    from paper_1910_05971_amd.serving import Server
    big = gg.rmat(18, 16, seed=81)
    small = [gg.er(4000, 9000, seed=82 + k) for k in range(6)]
    srv = Server(max_vertices=600_000, max_entries=12_000_000, max_slots=8)
    t_big = srv.submit(big.row_ptr, big.col)
    t_small = [srv.submit(g.row_ptr, g.col) for g in small]
    assert srv.cancel(t_small[2]) == fs.FASTSV_OK  # still queued
    assert srv.cancel(987654321) == fs.FASTSV_EINVAL
    got = {}
    srv.step()
    busy = 0
    while True:
        st = srv.cancel(t_big)
        if st == fs.FASTSV_OK:
            break
        assert st == fs.FASTSV_EBUSY
        busy += 1
        srv.step()
        assert busy < 10000
    for _ in range(10000):
        r, q = srv.step()
        for t, lab, its in srv.poll():
            got[t] = (lab.copy(), its)
        if r == 0 and q == 0:
            break
    assert t_big not in got and t_small[2] not in got
    for k, t in enumerate(t_small):
        if k == 2:
            continue
        lab, its = _expected(small[k])
        assert np.array_equal(got[t][0], lab) and got[t][1] == its
    assert srv.cancel(t_small[0]) == fs.FASTSV_EINVAL  # delivered
    st = srv.stats()
    assert st.cancelled == 2 and st.completed == len(small) - 1
    # the freed ranges serve the same graphs again
    t2 = [srv.submit(g.row_ptr, g.col) for g in [big] + small]
    got2 = {}
    for _ in range(10000):
        r, q = srv.step()
        for t, lab, its in srv.poll():
            got2[t] = (lab.copy(), its)
        if r == 0 and q == 0:
            break
    srv.close()
    for t, g in zip(t2, [big] + small):
        lab, its = _expected(g)
        assert np.array_equal(got2[t][0], lab) and got2[t][1] == its, g.name
