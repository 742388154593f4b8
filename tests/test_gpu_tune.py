"""Every option the autotuner may pick leaves the labels and the whole
trajectory (iteration count, changed counts per iteration) equal to the
oracle's Algorithm 2; the tuner's cache feeds cc_csr(tuned=True)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1910_05971_amd import graphgen as gg
from paper_1910_05971_amd import tune

pytestmark = pytest.mark.gpu


def test_every_candidate_keeps_the_trajectory(gpu_ok):
    import paper_1910_05971_amd as fs
    for g in (gg.rmat(16, 16, seed=91), gg.grid(300, 300, 0.55, seed=92), gg.er(50000, 150000, seed=93)):
        want = O.uf_labels(g.n, g.row_ptr, g.col)
        ref = O.fastsv_alg2(g.n, g.row_ptr, g.col, trace_cap=256, record_f=False)
        rp, col = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
        for c in tune.csr_candidates(g.n, g.nnz, all_bins=True):
            print(f"[gpu] tune candidate {g.name} {c}", flush=True)
            lab, st = fs.cc_csr(rp, col, binned=True, **c)
            assert np.array_equal(lab.cpu().numpy(), want), (g.name, c)
            assert st.iterations == ref.iterations, (g.name, c)
            assert st.changed_list() == ref.changed.tolist()[:64], (g.name, c)


def test_tuner_cache_feeds_tuned_calls(gpu_ok, tmp_path, monkeypatch):
    import paper_1910_05971_amd as fs
    monkeypatch.setenv("FASTSV_TUNING_CACHE", str(tmp_path / "tuning.json"))
    g = gg.rmat(15, 16, seed=94)
    rp, col = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
    rec = tune.tune_csr(rp, col, reps=1)
    assert len(rec["results"]) == len(tune.TAUS) and rec["best"]["ms"] > 0
    got = tune.lookup(0, g.n, g.nnz)
    assert got == rec["best"]["opts"]
    lab, st = fs.cc_csr(rp, col, tuned=True)
    assert np.array_equal(lab.cpu().numpy(), O.uf_labels(g.n, g.row_ptr, g.col))
    assert st.iterations == O.fastsv_alg2(g.n, g.row_ptr, g.col).iterations
    # a size class that was never tuned: no options
    assert tune.lookup(0, 10 * g.n, 10 * g.nnz) == {}
    # the batch threshold and the server's admission size
    b = gg.batch(32, seed=95, max_n=3000)
    t = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (b.vtx_off, b.edge_off, b.row_ptr, b.col)]
    rb = tune.tune_batch(*t, reps=1)
    assert rb["best"]["opts"]["frontier_tau"] in tune.TAUS
    from paper_1910_05971_amd import serving
    graphs = serving.pin_graphs([b.graph(i) for i in range(32)])
    rs = tune.tune_server(graphs, (200_000, 4_000_000, 64))
    assert rs["best"]["opts"]["admit_mb"] in tune.ADMIT_MB and rs["best"]["graphs_per_s"] > 0
    db = tune.load()
    assert {"csr", "batch", "server"} <= set(db[tune.device_key(0)])
