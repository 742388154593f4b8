"""fastsv_cc_csr_noalloc (the entry point that allocates no device memory)
against fastsv_cc_csr on the same graphs: labels bit-identical, the same
iteration count and per-iteration changed counts, on consecutive calls whose
second graph is smaller than the first (the scratch array keeps the first
call's contents), and the refusal of a graph whose workspace exceeds the
fixed scratch size."""
import numpy as np
import pytest
import torch

import oracle
from paper_1910_05971_amd import binding as b
from paper_1910_05971_amd import graphgen

pytestmark = pytest.mark.gpu


def _dev(g):
    return torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()


def _both(g, **kw):
    rp, col = _dev(g)
    want, ws = b.cc_csr(rp, col, **kw)
    got = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    got, gs = b.cc_csr_noalloc(rp, col, labels=got, **kw)
    torch.cuda.synchronize()
    return want.cpu().numpy(), ws, got.cpu().numpy(), gs


def _check(g, **kw):
    print(f"noalloc: {g.name} n={g.n} nnz={g.nnz} opts={kw}", flush=True)
    want, ws, got, gs = _both(g, **kw)
    assert np.array_equal(got, want)
    assert gs.iterations == ws.iterations
    assert gs.changed_list() == ws.changed_list()
    assert gs.sparse_list() == ws.sparse_list()
    return got, gs


def test_noalloc_equals_cc_csr_on_consecutive_calls(gpu_ok):
    big = graphgen.rmat(18, 16, seed=21)      # 262,144 vertices, about 8.4 M entries
    small = graphgen.er(5000, 9000, seed=22)  # ragged: several tiles and a partial last one
    got, st = _check(big)
    assert np.array_equal(got, oracle.uf_labels(big.n, big.row_ptr, big.col))
    got2, st2 = _check(small)
    assert np.array_equal(got2, oracle.uf_labels(small.n, small.row_ptr, small.col))
    ref = oracle.fastsv_alg2(small.n, small.row_ptr, small.col)
    assert st2.iterations == ref.iterations
    # again in the other order, with the sparse frontier off and then always on
    _check(big, frontier_tau=0.0)
    _check(small, frontier_tau=1.0)


def test_noalloc_options_and_edge_cases(gpu_ok):
    # dense-only, async, an ablation variant and a capped run through the same scratch
    g = graphgen.er(20000, 30000, seed=23)
    _check(g, frontier_tau=0.0)
    _check(g, sv_flags="sv2")
    rp, col = _dev(g)
    lab, st, code = b.cc_csr_noalloc(rp, col, max_iters=1, check=False)
    assert code == b.FASTSV_ENOTCONVERGED and st.iterations == 1
    lab_a, st_a = b.cc_csr_noalloc(rp, col, mode="async")
    assert np.array_equal(lab_a.cpu().numpy(), oracle.uf_labels(g.n, g.row_ptr, g.col))
    # no vertices, and vertices without edges
    e = graphgen.er(1, 0, seed=1)
    _check(e)
    iso = graphgen.er(300, 0, seed=1)
    got, _ = _check(iso)
    assert np.array_equal(got, np.arange(300, dtype=np.int32))
    rp0 = torch.zeros(1, dtype=torch.int32, device="cuda")
    col0 = torch.zeros(0, dtype=torch.int32, device="cuda")
    lab0, st0 = b.cc_csr_noalloc(rp0, col0)
    assert lab0.numel() == 0 and st0.iterations == 0


def test_noalloc_refuses_workspace_beyond_scratch(gpu_ok):
    # 4 M vertices need 5 int32[n] vectors = 80 MiB > 64 MiB: refused before
    # any launch, labels untouched
    n = 4 << 20
    assert b.workspace_bytes(n, 0, b.make_opts(binned=0)) > b.NOALLOC_SCRATCH_BYTES
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    lab = torch.full((n,), -5, dtype=torch.int32, device="cuda")
    _, _, code = b.cc_csr_noalloc(rp, col, labels=lab, check=False)
    assert code == b.FASTSV_ESCRATCH
    assert int((lab != -5).sum()) == 0
    # the largest vertex count that fits still runs (no edges: every vertex alone)
    n2 = 3 << 20
    assert b.workspace_bytes(n2, 0) <= b.NOALLOC_SCRATCH_BYTES
    rp2 = torch.zeros(n2 + 1, dtype=torch.int32, device="cuda")
    lab2, st2 = b.cc_csr_noalloc(rp2, col)
    assert st2.iterations == 1
    assert torch.equal(lab2, torch.arange(n2, dtype=torch.int32, device="cuda"))
