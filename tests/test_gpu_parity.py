"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Labels are compared element by element (bit-exact: integer work).  In the
default Jacobi mode the whole trajectory is deterministic (Sec. 2.4), so the
iteration count, the per-iteration count of changed grandparents and, on
moderate graphs, every iterate f_k (read back by capping max_iters at k) must
equal Algorithm 2's.
"""
import itertools
import json
import os
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


def to_dev(g):
    return (torch.from_numpy(np.ascontiguousarray(g.row_ptr)).cuda(),
            torch.from_numpy(np.ascontiguousarray(g.col)).cuda())


def solve(rp, col, expect_capped=None, **kw):
    """Solve; a capped run (max_iters) returns f after max_iters iterations.
    expect_capped=True asserts FASTSV_ENOTCONVERGED exactly (the cap fell
    before the termination test was met), False asserts FASTSV_OK; None
    accepts either for a capped run."""
    import paper_1910_05971_amd as fs
    labels, stats, st = fs.cc_csr(rp, col, check=False, **kw)
    torch.cuda.synchronize()
    if expect_capped is None:
        ok = (fs.FASTSV_OK, fs.FASTSV_ENOTCONVERGED) if kw.get("max_iters") else (fs.FASTSV_OK,)
    else:
        ok = (fs.FASTSV_ENOTCONVERGED,) if expect_capped else (fs.FASTSV_OK,)
    assert st in ok, f"status {st}, expected one of {ok}"
    return labels.cpu().numpy(), stats


def check_graph(g, taus=(0.05,), trajectory=False, oracle_alg2=True, **kw):
    _say(f"[gpu] {g.name} n={g.n} nnz={g.nnz} {kw}")
    rp, col = to_dev(g)
    want = O.uf_labels(g.n, g.row_ptr, g.col)
    ref = O.fastsv_alg2(g.n, g.row_ptr, g.col, trace_cap=256, record_f=trajectory) if oracle_alg2 else None
    for tau in taus:
        got, st = solve(rp, col, frontier_tau=tau, validate=True, **kw)
        assert np.array_equal(got, want), f"{g.name} tau={tau}: labels differ at {np.flatnonzero(got != want)[:10]}"
        if ref is not None:
            assert st.iterations == ref.iterations, (g.name, tau, st.iterations, ref.iterations)
            k = min(ref.iterations, 64)
            assert st.changed_list()[:k] == ref.changed[:k].tolist(), (g.name, tau)
    if trajectory and ref is not None:
        for k in range(1, ref.iterations + 1):
            for tau in taus:
                got, st = solve(rp, col, frontier_tau=tau, max_iters=k, expect_capped=k < ref.iterations, **kw)
                assert np.array_equal(got, ref.trace[k - 1]), f"{g.name} tau={tau}: f_{k} differs"
    return ref


def test_exhaustive_small_graphs(gpu_ok):
    # every graph on 5 vertices, dense and sparse-always
    n = 5
    pairs_all = list(itertools.combinations(range(n), 2))
    _say("[gpu] exhaustive n=5")
    for mask in range(1 << len(pairs_all)):
        pairs = [p for i, p in enumerate(pairs_all) if mask >> i & 1]
        rp_h, col_h = P.csr_from_pairs(n, pairs)
        want = P.py_bfs_labels(n, pairs)
        ref = O.fastsv_alg2(n, rp_h, col_h, trace_cap=16)
        rp, col = torch.from_numpy(rp_h).cuda(), torch.from_numpy(col_h).cuda()
        for tau in (0.0, 1.0):
            got, st = solve(rp, col, frontier_tau=tau)
            assert np.array_equal(got, want), (pairs, tau)
            assert st.iterations == ref.iterations, (pairs, tau)
            assert st.changed_list() == ref.changed.tolist(), (pairs, tau)


def test_golden_and_closed_forms(gpu_ok):
    import json
    import os
    for fname in sorted(os.listdir(P.GOLDEN)):
        if not fname.endswith(".json"):
            continue
        ex = json.load(open(os.path.join(P.GOLDEN, fname)))
        rp_h, col_h = P.csr_from_pairs(ex["n"], ex["edges"])
        rp, col = torch.from_numpy(rp_h).cuda(), torch.from_numpy(col_h).cuda()
        if "trajectory" in ex:
            for tau in (0.0, 1.0):
                for k, fk in enumerate(ex["trajectory"], start=1):
                    got, _ = solve(rp, col, frontier_tau=tau, max_iters=k, expect_capped=k < ex["iterations"])
                    assert got.tolist() == fk, (fname, tau, k)
        # hand-worked trajectories of the convergence-ablation variants
        for name, v in ex.get("variants", {}).items():
            for k, fk in enumerate(v["trajectory"], start=1):
                got, _ = solve(rp, col, sv_flags=v["flags"], max_iters=k, expect_capped=k < v["iterations"])
                assert got.tolist() == fk, (fname, name, k)
            _, st = solve(rp, col, sv_flags=v["flags"])
            assert st.iterations == v["iterations"] and st.changed_list() == v["changed"], (fname, name)
    for n in (1, 2, 3, 17, 64, 1000, 4097):
        rp_h, col_h = P.csr_from_pairs(n, [(u, u + 1) for u in range(n - 1)])
        rp, col = torch.from_numpy(rp_h).cuda(), torch.from_numpy(col_h).cuda()
        K = P.path_iterations(n)
        for tau in (0.0, 1.0):
            for k in range(1, K + 1):
                got, st = solve(rp, col, frontier_tau=tau, max_iters=k, expect_capped=k < K)
                assert np.array_equal(got, P.path_closed_form(n, k)), (n, tau, k)
            _, st = solve(rp, col, frontier_tau=tau)
            assert st.iterations == K


def test_random_trajectories(gpu_ok):
    graphs = [gg.er(3000, 3500, seed=41), gg.er(20000, 80000, seed=42), gg.rmat(14, 16, seed=43),
              gg.grid(100, 120, 0.55, seed=44), gg.rmat(12, 4, seed=45)]
    for g in graphs:
        check_graph(g, taus=(0.0, 0.05, 1.0), trajectory=True)


def test_edge_cases(gpu_ok):
    # empty vertex set
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    got, st = solve(rp, col)
    assert got.shape == (0,) and st.iterations == 0
    # edgeless
    for n in (1, 5, 100000):
        rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
        got, st = solve(rp, col)
        assert np.array_equal(got, np.arange(n)) and st.iterations == 1
    # self loops and duplicates only
    pairs = [(0, 0), (3, 3), (1, 2), (1, 2), (2, 1)]
    rp_h, col_h = P.csr_from_pairs(6, pairs)
    got, _ = solve(torch.from_numpy(rp_h).cuda(), torch.from_numpy(col_h).cuda())
    assert got.tolist() == [0, 1, 1, 3, 4, 5]


def test_hub_rows_and_ragged_tiles(gpu_ok):
    rng = np.random.default_rng(5)
    # one hub spanning hundreds of tiles, plus degree-15/16/17 rows around lane boundaries
    n = 300000
    hub = 123457
    pairs = [(hub, int(v)) for v in rng.choice(n, 150000, replace=False) if v != hub]
    for d in (15, 16, 17, 63, 64, 65, 1023, 1024, 1025):
        c = int(rng.integers(0, n))
        pairs += [(c, int(v)) for v in rng.integers(0, n, d) if v != c]
    rp_h, col_h = P.csr_from_pairs(n, pairs)
    g = gg.Graph("hub_ragged", n, rp_h, col_h, len(pairs))
    check_graph(g, taus=(0.0, 1.0), trajectory=True)


def test_sparse_rows_wide_windows(gpu_ok):
    # a few edges spread over a huge id range: tiles span far more rows than
    # the LDS window holds
    rng = np.random.default_rng(7)
    n = 3_000_000
    ids = np.sort(rng.choice(n, 4000, replace=False))
    pairs = [(int(ids[i]), int(ids[i + 1])) for i in range(0, 3999, 2)]
    pairs += [(int(ids[i]), int(ids[(i * 7) % 4000])) for i in range(0, 4000, 3)]
    rp_h, col_h = P.csr_from_pairs(n, pairs)
    g = gg.Graph("wide_windows", n, rp_h, col_h, len(pairs))
    check_graph(g, taus=(0.0, 1.0), trajectory=True)
    # the same through the binned passes (by default 256 bins, one per CU, of
    # 11719 rows; first iteration fused into the layout build at tau 0, built
    # lazily at tau 1)
    check_graph(g, taus=(0.0, 1.0), trajectory=True, binned=True)
    rp, col = to_dev(g)
    _, st = solve(rp, col, frontier_tau=0.0, binned=True)
    assert st.num_bins == 256 and st.bin_fused_first == 1


def test_binned_fill_window_edge(gpu_ok):
    # a cycle with sparse chords: its tiles of 1024 entries span 511 rows (the
    # fill's row window full, rows found by the scan over row starts) or 512-513
    # (one more than the window holds: rows found by searching row_ptr), mixed
    # in one layout build; checked iterate by iterate from the fused first
    # iteration on
    rng = np.random.default_rng(73)
    n = 200_000
    pairs = [(i, (i + 1) % n) for i in range(n)]
    pairs += [(int(a), int((a + n // 2 + 7) % n)) for a in rng.choice(n, 150, replace=False)]
    rp_h, col_h = P.csr_from_pairs(n, pairs)
    g = gg.Graph("chorded_cycle", n, rp_h, col_h, len(pairs))
    nnz = int(rp_h[-1])
    spans = []
    for e0 in range(0, nnz, 1024):
        e1 = min(nnz, e0 + 1024)
        r_lo = int(np.searchsorted(rp_h, e0, side="right")) - 1
        r_hi = int(np.searchsorted(rp_h, e1 - 1, side="right")) - 1
        spans.append(r_hi - r_lo + 1)
    assert 511 in spans and max(spans) > 511
    for shift in (12, 15):
        check_graph(g, taus=(0.0, 0.05), trajectory=True, binned=True, bin_shift=shift)


def test_binned_passes_trajectories(gpu_ok):
    # binned dense passes forced on moderate graphs with narrow bins: many bins,
    # bins shorter than one block-wide span of the dense pass (32768 entries),
    # and bins of one or several spans with a ragged last one (the R-MAT at
    # shift 10: about 32K entries per bin, at shift 12: about 131K)
    graphs = [(gg.rmat(14, 16, seed=61), 8), (gg.er(30000, 120000, seed=62), 8),
              (gg.grid(120, 150, 0.6, seed=63), 8), (gg.rmat(16, 8, seed=64), 8), (gg.er(40000, 90000, seed=65), 10),
              (gg.rmat(16, 16, seed=66), 10), (gg.rmat(16, 16, seed=68), 12)]
    for g, shift in graphs:
        ref = check_graph(g, taus=(0.0, 0.05), trajectory=True, binned=True, bin_shift=shift)
        rp, col = to_dev(g)
        _, st = solve(rp, col, frontier_tau=0.0, binned=True, bin_shift=shift)
        assert st.num_bins == (g.n + (1 << shift) - 1) >> shift
        assert st.binned_iterations == max(0, ref.iterations - 1), (g.name, st.binned_iterations)


def test_binned_span_choice(gpu_ok):
    # bins of at least 2^17 records take the filtered middle step (16 records
    # per lane and step), shorter ones the narrow one (8); 32 and 16 are also
    # asked for explicitly; each is checked iterate by iterate
    g = gg.rmat(16, 16, seed=69)
    for shift, ask, span in ((14, 0, 16), (14, 32, 32), (10, 0, 8), (10, 16, 16)):
        check_graph(g, taus=(0.0, 0.05), trajectory=True, binned=True, bin_shift=shift, bin_span=ask)
        rp, col = to_dev(g)
        _, st = solve(rp, col, frontier_tau=0.0, binned=True, bin_shift=shift, bin_span=ask)
        assert st.binned_iterations > 0 and st.bin_span == span, (shift, ask, st.bin_span)


def test_binned_automatic_width(gpu_ok):
    # more than 2^22 vertices: binned by default, with the automatic width of
    # ceil(5e6 / 256) = 19532 rows (not a power of two), one bin per CU
    g = gg.er(5_000_000, 15_000_000, seed=67)
    check_graph(g, taus=(0.0, 0.05))
    rp, col = to_dev(g)
    _, st = solve(rp, col)
    assert st.num_bins == 256 and st.binned_iterations > 0 and st.bin_fused_first == 1
    assert st.bin_span == 8  # about 117K records per bin


def test_binned_source_high_bits(gpu_ok):
    # graphs beyond 2^16 vertices, where the layout's records carry the low 16
    # bits of the source and markers the high bits:
    # * ER: tiles and fill rounds whose rows cross a multiple of 2^16;
    # * clusters far apart: one round whose rows span all 16 values of the high
    #   bits of a 10^6-vertex graph, most of them without entries (markers only);
    # * stars centred on both sides of a boundary, whose rows straddle tiles.
    g = gg.er(400_000, 1_200_000, seed=71)
    for shift in (12, 15):
        check_graph(g, taus=(0.0, 0.05), trajectory=True, binned=True, bin_shift=shift)
    # the same with each span of the dense pass asked for (the automatic one
    # is the narrow span here), so that every span meets markers mid-bin
    for span in (16, 32):
        check_graph(g, taus=(0.0,), trajectory=True, binned=True, bin_shift=15, bin_span=span)
    n = 1_000_000
    starts = (0, 70_000, 131_000, 300_000, 655_300, 999_900)
    pairs = []
    for s0 in starts:
        pairs += [(s0 + i, s0 + i + 1) for i in range(99)]
    pairs += [(starts[i] + 50, starts[i + 1] + 7) for i in range(0, len(starts) - 1, 2)]
    rp_h, col_h = P.csr_from_pairs(n, pairs)
    clusters = gg.Graph("far_clusters", n, rp_h, col_h, len(pairs))
    for shift in (12, 15):
        check_graph(clusters, taus=(0.0, 1.0), trajectory=True, binned=True, bin_shift=shift)
    rng = np.random.default_rng(72)
    n = 300_000
    pairs = [(65_535, int(v)) for v in rng.choice(n, 3000, replace=False) if v != 65_535]
    pairs += [(65_536, int(v)) for v in rng.choice(n, 3000, replace=False) if v != 65_536]
    pairs += [(131_071, int(v)) for v in rng.choice(n, 2000, replace=False) if v != 131_071]
    pairs += [(int(a), int(b)) for a, b in rng.integers(0, n, size=(20_000, 2)) if a != b]
    rp_h, col_h = P.csr_from_pairs(n, pairs)
    stars = gg.Graph("boundary_stars", n, rp_h, col_h, len(pairs))
    check_graph(stars, taus=(0.0, 0.05), trajectory=True, binned=True, bin_shift=13)


def test_binned_hub_and_unsorted_rows(gpu_ok):
    # a star centre with an entry in every bin, plus rows in random order
    n = 6000
    pairs = [(17, v) for v in range(n) if v != 17] + [(v, v + 1) for v in range(3000, 3100)]
    rp_h, col_h = P.csr_from_pairs(n, pairs)
    rng = np.random.default_rng(9)
    col_h = col_h.copy()
    for u in range(n):
        a, b = rp_h[u], rp_h[u + 1]
        col_h[a:b] = rng.permutation(col_h[a:b])
    g = gg.Graph("star_unsorted", n, rp_h, col_h, len(pairs))
    check_graph(g, taus=(0.0, 1.0), trajectory=True, binned=True, bin_shift=8)


def test_binned_too_many_bins_falls_back(gpu_ok):
    # 2049 bins of 2^8 vertices: more than the scatter pass supports, so the pull pass runs
    n = 2048 * 256 + 1
    pairs = [(0, n - 1), (5, 600000 % n), (300000, 300001)]
    rp_h, col_h = P.csr_from_pairs(n, pairs)
    g = gg.Graph("many_bins", n, rp_h, col_h, len(pairs))
    check_graph(g, taus=(0.0,), binned=True, bin_shift=8)
    rp, col = to_dev(g)
    _, st = solve(rp, col, frontier_tau=0.0, binned=True, bin_shift=8)
    assert st.num_bins == 0 and st.binned_iterations == 0


def test_validation_rejects_bad_graph(gpu_ok):
    import paper_1910_05971_amd as fs
    rp = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    col = torch.tensor([1, 7], dtype=torch.int32, device="cuda")  # 7 is out of range
    labels = torch.full((2,), -5, dtype=torch.int32, device="cuda")
    _, _, st = fs.cc_csr(rp, col, labels=labels, validate=True, check=False)
    assert st == fs.FASTSV_ERANGE
    assert labels.cpu().tolist() == [-5, -5]  # untouched
    rp_bad = torch.tensor([0, 2, 1], dtype=torch.int32, device="cuda")
    _, _, st = fs.cc_csr(rp_bad, torch.tensor([1], dtype=torch.int32, device="cuda"), validate=True,
                         check=False)
    assert st == fs.FASTSV_ERANGE


def test_deterministic_repeats(gpu_ok):
    g = gg.rmat(15, 16, seed=46)
    rp, col = to_dev(g)
    outs = set()
    for _ in range(5):
        got, st = solve(rp, col, max_iters=2)
        outs.add(got.tobytes())
    assert len(outs) == 1


def test_config_c1(gpu_ok):
    g = gg.c1_er()
    check_graph(g, taus=(0.0, 0.05, 1.0), trajectory=True)


@pytest.mark.slow
def test_config_c3_grid(gpu_ok):
    g = gg.c3_grid()
    ref = config_counts("grid_4096x4096_p0.55")
    assert (ref["n"], ref["nnz"]) == (g.n, g.nnz)
    _say(f"[gpu] C3 n={g.n} nnz={g.nnz}")
    rp, col = to_dev(g)
    want = O.uf_labels(g.n, g.row_ptr, g.col)
    for tau, binned in ((0.05, None), (0.05, False), (1.0, True)):
        got, st = solve(rp, col, frontier_tau=tau, binned=binned, validate=True)
        assert np.array_equal(got, want), f"C3 tau={tau} binned={binned}"
        assert st.iterations == ref["iterations"], (tau, binned, st.iterations)
        assert st.changed_list() == ref["changed"], (tau, binned, st.changed_list())


def config_counts(key):
    """Algorithm 2's iteration count and changed counts on a full-size
    workload, written by tests/golden/configs/make_alg2_counts.py (oracle
    only); the graph's size is checked so that a generator change shows."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "configs", "alg2_counts.json")
    with open(path) as fh:
        return json.load(fh)[key]


@pytest.mark.slow
def test_config_c2_rmat(gpu_ok):
    g = gg.c2_rmat()
    _say(f"[gpu] C2 n={g.n} nnz={g.nnz}")
    ref = config_counts("rmat_scale24_ef16")
    assert (ref["n"], ref["nnz"]) == (g.n, g.nnz)
    rp, col = to_dev(g)
    want = O.uf_labels(g.n, g.row_ptr, g.col)
    assert int(np.count_nonzero(want == np.arange(g.n))) == ref["components"]
    for tau, binned in ((0.0, False), (0.05, None), (0.0, True), (1.0, True)):
        got, st = solve(rp, col, frontier_tau=tau, binned=binned)
        _say(f"[gpu] C2 tau={tau} binned={binned} iterations={st.iterations} "
             f"changed={st.changed_list()} binned_iterations={st.binned_iterations}")
        assert np.array_equal(got, want), f"C2 tau={tau} binned={binned}"
        assert st.iterations == ref["iterations"], (tau, binned, st.iterations)
        assert st.changed_list() == ref["changed"], (tau, binned, st.changed_list())
    O.check_final(got, g.row_ptr, g.col)
