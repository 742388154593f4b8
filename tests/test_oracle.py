"""The CPU oracle against its pins (no GPU)."""
import numpy as np
import pytest

import oracle as O
import oracle_pins as P


@pytest.fixture(scope="module")
def orc():
    return O.default()


def test_exhaustive_n6(orc):
    P.pin_exhaustive(orc, n=6)


def test_exhaustive_n4_and_below(orc):
    for n in range(1, 5):
        P.pin_exhaustive(orc, n=n)


def test_path_closed_form(orc):
    P.pin_path_closed_form(orc)


def test_golden_hand_worked(orc):
    P.pin_golden(orc)


def test_small_closed_forms(orc):
    P.pin_small_closed_forms(orc)


def test_known_components(orc):
    P.pin_known_components(orc)


def test_percolation_extremes(orc):
    P.pin_percolation_extremes(orc)


def test_scipy_reference(orc):
    P.pin_scipy(orc)


def test_invariants_and_alg2_equals_alg3(orc):
    P.pin_invariants(orc)


def test_early_termination(orc):
    P.pin_early_termination(orc)


def test_iteration_cap(orc):
    P.pin_iteration_cap(orc)


def test_sv_variants_path_closed_form(orc):
    P.pin_sv_path_closed_form(orc)


def test_sv4_follows_alg2(orc):
    P.pin_sv4_follows_alg2(orc)


def test_sv_root_hooks_keep_trees(orc):
    P.pin_sv_root_hooks_keep_trees(orc)


def test_empty_graph(orc):
    rp = np.zeros(1, dtype=np.int32)
    col = np.zeros(0, dtype=np.int32)
    assert orc.fastsv_alg2(0, rp, col).iterations == 0
    assert orc.uf_labels(0, rp, col).shape == (0,)


def test_self_loops_and_duplicates(orc):
    # loops and repeated entries change nothing
    pairs = [(0, 0), (1, 2), (2, 1), (1, 2), (3, 3), (4, 2)]
    rp, col = P.csr_from_pairs(5, pairs)
    want = P.py_bfs_labels(5, pairs)
    for name, lab in P.final_labels_all(orc, 5, rp, col).items():
        assert np.array_equal(lab, want), name


def test_warm_start_from_final_is_fixed_point(orc):
    # Algorithm 3 takes f as input; from the converged labels one iteration
    # confirms and changes nothing (Lemma "f stays unchanged", Appendix A).
    g = P.gg.er(3000, 4000, seed=31)
    lab = orc.uf_labels(g.n, g.row_ptr, g.col)
    r = orc.fastsv_alg3(g.n, g.row_ptr, g.col, f_init=lab)
    assert r.iterations == 1
    assert np.array_equal(r.f, lab)


def test_sv_ablation_counts_reported(orc):
    # Sec. 5.2 reports that the optimisations reduce iteration counts on real
    # graphs; here it is only reported, and each variant must be correct.
    for g in P.random_small_graphs():
        want = P.scipy_min_labels(g.n, g.row_ptr, g.col)
        its = {}
        for name, flags in O.SV_FLAGS.items():
            r = orc.sv_variant(g.n, g.row_ptr, g.col, flags)
            assert np.array_equal(r.f, want), (g.name, name)
            its[name] = r.iterations
        assert its["sv5"] <= its["sv4"]
