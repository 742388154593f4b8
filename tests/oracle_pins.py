"""Pins for the CPU oracle: checks against facts that the paper and plain
mathematics fix, independent of the oracle's own code.

Every ``pin_*`` takes an ``oracle.Oracle`` (the default build or a test-only
mutant build) and raises AssertionError on a mismatch.  ``tests/test_oracle.py``
runs them on the real oracle; ``tests/test_oracle_mutants.py`` plants mistakes
in a copy of the oracle source and checks that some pin catches each one.
"""
from __future__ import annotations

import itertools
import json
import os
from collections import deque

import numpy as np

import oracle as O
from paper_1910_05971_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# Iteration cap for every oracle call made by a pin: far above what any pin
# graph needs, so a (planted) non-terminating variant fails instead of hanging.
CAP = 500


# ---------------------------------------------------------------- helpers

def csr_from_pairs(n, pairs):
    """Symmetric CSR built with numpy only (each pair stored both ways)."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    src = np.concatenate([pairs[:, 0], pairs[:, 1]])
    dst = np.concatenate([pairs[:, 1], pairs[:, 0]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, dst.astype(np.int32)


def py_bfs_labels(n, pairs):
    """Pure-Python brute force: label each component with its smallest vertex."""
    adj = [[] for _ in range(n)]
    for a, b in pairs:
        adj[a].append(b)
        adj[b].append(a)
    lab = [-1] * n
    for s in range(n):
        if lab[s] >= 0:
            continue
        lab[s] = s
        q = deque([s])
        while q:
            x = q.popleft()
            for y in adj[x]:
                if lab[y] < 0:
                    lab[y] = s
                    q.append(y)
    return np.array(lab, dtype=np.int32)


def scipy_min_labels(n, row_ptr, col):
    """Textbook routine (scipy's connected_components) mapped to min-id labels."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    a = sp.csr_matrix((np.ones(col.shape[0], dtype=np.int8), col, row_ptr), shape=(n, n))
    _, comp = connected_components(a, directed=False)
    mins = np.full(comp.max() + 1 if n else 0, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].astype(np.int32)


def final_labels_all(orc, n, rp, col):
    """Final labels from every oracle routine."""
    runs = {"alg2": orc.fastsv_alg2(n, rp, col, CAP), "alg3": orc.fastsv_alg3(n, rp, col, CAP)}
    for name, flags in O.SV_FLAGS.items():
        runs[name] = orc.sv_variant(n, rp, col, flags, CAP)
    out = {"uf": orc.uf_labels(n, rp, col), "bfs": orc.bfs_labels(n, rp, col)}
    for name, r in runs.items():
        assert r.iterations >= 0, f"{name} did not terminate within {CAP} iterations"
        out[name] = r.f
    f, it = orc.fastsv_async(n, rp, col, CAP)
    assert it >= 0, f"async did not terminate within {CAP} iterations"
    out["async"] = f
    return out


def path_closed_form(n, k):
    """Sorted path 0-1-...-(n-1): f_k[u] = max(0, u - (2^k - 1)).

    Derivation (Algorithm 2 with f_k of this form, a = 2^k - 1): the
    grandparent is g_k[u] = max(0, u - 2a); vertex u's best neighbour is u-1,
    offering g_k[u-1] = max(0, u - 1 - 2a) through aggressive hooking; the
    stochastic hook reaching x comes from u = x + a and offers
    max(0, x - 1 - a), never smaller; shortcutting offers g_k[x], never
    smaller.  Hence f_{k+1}[x] = max(0, x - (2a + 1)) and 2a + 1 = 2^{k+1} - 1.
    """
    a = (1 << k) - 1
    return np.maximum(0, np.arange(n, dtype=np.int64) - a).astype(np.int32)


def path_iterations(n):
    """g_{k-1} = g_k everywhere exactly when g_{k-1} is all zero, i.e. when
    (n-1) - 2(2^{k-1} - 1) <= 0, i.e. 2^k >= n + 1; the loop runs at least once."""
    return max(1, int(n).bit_length())


def random_small_graphs():
    """A few seeded random graphs of each workload shape (small sizes)."""
    gs = [gg.er(300, 400, seed=21), gg.er(2000, 2500, seed=22), gg.er(5000, 20000, seed=23),
          gg.rmat(12, 8, seed=24), gg.rmat(10, 4, seed=25),
          gg.grid(40, 50, 0.5, seed=26), gg.grid(64, 64, 0.55, seed=27)]
    return gs


# ---------------------------------------------------------------- pins

def pin_exhaustive(orc, n=6):
    """Every graph on n labelled vertices (all 2^(n(n-1)/2) edge sets): all
    routines agree with a pure-Python BFS; FastSV ends in a star forest."""
    all_pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(all_pairs)):
        pairs = [p for i, p in enumerate(all_pairs) if mask >> i & 1]
        rp, col = csr_from_pairs(n, pairs)
        want = py_bfs_labels(n, pairs)
        got = final_labels_all(orc, n, rp, col)
        for name, lab in got.items():
            assert np.array_equal(lab, want), f"n={n} edges={pairs}: {name} {lab} != {want}"
        r2 = orc.fastsv_alg2(n, rp, col, CAP)
        r3 = orc.fastsv_alg3(n, rp, col, CAP)
        assert r2.iterations == r3.iterations, f"edges={pairs}: iterations {r2.iterations} != {r3.iterations}"
        O.check_final(r2.f, rp, col)


def pin_path_closed_form(orc, sizes=(1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 33, 64, 100, 257)):
    """Trajectory and iteration count on the sorted path (closed form above)."""
    for n in sizes:
        rp, col = csr_from_pairs(n, [(u, u + 1) for u in range(n - 1)])
        K = path_iterations(n)
        for name, r in (("alg2", orc.fastsv_alg2(n, rp, col, CAP, trace_cap=64)),
                        ("alg3", orc.fastsv_alg3(n, rp, col, CAP, trace_cap=64))):
            assert r.iterations == K, f"path n={n} {name}: {r.iterations} iterations, expected {K}"
            prev_g = np.arange(n, dtype=np.int32)
            for k in range(1, K + 1):
                fk = path_closed_form(n, k)
                assert np.array_equal(r.trace[k - 1], fk), f"path n={n} {name}: f_{k} mismatch"
                gk = fk[fk]
                assert r.changed[k - 1] == int(np.count_nonzero(gk != prev_g)), \
                    f"path n={n} {name}: changed count at iteration {k}"
                prev_g = gk


def pin_golden(orc):
    """Hand-worked trajectories stored under tests/golden/: Algorithm 2's (run
    through Alg. 2, Alg. 3 and the sv5 variant) and, where a file lists them,
    those of the convergence-ablation variants sv1..sv4."""
    for fname in sorted(os.listdir(GOLDEN)):
        if not fname.endswith(".json"):
            continue
        with open(os.path.join(GOLDEN, fname)) as fh:
            ex = json.load(fh)
        n = ex["n"]
        rp, col = csr_from_pairs(n, ex["edges"])
        if "trajectory" in ex:
            for name, r in (("alg2", orc.fastsv_alg2(n, rp, col, CAP, trace_cap=32)),
                            ("alg3", orc.fastsv_alg3(n, rp, col, CAP, trace_cap=32)),
                            ("sv5", orc.sv_variant(n, rp, col, O.SV_FLAGS["sv5"], CAP, trace_cap=32))):
                assert r.iterations == ex["iterations"], f"{fname} {name}: iterations {r.iterations}"
                assert r.trace.tolist() == ex["trajectory"], f"{fname} {name}: trajectory {r.trace.tolist()}"
                assert r.changed.tolist() == ex["changed"], f"{fname} {name}: changed {r.changed.tolist()}"
        for name, v in ex.get("variants", {}).items():
            assert v["flags"] == O.SV_FLAGS[name], f"{fname}: flags of {name}"
            r = orc.sv_variant(n, rp, col, v["flags"], CAP, trace_cap=32)
            assert r.iterations == v["iterations"], f"{fname} {name}: iterations {r.iterations}"
            assert r.trace.tolist() == v["trajectory"], f"{fname} {name}: trajectory {r.trace.tolist()}"
            assert r.changed.tolist() == v["changed"], f"{fname} {name}: changed {r.changed.tolist()}"


def sv_path_closed_form(name, n, k):
    """Sorted path 0-1-...-(n-1), iterate k >= 1 of an ablation variant.

    sv1 and sv2 (Alg. 1, with or without grandparent hooking): in iteration 1
    every root u > 0 hooks onto u-1 and then shortcuts to u-2, so
    f_1[u] = max(0, u-2).  From then on a vertex whose parent is a root has
    parent 0 and no smaller neighbour parent, so no hook fires and each
    iteration is one pointer jump: f_k[u] = max(0, u - 2^k).
    sv3 (stochastic hooking without aggressive hooking): with f = max(0, u-a),
    the only vertex u whose parent is x > 0 is x + a; its neighbours' smallest
    grandparent is max(0, x - 1 - a), and the shortcut offers max(0, x - 2a),
    which is never larger for a >= 1.  From f_1[u] = max(0, u-1) this gives
    f_k[u] = max(0, u - 2^(k-1)).
    sv4 has Algorithm 2's iterates, f_k[u] = max(0, u - (2^k - 1)) (see
    path_closed_form).
    """
    u = np.arange(n, dtype=np.int64)
    a = {"sv1": 1 << k, "sv2": 1 << k, "sv3": 1 << (k - 1), "sv4": (1 << k) - 1}[name]
    return np.maximum(0, u - a).astype(np.int32)


def pin_sv_path_closed_form(orc, sizes=(1, 2, 3, 4, 5, 6, 9, 16, 17, 33, 100)):
    """Trajectories and iteration counts of sv1..sv4 on the sorted path.  They
    test f, so they stop at the first k with f_k = f_(k-1) (f_0 = iota)."""
    for n in sizes:
        rp, col = csr_from_pairs(n, [(u, u + 1) for u in range(n - 1)])
        for name in ("sv1", "sv2", "sv3", "sv4"):
            r = orc.sv_variant(n, rp, col, O.SV_FLAGS[name], CAP, trace_cap=64)
            prev = np.arange(n, dtype=np.int32)
            k = 0
            while True:
                k += 1
                fk = sv_path_closed_form(name, n, k)
                assert k <= r.iterations, f"path n={n} {name}: stopped after {r.iterations}, f_{k} still changes"
                assert np.array_equal(r.trace[k - 1], fk), f"path n={n} {name}: f_{k} {r.trace[k - 1]} != {fk}"
                assert r.changed[k - 1] == int(np.count_nonzero(fk != prev)), f"path n={n} {name}: changed[{k}]"
                if np.array_equal(fk, prev):
                    break
                prev = fk
            assert r.iterations == k, f"path n={n} {name}: {r.iterations} iterations, expected {k}"


def pin_sv4_follows_alg2(orc, graphs=None):
    """sv4 applies all three hooks of Algorithm 2 and tests f instead of f[f]
    (Sec. 3.4): its iterates are Algorithm 2's, continued by one iterate that
    Lemma T fixes (once f[f] is unchanged, f stays as it is), and it stops at
    the first iterate equal to its predecessor.  sv5 is Algorithm 2 itself."""
    for g in graphs or random_small_graphs():
        r2 = orc.fastsv_alg2(g.n, g.row_ptr, g.col, CAP, trace_cap=256)
        traj = list(r2.trace) + [r2.trace[-1]]  # Lemma T: the next iterate repeats
        prev = np.arange(g.n, dtype=np.int32)
        want_k = None
        for k, fk in enumerate(traj, start=1):
            if np.array_equal(fk, prev):
                want_k = k
                break
            prev = fk
        r4 = orc.sv_variant(g.n, g.row_ptr, g.col, O.SV_FLAGS["sv4"], CAP, trace_cap=256)
        assert r4.iterations == want_k, f"{g.name}: sv4 {r4.iterations} iterations, expected {want_k}"
        for k in range(want_k):
            assert np.array_equal(r4.trace[k], traj[k]), f"{g.name}: sv4 f_{k + 1}"
        r5 = orc.sv_variant(g.n, g.row_ptr, g.col, O.SV_FLAGS["sv5"], CAP, trace_cap=256)
        assert r5.iterations == r2.iterations, g.name
        assert np.array_equal(r5.trace, r2.trace) and np.array_equal(r5.changed, r2.changed), g.name


def pin_sv_root_hooks_keep_trees(orc, graphs=None):
    """Without stochastic hooking only roots are hooked (Alg. 1's test), so a
    tree is never split: two vertices with the same parent after an iterate
    keep a common root in every later iterate, and every hook lowers a root
    by moving it into a tree with a smaller id (Sec. 2.4)."""
    for g in graphs or random_small_graphs()[:4]:
        for name in ("sv1", "sv2"):
            r = orc.sv_variant(g.n, g.row_ptr, g.col, O.SV_FLAGS[name], CAP, trace_cap=256)
            assert r.iterations > 0, (g.name, name)
            steps = r.trace[:r.iterations]
            for k in range(1, len(steps)):
                a, b = steps[k - 1], steps[k]
                root_a, root_b = a.copy(), b.copy()
                for _ in range(24):  # pointer doubling: f^(2^24) reaches every root
                    root_a, root_b = root_a[root_a], root_b[root_b]
                # vertices in one tree of f_(k-1) share a tree of f_k
                order = np.argsort(root_a, kind="stable")
                ra, rb = root_a[order], root_b[order]
                same = ra[1:] == ra[:-1]
                assert np.all(rb[1:][same] == rb[:-1][same]), f"{g.name} {name}: a tree was split at {k + 1}"


def pin_small_closed_forms(orc):
    """Stars and cliques, worked by hand:
    * star centred at 0: every leaf hooks onto 0 in iteration 1 -> f_1 = 0,
      changed = [n-1, 0], 2 iterations;
    * star centred at n-1 (n >= 3): centre hooks onto 0 in iteration 1, leaves
      follow in iteration 2 -> changed = [1, n-2, 0], 3 iterations;
    * complete graph K_n: every u > 0 sees 0 -> f_1 = 0, 2 iterations;
    * edgeless graph: nothing changes, 1 iteration, f = iota."""
    for n in (3, 4, 9, 33):
        z = np.zeros(n, dtype=np.int32)
        cases = [
            ([(0, l) for l in range(1, n)], [n - 1, 0], [z, z]),
            ([(n - 1, l) for l in range(n - 1)], [1, n - 2, 0],
             [np.r_[np.arange(n - 1), 0].astype(np.int32), z, z]),
            (list(itertools.combinations(range(n), 2)), [n - 1, 0], [z, z]),
            ([], [0], [np.arange(n, dtype=np.int32)]),
        ]
        for pairs, changed, traj in cases:
            rp, col = csr_from_pairs(n, pairs)
            for name, r in (("alg2", orc.fastsv_alg2(n, rp, col, CAP, trace_cap=16)),
                            ("alg3", orc.fastsv_alg3(n, rp, col, CAP, trace_cap=16))):
                assert r.iterations == len(changed), f"n={n} {name} {pairs[:3]}: iterations {r.iterations}"
                assert r.changed.tolist() == changed, f"n={n} {name}: changed {r.changed.tolist()}"
                for k, fk in enumerate(traj):
                    assert np.array_equal(r.trace[k], fk), f"n={n} {name}: f_{k + 1}"


def _block_graph(blocks, rng):
    """Disjoint union of blocks, relabelled by a random permutation.
    Returns n, pairs, expected labels (smallest relabelled id per block)."""
    pairs, sizes = [], []
    base = 0
    for kind, s in blocks:
        ids = list(range(base, base + s))
        if kind == "path":
            pairs += [(ids[i], ids[i + 1]) for i in range(s - 1)]
        elif kind == "cycle":
            pairs += [(ids[i], ids[(i + 1) % s]) for i in range(s)] if s >= 3 else \
                [(ids[i], ids[i + 1]) for i in range(s - 1)]
        elif kind == "clique":
            pairs += list(itertools.combinations(ids, 2))
        elif kind == "star":
            pairs += [(ids[0], x) for x in ids[1:]]
        elif kind == "tree":
            pairs += [(ids[i], ids[int(rng.integers(0, i))]) for i in range(1, s)]
        sizes.append(s)
        base += s
    n = base
    perm = rng.permutation(n)
    pairs = [(int(perm[a]), int(perm[b])) for a, b in pairs]
    want = np.empty(n, dtype=np.int32)
    base = 0
    for s in sizes:
        members = perm[base:base + s]
        want[members] = members.min()
        base += s
    return n, pairs, want, len(sizes)


def pin_known_components(orc, trials=30, seed=7):
    """Disjoint unions of paths, cycles, cliques, stars and random trees under
    a random relabelling: k blocks give exactly k components, each labelled by
    its smallest (relabelled) vertex."""
    rng = np.random.default_rng(seed)
    kinds = ["path", "cycle", "clique", "star", "tree"]
    for _ in range(trials):
        blocks = [(kinds[int(rng.integers(0, 5))], int(rng.integers(1, 40))) for _ in range(int(rng.integers(1, 12)))]
        n, pairs, want, k = _block_graph(blocks, rng)
        rp, col = csr_from_pairs(n, pairs)
        for name, lab in final_labels_all(orc, n, rp, col).items():
            assert np.array_equal(lab, want), f"{blocks}: {name} labels"
            assert len(np.unique(lab)) == k, f"{blocks}: {name} component count"


def pin_percolation_extremes(orc):
    """Lattice with bond probability 0 has n components; with 1 it has one."""
    for p, expect in ((0.0, None), (1.0, 1)):
        g = gg.grid(23, 31, p, seed=5)
        want_count = g.n if expect is None else expect
        for name, lab in (("uf", orc.uf_labels(g.n, g.row_ptr, g.col)),
                          ("alg2", orc.fastsv_alg2(g.n, g.row_ptr, g.col, CAP).f)):
            assert len(np.unique(lab)) == want_count, f"grid p={p}: {name}"


def pin_scipy(orc, graphs=None):
    """Labels equal scipy's connected components mapped to min ids."""
    for g in graphs or random_small_graphs():
        want = scipy_min_labels(g.n, g.row_ptr, g.col)
        for name, lab in (("uf", orc.uf_labels(g.n, g.row_ptr, g.col)),
                          ("bfs", orc.bfs_labels(g.n, g.row_ptr, g.col)),
                          ("alg2", orc.fastsv_alg2(g.n, g.row_ptr, g.col, CAP).f),
                          ("alg3", orc.fastsv_alg3(g.n, g.row_ptr, g.col, CAP).f)):
            assert np.array_equal(lab, want), f"{g.name}: {name}"


def pin_invariants(orc, graphs=None):
    """Appendix A properties on every iterate, star forest at the end, and
    Algorithm 2 and Algorithm 3 produce the same iterates (both are written
    from the paper independently)."""
    for g in graphs or random_small_graphs():
        want = scipy_min_labels(g.n, g.row_ptr, g.col)
        r2 = orc.fastsv_alg2(g.n, g.row_ptr, g.col, CAP, trace_cap=256)
        r3 = orc.fastsv_alg3(g.n, g.row_ptr, g.col, CAP, trace_cap=256)
        assert r2.iterations > 0 and r2.iterations == r3.iterations, g.name
        assert np.array_equal(r2.trace, r3.trace), f"{g.name}: alg2 and alg3 iterates differ"
        assert np.array_equal(r2.changed, r3.changed), g.name
        O.check_invariants(r2.trace, want)
        O.check_final(r2.f, g.row_ptr, g.col)
        assert np.array_equal(r2.f, want), g.name
        # the termination count is the number of changed grandparents
        prev = np.arange(g.n, dtype=np.int32)
        for k, fk in enumerate(r2.trace):
            gk = fk[fk]
            assert r2.changed[k] == np.count_nonzero(gk != prev), f"{g.name}: changed[{k}]"
            prev = gk
        assert r2.changed[-1] == 0 and np.all(r2.changed[:-1] > 0), g.name


def pin_early_termination(orc, graphs=None):
    """Sec. 3.4: the grandparent test stops no later than the parent test and
    at most one iteration earlier, with the same final vector (sv5 vs sv4)."""
    for g in graphs or random_small_graphs():
        r5 = orc.sv_variant(g.n, g.row_ptr, g.col, O.SV_FLAGS["sv5"], CAP)
        r4 = orc.sv_variant(g.n, g.row_ptr, g.col, O.SV_FLAGS["sv4"], CAP)
        assert r5.iterations > 0 and r4.iterations > 0, g.name
        assert r5.iterations <= r4.iterations <= r5.iterations + 1, g.name
        assert np.array_equal(r5.f, r4.f), g.name


def pin_iteration_cap(orc):
    """max_iters below the true count returns -1 and the k-th iterate."""
    g = gg.grid(30, 30, 0.6, seed=9)
    full = orc.fastsv_alg2(g.n, g.row_ptr, g.col, CAP, trace_cap=256)
    assert full.iterations >= 3
    for k in (1, 2, full.iterations - 1):
        r = orc.fastsv_alg2(g.n, g.row_ptr, g.col, max_iters=k)
        assert r.iterations == -1
        assert np.array_equal(r.f, full.trace[k - 1])


ALL_PINS = [pin_path_closed_form, pin_golden, pin_small_closed_forms, pin_known_components,
            pin_percolation_extremes, pin_scipy, pin_invariants, pin_early_termination,
            pin_iteration_cap, pin_sv_path_closed_form, pin_sv4_follows_alg2, pin_sv_root_hooks_keep_trees]
