"""Planted mistakes in a COPY of the oracle source must be caught by the pins.

Each mutant edits one plausible mistake into a temporary copy of
``oracle/oracle.c`` (a dropped term, a wrong index, a transposed operand,
the wrong termination test), compiles it with gcc on the CPU and runs the pin
suite against it.  The real oracle is never modified.
"""
import os
import subprocess

import pytest

import oracle as O
import oracle_pins as P

MUTANTS = {
    # Algorithm 2
    "alg2_drop_stochastic": ("fn[f[u]] = min32(fn[f[u]], f[f[v]]);", ";"),
    "alg2_drop_aggressive": ("fn[u] = min32(fn[u], f[f[v]]);", ";"),
    "alg2_drop_shortcut": ("for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);\n        /* the next iteration", "/* the next iteration"),
    "alg2_hook_parent_not_grandparent": ("fn[f[u]] = min32(fn[f[u]], f[f[v]]);", "fn[f[u]] = min32(fn[f[u]], f[v]);"),
    "alg2_aggressive_parent_not_grandparent": ("fn[u] = min32(fn[u], f[f[v]]);", "fn[u] = min32(fn[u], f[v]);"),
    "alg2_stochastic_target_from_next": ("fn[f[u]] = min32(fn[f[u]], f[f[v]]);", "fn[fn[u]] = min32(fn[fn[u]], f[f[v]]);"),
    # (swapping u and v in the stochastic hook is an equivalent mutant: the
    # symmetric CSR holds both orientations of every edge)
    "alg2_stochastic_reads_u": ("fn[f[u]] = min32(fn[f[u]], f[f[v]]);", "fn[f[u]] = min32(fn[f[u]], f[f[u]]);"),
    "alg2_terminate_on_f": ("int32_t g = f[f[u]];\n            changed += (g != gprev[u]);", "int32_t g = f[u];\n            changed += (g != gprev[u]);"),
    "alg2_shortcut_parent": ("for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);\n        /* the next iteration", "for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[u]);\n        /* the next iteration"),
    # Algorithm 3
    # (indexing the assign by the partly updated f instead of value is an
    # equivalent mutant in increasing-i order: f[i] can only have been lowered
    # by some j with f[j] = i <= j, i.e. not before i itself is processed)
    "alg3_assign_value_gf": ("f[value[i]] = min32(f[value[i]], mngf[i]);", "f[value[i]] = min32(f[value[i]], gf[i]);"),
    "alg3_mxv_gathers_f": ("for (int32_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e) t = min32(t, gf[col[e]]);",
                           "for (int32_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e) t = min32(t, f[col[e]]);"),
    "alg3_drop_assign": ("for (int32_t i = 0; i < n; ++i) f[value[i]] = min32(f[value[i]], mngf[i]);", ";"),
    "alg3_drop_aggressive": ("for (int32_t i = 0; i < n; ++i) f[i] = min32(f[i], mngf[i]);", ";"),
    "alg3_mxv_skips_first": ("for (int32_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e) t = min32(t, gf[col[e]]);",
                             "for (int32_t e = row_ptr[i] + 1; e < row_ptr[i + 1]; ++e) t = gf[col[e]];"),
    "alg3_extract_parent": ("for (int32_t i = 0; i < n; ++i) gf[i] = f[value[i]];", "for (int32_t i = 0; i < n; ++i) gf[i] = f[i];"),
    "alg3_dup_not_updated": ("memcpy(dup, gf, (size_t)n * sizeof(int32_t));\n        ++it;", "++it;"),
    # convergence-ablation variants (Alg. 1 plus the changes of Sec. 3)
    "sv_root_test_dropped": ("if (f[u] == f[f[u]] && f[v] < f[u]) fn[f[u]]", "if (f[v] < f[u]) fn[f[u]]"),
    "sv_root_test_on_u": ("if (f[u] == f[f[u]] && f[v] < f[u]) fn[f[u]]", "if (f[u] == u && f[v] < f[u]) fn[f[u]]"),
    "sv_hook_condition_on_grandparent": ("if (f[u] == f[f[u]] && f[v] < f[u]) fn[f[u]]", "if (f[u] == f[f[u]] && h < f[u]) fn[f[u]]"),
    # (a non-strict f[v] <= f[u] is an equivalent mutant: with f[v] = f[u] a
    # root, both f[v] and f[f[v]] equal f[u], which the root already holds)
    "sv_grandparent_ignored": ("int32_t h = grand ? f[f[v]] : f[v];\n                    if (f[u] == f[f[u]]", "int32_t h = f[v];\n                    if (f[u] == f[f[u]]"),
    "sv_hook_target_u": ("if (f[u] == f[f[u]] && f[v] < f[u]) fn[f[u]] = min32(fn[f[u]], h);", "if (f[u] == f[f[u]] && f[v] < f[u]) fn[u] = min32(fn[u], h);"),
    "sv_shortcut_to_root_test_parent": ("if (f[u] != f[f[u]]) fn[u] = f[f[u]];", "if (f[u] != f[f[u]]) fn[u] = f[u];"),
    "sv_stochastic_skips_shortcut": ("for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);\n            memcpy", "memcpy"),
    "sv_stochastic_aggressive_always": ("                        fn[u] = min32(fn[u], h);\n                    }\n            for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);",
                                        "                        fn[u] = min32(fn[u], h);\n                    }\n            for (int32_t u = 0; u < n; ++u) for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) fn[u] = min32(fn[u], f[f[col[e]]]);\n            for (int32_t u = 0; u < n; ++u) fn[u] = min32(fn[u], f[f[u]]);"),
    "sv_termination_tests_f_when_early": ("int32_t x = early ? f[f[u]] : f[u];", "int32_t x = f[u];"),
    # union-find and BFS
    "uf_link_smaller_below_larger": ("if (a < b) labels[b] = a;\n            else if (b < a) labels[a] = b;\n        }\n    }",
                                     "if (a < b) labels[a] = b;\n            else if (b < a) labels[b] = a;\n        }\n    }"),
    "uf_skip_last_entry": ("for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {\n            int32_t a = uf_find",
                           "for (int32_t e = row_ptr[u]; e + 1 < row_ptr[u + 1]; ++e) {\n            int32_t a = uf_find"),
    "bfs_label_by_visit": ("if (labels[y] < 0) { labels[y] = s; queue[tail++] = y; }", "if (labels[y] < 0) { labels[y] = x; queue[tail++] = y; }"),
}

PINS = [lambda o: P.pin_exhaustive(o, n=5), P.pin_path_closed_form, P.pin_golden,
        P.pin_small_closed_forms, P.pin_known_components, P.pin_scipy, P.pin_invariants,
        P.pin_sv_path_closed_form, P.pin_sv4_follows_alg2, P.pin_sv_root_hooks_keep_trees]


def _build_mutant(tmp_path, name, old, new):
    src = open(O.SOURCE).read()
    assert src.count(old) == 1, f"mutation site for {name} must occur exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-w", str(path), "-o", str(lib)], check=True)
    return O.Oracle(str(lib))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    orc = _build_mutant(tmp_path, name, old, new)
    caught = []
    for pin in PINS:
        try:
            pin(orc)
        except AssertionError as e:
            caught.append(str(e)[:120])
            break
    assert caught, f"no pin catches mutant {name}"


def test_unmutated_copy_passes(tmp_path):
    orc = _build_mutant(tmp_path, "identity", "static inline int32_t min32", "static inline int32_t min32")
    for pin in PINS:
        pin(orc)
