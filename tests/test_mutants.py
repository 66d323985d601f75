"""The oracle's pins catch plausible mistakes in the oracle.

Each case below plants one mistake in a copy of the oracle package: in
``oracle.c`` (a dropped term, a wrong sign, weight or index, a transposed
operand, a flipped tie rule, a missing step of Alg. 6) or in its Python
half (the degree bound on harmonic centrality, the harmonic order, the
default reachability brackets, outputs handed back in the wrong order).
The copy is built in a directory of its own and the oracle's pin files run
against it in a fresh pytest process (``ORACLE_PKG_DIR`` puts the copy
first on the import path).  A mistake passes this test only if some pin
fails on it; the unaltered package, copied and built the same way, must
pass every pin.  Nothing here runs on a GPU, and the oracle's own files are
never touched.
"""
import concurrent.futures
import glob
import os
import re
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
PINS = sorted(p for p in glob.glob(os.path.join(HERE, "test_oracle_*.py")))
PINS.append(os.path.join(HERE, "test_generators.py"))

# (name, text in oracle.c, replacement); a tuple of texts and a tuple of
# replacements change several places at once.  Every text must occur
# exactly once.
MUTANTS = [
    # adjacency
    ("adj_undirected_wrong_end",
     "A->nbr[fill[u]++] = v; A->nbr[fill[v]++] = u; }",
     "A->nbr[fill[u]++] = v; A->nbr[fill[v]++] = v; }"),
    ("adj_keeps_repeated_arcs",
     "if (q == a || A->nbr[q] != A->nbr[q - 1]) A->nbr[w++] = A->nbr[q];",
     "A->nbr[w++] = A->nbr[q];"),
    ("adj_keeps_self_loops",
     ("if (u < 0 || v < 0 || u >= n || v >= n) return -2;\n        if (u == v) continue;",
      "int32_t u = ed[2 * e], v = ed[2 * e + 1];\n        if (u == v) continue;\n        if (!directed) { A->nbr"),
     ("if (u < 0 || v < 0 || u >= n || v >= n) return -2;",
      "int32_t u = ed[2 * e], v = ed[2 * e + 1];\n        if (!directed) { A->nbr")),
    # textbook search (Sect. 1)
    ("bfs_distance_off_by_one",
     "d++;\n        S += d * (tail - level_end);",
     "S += d * (tail - level_end);\n        d++;"),
    ("bfs_reach_without_source",
     "*r_out = tail;",
     "*r_out = tail - 1;"),
    ("bfs_visited_not_cleared",
     "for (int64_t q = 0; q < tail; q++) seen[queue[q] >> 6] = 0;",
     ""),
    ("sums_ignore_source_list",
     "int32_t s = src ? src[i] : (int32_t)i;\n            S[i] = bfs_sum",
     "int32_t s = (int32_t)i;\n            S[i] = bfs_sum"),
    # harmonic centrality
    ("harmonic_distance_off_by_one",
     "h += (double)nd / (double)d;",
     "h += (double)nd / (double)(d + 1);"),
    ("harmonic_counts_source",
     "int64_t q = 1;\n    while (q < tail) {",
     "int64_t q = 0;\n    while (q < tail) {"),
    ("harmonic_ignore_source_list",
     "int32_t s = src ? src[i] : (int32_t)i;\n            h[i] = bfs_harmonic",
     "int32_t s = (int32_t)i;\n            h[i] = bfs_harmonic"),
    # the exact order (Sect. 2, Eq. 1)
    ("order_transposed_cross_product",
     "u128 x = (u128)(uint64_t)Sa * db, y = (u128)(uint64_t)Sb * da;",
     "u128 x = (u128)(uint64_t)Sa * da, y = (u128)(uint64_t)Sb * db;"),
    ("order_unreachable_first",
     "if (ia || ib) return ia - ib;",
     "if (ia || ib) return ib - ia;"),
    ("order_r_squared_not_r_minus_one",
     "u128 da = (u128)(uint64_t)(ra - 1) * (uint64_t)(ra - 1);\n"
     "    u128 db = (u128)(uint64_t)(rb - 1) * (uint64_t)(rb - 1);",
     "u128 da = (u128)(uint64_t)ra * (uint64_t)ra;\n"
     "    u128 db = (u128)(uint64_t)rb * (uint64_t)rb;"),
    ("order_square_dropped",
     "u128 da = (u128)(uint64_t)(ra - 1) * (uint64_t)(ra - 1);\n"
     "    u128 db = (u128)(uint64_t)(rb - 1) * (uint64_t)(rb - 1);",
     "u128 da = (u128)(uint64_t)(ra - 1);\n"
     "    u128 db = (u128)(uint64_t)(rb - 1);"),
    ("order_tie_to_larger_id",
     "return c < 0 || (c == 0 && a < b);",
     "return c < 0 || (c == 0 && a > b);"),
    ("farness_n_not_n_minus_one",
     "((double)(n - 1) * (double)S)",
     "((double)n * (double)S)"),
    ("farness_unreachable_zero",
     "if (r <= 1) return __builtin_inf();",
     "if (r <= 1) return 0.0;"),
    ("component_size_off_by_one",
     "size[queue[q]] = t;",
     "size[queue[q]] = t - 1;"),
    # SCCs and Alg. 6 (Sect. 8.4)
    ("scc_second_pass_forward",
     "for (int64_t e = R->off[u]; e < R->off[u + 1]; e++) {\n                int32_t w = R->nbr[e];",
     "for (int64_t e = G->off[u]; e < G->off[u + 1]; e++) {\n                int32_t w = G->nbr[e];"),
    ("scc_graphs_swapped_in_alg6",
     "int32_t nc = scc_kosaraju(&G, &R, comp);\n    int64_t *wt",
     "int32_t nc = scc_kosaraju(&R, &G, comp);\n    int64_t *wt"),
    ("largest_scc_tie_to_larger_id",
     "(wt[c] == wt[big] && minid[c] < minid[big])",
     "(wt[c] == wt[big] && minid[c] > minid[big])"),
    ("alg6_no_refinement",
     "if (to_big[c]) o = o2 + oS[big];",
     ""),
    ("alg6_no_cap_at_n",
     "if (o > n) o = n;",
     ""),
    ("alg6_alpha_sums_successors",
     "if (aS[y] > a) a = aS[y];",
     "a += aS[y];"),
    ("alg6_omega_max_of_successors",
     "o += oS[y];",
     "if (oS[y] > o) o = oS[y];"),
    ("alg6_alpha_without_own_size",
     "a += wt[c]; o += wt[c];",
     "o += wt[c];"),
    ("alg6_largest_scc_reach_truncated",
     "for (int32_t c = big; c < nc; c++)\n        if (from_big[c])",
     "for (int32_t c = big + 1; c < nc; c++)\n        if (from_big[c])"),
    # neighbourhood-based bound (Sect. 5)
    ("nb_subtract_d_not_d_minus_one",
     "u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)(d - 1) * (uint64_t)g2[s];\n"
     "                    acc =",
     "u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)d * (uint64_t)g2[s];\n"
     "                    acc ="),
    ("nb_subtract_d_in_both_bounds",
     ("u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)(d - 1) * (uint64_t)g2[s];\n"
      "                    acc =",
      "u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)(d - 1) * (uint64_t)g2[s];\n"
      "                acc ="),
     ("u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)d * (uint64_t)g2[s];\n"
      "                    acc =",
      "u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)d * (uint64_t)g2[s];\n"
      "                acc =")),
    ("nb_no_tree_correction",
     "            if (!directed) {\n                int64_t d = A.off[s + 1] - A.off[s];\n"
     "                if (acc < NB_INF) {",
     "            if (0) {\n                int64_t d = A.off[s + 1] - A.off[s];\n"
     "                if (acc < NB_INF) {"),
    ("nb_level_weight_minus_one",
     "rat_min(&num[s], &den[s], ps + k * (o - pv), (o - 1) * (o - 1));",
     "rat_min(&num[s], &den[s], ps + (k - 1) * (o - pv), (o - 1) * (o - 1));"),
    ("nb_first_level_sum_dropped",
     "if (nv < a) { sum[s] = d; vis[s] = nv; }",
     "if (nv < a) { sum[s] = 0; vis[s] = nv; }"),
    ("nb_alpha_end_skipped",
     "                if (!started[s]) {\n"
     "                    rat_min(&num[s], &den[s], ps + k * (a - pv), (a - 1) * (a - 1));",
     "                if (!started[s]) {\n"
     "                    rat_min(&num[s], &den[s], ps + k * (o - pv), (o - 1) * (o - 1));"),
    ("nb_harmonic_level_denominator",
     "ub[s] += (double)take / (double)k;",
     "ub[s] += (double)take / (double)(k + 1);"),
    ("nb_harmonic_fill_uncapped",
     "int64_t take = gk[s] < room ? gk[s] : room;",
     "int64_t take = gk[s];"),
    # BFSCut (Sect. 6, Lemma 6.1, Sect. 8.2)
    ("cut_paper_form_weight",
     "*paper = SD - U + (D + 2) * rem;",
     "*paper = SD - U + (D + 1) * rem;"),
    ("cut_tight_form_weight",
     "*tight = SD + (D + 1) * rem + (extra > 0 ? extra : 0);",
     "*tight = SD + (D + 2) * rem + (extra > 0 ? extra : 0);"),
    ("cut_undirected_parent_arc_counted",
     "U += (directed || D == 0) ? d : d - 1;",
     "U += d;"),
    ("cut_kink_candidate_dropped",
     "int64_t cands[3] = {a1, o1, nD + U};",
     "int64_t cands[3] = {a1, o1, a1};"),
    ("cut_level_distance_off_by_one",
     "dist[w] = D + 1; SD += D + 1;",
     "dist[w] = D + 1; SD += D;"),
    # level-based bound (Sect. 7, Eq. 4-5, Lemma 7.2, Sect. 8.3)
    ("lb_definition_near_weight",
     "                L += (t <= 1 ? 2 : t) * gam[j];\n            }\n            lev[i] = L;",
     "                L += (t <= 1 ? 1 : t) * gam[j];\n            }\n            lev[i] = L;"),
    ("lb_near_weight_in_definition_and_first_level",
     ("                L += (t <= 1 ? 2 : t) * gam[j];\n            }\n            lev[i] = L;",
      "            L += (t <= 1 ? 2 : t) * gam[j];\n        }\n        lev[1] = L;"),
     ("                L += (t <= 1 ? 1 : t) * gam[j];\n            }\n            lev[i] = L;",
      "            L += (t <= 1 ? 1 : t) * gam[j];\n        }\n        lev[1] = L;")),
    ("lb_recurrence_upper_index",
     "for (int32_t j = i + 2; j <= maxD; j++) hi += gam[j];",
     "for (int32_t j = i + 1; j <= maxD; j++) hi += gam[j];"),
    ("lb_recurrence_lower_index",
     "for (int32_t j = 0; j < i - 2; j++) lo += gam[j];",
     "for (int32_t j = 0; j <= i - 2; j++) lo += gam[j];"),
    ("lb_degree_not_subtracted",
     "int64_t b = lev[dist[v]] - d;",
     "int64_t b = lev[dist[v]];"),
    ("lb_outside_scc",
     "if (directed && scc && scc[v] != scc[s]) continue;\n"
     "        int64_t d = A.off[v + 1] - A.off[v];\n        int64_t b",
     "int64_t d = A.off[v + 1] - A.off[v];\n        int64_t b"),
    ("lb_harmonic_self_term_kept",
     "lev[l] = x - 0.5;",
     "lev[l] = x;"),
    ("lb_harmonic_neighbour_weight",
     "ub[v] = lev[dist[v]] + 0.5 * (double)d;",
     "ub[v] = lev[dist[v]] + 1.0 * (double)d;"),
    ("lb_harmonic_outside_scc",
     "if (directed && scc && scc[v] != scc[s]) continue;\n"
     "        int64_t d = A.off[v + 1] - A.off[v];\n        ub[v]",
     "int64_t d = A.off[v + 1] - A.off[v];\n        ub[v]"),
    ("lb_harmonic_undirected_signed_distance",
     "int64_t t = directed ? (int64_t)i - l : (i > l ? (int64_t)i - l : (int64_t)l - i);",
     "int64_t t = (int64_t)i - l;"),
    ("lb_undirected_signed_distance",
     "int64_t t = directed ? (int64_t)j - i : (j > i ? (int64_t)j - i : (int64_t)i - j);",
     "int64_t t = (int64_t)j - i;"),
]

# the same for oracle/__init__.py
PY_MUTANTS = [
    ("py_harmonic_order_tie_to_larger_id",
     "order = np.lexsort((np.arange(h.size), -h))",
     "order = np.lexsort((-np.arange(h.size), -h))"),
    ("py_harmonic_order_ascending",
     "order = np.lexsort((np.arange(h.size), -h))",
     "order = np.lexsort((np.arange(h.size), h))"),
    ("py_deg_bound_keeps_repeated_arcs",
     "e = np.unique(e[:, 0] * max(n, 1) + e[:, 1])",
     "e = e[:, 0] * max(n, 1) + e[:, 1]"),
    ("py_deg_bound_keeps_self_loops",
     "e = e[e[:, 0] != e[:, 1]]\n",
     "e = e\n"),
    ("py_deg_bound_undirected_one_way",
     "e = np.concatenate([e, e[:, ::-1]])",
     "e = np.concatenate([e, e])"),
    ("py_deg_bound_far_weight",
     "float(omega[v] - 1 - deg[v]) / 2.0",
     "float(omega[v] - 1 - deg[v]) / 3.0"),
    ("py_deg_bound_far_weight_loose",
     "float(omega[v] - 1 - deg[v]) / 2.0",
     "float(omega[v] - 1 - deg[v]) / 1.0"),
    ("py_deg_bound_near_weight",
     "out[v] = float(deg[v]) + float(omega[v] - 1 - deg[v]) / 2.0",
     "out[v] = float(deg[v]) / 2.0 + float(omega[v] - 1 - deg[v]) / 2.0"),
    ("py_walk_bound_stops_at_alpha",
     "        omega = reach_bounds(n, edges, directed)[1]\n    o = np.ascontiguousarray(omega",
     "        omega = reach_bounds(n, edges, directed)[0]\n    o = np.ascontiguousarray(omega"),
    ("py_nb_brackets_swapped",
     "        alpha, omega, _ = reach_bounds(n, edges, directed)",
     "        omega, alpha, _ = reach_bounds(n, edges, directed)"),
    ("py_sums_outputs_swapped",
     "return S[:cnt], r[:cnt]",
     "return r[:cnt], S[:cnt]"),
    ("py_nb_outputs_swapped",
     "return num[:n], den[:n]",
     "return den[:n], num[:n]"),
    ("py_alpha_omega_swapped",
     "return a[:n], o[:n], comp[:n]",
     "return o[:n], a[:n], comp[:n]"),
    ("py_lb_harmonic_ignores_scc",
     "        ptr = sc.ctypes.data_as(ctypes.c_void_p)\n    else:\n        sc = None\n        ptr = None\n"
     "    r = _L().oracle_lb_harmonic",
     "        ptr = None\n    else:\n        sc = None\n        ptr = None\n"
     "    r = _L().oracle_lb_harmonic"),
    ("py_closeness_farness_by_rank",
     "far = np.array([farness(n, S[i], r[i]) for i in ids], dtype=np.float64)",
     "far = np.array([farness(n, S[i], r[i]) for i in range(len(ids))], dtype=np.float64)"),
]

_BASE = "unaltered"


def _mutate(src, old, new):
    olds, news = (old, new) if isinstance(old, tuple) else ((old,), (new,))
    assert len(olds) == len(news)
    for o, w in zip(olds, news):
        assert src.count(o) == 1, "text must occur once: %r" % o
        src = src.replace(o, w)
    return src


def _run_one(tmp, name, c_text, py_text):
    d = os.path.join(tmp, name)
    pkg = os.path.join(d, "oracle")
    os.makedirs(pkg, exist_ok=True)
    for fname, text in (("oracle.c", c_text), ("__init__.py", py_text)):
        with open(os.path.join(pkg, fname), "w") as fh:
            fh.write(text)
    lib = os.path.join(pkg, "liboracle.so")
    b = subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-w", "-o", lib,
                        os.path.join(pkg, "oracle.c")], capture_output=True, text=True)
    if b.returncode:
        return ("build", b.stderr[-2000:])
    env = dict(os.environ, ORACLE_PKG_DIR=d, OMP_NUM_THREADS="1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           "--hypothesis-seed=0", "--timeout", "120", *PINS]
    try:
        p = subprocess.run(cmd, cwd=d, env=env, capture_output=True, text=True, timeout=600)
    except subprocess.TimeoutExpired:
        return ("timeout", "")
    out = p.stdout + p.stderr
    failed = re.findall(r"^FAILED (\S+)", out, re.M)
    return (p.returncode, failed[0] if failed else out[-2000:])


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    here = os.path.dirname(oracle.__file__)
    with open(os.path.join(here, "oracle.c")) as fh:
        c_src = fh.read()
    with open(os.path.join(here, "__init__.py")) as fh:
        py_src = fh.read()
    cases = {_BASE: (c_src, py_src)}
    for name, old, new in MUTANTS:
        cases[name] = (_mutate(c_src, old, new), py_src)
    for name, old, new in PY_MUTANTS:
        cases[name] = (c_src, _mutate(py_src, old, new))
    tmp = str(tmp_path_factory.mktemp("mutants"))
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        futs = {nm: ex.submit(_run_one, tmp, nm, c, py) for nm, (c, py) in cases.items()}
        return {nm: f.result() for nm, f in futs.items()}


def test_mutant_names_unique():
    names = [m[0] for m in MUTANTS + PY_MUTANTS]
    assert len(names) == len(set(names))


def test_unaltered_source_passes_the_pins(outcomes):
    rc, info = outcomes[_BASE]
    assert rc == 0, info


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS + PY_MUTANTS])
def test_pins_catch(outcomes, name):
    rc, info = outcomes[name]
    # 1: pytest ran and some pin failed (not a crash, a time-out or a build error)
    assert rc == 1, "mutant %s: pytest status %r\n%s" % (name, rc, info)
