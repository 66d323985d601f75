"""Reachability bounds of directed graphs on the device (Sect. 8.4, Alg. 6).

The device path (trimming, a forward/backward search from a pivot, colour
propagation, the component DAG by sorting) must give alpha and omega bit
for bit equal to the oracle's, the same partition into strongly connected
components, and ids in a topological order of the component DAG.  Inputs
with long chains of components meet the parallel steps' round caps, and a
one-thread device pass finishes them; it must agree as well.
"""
import functools

import numpy as np
import pytest

import graphgen
import oracle
from conftest import hip_available

pytestmark = pytest.mark.gpu

if hip_available():
    from paper_1704_01077_amd import tkc
else:
    tkc = None


@pytest.fixture(scope="module")
def ctx():
    if not hip_available():
        pytest.skip("no GPU")
    import torch
    torch.cuda.init()
    c = tkc.Context(0)
    yield c
    c.close()


def _g(name, n, edges, directed=True):
    return graphgen.make(name, n, np.asarray(edges, dtype=np.int32).reshape(-1, 2), directed)


def _cycle(vs):
    return [(vs[i], vs[(i + 1) % len(vs)]) for i in range(len(vs))]


@functools.lru_cache(maxsize=None)
def graph(name):
    if name == "gnp_d":
        return _g(name, 600, graphgen.gnp(600, 0.004, True, 22))
    if name == "gnp_giant":       # one giant component plus tendrils
        return _g(name, 3000, graphgen.gnp(3000, 0.0012, True, 41))
    if name == "rmat11":
        return graphgen.rmat_graph(11, 8, seed=12)
    if name == "rmat13":
        return graphgen.rmat_graph(13, 16, seed=13)
    if name == "rmat15":
        return graphgen.rmat_graph(15, 8, seed=15)
    if name == "dpath":
        return _g(name, 90, [(i, i + 1) for i in range(89)])
    if name == "sinks":
        return _g(name, 40, np.zeros((0, 2), np.int32))
    if name == "scc_mix":
        # cycles of sizes 5, 3, 5, 2 and 1-vertex components, joined by a DAG;
        # two largest components of equal size (ties: the one with vertex 0)
        e = _cycle([7, 0, 9, 3, 11]) + _cycle([1, 4, 6]) + _cycle([2, 5, 8, 10, 12]) + _cycle([13, 14])
        e += [(1, 0), (2, 1), (12, 13), (14, 15), (3, 16), (16, 17), (6, 17), (18, 2), (18, 19), (19, 14)]
        return _g(name, 21, e)
    if name == "two_big_rev":
        # the same, with the tied components listed the other way round
        e = _cycle([2, 5, 8, 10, 12]) + _cycle([7, 0, 9, 3, 11]) + [(0, 2), (12, 13)]
        return _g(name, 14, e)
    if name == "cycle_chain":     # 2-cycles in a chain: many small components
        e = []
        for i in range(0, 400, 2):
            e += [(i, i + 1), (i + 1, i)]
            if i + 2 < 400:
                e.append((i + 1, i + 2))
        return _g(name, 400, e)
    if name == "dpath_desc":      # a long chain with decreasing ids
        n = 6000
        return _g(name, n, [(i + 1, i) for i in range(n - 1)])
    if name == "dpath_long":      # a long chain with increasing ids
        n = 6000
        return _g(name, n, [(i, i + 1) for i in range(n - 1)])
    if name == "cycle_chain_long":   # 3,000 2-cycles in a chain, ids falling along it
        n = 6000
        e = []
        for i in range(0, n, 2):
            a, b = n - 1 - i, n - 2 - i
            e += [(a, b), (b, a)]
            if b - 1 >= 0:
                e.append((b, b - 1))
        return _g(name, n, e)
    if name == "dag_deep":      # triangles in a chain of 300, plus side sinks: a deep DAG
        e = []
        for t in range(300):
            x, y, z = 3 * t, 3 * t + 1, 3 * t + 2
            e += [(x, y), (y, z), (z, x)]
            if t + 1 < 300:
                e.append((z, 3 * t + 3))
            e.append((x, 900 + t))
        return _g(name, 1200, e)
    raise KeyError(name)


DEVICE = ["gnp_d", "gnp_giant", "rmat11", "rmat13", "rmat15", "sinks", "scc_mix", "two_big_rev"]
# chains past the parallel steps' round caps (the component DAGs of dpath
# and cycle_chain are 89 and 199 deep)
SEQ = ["dpath", "cycle_chain", "dpath_desc", "dpath_long", "cycle_chain_long", "dag_deep"]


def check(g, a, o, sc):
    wa, wo, wc = oracle.alpha_omega(g.n, g.edges)
    assert np.array_equal(a, wa) and np.array_equal(o, wo)
    pairs = set(zip(sc.tolist(), wc.tolist()))
    assert len(pairs) == len(set(sc.tolist())) == len(set(wc.tolist()))
    # ids are 0..nc-1 and every arc goes forward (or stays in its component)
    assert np.array_equal(np.unique(sc), np.arange(len(set(sc.tolist()))))
    if len(g.edges):
        u, v = g.edges[:, 0], g.edges[:, 1]
        assert np.all(sc[u] <= sc[v])


@pytest.mark.parametrize("name", DEVICE + SEQ)
def test_reach_device_path(ctx, name):
    g = graph(name)
    dg = tkc.Graph.from_graphgen(ctx, g, validate=True)
    try:
        assert dg.reach_info()[0] == 0
        a, o, sc = dg.reach()
        check(g, a, o, sc)
        path, ms = dg.reach_info()
        assert path == (2 if name in SEQ else 1), (name, path)
        assert ms >= 0
        # cached: a second call gives the same arrays
        a2, o2, sc2 = dg.reach()
        assert np.array_equal(a, a2) and np.array_equal(o, o2) and np.array_equal(sc, sc2)
    finally:
        dg.free()


@pytest.mark.parametrize("name", ["dpath_desc", "cycle_chain_long", "dag_deep"])
def test_reach_seq_pass_exact(ctx, name):
    """Graphs whose chains exceed the parallel steps' round caps: the
    one-thread device pass finishes them, bit for bit equal to the oracle."""
    g = graph(name)
    dg = tkc.Graph.from_graphgen(ctx, g)
    try:
        a, o, sc = dg.reach()
        check(g, a, o, sc)
        assert dg.reach_info()[0] == 2
    finally:
        dg.free()


@pytest.mark.parametrize("name", ["rmat13", "scc_mix", "dpath_desc"])
def test_topk_after_device_reach(ctx, name):
    """Queries on graphs whose bounds came from either path stay exact."""
    g = graph(name)
    dg = tkc.Graph.from_graphgen(ctx, g)
    try:
        S, r = oracle.sums(g.n, g.edges, True)
        for k in (1, 10):
            ids, S1, r1, f1, _ = tkc.topk_closeness(dg, k, "nbcut", "batched")
            want = oracle.topk(S, r, k)
            assert np.array_equal(ids, want) and np.array_equal(S1, S[want]) and np.array_equal(r1, r[want])
    finally:
        dg.free()
