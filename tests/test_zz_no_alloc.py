"""The no-allocation reachability entry point against tkc_graph_reach.

tkc_graph_reach_noalloc takes its scratch from a static device array
instead of allocating; on the same graph it must give the same alpha and
omega bit for bit, and the same partition into strongly connected
components with ids in a topological order (the numbering itself is not
unique).  Two calls in a row, the second on a smaller graph, check that
nothing left in the shared array from the first call leaks into the second.
"""
import numpy as np
import pytest

import graphgen
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


def _noalloc(dg):
    import torch
    a = torch.full((dg.n,), -7, dtype=torch.int64, device="cuda")
    o = torch.full((dg.n,), -7, dtype=torch.int64, device="cuda")
    s = torch.full((dg.n,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    tkc.tkc_graph_reach_noalloc(dg.h, a, o, s if dg.directed else None)
    return a.cpu().numpy(), o.cpu().numpy(), (s.cpu().numpy() if dg.directed else None)


def _same(g, dg, got):
    a, o, sc = got
    wa, wo, ws = dg.reach()
    assert np.array_equal(a, wa) and np.array_equal(o, wo)
    if g.directed:
        pairs = set(zip(sc.tolist(), ws.tolist()))
        assert len(pairs) == len(set(sc.tolist())) == len(set(ws.tolist()))
        assert np.array_equal(np.unique(sc), np.arange(len(set(sc.tolist()))))
        u, v = g.edges[:, 0], g.edges[:, 1]
        assert np.all(sc[u] <= sc[v])


@pytest.mark.parametrize("pair", [("rmat13", "rmat11"), ("ba5000", "ba2000"), ("gnp_d", "dchain")])
def test_noalloc_matches_reach_twice(ctx, pair):
    graphs = {
        "rmat13": lambda: graphgen.rmat_graph(13, 16, seed=13),
        "rmat11": lambda: graphgen.rmat_graph(11, 8, seed=12),
        "ba5000": lambda: graphgen.ba_graph(5000, 5, 31),
        "ba2000": lambda: graphgen.ba_graph(2000, 3, 32),
        "gnp_d": lambda: graphgen.make("gnp_d", 3000, graphgen.gnp(3000, 0.0012, True, 41), True),
        # a long chain: the one-thread passes run inside the shared array
        "dchain": lambda: graphgen.make("dchain", 1500, np.array([(i + 1, i) for i in range(1499)],
                                                                  np.int32), True),
    }
    for name in pair:
        g = graphs[name]()
        dg = tkc.Graph.from_graphgen(ctx, g)
        try:
            _same(g, dg, _noalloc(dg))
        finally:
            dg.free()


def test_noalloc_scc_may_be_null(ctx):
    import torch
    g = graphgen.rmat_graph(12, 8, seed=14)
    dg = tkc.Graph.from_graphgen(ctx, g)
    try:
        a = torch.zeros(dg.n, dtype=torch.int64, device="cuda")
        o = torch.zeros(dg.n, dtype=torch.int64, device="cuda")
        tkc.tkc_graph_reach_noalloc(dg.h, a, o, None)
        wa, wo, _ = dg.reach()
        assert np.array_equal(a.cpu().numpy(), wa) and np.array_equal(o.cpu().numpy(), wo)
    finally:
        dg.free()


def test_noalloc_rejects_graphs_beyond_the_limit(ctx):
    import torch
    g = graphgen.rmat_graph(17, 16, seed=15)     # needs about 100 MB of scratch
    dg = tkc.Graph.from_graphgen(ctx, g)
    try:
        a = torch.zeros(dg.n, dtype=torch.int64, device="cuda")
        o = torch.zeros(dg.n, dtype=torch.int64, device="cuda")
        s = torch.zeros(dg.n, dtype=torch.int32, device="cuda")
        with pytest.raises(tkc.TkcError) as e:
            tkc.tkc_graph_reach_noalloc(dg.h, a, o, s)
        assert e.value.code == tkc.TKC_EINVAL
        assert "limit" in str(e.value)
    finally:
        dg.free()
