"""Graphs uploaded with TKC_RELABEL: stored with their vertices renumbered by
decreasing out-degree, answered in the caller's ids.

The order of Alg. 1's output breaks ties on the smaller id (Sect. 2), and
Alg. 6 takes the largest strongly connected component with the smallest
id on ties, so every comparison must use the caller's ids.  Each test
below compares a relabelled upload with the oracle on the original
numbering: top-k closeness for every variant and engine, harmonic
centrality, the all-ties output, α and ω, and the entry points that
refuse a relabelled graph.
"""
import functools

import numpy as np
import pytest

import graphgen
import oracle
from conftest import hip_available
from test_gpu_parity import graph, expect, SMALL
from test_gpu_variants import expect_ties

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


_DEV = {}


def dev(ctx, name):
    if name not in _DEV:
        _DEV[name] = tkc.Graph.from_graphgen(ctx, graph(name), validate=True, relabel=True)
    return _DEV[name]


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("variant", ["degcut", "nbcut", "nbbound", "nbcutlb", "auto"])
@pytest.mark.parametrize("mode", ["plain", "batched", "hybrid"])
@pytest.mark.parametrize("k", [1, 10, 100])
def test_relabel_topk(ctx, name, variant, mode, k):
    ids, S, r, f, _ = tkc.topk_closeness(dev(ctx, name), k, variant, mode)
    wids, wS, wr, wf = expect(name, k)
    assert np.array_equal(ids, wids), (ids[:10], wids[:10])
    assert np.array_equal(S, wS) and np.array_equal(r, wr) and np.array_equal(f, wf)


@pytest.mark.parametrize("name", ["ba20k", "grid150", "rmat13"])
@pytest.mark.parametrize("mode", ["batched", "hybrid"])
@pytest.mark.parametrize("variant", ["nbcut", "degcut", "nbbound", "nbcutlb"])
def test_relabel_topk_medium(ctx, name, mode, variant):
    for k in (1, 10, 100):
        ids, S, r, f, _ = tkc.topk_closeness(dev(ctx, name), k, variant, mode)
        wids, wS, wr, wf = expect(name, k)
        assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)


@pytest.mark.parametrize("width", [32, 128, 256])
def test_relabel_batch_widths(ctx, width):
    keep = ctx.tuning()
    try:
        ctx.tune(batch_width=width)
        for name in ("rmat13", "ba20k"):
            ids, S, r, f, _ = tkc.topk_closeness(dev(ctx, name), 10, "nbcut", "batched")
            wids, wS, wr, _ = expect(name, 10)
            assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)
    finally:
        ctx.tune(**keep)


@functools.lru_cache(maxsize=None)
def harmonic_truth(name):
    g = graph(name)
    return oracle.harmonic(g.n, g.edges, g.directed)


@pytest.mark.parametrize("name", ["ba2k", "grid60", "rmat11", "gnp_d", "ties", "star", "sinks", "rmat13"])
@pytest.mark.parametrize("variant", ["nbcut", "degcut", "nbbound"])
@pytest.mark.parametrize("mode", ["plain", "batched", "hybrid"])
def test_relabel_harmonic(ctx, name, variant, mode):
    h = harmonic_truth(name)
    for k in (1, 10):
        ids, hv, _ = tkc.topk_harmonic(dev(ctx, name), k, variant, mode)
        want = oracle.harmonic_topk(h, k)
        assert np.array_equal(ids, want) and np.array_equal(hv, h[want])


@pytest.mark.parametrize("name", ["cycle", "complete", "star", "ties", "grid60", "gnp_d", "forest", "sinks"])
@pytest.mark.parametrize("k", [1, 5])
def test_relabel_all_ties(ctx, name, k):
    wids, wS, wr, wf = expect_ties(name, k)
    for variant, mode in (("nbcut", "batched"), ("degcut", "hybrid"), ("nbbound", "batched"), ("degcut", "plain")):
        ids, S, r, f, _ = tkc.topk_closeness_ties(dev(ctx, name), k, variant, mode)
        assert np.array_equal(ids, wids), (variant, mode, ids[:20], wids[:20])
        assert np.array_equal(S, wS) and np.array_equal(r, wr) and np.array_equal(f, wf)


@pytest.mark.parametrize("name", ["gnp_d", "rmat11", "rmat13", "ties", "reduction", "dpath", "sinks"])
def test_relabel_reach(ctx, name):
    """α, ω and the partition by the caller's ids; the largest component's
    tie goes to the one holding the smallest caller's id."""
    g = graph(name)
    a, o, sc = dev(ctx, name).reach()
    wa, wo, wc = oracle.alpha_omega(g.n, g.edges)
    assert np.array_equal(a, wa) and np.array_equal(o, wo)
    pairs = set(zip(sc.tolist(), wc.tolist()))
    assert len(pairs) == len(set(sc.tolist())) == len(set(wc.tolist()))


def test_relabel_reach_tied_components(ctx):
    """Two largest components of equal size: ω depends on which one is C~,
    so the choice must follow the caller's ids even when the renumbering
    puts the other one first."""
    # component A = {0..4} (a 5-cycle of low out-degree), component B =
    # {5..9} (a 5-cycle whose vertices also point at the sinks 10..19:
    # high out-degree, so the renumbering lists B first); A reaches B
    e = [(i, (i + 1) % 5) for i in range(5)] + [(5 + i, 5 + (i + 1) % 5) for i in range(5)]
    e += [(5 + i, 10 + 2 * i + j) for i in range(5) for j in range(2)] + [(0, 5)]
    g = graphgen.make("tied_big", 20, np.asarray(e, np.int32), True)
    dg = tkc.Graph.from_graphgen(ctx, g, validate=True, relabel=True)
    try:
        a, o, _ = dg.reach()
        wa, wo, _ = oracle.alpha_omega(g.n, g.edges)
        assert np.array_equal(a, wa) and np.array_equal(o, wo)
        S, r = oracle.sums(g.n, g.edges, True)
        for k in (1, 5, 20):
            ids, S1, r1, _, _ = tkc.topk_closeness(dg, k, "nbcut", "hybrid")
            want = oracle.topk(S, r, k)
            assert np.array_equal(ids, want) and np.array_equal(S1, S[want]) and np.array_equal(r1, r[want])
    finally:
        dg.free()


def test_relabel_refusals(ctx):
    dg = dev(ctx, "rmat11")
    n = graph("rmat11").n
    calls = [
        lambda: dg.bounds("nbcut"),
        lambda: dg.harmonic_bounds("nbcut"),
        lambda: dg.sums([0, 1]),
        lambda: dg.lb_update([0], np.zeros(n, np.int64), np.zeros(n, np.int64)),
        lambda: dg.harmonic_lb_update([0], np.zeros(n, np.float64)),
        lambda: tkc.tkc_graph_reach_noalloc(dg.h, np.zeros(n, np.int64), np.zeros(n, np.int64),
                                            np.zeros(n, np.int32)),
        lambda: tkc.Pack(ctx, [dg]),
    ]
    for call in calls:
        with pytest.raises(tkc.TkcError) as e:
            call()
        assert e.value.code == tkc.TKC_EINVAL


def test_relabel_serving(ctx):
    """A server holding relabelled and plain graphs: packing takes only the
    plain ones, and every served answer is in the caller's ids."""
    names = ["rmat11", "ba2k", "gnp_d", "forest", "rmat13"]
    relabelled = {"rmat11", "ba2k", "rmat13"}
    gs = {nm: tkc.Graph.from_graphgen(ctx, graph(nm), validate=True, relabel=nm in relabelled) for nm in names}
    srv = tkc.Server(ctx, 8 << 30, 2)
    try:
        gid = {nm: srv.add(gs[nm]) for nm in names}
        srv.enable_packing(10000)     # gnp_d (directed) and forest (undirected): one member each
        rng = np.random.default_rng(5)
        reqs = []
        for _ in range(80):
            nm = names[int(rng.integers(len(names)))]
            reqs.append((nm, int(rng.choice([1, 10, 100])), ("nbcut", "degcut", "auto", "nbbound")[int(rng.integers(4))]))
        tickets = [srv.submit(gid[nm], k, var) for nm, k, var in reqs]
        for (nm, k, var), t in zip(reqs, tickets):
            ids, S, r, f, _ = srv.result(t, k)
            wids, wS, wr, wf = expect(nm, k)
            assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr), (nm, k, var)
            assert np.array_equal(f, wf)
        assert srv.info()["served"] == len(reqs)
    finally:
        srv.close()
        for g in gs.values():
            g.free()
