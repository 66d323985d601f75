"""In-closeness (the reversed graph's out-closeness) and the all-ties output
of Alg. 1, through the C ABI, against the oracle on the same inputs.

All-ties: the first min(k, n) vertices in the exact (f, id) order, then
every other vertex whose farness equals the k-th's exactly, by increasing
id.  In-closeness: the oracle's answer on the edge list with every arc
reversed.
"""
import numpy as np
import pytest

import graphgen
import oracle
from conftest import hip_available
from test_gpu_parity import graph, upload, expect

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


def expect_ties(name, k):
    g = graph(name)
    S, r = oracle.sums(g.n, g.edges, g.directed)
    ids = list(oracle.topk(S, r, k))
    kth = ids[-1]
    chosen = set(ids)
    tied = [v for v in range(g.n) if v not in chosen and oracle.cmp(S[v], r[v], S[kth], r[kth]) == 0]
    out = np.array(ids + tied, dtype=np.int32)
    far = np.array([oracle.farness(g.n, S[v], r[v]) for v in out])
    return out, S[out], r[out], far


TIE_GRAPHS = ["cycle", "complete", "star", "ties", "grid60", "king40", "ba2k", "gnp_d", "gnp_u", "forest",
              "sinks", "edgeless", "single", "reduction"]


@pytest.mark.parametrize("name", TIE_GRAPHS)
@pytest.mark.parametrize("k", [1, 3, 10])
def test_all_ties(ctx, name, k):
    dg = upload(ctx, name)
    wids, wS, wr, wf = expect_ties(name, k)
    for variant, mode in (("nbcut", "batched"), ("degcut", "hybrid"), ("nbbound", "batched"),
                          ("degcut", "plain"), ("auto", "auto")):
        ids, S, r, f, st = tkc.topk_closeness_ties(dg, k, variant, mode)
        assert np.array_equal(ids, wids), (variant, mode, ids[:20], wids[:20])
        assert np.array_equal(S, wS) and np.array_equal(r, wr) and np.array_equal(f, wf)
    # the first min(k, n) entries are the ordinary answer
    ids0, S0, r0, f0, _ = tkc.topk_closeness(dg, k, "nbcut", "hybrid")
    assert np.array_equal(ids0, wids[:len(ids0)])


def test_all_ties_capacity(ctx):
    g = graph("cycle")
    dg = upload(ctx, "cycle")
    ids = np.zeros(4, np.int32)
    rc, n_out, _ = tkc.tkc_topk_closeness_ties(dg.h, 2, tkc.TKC_NB_CUT, tkc.TKC_BATCHED, 4, ids)
    assert rc == tkc.TKC_EINVAL and n_out == g.n      # every cycle vertex ties
    with pytest.raises(tkc.TkcError) as e:            # cap below min(k, n)
        tkc.tkc_topk_closeness_ties(dg.h, 10, tkc.TKC_NB_CUT, tkc.TKC_BATCHED, 5, ids)
    assert e.value.code == tkc.TKC_EINVAL


@pytest.mark.parametrize("name", ["gnp_d", "rmat11", "rmat13", "dpath", "ties", "reduction", "sinks"])
def test_in_closeness(ctx, name):
    g = graph(name)
    rev = graphgen.make(name + "_rev", g.n, np.ascontiguousarray(g.edges[:, ::-1]), True)
    S, r = oracle.sums(rev.n, rev.edges, True)
    dg = tkc.Graph.from_graphgen(ctx, g, validate=True, reverse=True)
    try:
        for k in (1, 10, 50):
            wids = oracle.topk(S, r, k)
            for variant, mode in (("nbcut", "hybrid"), ("nbbound", "batched"), ("degcut", "plain")):
                ids, S2, r2, f2, st = tkc.topk_closeness(dg, k, variant, mode)
                assert np.array_equal(ids, wids) and np.array_equal(S2, S[wids]) and np.array_equal(r2, r[wids])
    finally:
        dg.free()


def test_reverse_is_a_no_op_when_undirected(ctx):
    g = graph("ba2k")
    dg = tkc.Graph.from_graphgen(ctx, g, reverse=True)
    try:
        ids, S, r, f, st = tkc.topk_closeness(dg, 10, "nbcut", "hybrid")
        wids, wS, wr, wf = expect("ba2k", 10)
        assert np.array_equal(ids, wids) and np.array_equal(S, wS)
    finally:
        dg.free()


@pytest.mark.parametrize("name", ["ba2k", "gnp_d", "rmat11", "grid60"])
def test_budget_plain(ctx, name):
    """tkc_topk_closeness_budget: a cap above the searches plain mode needs
    gives its exact answer; a cap below stops with TKC_ECANCELED, no answer,
    and counters of exactly that many searches."""
    dg = upload(ctx, name)
    want = expect(name, 10)
    ids, S, r, f, st = tkc.topk_closeness(dg, 10, "nbcut", "plain")
    assert np.array_equal(ids, want[0])
    need = st["bfs_started"]
    done, res, st2 = tkc.topk_closeness_budget(dg, 10, "nbcut", need + 5)
    assert done and np.array_equal(res[0], want[0]) and np.array_equal(res[1], want[1])
    assert st2["m_vis"] == st["m_vis"]
    if need >= 2:
        done, res, st3 = tkc.topk_closeness_budget(dg, 10, "nbcut", 1)
        assert not done and res is None
        assert st3["m_vis"] > 0
        # the answer of a later full query is unaffected
        ids4, S4, _, _, _ = tkc.topk_closeness(dg, 10, "nbcut", "plain")
        assert np.array_equal(ids4, want[0]) and np.array_equal(S4, want[1])
