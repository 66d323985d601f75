"""Serving: graphs stay resident and top-k requests are admitted while
others run (continuous batching), within an HBM budget.

Every served result must equal the same request run alone on its own
context and the oracle's answer (tolerance zero: ids, S and r bit for bit,
farness from the fixed formula), whatever else was in flight.  Admission,
cancellation, graph lifetime and autotuned graphs are covered too.
"""
import functools
import time

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

GIB = 1 << 30


@pytest.fixture(scope="module")
def ctx():
    if not hip_available():
        pytest.skip("no GPU")
    import torch
    torch.cuda.init()
    c = tkc.Context(0)
    yield c
    c.close()


def _g(name, n, edges, directed):
    return graphgen.make(name, n, np.asarray(edges, dtype=np.int32).reshape(-1, 2), directed)


@functools.lru_cache(maxsize=None)
def graph(name):
    if name == "ba20k":
        return graphgen.ba_graph(20000, 5, 7)
    if name == "ba3k":
        return graphgen.ba_graph(3000, 3, 17)
    if name == "rmat13":
        return graphgen.rmat_graph(13, 16, seed=13)
    if name == "rmat11":
        return graphgen.rmat_graph(11, 8, seed=12)
    if name == "grid150":
        return graphgen.grid_graph(150, 0.05, 6, seed=6)
    if name == "king40":
        return graphgen.grid_graph(40, 0.05, 2, seed=8, king=True)
    if name == "gnp_d":
        return _g(name, 600, graphgen.gnp(600, 0.004, True, 22), True)
    if name == "forest":
        e1 = graphgen.tree(300, 31)
        e2 = graphgen.tree(200, 32) + 300
        return _g(name, 520, np.concatenate([e1, e2]), False)
    raise KeyError(name)


POOL = ["ba20k", "ba3k", "rmat13", "rmat11", "grid150", "king40", "gnp_d", "forest"]
VARIANTS = ["auto", "degcut", "nbcut", "degbound", "nbbound"]


@functools.lru_cache(maxsize=None)
def truth(name):
    g = graph(name)
    return oracle.sums(g.n, g.edges, g.directed)


def expect(name, k):
    g = graph(name)
    S, r = truth(name)
    ids = oracle.topk(S, r, k)
    far = np.array([oracle.farness(g.n, S[i], r[i]) for i in ids])
    return ids, S[ids], r[ids], far


@pytest.fixture(scope="module")
def pool(ctx):
    return {name: tkc.Graph.from_graphgen(ctx, graph(name)) for name in POOL}


def requests(count, seed):
    rng = np.random.default_rng(seed)
    return [(POOL[int(rng.integers(len(POOL)))], int(rng.choice([1, 10, 100])),
             VARIANTS[int(rng.integers(len(VARIANTS)))]) for _ in range(count)]


def test_served_equals_solo_and_oracle(ctx, pool):
    """Requests arrive in waves while earlier ones still run; each result
    equals its solo run and the oracle."""
    srv = tkc.Server(ctx, 8 * GIB, 4)
    try:
        gid = {name: srv.add(pool[name]) for name in POOL}
        reqs = requests(96, 1)
        tickets = []
        for i, (name, k, var) in enumerate(reqs):
            tickets.append(srv.submit(gid[name], k, var))
            if i % 8 == 7:
                time.sleep(0.002)   # let some of the wave start before the next arrives
        solo_ctx = tkc.Context(0)
        solo = {}
        try:
            for name in POOL:
                solo[name] = tkc.Graph.from_graphgen(solo_ctx, graph(name))
            for (name, k, var), t in zip(reqs, tickets):
                ids, S, r, f, lat = srv.result(t, k)
                wids, wS, wr, wf = expect(name, k)
                assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr), (name, k, var)
                assert np.array_equal(f, wf)
                assert lat >= 0
                sids, sS, sr, sf, _ = tkc.topk_closeness(solo[name], k, var, "hybrid")
                assert np.array_equal(ids, sids) and np.array_equal(S, sS) and np.array_equal(r, sr)
        finally:
            for g in solo.values():
                g.free()
            solo_ctx.close()
    finally:
        srv.close()


def test_tight_budget_still_serves(ctx, pool):
    """A budget far below four concurrent workspaces delays admission but
    still serves everything correctly."""
    srv = tkc.Server(ctx, 256 << 20, 4)
    try:
        gid = {name: srv.add(pool[name]) for name in ("ba3k", "gnp_d", "king40", "rmat11")}
        reqs = [(name, k, var) for name in gid for k in (1, 10) for var in ("nbcut", "nbbound")]
        tickets = [srv.submit(gid[name], k, var) for name, k, var in reqs]
        for (name, k, var), t in zip(reqs, tickets):
            ids, S, r, f, lat = srv.result(t, k)
            wids, wS, wr, wf = expect(name, k)
            assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)
    finally:
        srv.close()


def test_never_fitting_request_is_refused(ctx, pool):
    srv = tkc.Server(ctx, 1 << 20, 2)
    try:
        gid = srv.add(pool["ba20k"])
        with pytest.raises(tkc.TkcError) as e:
            srv.submit(gid, 10, "nbcut")
        assert e.value.code == tkc.TKC_EBUSY
    finally:
        srv.close()


def test_cancel_queued_request(ctx, pool):
    srv = tkc.Server(ctx, 8 * GIB, 1)
    try:
        gid = srv.add(pool["ba20k"])
        tickets = [srv.submit(gid, 100, "degcut") for _ in range(6)]
        srv.cancel(tickets[-1])
        with pytest.raises(tkc.TkcError) as e:
            srv.result(tickets[-1], 100)
        assert e.value.code == tkc.TKC_ECANCELED
        wids, wS, wr, wf = expect("ba20k", 100)
        for t in tickets[:-1]:
            ids, S, r, f, lat = srv.result(t, 100)
            assert np.array_equal(ids, wids) and np.array_equal(S, wS)
        with pytest.raises(tkc.TkcError) as e:
            srv.submit(gid + 5, 10, "nbcut")
        assert e.value.code == tkc.TKC_EINVAL
    finally:
        srv.close()


def test_graph_held_by_server_cannot_be_freed(ctx):
    g = tkc.Graph.from_graphgen(ctx, graph("forest"))
    srv = tkc.Server(ctx, GIB, 1)
    srv.add(g)
    with pytest.raises(tkc.TkcError) as e:
        tkc.tkc_graph_free(g.h)
    assert e.value.code == tkc.TKC_EBUSY
    srv.close()
    g.free()


def test_autotuned_graph_in_server(ctx):
    g = tkc.Graph.from_graphgen(ctx, graph("rmat13"))
    try:
        best, ms = g.autotune(10, "auto", budget_ms=2000.0)
        srv = tkc.Server(ctx, 8 * GIB, 2)
        try:
            gid = srv.add(g)
            tickets = [(k, srv.submit(gid, k, "auto")) for k in (1, 10, 100, 10)]
            for k, t in tickets:
                ids, S, r, f, lat = srv.result(t, k)
                wids, wS, wr, wf = expect("rmat13", k)
                assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)
        finally:
            srv.close()
    finally:
        g.free()


def test_packed_serving_equals_oracle(ctx, pool):
    """With packing on, requests on the small graphs are served together in
    packed launches; every answer still equals the oracle's, and requests
    that cannot be packed (level-based variants, two on one graph at once)
    are served alone."""
    srv = tkc.Server(ctx, 8 * GIB, 2)
    try:
        gid = {name: srv.add(pool[name]) for name in POOL}
        srv.enable_packing(10000)     # ba3k, rmat11, king40, gnp_d, forest (and not the rest)
        info = srv.info()
        assert info["packs"] == 2     # undirected and directed
        rng = np.random.default_rng(3)
        small = ["ba3k", "rmat11", "king40", "gnp_d", "forest"]
        reqs = []
        for _ in range(120):
            name = small[int(rng.integers(len(small)))] if rng.random() < 0.85 else POOL[int(rng.integers(len(POOL)))]
            reqs.append((name, int(rng.choice([1, 10, 100])), ("nbcut", "degcut", "auto", "nbbound")[int(rng.integers(4))]))
        tickets = [srv.submit(gid[name], k, var) for name, k, var in reqs]
        for (name, k, var), t in zip(reqs, tickets):
            ids, S, r, f, lat = srv.result(t, k)
            wids, wS, wr, wf = expect(name, k)
            assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr), (name, k, var)
            assert np.array_equal(f, wf)
        info = srv.info()
        assert info["served"] == len(reqs)
        assert info["packed"] >= 2 and info["pack_calls"] >= 1, info
        with pytest.raises(tkc.TkcError) as e:   # a pack's members stay held
            tkc.tkc_graph_free(pool["ba3k"].h)
        assert e.value.code == tkc.TKC_EBUSY
    finally:
        srv.close()
