"""GPU parity at the full sizes of the benchmark workloads, in the launch
configurations that bench.py times (and the autotuner picks).

The oracle cannot run every source at these sizes (hours of CPU), so each
check is on outputs it computes one at a time, or on properties that hold at
any size:
  - every returned (id, S, r) equals the oracle's textbook BFS from that id;
  - the returned list is strictly increasing in the exact (f, id) order, and
    each farness double follows from (S, r) by the fixed formula;
  - no sampled vertex outside the result (seeded random vertices plus the
    highest-degree ones, the likeliest central vertices) precedes the k-th
    result in that order;
  - every mode and batch width returns the same answer;
  - step outputs at full size: (S, r) of sampled sources from the batched
    engine, reachability (alpha / omega / SCC) and the NB bound bit for bit,
    and the LB update of a few complete searches on the grid.
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


@functools.lru_cache(maxsize=None)
def workload(name):
    return graphgen.workload(name)


_DEV = {}


def dev(ctx, name):
    if name not in _DEV:
        _DEV[name] = tkc.Graph.from_graphgen(ctx, workload(name))
    return _DEV[name]


def sample_sources(g, count, seed, top_degree=0, exclude=()):
    rng = np.random.default_rng(seed)
    pick = set(rng.integers(0, g.n, size=count).tolist())
    if top_degree:
        deg = np.diff(g.row_ptr)
        pick |= set(np.argsort(-deg, kind="stable")[:top_degree].tolist())
    pick -= set(int(v) for v in exclude)
    return np.array(sorted(pick), dtype=np.int32)


def check_topk(g, k, ids, S, r, f):
    kk = min(k, g.n)
    assert len(ids) == kk and len(set(ids.tolist())) == kk
    wS, wr = oracle.sums(g.n, g.edges, g.directed, sources=ids)
    assert np.array_equal(S, wS) and np.array_equal(r, wr)
    for i in range(kk):
        assert f[i] == oracle.farness(g.n, S[i], r[i]) or (np.isinf(f[i]) and r[i] <= 1)
    for i in range(1, kk):
        c = oracle.cmp(S[i - 1], r[i - 1], S[i], r[i])
        assert c < 0 or (c == 0 and ids[i - 1] < ids[i])
    # sampled outsiders never precede the k-th result
    out = sample_sources(g, 256, 11 + k, top_degree=32, exclude=ids)
    oS, orr = oracle.sums(g.n, g.edges, g.directed, sources=out)
    for v, sv, rv in zip(out.tolist(), oS.tolist(), orr.tolist()):
        c = oracle.cmp(sv, rv, S[-1], r[-1])
        assert c > 0 or (c == 0 and v > ids[-1]), (v, sv, rv)


# the bench configuration of the BA graph (hybrid, default knobs) for k = 1,
# 10, 100; other modes must agree
@pytest.mark.parametrize("k", [1, 10, 100])
def test_full_ba1m_topk(ctx, k):
    g = workload("ba1m")
    dg = dev(ctx, "ba1m")
    ids, S, r, f, st = tkc.topk_closeness(dg, k, "auto", "hybrid")
    check_topk(g, k, ids, S, r, f)
    modes = ("batched", "plain") if k == 10 else ("batched",)
    for mode in modes:
        ids2, S2, r2, f2, _ = tkc.topk_closeness(dg, k, "auto", mode)
        assert np.array_equal(ids2, ids) and np.array_equal(S2, S) and np.array_equal(r2, r)


# R-MAT: the autotuned configuration (batched, W = 128, four workgroups per
# CU) and the other modes and widths
def test_full_rmat20_topk(ctx):
    g = workload("rmat20")
    dg = dev(ctx, "rmat20")
    keep = ctx.tuning()
    try:
        ctx.tune(batch_width=128, blocks_per_cu=4)
        ids, S, r, f, st = tkc.topk_closeness(dg, 10, "auto", "batched")
        check_topk(g, 10, ids, S, r, f)
        ctx.tune(**keep)
        for mode in ("hybrid", "plain"):
            ids2, S2, r2, _, _ = tkc.topk_closeness(dg, 10, "auto", mode)
            assert np.array_equal(ids2, ids) and np.array_equal(S2, S) and np.array_equal(r2, r)
        ctx.tune(batch_width=256)
        ids2, S2, r2, _, _ = tkc.topk_closeness(dg, 10, "degcut", "batched")
        assert np.array_equal(ids2, ids) and np.array_equal(S2, S) and np.array_equal(r2, r)
    finally:
        ctx.tune(**keep)


# the road-like grid: AUTO picks NB + level-based updates, batched
def test_full_grid2000_topk(ctx):
    g = workload("grid2000")
    dg = dev(ctx, "grid2000")
    ids, S, r, f, st = tkc.topk_closeness(dg, 10, "auto", "batched")
    assert st["variant_used"] == tkc.TKC_NB_BOUND
    check_topk(g, 10, ids, S, r, f)


# Cut and level-based updates combined: the same answer on every workload
@pytest.mark.parametrize("name", ["ba1m", "rmat20", "grid2000"])
def test_full_cutlb_topk(ctx, name):
    g = workload(name)
    dg = dev(ctx, name)
    ids, S, r, f, st = tkc.topk_closeness(dg, 10, "nbcutlb", "batched")
    check_topk(g, 10, ids, S, r, f)
    assert st["variant_used"] == tkc.TKC_NB_CUTLB


@pytest.mark.parametrize("name", ["ba1m", "rmat20", "grid2000"])
def test_full_sums(ctx, name):
    g = workload(name)
    dg = dev(ctx, name)
    src = sample_sources(g, 160, 3)
    S, R = dg.sums(src)
    wS, wR = oracle.sums(g.n, g.edges, g.directed, sources=src)
    assert np.array_equal(S, wS) and np.array_equal(R, wR)


@pytest.mark.parametrize("name", ["ba1m", "rmat20", "grid2000"])
def test_full_reach(ctx, name):
    g = workload(name)
    dg = dev(ctx, name)
    a, o, sc = dg.reach()
    wa, wo, wc = oracle.reach_bounds(g.n, g.edges, g.directed)
    assert np.array_equal(a, wa) and np.array_equal(o, wo)
    if g.directed:
        pairs = set(zip(sc.tolist(), wc.tolist()))
        assert len(pairs) == len(set(sc.tolist())) == len(set(wc.tolist()))


def rat_equal(n1, d1, n2, d2):
    n1, d1, n2, d2 = (np.asarray(x, dtype=object) for x in (n1, d1, n2, d2))
    inf1, inf2 = d1 == 0, d2 == 0
    if not np.array_equal(inf1, inf2):
        return False
    fin = ~inf1
    return bool(np.all(n1[fin] * d2[fin] == n2[fin] * d1[fin]))


@pytest.mark.parametrize("name", ["ba1m", "rmat20"])
def test_full_nb_bound(ctx, name):
    g = workload(name)
    dg = dev(ctx, name)
    num, den, order = dg.bounds("nbcut")
    a, o, _ = oracle.reach_bounds(g.n, g.edges, g.directed)
    wn, wd = oracle.nb(g.n, g.edges, g.directed, a, o)
    assert rat_equal(num, den, wn, wd)
    assert np.array_equal(np.sort(order), np.arange(g.n))


def test_full_grid_lb_update(ctx):
    """The grid is connected, so every bound has the denominator (n-1)^2 and
    the level-based update is a plain integer maximum of numerators."""
    g = workload("grid2000")
    dg = dev(ctx, "grid2000")
    num0, den0, _ = dg.bounds("nbbound")
    d = (g.n - 1) ** 2
    assert np.all(den0 == d)
    src = sample_sources(g, 3, 17)
    num, den = dg.lb_update(src, num0, den0)
    assert np.all(den == d)
    want = num0.copy()
    for s in src.tolist():
        rs, b = oracle.lb_source(g.n, g.edges, g.directed, s, None)
        assert rs == g.n
        want = np.maximum(want, np.where(b >= 0, b, -1))
    assert np.array_equal(num, want)
