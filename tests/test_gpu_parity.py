"""GPU parity: every step of the HIP path, called through the C ABI, against
the CPU oracle on the same seeded inputs.

Integer results (ids, S, r, reachability, bounds as exact rationals, the
processing order) must match bit for bit; the farness doubles follow from
(S, r) by one fixed formula and must be identical too.
"""
import functools
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle
from conftest import hip_available

pytestmark = pytest.mark.gpu

if hip_available():
    from paper_1704_01077_amd import tkc
else:   # collected on CPU only to be skipped
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


def _g(name, n, edges, directed):
    return graphgen.make(name, n, np.asarray(edges, dtype=np.int32).reshape(-1, 2), directed)


@functools.lru_cache(maxsize=None)
def graph(name):
    """Small and medium inputs: several tiles, ragged tails, the method's
    degenerate cases (sinks, isolated vertices, ties, disconnection)."""
    if name == "ba2k":
        return graphgen.workload("ba2k")
    if name == "ba20k":
        return graphgen.ba_graph(20000, 5, 7)
    if name == "ba3k_m2":
        return graphgen.ba_graph(3000, 2, 11)
    if name == "ba_path":     # BA with a hanging path: open vertices linger for many levels
        b = graphgen.ba(3000, 3, 17)
        return _g(name, 3030, np.concatenate([b, [(2999 + i, 3000 + i) for i in range(30)]]), False)
    if name == "grid60":
        return graphgen.grid_graph(60, 0.05, 3, seed=5)
    if name == "grid150":
        return graphgen.grid_graph(150, 0.05, 6, seed=6)
    if name == "king40":
        return graphgen.grid_graph(40, 0.05, 2, seed=8, king=True)
    if name == "rmat11":
        return graphgen.rmat_graph(11, 8, seed=12)
    if name == "rmat13":
        return graphgen.rmat_graph(13, 16, seed=13)
    if name == "gnp_u":       # undirected, disconnected, isolated vertices
        return _g(name, 700, graphgen.gnp(700, 0.002, False, 21), False)
    if name == "gnp_d":       # directed, many sinks, not strongly connected
        return _g(name, 600, graphgen.gnp(600, 0.004, True, 22), True)
    if name == "forest":      # two trees and isolated vertices
        e1 = graphgen.tree(300, 31)
        e2 = graphgen.tree(200, 32) + 300
        return _g(name, 520, np.concatenate([e1, e2]), False)
    if name == "cycle":
        return _g(name, 257, [(i, (i + 1) % 257) for i in range(257)], False)
    if name == "complete":
        return _g(name, 40, [(i, j) for i in range(40) for j in range(i + 1, 40)], False)
    if name == "star":
        return _g(name, 130, [(0, i) for i in range(1, 130)], False)
    if name == "dpath":
        return _g(name, 90, [(i, i + 1) for i in range(89)], True)
    if name == "ties":
        e = [(0, 1), (0, 2), (3, 4), (4, 5), (4, 6), (5, 7), (8, 9), (8, 10), (8, 11),
             (12, 13), (12, 14), (13, 15), (14, 16), (15, 17), (16, 18)]
        return _g(name, 19, e, True)
    if name == "reduction":
        sets = [{0}, {0, 1}, {2}, {1, 2, 3}, {3}, {0, 3}]
        n, e, _ = graphgen.reduction_graph(sets, 4, 7, 36)
        return _g(name, n, e, True)
    if name == "single":
        return _g(name, 1, np.zeros((0, 2), np.int32), False)
    if name == "edgeless":
        return _g(name, 50, np.zeros((0, 2), np.int32), False)
    if name == "sinks":
        return _g(name, 40, np.zeros((0, 2), np.int32), True)
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def truth(name):
    g = graph(name)
    S, r = oracle.sums(g.n, g.edges, g.directed)
    return S, r


@functools.lru_cache(maxsize=None)
def dev_graph(ctx_id, name):
    return tkc.Graph.from_graphgen(_CTX[0], graph(name), validate=True)


_CTX = [None]


def upload(ctx, name):
    _CTX[0] = ctx
    return dev_graph(id(ctx), name)


def expect(name, k):
    g = graph(name)
    S, r = truth(name)
    ids = oracle.topk(S, r, k)
    far = np.array([oracle.farness(g.n, S[i], r[i]) for i in ids])
    return ids, S[ids], r[ids], far


SMALL = ["ba2k", "ba3k_m2", "ba_path", "grid60", "king40", "rmat11", "gnp_u", "gnp_d", "forest", "cycle", "complete",
         "star", "dpath", "ties", "reduction", "single", "edgeless", "sinks"]


# ----------------------------------------------------------- step parity
@pytest.mark.parametrize("name", ["ba2k", "gnp_u", "forest", "grid60", "edgeless", "single"])
def test_reach_undirected(ctx, name):
    g = graph(name)
    dg = upload(ctx, name)
    a, o, _ = dg.reach()
    want = oracle.component_sizes(g.n, g.edges)
    assert np.array_equal(a, want) and np.array_equal(o, want)


@pytest.mark.parametrize("name", ["gnp_d", "rmat11", "rmat13", "ties", "reduction", "dpath", "sinks"])
def test_reach_directed(ctx, name):
    g = graph(name)
    dg = upload(ctx, name)
    a, o, sc = dg.reach()
    wa, wo, wc = oracle.alpha_omega(g.n, g.edges)
    assert np.array_equal(a, wa) and np.array_equal(o, wo)
    # same partition into strongly connected components
    pairs = set(zip(sc.tolist(), wc.tolist()))
    assert len(pairs) == len(set(sc.tolist())) == len(set(wc.tolist()))


def rat_equal(n1, d1, n2, d2):
    n1, d1, n2, d2 = (np.asarray(x, dtype=object) for x in (n1, d1, n2, d2))
    inf1, inf2 = d1 == 0, d2 == 0
    if not np.array_equal(inf1, inf2):
        return False
    fin = ~inf1
    return bool(np.all(n1[fin] * d2[fin] == n2[fin] * d1[fin]))


# the NB rounds' tail (a round over the few open vertices alone) succeeds on
# grid60 and gnp_u, fails and falls back to full rounds on gnp_d and ba_path
@pytest.mark.parametrize("name", ["ba2k", "ba20k", "ba_path", "grid60", "king40", "rmat11", "rmat13", "gnp_u",
                                  "gnp_d", "forest", "cycle", "star", "dpath", "reduction", "sinks", "single"])
def test_nb_bound_parity(ctx, name):
    g = graph(name)
    dg = upload(ctx, name)
    num, den, order = dg.bounds("nbcut")
    a, o, _ = oracle.reach_bounds(g.n, g.edges, g.directed)
    wn, wd = oracle.nb(g.n, g.edges, g.directed, a, o)
    assert rat_equal(num, den, wn, wd)
    # order: ascending bound, ties by id; the keys keep 12 mantissa bits of
    # the bound, so check monotonicity with a relative slack of 2^-11
    vals = [float("inf") if den[v] == 0 else num[v] / den[v] for v in order]
    assert sorted(order.tolist()) == list(range(g.n))
    for i in range(1, len(vals)):
        assert vals[i] >= vals[i - 1] * (1 - 2.0 ** -11) or vals[i - 1] == 0


@pytest.mark.parametrize("name", ["ba2k", "gnp_d", "star", "sinks", "edgeless"])
def test_deg_order(ctx, name):
    g = graph(name)
    dg = upload(ctx, name)
    num, den, order = dg.bounds("degcut")
    deg = np.diff(g.row_ptr)
    a, o, _ = oracle.reach_bounds(g.n, g.edges, g.directed)
    key = [(o[v] <= 1, -deg[v], v) for v in range(g.n)]
    assert order.tolist() == [v for _, _, v in sorted(key)]
    assert np.array_equal(den == 0, o <= 1) and np.all(num == 0)


@pytest.mark.parametrize("name", ["ba2k", "grid60", "rmat11", "gnp_d", "gnp_u", "reduction", "sinks"])
@pytest.mark.parametrize("width", [32, 64, 128, 256])
def test_sums_parity(ctx, name, width):
    g = graph(name)
    dg = upload(ctx, name)
    ctx.tune(batch_width=width)
    try:
        rng = np.random.default_rng(5)
        src = rng.integers(0, g.n, size=min(g.n, 3 * width + 7)).astype(np.int32)
        S, R = dg.sums(src)
        wS, wR = truth(name)
        assert np.array_equal(S, wS[src]) and np.array_equal(R, wR[src])
    finally:
        ctx.tune(batch_width=64)


@pytest.mark.parametrize("name", ["grid60", "ba2k", "gnp_u", "forest", "gnp_d", "rmat11", "reduction"])
def test_lb_update_parity(ctx, name):
    g = graph(name)
    dg = upload(ctx, name)
    num0, den0, _ = dg.bounds("nbbound")
    rng = np.random.default_rng(9)
    src = np.unique(rng.integers(0, g.n, size=70)).astype(np.int32)
    num, den = dg.lb_update(src, num0, den0)
    # oracle: the level-based bound of every source, kept when it beats the current one
    sc = oracle.scc(g.n, g.edges)[1] if g.directed else None
    S, r = truth(name)
    wn = [Fraction(int(num0[v]), int(den0[v])) if den0[v] else None for v in range(g.n)]
    for s in src:
        if r[s] <= 1:
            continue
        _, b = oracle.lb_source(g.n, g.edges, g.directed, int(s), sc)
        for v in range(g.n):
            if b[v] >= 0 and wn[v] is not None:
                cand = Fraction(int(b[v]), int(r[s] - 1) ** 2)
                if cand > wn[v]:
                    wn[v] = cand
    for v in range(g.n):
        got = None if den[v] == 0 else Fraction(int(num[v]), int(den[v]))
        assert got == wn[v], (v, got, wn[v])
        # still a lower bound on the exact farness
        if r[v] > 1:
            assert got <= Fraction(int(S[v]), int(r[v] - 1) ** 2)


# ------------------------------------------------------------- top-k parity
@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("variant", ["degcut", "nbcut", "degbound", "nbbound", "degcutlb", "nbcutlb", "auto"])
@pytest.mark.parametrize("mode", ["plain", "batched", "hybrid"])
@pytest.mark.parametrize("k", [1, 10, 100])
def test_topk_parity(ctx, name, variant, mode, k):
    g = graph(name)
    dg = upload(ctx, name)
    ids, S, r, f, st = tkc.topk_closeness(dg, k, variant, mode)
    wids, wS, wr, wf = expect(name, k)
    assert np.array_equal(ids, wids), (ids[:10], wids[:10])
    assert np.array_equal(S, wS) and np.array_equal(r, wr)
    assert np.array_equal(f, wf)
    assert st["bfs_exact"] >= min(k, g.n) or variant in ("degbound", "nbbound", "degcutlb", "nbcutlb", "auto")


@pytest.mark.parametrize("name", ["ba20k", "grid150", "rmat13"])
@pytest.mark.parametrize("mode", ["batched", "hybrid"])
@pytest.mark.parametrize("variant", ["nbcut", "degcut", "nbbound", "nbcutlb", "degcutlb"])
def test_topk_parity_medium(ctx, name, mode, variant):
    for k in (1, 10, 100):
        dg = upload(ctx, name)
        ids, S, r, f, st = tkc.topk_closeness(dg, k, variant, mode)
        wids, wS, wr, wf = expect(name, k)
        assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)


def test_k_larger_than_n_and_full_ranking(ctx):
    name = "ties"
    g = graph(name)
    dg = upload(ctx, name)
    for k in (g.n, g.n + 5, 1000):
        for mode in ("plain", "batched", "hybrid"):
            ids, S, r, f, st = tkc.topk_closeness(dg, k, "nbcut", mode)
            wids, wS, wr, wf = expect(name, g.n)
            assert len(ids) == g.n and np.array_equal(ids, wids)


@pytest.mark.parametrize("width", [32, 128, 256])
def test_batch_widths_topk(ctx, width):
    ctx.tune(batch_width=width)
    try:
        for name in ("ba2k", "gnp_d", "grid60"):
            dg = upload(ctx, name)
            for variant in ("nbcut", "nbbound"):
                ids, S, r, f, st = tkc.topk_closeness(dg, 10, variant, "batched")
                wids, wS, wr, wf = expect(name, 10)
                assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)
    finally:
        ctx.tune(batch_width=64)


def test_small_swarm_queue_defers(ctx):
    """A tiny per-workgroup queue forces deferrals; past batch-width of them
    the engine closes and the rest of the order runs batched."""
    keep = ctx.tuning()
    ctx.tune(swarm_qcap=64, batch_width=32)
    try:
        for name in ("ba20k", "rmat13"):
            dg = upload(ctx, name)
            ids, S, r, f, st = tkc.topk_closeness(dg, 10, "degcut", "hybrid")
            wids, wS, wr, wf = expect(name, 10)
            assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)
            assert st["deferred"] > 0
    finally:
        ctx.tune(**keep)


# ---------------------------------------------------------------- tuning
def test_tuning_roundtrip_and_validation(ctx):
    keep = ctx.tuning()
    assert keep["batch_width"] in (32, 64, 128, 256) and keep["mode"] in (0, 1, 2)
    try:
        ctx.tune(batch_width=128, blocks_per_cu=3, mode="hybrid", batch_alpha=5)
        t = ctx.tuning()
        assert (t["batch_width"], t["blocks_per_cu"], t["mode"], t["batch_alpha"]) == (128, 3, 2, 5)
        for bad in (dict(batch_width=96), dict(blocks_per_cu=0), dict(blocks_per_cu=9), dict(mode=3),
                    dict(swarm_qcap=8), dict(batch_alpha=0), dict(seed_lanes=300)):
            with pytest.raises(tkc.TkcError) as e:
                ctx.tune(**bad)
            assert e.value.code == tkc.TKC_EINVAL
        assert ctx.tuning() == t        # a refused setting changes nothing
    finally:
        ctx.tune(**keep)


@pytest.mark.parametrize("blocks", [1, 3, 4])
def test_blocks_per_cu_topk(ctx, blocks):
    keep = ctx.tuning()
    ctx.tune(blocks_per_cu=blocks)
    try:
        for name in ("ba20k", "gnp_d", "grid60"):
            dg = upload(ctx, name)
            for variant, mode in (("nbcut", "plain"), ("nbcut", "batched"), ("nbbound", "batched"),
                                  ("degcut", "hybrid")):
                ids, S, r, f, st = tkc.topk_closeness(dg, 10, variant, mode)
                wids, wS, wr, wf = expect(name, 10)
                assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)
    finally:
        ctx.tune(**keep)


@pytest.mark.parametrize("name", ["ba20k", "rmat13", "grid150"])
def test_autotune_then_auto_mode(ctx, name):
    keep = ctx.tuning()
    dg = upload(ctx, name)
    best, ms = dg.autotune(10, "auto", budget_ms=3000.0)
    assert ms > 0 and best["batch_width"] in (32, 64, 128, 256) and best["mode"] in (1, 2)
    assert 1 <= best["blocks_per_cu"] <= 8
    assert ctx.tuning() == keep       # the context's own knobs are untouched
    for k in (1, 10, 37):
        ids, S, r, f, st = tkc.topk_closeness(dg, k, "auto", "auto")
        wids, wS, wr, wf = expect(name, k)
        assert np.array_equal(ids, wids) and np.array_equal(S, wS) and np.array_equal(r, wr)
        assert np.array_equal(f, wf)
        assert st["batch_width"] == best["batch_width"] and st["mode_used"] == best["mode"]


# ---------------------------------------------------------------- errors
def test_error_codes(ctx):
    g = graph("ba2k")
    dg = upload(ctx, "ba2k")
    with pytest.raises(tkc.TkcError) as e:
        tkc.topk_closeness(dg, 0, "nbcut", "hybrid")
    assert e.value.code == tkc.TKC_EINVAL
    bad = g.col_idx.copy()
    bad[3] = g.n + 7
    with pytest.raises(tkc.TkcError) as e:
        tkc.Graph(ctx, g.n, g.row_ptr, bad, validate=True)
    assert e.value.code == tkc.TKC_EINVAL
    loop = g.col_idx.copy()
    loop[g.row_ptr[5]] = 5
    with pytest.raises(tkc.TkcError) as e:
        tkc.Graph(ctx, g.n, g.row_ptr, loop, validate=True)
    assert e.value.code == tkc.TKC_EINVAL
    asym = graph("gnp_d")
    with pytest.raises(tkc.TkcError) as e:   # directed arcs passed as an undirected graph
        tkc.Graph(ctx, asym.n, asym.row_ptr, asym.col_idx, validate=True)
    assert e.value.code == tkc.TKC_EINVAL
    with pytest.raises(tkc.TkcError) as e:
        tkc.tkc_graph_upload(ctx.h, g.n, g.arcs, g.row_ptr, g.col_idx, None, None, tkc.TKC_DIRECTED)
    assert e.value.code == tkc.TKC_EINVAL
    # checked on every upload, validate or not: ids out of range, row
    # pointers that decrease or do not end at m, n < 1, m out of range
    for v in (-1, g.n):
        bad = g.col_idx.copy()
        bad[-1] = v
        with pytest.raises(tkc.TkcError) as e:
            tkc.Graph(ctx, g.n, g.row_ptr, bad)
        assert e.value.code == tkc.TKC_EINVAL
    rp = g.row_ptr.copy()
    rp[7], rp[8] = rp[8], rp[7]
    with pytest.raises(tkc.TkcError) as e:
        tkc.Graph(ctx, g.n, rp, g.col_idx)
    assert e.value.code == tkc.TKC_EINVAL
    with pytest.raises(tkc.TkcError) as e:
        tkc.tkc_graph_upload(ctx.h, g.n, g.arcs - 1, g.row_ptr, g.col_idx, None, None, 0)
    assert e.value.code == tkc.TKC_EINVAL
    for nn, mm in ((0, 0), (g.n, -1), (g.n, 1 << 31)):
        with pytest.raises(tkc.TkcError) as e:
            tkc.tkc_graph_upload(ctx.h, nn, mm, g.row_ptr, g.col_idx, None, None, 0)
        assert e.value.code == tkc.TKC_EINVAL
    d = graph("gnp_d")
    badr = d.rcol_idx.copy()
    badr[0] = d.n + 3
    with pytest.raises(tkc.TkcError) as e:
        tkc.Graph(ctx, d.n, d.row_ptr, d.col_idx, d.rrow_ptr, badr)
    assert e.value.code == tkc.TKC_EINVAL


def test_device_pointer_upload(ctx):
    import torch
    g = graph("gnp_d")
    t = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col_idx, g.rrow_ptr, g.rcol_idx)]
    torch.cuda.synchronize()
    dg = tkc.Graph(ctx, g.n, *t, validate=True, device_ptrs=True)
    ids, S, r, f, st = tkc.topk_closeness(dg, 10, "nbcut", "hybrid")
    wids, wS, wr, wf = expect("gnp_d", 10)
    assert np.array_equal(ids, wids) and np.array_equal(S, wS)
    dg.free()
    # from_csr: device tensors are detected, host tensors and arrays copied
    for arrs in (t, [x.cpu() for x in t], [g.row_ptr, g.col_idx, g.rrow_ptr, g.rcol_idx]):
        dg = tkc.Graph.from_csr(ctx, *arrs, validate=True)
        ids, S, r, f, st = tkc.topk_closeness(dg, 10, "nbcut", "batched")
        assert np.array_equal(ids, wids) and np.array_equal(S, wS)
        dg.free()


def test_repeatable(ctx):
    """Two runs give identical results and identical work counts."""
    dg = upload(ctx, "ba20k")
    a = tkc.topk_closeness(dg, 10, "nbcut", "batched")
    b = tkc.topk_closeness(dg, 10, "nbcut", "batched")
    assert np.array_equal(a[0], b[0]) and a[4]["m_vis"] == b[4]["m_vis"]
