"""Top-k harmonic centrality on the GPU (Sect. 2 with f(d) = 1/d, ranked in
Sect. 9.1) against the oracle.

The library and the oracle evaluate h in the same binary64 reading (terms
n_d / d added in increasing d), so ids and values are compared bit for bit.
The upper bounds the searches start from are compared with the oracle's
bounds (raised by the same 1e-9 margin), and the full-size runs are checked
on the outputs the oracle can compute one by one: every returned value, the
order, and sampled outsiders.
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

MARGIN = 1.0 + 1e-9


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
    if name == "ba2k":
        return graphgen.workload("ba2k")
    if name == "ba20k":
        return graphgen.ba_graph(20000, 5, 7)
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
    if name == "gnp_u":
        return _g(name, 700, graphgen.gnp(700, 0.002, False, 21), False)
    if name == "gnp_d":
        return _g(name, 600, graphgen.gnp(600, 0.004, True, 22), True)
    if name == "forest":
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
    if name == "single":
        return _g(name, 1, np.zeros((0, 2), np.int32), False)
    if name == "edgeless":
        return _g(name, 50, np.zeros((0, 2), np.int32), False)
    if name == "sinks":
        return _g(name, 40, np.zeros((0, 2), np.int32), True)
    if name in ("ba1m", "rmat20", "grid2000"):
        return graphgen.workload(name)
    raise KeyError(name)


SMALL = ["ba2k", "ba_path", "grid60", "king40", "rmat11", "gnp_u", "gnp_d", "forest", "cycle", "complete", "star",
         "dpath", "single", "edgeless", "sinks"]
_DEV = {}


def dev(ctx, name):
    if name not in _DEV:
        _DEV[name] = tkc.Graph.from_graphgen(ctx, graph(name), validate=name not in ("ba1m", "rmat20", "grid2000"))
    return _DEV[name]


@functools.lru_cache(maxsize=None)
def truth(name):
    g = graph(name)
    return oracle.harmonic(g.n, g.edges, g.directed)


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("variant", ["degcut", "nbcut", "degbound", "nbbound", "degcutlb", "nbcutlb", "auto"])
@pytest.mark.parametrize("mode", ["plain", "batched", "hybrid"])
@pytest.mark.parametrize("k", [1, 10, 100])
def test_harmonic_topk_parity(ctx, name, variant, mode, k):
    g = graph(name)
    h = truth(name)
    ids, hv, st = tkc.topk_harmonic(dev(ctx, name), k, variant, mode)
    want = oracle.harmonic_topk(h, k)
    assert np.array_equal(ids, want), (ids[:10], want[:10])
    assert np.array_equal(hv, h[want])
    assert st["bfs_exact"] >= min(k, g.n) or st["bfs_exact"] + st["skipped"] >= 0


@pytest.mark.parametrize("name", ["ba20k", "grid150", "rmat13", "king40"])
@pytest.mark.parametrize("variant", ["degcut", "nbcut", "nbbound", "nbcutlb"])
@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_harmonic_topk_medium(ctx, name, variant, mode):
    h = truth(name)
    for k in (1, 10, 100):
        ids, hv, st = tkc.topk_harmonic(dev(ctx, name), k, variant, mode)
        want = oracle.harmonic_topk(h, k)
        assert np.array_equal(ids, want) and np.array_equal(hv, h[want])


@pytest.mark.parametrize("width", [32, 128, 256])
def test_harmonic_batch_widths(ctx, width):
    keep = ctx.tuning()
    ctx.tune(batch_width=width)
    try:
        for name in ("ba2k", "gnp_d", "rmat11"):
            h = truth(name)
            ids, hv, st = tkc.topk_harmonic(dev(ctx, name), 10, "nbcut", "batched")
            want = oracle.harmonic_topk(h, 10)
            assert np.array_equal(ids, want) and np.array_equal(hv, h[want])
    finally:
        ctx.tune(**keep)


@pytest.mark.parametrize("name", ["ba2k", "ba_path", "grid60", "gnp_u", "gnp_d", "forest", "rmat11", "dpath",
                                  "star", "sinks"])
def test_harmonic_bounds_parity(ctx, name):
    """Walk-count bounds bit for bit (the same terms in the same order as the
    oracle's), degree bounds likewise, both above h, and the order."""
    g = graph(name)
    h = truth(name)
    dg = dev(ctx, name)
    for variant, ref in (("nbcut", oracle.nb_harmonic), ("degcut", oracle.deg_harmonic)):
        ub, order = dg.harmonic_bounds(variant)
        want = ref(g.n, g.edges, g.directed) * MARGIN
        assert np.array_equal(ub, want), (variant, np.flatnonzero(ub != want)[:5])
        assert np.all(ub >= h)
        # order: 32-bit keys (the complement of the top half of the bound's
        # bit pattern) ascending, ties by id: the largest bound first, up to
        # the keys' 2^-20 relative resolution
        key = ~(ub.view(np.uint64) >> np.uint64(32)).astype(np.uint32)
        assert np.array_equal(order, np.lexsort((np.arange(g.n), key)).astype(np.int32))
        assert np.all(np.diff(ub[order]) <= ub[order][:-1] * 2.0 ** -19)


def test_harmonic_rejects_unknown_variant(ctx):
    dg = dev(ctx, "ba2k")
    with pytest.raises(tkc.TkcError) as e:
        tkc.topk_harmonic(dg, 10, 7, "batched")
    assert e.value.code == tkc.TKC_EINVAL


@pytest.mark.parametrize("name", ["ba2k", "gnp_u", "forest", "grid60", "gnp_d", "rmat11", "dpath", "star"])
def test_harmonic_lb_update_parity(ctx, name):
    """The level-based update of a few complete searches, bit for bit: the
    least of the old bound and the oracle's bounds (raised by the margin)."""
    g = graph(name)
    dg = dev(ctx, name)
    ub0, _ = dg.harmonic_bounds("nbcut")
    rng = np.random.default_rng(3)
    src = np.unique(rng.integers(0, g.n, size=5)).astype(np.int32)
    got = dg.harmonic_lb_update(src, ub0)
    scc = oracle.scc(g.n, g.edges)[1] if g.directed else None
    want = ub0.copy()
    for s_ in src.tolist():
        _, b = oracle.lb_harmonic(g.n, g.edges, g.directed, s_, scc)
        ok = b >= 0
        want[ok] = np.minimum(want[ok], b[ok] * MARGIN)
    assert np.array_equal(got, want), np.flatnonzero(got != want)[:5]
    assert np.all(got >= truth(name))


def test_harmonic_and_closeness_interleave(ctx):
    """A harmonic query between closeness queries leaves both exact."""
    name = "rmat11"
    g = graph(name)
    dg = dev(ctx, name)
    S, r = oracle.sums(g.n, g.edges, g.directed)
    cw = oracle.topk(S, r, 10)
    for _ in range(2):
        ids, S1, r1, f1, _ = tkc.topk_closeness(dg, 10, "nbcut", "hybrid")
        assert np.array_equal(ids, cw)
        hid, hv, _ = tkc.topk_harmonic(dg, 10, "nbcut", "batched")
        assert np.array_equal(hid, oracle.harmonic_topk(truth(name), 10))


# full size: every returned value from the oracle one source at a time, the
# order, and sampled outsiders (random plus the highest-degree vertices)
@pytest.mark.parametrize("name", ["ba1m", "rmat20", "grid2000"])
def test_harmonic_full(ctx, name):
    g = graph(name)
    dg = dev(ctx, name)
    ids, hv, st = tkc.topk_harmonic(dg, 10, "auto", "batched")
    assert len(ids) == 10 and len(set(ids.tolist())) == 10
    assert np.array_equal(hv, oracle.harmonic(g.n, g.edges, g.directed, sources=ids))
    for i in range(1, 10):
        assert hv[i - 1] > hv[i] or (hv[i - 1] == hv[i] and ids[i - 1] < ids[i])
    rng = np.random.default_rng(31)
    pick = set(rng.integers(0, g.n, size=256).tolist())
    deg = np.diff(g.row_ptr)
    pick |= set(np.argsort(-deg, kind="stable")[:64].tolist())
    pick -= set(ids.tolist())
    out = np.array(sorted(pick), np.int32)
    ho = oracle.harmonic(g.n, g.edges, g.directed, sources=out)
    for v, x in zip(out.tolist(), ho.tolist()):
        assert x < hv[-1] or (x == hv[-1] and v > ids[-1]), (v, x)
    if name == "grid2000":
        assert st["variant_used"] == tkc.TKC_NB_BOUND
        return
    ids2, hv2, _ = tkc.topk_harmonic(dg, 10, "nbcut", "plain")
    assert np.array_equal(ids2, ids) and np.array_equal(hv2, hv)
    ids3, hv3, _ = tkc.topk_harmonic(dg, 10, "degcut", "batched")
    assert np.array_equal(ids3, ids) and np.array_equal(hv3, hv)
    ids4, hv4, st4 = tkc.topk_harmonic(dg, 10, "nbcut", "hybrid")
    assert np.array_equal(ids4, ids) and np.array_equal(hv4, hv)
    assert st4["mode_used"] == tkc.TKC_HYBRID
