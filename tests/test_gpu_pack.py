"""Packed requests: top-k queries on several graphs in one batched launch.

A pack is the disjoint union of member graphs; the requests of one call
share the lanes of one cooperative launch, each with its own order, bounds
and k-th farness.  Every request's answer must equal the oracle's exact
top k on its own member (and the same query run alone), element by element,
whatever the mix of requests, their k and the batch width.
"""
import numpy as np
import pytest

from conftest import hip_available
from test_gpu_parity import expect, graph, upload

pytestmark = pytest.mark.gpu

if hip_available():
    from paper_1704_01077_amd import tkc
else:
    tkc = None

UNDIRECTED = ["ba2k", "ba3k_m2", "grid60", "king40", "gnp_u", "forest", "cycle", "complete", "star", "ba_path"]
DIRECTED = ["rmat11", "gnp_d", "dpath"]


@pytest.fixture(scope="module")
def ctx():
    if not hip_available():
        pytest.skip("no GPU")
    import torch
    torch.cuda.init()
    c = tkc.Context(0)
    yield c
    c.close()


def check(names, members, ks, res):
    for (ids, S, r, f), m, k in zip(res, members, ks):
        want = expect(names[m], k)
        assert np.array_equal(ids, want[0]), (names[m], k, ids[:5], want[0][:5])
        assert np.array_equal(S, want[1]) and np.array_equal(r, want[2])
        assert np.array_equal(f, want[3])


@pytest.mark.parametrize("names", [UNDIRECTED, DIRECTED], ids=["undirected", "directed"])
@pytest.mark.parametrize("variant", ["nbcut", "degcut"])
def test_pack_all_members(ctx, names, variant):
    p = tkc.Pack(ctx, [upload(ctx, x) for x in names])
    try:
        for k in (1, 10, 100):
            members = list(range(len(names)))
            res, st = p.topk(members, [k] * len(names), variant)
            check(names, members, [k] * len(names), res)
        # mixed k, a subset, in another order; twice in a row
        members = list(range(len(names)))[::-2]
        ks = [(1, 10, 100, 3)[i % 4] for i in range(len(members))]
        for _ in range(2):
            res, st = p.topk(members, ks, variant)
            check(names, members, ks, res)
    finally:
        p.close()


@pytest.mark.parametrize("width", [32, 128, 256])
def test_pack_widths(ctx, width):
    names = UNDIRECTED
    p = tkc.Pack(ctx, [upload(ctx, x) for x in names])
    keep = ctx.tuning()
    try:
        ctx.tune(batch_width=width)
        members = list(range(len(names)))
        ks = [10] * len(names)
        res, _ = p.topk(members, ks, "nbcut")
        check(names, members, ks, res)
    finally:
        ctx.tune(**keep)
        p.close()


def test_pack_equals_solo(ctx):
    """The packed answer of each request is the same query run alone."""
    names = ["ba2k", "grid60", "king40"]
    dgs = [upload(ctx, x) for x in names]
    p = tkc.Pack(ctx, dgs)
    try:
        res, _ = p.topk([0, 1, 2], [10, 10, 10], "nbcut")
        for (ids, S, r, f), dg in zip(res, dgs):
            ids2, S2, r2, f2, _ = tkc.topk_closeness(dg, 10, "nbcut", "batched")
            assert np.array_equal(ids, ids2) and np.array_equal(S, S2) and np.array_equal(r, r2)
    finally:
        p.close()


def test_pack_errors(ctx):
    p = tkc.Pack(ctx, [upload(ctx, "ba2k"), upload(ctx, "grid60")])
    try:
        with pytest.raises(tkc.TkcError) as e:
            p.topk([0, 0], [10, 10])          # two requests on one member
        assert e.value.code == tkc.TKC_EINVAL
        with pytest.raises(tkc.TkcError) as e:
            p.topk([0], [10], "nbbound")      # level-based variants run alone
        assert e.value.code == tkc.TKC_EINVAL
        with pytest.raises(tkc.TkcError) as e:
            tkc.tkc_graph_free(upload(ctx, "grid60").h)   # held by the pack
        assert e.value.code == tkc.TKC_EBUSY
    finally:
        p.close()
    with pytest.raises(tkc.TkcError) as e:
        tkc.Pack(ctx, [upload(ctx, "ba2k"), upload(ctx, "rmat11")])   # mixed directedness
    assert e.value.code == tkc.TKC_EINVAL
