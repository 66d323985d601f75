"""Top-k parity against the oracle's full answer, element by element.

tests/golden/full_<name>.txt holds the exact top-100 of a workload, written
by tests/golden/make_full.py from the oracle's all-sources textbook search
(Sect. 1) and the exact order of Lin's index (Sect. 2, Eq. 1; the smaller
id wins a tie).  Alg. 1 reaches exactly that answer (Sect. 4), so for
k = 1, 10 and 100 the device's (id, S, r) must equal the file's first k rows
and each farness double must follow from (S, r) by the fixed formula.

Medium graphs (BA 2^17, R-MAT scale 16, grid 500^2) run every variant and
engine, and harmonic centrality (full_<name>_harmonic.txt, bit for bit).
They hold hubs of in-degree above 1024 (the batched pull's hub chunks), walk
counts beyond 2^31 (the NB rounds' capped 32-bit copy) and NB tail rounds.
The full-size workloads (BA 2^20, R-MAT scale 20) run in the configurations
bench.py times.  Each file's graph digest is checked first.
"""
import functools
import os

import numpy as np
import pytest

import graphgen
import oracle
from conftest import hip_available

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

if hip_available():
    from paper_1704_01077_amd import tkc
else:
    tkc = None


def load(name, harmonic=False):
    path = os.path.join(GOLDEN, "full_%s%s.txt" % (name, "_harmonic" if harmonic else ""))
    if not os.path.exists(path):
        pytest.skip("no oracle answer stored for %s" % name)
    meta, rows = {}, []
    with open(path) as fp:
        for line in fp:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0].isdigit():
                rows.append(t[1:])
            else:
                meta[t[0]] = t[1]
    return meta, rows


@functools.lru_cache(maxsize=None)
def workload(name):
    return graphgen.workload(name)


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


def dev(ctx, name, relabel=False):
    if (name, relabel) not in _DEV:
        g = workload(name)
        meta, _ = load(name)
        assert meta["digest"] == g.digest(), "the stored answer is for another graph"
        _DEV[(name, relabel)] = tkc.Graph.from_graphgen(ctx, g, relabel=relabel)
    return _DEV[(name, relabel)]


def expect(name, k):
    meta, rows = load(name)
    kk = min(k, int(meta["n"]))
    ids = np.array([int(r[0]) for r in rows[:kk]], np.int32)
    S = np.array([int(r[1]) for r in rows[:kk]], np.int64)
    R = np.array([int(r[2]) for r in rows[:kk]], np.int64)
    return ids, S, R


def check(name, k, ids, S, r, f):
    wi, wS, wr = expect(name, k)
    assert np.array_equal(ids, wi), (name, k, ids[:8], wi[:8])
    assert np.array_equal(S, wS) and np.array_equal(r, wr)
    n = workload(name).n
    for i in range(len(ids)):
        assert f[i] == oracle.farness(n, S[i], r[i])


MEDIUM = ["ba128k", "rmat16", "grid500"]
VARIANTS = ["auto", "degcut", "nbcut", "degbound", "nbbound", "nbcutlb"]


@pytest.mark.parametrize("name", MEDIUM)
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("mode", ["batched", "hybrid"])
def test_medium_topk(ctx, name, variant, mode):
    dg = dev(ctx, name)
    for k in (1, 10, 100):
        ids, S, r, f, _ = tkc.topk_closeness(dg, k, variant, mode)
        check(name, k, ids, S, r, f)


@pytest.mark.parametrize("name", ["ba128k", "rmat16"])
@pytest.mark.parametrize("variant", ["degcut", "nbcut"])
def test_medium_topk_plain(ctx, name, variant):
    dg = dev(ctx, name)
    for k in (1, 10, 100):
        ids, S, r, f, _ = tkc.topk_closeness(dg, k, variant, "plain")
        check(name, k, ids, S, r, f)


@pytest.mark.parametrize("name", MEDIUM)
@pytest.mark.parametrize("width", [32, 128, 256])
def test_medium_topk_widths(ctx, name, width):
    dg = dev(ctx, name)
    keep = ctx.tuning()
    try:
        ctx.tune(batch_width=width)
        for k in (10, 100):
            ids, S, r, f, _ = tkc.topk_closeness(dg, k, "nbcut", "batched")
            check(name, k, ids, S, r, f)
    finally:
        ctx.tune(**keep)


@pytest.mark.parametrize("name", MEDIUM)
@pytest.mark.parametrize("variant", ["auto", "nbcut", "nbbound"])
def test_medium_harmonic(ctx, name, variant):
    meta, rows = load(name, harmonic=True)
    assert meta["digest"] == workload(name).digest()
    dg = dev(ctx, name)
    for k in (1, 10, 100):
        ids, h, _ = tkc.topk_harmonic(dg, k, variant, "batched")
        kk = min(k, len(rows))
        want_ids = np.array([int(r[0]) for r in rows[:kk]], np.int32)
        want_h = np.array([float.fromhex(r[1]) for r in rows[:kk]], np.float64)
        assert np.array_equal(ids, want_ids), (name, variant, k)
        assert np.array_equal(h.view(np.uint64), want_h.view(np.uint64))


# full size, in the configurations bench.py times: BA 2^20 in hybrid mode
# with the default knobs, R-MAT scale 20 batched at W = 256 and four
# workgroups per CU
@pytest.mark.parametrize("k", [1, 10, 100])
def test_full_ba1m_exact(ctx, k):
    dg = dev(ctx, "ba1m")
    ids, S, r, f, _ = tkc.topk_closeness(dg, k, "auto", "hybrid")
    check("ba1m", k, ids, S, r, f)


@pytest.mark.parametrize("k", [1, 10, 100])
def test_full_rmat20_exact(ctx, k):
    dg = dev(ctx, "rmat20")
    keep = ctx.tuning()
    try:
        ctx.tune(batch_width=256, blocks_per_cu=4)
        ids, S, r, f, _ = tkc.topk_closeness(dg, k, "auto", "batched")
        check("rmat20", k, ids, S, r, f)
    finally:
        ctx.tune(**keep)


# graphs uploaded with TKC_RELABEL answer in the caller's ids: the medium
# tier in every engine, and R-MAT scale 20 in bench.py's C3 configuration.
# (A degree order scatters a grid's neighbours, so the one-source-at-a-time
# engine on the relabelled grid is left out: each of its ~1,000-level
# searches then takes far longer, and grids are not what relabelling is for.)
@pytest.mark.parametrize("name,mode", [(nm, md) for nm in MEDIUM for md in ("plain", "batched", "hybrid")
                                       if not (nm == "grid500" and md == "plain")])
@pytest.mark.parametrize("variant", ["auto", "nbcut", "nbbound", "nbcutlb"])
def test_medium_topk_relabel(ctx, name, variant, mode):
    dg = dev(ctx, name, relabel=True)
    for k in (1, 10, 100):
        ids, S, r, f, _ = tkc.topk_closeness(dg, k, variant, mode)
        check(name, k, ids, S, r, f)


@pytest.mark.parametrize("k", [1, 10, 100])
def test_full_rmat20_relabel_exact(ctx, k):
    dg = dev(ctx, "rmat20", relabel=True)
    keep = ctx.tuning()
    try:
        ctx.tune(batch_width=256, blocks_per_cu=4)
        ids, S, r, f, _ = tkc.topk_closeness(dg, k, "auto", "batched")
        check("rmat20", k, ids, S, r, f)
    finally:
        ctx.tune(**keep)
