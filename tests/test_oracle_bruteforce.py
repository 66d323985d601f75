"""Pins of the oracle against brute force: Floyd-Warshall distances and an
exact Fraction sort on tiny random graphs (directed and undirected, from
sparse and disconnected to dense)."""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen
import oracle


def brute(n, edges, directed):
    d = oracle.floyd_warshall(n, edges, directed)
    S = np.where(d >= 0, d, 0).sum(axis=1).astype(np.int64)
    r = (d >= 0).sum(axis=1).astype(np.int64)
    return S, r


def brute_order(n, S, r):
    key = []
    for v in range(n):
        if r[v] <= 1:
            key.append((1, Fraction(0), v))
        else:
            key.append((0, Fraction(int(S[v]), int(r[v] - 1) ** 2), v))
    return [v for _, _, v in sorted(key)]


@pytest.mark.parametrize("directed", [False, True])
def test_floyd_warshall_many(directed):
    count = 0
    for seed in range(600):
        n = 1 + seed % 40
        p = [0.02, 0.05, 0.1, 0.2, 0.5][seed % 5]
        e = graphgen.gnp(n, p, directed, 1000 + seed)
        S, r = oracle.sums(n, e, directed)
        S2, r2 = brute(n, e, directed)
        assert (S == S2).all() and (r == r2).all(), (seed, n, p)
        assert list(oracle.topk(S, r, n)) == brute_order(n, S2, r2)
        count += 1
    assert count == 600


@settings(max_examples=200, deadline=None)
@given(st.integers(1, 24), st.lists(st.tuples(st.integers(0, 23), st.integers(0, 23)), max_size=80),
       st.booleans(), st.integers(1, 30))
def test_hypothesis_edge_lists(n, pairs, directed, k):
    """Arbitrary edge lists with repeats and self-loops."""
    e = np.array([(a % n, b % n) for a, b in pairs], dtype=np.int32).reshape(-1, 2)
    S, r = oracle.sums(n, e, directed)
    S2, r2 = brute(n, e, directed)
    assert (S == S2).all() and (r == r2).all()
    want = brute_order(n, S2, r2)[: min(k, n)]
    assert list(oracle.topk(S, r, k)) == want


def test_sources_subset_matches_all():
    e = graphgen.gnp(60, 0.05, True, 7)
    S, r = oracle.sums(60, e, True)
    src = np.array([5, 0, 59, 5, 17], dtype=np.int32)
    S2, r2 = oracle.sums(60, e, True, sources=src)
    assert (S2 == S[src]).all() and (r2 == r[src]).all()


def test_topk_edge_cases():
    assert list(oracle.topk(np.zeros(0, np.int64), np.zeros(0, np.int64), 5)) == []
    S = np.array([0], np.int64)
    r = np.array([1], np.int64)
    assert list(oracle.topk(S, r, 3)) == [0]
    assert list(oracle.topk(S, r, 0)) == []


@pytest.mark.parametrize("directed", [False, True])
def test_closeness_topk_against_brute(directed):
    """The oracle's whole answer (ids, S, r and the farness doubles) against
    Floyd-Warshall: each returned double belongs to its own vertex and lies
    within a few ulps of the exact rational (n-1) S / (r-1)^2 (the binary64
    formula rounds three times: two products and the quotient)."""
    for seed in range(120):
        n = 2 + seed % 30
        e = graphgen.gnp(n, [0.05, 0.1, 0.3][seed % 3], directed, 77000 + seed)
        S2, r2 = brute(n, e, directed)
        want = brute_order(n, S2, r2)
        for k in (1, 5, n):
            ids, S, r, far = oracle.closeness_topk(n, e, directed, k)
            assert list(ids) == want[:k], (seed, k)
            assert (S == S2[ids]).all() and (r == r2[ids]).all()
            for v, f in zip(ids, far):
                if r2[v] <= 1:
                    assert f == float("inf")
                    continue
                exact = Fraction((n - 1) * int(S2[v]), int(r2[v] - 1) ** 2)
                assert abs(Fraction(f) - exact) <= 4 * 2.0 ** -52 * exact, (seed, v, f)
