"""Pins of the oracle against closed forms (Sect. 2, Eq. 1; Sect. 3 reduction).

Each expected value below is derived from the definition of S(v), r(v)
(Table 1) on a graph whose distances are known in closed form, not from the
oracle's own code.
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle


def farn(n, S, r):
    """Exact farness as a Fraction, None for +inf (Eq. 1, r = 1 rule)."""
    return None if r <= 1 else Fraction((n - 1) * S, (r - 1) ** 2)


def path_edges(n):
    return np.array([(i, i + 1) for i in range(n - 1)], dtype=np.int32).reshape(-1, 2)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 10, 33])
def test_path(n):
    S, r = oracle.sums(n, path_edges(n), False)
    for i in range(n):
        assert S[i] == i * (i + 1) // 2 + (n - 1 - i) * (n - i) // 2
        assert r[i] == n


@pytest.mark.parametrize("n", [3, 4, 5, 8, 9, 20, 21])
def test_cycle(n):
    e = np.array([(i, (i + 1) % n) for i in range(n)], dtype=np.int32)
    S, r = oracle.sums(n, e, False)
    want = (n * n - 1) // 4 if n % 2 else n * n // 4
    assert (S == want).all() and (r == n).all()


@pytest.mark.parametrize("n", [2, 3, 6, 50])
def test_star(n):
    e = np.array([(0, i) for i in range(1, n)], dtype=np.int32)
    S, r = oracle.sums(n, e, False)
    assert S[0] == n - 1
    assert all(S[i] == 2 * n - 3 for i in range(1, n))
    ids = oracle.topk(S, r, 3)
    assert ids[0] == 0 and list(ids[1:]) == list(range(1, min(3, n)))


@pytest.mark.parametrize("n", [2, 5, 12])
def test_complete(n):
    e = np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.int32)
    S, r = oracle.sums(n, e, False)
    assert (S == n - 1).all() and (r == n).all()
    # every vertex ties: the k smallest ids win
    assert list(oracle.topk(S, r, 4)) == list(range(min(4, n)))


@pytest.mark.parametrize("a,b", [(1, 5), (2, 2), (3, 7), (6, 6), (9, 4)])
def test_grid(a, b):
    e = []
    for i in range(a):
        for j in range(b):
            u = i * b + j
            if j + 1 < b:
                e.append((u, u + 1))
            if i + 1 < a:
                e.append((u, u + b))
    n = a * b
    S, r = oracle.sums(n, np.array(e, dtype=np.int32).reshape(-1, 2), False)
    for i in range(a):
        for j in range(b):
            want = b * (i * (i + 1) // 2 + (a - 1 - i) * (a - i) // 2) + \
                a * (j * (j + 1) // 2 + (b - 1 - j) * (b - j) // 2)
            assert S[i * b + j] == want


@pytest.mark.parametrize("n", [2, 3, 8, 15])
def test_directed_path_reachable_set(n):
    """0 -> 1 -> ... -> n-1: vertex i reaches m = n-1-i others at 1..m, so
    f = (n-1)(m+1)/(2m); the last vertex reaches nothing (f = +inf)."""
    S, r = oracle.sums(n, path_edges(n), True)
    for i in range(n):
        m = n - 1 - i
        assert r[i] == m + 1 and S[i] == m * (m + 1) // 2
        f = oracle.farness(n, S[i], r[i])
        if m == 0:
            assert f == float("inf")
        else:
            assert f == pytest.approx((n - 1) * (m + 1) / (2 * m), rel=1e-15)
    # most central: vertex 0 (largest m gives the smallest (m+1)/(2m))
    ids = oracle.topk(S, r, n)
    assert list(ids) == list(range(n))


def test_disjoint_union_with_isolated_vertices():
    """P_4 on 0..3, K_3 on 4..6, isolated 7 and 8: r = component size."""
    e = [(0, 1), (1, 2), (2, 3), (4, 5), (5, 6), (4, 6)]
    n = 9
    S, r = oracle.sums(n, np.array(e, dtype=np.int32), False)
    assert list(r) == [4, 4, 4, 4, 3, 3, 3, 1, 1]
    assert list(S) == [6, 4, 4, 6, 2, 2, 2, 0, 0]
    # f(K3 vertex) = 8*2/4 = 4; f(P4 centre) = 8*4/9 < 4; f(P4 end) = 8*6/9
    ids = oracle.topk(S, r, 9)
    assert list(ids) == [1, 2, 4, 5, 6, 0, 3, 7, 8]
    assert oracle.farness(n, 0, 1) == float("inf")


def test_exact_ties_with_different_S_and_r():
    """Exact ties S/(r-1)^2 = 1/2 from (S, r) = (2, 3) and (8, 5), and 1/3 from
    (3, 4) and (12, 7): the smaller id wins, never a floating-point order."""
    e = [(0, 1), (0, 2),                          # 0: S=2, r=3
         (3, 4), (4, 5), (4, 6), (5, 7),          # 3: S=8, r=5
         (8, 9), (8, 10), (8, 11),                # 8: S=3, r=4
         (12, 13), (12, 14), (13, 15), (14, 16), (15, 17), (16, 18)]  # 12: S=12, r=7
    n = 19
    S, r = oracle.sums(n, np.array(e, dtype=np.int32), True)
    assert (S[0], r[0], S[3], r[3]) == (2, 3, 8, 5)
    assert (S[8], r[8], S[12], r[12]) == (3, 4, 12, 7)
    assert oracle.cmp(S[0], r[0], S[3], r[3]) == 0
    assert oracle.cmp(S[8], r[8], S[12], r[12]) == 0
    ids = list(oracle.topk(S, r, n))
    assert ids.index(0) + 1 == ids.index(3)
    assert ids.index(8) + 1 == ids.index(12)
    # the full order matches an exact Fraction sort
    key = [(farn(n, S[v], r[v]) is None, farn(n, S[v], r[v]) or 0, v) for v in range(n)]
    assert ids == [v for _, _, v in sorted(key)]


def test_reduction_graph_closed_forms():
    """Sect. 3: closeness of every vertex class of the reduction graph with
    p = 7, q = 36 (g(p) = 35), on the family X = {0,1,2,3},
    sets {0}, {0,1}, {2}, {1,2,3}, {3}."""
    sets = [{0}, {0, 1}, {2}, {1, 2, 3}, {3}]
    X = 4
    p, q = 7, 36
    n, e, cls = graphgen.reduction_graph(sets, X, p, q)
    C = len(sets)
    assert n == q * C + q + C + 2 * X + p * C
    S, r = oracle.sums(n, e, True)
    g = (p + 1) * (p + 2) // 2 - 1
    assert g == 35

    def clos(v):
        return Fraction(0) if r[v] <= 1 else Fraction((r[v] - 1) ** 2, (n - 1) * S[v])
    for ci, s in enumerate(sets):
        R = sum(1 for t in sets if s & t)
        want = Fraction((q * (1 + C) + X + p * R) ** 2, (q * (1 + 2 * C) + X + g * R) * (n - 1))
        assert clos(cls["C0"][ci]) == want
    for y in cls["Y"]:
        assert clos(y) == Fraction(C, n - 1)
    for i in range(1, p + 1):
        for v in cls["C%d" % i]:
            want = Fraction(2 * (p - i), (n - 1) * (p - i + 1)) if i < p else Fraction(0)
            assert clos(v) == want
    for x in range(X):
        Nx = sum(1 for t in sets if x in t)
        want = Fraction(2 * p * Nx, (n - 1) * (p + 1)) if Nx else Fraction(0)
        assert clos(cls["X1"][x]) == want
    for v in cls["Z"] + cls["X2"]:
        assert clos(v) == 0
    # the most central vertex is the C0 vertex with the smallest R_C
    S64, r64 = S.astype(np.int64), r.astype(np.int64)
    top = oracle.topk(S64, r64, 1)[0]
    Rc = [sum(1 for t in sets if s & t) for s in sets]
    assert top == cls["C0"][int(np.argmin(Rc))]


def test_farness_double_formula():
    n = 1000
    for S, r in [(999, 1000), (12345, 777), (2, 3), (10 ** 10, 4 * 10 ** 6)]:
        want = (float(n - 1) * float(S)) / (float(r - 1) * float(r - 1))
        assert oracle.farness(n, S, r) == want
    assert oracle.farness(n, 0, 1) == float("inf")
