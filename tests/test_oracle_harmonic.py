"""Pins of the oracle's harmonic centrality (Sect. 2 with f(d) = 1/d, the
measure Sect. 9.1 also ranks).

The expected values come from closed forms on graphs whose distances are
known, and from Floyd-Warshall distances on tiny random graphs, never from
the oracle's own code.  Two bars:
  - the exact rational value (Fractions), within the rounding that a sum of
    ecc(v) binary64 terms allows;
  - bit for bit, the binary64 reading the library and the oracle share: the
    terms n_d / d added in increasing d, with the level counts n_d taken
    from Floyd-Warshall distances.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def H(m):
    """Harmonic number H_m as a Fraction."""
    return sum((Fraction(1, j) for j in range(1, m + 1)), Fraction(0))


def close(got, want, terms):
    """|got - want| within terms+1 units of 2^-52 relative (want a Fraction)."""
    w = float(want)
    return abs(got - w) <= (terms + 1) * 2.0 ** -52 * max(abs(w), 1e-300)


def E(pairs):
    return np.array(pairs, dtype=np.int32).reshape(-1, 2)


@pytest.mark.parametrize("n", [1, 2, 3, 6, 17, 40])
def test_complete_graph(n):
    e = E([(i, j) for i in range(n) for j in range(i + 1, n)])
    h = oracle.harmonic(n, e, False)
    assert np.all(h == float(n - 1))


@pytest.mark.parametrize("n", [2, 3, 5, 12, 101])
def test_star(n):
    h = oracle.harmonic(n, E([(0, i) for i in range(1, n)]), False)
    assert h[0] == float(n - 1)
    for i in range(1, n):
        assert close(h[i], 1 + Fraction(n - 2, 2), 2)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 30, 257])
def test_path(n):
    h = oracle.harmonic(n, E([(i, i + 1) for i in range(n - 1)]), False)
    for i in range(n):
        assert close(h[i], H(i) + H(n - 1 - i), n)


@pytest.mark.parametrize("n", [2, 5, 64])
def test_directed_path(n):
    h = oracle.harmonic(n, E([(i, i + 1) for i in range(n - 1)]), True)
    for i in range(n):
        assert close(h[i], H(n - 1 - i), n)
    assert h[n - 1] == 0.0


@pytest.mark.parametrize("n", [3, 4, 7, 10, 31, 64])
def test_cycle(n):
    h = oracle.harmonic(n, E([(i, (i + 1) % n) for i in range(n)]), False)
    m = n // 2
    want = 2 * H(m) if n % 2 else 2 * H(m - 1) + Fraction(1, m)
    assert np.all([close(x, want, n) for x in h])
    # a directed cycle: every vertex sees 1, 2, ..., n-1 once
    hd = oracle.harmonic(n, E([(i, (i + 1) % n) for i in range(n)]), True)
    assert np.all([close(x, H(n - 1), n) for x in hd])


def test_edgeless_and_isolated():
    h = oracle.harmonic(6, E([(0, 1)]), False)
    assert list(h) == [1.0, 1.0, 0.0, 0.0, 0.0, 0.0]
    assert list(oracle.harmonic(4, np.zeros((0, 2), np.int32), True)) == [0.0] * 4


def fw_levels(n, edges, directed):
    """Level counts per source from Floyd-Warshall distances."""
    d = oracle.floyd_warshall(n, edges, directed)
    out = []
    for v in range(n):
        row = d[v]
        lv = {}
        for w in range(n):
            if w != v and row[w] >= 0:
                lv[int(row[w])] = lv.get(int(row[w]), 0) + 1
        out.append(lv)
    return out


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_tiny(directed, seed):
    rng = np.random.default_rng(900 + seed + (1000 if directed else 0))
    n = int(rng.integers(1, 16))
    p = float(rng.uniform(0.05, 0.5))
    pairs = set()
    for u in range(n):
        for w in range(n):
            if u != w and rng.random() < p and (directed or u < w):
                pairs.add((u, w))
    e = E(sorted(pairs))
    h = oracle.harmonic(n, e, directed)
    for v, lv in enumerate(fw_levels(n, e, directed)):
        exact = sum((Fraction(c, d) for d, c in lv.items()), Fraction(0))
        assert close(h[v], exact, len(lv))
        # the binary64 reading, bit for bit
        x = 0.0
        for d in sorted(lv):
            x += float(lv[d]) / float(d)
        assert h[v] == x, (v, h[v], x)
    # the order: larger first, ties to the smaller id, against a plain sort
    want = sorted(range(n), key=lambda v: (-h[v], v))
    for k in (1, 3, n, n + 2):
        assert list(oracle.harmonic_topk(h, k)) == want[:k]


def test_sources_subset_matches_all():
    rng = np.random.default_rng(5)
    n = 300
    e = E(sorted({(int(a), int(b)) for a, b in rng.integers(0, n, size=(900, 2)) if a != b}))
    h = oracle.harmonic(n, e, True)
    src = np.array([0, 7, 299, 150], np.int32)
    assert np.array_equal(oracle.harmonic(n, e, True, sources=src), h[src])


# ------------------------------------------------ upper bounds (Sect. 5, 8.4)
def random_tree(n, rng):
    return E([(i, int(rng.integers(0, i))) for i in range(1, n)])


@pytest.mark.parametrize("seed", range(30))
def test_nb_bound_exact_on_trees(seed):
    """On a tree the walk counts are the level sizes, so the bound is h
    itself, bit for bit (the same terms in the same order)."""
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(1, 60))
    e = random_tree(n, rng)
    h = oracle.harmonic(n, e, False)
    ub = oracle.nb_harmonic(n, e, False)
    assert np.array_equal(ub, h)


@pytest.mark.parametrize("n", [3, 4, 7, 10, 31, 64])
def test_nb_bound_on_cycles(n):
    """Undirected cycle: the walks that never step straight back are two of
    each length, and up to length n/2 they end at the two distinct vertices
    at that distance, except the one antipode of an even cycle.  Placing
    vertices stops at omega = n, so the antipode level takes one vertex: the
    bound is h bit for bit (the same terms in the same order), the closed
    form of the cycle.  Directed cycle: one walk per length, h = H(n-1)."""
    e = E([(i, (i + 1) % n) for i in range(n)])
    h = oracle.harmonic(n, e, False)
    ub = oracle.nb_harmonic(n, e, False)
    assert np.array_equal(ub, h)
    m = n // 2
    want = 2 * H(m) if n % 2 else 2 * H(m - 1) + Fraction(1, m)
    assert np.all([close(x, want, n) for x in ub])
    hd = oracle.harmonic(n, e, True)
    ubd = oracle.nb_harmonic(n, e, True)
    assert np.array_equal(ubd, hd)
    assert np.all([close(x, H(n - 1), n) for x in ubd])


def test_nb_bound_forest_with_isolated_vertices():
    rng = np.random.default_rng(77)
    e1 = random_tree(30, rng)
    e2 = random_tree(20, rng) + 30
    e = np.concatenate([e1, e2])
    n = 55   # vertices 50..54 isolated
    h = oracle.harmonic(n, e, False)
    ub = oracle.nb_harmonic(n, e, False)
    assert np.array_equal(ub, h)
    assert np.all(ub[50:] == 0.0)


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("seed", range(40))
def test_bounds_above_h(directed, seed):
    """Both upper bounds hold on random graphs (connected or not), with
    alpha / omega from the reachability bounds for directed ones."""
    rng = np.random.default_rng(5000 + seed + (1000 if directed else 0))
    n = int(rng.integers(2, 40))
    p = float(rng.uniform(0.02, 0.3))
    pairs = {(u, w) for u in range(n) for w in range(n)
             if u != w and rng.random() < p and (directed or u < w)}
    e = E(sorted(pairs))
    # exact h from Floyd-Warshall levels, as Fractions
    for v, lv in enumerate(fw_levels(n, e, directed)):
        exact = sum((Fraction(c, d) for d, c in lv.items()), Fraction(0))
        ub_nb = oracle.nb_harmonic(n, e, directed)[v]
        ub_deg = oracle.deg_harmonic(n, e, directed)[v]
        tol = 1e-12 * max(1.0, float(exact))
        assert ub_nb >= float(exact) - tol, (v, ub_nb, exact)
        assert ub_deg >= float(exact) - tol, (v, ub_deg, exact)


def test_deg_bound_closed_forms():
    # star: the centre's bound is exact (n-1); a leaf sees 1 at distance 1
    # and n-2 at distance 2, also exact
    n = 9
    e = E([(0, i) for i in range(1, n)])
    ub = oracle.deg_harmonic(n, e, False)
    assert ub[0] == n - 1 and np.all(ub[1:] == 1 + (n - 2) / 2)
    # complete graph: n-1 everywhere
    e = E([(i, j) for i in range(6) for j in range(i + 1, 6)])
    assert np.all(oracle.deg_harmonic(6, e, False) == 5.0)


@pytest.mark.parametrize("directed", [False, True])
def test_repeated_arcs_and_self_loops_count_once(directed):
    """The measure is on the simple graph: repeats and self-loops change
    neither h nor its bounds."""
    clean = E([(0, 1), (1, 2), (2, 3), (3, 0), (0, 4)])
    noisy = E([(0, 1), (0, 1), (1, 2), (2, 2), (2, 3), (3, 0), (0, 4), (0, 4), (4, 4)])
    for f in (oracle.harmonic, oracle.nb_harmonic, oracle.deg_harmonic):
        assert np.array_equal(f(6, noisy, directed), f(6, clean, directed)), f.__name__


# ------------------------------------------- level-based bound (Sect. 7, 8.3)
def test_lb_exact_on_path_and_star():
    """Paths (from an end) and stars (from a leaf): the level structure pins
    every distance, so the bound is h itself up to rounding."""
    n = 40
    e = E([(i, i + 1) for i in range(n - 1)])
    h = oracle.harmonic(n, e, False)
    r, ub = oracle.lb_harmonic(n, e, False, 0)
    assert r == n and ub[0] == -1.0
    for w in range(1, n):
        assert close(ub[w], H(w) + H(n - 1 - w), 2 * n)
    n = 12
    e = E([(0, i) for i in range(1, n)])
    r, ub = oracle.lb_harmonic(n, e, False, 3)
    assert ub[0] == n - 1                       # the centre: n-1 neighbours
    for w in range(1, n):
        if w != 3:
            assert ub[w] == n / 2               # a leaf: 1 + (n-2)/2


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("seed", range(40))
def test_lb_above_h(directed, seed):
    """Every applicable bound (same component, or same SCC) stays above the
    exact Floyd-Warshall value, from every source."""
    rng = np.random.default_rng(7000 + seed + (1000 if directed else 0))
    n = int(rng.integers(2, 30))
    p = float(rng.uniform(0.05, 0.4))
    pairs = {(u, w) for u in range(n) for w in range(n)
             if u != w and rng.random() < p and (directed or u < w)}
    e = E(sorted(pairs))
    exact = [sum((Fraction(c, d) for d, c in lv.items()), Fraction(0)) for lv in fw_levels(n, e, directed)]
    scc = oracle.scc(n, e)[1] if directed else None
    for s in range(n):
        r, ub = oracle.lb_harmonic(n, e, directed, s, scc)
        for w in range(n):
            if ub[w] >= 0:
                assert ub[w] >= float(exact[w]) - 1e-12 * max(1.0, float(exact[w])), (s, w)
                if directed:
                    assert scc[w] == scc[s]
