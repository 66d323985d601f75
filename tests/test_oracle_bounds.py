"""Pins of the oracle's reference bounds.

* Prop. 5.1 / Sect. 5: the NB bound never exceeds the exact farness, and on
  trees it is exact (the recurrence of Alg. 2 counts each level exactly).
* Lemma 6.1 and Sect. 8.2: every per-level BFSCut bound stays below the
  exact farness; at the last level the tightened bound equals it when r is
  known.
* Sect. 7 (Eq. 4 / Eq. 5, Lemma 7.2): the level-based bound stays below S(v);
  the recurrence gives the same level table as the direct definition.
* Sect. 8.4 (Alg. 6): alpha <= r <= omega, exact on strongly connected graphs.
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle


def le(num, den, S, r):
    """bound num/den <= S/(r-1)^2 (den 0 = +inf)."""
    if r <= 1:
        return True
    if den == 0:
        return False
    return Fraction(int(num), int(den)) <= Fraction(int(S), int(r - 1) ** 2)


def graphs(directed, count=150):
    for seed in range(count):
        n = 2 + seed % 30
        p = [0.03, 0.08, 0.15, 0.3][seed % 4]
        yield seed, n, graphgen.gnp(n, p, directed, 5000 + seed)
    # sparse trees with a few chords, some split in two
    for seed in range(count):
        n = 3 + seed % 28
        e = graphgen.tree(n, 9000 + seed)
        extra = graphgen.gnp(n, 0.04, directed, 9500 + seed)
        ee = np.concatenate([e, extra]) if len(extra) else e
        if seed % 3 == 0 and len(ee) > 2:
            ee = ee[:-2]
        yield seed, n, ee


@pytest.mark.parametrize("directed", [False, True])
def test_nb_bound_valid(directed):
    for seed, n, e in graphs(directed):
        S, r = oracle.sums(n, e, directed)
        num, den = oracle.nb(n, e, directed)
        for v in range(n):
            assert le(num[v], den[v], S[v], r[v]), (seed, v)
            if r[v] <= 1:
                assert den[v] == 0


def test_nb_exact_on_trees():
    for seed in range(300):
        n = 2 + seed % 40
        e = graphgen.tree(n, 100 + seed)
        S, r = oracle.sums(n, e, False)
        num, den = oracle.nb(n, e, False)
        assert (den == (n - 1) ** 2).all()
        assert (num == S).all(), seed


def test_nb_exact_on_directed_paths_and_stars():
    """On a directed path every walk count is exact (one walk per length)."""
    n = 12
    e = np.array([(i, i + 1) for i in range(n - 1)], dtype=np.int32)
    a, o, _ = oracle.alpha_omega(n, e)
    S, r = oracle.sums(n, e, True)
    num, den = oracle.nb(n, e, True, a, o)
    for v in range(n - 1):
        assert Fraction(int(num[v]), int(den[v])) == Fraction(int(S[v]), int(r[v] - 1) ** 2)


def test_nb_known_small_values():
    """Hand-computed: path 0-1-2-3 (undirected).  Vertex 0: gamma = 1,1,1 so
    S_NB = 1+2+3 = 6 (exact).  Cycle C_4, vertex 0: gamma_1 = 2, gamma_2 =
    2 (non-backtracking walks, they reach the same vertex), r = 4, so
    S_NB = 2*1 + 2*1 (one slot left) = 4 = exact S."""
    e = np.array([(0, 1), (1, 2), (2, 3)], dtype=np.int32)
    num, den = oracle.nb(4, e, False)
    assert list(num) == [6, 4, 4, 6] and list(den) == [9] * 4
    c4 = np.array([(0, 1), (1, 2), (2, 3), (3, 0)], dtype=np.int32)
    num, den = oracle.nb(4, c4, False)
    assert list(num) == [4] * 4


def walk_counts(n, e, directed, s, kmax):
    """gamma_1(s) .. gamma_kmax(s) counted by enumeration, as the arcs the
    walks end on: directed, every walk of length k out of s (Eq. 3);
    undirected, every walk that never steps straight back along the edge it
    came by, which is what the tree recurrence of Sect. 5 (Eq. 2, Alg. 3)
    counts.  Self-loops and repeated arcs are dropped, as in the oracle."""
    arcs = {(int(u), int(v)) for u, v in e if u != v}
    if not directed:
        arcs |= {(v, u) for u, v in arcs}
    out = {u: [] for u in range(n)}
    for u, v in sorted(arcs):
        out[u].append(v)
    cur = {(s, c): 1 for c in out[s]}
    g = []
    for _ in range(kmax):
        g.append(sum(cur.values()))
        nxt = {}
        for (p, c), w in cur.items():
            for x in out[c]:
                if directed or x != p:
                    nxt[(c, x)] = nxt.get((c, x), 0) + w
        cur = nxt
    return g


def nb_by_enumeration(n, e, directed, s, a, o):
    """Prop. 5.1 with alpha <= r <= omega (Sect. 8.1), by exhaustion: for
    every integer r in [alpha, omega], place r - 1 vertices at levels 1, 2,
    ... with at most gamma_k at level k (r is impossible when the walks die
    out first) and keep the least S_NB(r) / (r-1)^2; None when no r >= 2 is
    possible (+inf)."""
    g = walk_counts(n, e, directed, s, max(1, int(o)))
    best = None
    for r in range(max(2, int(a)), int(o) + 1):
        placed, S = 1, 0
        for k, gk in enumerate(g, start=1):
            take = min(gk, r - placed)
            S += k * take
            placed += take
            if placed == r:
                break
        if placed < r:
            continue
        f = Fraction(S, (r - 1) ** 2)
        best = f if best is None or f < best else best
    return best


@pytest.mark.parametrize("directed", [False, True])
def test_nb_matches_enumeration(directed):
    """The oracle evaluates Prop. 5.1 only at alpha, omega and the level
    boundaries between them, from the recurrence; the enumeration tries
    every r from walks it lists one by one.  Reachability bounds: Alg. 6 on
    digraphs, exact r, and the loose 1 <= r <= n."""
    checks = 0
    for seed in range(60):
        n = 2 + seed % 13
        e = graphgen.gnp(n, [0.08, 0.15, 0.3][seed % 3], directed, 41000 + seed)
        S, r = oracle.sums(n, e, directed)
        ab, ob, _ = oracle.reach_bounds(n, e, directed)
        for a, o in ((ab, ob), (r, r), (np.ones(n, np.int64), np.full(n, n, np.int64))):
            num, den = oracle.nb(n, e, directed, a, o)
            for v in range(n):
                want = nb_by_enumeration(n, e, directed, v, a[v], o[v])
                if want is None:
                    assert den[v] == 0, (seed, v)
                else:
                    assert den[v] > 0 and Fraction(int(num[v]), int(den[v])) == want, (seed, v, a[v], o[v])
                checks += 1
    assert checks > 1000


@pytest.mark.parametrize("directed", [False, True])
def test_cut_bounds_valid(directed):
    checks = 0
    for seed, n, e in graphs(directed, 80):
        S, r = oracle.sums(n, e, directed)
        a, o, _ = oracle.reach_bounds(n, e, directed)
        for v in range(n):
            num, den, pnum, pden = oracle.cut_levels(n, e, directed, v, a[v], o[v])
            for D in range(len(num)):
                assert le(num[D], den[D], S[v], r[v]), (seed, v, D)
                if r[v] > 1:
                    assert Fraction(int(pnum[D]), int(pden[D])) <= Fraction(int(S[v]), int(r[v] - 1) ** 2)
                checks += 1
            if r[v] > 1 and a[v] == o[v]:
                assert Fraction(int(num[-1]), int(den[-1])) == Fraction(int(S[v]), int(r[v] - 1) ** 2)
    assert checks > 1000


def test_cut_bound_hand_values():
    """Star with centre 0 and 5 leaves, source = leaf 1, r = 6.
    D=0: n_0 = 1, S_0 = 0, U = deg(1) = 1:
         tightened = 0 + 1*5 + max(0, 5-1) = 9, paper = 0 - 1 + 2*5 = 9.
    D=1: n_1 = 2, S_1 = 1, U = deg(0) - 1 = 4: tightened = 1 + 2*4 + 0 = 9 = S."""
    e = np.array([(0, i) for i in range(1, 6)], dtype=np.int32)
    num, den, pnum, pden = oracle.cut_levels(6, e, False, 1, 6, 6)
    assert list(num) == [9, 9, 9] and list(den) == [25] * 3
    assert list(pnum[:2]) == [9, 9]


@pytest.mark.parametrize("directed", [False, True])
def test_lb_valid_and_recurrence(directed):
    for seed, n, e in graphs(directed, 100):
        S, r = oracle.sums(n, e, directed)
        sc = oracle.scc(n, e)[1] if directed else None
        for s in range(0, n, 3):
            rs, b = oracle.lb_source(n, e, directed, s, sc)
            rs2, b2 = oracle.lb_source(n, e, directed, s, sc, direct=True)
            assert (b == b2).all(), (seed, s)
            assert rs == r[s]
            for v in range(n):
                if b[v] >= 0:
                    assert b[v] <= S[v], (seed, s, v)
                    assert r[v] == r[s]


def test_lb_hand_values():
    """Path 0-1-2-3-4 from s = 0: gamma = (1,1,1,1,1).
    Lev(i) = 2*(#levels within 1) + sum_{|j-i|>1} |j-i| - 2.
    v=2 (i=2): near {1,2,3} -> 6, far: j=0 (2) + j=4 (2) -> 4; Lev = 8,
    bound = 8 - deg(2) = 6 = S(2)."""
    e = np.array([(i, i + 1) for i in range(4)], dtype=np.int32)
    _, b = oracle.lb_source(5, e, False, 0)
    assert b[2] == 6
    S, _ = oracle.sums(5, e, False)
    assert S[2] == 6


def test_alpha_omega_brackets_r():
    for seed in range(400):
        n = 2 + seed % 16
        e = graphgen.gnp(n, [0.05, 0.1, 0.2][seed % 3], True, 20000 + seed)
        S, r = oracle.sums(n, e, True)
        a, o, comp = oracle.alpha_omega(n, e)
        assert (a <= r).all() and (r <= o).all(), seed
        assert (o <= n).all()
        # vertices of the largest SCC (ties: smallest id) get r exactly
        nc, c2 = oracle.scc(n, e)
        sizes = np.bincount(c2, minlength=nc)
        big = max(range(nc), key=lambda c: (sizes[c], -int(np.min(np.nonzero(c2 == c)[0]))))
        for v in np.nonzero(c2 == big)[0]:
            assert a[v] == r[v] == o[v]


def test_alpha_omega_strongly_connected_exact():
    n = 30
    e = np.array([(i, (i + 1) % n) for i in range(n)] + [(0, 15), (7, 3)], dtype=np.int32)
    a, o, _ = oracle.alpha_omega(n, e)
    assert (a == n).all() and (o == n).all()


def test_scc_matches_mutual_reachability():
    for seed in range(100):
        n = 2 + seed % 20
        e = graphgen.gnp(n, 0.1, True, 30000 + seed)
        d = oracle.floyd_warshall(n, e, True)
        nc, comp = oracle.scc(n, e)
        for u in range(n):
            for v in range(n):
                same = d[u, v] >= 0 and d[v, u] >= 0
                assert (comp[u] == comp[v]) == same
        # numbering is topological: an arc never goes to a smaller component
        for u, v in e:
            if comp[u] != comp[v]:
                assert comp[u] < comp[v]
