"""The oracle's Alg. 6 (Sect. 8.4) against digraphs worked out by hand.

Each fixture under tests/golden/alg6_*.txt lists a digraph and, per vertex,
the alpha and omega that the steps of Alg. 6 give (worked in the file's
comments, step by step) and the exact reach r.  The three cover: the
refinement through the largest SCC changing omega; a component that reaches
the largest SCC only through another one (the listing counts its reach
twice and the cap at n binds); and the tie between two largest SCCs.
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FIXTURES = ["alg6_refine.txt", "alg6_through.txt", "alg6_tie.txt"]


def load(name):
    n, arcs, rows = None, [], {}
    with open(os.path.join(GOLDEN, name)) as fp:
        for line in fp:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "n":
                n = int(t[1])
            elif t[0] == "arc":
                arcs.append((int(t[1]), int(t[2])))
            elif t[0] == "v":
                rows[int(t[1])] = tuple(int(x) for x in t[2:5])
    assert n is not None and sorted(rows) == list(range(n)), name
    a = np.array([rows[v][0] for v in range(n)], np.int64)
    o = np.array([rows[v][1] for v in range(n)], np.int64)
    r = np.array([rows[v][2] for v in range(n)], np.int64)
    return n, np.array(arcs, np.int32).reshape(-1, 2), a, o, r


@pytest.mark.parametrize("name", FIXTURES)
def test_alpha_omega_by_hand(name):
    n, e, a, o, r = load(name)
    ga, go, _ = oracle.alpha_omega(n, e)
    assert np.array_equal(ga, a), (name, ga.tolist(), a.tolist())
    assert np.array_equal(go, o), (name, go.tolist(), o.tolist())


@pytest.mark.parametrize("name", FIXTURES)
def test_hand_reach_counts(name):
    """The r column is the reach count of each vertex, which the textbook
    search must give, and alpha <= r <= omega holds."""
    n, e, a, o, r = load(name)
    _, gr = oracle.sums(n, e, True)
    assert np.array_equal(gr, r), (name, gr.tolist(), r.tolist())
    assert np.all(a <= r) and np.all(r <= o)
