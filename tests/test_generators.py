"""Input generators: sizes, determinism, simple-graph CSR invariants."""
import numpy as np
import pytest

import graphgen
import oracle


def test_ba_counts_and_determinism():
    e = graphgen.ba(2000, 5, 1)
    assert len(e) == 9985
    assert (e == graphgen.ba(2000, 5, 1)).all()
    assert not (e == graphgen.ba(2000, 5, 2)).all()
    assert graphgen._L().gg_ba_count(1 << 20, 5) == 5242865
    g = graphgen.make("ba", 2000, e, False)
    assert g.arcs == 2 * 9985  # BA never repeats an edge
    assert oracle.check_csr(2000, e, False, g.row_ptr, g.col_idx)
    assert (oracle.component_sizes(2000, e) == 2000).all()


def test_csr_is_simple_and_matches_oracle():
    for directed in (False, True):
        e = np.array([(0, 1), (1, 0), (1, 1), (2, 3), (2, 3), (3, 4), (4, 0)], dtype=np.int32)
        g = graphgen.make("t", 6, e, directed)
        for u in range(6):
            row = g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]
            assert (np.diff(row) > 0).all() and u not in row
        assert oracle.check_csr(6, e, directed, g.row_ptr, g.col_idx)
        if directed:
            assert oracle.check_csr(6, e, True, g.rrow_ptr, g.rcol_idx, reverse=True)


def test_rmat_small():
    g = graphgen.rmat_graph(10, 8, seed=11)
    assert g.n == 1024 and g.directed
    assert g.arcs <= 8 * 1024
    assert oracle.check_csr(g.n, g.edges, True, g.row_ptr, g.col_idx)
    assert oracle.check_csr(g.n, g.edges, True, g.rrow_ptr, g.rcol_idx, reverse=True)
    g2 = graphgen.rmat_graph(10, 8, seed=11)
    assert g.digest() == g2.digest()


def test_grid_lattice():
    side = 40
    ne = graphgen._L().gg_lattice_count(side, 0)
    assert ne == 2 * side * (side - 1)
    e = graphgen.lattice(side, False, 100, 7, 3)
    assert len(e) == ne - 100 + 7
    g = graphgen.grid_graph(side, 0.05, 7, seed=3)
    assert (oracle.component_sizes(g.n, g.edges) == g.n).all()
    assert g.n <= side * side
    k = graphgen._L().gg_lattice_count(side, 1)
    assert k == 2 * side * (side - 1) + 2 * (side - 1) ** 2


def test_grid2000_recipe_counts():
    """The 2000^2 workload: 7,996,000 lattice edges, 399,800 deleted (5%)."""
    assert graphgen._L().gg_lattice_count(2000, 0) == 7996000
    assert round(0.05 * 7996000) == 399800


def test_tree_and_gnp():
    e = graphgen.tree(50, 1)
    assert len(e) == 49
    assert (oracle.component_sizes(50, e) == 50).all()
    g = graphgen.gnp(30, 0.0, False, 1)
    assert len(g) == 0


def test_rng_stream_deterministic():
    a = graphgen.rng_stream(42, 100)
    b = graphgen.rng_stream(42, 100)
    assert (a == b).all() and len(set(a.tolist())) == 100
    # rough uniformity of the top bit
    big = graphgen.rng_stream(7, 20000)
    frac = float(((big >> np.uint64(63)) & np.uint64(1)).mean())
    assert 0.47 < frac < 0.53
