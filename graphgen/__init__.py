"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

The module only generates graphs (edge lists) and turns them into simple
CSR arrays (self-loops and duplicate arcs removed, rows sorted).  It holds
none of the closeness arithmetic.  The C core (``gen.c``) is compiled with
gcc into ``libgraphgen.so`` next to this file by :func:`build`.

Workload recipes (the paper measures on real networks that stand in here as
synthetic graphs of the same shape):

* ``ba(n, m, seed)``: Barabasi-Albert, clique K_{m+1} seed, m distinct
  degree-proportional targets per new vertex (undirected complex networks).
* ``rmat(scale, ef, a, b, c, seed)``: R-MAT arcs, ids permuted (directed
  web/social graphs; not strongly connected).
* ``lattice(side, king, n_delete, n_short, seed)`` then ``lcc``: perturbed
  4- or 8-neighbour grids (road networks, diameter in the hundreds).
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c with gcc into libgraphgen.so (always recompiles when force)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        c = ctypes
        lib.gg_rng_stream.argtypes = [c.c_uint64, c.c_int64, u64p]
        lib.gg_ba_count.argtypes = [c.c_int32, c.c_int32]
        lib.gg_ba_count.restype = c.c_int64
        lib.gg_ba.argtypes = [c.c_int32, c.c_int32, c.c_uint64, i32p]
        lib.gg_ba.restype = c.c_int64
        lib.gg_rmat.argtypes = [c.c_int32, c.c_int64, c.c_double, c.c_double, c.c_double,
                                c.c_uint64, c.c_int, i32p]
        lib.gg_lattice_count.argtypes = [c.c_int32, c.c_int]
        lib.gg_lattice_count.restype = c.c_int64
        lib.gg_lattice.argtypes = [c.c_int32, c.c_int, c.c_int64, c.c_int64, c.c_uint64, i32p]
        lib.gg_lattice.restype = c.c_int64
        lib.gg_gnp.argtypes = [c.c_int32, c.c_double, c.c_int, c.c_uint64, i32p]
        lib.gg_gnp.restype = c.c_int64
        lib.gg_tree.argtypes = [c.c_int32, c.c_uint64, i32p]
        lib.gg_csr.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, c.c_int, i32p, i32p]
        lib.gg_csr.restype = c.c_int64
        lib.gg_lcc.argtypes = [c.c_int32, c.c_int64, i32p, i32p, c.POINTER(c.c_int32)]
        lib.gg_lcc.restype = c.c_int64
        _lib = lib
    return _lib


# ---------------------------------------------------------------- raw draws
def rng_stream(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _L().gg_rng_stream(seed, count, out)
    return out


def ba(n: int, m: int, seed: int) -> np.ndarray:
    ne = _L().gg_ba_count(n, m)
    if ne < 0:
        raise ValueError("BA needs m >= 1 and n >= m + 1")
    e = np.zeros(2 * ne, dtype=np.int32)
    got = _L().gg_ba(n, m, seed, e)
    assert got == ne
    return e.reshape(-1, 2)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         permute: bool = True) -> np.ndarray:
    n_arcs = edge_factor << scale
    e = np.zeros(2 * n_arcs, dtype=np.int32)
    _L().gg_rmat(scale, n_arcs, a, b, c, seed, int(permute), e)
    return e.reshape(-1, 2)


def lattice(side: int, king: bool, n_delete: int, n_short: int, seed: int) -> np.ndarray:
    ne = _L().gg_lattice_count(side, int(king))
    e = np.zeros(2 * (ne + n_short), dtype=np.int32)
    got = _L().gg_lattice(side, int(king), n_delete, n_short, seed, e)
    if got < 0:
        raise ValueError("bad lattice parameters")
    return e[: 2 * got].reshape(-1, 2)


def gnp(n: int, p: float, directed: bool, seed: int) -> np.ndarray:
    e = np.zeros(2 * max(1, n * n), dtype=np.int32)
    got = _L().gg_gnp(n, p, int(directed), seed, e)
    return e[: 2 * got].reshape(-1, 2)


def tree(n: int, seed: int) -> np.ndarray:
    e = np.zeros(2 * max(1, n - 1), dtype=np.int32)
    if n > 1:
        _L().gg_tree(n, seed, e)
    return e[: 2 * max(0, n - 1)].reshape(-1, 2)


def csr(n: int, edges: np.ndarray, directed: bool, transpose: bool = False):
    """Simple-graph CSR (int32 row_ptr[n+1], col_idx[arcs])."""
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1)
    ne = edges.size // 2
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(max(1, (1 if directed else 2) * ne), dtype=np.int32)
    arcs = _L().gg_csr(n, ne, edges, int(directed), int(transpose), row_ptr, col)
    if arcs < 0:
        raise ValueError("edge endpoint out of range")
    return row_ptr, col[:arcs].copy()


def lcc(n: int, edges: np.ndarray):
    """Largest weakly connected component, relabelled by increasing old id."""
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1).copy()
    new_id = np.zeros(max(1, n), dtype=np.int32)
    n_out = ctypes.c_int32(0)
    ne = _L().gg_lcc(n, e.size // 2, e, new_id, ctypes.byref(n_out))
    return int(n_out.value), e[: 2 * ne].reshape(-1, 2), new_id[:n]


# ------------------------------------------------------------- graph bundle
@dataclasses.dataclass
class Graph:
    """A simple graph: raw edge list plus its CSR (and reverse CSR if directed)."""
    name: str
    n: int
    directed: bool
    edges: np.ndarray            # (ne, 2) int32 raw list (may hold loops/dups)
    row_ptr: np.ndarray          # int32[n+1]
    col_idx: np.ndarray          # int32[arcs]
    rrow_ptr: np.ndarray | None = None
    rcol_idx: np.ndarray | None = None

    @property
    def arcs(self) -> int:
        return int(self.row_ptr[-1])

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64([self.n, int(self.directed)]).tobytes())
        h.update(self.row_ptr.tobytes())
        h.update(self.col_idx.tobytes())
        return h.hexdigest()[:16]


def make(name: str, n: int, edges: np.ndarray, directed: bool) -> Graph:
    rp, ci = csr(n, edges, directed)
    g = Graph(name, n, directed, np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2), rp, ci)
    if directed:
        g.rrow_ptr, g.rcol_idx = csr(n, edges, True, transpose=True)
    return g


# ------------------------------------------------- the five workload recipes
def ba_graph(n: int, m: int = 5, seed: int = 1) -> Graph:
    return make("ba_n%d_m%d_s%d" % (n, m, seed), n, ba(n, m, seed), False)


def rmat_graph(scale: int, edge_factor: int = 16, seed: int = 3,
               abc=(0.57, 0.19, 0.19)) -> Graph:
    e = rmat(scale, edge_factor, abc[0], abc[1], abc[2], seed)
    return make("rmat_s%d_ef%d_s%d" % (scale, edge_factor, seed), 1 << scale, e, True)


def grid_graph(side: int, del_frac: float = 0.05, n_short: int | None = None,
               seed: int = 4, king: bool = False) -> Graph:
    """Perturbed lattice restricted to its largest connected component.

    The 2000 x 2000 road-like workload deletes exactly 399,800 of its
    7,996,000 edges (5%) and adds 1,000 shortcuts."""
    ne = _L().gg_lattice_count(side, int(king))
    n_del = int(round(del_frac * ne))
    if n_short is None:
        n_short = max(1, math.ceil(side * side / 4000))
    e = lattice(side, king, n_del, n_short, seed)
    n2, e2, _ = lcc(side * side, e)
    kind = "king" if king else "grid"
    return make("%s%d_d%d_sc%d_s%d" % (kind, side, n_del, n_short, seed), n2, e2, False)


def workload(name: str) -> Graph:
    """Named full-size workloads."""
    if name == "ba2k":          # undirected BA, n=2,000, m=5, seed 1
        return ba_graph(2000, 5, 1)
    if name == "ba1m":          # undirected BA, n=2^20, m=5, seed 2
        return ba_graph(1 << 20, 5, 2)
    if name == "rmat20":        # directed R-MAT scale 20, edge factor 16, seed 3
        return rmat_graph(20, 16, 3)
    if name == "grid2000":      # 2000^2 grid, 5% deleted, 1,000 shortcuts, LCC
        return grid_graph(2000, 0.05, 1000, 4)
    # medium tier: the same shapes at sizes whose all-sources answer takes
    # minutes of CPU, large enough to hold hubs of in-degree > 1024 and
    # walk counts beyond 2^31
    if name == "ba128k":        # undirected BA, n=2^17, m=5, seed 6
        return ba_graph(1 << 17, 5, 6)
    if name == "rmat16":        # directed R-MAT scale 16, edge factor 16, seed 7
        return rmat_graph(16, 16, 7)
    if name == "grid500":       # 500^2 grid, 5% deleted, 63 shortcuts, seed 8, LCC
        return grid_graph(500, 0.05, 63, 8)
    raise KeyError(name)


def serving_pool(count: int = 64, seed: int = 5, n_lo: float = 1e3, n_hi: float = 1e6):
    """The serving mix: family i mod 3 in {BA, R-MAT, king lattice}; n log-uniform
    in [n_lo, n_hi]; target average degree uniform in [8, 16].  A 4-neighbour
    grid cannot reach degree 8, so the lattice family uses 8-neighbour (king)
    moves with 5% deletions and ceil(n/4000) shortcuts."""
    out = []
    st = rng_stream(seed, 3 * count)
    u = st.astype(np.float64) / 2.0 ** 64
    for i in range(count):
        n_i = int(round(10 ** (math.log10(n_lo) + (math.log10(n_hi) - math.log10(n_lo)) * u[3 * i])))
        d_i = 8.0 + 8.0 * u[3 * i + 1]
        gseed = int(st[3 * i + 2] & 0x7FFFFFFF)
        fam = i % 3
        if fam == 0:
            m = max(1, int(round(d_i / 2)))
            out.append(ba_graph(max(n_i, m + 2), m, gseed))
        elif fam == 1:
            scale = max(4, int(round(math.log2(n_i))))
            out.append(rmat_graph(scale, max(1, int(round(d_i))), gseed))
        else:
            side = max(4, int(round(math.sqrt(n_i))))
            out.append(grid_graph(side, 0.05, None, gseed, king=True))
    return out


def reduction_graph(sets, n_ground: int, p: int = 7, q: int = 36):
    """The directed reduction graph of the hardness section (Sect. 3): vertex
    classes Z, Y, C_0, X_1, X_2, C_1..C_p for a family `sets` of subsets of
    range(n_ground).  Returns (n, edges, classes) where classes maps a class
    name to its list of vertex ids (C_0 in family order)."""
    nc = len(sets)
    ids = {}
    nxt = [0]

    def alloc(cls, count):
        ids[cls] = list(range(nxt[0], nxt[0] + count))
        nxt[0] += count
    alloc("Z", q * nc)
    alloc("Y", q)
    alloc("C0", nc)
    alloc("X1", n_ground)
    alloc("X2", n_ground)
    for i in range(1, p + 1):
        alloc("C%d" % i, nc)
    e = []
    for yi, y in enumerate(ids["Y"]):
        for j in range(nc):
            e.append((y, ids["Z"][yi * nc + j]))
    for ci, s in enumerate(sets):
        c0 = ids["C0"][ci]
        for y in ids["Y"]:
            e.append((c0, y))
        for x in range(n_ground):
            if x in s:
                e.append((c0, ids["X1"][x]))
                e.append((ids["X1"][x], ids["C1"][ci]))
            else:
                e.append((c0, ids["X2"][x]))
        for i in range(1, p):
            e.append((ids["C%d" % i][ci], ids["C%d" % (i + 1)][ci]))
    return nxt[0], np.array(e, dtype=np.int32).reshape(-1, 2), ids
