"""ORACLE -- test infrastructure only.

Plain CPU reference for exact top-k closeness: textbook all-sources BFS,
Lin's index with the reachable-set generalisation, the exact (farness, id)
order, and reference versions of the NB / BFSCut / LB bounds and of the
alpha/omega reachability bounds.  See ``oracle.c`` for the passage each part
follows.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import this package; the product path never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        c = ctypes
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        lib.oracle_check_csr.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, c.c_int, i32p, i32p]
        lib.oracle_sums.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, c.c_void_p, c.c_int64,
                                    i64p, i64p, c.c_int]
        lib.oracle_harmonic.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, c.c_void_p, c.c_int64,
                                         np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS"), c.c_int]
        lib.oracle_nb_harmonic.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, i64p,
                                            np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")]
        lib.oracle_lb_harmonic.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, c.c_int32, c.c_void_p,
                                            np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")]
        lib.oracle_lb_harmonic.restype = c.c_int64
        lib.oracle_threads.restype = c.c_int
        lib.oracle_arcs.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int]
        lib.oracle_arcs.restype = c.c_int64
        lib.oracle_topk.argtypes = [c.c_int32, i64p, i64p, c.c_int32, i32p]
        lib.oracle_topk.restype = c.c_int32
        lib.oracle_cmp.argtypes = [c.c_int64] * 4
        lib.oracle_cmp.restype = c.c_int
        lib.oracle_farness.argtypes = [c.c_int32, c.c_int64, c.c_int64]
        lib.oracle_farness.restype = c.c_double
        lib.oracle_floyd_warshall.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, i32p]
        lib.oracle_component_sizes.argtypes = [c.c_int32, c.c_int64, i32p, i64p]
        lib.oracle_scc.argtypes = [c.c_int32, c.c_int64, i32p, i32p]
        lib.oracle_scc.restype = c.c_int32
        lib.oracle_alpha_omega.argtypes = [c.c_int32, c.c_int64, i32p, i64p, i64p, i32p]
        lib.oracle_nb.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, i64p, i64p, i64p, i64p]
        lib.oracle_cut_levels.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, c.c_int32,
                                          c.c_int64, c.c_int64, c.c_int32, i64p, i64p, i64p, i64p]
        lib.oracle_cut_levels.restype = c.c_int32
        lib.oracle_lb_source.argtypes = [c.c_int32, c.c_int64, i32p, c.c_int, c.c_int32,
                                         c.c_void_p, c.c_int, i64p]
        lib.oracle_lb_source.restype = c.c_int64
        _lib = lib
    return _lib


def _edges(edges) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))


def threads() -> int:
    return int(_L().oracle_threads())


def check_csr(n, edges, directed, row_ptr, col_idx, reverse=False) -> bool:
    e = _edges(edges)
    return _L().oracle_check_csr(n, e.size // 2, e, int(directed), int(reverse),
                                 np.ascontiguousarray(row_ptr, dtype=np.int32),
                                 np.ascontiguousarray(col_idx, dtype=np.int32)) == 0


def sums(n, edges, directed, sources=None, nthreads=0):
    """Exact (S, r) per source by textbook BFS (all vertices if sources is None)."""
    e = _edges(edges)
    if sources is None:
        cnt = n
        src_ptr = None
        src = None
    else:
        src = np.ascontiguousarray(sources, dtype=np.int32)
        cnt = src.size
        src_ptr = src.ctypes.data_as(ctypes.c_void_p)
    S = np.zeros(max(1, cnt), dtype=np.int64)
    r = np.zeros(max(1, cnt), dtype=np.int64)
    rc = _L().oracle_sums(n, e.size // 2, e, int(directed), src_ptr, cnt, S, r, nthreads)
    if rc:
        raise ValueError("bad edge list")
    return S[:cnt], r[:cnt]


def harmonic(n, edges, directed, sources=None, nthreads=0):
    """Harmonic centrality per source (Sect. 2 with f(d) = 1/d): the binary64
    sum over d = 1, 2, ... of n_d / d, added in increasing d (oracle.c)."""
    e = _edges(edges)
    if sources is None:
        cnt = n
        src_ptr = None
    else:
        src = np.ascontiguousarray(sources, dtype=np.int32)
        cnt = src.size
        src_ptr = src.ctypes.data_as(ctypes.c_void_p)
    h = np.zeros(max(1, cnt), dtype=np.float64)
    rc = _L().oracle_harmonic(n, e.size // 2, e, int(directed), src_ptr, cnt, h, nthreads)
    if rc:
        raise ValueError("bad edge list")
    return h[:cnt]


def nb_harmonic(n, edges, directed, omega=None):
    """Walk-count upper bound on the harmonic centrality (oracle.c); omega
    defaults to the reachability upper bounds of Sect. 8.4."""
    e = _edges(edges)
    if omega is None:
        omega = reach_bounds(n, edges, directed)[1]
    o = np.ascontiguousarray(omega, dtype=np.int64)
    ub = np.zeros(max(1, n), dtype=np.float64)
    if _L().oracle_nb_harmonic(n, e.size // 2, e, int(directed), o, ub):
        raise ValueError("bad edge list")
    return ub[:n]


def deg_harmonic(n, edges, directed, omega=None):
    """Degree upper bound on the harmonic centrality: the distinct
    out-neighbours at distance 1, every other vertex v may reach at
    distance >= 2 (self-loops and repeated arcs count once, as in the
    adjacency oracle.c builds)."""
    e = _edges(edges).reshape(-1, 2).astype(np.int64)
    e = e[e[:, 0] != e[:, 1]]
    if not directed:
        e = np.concatenate([e, e[:, ::-1]])
    e = np.unique(e[:, 0] * max(n, 1) + e[:, 1])
    if omega is None:
        omega = reach_bounds(n, edges, directed)[1]
    deg = np.bincount((e // max(n, 1)).astype(np.int64), minlength=n)
    out = np.zeros(n, dtype=np.float64)
    for v in range(n):
        if omega[v] > 1:
            out[v] = float(deg[v]) + float(omega[v] - 1 - deg[v]) / 2.0
    return out


def lb_harmonic(n, edges, directed, s, scc_ids=None):
    """Level-based upper bound on the harmonic centrality from a complete
    search at s (oracle.c); -1 where it does not apply.  Returns (r(s), ub)."""
    e = _edges(edges)
    out = np.zeros(max(1, n), dtype=np.float64)
    if scc_ids is not None:
        sc = np.ascontiguousarray(scc_ids, dtype=np.int32)
        ptr = sc.ctypes.data_as(ctypes.c_void_p)
    else:
        sc = None
        ptr = None
    r = _L().oracle_lb_harmonic(n, e.size // 2, e, int(directed), int(s), ptr, out)
    return int(r), out[:n]


def harmonic_topk(h, k):
    """The first min(k, n) vertices: larger h first, an exact tie to the smaller id."""
    h = np.asarray(h, dtype=np.float64)
    order = np.lexsort((np.arange(h.size), -h))
    return order[:max(0, min(k, h.size))].astype(np.int32)


def arcs(n, edges, directed) -> int:
    e = _edges(edges)
    return int(_L().oracle_arcs(n, e.size // 2, e, int(directed)))


def topk(S, r, k):
    S = np.ascontiguousarray(S, dtype=np.int64)
    r = np.ascontiguousarray(r, dtype=np.int64)
    n = S.size
    ids = np.zeros(max(1, min(max(k, 0), n)), dtype=np.int32)
    c = _L().oracle_topk(n, S, r, k, ids)
    return ids[:c]


def cmp(Sa, ra, Sb, rb) -> int:
    return int(_L().oracle_cmp(int(Sa), int(ra), int(Sb), int(rb)))


def farness(n, S, r) -> float:
    return float(_L().oracle_farness(int(n), int(S), int(r)))


def closeness_topk(n, edges, directed, k, nthreads=0):
    """Oracle answer: (ids, S, r, farness) of the first min(k, n) vertices."""
    S, r = sums(n, edges, directed, nthreads=nthreads)
    ids = topk(S, r, k)
    far = np.array([farness(n, S[i], r[i]) for i in ids], dtype=np.float64)
    return ids, S[ids], r[ids], far


def floyd_warshall(n, edges, directed):
    e = _edges(edges)
    d = np.zeros(max(1, n * n), dtype=np.int32)
    _L().oracle_floyd_warshall(n, e.size // 2, e, int(directed), d)
    return d[: n * n].reshape(n, n)


def component_sizes(n, edges):
    e = _edges(edges)
    out = np.zeros(max(1, n), dtype=np.int64)
    _L().oracle_component_sizes(n, e.size // 2, e, out)
    return out[:n]


def scc(n, edges):
    e = _edges(edges)
    comp = np.zeros(max(1, n), dtype=np.int32)
    nc = _L().oracle_scc(n, e.size // 2, e, comp)
    return int(nc), comp[:n]


def alpha_omega(n, edges):
    e = _edges(edges)
    a = np.zeros(max(1, n), dtype=np.int64)
    o = np.zeros(max(1, n), dtype=np.int64)
    comp = np.zeros(max(1, n), dtype=np.int32)
    _L().oracle_alpha_omega(n, e.size // 2, e, a, o, comp)
    return a[:n], o[:n], comp[:n]


def reach_bounds(n, edges, directed):
    """(alpha, omega, scc) with alpha = omega = r for undirected graphs."""
    if not directed:
        r = component_sizes(n, edges)
        return r, r.copy(), None
    return alpha_omega(n, edges)


def nb(n, edges, directed, alpha=None, omega=None):
    """Neighbourhood-based farness bound as (num, den): bound = (n-1) num / den, den 0 = inf."""
    e = _edges(edges)
    if alpha is None:
        alpha, omega, _ = reach_bounds(n, edges, directed)
    a = np.ascontiguousarray(alpha, dtype=np.int64)
    o = np.ascontiguousarray(omega, dtype=np.int64)
    num = np.zeros(max(1, n), dtype=np.int64)
    den = np.zeros(max(1, n), dtype=np.int64)
    _L().oracle_nb(n, e.size // 2, e, int(directed), a, o, num, den)
    return num[:n], den[:n]


def cut_levels(n, edges, directed, v, alpha, omega, cap=100000):
    e = _edges(edges)
    cap = max(1, min(cap, n + 1))
    bufs = [np.zeros(cap, dtype=np.int64) for _ in range(4)]
    lv = _L().oracle_cut_levels(n, e.size // 2, e, int(directed), int(v), int(alpha), int(omega),
                                cap, *bufs)
    lv = min(lv, cap)
    return tuple(b[:lv] for b in bufs)


def lb_source(n, edges, directed, s, scc_ids=None, direct=False):
    """Level-based bound on S(v) from a BFS at s; -1 where it does not apply."""
    e = _edges(edges)
    out = np.zeros(max(1, n), dtype=np.int64)
    if scc_ids is not None:
        sc = np.ascontiguousarray(scc_ids, dtype=np.int32)
        ptr = sc.ctypes.data_as(ctypes.c_void_p)
    else:
        sc = None
        ptr = None
    r = _L().oracle_lb_source(n, e.size // 2, e, int(directed), int(s), ptr, int(direct), out)
    return int(r), out[:n]
