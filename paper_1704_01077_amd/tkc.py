"""Python binding of libtkc.so (argument marshalling only).

Every entry point of ``include/tkc.h`` is exposed under the same name; the
helpers ``Graph`` / ``topk_closeness`` wrap them for numpy arrays and torch
tensors.  Nothing here computes any part of the method: all of it runs in
the HIP library, and importing this module fails loudly when the library is
missing or cannot be loaded.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtkc.so")

TKC_OK = 0
TKC_EINVAL = -1
TKC_ENOMEM = -2
TKC_EDEVICE = -3
TKC_ENOTSUP = -4
TKC_EBUSY = -5
TKC_ECANCELED = -6

TKC_AUTO, TKC_DEG_CUT, TKC_NB_CUT, TKC_DEG_BOUND, TKC_NB_BOUND = 0, 1, 2, 3, 4
TKC_DEG_CUTLB, TKC_NB_CUTLB = 5, 6
TKC_PLAIN, TKC_BATCHED, TKC_HYBRID, TKC_MODE_AUTO = 0, 1, 2, 3
TKC_DIRECTED, TKC_VALIDATE, TKC_DEVICE_PTRS, TKC_REVERSE, TKC_RELABEL = 1, 2, 4, 8, 16

VARIANTS = {"auto": TKC_AUTO, "degcut": TKC_DEG_CUT, "nbcut": TKC_NB_CUT,
            "degbound": TKC_DEG_BOUND, "nbbound": TKC_NB_BOUND,
            "degcutlb": TKC_DEG_CUTLB, "nbcutlb": TKC_NB_CUTLB}
MODES = {"plain": TKC_PLAIN, "batched": TKC_BATCHED, "hybrid": TKC_HYBRID, "auto": TKC_MODE_AUTO}

EXPORTS = [
    "tkc_ctx_create", "tkc_ctx_destroy", "tkc_ctx_get_tuning", "tkc_ctx_set_tuning", "tkc_graph_upload",
    "tkc_graph_free", "tkc_topk_closeness", "tkc_topk_closeness_budget", "tkc_topk_closeness_ties", "tkc_autotune", "tkc_graph_reach", "tkc_graph_reach_info", "tkc_graph_reach_noalloc", "tkc_graph_bounds", "tkc_topk_harmonic", "tkc_graph_harmonic_bounds", "tkc_graph_harmonic_lb_update", "tkc_graph_lb_update",
    "tkc_graph_sums", "tkc_server_create", "tkc_server_add_graph", "tkc_server_submit",
    "tkc_server_poll", "tkc_server_result", "tkc_server_cancel", "tkc_server_destroy",
    "tkc_pack_create", "tkc_pack_topk", "tkc_pack_free", "tkc_server_enable_packing", "tkc_server_info",
    "tkc_last_error", "tkc_version",
]


class tkc_stats(ctypes.Structure):
    _fields_ = [
        ("m_vis", ctypes.c_int64), ("bfs_started", ctypes.c_int64), ("bfs_exact", ctypes.c_int64),
        ("bfs_cut", ctypes.c_int64), ("skipped", ctypes.c_int64), ("deferred", ctypes.c_int64),
        ("max_level", ctypes.c_int32), ("batch_width", ctypes.c_int32), ("variant_used", ctypes.c_int32),
        ("mode_used", ctypes.c_int32), ("nb_rounds", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("ms_reach", ctypes.c_double), ("ms_bounds", ctypes.c_double), ("ms_traverse", ctypes.c_double),
        ("ms_total", ctypes.c_double), ("ms_kernel_main", ctypes.c_double),
        ("main_launches", ctypes.c_int32), ("main_kernel", ctypes.c_int32), ("bytes_main", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


class tkc_tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("batch_width", "td_bu_alpha", "bu_td_beta", "batch_alpha",
                                              "swarm_qcap", "seed_lanes", "blocks_per_cu", "mode")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TkcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tkc error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtkc.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1704_01077_amd.build)")
    # torch's HIP runtime must be the one this library binds to: streams and
    # device pointers handed over from torch are only valid there, and a
    # second runtime loaded first does not see the device once torch has
    # initialised its own
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp, i32, i64, u32, u64 = c.c_void_p, c.c_int32, c.c_int64, c.c_uint32, c.c_uint64
    P = c.POINTER
    sig = {
        "tkc_ctx_create": [c.c_int, vp, P(vp)],
        "tkc_ctx_destroy": [vp],
        "tkc_ctx_get_tuning": [vp, P(tkc_tuning)],
        "tkc_ctx_set_tuning": [vp, P(tkc_tuning)],
        "tkc_autotune": [vp, i32, i32, c.c_double, P(tkc_tuning), P(c.c_double)],
        "tkc_graph_upload": [vp, i32, i64, vp, vp, vp, vp, u32, P(vp)],
        "tkc_graph_free": [vp],
        "tkc_topk_closeness": [vp, i32, i32, i32, vp, vp, vp, vp, P(i32), P(tkc_stats)],
        "tkc_topk_closeness_ties": [vp, i32, i32, i32, i32, vp, vp, vp, vp, P(i32), P(tkc_stats)],
        "tkc_topk_closeness_budget": [vp, i32, i32, i64, vp, vp, vp, vp, P(i32), P(tkc_stats)],
        "tkc_pack_create": [vp, vp, i32, P(vp)],
        "tkc_pack_topk": [vp, i32, vp, vp, i32, vp, vp, vp, vp, vp, P(tkc_stats)],
        "tkc_pack_free": [vp],
        "tkc_server_enable_packing": [vp, i32],
        "tkc_server_info": [vp, P(i64), P(i64), P(i64), P(i32)],
        "tkc_graph_reach": [vp, vp, vp, vp],
        "tkc_graph_reach_info": [vp, P(i32), P(c.c_double)],
        "tkc_graph_reach_noalloc": [vp, vp, vp, vp],
        "tkc_topk_harmonic": [vp, i32, i32, i32, vp, vp, P(i32), P(tkc_stats)],
        "tkc_graph_harmonic_bounds": [vp, i32, vp, vp],
        "tkc_graph_harmonic_lb_update": [vp, vp, i32, vp],
        "tkc_graph_bounds": [vp, i32, vp, vp, vp],
        "tkc_graph_lb_update": [vp, vp, i32, vp, vp],
        "tkc_graph_sums": [vp, vp, i32, vp, vp],
        "tkc_server_create": [vp, c.c_size_t, i32, P(vp)],
        "tkc_server_add_graph": [vp, vp, P(i32)],
        "tkc_server_submit": [vp, i32, i32, i32, P(u64)],
        "tkc_server_poll": [vp, u64, P(i32)],
        "tkc_server_result": [vp, u64, vp, vp, vp, vp, P(i32), P(c.c_double)],
        "tkc_server_cancel": [vp, u64],
        "tkc_server_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c.c_int
    lib.tkc_last_error.restype = c.c_char_p
    lib.tkc_last_error.argtypes = []
    lib.tkc_version.restype = c.c_char_p
    lib.tkc_version.argtypes = []
    return lib


lib = _load()


def _check(rc):
    if rc != TKC_OK:
        raise TkcError(rc, lib.tkc_last_error().decode())
    return rc


def _ptr(a):
    """Device or host pointer of a numpy array / torch tensor (or None)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())   # torch tensor


# ---------------------------------------------------------- raw entry points
def tkc_ctx_create(device: int = 0, hip_stream: int | None = None):
    h = ctypes.c_void_p()
    _check(lib.tkc_ctx_create(device, ctypes.c_void_p(hip_stream) if hip_stream else None, ctypes.byref(h)))
    return h


def tkc_ctx_destroy(ctx):
    _check(lib.tkc_ctx_destroy(ctx))


def tkc_ctx_get_tuning(ctx) -> dict:
    t = tkc_tuning()
    _check(lib.tkc_ctx_get_tuning(ctx, ctypes.byref(t)))
    return t.as_dict()


def tkc_ctx_set_tuning(ctx, **kw):
    """Set the named knobs; the others keep their current values."""
    t = tkc_tuning()
    _check(lib.tkc_ctx_get_tuning(ctx, ctypes.byref(t)))
    for k, v in kw.items():
        if k == "mode":
            v = MODES.get(v, v)
        if k not in t.as_dict():
            raise TypeError("unknown tuning knob %r" % k)
        setattr(t, k, int(v))
    _check(lib.tkc_ctx_set_tuning(ctx, ctypes.byref(t)))


def tkc_autotune(g, k, variant=TKC_AUTO, budget_ms=10000.0):
    """Returns (best knob dict, best query ms); the graph keeps the setting."""
    t = tkc_tuning()
    ms = ctypes.c_double()
    _check(lib.tkc_autotune(g, int(k), VARIANTS.get(variant, variant), float(budget_ms), ctypes.byref(t),
                            ctypes.byref(ms)))
    return t.as_dict(), ms.value


def tkc_graph_upload(ctx, n, m_arcs, row_ptr, col_idx, rrow_ptr=None, rcol_idx=None, flags=0):
    h = ctypes.c_void_p()
    _check(lib.tkc_graph_upload(ctx, n, m_arcs, _ptr(row_ptr), _ptr(col_idx), _ptr(rrow_ptr),
                                _ptr(rcol_idx), flags, ctypes.byref(h)))
    return h


def tkc_graph_free(g):
    _check(lib.tkc_graph_free(g))


def tkc_topk_closeness(g, k, variant, mode, ids, sum_dist=None, reach=None, farness=None):
    n_out = ctypes.c_int32(0)
    st = tkc_stats()
    _check(lib.tkc_topk_closeness(g, k, variant, mode, _ptr(ids), _ptr(sum_dist), _ptr(reach),
                                  _ptr(farness), ctypes.byref(n_out), ctypes.byref(st)))
    return n_out.value, st


def tkc_topk_closeness_ties(g, k, variant, mode, cap, ids, sum_dist=None, reach=None, farness=None):
    """Returns (rc, n_out, stats): rc is TKC_EINVAL with n_out = the needed
    capacity when the answer does not fit cap; other errors raise."""
    n_out = ctypes.c_int32(0)
    st = tkc_stats()
    rc = lib.tkc_topk_closeness_ties(g, k, variant, mode, cap, _ptr(ids), _ptr(sum_dist), _ptr(reach),
                                     _ptr(farness), ctypes.byref(n_out), ctypes.byref(st))
    if rc != TKC_OK and not (rc == TKC_EINVAL and n_out.value > cap):
        _check(rc)
    return rc, n_out.value, st


def tkc_topk_closeness_budget(g, k, variant, max_searches, ids, sum_dist=None, reach=None, farness=None):
    """Returns (rc, n_out, stats): rc is TKC_OK with the answer, or
    TKC_ECANCELED (no answer, stats filled) when the search cap was met;
    other errors raise."""
    n_out = ctypes.c_int32(0)
    st = tkc_stats()
    rc = lib.tkc_topk_closeness_budget(g, k, variant, max_searches, _ptr(ids), _ptr(sum_dist), _ptr(reach),
                                       _ptr(farness), ctypes.byref(n_out), ctypes.byref(st))
    if rc not in (TKC_OK, TKC_ECANCELED):
        _check(rc)
    return rc, n_out.value, st


def tkc_graph_reach(g, alpha, omega, scc=None):
    _check(lib.tkc_graph_reach(g, _ptr(alpha), _ptr(omega), _ptr(scc)))


def tkc_graph_reach_info(g):
    path = ctypes.c_int32(0)
    ms = ctypes.c_double(0)
    _check(lib.tkc_graph_reach_info(g, ctypes.byref(path), ctypes.byref(ms)))
    return path.value, ms.value


def tkc_graph_reach_noalloc(g, alpha, omega, scc=None):
    """alpha, omega, scc: device tensors (int64, int64, int32) of n entries."""
    _check(lib.tkc_graph_reach_noalloc(g, _ptr(alpha), _ptr(omega), _ptr(scc)))


def tkc_graph_bounds(g, variant, num, den, order=None):
    _check(lib.tkc_graph_bounds(g, variant, _ptr(num), _ptr(den), _ptr(order)))


def tkc_graph_lb_update(g, sources, num, den):
    _check(lib.tkc_graph_lb_update(g, _ptr(sources), len(sources), _ptr(num), _ptr(den)))


def tkc_graph_sums(g, sources, S, R):
    _check(lib.tkc_graph_sums(g, _ptr(sources), len(sources), _ptr(S), _ptr(R)))


def tkc_server_create(ctx, hbm_budget_bytes, max_inflight):
    h = ctypes.c_void_p()
    _check(lib.tkc_server_create(ctx, hbm_budget_bytes, max_inflight, ctypes.byref(h)))
    return h


def tkc_server_add_graph(s, g):
    gid = ctypes.c_int32(0)
    _check(lib.tkc_server_add_graph(s, g, ctypes.byref(gid)))
    return gid.value


def tkc_server_submit(s, graph_id, k, variant=TKC_AUTO):
    t = ctypes.c_uint64(0)
    _check(lib.tkc_server_submit(s, graph_id, k, variant, ctypes.byref(t)))
    return t.value


def tkc_server_poll(s, ticket):
    d = ctypes.c_int32(0)
    _check(lib.tkc_server_poll(s, ticket, ctypes.byref(d)))
    return bool(d.value)


def tkc_server_result(s, ticket, ids, sum_dist=None, reach=None, farness=None):
    n_out = ctypes.c_int32(0)
    lat = ctypes.c_double(0)
    _check(lib.tkc_server_result(s, ticket, _ptr(ids), _ptr(sum_dist), _ptr(reach), _ptr(farness),
                                 ctypes.byref(n_out), ctypes.byref(lat)))
    return n_out.value, lat.value


def tkc_server_cancel(s, ticket):
    _check(lib.tkc_server_cancel(s, ticket))


def tkc_server_destroy(s):
    _check(lib.tkc_server_destroy(s))


def tkc_last_error() -> str:
    return lib.tkc_last_error().decode()


def tkc_version() -> str:
    return lib.tkc_version().decode()


# ------------------------------------------------------------ convenience
class Context:
    def __init__(self, device=0, stream=None):
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:
                stream = None
        self.h = tkc_ctx_create(device, stream)

    def tune(self, **kw):
        tkc_ctx_set_tuning(self.h, **kw)

    def tuning(self) -> dict:
        return tkc_ctx_get_tuning(self.h)

    def close(self):
        if self.h:
            tkc_ctx_destroy(self.h)
            self.h = None


class Graph:
    """A graph resident on the device (CSR copied at construction)."""

    def __init__(self, ctx: Context, n, row_ptr, col_idx, rrow_ptr=None, rcol_idx=None,
                 validate=False, device_ptrs=False, reverse=False, relabel=False):
        row_ptr = _as_i32(row_ptr)
        col_idx = _as_i32(col_idx)
        flags = (TKC_DIRECTED if rrow_ptr is not None else 0) | (TKC_VALIDATE if validate else 0)
        # device tensors (torch on the GPU) are copied device to device
        if device_ptrs or getattr(row_ptr, "is_cuda", False):
            flags |= TKC_DEVICE_PTRS
        if reverse:
            flags |= TKC_REVERSE
        if relabel:
            flags |= TKC_RELABEL
        if rrow_ptr is not None:
            rrow_ptr, rcol_idx = _as_i32(rrow_ptr), _as_i32(rcol_idx)
        self.n = int(n)
        self.m = int(col_idx.shape[0])
        self.directed = rrow_ptr is not None
        self._keep = (row_ptr, col_idx, rrow_ptr, rcol_idx)
        self.h = tkc_graph_upload(ctx.h, self.n, self.m, row_ptr, col_idx, rrow_ptr, rcol_idx, flags)

    @classmethod
    def from_csr(cls, ctx, row_ptr, col_idx, rrow_ptr=None, rcol_idx=None, validate=False, reverse=False,
                 relabel=False):
        """From int32 CSR arrays (numpy, or torch tensors on the host or the
        GPU); the reverse CSR is given iff the graph is directed."""
        return cls(ctx, len(row_ptr) - 1, row_ptr, col_idx, rrow_ptr, rcol_idx, validate=validate, reverse=reverse,
                   relabel=relabel)

    @classmethod
    def from_graphgen(cls, ctx, g, validate=False, reverse=False, relabel=False):
        return cls(ctx, g.n, g.row_ptr, g.col_idx, g.rrow_ptr, g.rcol_idx, validate=validate, reverse=reverse,
                   relabel=relabel)

    def free(self):
        if self.h:
            tkc_graph_free(self.h)
            self.h = None

    def autotune(self, k, variant="auto", budget_ms=10000.0):
        return tkc_autotune(self.h, k, variant, budget_ms)

    def reach(self):
        a = np.zeros(self.n, np.int64)
        o = np.zeros(self.n, np.int64)
        s = np.zeros(self.n, np.int32)
        tkc_graph_reach(self.h, a, o, s)
        return a, o, (s if self.directed else None)

    def reach_info(self):
        """(path, ms): 0 not computed yet, 1 the parallel device steps, 2 with
        the one-thread device pass for long chains."""
        return tkc_graph_reach_info(self.h)

    def harmonic_bounds(self, variant):
        """(upper bounds with the search's margin, processing order)."""
        ub = np.zeros(self.n, np.float64)
        order = np.zeros(self.n, np.int32)
        tkc_graph_harmonic_bounds(self.h, VARIANTS.get(variant, variant), ub, order)
        return ub, order

    def harmonic_lb_update(self, sources, ub):
        ub = np.ascontiguousarray(ub, dtype=np.float64).copy()
        tkc_graph_harmonic_lb_update(self.h, np.ascontiguousarray(sources, dtype=np.int32), ub)
        return ub

    def bounds(self, variant):
        num = np.zeros(self.n, np.int64)
        den = np.zeros(self.n, np.int64)
        order = np.zeros(self.n, np.int32)
        tkc_graph_bounds(self.h, VARIANTS.get(variant, variant), num, den, order)
        return num, den, order

    def lb_update(self, sources, num, den):
        num = np.ascontiguousarray(num, dtype=np.int64).copy()
        den = np.ascontiguousarray(den, dtype=np.int64).copy()
        tkc_graph_lb_update(self.h, np.ascontiguousarray(sources, dtype=np.int32), num, den)
        return num, den

    def sums(self, sources):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        S = np.zeros(max(1, src.size), np.int64)
        R = np.zeros(max(1, src.size), np.int64)
        if src.size:
            tkc_graph_sums(self.h, src, S, R)
        return S[: src.size], R[: src.size]


def tkc_pack_create(ctx, graph_handles):
    arr = (ctypes.c_void_p * len(graph_handles))(*[h.value for h in graph_handles])
    h = ctypes.c_void_p()
    _check(lib.tkc_pack_create(ctx, arr, len(graph_handles), ctypes.byref(h)))
    return h


def tkc_pack_topk(p, members, ks, variant, ids, sum_dist, reach, farness, n_out):
    st = tkc_stats()
    _check(lib.tkc_pack_topk(p, len(members), _ptr(members), _ptr(ks), variant, _ptr(ids), _ptr(sum_dist),
                             _ptr(reach), _ptr(farness), _ptr(n_out), ctypes.byref(st)))
    return st


def tkc_pack_free(p):
    _check(lib.tkc_pack_free(p))


class Pack:
    """Several resident graphs whose top-k requests share one batched launch."""

    def __init__(self, ctx: Context, graphs):
        self.graphs = list(graphs)
        self.h = tkc_pack_create(ctx.h, [g.h for g in self.graphs])

    def topk(self, members, ks, variant="nbcut"):
        """Requests (members[i], ks[i]) on distinct members: a list of (ids, S,
        r, farness) per request, and the launch's stats."""
        members = np.ascontiguousarray(members, dtype=np.int32)
        ks = np.ascontiguousarray(ks, dtype=np.int32)
        tot = int(sum(min(int(k), self.graphs[int(m)].n) for m, k in zip(members, ks)))
        ids = np.zeros(max(1, tot), np.int32)
        S = np.zeros(max(1, tot), np.int64)
        R = np.zeros(max(1, tot), np.int64)
        F = np.zeros(max(1, tot), np.float64)
        n_out = np.zeros(len(members), np.int32)
        st = tkc_pack_topk(self.h, members, ks, VARIANTS.get(variant, variant), ids, S, R, F, n_out)
        out, o = [], 0
        for c in n_out.tolist():
            out.append((ids[o:o + c], S[o:o + c], R[o:o + c], F[o:o + c]))
            o += c
        return out, st.as_dict()

    def close(self):
        if self.h:
            tkc_pack_free(self.h)
            self.h = None


def tkc_server_enable_packing(s, max_vertices):
    _check(lib.tkc_server_enable_packing(s, int(max_vertices)))


def tkc_server_info(s):
    a, b, c2 = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    d = ctypes.c_int32(0)
    _check(lib.tkc_server_info(s, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c2), ctypes.byref(d)))
    return {"served": a.value, "packed": b.value, "pack_calls": c2.value, "packs": d.value}


class Server:
    """Request server over resident graphs (continuous batching)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_inflight: int = 4):
        self.h = tkc_server_create(ctx.h, int(hbm_budget_bytes), int(max_inflight))
        self.graphs = []

    def add(self, g: "Graph") -> int:
        gid = tkc_server_add_graph(self.h, g.h)
        self.graphs.append(g)
        return gid

    def enable_packing(self, max_vertices: int):
        """Serve requests on graphs of at most max_vertices vertices in
        packed launches (0 turns packing off)."""
        tkc_server_enable_packing(self.h, max_vertices)

    def info(self) -> dict:
        return tkc_server_info(self.h)

    def submit(self, graph_id: int, k: int, variant="auto") -> int:
        return tkc_server_submit(self.h, int(graph_id), int(k), VARIANTS.get(variant, variant))

    def poll(self, ticket: int) -> bool:
        return tkc_server_poll(self.h, ticket)

    def result(self, ticket: int, k: int):
        """(ids, S, r, farness, latency_ms); blocks until the request is done."""
        ids = np.zeros(max(1, k), np.int32)
        S = np.zeros(max(1, k), np.int64)
        r = np.zeros(max(1, k), np.int64)
        f = np.zeros(max(1, k), np.float64)
        c, lat = tkc_server_result(self.h, ticket, ids, S, r, f)
        return ids[:c], S[:c], r[:c], f[:c], lat

    def cancel(self, ticket: int):
        tkc_server_cancel(self.h, ticket)

    def close(self):
        if self.h:
            tkc_server_destroy(self.h)
            self.h = None


def _as_i32(a):
    if isinstance(a, np.ndarray):
        return np.ascontiguousarray(a, dtype=np.int32)
    return a   # torch tensor (host or device), int32 and contiguous


def topk_closeness(g: Graph, k: int, variant="auto", mode="hybrid"):
    """(ids int32, S int64, r int64, farness float64, stats) of the top min(k, n)."""
    kk = min(int(k), g.n) if k > 0 else k
    cap = max(1, kk)
    ids = np.zeros(cap, np.int32)
    S = np.zeros(cap, np.int64)
    R = np.zeros(cap, np.int64)
    F = np.zeros(cap, np.float64)
    n_out, st = tkc_topk_closeness(g.h, int(k), VARIANTS.get(variant, variant), MODES.get(mode, mode),
                                   ids, S, R, F)
    return ids[:n_out], S[:n_out], R[:n_out], F[:n_out], st.as_dict()


def topk_closeness_budget(g: Graph, k: int, variant="auto", max_searches=1000):
    """Plain mode with at most max_searches searches: (finished, result,
    stats) where result is (ids, S, r, farness) when finished, else None."""
    cap = max(1, min(int(k), g.n))
    ids = np.zeros(cap, np.int32)
    S = np.zeros(cap, np.int64)
    R = np.zeros(cap, np.int64)
    F = np.zeros(cap, np.float64)
    rc, n_out, st = tkc_topk_closeness_budget(g.h, int(k), VARIANTS.get(variant, variant), int(max_searches),
                                              ids, S, R, F)
    if rc == TKC_OK:
        return True, (ids[:n_out], S[:n_out], R[:n_out], F[:n_out]), st.as_dict()
    return False, None, st.as_dict()


def tkc_topk_harmonic(g, k, variant, mode, ids, harmonic):
    n_out = ctypes.c_int32(0)
    st = tkc_stats()
    _check(lib.tkc_topk_harmonic(g, k, variant, mode, _ptr(ids), _ptr(harmonic), ctypes.byref(n_out),
                                 ctypes.byref(st)))
    return n_out.value, st


def tkc_graph_harmonic_bounds(g, variant, ub, order=None):
    _check(lib.tkc_graph_harmonic_bounds(g, variant, _ptr(ub), _ptr(order)))


def tkc_graph_harmonic_lb_update(g, sources, ub):
    _check(lib.tkc_graph_harmonic_lb_update(g, _ptr(sources), len(sources), _ptr(ub)))


def topk_harmonic(g: Graph, k: int, variant="auto", mode="batched"):
    """(ids int32, harmonic float64, stats) of the top min(k, n) by harmonic
    centrality, larger first, ties to the smaller id."""
    cap = max(1, min(int(k), g.n) if k > 0 else 1)
    ids = np.zeros(cap, np.int32)
    h = np.zeros(cap, np.float64)
    n_out, st = tkc_topk_harmonic(g.h, int(k), VARIANTS.get(variant, variant), MODES.get(mode, mode), ids, h)
    return ids[:n_out], h[:n_out], st.as_dict()


def topk_closeness_ties(g: Graph, k: int, variant="auto", mode="hybrid", cap=None):
    """Top k with every vertex tied with the k-th: (ids, S, r, farness, stats).
    Retries once with the capacity the library reports when cap is short."""
    kk = min(int(k), g.n)
    cap = max(kk, int(cap) if cap else kk + 64)
    for _ in range(2):
        ids = np.zeros(cap, np.int32)
        S = np.zeros(cap, np.int64)
        R = np.zeros(cap, np.int64)
        F = np.zeros(cap, np.float64)
        rc, n_out, st = tkc_topk_closeness_ties(g.h, int(k), VARIANTS.get(variant, variant), MODES.get(mode, mode),
                                                cap, ids, S, R, F)
        if rc == TKC_OK:
            return ids[:n_out], S[:n_out], R[:n_out], F[:n_out], st.as_dict()
        cap = n_out
    raise TkcError(TKC_EINVAL, "tie output did not fit")
