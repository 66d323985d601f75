"""Write the exact top-100 of the full-size and medium workloads.

Every value written here comes from the oracle alone: the all-sources
textbook breadth-first search of the introduction (Sect. 1) gives S(v) and
r(v) for every vertex, and the exact order of Lin's index (Sect. 2, Eq. 1:
farness (n-1) S / (r-1)^2 ascending, the smaller id winning an exact tie)
picks the first 100.  Alg. 1 reaches exactly this answer (Sect. 4), so the
device's top-k must equal a prefix of it.  For the medium graphs the
harmonic centrality (Sect. 2 with f(d) = 1/d, in the oracle's binary64
reading) is written too.

Usage:
    python tests/golden/make_full.py --cache DIR [--threads T] [--harmonic] NAME...

The per-chunk (S, r) arrays go to DIR/<graph digest>/, so an interrupted
run resumes where it stopped.  The result is tests/golden/full_<NAME>.txt
(and full_<NAME>_harmonic.txt), keyed by the graph digest that the tests
check before they compare.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

TOP = 100
CHUNK = 32768


def all_sources(g, cache, threads, harmonic):
    d = os.path.join(cache, g.digest())
    os.makedirs(d, exist_ok=True)
    nchunks = (g.n + CHUNK - 1) // CHUNK
    S = np.zeros(g.n, np.int64)
    r = np.zeros(g.n, np.int64)
    h = np.zeros(g.n, np.float64) if harmonic else None
    t0 = time.time()
    for c in range(nchunks):
        lo, hi = c * CHUNK, min(g.n, (c + 1) * CHUNK)
        f = os.path.join(d, "sums_%05d.npz" % c)
        if not os.path.exists(f):
            src = np.arange(lo, hi, dtype=np.int32)
            cs, cr = oracle.sums(g.n, g.edges, g.directed, sources=src, nthreads=threads)
            np.savez(f + ".tmp.npz", S=cs, r=cr)
            os.replace(f + ".tmp.npz", f)
        z = np.load(f)
        S[lo:hi], r[lo:hi] = z["S"], z["r"]
        if harmonic:
            fh = os.path.join(d, "harm_%05d.npy" % c)
            if not os.path.exists(fh):
                src = np.arange(lo, hi, dtype=np.int32)
                np.save(fh + ".tmp.npy", oracle.harmonic(g.n, g.edges, g.directed, sources=src,
                                                         nthreads=threads))
                os.replace(fh + ".tmp.npy", fh)
            h[lo:hi] = np.load(fh)
        print("%s chunk %d/%d done, %.0f s" % (g.name, c + 1, nchunks, time.time() - t0), flush=True)
    return S, r, h


def write(name, g, S, r, h):
    head = ["# %s: exact top-%d by closeness (Lin's index, Sect. 2 Eq. 1)" % (name, TOP),
            "# from the oracle's all-sources breadth-first search (Sect. 1); written by",
            "# tests/golden/make_full.py, which calls only the oracle and the seeded generators",
            "digest %s" % g.digest(),
            "n %d" % g.n,
            "arcs %d" % g.arcs,
            "directed %d" % int(g.directed),
            "sum_S %d" % int(S.sum()),
            "sum_r %d" % int(r.sum()),
            "# rank id S r"]
    ids = oracle.topk(S, r, TOP)
    rows = ["%d %d %d %d" % (i, v, S[v], r[v]) for i, v in enumerate(ids)]
    with open(os.path.join(HERE, "full_%s.txt" % name), "w") as fp:
        fp.write("\n".join(head + rows) + "\n")
    if h is not None:
        hid = oracle.harmonic_topk(h, TOP)
        head = ["# %s: exact top-%d by harmonic centrality (Sect. 2 with f(d) = 1/d)" % (name, TOP),
                "# in the oracle's binary64 reading, from its all-sources search; written by",
                "# tests/golden/make_full.py",
                "digest %s" % g.digest(),
                "n %d" % g.n,
                "# rank id h(hex)"]
        rows = ["%d %d %s" % (i, v, float(h[v]).hex()) for i, v in enumerate(hid)]
        with open(os.path.join(HERE, "full_%s_harmonic.txt" % name), "w") as fp:
            fp.write("\n".join(head + rows) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", required=True)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--harmonic", action="store_true")
    ap.add_argument("names", nargs="+")
    a = ap.parse_args()
    for name in a.names:
        g = graphgen.workload(name)
        S, r, h = all_sources(g, a.cache, a.threads, a.harmonic)
        write(name, g, S, r, h)
        print("wrote", name, flush=True)


if __name__ == "__main__":
    main()
