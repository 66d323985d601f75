/*
 * ORACLE -- test infrastructure only.  Plain, slow, obviously correct CPU
 * reference for exact top-k closeness (Bergamini, Borassi, Crescenzi,
 * Marino, Meyerhenke, "Computing top-k Closeness Centrality Faster in
 * Unweighted Graphs").  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this file's library; the GPU product path
 * never does.  It shares no code with the GPU path or the input generators:
 * it builds its own adjacency from the raw edge list.
 *
 * What it computes, and the passage each part follows:
 *
 *  - Distances: one FIFO breadth-first search per source (the textbook
 *    algorithm of the introduction, Sect. 1).  S(v) = sum of d(v,w) over the
 *    vertices w reachable from v, r(v) = number of reachable vertices with v
 *    itself counted (Table 1, "Reachability set function").
 *  - Farness (Sect. 2, Eq. 1, Lin's index):
 *        f(v) = (n-1) S(v) / (r(v)-1)^2  for r(v) >= 2,
 *        f(v) = +inf (closeness 0) when v reaches nothing else (r(v) = 1).
 *  - Order: v precedes w iff f(v) < f(w), or f(v) = f(w) and v < w (the
 *    smaller id wins an exact tie; Sect. 4 returns every tied vertex, this
 *    library returns exactly min(k, n)).  f is compared as an exact
 *    rational: S(v)(r(w)-1)^2 against S(w)(r(v)-1)^2 in unsigned 128-bit
 *    arithmetic (n-1 cancels).
 *  - Reported double: ((double)(n-1) * (double)S) / ((double)(r-1) * (double)(r-1)),
 *    IEEE binary64 round-to-nearest, +inf when r = 1.
 *
 * Reference implementations of the lower bounds (used to pin the bound
 * kernels bit for bit and to check that every bound stays below the exact
 * farness), each taking the paper's steps in the paper's order:
 *  - oracle_nb:      neighbourhood-based bound, Sect. 5 (Prop. 5.1, Eq. 2,
 *                    Alg. 3, directed Eq. 3) and the disconnected form of
 *                    Sect. 8.1 (Eq. nblbdisc).
 *  - oracle_cut_levels: the BFSCut bound of Sect. 6 (Lemma 6.1 and its
 *                    corollary) at every level boundary; disconnected
 *                    directed graphs via Lemma 8.1 / Sect. 8.2.
 *  - oracle_lb_source: the level-based bound of Sect. 7 (Eq. 4, Lemma 7.2,
 *                    Alg. 5; directed Eq. 5, same-SCC rule of Sect. 8.3).
 *  - oracle_alpha_omega: reachability bounds of Sect. 8.4 (Alg. 6).
 *  - oracle_harmonic: harmonic centrality, the measure of Sect. 2 with
 *                    f(d) = 1/d that Sect. 9.1 also ranks.
 * Readings taken where the text is silent or garbled are listed at each
 * function.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ------------------------------------------------------------ adjacency */
typedef struct {
    int32_t n;
    int64_t *off;   /* n+1 */
    int32_t *nbr;   /* off[n] */
} oadj;

static int cmp_int(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Out-adjacency (reverse=0) or in-adjacency (reverse=1) of the simple graph
 * given by an edge list: self-loops ignored, repeated arcs kept once, an
 * undirected edge {u,v} gives arcs u->v and v->u. */
static int adj_build(int32_t n, int64_t ne, const int32_t *ed, int directed, int reverse, oadj *A) {
    A->n = n;
    A->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!A->off) return -1;
    for (int64_t e = 0; e < ne; e++) {
        int32_t u = ed[2 * e], v = ed[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n) return -2;
        if (u == v) continue;
        if (!directed) { A->off[u + 1]++; A->off[v + 1]++; }
        else if (!reverse) A->off[u + 1]++;
        else A->off[v + 1]++;
    }
    for (int32_t i = 0; i < n; i++) A->off[i + 1] += A->off[i];
    int64_t tot = A->off[n];
    A->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot ? tot : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, A->off, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < ne; e++) {
        int32_t u = ed[2 * e], v = ed[2 * e + 1];
        if (u == v) continue;
        if (!directed) { A->nbr[fill[u]++] = v; A->nbr[fill[v]++] = u; }
        else if (!reverse) A->nbr[fill[u]++] = v;
        else A->nbr[fill[v]++] = u;
    }
    free(fill);
    /* sort each list and squeeze out repeats */
    int64_t w = 0;
    int64_t start = 0;
    for (int32_t i = 0; i < n; i++) {
        int64_t a = start, b = A->off[i + 1];
        qsort(A->nbr + a, (size_t)(b - a), sizeof(int32_t), cmp_int);
        A->off[i] = w;
        for (int64_t q = a; q < b; q++)
            if (q == a || A->nbr[q] != A->nbr[q - 1]) A->nbr[w++] = A->nbr[q];
        start = b;
    }
    A->off[n] = w;
    return 0;
}
static void adj_free(oadj *A) { free(A->off); free(A->nbr); }

/* 0 if the given CSR equals the oracle's own adjacency of the edge list. */
int oracle_check_csr(int32_t n, int64_t ne, const int32_t *ed, int directed, int reverse,
                     const int32_t *row_ptr, const int32_t *col_idx) {
    oadj A;
    if (adj_build(n, ne, ed, directed, reverse, &A)) return -1;
    int bad = 0;
    for (int32_t i = 0; i <= n && !bad; i++) if ((int64_t)row_ptr[i] != A.off[i]) bad = 1;
    for (int64_t q = 0; q < A.off[n] && !bad; q++) if (col_idx[q] != A.nbr[q]) bad = 2;
    adj_free(&A);
    return bad;
}

/* ------------------------------------------------- textbook BFS (Sect. 1) */
/* One FIFO breadth-first search from s: returns S(s) and writes r(s).
 * The queue holds the vertices in the order they are found, so it is the
 * levels one after the other: queue[0] = s is level 0, and while level d is
 * being expanded every vertex appended belongs to level d + 1.  S adds d
 * once per vertex of level d.  seen[] is a bitmap of n bits, all clear on
 * entry and cleared again on exit; queue holds n entries.  The two
 * prefetches only warm the cache for rows a few entries ahead in the queue
 * and change nothing computed. */
static int64_t bfs_sum(const oadj *A, int32_t s, uint64_t *seen, int32_t *queue, int64_t *r_out) {
    int64_t head = 0, tail = 0, S = 0, d = 0;
    seen[s >> 6] |= 1ull << (s & 63);
    queue[tail++] = s;
    while (head < tail) {
        int64_t level_end = tail;   /* queue[head, level_end) is level d */
        while (head < level_end) {
            if (head + 16 < tail) __builtin_prefetch(&A->off[queue[head + 16]]);
            if (head + 6 < tail) __builtin_prefetch(&A->nbr[A->off[queue[head + 6]]]);
            int32_t u = queue[head++];
            for (int64_t q = A->off[u]; q < A->off[u + 1]; q++) {
                int32_t w = A->nbr[q];
                uint64_t bit = 1ull << (w & 63);
                if (!(seen[w >> 6] & bit)) { seen[w >> 6] |= bit; queue[tail++] = w; }
            }
        }
        d++;
        S += d * (tail - level_end);   /* the vertices just appended are at distance d */
    }
    for (int64_t q = 0; q < tail; q++) seen[queue[q] >> 6] = 0;
    *r_out = tail;
    return S;
}

/* S and r for every source in src[0..ns) (src == NULL: all n vertices). */
int oracle_sums(int32_t n, int64_t ne, const int32_t *ed, int directed,
                const int32_t *src, int64_t ns, int64_t *S, int64_t *r, int nthreads) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int64_t cnt = src ? ns : n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    #pragma omp parallel
    {
        uint64_t *seen = (uint64_t *)calloc(((size_t)n + 63) / 64 + 1, sizeof(uint64_t));
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < cnt; i++) {
            int32_t s = src ? src[i] : (int32_t)i;
            S[i] = bfs_sum(&A, s, seen, queue, &r[i]);
        }
        free(seen); free(queue);
    }
    adj_free(&A);
    return 0;
}

/* ------------------------------------ harmonic centrality (Sect. 2, 9.1) */
/* h(v) = sum over the vertices w != v that v reaches of 1/d(v,w): the
 * centrality of the form sum f(d(v,w)) with f(d) = 1/d, f(inf) = 0.
 * Larger is more central; an exact tie goes to the smaller id.
 * Reading (the paper fixes no precision): h is the IEEE binary64 value of
 *     sum over d = 1, 2, ..., ecc(v) of  (double)n_d / (double)d,
 * n_d the number of vertices at distance exactly d, each quotient rounded
 * to nearest and the terms added in increasing d, rounding to nearest after
 * each addition.  It differs from the exact rational by at most ecc(v)
 * units in the last place. */
static double bfs_harmonic(const oadj *A, int32_t s, int32_t *dist, int32_t *queue) {
    int64_t head = 0, tail = 0;
    dist[s] = 0; queue[tail++] = s;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t q = A->off[u]; q < A->off[u + 1]; q++) {
            int32_t w = A->nbr[q];
            if (dist[w] < 0) { dist[w] = dist[u] + 1; queue[tail++] = w; }
        }
    }
    /* a FIFO search emits the vertices in nondecreasing distance: the queue
     * is the levels one after the other */
    double h = 0.0;
    int64_t q = 1;
    while (q < tail) {
        int32_t d = dist[queue[q]];
        int64_t nd = 0;
        while (q < tail && dist[queue[q]] == d) { nd++; q++; }
        h += (double)nd / (double)d;
    }
    for (int64_t i = 0; i < tail; i++) dist[queue[i]] = -1;
    return h;
}

int oracle_harmonic(int32_t n, int64_t ne, const int32_t *ed, int directed,
                    const int32_t *src, int64_t ns, double *h, int nthreads) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int64_t cnt = src ? ns : n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    #pragma omp parallel
    {
        int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
        for (int32_t i = 0; i < n; i++) dist[i] = -1;
        #pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < cnt; i++) {
            int32_t s = src ? src[i] : (int32_t)i;
            h[i] = bfs_harmonic(&A, s, dist, queue);
        }
        free(dist); free(queue);
    }
    adj_free(&A);
    return 0;
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* number of arcs each BFS scans: sum of out-degrees over R(s) */
int64_t oracle_arcs(int32_t n, int64_t ne, const int32_t *ed, int directed) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int64_t m = A.off[n];
    adj_free(&A);
    return m;
}

/* ------------------------------------------------- exact farness order */
/* sign of f(a) - f(b) with f = S/(r-1)^2, +inf when r <= 1 */
static int farn_cmp(int64_t Sa, int64_t ra, int64_t Sb, int64_t rb) {
    int ia = ra <= 1, ib = rb <= 1;
    if (ia || ib) return ia - ib;
    u128 da = (u128)(uint64_t)(ra - 1) * (uint64_t)(ra - 1);
    u128 db = (u128)(uint64_t)(rb - 1) * (uint64_t)(rb - 1);
    u128 x = (u128)(uint64_t)Sa * db, y = (u128)(uint64_t)Sb * da;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* merge sort of ids by (f, id); stable and self-contained */
static const int64_t *g_S, *g_r;
static int prec(int32_t a, int32_t b) {
    int c = farn_cmp(g_S[a], g_r[a], g_S[b], g_r[b]);
    return c < 0 || (c == 0 && a < b);
}
static void msort(int32_t *x, int32_t *t, int64_t len) {
    if (len < 2) return;
    int64_t h = len / 2;
    msort(x, t, h); msort(x + h, t, len - h);
    int64_t i = 0, j = h, o = 0;
    while (i < h && j < len) t[o++] = prec(x[j], x[i]) ? x[j++] : x[i++];
    while (i < h) t[o++] = x[i++];
    while (j < len) t[o++] = x[j++];
    memcpy(x, t, sizeof(int32_t) * (size_t)len);
}

/* the first min(k, n) vertices under the exact order; returns the count */
int32_t oracle_topk(int32_t n, const int64_t *S, const int64_t *r, int32_t k, int32_t *ids) {
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *t = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int32_t i = 0; i < n; i++) x[i] = i;
    g_S = S; g_r = r;
    msort(x, t, n);
    int32_t c = k < n ? k : n;
    if (c < 0) c = 0;
    memcpy(ids, x, sizeof(int32_t) * (size_t)c);
    free(x); free(t);
    return c;
}

int oracle_cmp(int64_t Sa, int64_t ra, int64_t Sb, int64_t rb) { return farn_cmp(Sa, ra, Sb, rb); }

double oracle_farness(int32_t n, int64_t S, int64_t r) {
    if (r <= 1) return __builtin_inf();
    return ((double)(n - 1) * (double)S) / ((double)(r - 1) * (double)(r - 1));
}

/* ------------------------------------------- brute force distances (pin) */
/* Floyd-Warshall over the adjacency; dist[i*n+j] = -1 when unreachable */
int oracle_floyd_warshall(int32_t n, int64_t ne, const int32_t *ed, int directed, int32_t *dist) {
    const int32_t INF = 1 << 29;
    for (int64_t i = 0; i < (int64_t)n * n; i++) dist[i] = INF;
    for (int32_t i = 0; i < n; i++) dist[(int64_t)i * n + i] = 0;
    for (int64_t e = 0; e < ne; e++) {
        int32_t u = ed[2 * e], v = ed[2 * e + 1];
        if (u == v) continue;
        dist[(int64_t)u * n + v] = 1;
        if (!directed) dist[(int64_t)v * n + u] = 1;
    }
    for (int32_t k = 0; k < n; k++)
        for (int32_t i = 0; i < n; i++)
            for (int32_t j = 0; j < n; j++) {
                int32_t c = dist[(int64_t)i * n + k] + dist[(int64_t)k * n + j];
                if (c < dist[(int64_t)i * n + j]) dist[(int64_t)i * n + j] = c;
            }
    for (int64_t i = 0; i < (int64_t)n * n; i++) if (dist[i] >= INF) dist[i] = -1;
    return 0;
}

/* ---------------------------------------------- connected components */
/* undirected: size of each vertex's component (= r(v), Sect. 4) */
int oracle_component_sizes(int32_t n, int64_t ne, const int32_t *ed, int64_t *size) {
    oadj A;
    if (adj_build(n, ne, ed, 0, 0, &A)) return -1;
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int32_t i = 0; i < n; i++) lab[i] = -1;
    for (int32_t s = 0; s < n; s++) {
        if (lab[s] >= 0) continue;
        int64_t h = 0, t = 0;
        lab[s] = s; queue[t++] = s;
        while (h < t) {
            int32_t u = queue[h++];
            for (int64_t q = A.off[u]; q < A.off[u + 1]; q++)
                if (lab[A.nbr[q]] < 0) { lab[A.nbr[q]] = s; queue[t++] = A.nbr[q]; }
        }
        for (int64_t q = 0; q < t; q++) size[queue[q]] = t;
    }
    free(lab); free(queue); adj_free(&A);
    return 0;
}

/* --------------------------------------- SCCs and alpha/omega (Sect. 8.4) */
/*
 * Strongly connected components by Kosaraju's two passes (iterative DFS):
 * finishing order on G, then components on the reverse graph in decreasing
 * finishing time.  Components come out numbered in a topological order of
 * the component DAG (a component's number is smaller than those of every
 * component it reaches).
 */
static int32_t scc_kosaraju(const oadj *G, const oadj *R, int32_t *comp) {
    int32_t n = G->n;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *stk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *it = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    char *seen = (char *)calloc((size_t)(n ? n : 1), 1);
    int32_t no = 0;
    for (int32_t s = 0; s < n; s++) {
        if (seen[s]) continue;
        int32_t sp = 0;
        stk[sp++] = s; seen[s] = 1; it[s] = G->off[s];
        while (sp) {
            int32_t u = stk[sp - 1];
            if (it[u] < G->off[u + 1]) {
                int32_t w = G->nbr[it[u]++];
                if (!seen[w]) { seen[w] = 1; it[w] = G->off[w]; stk[sp++] = w; }
            } else { order[no++] = u; sp--; }
        }
    }
    for (int32_t i = 0; i < n; i++) comp[i] = -1;
    int32_t nc = 0;
    for (int32_t q = n - 1; q >= 0; q--) {
        int32_t s = order[q];
        if (comp[s] >= 0) continue;
        int32_t sp = 0;
        stk[sp++] = s; comp[s] = nc;
        while (sp) {
            int32_t u = stk[--sp];
            for (int64_t e = R->off[u]; e < R->off[u + 1]; e++) {
                int32_t w = R->nbr[e];
                if (comp[w] < 0) { comp[w] = nc; stk[sp++] = w; }
            }
        }
        nc++;
    }
    free(order); free(stk); free(it); free(seen);
    return nc;
}

int32_t oracle_scc(int32_t n, int64_t ne, const int32_t *ed, int32_t *comp) {
    oadj G, R;
    if (adj_build(n, ne, ed, 1, 0, &G) || adj_build(n, ne, ed, 1, 1, &R)) return -1;
    int32_t nc = scc_kosaraju(&G, &R, comp);
    adj_free(&G); adj_free(&R);
    return nc;
}

/*
 * Alg. 6 (Sect. 8.4): alpha(C) = w(C) + the largest alpha of C's successors,
 * omega(C) = w(C) + the sum of their omegas, taken sinks first, with the
 * largest SCC's reach counted exactly.  For a component that reaches the
 * largest SCC, omega sums only the successors that the largest SCC does not
 * reach and then adds the largest SCC's reach once.
 * Readings: the pseudocode's reachability test inside the successor loop
 * names a variable that is never bound; it is read as a test on the
 * successor being examined.  The largest SCC's ties go to the component
 * holding the smallest vertex id.  The successors' omegas are taken as
 * computed (a successor that itself reaches the largest SCC already holds
 * that SCC's reach, so it can be counted twice; the bound stays valid), and
 * every omega is capped at n after it is formed, since r <= n always holds.
 * tests/golden/alg6_*.txt work three small digraphs out by hand.
 */
int oracle_alpha_omega(int32_t n, int64_t ne, const int32_t *ed, int64_t *alpha, int64_t *omega,
                       int32_t *scc_out) {
    oadj G, R;
    if (adj_build(n, ne, ed, 1, 0, &G) || adj_build(n, ne, ed, 1, 1, &R)) return -1;
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t nc = scc_kosaraju(&G, &R, comp);
    int64_t *wt = (int64_t *)calloc((size_t)(nc ? nc : 1), sizeof(int64_t));
    int32_t *minid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc ? nc : 1));
    for (int32_t c = 0; c < nc; c++) minid[c] = n;
    for (int32_t v = 0; v < n; v++) { wt[comp[v]]++; if (v < minid[comp[v]]) minid[comp[v]] = v; }
    int32_t big = 0;
    for (int32_t c = 1; c < nc; c++)
        if (wt[c] > wt[big] || (wt[c] == wt[big] && minid[c] < minid[big])) big = c;
    /* component DAG: successor lists (deduplicated) */
    int64_t *doff = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    for (int32_t u = 0; u < n; u++)
        for (int64_t e = G.off[u]; e < G.off[u + 1]; e++)
            if (comp[G.nbr[e]] != comp[u]) doff[comp[u] + 1]++;
    for (int32_t c = 0; c < nc; c++) doff[c + 1] += doff[c];
    int32_t *dnb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(doff[nc] ? doff[nc] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nc + 1));
    memcpy(fill, doff, sizeof(int64_t) * ((size_t)nc + 1));
    for (int32_t u = 0; u < n; u++)
        for (int64_t e = G.off[u]; e < G.off[u + 1]; e++)
            if (comp[G.nbr[e]] != comp[u]) dnb[fill[comp[u]]++] = comp[G.nbr[e]];
    /* dedup each successor list */
    int64_t w = 0, st = 0;
    for (int32_t c = 0; c < nc; c++) {
        int64_t a = st, b = doff[c + 1];
        qsort(dnb + a, (size_t)(b - a), sizeof(int32_t), cmp_int);
        doff[c] = w;
        for (int64_t q = a; q < b; q++) if (q == a || dnb[q] != dnb[q - 1]) dnb[w++] = dnb[q];
        st = b;
    }
    doff[nc] = w;
    /* components reachable from C~ (forward) and able to reach C~ (backward):
     * numbering is topological, so one sweep each way suffices */
    char *from_big = (char *)calloc((size_t)(nc ? nc : 1), 1);
    char *to_big = (char *)calloc((size_t)(nc ? nc : 1), 1);
    from_big[big] = 1;
    for (int32_t c = big; c < nc; c++)
        if (from_big[c]) for (int64_t q = doff[c]; q < doff[c + 1]; q++) from_big[dnb[q]] = 1;
    to_big[big] = 1;
    for (int32_t c = big; c >= 0; c--)
        for (int64_t q = doff[c]; q < doff[c + 1]; q++) if (to_big[dnb[q]]) { to_big[c] = 1; break; }
    int64_t reach_big = 0;
    for (int32_t c = 0; c < nc; c++) if (from_big[c]) reach_big += wt[c];
    int64_t *aS = (int64_t *)calloc((size_t)(nc ? nc : 1), sizeof(int64_t));
    int64_t *oS = (int64_t *)calloc((size_t)(nc ? nc : 1), sizeof(int64_t));
    aS[big] = oS[big] = reach_big;
    for (int32_t c = nc - 1; c >= 0; c--) {          /* reverse topological */
        if (c == big) continue;
        int64_t a = 0, o = 0, o2 = 0;
        for (int64_t q = doff[c]; q < doff[c + 1]; q++) {
            int32_t y = dnb[q];
            if (aS[y] > a) a = aS[y];
            o += oS[y];
            if (!from_big[y]) o2 += oS[y];
        }
        if (to_big[c]) o = o2 + oS[big];
        a += wt[c]; o += wt[c];
        if (o > n) o = n;
        aS[c] = a; oS[c] = o;
    }
    for (int32_t v = 0; v < n; v++) {
        alpha[v] = aS[comp[v]]; omega[v] = oS[comp[v]];
        if (scc_out) scc_out[v] = comp[v];
    }
    free(comp); free(wt); free(minid); free(doff); free(dnb); free(fill);
    free(from_big); free(to_big); free(aS); free(oS);
    adj_free(&G); adj_free(&R);
    return 0;
}

/* ------------------------------------- neighbourhood-based bound (Sect. 5) */
#define NB_INF ((int64_t)1 << 62)
static inline int64_t sat_add(int64_t a, int64_t b) {
    int64_t s = a + b;   /* both operands are in [0, 2^62] */
    return s >= NB_INF ? NB_INF : s;
}
/* keep the smaller of (num, den) and (cn, cd); den > 0 */
static void rat_min(int64_t *num, int64_t *den, int64_t cn, int64_t cd) {
    if (*den == 0) { *num = cn; *den = cd; return; }
    u128 x = (u128)(uint64_t)cn * (uint64_t)(*den), y = (u128)(uint64_t)(*num) * (uint64_t)cd;
    if (x < y) { *num = cn; *den = cd; }
}

/*
 * Lower bound on the farness of every vertex from walk counts.
 * gamma_k(s) bounds the number of vertices at distance k from s:
 *   undirected (Eq. 2, the tree recurrence of Alg. 2/3):
 *     gamma_1(s) = deg(s),
 *     gamma_2(s) = sum_{w in N(s)} gamma_1(w) - deg(s),
 *     gamma_k(s) = sum_{w in N(s)} gamma_{k-1}(w) - (deg(s)-1) gamma_{k-2}(s), k >= 3;
 *   directed (Eq. 3): gamma_k(s) = sum over out-neighbours of gamma_{k-1}(w).
 * Prop. 5.1 turns them into a bound on S(s) by filling levels 1, 2, ...
 * with gamma_k vertices until r(s) vertices are placed.  With only
 * alpha(s) <= r(s) <= omega(s) known (Sect. 8.1) the farness bound is the
 * minimum of (n-1) S_NB(r)/(r-1)^2 over r in {alpha, omega} and over the
 * cumulative sums 1 + gamma_1 + ... + gamma_l lying strictly between them.
 * With r known pass alpha = omega = r.
 * Readings: the vertex that finishes keeps updating its gamma values (only
 * its sum and visited count stop), so neighbours always read current
 * counts; counts saturate at 2^62, which is treated as "at least that many";
 * when gamma_k(s) = 0 (all walks from s die out, possible in a directed
 * graph with omega(s) > r(s)) nothing lies at distance >= k, r(s) is at most
 * the visited count, and s finishes with the candidates already taken.
 * Output: farness bound = (n-1) * num / den, den = (r-1)^2 of the minimising
 * r; den = 0 encodes +inf (r = 1, nothing reachable).
 */
int oracle_nb(int32_t n, int64_t ne, const int32_t *ed, int directed,
              const int64_t *alpha, const int64_t *omega, int64_t *num, int64_t *den) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int64_t *g1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));   /* gamma_{k-1} */
    int64_t *g2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));   /* gamma_{k-2} */
    int64_t *gk = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *sum = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *vis = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    char *fin = (char *)malloc((size_t)(n ? n : 1));
    char *started = (char *)malloc((size_t)(n ? n : 1));
    int32_t nfin = 0;
    for (int32_t s = 0; s < n; s++) {
        int64_t d = A.off[s + 1] - A.off[s];
        g1[s] = d; g2[s] = 1;
        num[s] = 0; den[s] = 0; fin[s] = 0; started[s] = 0;
        /* level 1: previous visited 1 (s itself), previous sum 0 */
        int64_t a = alpha[s], o = omega[s];
        if (o <= 1) { fin[s] = 1; nfin++; sum[s] = 0; vis[s] = 1; continue; }
        int64_t pv = 1, ps = 0, nv = 1 + d;
        if (nv < a) { sum[s] = d; vis[s] = nv; }
        else if (nv < o) {
            rat_min(&num[s], &den[s], ps + 1 * (a - pv), (a - 1) * (a - 1));
            started[s] = 1;
            sum[s] = d; vis[s] = nv;
            rat_min(&num[s], &den[s], sum[s], (nv - 1) * (nv - 1));
        } else {
            if (!started[s]) rat_min(&num[s], &den[s], ps + 1 * (a - pv), (a - 1) * (a - 1));
            rat_min(&num[s], &den[s], ps + 1 * (o - pv), (o - 1) * (o - 1));
            fin[s] = 1; nfin++;
        }
    }
    for (int64_t k = 2; nfin < n; k++) {
        for (int32_t s = 0; s < n; s++) {
            int64_t acc = 0;
            for (int64_t q = A.off[s]; q < A.off[s + 1]; q++) acc = sat_add(acc, g1[A.nbr[q]]);
            if (!directed) {
                int64_t d = A.off[s + 1] - A.off[s];
                if (acc < NB_INF) {
                    /* exact counts: the subtrahend never exceeds the sum */
                    u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)(d - 1) * (uint64_t)g2[s];
                    acc = (u128)acc >= sub ? (int64_t)((u128)acc - sub) : 0;
                }
            }
            gk[s] = acc;
        }
        for (int32_t s = 0; s < n; s++) {
            g2[s] = g1[s]; g1[s] = gk[s];
            if (fin[s]) continue;
            int64_t a = alpha[s], o = omega[s];
            int64_t pv = vis[s], ps = sum[s];
            if (gk[s] == 0) {
                /* no walk of length k: nothing lies at distance >= k, so
                 * r <= pv and every candidate r in [alpha, pv] has already
                 * been evaluated (alpha <= r <= pv means alpha was reached) */
                if (!started[s]) rat_min(&num[s], &den[s], ps, (pv - 1) * (pv - 1));
                fin[s] = 1; nfin++;
                continue;
            }
            int64_t nv = sat_add(pv, gk[s]);
            if (nv < a) { sum[s] = ps + k * gk[s]; vis[s] = nv; }
            else if (nv < o) {
                if (!started[s]) {
                    rat_min(&num[s], &den[s], ps + k * (a - pv), (a - 1) * (a - 1));
                    started[s] = 1;
                }
                sum[s] = ps + k * gk[s]; vis[s] = nv;
                rat_min(&num[s], &den[s], sum[s], (nv - 1) * (nv - 1));
            } else {
                if (!started[s]) rat_min(&num[s], &den[s], ps + k * (a - pv), (a - 1) * (a - 1));
                rat_min(&num[s], &den[s], ps + k * (o - pv), (o - 1) * (o - 1));
                fin[s] = 1; nfin++;
            }
        }
    }
    free(g1); free(g2); free(gk); free(sum); free(vis); free(fin); free(started);
    adj_free(&A);
    return 0;
}

/* Upper bound on the harmonic centrality of every vertex from the walk
 * counts of Sect. 5 (the same gamma_k as oracle_nb): h(s) is largest when
 * the vertices s reaches sit as close as the counts allow, so level k takes
 * min(gamma_k(s), omega(s) - placed) of them, placed starting at 1 (s
 * itself), until omega(s) vertices are placed or gamma_k(s) = 0.  omega(s)
 * >= r(s) (Sect. 8.4), so the fill never undercounts.  The bound is the
 * binary64 sum of placed_k / k in increasing k, as for h itself; on a tree
 * the counts are exact and the bound equals h bit for bit. */
int oracle_nb_harmonic(int32_t n, int64_t ne, const int32_t *ed, int directed,
                       const int64_t *omega, double *ub) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int64_t *g1 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *g2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *gk = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *placed = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    char *done = (char *)malloc((size_t)(n ? n : 1));
    int32_t ndone = 0;
    for (int32_t s = 0; s < n; s++) {
        int64_t d = A.off[s + 1] - A.off[s];
        g2[s] = 1; g1[s] = d;
        ub[s] = 0.0; placed[s] = 1; done[s] = 0;
        if (omega[s] <= 1 || d == 0) { done[s] = 1; ndone++; continue; }
        int64_t take = d < omega[s] - 1 ? d : omega[s] - 1;
        ub[s] += (double)take / 1.0;
        placed[s] += take;
        if (placed[s] >= omega[s]) { done[s] = 1; ndone++; }
    }
    for (int64_t k = 2; ndone < n; k++) {
        for (int32_t s = 0; s < n; s++) {
            int64_t acc = 0;
            for (int64_t q = A.off[s]; q < A.off[s + 1]; q++) acc = sat_add(acc, g1[A.nbr[q]]);
            if (!directed && acc < NB_INF) {
                int64_t d = A.off[s + 1] - A.off[s];
                u128 sub = (k == 2) ? (u128)d : (u128)(uint64_t)(d - 1) * (uint64_t)g2[s];
                acc = (u128)acc >= sub ? (int64_t)((u128)acc - sub) : 0;
            }
            gk[s] = acc;
        }
        for (int32_t s = 0; s < n; s++) {
            g2[s] = g1[s]; g1[s] = gk[s];
            if (done[s]) continue;
            if (gk[s] == 0) { done[s] = 1; ndone++; continue; }
            int64_t room = omega[s] - placed[s];
            int64_t take = gk[s] < room ? gk[s] : room;
            ub[s] += (double)take / (double)k;
            placed[s] += take;
            if (placed[s] >= omega[s]) { done[s] = 1; ndone++; }
        }
    }
    free(g1); free(g2); free(gk); free(placed); free(done);
    adj_free(&A);
    return 0;
}

/* ---------------------------------------------------- BFSCut bound (Sect. 6) */
/*
 * Full BFS from v; after the vertices at distance <= D are all known
 * (n_D of them, distance sum S_D) the bound on S(v) for a reachable count r
 * is, with U = sum of out-degrees over the level-D vertices (undirected:
 * sum of (deg - 1), or deg(v) when D = 0) bounding the next level:
 *   paper form (Lemma 6.1):  S_D - U + (D+2)(r - n_D)
 *   tightened:               S_D + (D+1)(r - n_D) + max(0, r - n_D - U)
 * (the tightened form is the max of the paper form and S_D + (D+1)(r-n_D),
 * i.e. every unseen vertex is at distance at least D+1).  With r known the
 * farness bound is (n-1) bound / (r-1)^2.  With alpha <= r <= omega
 * (Sect. 8.2) r ranges over [a', o'] with a' = max(alpha, n_D) and
 * o' = max(omega, a'); the paper form is linear in r so its minimum over
 * the range sits at an end (Lemma 8.1); the tightened form is convex with
 * one kink at r = n_D + U, which is added to the candidates.
 * Writes, per level D = 0 .. ecc(v), the tightened bound as (num, den) and
 * the paper-form bound as (pnum, pden); returns the number of levels
 * (ecc(v)+1), or -1.  Levels beyond cap are not written.
 */
static void cut_eval(int64_t SD, int64_t nD, int64_t U, int64_t D, int64_t r,
                     int64_t *tight, int64_t *paper) {
    int64_t rem = r - nD;
    *paper = SD - U + (D + 2) * rem;
    int64_t extra = rem - U;
    *tight = SD + (D + 1) * rem + (extra > 0 ? extra : 0);
}
int32_t oracle_cut_levels(int32_t n, int64_t ne, const int32_t *ed, int directed, int32_t v,
                          int64_t alpha, int64_t omega, int32_t cap,
                          int64_t *num, int64_t *den, int64_t *pnum, int64_t *pden) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; i++) dist[i] = -1;
    int64_t head = 0, tail = 0;
    dist[v] = 0; queue[tail++] = v;
    int64_t SD = 0, nD = 1;
    int32_t D = 0;
    int64_t lev_start = 0;
    for (;;) {
        /* level D fully known: vertices queue[lev_start .. tail) */
        int64_t U = 0;
        for (int64_t q = lev_start; q < tail; q++) {
            int32_t u = queue[q];
            int64_t d = A.off[u + 1] - A.off[u];
            U += (directed || D == 0) ? d : d - 1;
        }
        if (D < cap) {
            int64_t a1 = alpha > nD ? alpha : nD;
            int64_t o1 = omega > a1 ? omega : a1;
            int64_t cands[3] = {a1, o1, nD + U};
            if (cands[2] < a1) cands[2] = a1;
            if (cands[2] > o1) cands[2] = o1;
            num[D] = 0; den[D] = 0; pnum[D] = 0; pden[D] = 0;
            for (int c = 0; c < 3; c++) {
                int64_t r = cands[c];
                if (r <= 1) continue;
                int64_t t, p;
                cut_eval(SD, nD, U, D, r, &t, &p);
                rat_min(&num[D], &den[D], t, (r - 1) * (r - 1));
                if (c < 2) {
                    /* paper form: endpoints only; it may be negative */
                    if (pden[D] == 0) { pnum[D] = p; pden[D] = (r - 1) * (r - 1); }
                    else {
                        __int128 x = (__int128)p * pden[D], y = (__int128)pnum[D] * ((r - 1) * (r - 1));
                        if (x < y) { pnum[D] = p; pden[D] = (r - 1) * (r - 1); }
                    }
                }
            }
        }
        /* expand level D */
        int64_t end = tail;
        for (; head < end; head++) {
            int32_t u = queue[head];
            for (int64_t q = A.off[u]; q < A.off[u + 1]; q++) {
                int32_t w = A.nbr[q];
                if (dist[w] < 0) { dist[w] = D + 1; SD += D + 1; nD++; queue[tail++] = w; }
            }
        }
        if (tail == end) break;
        lev_start = end;
        D++;
    }
    free(dist); free(queue); adj_free(&A);
    return D + 1;
}

/* ------------------------------------------------ level-based bound (Sect. 7) */
/*
 * Full BFS from s, level counts gamma_j over R(s) with s itself at level 0
 * (gamma_0 = 1).  Undirected (Eq. 4): for v at level i,
 *   S(v) >= Lev(i) - deg(v),
 *   Lev(i) = 2 sum_{|j-i|<=1} gamma_j + sum_{|j-i|>1} |j-i| gamma_j - 2.
 * Lev(1) is formed from this definition and Lev(i), i >= 2, by the
 * recurrence of Lemma 7.2: Lev(i) = Lev(i-1) + sum_{j<i-2} gamma_j - sum_{j>i+1} gamma_j.
 * Directed (Eq. 5): Lev(i) = 2 #{w: j - i <= 1} + sum_{j-i>1} (j-i) gamma_j - 2
 * with the out-degree, applied only to v in the SCC of s (Sect. 8.3), built
 * level by level with Lev(i) = Lev(i-1) - sum_{j>i+1} gamma_j.
 * Readings: counts run over R(s), never over all of V (Alg. 5 writes |V|,
 * which over-counts on a disconnected graph and can break the bound);
 * Lev(1) is taken from the definition (the printed closed form for it does
 * not match the definition).
 * Writes bound[v] (a bound on S(v); -1 where it does not apply: v outside
 * R(s) or outside the SCC of s, and v = s) and returns r(s).
 */
int64_t oracle_lb_source(int32_t n, int64_t ne, const int32_t *ed, int directed, int32_t s,
                         const int32_t *scc, int direct_definition, int64_t *bound) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; i++) dist[i] = -1;
    int64_t head = 0, tail = 0;
    dist[s] = 0; queue[tail++] = s;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t q = A.off[u]; q < A.off[u + 1]; q++)
            if (dist[A.nbr[q]] < 0) { dist[A.nbr[q]] = dist[u] + 1; queue[tail++] = A.nbr[q]; }
    }
    int32_t maxD = dist[queue[tail - 1]];
    int64_t *gam = (int64_t *)calloc((size_t)maxD + 3, sizeof(int64_t));
    for (int64_t q = 0; q < tail; q++) gam[dist[queue[q]]]++;
    int64_t *lev = (int64_t *)calloc((size_t)maxD + 2, sizeof(int64_t));
    if (direct_definition || maxD < 1) {
        for (int32_t i = 0; i <= maxD; i++) {
            int64_t L = -2;
            for (int32_t j = 0; j <= maxD; j++) {
                int64_t t = directed ? (int64_t)j - i : (j > i ? (int64_t)j - i : (int64_t)i - j);
                L += (t <= 1 ? 2 : t) * gam[j];
            }
            lev[i] = L;
        }
    } else {
        /* Lev(1) from the definition */
        int64_t L = -2;
        for (int32_t j = 0; j <= maxD; j++) {
            int64_t t = directed ? (int64_t)j - 1 : (j > 1 ? (int64_t)j - 1 : 1 - (int64_t)j);
            L += (t <= 1 ? 2 : t) * gam[j];
        }
        lev[1] = L;
        for (int32_t i = 2; i <= maxD; i++) {
            int64_t lo = 0, hi = 0;
            if (!directed) for (int32_t j = 0; j < i - 2; j++) lo += gam[j];
            for (int32_t j = i + 2; j <= maxD; j++) hi += gam[j];
            lev[i] = lev[i - 1] + lo - hi;
        }
    }
    for (int32_t v = 0; v < n; v++) bound[v] = -1;
    for (int64_t q = 1; q < tail; q++) {
        int32_t v = queue[q];
        if (directed && scc && scc[v] != scc[s]) continue;
        int64_t d = A.off[v + 1] - A.off[v];
        int64_t b = lev[dist[v]] - d;
        bound[v] = b > 0 ? b : 0;
    }
    free(gam); free(lev); free(dist); free(queue); adj_free(&A);
    return tail;
}

/* Level-based upper bound on the harmonic centrality from one complete
 * search at s (Sect. 7's argument with f(d) = 1/d): a vertex x at level i
 * and w at level l satisfy d(w,x) >= |i - l| (undirected; directed and in
 * the SCC of s, d(w,x) >= i - l, Sect. 8.3), and d(w,x) >= 2 for every x
 * but w's deg(w) out-neighbours, which sit at exactly 1.  So
 *   h(w) <= sum over x != w of 1 / max(2, t(x)) + deg(w) / 2,
 * t = |i - l| or i - l.  w reaches exactly what s reaches (same component,
 * or same SCC), so the sum runs over the vertices s reached.
 * Binary64 reading (the device computes the same): per level l, the terms
 * n_i / max(2, t) added in increasing i, then 1/2 (w itself) subtracted;
 * the bound is that plus 0.5 * deg(w).  ub[v] = -1 where it does not apply
 * (v = s, not reached, or another SCC).  Returns r(s). */
int64_t oracle_lb_harmonic(int32_t n, int64_t ne, const int32_t *ed, int directed, int32_t s,
                           const int32_t *scc, double *ub) {
    oadj A;
    if (adj_build(n, ne, ed, directed, 0, &A)) return -1;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; i++) dist[i] = -1;
    int64_t head = 0, tail = 0;
    dist[s] = 0; queue[tail++] = s;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t q = A.off[u]; q < A.off[u + 1]; q++)
            if (dist[A.nbr[q]] < 0) { dist[A.nbr[q]] = dist[u] + 1; queue[tail++] = A.nbr[q]; }
    }
    int32_t maxD = dist[queue[tail - 1]];
    int64_t *cnt = (int64_t *)calloc((size_t)maxD + 1, sizeof(int64_t));
    for (int64_t q = 0; q < tail; q++) cnt[dist[queue[q]]]++;
    double *lev = (double *)calloc((size_t)maxD + 1, sizeof(double));
    for (int32_t l = 0; l <= maxD; l++) {
        double x = 0.0;
        for (int32_t i = 0; i <= maxD; i++) {
            int64_t t = directed ? (int64_t)i - l : (i > l ? (int64_t)i - l : (int64_t)l - i);
            x += (double)cnt[i] / (double)(t < 2 ? 2 : t);
        }
        lev[l] = x - 0.5;
    }
    for (int32_t v = 0; v < n; v++) ub[v] = -1.0;
    for (int64_t q = 1; q < tail; q++) {
        int32_t v = queue[q];
        if (directed && scc && scc[v] != scc[s]) continue;
        int64_t d = A.off[v + 1] - A.off[v];
        ub[v] = lev[dist[v]] + 0.5 * (double)d;
    }
    free(cnt); free(lev); free(dist); free(queue); adj_free(&A);
    return tail;
}
