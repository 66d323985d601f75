/*
 * Seeded synthetic graph generators and the simple-graph CSR builder.
 *
 * This module holds no part of the closeness method: it only produces
 * inputs (edge lists and CSR arrays) that both the oracle and the GPU path
 * consume.  Every random draw comes from xoshiro256** seeded through
 * splitmix64 (Blackman & Vigna, "Scrambled linear pseudorandom number
 * generators", 2018), with integers mapped to [0, n) by Lemire's
 * multiply-and-reject method, so a given seed yields the same graph on
 * every machine.
 *
 * Workload shapes (the paper's real graphs are replaced by these):
 *  - Barabasi-Albert preferential attachment: undirected complex networks.
 *  - R-MAT (Chakrabarti, Zhan, Faloutsos 2004): directed web/social graphs.
 *  - Perturbed 4- or 8-neighbour lattices: road networks (high diameter).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ PRNG */
typedef struct { uint64_t s[4]; } gg_rng;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static void rng_seed(gg_rng *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t rng_next(gg_rng *r) {
    uint64_t *s = r->s;
    uint64_t out = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return out;
}
/* uniform integer in [0, n), n >= 1, unbiased (Lemire 2019) */
static inline uint64_t rng_below(gg_rng *r, uint64_t n) {
    uint64_t x = rng_next(r);
    __uint128_t m = (__uint128_t)x * n;
    uint64_t l = (uint64_t)m;
    if (l < n) {
        uint64_t t = (0 - n) % n;
        while (l < t) {
            x = rng_next(r);
            m = (__uint128_t)x * n;
            l = (uint64_t)m;
        }
    }
    return (uint64_t)(m >> 64);
}
/* uniform double in [0, 1) from the top 53 bits */
static inline double rng_unit(gg_rng *r) {
    return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

/* exported so tests can pin the stream against the published reference
 * outputs of splitmix64 / xoshiro256** */
void gg_rng_stream(uint64_t seed, int64_t count, uint64_t *out) {
    gg_rng r; rng_seed(&r, seed);
    for (int64_t i = 0; i < count; i++) out[i] = rng_next(&r);
}

/* ----------------------------------------------------- Barabasi-Albert */
/*
 * Start from the clique on vertices 0..m; every new vertex v = m+1..n-1
 * attaches to m distinct earlier vertices, each drawn with probability
 * proportional to current degree (a uniform pick from the list of all edge
 * endpoints so far; a repeated target is re-drawn).  Writes 2 * n_edges
 * int32 (u, v) pairs; returns the number of edges, -1 on bad arguments.
 * Edge count = m(m+1)/2 + (n-m-1)*m.
 */
int64_t gg_ba_count(int32_t n, int32_t m) {
    if (m < 1 || n < m + 1) return -1;
    return (int64_t)m * (m + 1) / 2 + (int64_t)(n - m - 1) * m;
}
int64_t gg_ba(int32_t n, int32_t m, uint64_t seed, int32_t *edges) {
    int64_t ne = gg_ba_count(n, m);
    if (ne < 0) return -1;
    gg_rng r; rng_seed(&r, seed);
    int32_t *ends = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)ne);
    int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    if (!ends || !pick) { free(ends); free(pick); return -1; }
    int64_t e = 0, ne2 = 0;
    for (int32_t i = 0; i <= m; i++)
        for (int32_t j = i + 1; j <= m; j++) {
            edges[2 * e] = i; edges[2 * e + 1] = j; e++;
            ends[ne2++] = i; ends[ne2++] = j;
        }
    for (int32_t v = m + 1; v < n; v++) {
        int32_t got = 0;
        while (got < m) {
            int32_t t = ends[rng_below(&r, (uint64_t)ne2)];
            int dup = 0;
            for (int32_t q = 0; q < got; q++) if (pick[q] == t) { dup = 1; break; }
            if (!dup) pick[got++] = t;
        }
        for (int32_t q = 0; q < m; q++) {
            edges[2 * e] = v; edges[2 * e + 1] = pick[q]; e++;
            ends[ne2++] = v; ends[ne2++] = pick[q];
        }
    }
    free(ends); free(pick);
    return e;
}

/* --------------------------------------------------------------- R-MAT */
/*
 * n_arcs draws of one directed arc each: every one of the `scale` bit levels
 * picks a quadrant with probabilities (a, b, c, 1-a-b-c) (a: top-left,
 * b: top-right, c: bottom-left), no per-level noise.  Self-loops and
 * duplicates are kept here (the CSR builder removes them).  Afterwards the
 * vertex ids are relabelled by a seeded uniform permutation.
 */
void gg_rmat(int32_t scale, int64_t n_arcs, double a, double b, double c,
             uint64_t seed, int permute, int32_t *edges) {
    gg_rng r; rng_seed(&r, seed);
    double ab = a + b, abc = a + b + c;
    for (int64_t e = 0; e < n_arcs; e++) {
        uint32_t u = 0, v = 0;
        for (int32_t l = 0; l < scale; l++) {
            double x = rng_unit(&r);
            u <<= 1; v <<= 1;
            if (x < a) { }
            else if (x < ab) { v |= 1; }
            else if (x < abc) { u |= 1; }
            else { u |= 1; v |= 1; }
        }
        edges[2 * e] = (int32_t)u; edges[2 * e + 1] = (int32_t)v;
    }
    if (permute) {
        int32_t n = (int32_t)1 << scale;
        int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        for (int32_t i = 0; i < n; i++) perm[i] = i;
        for (int32_t i = n - 1; i > 0; i--) {
            int32_t j = (int32_t)rng_below(&r, (uint64_t)i + 1);
            int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
        for (int64_t e = 0; e < 2 * n_arcs; e++) edges[e] = perm[edges[e]];
        free(perm);
    }
}

/* --------------------------------------------------- perturbed lattices */
/* key of an undirected pair for the shortcut-uniqueness hash */
static inline uint64_t pair_key(int32_t u, int32_t v) {
    if (u > v) { int32_t t = u; u = v; v = t; }
    return ((uint64_t)(uint32_t)u << 32) | (uint32_t)v;
}
typedef struct { uint64_t *slot; uint64_t cap; } gg_set;
static uint64_t mix(uint64_t k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdULL; k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL; k ^= k >> 33; return k;
}
static int set_insert(gg_set *s, uint64_t key) { /* 1 if inserted, 0 if present */
    uint64_t h = mix(key) & (s->cap - 1);
    uint64_t k1 = key + 1; /* 0 marks an empty slot */
    while (s->slot[h]) {
        if (s->slot[h] == k1) return 0;
        h = (h + 1) & (s->cap - 1);
    }
    s->slot[h] = k1;
    return 1;
}

/*
 * side x side lattice, id = row*side + col.  king=0: 4-neighbour (right,
 * down); king=1: 8-neighbour (right, down, down-right, down-left).  Lattice
 * edges are enumerated row-major; exactly n_delete of them are removed
 * uniformly without replacement (partial Fisher-Yates), then n_short
 * shortcuts between uniform vertex pairs are added (self pairs, lattice
 * edges that survived and repeated shortcuts are re-drawn).
 * Returns the number of edges written (lattice - deleted + shortcuts).
 */
int64_t gg_lattice_count(int32_t side, int king) {
    int64_t s = side;
    int64_t e = 2 * s * (s - 1);
    if (king) e += 2 * (s - 1) * (s - 1);
    return e;
}
int64_t gg_lattice(int32_t side, int king, int64_t n_delete, int64_t n_short,
                   uint64_t seed, int32_t *edges) {
    gg_rng r; rng_seed(&r, seed);
    int64_t ne = gg_lattice_count(side, king);
    if (n_delete > ne || side < 2) return -1;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)ne);
    if (!tmp) return -1;
    int64_t e = 0;
    for (int32_t i = 0; i < side; i++)
        for (int32_t j = 0; j < side; j++) {
            int32_t u = i * side + j;
            if (j + 1 < side) { tmp[2 * e] = u; tmp[2 * e + 1] = u + 1; e++; }
            if (i + 1 < side) { tmp[2 * e] = u; tmp[2 * e + 1] = u + side; e++; }
            if (king && i + 1 < side) {
                if (j + 1 < side) { tmp[2 * e] = u; tmp[2 * e + 1] = u + side + 1; e++; }
                if (j > 0) { tmp[2 * e] = u; tmp[2 * e + 1] = u + side - 1; e++; }
            }
        }
    /* move n_delete uniformly chosen edges to the tail, then drop the tail */
    for (int64_t t = 0; t < n_delete; t++) {
        int64_t last = ne - 1 - t;
        int64_t j = (int64_t)rng_below(&r, (uint64_t)last + 1);
        int32_t a0 = tmp[2 * j], a1 = tmp[2 * j + 1];
        tmp[2 * j] = tmp[2 * last]; tmp[2 * j + 1] = tmp[2 * last + 1];
        tmp[2 * last] = a0; tmp[2 * last + 1] = a1;
    }
    int64_t keep = ne - n_delete;
    uint64_t cap = 1;
    while (cap < (uint64_t)(2 * (keep + n_short) + 16)) cap <<= 1;
    gg_set set; set.cap = cap; set.slot = (uint64_t *)calloc(cap, sizeof(uint64_t));
    if (!set.slot) { free(tmp); return -1; }
    for (int64_t q = 0; q < keep; q++) {
        edges[2 * q] = tmp[2 * q]; edges[2 * q + 1] = tmp[2 * q + 1];
        set_insert(&set, pair_key(tmp[2 * q], tmp[2 * q + 1]));
    }
    free(tmp);
    int64_t nv = (int64_t)side * side;
    int64_t out = keep;
    for (int64_t q = 0; q < n_short; q++) {
        for (;;) {
            int32_t u = (int32_t)rng_below(&r, (uint64_t)nv);
            int32_t v = (int32_t)rng_below(&r, (uint64_t)nv);
            if (u == v) continue;
            if (!set_insert(&set, pair_key(u, v))) continue;
            edges[2 * out] = u; edges[2 * out + 1] = v; out++;
            break;
        }
    }
    free(set.slot);
    return out;
}

/* ---------------------------------------------- small random test graphs */
/* G(n, p): every ordered (directed) or unordered (undirected) pair is an
 * arc/edge with probability p.  Returns the count; edges must hold n*n pairs. */
int64_t gg_gnp(int32_t n, double p, int directed, uint64_t seed, int32_t *edges) {
    gg_rng r; rng_seed(&r, seed);
    int64_t e = 0;
    for (int32_t u = 0; u < n; u++)
        for (int32_t v = directed ? 0 : u + 1; v < n; v++) {
            if (u == v) continue;
            if (rng_unit(&r) < p) { edges[2 * e] = u; edges[2 * e + 1] = v; e++; }
        }
    return e;
}
/* random recursive tree: vertex i > 0 attaches to a uniform j < i;
 * ids are then shuffled.  Writes n-1 edges. */
void gg_tree(int32_t n, uint64_t seed, int32_t *edges) {
    gg_rng r; rng_seed(&r, seed);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; i++) perm[i] = i;
    for (int32_t i = n - 1; i > 0; i--) {
        int32_t j = (int32_t)rng_below(&r, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    for (int32_t i = 1; i < n; i++) {
        int32_t j = (int32_t)rng_below(&r, (uint64_t)i);
        edges[2 * (i - 1)] = perm[i]; edges[2 * (i - 1) + 1] = perm[j];
    }
    free(perm);
}

/* ------------------------------------------------------- CSR building */
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}
/*
 * Simple-graph CSR from an edge list: self-loops dropped, undirected edges
 * stored in both directions, each row sorted ascending and deduplicated.
 * row_ptr has n+1 entries; col_idx must hold 2*ne (undirected) or ne
 * (directed) entries; the arc count (< 2^31) is returned, -2 on an id out
 * of range.  transpose=1 builds the in-arc (reverse) CSR of a directed graph.
 */
int64_t gg_csr(int32_t n, int64_t ne, const int32_t *edges, int directed,
               int transpose, int32_t *row_ptr, int32_t *col_idx) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int64_t e = 0; e < ne; e++) {
        int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u == v) continue;
        if (u < 0 || v < 0 || u >= n || v >= n) { free(cnt); return -2; }
        if (directed) cnt[transpose ? v : u]++;
        else { cnt[u]++; cnt[v]++; }
    }
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    off[0] = 0;
    for (int32_t i = 0; i < n; i++) off[i + 1] = off[i] + cnt[i];
    int64_t total = off[n];
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int64_t *pos = cnt; /* reuse as cursor */
    for (int32_t i = 0; i <= n; i++) pos[i] = off[i];
    for (int64_t e = 0; e < ne; e++) {
        int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u == v) continue;
        if (directed) {
            if (transpose) tmp[pos[v]++] = u; else tmp[pos[u]++] = v;
        } else { tmp[pos[u]++] = v; tmp[pos[v]++] = u; }
    }
    int64_t w = 0;
    int64_t arcs = 0;
    for (int32_t i = 0; i < n; i++) {
        int64_t a = off[i], b = off[i + 1];
        qsort(tmp + a, (size_t)(b - a), sizeof(int32_t), cmp_i32);
        int64_t start = w;
        for (int64_t q = a; q < b; q++)
            if (q == a || tmp[q] != tmp[q - 1]) tmp[w++] = tmp[q];
        if (row_ptr) row_ptr[i] = (int32_t)start;
        arcs = w;
    }
    if (row_ptr) row_ptr[n] = (int32_t)w;
    if (col_idx) memcpy(col_idx, tmp, sizeof(int32_t) * (size_t)w);
    free(tmp); free(off); free(cnt);
    return arcs;
}

/* -------------------------------------------- largest connected component */
static int32_t uf_find(int32_t *p, int32_t x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
}
/*
 * Keeps the largest weakly connected component (ties: the one holding the
 * smallest vertex id) and relabels its vertices in increasing original id.
 * new_id[v] = new label or -1.  Edges are rewritten in place (edges outside
 * the component dropped); returns the new edge count and writes the new n.
 */
int64_t gg_lcc(int32_t n, int64_t ne, int32_t *edges, int32_t *new_id, int32_t *n_out) {
    int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *sz = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int32_t i = 0; i < n; i++) p[i] = i;
    for (int64_t e = 0; e < ne; e++) {
        int32_t a = uf_find(p, edges[2 * e]), b = uf_find(p, edges[2 * e + 1]);
        if (a != b) { if (a < b) p[b] = a; else p[a] = b; }
    }
    for (int32_t i = 0; i < n; i++) sz[uf_find(p, i)]++;
    int32_t best = 0;
    for (int32_t i = 0; i < n; i++) if (sz[i] > sz[best]) best = i;
    int32_t c = 0;
    for (int32_t i = 0; i < n; i++) new_id[i] = (uf_find(p, i) == best) ? c++ : -1;
    int64_t w = 0;
    for (int64_t e = 0; e < ne; e++) {
        int32_t a = new_id[edges[2 * e]], b = new_id[edges[2 * e + 1]];
        if (a < 0 || b < 0) continue;
        edges[2 * w] = a; edges[2 * w + 1] = b; w++;
    }
    *n_out = c;
    free(p); free(sz);
    return w;
}
