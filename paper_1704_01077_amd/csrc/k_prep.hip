// Preprocessing kernels: out-degrees, connected components (r(v) of an
// undirected graph), the neighbourhood-based lower bound of Sect. 5 and the
// keys of the processing order (Sect. 4, computeBounds).
#include <stdlib.h>

#include <algorithm>

#include "dev_common.hpp"
#include "engine.hpp"

#define NB_INF ((int64_t)1 << 62)

// --------------------------------------------------------------- degrees
__global__ void k_degrees(int32_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ deg) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) deg[v] = rp[v + 1] - rp[v];
}


// ----------------------------------------------- connected components
// r(v) of an undirected graph is the size of v's component (Sect. 4).
// Lock-free union-find in the style of Afforest (Sutton, Ben-Nun, Barak,
// 2018): every vertex first links to its first two neighbours, the
// dominant component G is read off a sample of roots, and only vertices
// outside G then link their remaining neighbours (an edge from G to a
// vertex outside it is seen from the outside end, so nothing is missed).
// Roots only ever point to smaller ids: every component ends rooted at its
// smallest vertex and parent chains strictly decrease, so a find that reads
// a stale parent still terminates; the compare-and-swap that links a root
// is the only authority, and a failed swap retries with coherent reads.
TKC_DEV int32_t uf_find_plain(const int32_t* parent, int32_t x) {
    int32_t p = parent[x];
    while (p != x) { x = p; p = parent[x]; }
    return x;
}
TKC_DEV int32_t uf_find_coherent(int32_t* parent, int32_t x) {
    for (;;) {
        int32_t p = ld_rlx(&parent[x]);
        if (p == x) return x;
        x = p;
    }
}
TKC_DEV void uf_union(int32_t* parent, int32_t a, int32_t b) {
    int32_t ra = uf_find_plain(parent, a), rb = uf_find_plain(parent, b);
    for (;;) {
        if (ra == rb) return;
        int32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
        int32_t exp = hi;
        if (__hip_atomic_compare_exchange_strong(&parent[hi], &exp, lo, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        ra = uf_find_coherent(parent, a);
        rb = uf_find_coherent(parent, b);
    }
}
__global__ void k_cc_init(int32_t n, int32_t* parent) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) parent[v] = v;
}
// phase 1: link every vertex to its neighbour number `which` (one per
// round, so in a round a thread mostly swaps only its own root entry)
__global__ void k_cc_link_one(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              int32_t which, int32_t* parent) {
    int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int32_t q = rp[u] + which;
    if (q < rp[u + 1]) uf_union(parent, u, ci[q]);
}
// full path compression; with in_giant, a snapshot of membership in the
// component rooted at *giant
// (zero, when given, has its n + 1 counters cleared for the counting pass)
__global__ void k_cc_compress(int32_t n, int32_t* parent, const int32_t* giant, uint8_t* in_giant,
                              int64_t* zero) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (zero && v == 0) zero[n] = 0;
    if (v >= n) return;
    if (zero) zero[v] = 0;
    int32_t r = uf_find_coherent(parent, v);
    parent[v] = r;
    if (in_giant) in_giant[v] = (r == *giant);
}
// the most frequent root among ns evenly spaced samples of the (compressed)
// parents, ties to the smallest: one block of CC_NS threads, each counting
// the copies of its own sample (every thread reads the same LDS words at
// the same step: broadcasts, four at a time; padding never matches a root)
#define CC_NS 256
__global__ void __launch_bounds__(CC_NS) k_cc_mode(int32_t n, int32_t ns, const int32_t* __restrict__ parent,
                                                   int32_t* out) {
    __shared__ __align__(16) int32_t a[CC_NS];
    __shared__ unsigned long long best[CC_NS / 64];
    const int t = threadIdx.x;
    a[t] = t < ns ? parent[(int64_t)t * n / ns] : -1;
    __syncthreads();
    unsigned long long key = 0;
    if (t < ns) {
        const int32_t mine = a[t];
        const int4* a4 = (const int4*)a;
        int32_t c = 0;
        for (int j = 0; j < CC_NS / 4; j++) {
            const int4 q = a4[j];
            c += (q.x == mine) + (q.y == mine) + (q.z == mine) + (q.w == mine);
        }
        key = ((unsigned long long)c << 32) | (0xffffffffull - (uint32_t)mine);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(key, o, 64);
        key = y > key ? y : key;
    }
    if (lane_id() == 0) best[t >> 6] = key;
    __syncthreads();
    if (t == 0) {
        unsigned long long m = 0;
        for (int w = 0; w < CC_NS / 64; w++) m = best[w] > m ? best[w] : m;
        *out = (int32_t)(0xffffffffull - (m & 0xffffffffull));
    }
}
// phase 2: vertices outside the dominant component link their other
// neighbours (light: one thread each; heavy: one wave each)
__global__ void k_cc_link_rest(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               const int32_t* __restrict__ deg, const int32_t* __restrict__ heavy,
                               int32_t nheavy, int32_t nlight_blocks, int32_t first,
                               const uint8_t* __restrict__ in_giant, int32_t* parent) {
    if ((int32_t)blockIdx.x < nlight_blocks) {
        int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
        if (u >= n || deg[u] > HEAVY_DEG || in_giant[u]) return;
        for (int32_t q = rp[u] + first; q < rp[u + 1]; q++) uf_union(parent, u, ci[q]);
    } else {
        int32_t wv = ((blockIdx.x - nlight_blocks) * blockDim.x + threadIdx.x) >> 6;
        if (wv >= nheavy) return;
        int32_t u = heavy[wv];
        if (in_giant[u]) return;
        for (int32_t q = rp[u] + first + lane_id(); q < rp[u + 1]; q += 64) uf_union(parent, u, ci[q]);
    }
}
// sizes: vertices outside the dominant component count into their root,
// the dominant component's size is n minus all of those
// (the dominant component's root: the final root of its sampled root,
// which later links may have put under a smaller one)
__global__ void k_cc_count(int32_t n, const int32_t* __restrict__ parent, const int32_t* giant_dev, int64_t* size,
                           int64_t* outside) {
    __shared__ int64_t part[4];
    const int32_t giant = parent[*giant_dev];
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    int64_t mine = 0;
    if (v < n) {
        int32_t r = parent[v];
        if (r != giant) { fadd_rlx(&size[r], (int64_t)1); mine = 1; }
    }
    int64_t s = wave_sum_i64(mine);
    if (lane_id() == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = part[0] + part[1] + part[2] + part[3];
        if (t) fadd_rlx(outside, t);
    }
}
__global__ void k_cc_assign(int32_t n, const int32_t* parent, const int64_t* size, const int32_t* giant_dev,
                            const int64_t* outside, int64_t* alpha, int64_t* omega) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t giant = parent[*giant_dev];
    int32_t r = parent[v];
    int64_t s = (r == giant) ? (int64_t)n - *outside : size[r];
    alpha[v] = s;
    omega[v] = s;
}

// ------------------------------------------- NB bound (Sect. 5, Alg. 3)
// gamma_k(s) bounds the number of vertices at distance k.  Undirected: the
// non-backtracking walk recurrence of Eq. 2; directed: plain walk counts
// (Eq. 3).  Three rotating buffers hold gamma_{k-2}, gamma_{k-1}, gamma_k so
// one kernel per round both gathers the new counts and advances each
// vertex's sum (Prop. 5.1) -- a vertex only ever writes its own state.
// Counts saturate at 2^62 ("at least that many").  A finished vertex keeps
// updating its counts because its neighbours still read them.
// Disconnected directed graphs (Sect. 8.1): with alpha <= r <= omega the
// bound is the least value over r in {alpha, omega} and the cumulative
// counts strictly between them; with r known alpha = omega = r.
struct NBState {
    int64_t* sum;
    int64_t* vis;
    uint8_t* flags;   // bit0 finished, bit1 alpha reached
    int64_t* num;
    int64_t* den;
    double* hub;      // harmonic upper bound (null: closeness only)
    // 32-bit copy of the level being written, min(count, NB_C32) (null: none);
    // the next round gathers it and re-reads a row exactly from the 64-bit
    // counts when it meets NB_C32
    int32_t* c32;
};
#define NB_C32 0x7fffffff
// Finish counts: one add per workgroup, into NB_NCTR counters 128 B apart.
// Adds to one address are done one after another at the cache; with one
// add per wave on a single counter, a round in which most waves finish a
// vertex queued ~16K adds there and took twice as long.  k_nb_total sums
// the counters for the host check.
#define NB_NCTR 32
#define NB_CTR_WORDS 32
#define NB_TOTAL_WORD (NB_NCTR * NB_CTR_WORDS)
#define NB_TAILCNT_WORD (NB_TOTAL_WORD + 32)
// every thread of the block calls it; lds holds one int per wave
TKC_DEV void nb_count(bool fin, int32_t* nfin, int32_t* lds) {
    int tot;
    wave_rank(fin, &tot);
    if (lane_id() == 0) lds[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); i++) t += lds[i];
        if (t) fadd_rlx(nfin + (blockIdx.x % NB_NCTR) * NB_CTR_WORDS, t);
    }
}
// one wave: the counters' sum into nfin[NB_TOTAL_WORD]; it also clears the
// tail list's count, which a collect after the check starts from
__global__ void k_nb_total(int32_t* nfin) {
    int32_t v = lane_id() < NB_NCTR ? nfin[lane_id() * NB_CTR_WORDS] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane_id() == 0) {
        nfin[NB_TOTAL_WORD] = v;
        nfin[NB_TAILCNT_WORD] = 0;
    }
}

// Harmonic centrality from the same counts: level k takes min(gamma_k,
// omega - placed) vertices (placed = the visited count, s included), the
// closest placement the counts allow, and adds that many times 1/k.  Called
// before nb_advance, while s is unfinished (so placed < omega).
TKC_DEV void nb_harm(double* hub, int32_t s, int64_t k, int64_t gk, int64_t o, int64_t pv) {
    const int64_t room = o - pv;
    const int64_t take = gk < room ? gk : room;
    if (take > 0) hub[s] += (double)take / (double)k;
}
TKC_DEV void rat_keep_min(int64_t* num, int64_t* den, int64_t cn, int64_t cd) {
    if (*den == 0 || rat_cmp(cn, cd, *num, *den) < 0) { *num = cn; *den = cd; }
}
// advance vertex s by one level (level k, count gk); returns true when s finishes now
TKC_DEV bool nb_advance(int64_t k, int64_t gk, int64_t a, int64_t o, int64_t& pv, int64_t& ps,
                        uint8_t& fl, int64_t& num, int64_t& den) {
    if (gk == 0) {
        // nothing at distance >= k: r <= pv and alpha was already reached
        if (!(fl & 2)) rat_keep_min(&num, &den, ps, sq64(pv - 1));
        fl |= 1;
        return true;
    }
    int64_t nv = pv + gk;
    if (nv > NB_INF) nv = NB_INF;
    if (nv < a) {
        ps += k * gk; pv = nv;
        return false;
    }
    if (nv < o) {
        if (!(fl & 2)) { rat_keep_min(&num, &den, ps + k * (a - pv), sq64(a - 1)); fl |= 2; }
        ps += k * gk; pv = nv;
        rat_keep_min(&num, &den, ps, sq64(nv - 1));
        return false;
    }
    if (!(fl & 2)) rat_keep_min(&num, &den, ps + k * (a - pv), sq64(a - 1));
    rat_keep_min(&num, &den, ps + k * (o - pv), sq64(o - 1));
    fl |= 1;
    return true;
}

__global__ void k_nb_init(int32_t n, const int32_t* __restrict__ deg, const int64_t* __restrict__ alpha,
                          const int64_t* __restrict__ omega, int64_t* g0, int64_t* g1, NBState st,
                          int32_t* nfin) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    bool fin = false;
    if (s < n) {
        int64_t d = deg[s];
        g0[s] = 1;
        g1[s] = d;
        int64_t a = alpha[s], o = omega[s];
        int64_t pv = 1, ps = 0, num = 0, den = 0;
        uint8_t fl = 0;
        if (st.hub) st.hub[s] = 0.0;
        if (o <= 1) { fl = 1; fin = true; }
        else {
            if (st.hub) nb_harm(st.hub, s, 1, d, o, pv);
            fin = nb_advance(1, d, a, o, pv, ps, fl, num, den);
        }
        st.sum[s] = ps; st.vis[s] = pv; st.flags[s] = fl; st.num[s] = num; st.den[s] = den;
    }
    __shared__ int32_t lds[16];
    nb_count(fin, nfin, lds);
}

// adv = false only writes the count (the vertex's state was advanced at this
// level already, by a tail round over the open vertices)
template <bool DIRECTED>
TKC_DEV void nb_finish_vertex(int32_t s, uint64_t acc, int64_t k, int32_t d, const int64_t* g2,
                              int64_t* gk, const int64_t* alpha, const int64_t* omega, NBState st,
                              bool adv, bool* fin_now) {
    int64_t val;
    if (acc >= (uint64_t)NB_INF) val = NB_INF;
    else {
        val = (int64_t)acc;
        if (!DIRECTED) {
            // exact counts: the subtracted walks never exceed the sum
            tkc_u128 sub = (k == 2) ? (tkc_u128)d : (tkc_u128)(uint64_t)(d - 1) * (uint64_t)g2[s];
            val = ((tkc_u128)(uint64_t)val >= sub) ? (int64_t)((tkc_u128)(uint64_t)val - sub) : 0;
        }
    }
    gk[s] = val;
    if (st.c32) st.c32[s] = val >= (int64_t)NB_C32 ? NB_C32 : (int32_t)val;
    *fin_now = false;
    if (!adv) return;
    uint8_t fl = st.flags[s];
    if (fl & 1) return;
    int64_t pv = st.vis[s], ps = st.sum[s], num = st.num[s], den = st.den[s];
    if (st.hub) nb_harm(st.hub, s, k, val, omega[s], pv);
    *fin_now = nb_advance(k, val, alpha[s], omega[s], pv, ps, fl, num, den);
    st.vis[s] = pv; st.sum[s] = ps; st.flags[s] = fl; st.num[s] = num; st.den[s] = den;
}

// LPV lanes share one light vertex (its arcs strided over them), so a wave
// waits on the longest of 64 / LPV rows rather than of 64
// G: the type of the previous level's counts as gathered (the first round
// reads gamma_1, the out-degrees, from the int32 degree array: half the
// bytes per gather)
template <bool DIRECTED, int LPV, typename G>
__global__ void k_nb_round(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const int32_t* __restrict__ deg, const int32_t* __restrict__ ch_beg,
                           const int32_t* __restrict__ ch_end, int32_t nchunks, int32_t nlight_blocks,
                           int64_t k, const G* __restrict__ g1, const int64_t* __restrict__ g1x,
                           const int64_t* __restrict__ g2,
                           int64_t* __restrict__ gk, const int64_t* __restrict__ alpha,
                           const int64_t* __restrict__ omega, NBState st, uint64_t* partial, int32_t* nfin,
                           int32_t adv) {
    if ((int32_t)blockIdx.x < nlight_blocks && LPV > 1) {
        // light vertices: LPV lanes each, finished in place by the first
        const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const int32_t s = (int32_t)(gt / LPV);
        const int sub = (int)(gt & (LPV - 1));
        const bool mine = s < n && deg[s] <= HEAVY_DEG;   // the same on the LPV lanes of s
        uint64_t acc = 0;
        bool redo = false;
        if (mine) {
            int32_t e = rp[s] + sub;
            const int32_t end = rp[s + 1];
            for (; e + LPV < end; e += 2 * LPV) {
                // both terms at most 2^62: their sum fits, then clamp
                const G v0 = g1[ci[e]], v1 = g1[ci[e + LPV]];
                if (sizeof(G) == 4) redo |= (v0 == (G)NB_C32) | (v1 == (G)NB_C32);
                uint64_t s01 = (uint64_t)v0 + (uint64_t)v1;
                if (s01 > (uint64_t)NB_INF) s01 = NB_INF;
                acc += s01;
                if (acc > (uint64_t)NB_INF) acc = NB_INF;
            }
            if (e < end) {
                const G v0 = g1[ci[e]];
                if (sizeof(G) == 4) redo |= v0 == (G)NB_C32;
                acc += (uint64_t)v0;
                if (acc > (uint64_t)NB_INF) acc = NB_INF;
            }
        }
        if (sizeof(G) == 4) {
            // a capped count in the row: the vertex's LPV lanes sum it again
            // from the exact 64-bit counts
#pragma unroll
            for (int o = 1; o < LPV; o <<= 1) redo |= __shfl_xor((int)redo, o, 64) != 0;
            if (mine && redo) {
                acc = 0;
                for (int32_t e = rp[s] + sub; e < rp[s + 1]; e += LPV) {
                    acc += (uint64_t)g1x[ci[e]];
                    if (acc > (uint64_t)NB_INF) acc = NB_INF;
                }
            }
        }
        // the LPV partial sums (xor partners stay inside the group of s)
#pragma unroll
        for (int o = 1; o < LPV; o <<= 1) {
            acc += __shfl_xor(acc, o, 64);
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
        bool fin = false;
        if (mine && sub == 0)
            nb_finish_vertex<DIRECTED>(s, acc, k, deg[s], g2, gk, alpha, omega, st, adv != 0, &fin);
        __shared__ int32_t lds[16];
        nb_count(fin, nfin, lds);   // the branch is uniform over the workgroup
    } else if ((int32_t)blockIdx.x < nlight_blocks) {
        // light vertices: one thread each, finished in place
        bool fin = false;
        int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
        if (s < n && deg[s] <= HEAVY_DEG) {
            uint64_t acc = 0;
            int32_t e = rp[s], end = rp[s + 1];
            for (; e + 4 <= end; e += 4) {
                uint64_t a0 = g1[ci[e]], a1 = g1[ci[e + 1]], a2 = g1[ci[e + 2]], a3 = g1[ci[e + 3]];
                // every term is at most 2^62: clamp the pairs before adding
                // so no partial sum passes 2^64 (acc + 2 clamped pairs <
                // 2^62 + 2^63)
                uint64_t s01 = a0 + a1, s23 = a2 + a3;
                if (s01 > (uint64_t)NB_INF) s01 = NB_INF;
                if (s23 > (uint64_t)NB_INF) s23 = NB_INF;
                acc += s01 + s23;
                if (acc > (uint64_t)NB_INF) acc = NB_INF;
            }
            for (; e < end; e++) {
                acc += (uint64_t)g1[ci[e]];
                if (acc > (uint64_t)NB_INF) acc = NB_INF;
            }
            nb_finish_vertex<DIRECTED>(s, acc, k, deg[s], g2, gk, alpha, omega, st, adv != 0, &fin);
        }
        __shared__ int32_t lds[16];
        nb_count(fin, nfin, lds);   // the branch is uniform over the workgroup
    } else {
        // arcs of heavy vertices: one wave per chunk, saturating partial sum
        int32_t c = ((blockIdx.x - nlight_blocks) * blockDim.x + threadIdx.x) >> 6;
        if (c >= nchunks) return;   // wave-uniform
        // (the exact 64-bit counts: a 512-arc chunk meets a capped count
        // far more often than a light row)
        uint64_t acc = 0;
        for (int32_t e = ch_beg[c] + lane_id(); e < ch_end[c]; e += 64) {
            acc += (uint64_t)g1x[ci[e]];
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            acc += __shfl_xor(acc, o, 64);
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
        if (lane_id() == 0) partial[c] = acc;
    }
}
// heavy vertices: sum their chunks' partials and finish (one thread each)
template <bool DIRECTED>
__global__ void k_nb_heavy(int32_t nheavy, const int32_t* __restrict__ heavy, const int32_t* __restrict__ hcb,
                           const uint64_t* __restrict__ partial, const int32_t* __restrict__ deg, int64_t k,
                           const int64_t* __restrict__ g2, int64_t* __restrict__ gk,
                           const int64_t* __restrict__ alpha, const int64_t* __restrict__ omega, NBState st,
                           int32_t* nfin, int32_t adv) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool fin = false;
    if (i < nheavy) {
        uint64_t acc = 0;
        for (int32_t c = hcb[i]; c < hcb[i + 1]; c++) {
            acc += partial[c];
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
        int32_t s = heavy[i];
        nb_finish_vertex<DIRECTED>(s, acc, k, deg[s], g2, gk, alpha, omega, st, adv != 0, &fin);
    }
    __shared__ int32_t lds[16];
    nb_count(fin, nfin, lds);
}

// The open (unfinished) vertices, in no particular order: the tail round
// treats each on its own, so the order changes no result.  At most cap are
// written; *cnt counts them all.  One add per workgroup of 1024 threads.
__global__ void k_nb_collect(int32_t n, const uint8_t* __restrict__ flags, int32_t cap, int32_t* list,
                             int32_t* cnt) {
    __shared__ int32_t wbase[16];
    __shared__ int32_t bbase;
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool open = s < n && !(flags[s] & 1);
    int tot;
    const int r = wave_rank(open, &tot);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) wbase[w] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < (int)((blockDim.x + 63) >> 6); i++) {
            const int x = wbase[i];
            wbase[i] = t;
            t += x;
        }
        bbase = t ? fadd_rlx(cnt, t) : 0;
    }
    __syncthreads();
    const int32_t pos = bbase + wbase[w] + r;
    if (open && pos < cap) list[pos] = s;
}
// A round over the listed vertices alone (one wave each): the same
// saturating sum as the full round (min(sum, 2^62) in any order), then the
// same finish.  Only the listed vertices' counts at level k are written.
template <bool DIRECTED>
__global__ void k_nb_tail(const int32_t* __restrict__ cnt, int32_t cap, const int32_t* __restrict__ list,
                          const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const int32_t* __restrict__ deg, int64_t k, const int64_t* __restrict__ g1,
                          const int64_t* __restrict__ g2, int64_t* __restrict__ gk,
                          const int64_t* __restrict__ alpha, const int64_t* __restrict__ omega, NBState st,
                          int32_t* nfin) {
    const int32_t w = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int32_t m = *cnt < cap ? *cnt : cap;
    bool fin = false;
    if (w < m) {   // wave-uniform
        const int32_t s = list[w];
        uint64_t acc = 0;
        for (int32_t e = rp[s] + lane_id(); e < rp[s + 1]; e += 64) {
            acc += (uint64_t)g1[ci[e]];
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            acc += __shfl_xor(acc, o, 64);
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
        if (lane_id() == 0)
            nb_finish_vertex<DIRECTED>(s, acc, k, deg[s], g2, gk, alpha, omega, st, true, &fin);
    }
    __shared__ int32_t lds[16];
    nb_count(fin, nfin, lds);
}

// ------------------------------------------------------ order keys (Sect. 4)
// Deg: L = 0 (the bound is the trivial one) and the key is the degree,
// largest first; NB: the key is the bound itself.  Vertices that reach
// nothing get L = +inf and the last key.
__global__ void k_deg_bounds(int32_t n, const int32_t* __restrict__ deg, const int64_t* __restrict__ omega,
                             int64_t* num, int64_t* den, uint32_t* key, int32_t* val) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    bool inf = omega[v] <= 1;
    num[v] = 0;
    den[v] = inf ? 0 : 1;
    key[v] = inf ? 0xffffffffu : (uint32_t)(0x7fffffff - deg[v]);
    val[v] = v;
}
__global__ void k_nb_keys(int32_t n, const int64_t* __restrict__ num, const int64_t* __restrict__ den,
                          uint32_t* key, int32_t* val) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    // 24 bits (12 of mantissa, 2^-12 relative) order the candidates as well
    // as 32 and save the sort two of its 4-bit passes; truncating further
    // keeps every key a lower bound of its vertex's bound, so the stop test
    // stays valid (+inf keeps its all-ones key)
    const uint32_t k = order_key(num[v], den[v]);
    key[v] = k == 0xffffffffu ? k : (k & 0xffffff00u);
    val[v] = v;
}

// harmonic centrality: bounds and keys carry harm_enc of the upper bound
// (with its margin), so the order runs from the largest bound down and the
// skip and stop tests compare with x as for closeness
__global__ void k_harm_deg_bounds(int32_t n, const int32_t* __restrict__ deg, const int64_t* __restrict__ omega,
                                  int64_t* num, int64_t* den, uint32_t* key, int32_t* val) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t o = omega[v], d = deg[v];
    // the out-neighbours at distance 1, every other reachable vertex at >= 2
    const double ub = o > 1 ? (double)d + (double)(o - 1 - d) / 2.0 : 0.0;
    const double ubm = ub * (1.0 + HARM_MARGIN);
    num[v] = harm_enc(ubm);
    den[v] = 1;
    key[v] = harm_key(ubm);
    val[v] = v;
}
__global__ void k_harm_nb_keys(int32_t n, const double* __restrict__ hub, int64_t* num, int64_t* den,
                               uint32_t* key, int32_t* val) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double ubm = hub[v] * (1.0 + HARM_MARGIN);
    num[v] = harm_enc(ubm);
    den[v] = 1;
    key[v] = harm_key(ubm);
    val[v] = v;
}

// ------------------------------------------------------------ host side
static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

int tkc_launch_degrees(const DevGraph& g, hipStream_t s) {
    int32_t n = g.n;
    hipLaunchKernelGGL(k_degrees, dim3(nblk(n, 256)), dim3(256), 0, s, n, g.rp, g.deg);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Components (undirected reachability): size holds n + 2 int64, in_giant n bytes.
int tkc_launch_cc(const DevGraph& g, int32_t* parent, int64_t* size, int64_t* alpha, int64_t* omega,
                  uint8_t* in_giant, int32_t* sample_host, hipStream_t s) {
    (void)sample_host;   // the dominant component is found on the device
    int32_t n = g.n;
    const int32_t* heavy = g.heavy;
    const int32_t nheavy = g.nheavy;
    int nl = nblk(n, 256);
    const int32_t first = 2;
    hipLaunchKernelGGL(k_cc_init, dim3(nl), dim3(256), 0, s, n, parent);
    for (int32_t which = 0; which < first; which++) {
        hipLaunchKernelGGL(k_cc_link_one, dim3(nl), dim3(256), 0, s, n, g.rp, g.ci, which, parent);
        hipLaunchKernelGGL(k_cc_compress, dim3(nl), dim3(256), 0, s, n, parent, (const int32_t*)nullptr,
                           (uint8_t*)nullptr, (int64_t*)nullptr);
    }
    // dominant component: most frequent root among evenly spaced samples,
    // found on the device (no host round trip); it sits in size[n + 1],
    // past what the counting below clears
    int ns = n < CC_NS ? n : CC_NS;
    int32_t* giant_sample = (int32_t*)(size + n + 1);
    hipLaunchKernelGGL(k_cc_mode, dim3(1), dim3(CC_NS), 0, s, n, ns, (const int32_t*)parent, giant_sample);
    hipLaunchKernelGGL(k_cc_compress, dim3(nl), dim3(256), 0, s, n, parent, (const int32_t*)giant_sample, in_giant,
                       (int64_t*)nullptr);
    int nh = nblk((int64_t)nheavy * 64, 256);
    hipLaunchKernelGGL(k_cc_link_rest, dim3(nl + nh), dim3(256), 0, s, n, g.rp, g.ci, g.deg, heavy, nheavy,
                       nl, first, in_giant, parent);
    // the last compression also clears the component counters
    hipLaunchKernelGGL(k_cc_compress, dim3(nl), dim3(256), 0, s, n, parent, (const int32_t*)nullptr,
                       (uint8_t*)nullptr, size);
    hipLaunchKernelGGL(k_cc_count, dim3(nl), dim3(256), 0, s, n, parent, (const int32_t*)giant_sample, size,
                       size + n);
    hipLaunchKernelGGL(k_cc_assign, dim3(nl), dim3(256), 0, s, n, parent, size, (const int32_t*)giant_sample,
                       size + n, alpha, omega);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// open vertices below which a round first treats them alone
#define NB_TAIL_DIV 64

// lanes per light vertex in a full round; TKC_NB_LPV = 1, 2, 4 or 8 picks
// one for experiments
#define NB_LPV_DEFAULT 4
static int nb_lpv() {
    static const int v = [] {
        const char* e = getenv("TKC_NB_LPV");
        const int x = e ? atoi(e) : NB_LPV_DEFAULT;
        return (x == 1 || x == 2 || x == 4 || x == 8) ? x : NB_LPV_DEFAULT;
    }();
    return v;
}
// experiment switch: TKC_NB_C32=0 gathers the 64-bit counts only
static bool nb_c32() {
    static const bool v = [] {
        const char* e = getenv("TKC_NB_C32");
        return !(e && atoi(e) == 0);
    }();
    return v;
}
template <bool DIRECTED, typename G, typename... A>
static void launch_nb_round(int lpv, dim3 grid, hipStream_t s, A... args) {
    switch (lpv) {
        case 1:
            // one lane per vertex has no capped-count fallback: 64-bit only
            // (the caller takes the 32-bit copy only with lpv > 1, and the
            // grid is sized for lpv, so no other width may stand in)
            if constexpr (sizeof(G) == 8)
                hipLaunchKernelGGL((k_nb_round<DIRECTED, 1, G>), grid, dim3(256), 0, s, args...);
            break;
        case 2: hipLaunchKernelGGL((k_nb_round<DIRECTED, 2, G>), grid, dim3(256), 0, s, args...); break;
        case 8: hipLaunchKernelGGL((k_nb_round<DIRECTED, 8, G>), grid, dim3(256), 0, s, args...); break;
        default: hipLaunchKernelGGL((k_nb_round<DIRECTED, 4, G>), grid, dim3(256), 0, s, args...); break;
    }
}

// NB bound: returns the number of rounds, -1 on error.  gbuf holds 3*n int64
// and then 2*n int32;
// partial holds the heavy chunks' partial sums and also at least
// n / NB_TAIL_DIV int32; nfin_dev holds NB_TAILCNT_WORD + 1 int32 (the
// finish counters, their total, the tail list's count).
int tkc_launch_nb(const DevGraph& g, const int64_t* alpha, const int64_t* omega, int64_t* gbuf, int64_t* sum,
                  int64_t* vis, uint8_t* flags, int64_t* num, int64_t* den, uint64_t* partial,
                  int32_t* nfin_dev, int32_t* nfin_host, hipStream_t s, double* hub,
                  const std::function<int()>* fin, bool* fin_done) {
    int32_t n = g.n;
    if (fin_done) *fin_done = false;
    int nl = nblk(n, 256);
    int nc = nblk((int64_t)g.nchunks * 64, 256);
    int nhb = nblk(g.nheavy, 256);
    NBState st{sum, vis, flags, num, den, hub, nullptr};
    int64_t* buf[3] = {gbuf, gbuf + n, gbuf + 2 * (int64_t)n};
    hipMemsetAsync(nfin_dev, 0, sizeof(int32_t) * NB_TOTAL_WORD, s);
    // gamma_0 -> buf[0], gamma_1 -> buf[1]
    hipLaunchKernelGGL(k_nb_init, dim3(nl), dim3(256), 0, s, n, g.deg, alpha, omega, buf[0], buf[1],
                       st, nfin_dev);
    if (hipGetLastError() != hipSuccess) return -1;
    int32_t done = 0;
    int64_t k = 2;
    const int64_t kmax = (int64_t)n + 2;
    // a full round at level k (adv = 0: counts only, no vertex advances)
    const int lpv = nb_lpv();
    const int nlr = nblk((int64_t)n * lpv, 256);
    // 32-bit copies of two consecutive levels follow the three 64-bit buffers
    int32_t* c32[2] = {(int32_t*)(gbuf + 3 * (int64_t)n), (int32_t*)(gbuf + 3 * (int64_t)n) + n};
    const bool use32 = lpv > 1 && nb_c32();
    auto round = [&](int64_t lv, int32_t adv) {
        int64_t* g1 = buf[(lv - 1) % 3];
        int64_t* g2 = buf[(lv - 2) % 3];
        int64_t* gk = buf[lv % 3];
        NBState rs = st;
        if (use32) {
            // gamma_1 is the out-degree (k_nb_init stores the same values)
            rs.c32 = c32[lv & 1];
            const int32_t* g1c = lv == 2 ? g.deg : c32[(lv - 1) & 1];
            if (g.directed)
                launch_nb_round<true, int32_t>(lpv, dim3(nlr + nc), s, n, g.rp, g.ci, g.deg, g.ch_beg, g.ch_end,
                                               g.nchunks, nlr, lv, g1c, (const int64_t*)g1, (const int64_t*)g2, gk,
                                               alpha, omega, rs, partial, nfin_dev, adv);
            else
                launch_nb_round<false, int32_t>(lpv, dim3(nlr + nc), s, n, g.rp, g.ci, g.deg, g.ch_beg, g.ch_end,
                                                g.nchunks, nlr, lv, g1c, (const int64_t*)g1, (const int64_t*)g2, gk,
                                                alpha, omega, rs, partial, nfin_dev, adv);
        } else if (g.directed) {
            launch_nb_round<true, int64_t>(lpv, dim3(nlr + nc), s, n, g.rp, g.ci, g.deg, g.ch_beg, g.ch_end,
                                           g.nchunks, nlr, lv, (const int64_t*)g1, (const int64_t*)g1,
                                           (const int64_t*)g2, gk, alpha, omega, rs, partial, nfin_dev, adv);
        } else {
            launch_nb_round<false, int64_t>(lpv, dim3(nlr + nc), s, n, g.rp, g.ci, g.deg, g.ch_beg, g.ch_end,
                                            g.nchunks, nlr, lv, (const int64_t*)g1, (const int64_t*)g1,
                                            (const int64_t*)g2, gk, alpha, omega, rs, partial, nfin_dev, adv);
        }
        if (g.nheavy) {
            if (g.directed)
                hipLaunchKernelGGL(k_nb_heavy<true>, dim3(nhb), dim3(256), 0, s, g.nheavy, g.heavy, g.hcb, partial,
                                   g.deg, lv, (const int64_t*)g2, gk, alpha, omega, rs, nfin_dev, adv);
            else
                hipLaunchKernelGGL(k_nb_heavy<false>, dim3(nhb), dim3(256), 0, s, g.nheavy, g.heavy, g.hcb,
                                   partial, g.deg, lv, (const int64_t*)g2, gk, alpha, omega, rs, nfin_dev, adv);
        }
    };
    // the finish count after the rounds queued so far; with `ahead`, round k
    // is queued behind the count's copy, so the GPU works while the host
    // waits for the copy alone (a round after every vertex has finished
    // changes no bound)
    hipEvent_t ev_copy = nullptr;
    if (hipEventCreateWithFlags(&ev_copy, hipEventDisableTiming) != hipSuccess) return -1;
    struct EventGuard {
        hipEvent_t e;
        ~EventGuard() { hipEventDestroy(e); }
    } ev_guard{ev_copy};
    auto check = [&](bool ahead) -> bool {
        hipLaunchKernelGGL(k_nb_total, dim3(1), dim3(64), 0, s, nfin_dev);
        if (hipGetLastError() != hipSuccess) return false;
        if (hipMemcpyAsync(nfin_host, nfin_dev + NB_TOTAL_WORD, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess)
            return false;
        if (ahead) {
            if (hipEventRecord(ev_copy, s) != hipSuccess) return false;
            round(k, 1);
            k++;
            if (hipEventSynchronize(ev_copy) != hipSuccess) return false;
        } else if (hipStreamSynchronize(s) != hipSuccess) {
            return false;
        }
        done = *nfin_host;
        return true;
    };
    // tail rounds: once at most n / NB_TAIL_DIV vertices are open, a round
    // first treats them alone (their list sits in `partial`, which the
    // tail round does not use); if some stay open, a full round at the
    // same level then supplies every other vertex's count, and the next
    // try waits until four times fewer are open
    const int32_t tail_cap = n / NB_TAIL_DIV;
    int32_t tail_at = tail_cap;
    int32_t* tail_list = (int32_t*)partial;
    int32_t* tail_cnt = nfin_dev + NB_TAILCNT_WORD;
    bool checked = false;
    int ahead = 0;   // rounds of the current pair already queued by a check
    while (k <= kmax) {
        const int32_t open = n - done;   // may count some that a queued round finished
        if (checked && open <= tail_at) {
            ahead = 0;
            // tail_cnt was cleared by the check's k_nb_total
            hipLaunchKernelGGL(k_nb_collect, dim3(nblk(n, 1024)), dim3(1024), 0, s, n, (const uint8_t*)flags,
                               tail_cap, tail_list, tail_cnt);
            const int nt = nblk((int64_t)open * 64, 256);
            const int64_t* g1 = buf[(k - 1) % 3];
            const int64_t* g2 = buf[(k - 2) % 3];
            int64_t* gk = buf[k % 3];
            if (g.directed)
                hipLaunchKernelGGL(k_nb_tail<true>, dim3(nt), dim3(256), 0, s, (const int32_t*)tail_cnt, tail_cap,
                                   (const int32_t*)tail_list, g.rp, g.ci, g.deg, k, g1, g2, gk, alpha, omega, st,
                                   nfin_dev);
            else
                hipLaunchKernelGGL(k_nb_tail<false>, dim3(nt), dim3(256), 0, s, (const int32_t*)tail_cnt, tail_cap,
                                   (const int32_t*)tail_list, g.rp, g.ci, g.deg, k, g1, g2, gk, alpha, omega, st,
                                   nfin_dev);
            // a tail round usually finishes every vertex: the caller's work
            // on the final bounds goes ahead of the check's wait
            if (fin && (*fin)()) return -1;
            if (!check(false)) return -1;
            if (done < n) {
                round(k, 0);
                tail_at = (n - done) / 4;
            }
            k++;
            if (done >= n) {
                if (fin_done) *fin_done = fin != nullptr;
                break;
            }
            continue;
        }
        // two full rounds per host check (the first pair without one: the
        // initial level rarely finishes every vertex, so the first check
        // also queues the next round ahead of its wait); once every vertex
        // has finished, further rounds change no bound
        for (int rep = ahead; rep < 2 && k <= kmax; rep++, k++) round(k, 1);
        const bool spec = !checked && k <= kmax;
        if (!check(spec)) return -1;
        ahead = spec ? 1 : 0;
        checked = true;
        if (done >= n) break;
    }
    return (int)(k - 2);
}

int tkc_launch_deg_bounds(const DevGraph& g, const int64_t* omega, int64_t* num, int64_t* den,
                          uint32_t* key, int32_t* val, hipStream_t s) {
    hipLaunchKernelGGL(k_deg_bounds, dim3(nblk(g.n, 256)), dim3(256), 0, s, g.n, g.deg, omega, num,
                       den, key, val);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
int tkc_launch_harm_bounds(const DevGraph& g, const int64_t* omega, const double* hub, int64_t* num,
                           int64_t* den, uint32_t* key, int32_t* val, hipStream_t s) {
    if (hub)
        hipLaunchKernelGGL(k_harm_nb_keys, dim3(nblk(g.n, 256)), dim3(256), 0, s, g.n, hub, num, den, key, val);
    else
        hipLaunchKernelGGL(k_harm_deg_bounds, dim3(nblk(g.n, 256)), dim3(256), 0, s, g.n, g.deg, omega, num, den,
                           key, val);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
int tkc_launch_nb_keys(int32_t n, const int64_t* num, const int64_t* den, uint32_t* key, int32_t* val,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_nb_keys, dim3(nblk(n, 256)), dim3(256), 0, s, n, num, den, key, val);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
