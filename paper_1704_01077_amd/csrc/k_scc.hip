// Reachability bounds of a directed graph on the device (Sect. 8.4, Alg. 6):
// strongly connected components, their DAG, and
//   alpha(C) = w(C) + max over successors D of alpha(D)
//   omega(C) = w(C) + sum over successors D of omega(D)
// with the refinement through the largest component C~ (its reach is
// counted exactly; a component that reaches C~ sums only the successors C~
// does not reach, plus omega(C~) once), omega capped at n.  The values
// depend only on the component partition and its DAG, so they equal the
// host computation exactly.
//
// Components: (1) trimming -- a vertex with no remaining in-arcs or
// out-arcs is a component of its own, repeated; (2) one forward/backward
// search from a high-degree pivot (the giant component of complex
// networks); (3) trimming again; (4) max-colour propagation (a vertex takes
// the largest id that reaches it), then each colour root collects the
// vertices of its colour that reach it -- repeated until every vertex has a
// component.  Each of these steps has a round cap; a step that meets it
// (long chains of components) hands every vertex still unassigned to
// Tarjan's algorithm run by one device thread.
//
// The DAG: every arc between components as a (source, target) pair, sorted
// by two stable radix passes and deduplicated.  Heights (longest path to a
// sink) order the dynamic programme, and components are numbered in
// decreasing height, a topological order.  A DAG deeper than the
// relaxation cap is swept by one device thread in the order of a sinks-first
// peel instead.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dev_common.hpp"
#include "engine.hpp"

#define SB 256
#define SCAN_T 1024
#define SCAN_I 4

static inline int nblk(int64_t n, int per = SB) { return (int)((n + per - 1) / per); }
// blocks for one wave per item, grid-strided beyond 16384 blocks
static inline int wblk(int64_t items) {
    const int64_t b = (items * 64 + SB - 1) / SB;
    return (int)(b < 1 ? 1 : (b < 16384 ? b : 16384));
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(v, o, 64);
        v = y > v ? y : v;
    }
    return v;
}

// Reductions and appends to one global address are aggregated per block
// (grid-strided over at most RB blocks): same-address atomics serialise,
// so one per wave over a million vertices costs a few hundred microseconds.
#define RB 1024
static inline int rblk(int64_t n) {
    const int b = nblk(n);
    return b < 1 ? 1 : (b < RB ? b : RB);
}
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v, unsigned long long* sh) {
    v = wave_max_u64(v);
    if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long r = sh[0];
    for (int w = 1; w < SB / 64; w++) r = sh[w] > r ? sh[w] : r;
    __syncthreads();
    return r;
}
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* sh) {
    v = wave_sum_i64(v);
    if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t r = 0;
    for (int w = 0; w < SB / 64; w++) r += sh[w];
    __syncthreads();
    return r;
}
// block-wide append of the threads whose pred holds: one atomic per call
__device__ __forceinline__ int32_t block_append_base(bool pred, int32_t* cnt, int32_t* sh, int32_t* rank) {
    const uint64_t m = __ballot(pred);
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) sh[wv] = __popcll(m);
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < SB / 64; w++) {
        pre += w < wv ? sh[w] : 0;
        tot += sh[w];
    }
    if (threadIdx.x == 0) sh[SB / 64] = tot ? atomicAdd(cnt, tot) : 0;
    __syncthreads();
    const uint64_t below = lane_id() ? (~0ull >> (64 - lane_id())) : 0ull;
    *rank = pre + __popcll(m & below);
    const int32_t base = sh[SB / 64];
    __syncthreads();
    return base;
}

// ------------------------------------------------------------------ scan
// exclusive scan of n int32 in place (three passes)
__global__ void __launch_bounds__(SCAN_T) k_scan_blocks(int32_t* a, int64_t n, int32_t* bsum) {
    __shared__ int32_t ws[SCAN_T / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_T * SCAN_I + (int64_t)threadIdx.x * SCAN_I;
    int32_t v[SCAN_I], s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_I; j++) {
        v[j] = base + j < n ? a[base + j] : 0;
        s += v[j];
    }
    int32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane_id() >= o) x += y;
    }
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 63) ws[wv] = x;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < SCAN_T / 64; w++) {
        if (w < wv) pre += ws[w];
        tot += ws[w];
    }
    int32_t run = pre + x - s;
#pragma unroll
    for (int j = 0; j < SCAN_I; j++) {
        if (base + j < n) a[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}
__global__ void __launch_bounds__(SCAN_T) k_scan_top(int32_t* b, int32_t nb, int32_t* total) {
    __shared__ int32_t ws[SCAN_T / 64];
    const int32_t per = (nb + SCAN_T - 1) / SCAN_T;
    const int32_t lo = threadIdx.x * per;
    const int32_t hi = lo + per < nb ? lo + per : nb;
    int32_t s = 0;
    for (int32_t i = lo; i < hi; i++) s += b[i];
    int32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane_id() >= o) x += y;
    }
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 63) ws[wv] = x;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < SCAN_T / 64; w++) {
        if (w < wv) pre += ws[w];
        tot += ws[w];
    }
    int32_t run = pre + x - s;
    for (int32_t i = lo; i < hi; i++) {
        const int32_t t = b[i];
        b[i] = run;
        run += t;
    }
    if (threadIdx.x == 0) *total = tot;
}
__global__ void k_scan_add(int32_t* a, int64_t n, const int32_t* bsum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += bsum[i / (SCAN_T * SCAN_I)];
}

// ------------------------------------------------------ components: state
__global__ void k_scc_init(int32_t n, const int32_t* rp, const int32_t* rrp, int32_t* scc, int32_t* in_rem,
                           int32_t* out_rem, uint32_t* mark) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    scc[v] = -1;
    in_rem[v] = rrp[v + 1] - rrp[v];
    out_rem[v] = rp[v + 1] - rp[v];
    mark[v] = 0;
}

// a vertex without remaining in-arcs or out-arcs is a component of its own
__global__ void __launch_bounds__(SB) k_scc_trim(int32_t n, int32_t* scc, const int32_t* in_rem,
                                                 const int32_t* out_rem, int32_t* list, int32_t* cnt) {
    __shared__ int32_t sh[SB / 64 + 1];
    for (int64_t b0 = (int64_t)blockIdx.x * SB; b0 < n; b0 += (int64_t)gridDim.x * SB) {
        const int64_t v = b0 + threadIdx.x;
        const bool take = v < n && scc[v] < 0 && (in_rem[v] <= 0 || out_rem[v] <= 0);
        int32_t rank;
        const int32_t base = block_append_base(take, cnt, sh, &rank);
        if (take) {
            scc[v] = (int32_t)v;
            list[base + rank] = (int32_t)v;
        }
    }
}
// removed vertices take their arcs away from their neighbours' counts
__global__ void k_scc_trim_update(const int32_t* list, int32_t cnt, const int32_t* rp, const int32_t* ci,
                                  const int32_t* rrp, const int32_t* rci, int32_t* in_rem, int32_t* out_rem) {
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    for (int64_t i = gw; i < cnt; i += nw) {
        const int32_t v = list[i];
        for (int32_t e = rp[v] + lane_id(); e < rp[v + 1]; e += 64) atomicSub(&in_rem[ci[e]], 1);
        for (int32_t e = rrp[v] + lane_id(); e < rrp[v + 1]; e += 64) atomicSub(&out_rem[rci[e]], 1);
    }
}

// pivot: the unassigned vertex with the largest (in+1)(out+1), smallest id on ties
__global__ void __launch_bounds__(SB) k_scc_pivot(int32_t n, const int32_t* scc, const int32_t* in_rem,
                                                  const int32_t* out_rem, unsigned long long* best) {
    __shared__ unsigned long long sh[SB / 64];
    unsigned long long key = 0;
    for (int64_t v = (int64_t)blockIdx.x * SB + threadIdx.x; v < n; v += (int64_t)gridDim.x * SB) {
        if (scc[v] >= 0) continue;
        uint64_t p = (uint64_t)(in_rem[v] + 1) * (uint64_t)(out_rem[v] + 1);
        if (p > 0x7fffffffull) p = 0x7fffffffull;
        const unsigned long long k = ((unsigned long long)p << 32) | (0xffffffffull - (uint32_t)v);
        key = k > key ? k : key;
    }
    key = block_max_u64(key, sh);
    if (threadIdx.x == 0 && key) atomicMax(best, key);
}

// the same level as a pull: an unassigned vertex not yet found looks for a
// predecessor found at level nl - 1 (its own thread, first hit ends it);
// used when the frontier is a large part of the graph
__global__ void k_scc_pull(int32_t n, const int32_t* prp, const int32_t* pci, const int32_t* scc, uint32_t* mark,
                           uint32_t bit, int32_t* lev, int32_t nl) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (scc[v] >= 0 || (mark[v] & bit)) continue;
        for (int32_t e = prp[v]; e < prp[v + 1]; e++) {
            if (__hip_atomic_load(&lev[pci[e]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nl - 1) {
                mark[v] |= bit;
                __hip_atomic_store(&lev[v], nl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
}
// out-degrees (in the search's direction) of the frontier entries, zero
// past its end: an exclusive scan of these spreads its arcs evenly
__global__ void k_front_deg(int32_t n, const int32_t* fr, const int32_t* fcnt_dev, const int32_t* arp, int32_t* deg) {
    const int32_t fcnt = *fcnt_dev;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        deg[i] = i < fcnt ? arp[fr[i] + 1] - arp[fr[i]] : 0;
}
// one level of a push over the frontier's arcs, one thread per arc: arc j
// belongs to the last entry whose prefix pre[] is <= j
__global__ void k_scc_push(const int32_t* fr, const int32_t* pre, int32_t fcnt, int64_t farcs, const int32_t* arp,
                           const int32_t* aci, const int32_t* scc, uint32_t* mark, uint32_t bit, int32_t* lev,
                           int32_t nl) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < farcs;
         j += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = fcnt - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= j) lo = mid;
            else hi = mid - 1;
        }
        const int32_t u = fr[lo];
        const int32_t w = aci[arp[u] + (int32_t)(j - pre[lo])];
        if (scc[w] < 0 && !(mark[w] & bit) && !(atomicOr(&mark[w], bit) & bit)) lev[w] = nl;
    }
}
// the vertices of level nl, in id order: flags, then (after a scan) scatter
__global__ void k_lev_flag(int32_t n, const int32_t* lev, int32_t nl, int32_t* flag) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = lev[v] == nl;
}
__global__ void k_lev_scatter(int32_t n, const int32_t* lev, int32_t nl, const int32_t* pos, int32_t* out) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && lev[v] == nl) out[pos[v]] = v;
}
__global__ void k_scc_seed(int32_t* list, uint32_t* mark, int32_t* lev, int32_t pivot, uint32_t bit,
                           int32_t* fcnt_dev) {
    if (threadIdx.x == 0) {
        list[0] = pivot;
        mark[pivot] |= bit;
        lev[pivot] = 0;
        *fcnt_dev = 1;
    }
}
__global__ void k_scc_assign_fb(int32_t n, int32_t* scc, uint32_t* mark, int32_t pivot) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (scc[v] < 0 && (mark[v] & 3u) == 3u) scc[v] = pivot;
    mark[v] = 0;
}

// arcs between unassigned vertices only (one wave per vertex)
__global__ void k_scc_recount(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* rrp, const int32_t* rci,
                              const int32_t* scc, int32_t* in_rem, int32_t* out_rem) {
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    for (int64_t v = gw; v < n; v += nw) {
        if (scc[v] >= 0) continue;
        int32_t a = 0, b = 0;
        for (int32_t e = rrp[v] + lane_id(); e < rrp[v + 1]; e += 64) a += scc[rci[e]] < 0;
        for (int32_t e = rp[v] + lane_id(); e < rp[v + 1]; e += 64) b += scc[ci[e]] < 0;
        a = wave_sum_i32(a);
        b = wave_sum_i32(b);
        if (lane_id() == 0) {
            in_rem[v] = a;
            out_rem[v] = b;
        }
    }
}

// colouring: every unassigned vertex takes the largest id that reaches it
__global__ void __launch_bounds__(SB) k_col_init(int32_t n, const int32_t* scc, int32_t* color,
                                                 int32_t* unassigned) {
    __shared__ int64_t sh[SB / 64];
    int64_t c = 0;
    for (int64_t v = (int64_t)blockIdx.x * SB + threadIdx.x; v < n; v += (int64_t)gridDim.x * SB) {
        const bool un = scc[v] < 0;
        color[v] = un ? (int32_t)v : -1;
        c += un;
    }
    c = block_sum_i64(c, sh);
    if (threadIdx.x == 0 && c) atomicAdd(unassigned, (int32_t)c);
}
__global__ void k_col_prop(int32_t n, const int32_t* rrp, const int32_t* rci, const int32_t* scc, int32_t* color,
                           int32_t* changed) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || scc[v] >= 0) return;
    int32_t c = color[v];
    const int32_t c0 = c;
    for (int32_t e = rrp[v]; e < rrp[v + 1]; e++) {
        const int32_t cu = __hip_atomic_load(&color[rci[e]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cu > c) c = cu;
    }
    if (c > c0) {
        atomicMax(&color[v], c);
        *changed = 1;
    }
}
// roots collect the vertices of their colour that reach them
__global__ void k_col_close_init(int32_t n, const int32_t* scc, const int32_t* color, uint32_t* mark) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) mark[v] = (scc[v] < 0 && color[v] == v) ? 1u : 0u;
}
__global__ void k_col_close(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* scc,
                            const int32_t* color, uint32_t* mark, int32_t* changed) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || scc[v] >= 0 || mark[v]) return;
    const int32_t c = color[v];
    for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
        const int32_t w = ci[e];
        if (color[w] == c && __hip_atomic_load(&mark[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            mark[v] = 1u;
            *changed = 1;
            return;
        }
    }
}
__global__ void k_col_assign(int32_t n, int32_t* scc, const int32_t* color, uint32_t* mark) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (scc[v] < 0 && mark[v]) scc[v] = color[v];
    mark[v] = 0;
}

// ------------------------------------------------------- dense component ids
__global__ void k_rep_flag(int32_t n, const int32_t* scc, int32_t* cid) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) cid[v] = scc[v] == v ? 1 : 0;
}
__global__ void k_comp_of(int32_t n, const int32_t* scc, const int32_t* cid, int32_t* comp) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) comp[v] = cid[scc[v]];
}
// minid: the smallest caller's id in each component (oid: the caller's id of
// each vertex of a relabelled graph, or null)
__global__ void __launch_bounds__(SB) k_comp_stats(int32_t n, const int32_t* comp, int32_t pivot, int32_t* wt,
                                                   int32_t* minid, const int32_t* oid) {
    // the pivot's component holds most vertices: one atomic per block for it
    __shared__ int64_t sh[SB / 64];
    __shared__ unsigned long long shm[SB / 64];
    const int32_t hot = pivot >= 0 ? comp[pivot] : -1;
    int64_t hc = 0;
    unsigned long long hm = 0;   // 0xffffffff - smallest id of the hot component seen
    for (int64_t v = (int64_t)blockIdx.x * SB + threadIdx.x; v < n; v += (int64_t)gridDim.x * SB) {
        const int32_t c = comp[v];
        const int32_t id = oid ? oid[v] : (int32_t)v;
        if (c == hot) {
            hc++;
            const unsigned long long k = 0xffffffffull - (uint32_t)id;
            hm = k > hm ? k : hm;
        } else {
            atomicAdd(&wt[c], 1);
            atomicMin(&minid[c], id);
        }
    }
    hc = block_sum_i64(hc, sh);
    hm = block_max_u64(hm, shm);
    if (threadIdx.x == 0 && hc) {
        atomicAdd(&wt[hot], (int32_t)hc);
        atomicMin(&minid[hot], (int32_t)(0xffffffffull - hm));
    }
}
// the largest component, ties to the one holding the smallest vertex id
__global__ void __launch_bounds__(SB) k_comp_big(int32_t nc, const int32_t* wt, const int32_t* minid,
                                                 unsigned long long* best) {
    __shared__ unsigned long long sh[SB / 64];
    unsigned long long key = 0;
    for (int64_t c = (int64_t)blockIdx.x * SB + threadIdx.x; c < nc; c += (int64_t)gridDim.x * SB) {
        const unsigned long long k = ((unsigned long long)(uint32_t)wt[c] << 32) | (0xffffffffull - (uint32_t)minid[c]);
        key = k > key ? k : key;
    }
    key = block_max_u64(key, sh);
    if (threadIdx.x == 0 && key) atomicMax(best, key);
}

__global__ void k_set_big(const int32_t* comp, int32_t bmin, const int32_t* nid, int32_t* tob, int32_t* frb,
                          int32_t* out) {
    if (threadIdx.x == 0) {
        const int32_t c = comp[nid ? nid[bmin] : bmin];
        tob[c] = 1;
        frb[c] = 1;
        *out = c;
    }
}

// --------------------------------------------------------------- the DAG
// arcs leaving each vertex's component: a thread per light vertex, a wave
// per heavy one (more than HEAVY_DEG out-arcs)
__global__ void k_dag_count(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* comp, int32_t* cnt) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        if (rp[u + 1] - rp[u] > HEAVY_DEG) continue;
        const int32_t cu = comp[u];
        int32_t c = 0;
        for (int32_t e = rp[u]; e < rp[u + 1]; e++) c += comp[ci[e]] != cu;
        cnt[u] = c;
    }
}
// heavy vertices: one wave per chunk of CHUNK_ARCS arcs, then each heavy
// vertex sums its chunks and notes where they start
__global__ void k_dag_chunk_count(int32_t nchunks, const int32_t* ch_beg, const int32_t* ch_end,
                                  const int32_t* ch_vtx, const int32_t* ci, const int32_t* comp, int32_t* ccnt) {
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    for (int64_t c = gw; c < nchunks; c += nw) {
        const int32_t cu = comp[ch_vtx[c]];
        int32_t k = 0;
        for (int32_t e = ch_beg[c] + lane_id(); e < ch_end[c]; e += 64) k += comp[ci[e]] != cu;
        k = wave_sum_i32(k);
        if (lane_id() == 0) ccnt[c] = k;
    }
}
__global__ void k_dag_heavy_sum(int32_t nheavy, const int32_t* heavy, const int32_t* hcb, const int32_t* ccnt,
                                int32_t* cnt, int32_t* cfirst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nheavy) return;
    int32_t k = 0;
    for (int32_t c = hcb[i]; c < hcb[i + 1]; c++) {
        k += ccnt[c];
        cfirst[c] = hcb[i];
    }
    cnt[heavy[i]] = k;
}
__global__ void k_dag_pairs(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* comp, const int32_t* off,
                            uint32_t* key, int32_t* val) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        if (rp[u + 1] - rp[u] > HEAVY_DEG) continue;
        const int32_t cu = comp[u];
        int32_t o = off[u];
        for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
            const int32_t cw = comp[ci[e]];
            if (cw != cu) {
                key[o] = (uint32_t)cw;   // first pass: by target
                val[o] = cu;
                o++;
            }
        }
    }
}
// chunk c writes from off[owner] + (its owner's arcs in earlier chunks),
// cpre[] being the exclusive scan of the chunk counts
__global__ void k_dag_chunk_pairs(int32_t nchunks, const int32_t* ch_beg, const int32_t* ch_end,
                                  const int32_t* ch_vtx, const int32_t* ci, const int32_t* comp, const int32_t* off,
                                  const int32_t* cpre, const int32_t* cfirst, uint32_t* key, int32_t* val) {
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
    const uint64_t below = lane_id() ? (~0ull >> (64 - lane_id())) : 0ull;
    for (int64_t c = gw; c < nchunks; c += nw) {
        const int32_t u = ch_vtx[c];
        const int32_t cu = comp[u];
        int32_t o = off[u] + cpre[c] - cpre[cfirst[c]];
        for (int32_t e0 = ch_beg[c]; e0 < ch_end[c]; e0 += 64) {
            const int32_t e = e0 + lane_id();
            int32_t cw = cu;
            if (e < ch_end[c]) cw = comp[ci[e]];
            const bool x = cw != cu;
            const uint64_t m = __ballot(x);
            if (x) {
                const int32_t p = o + __popcll(m & below);
                key[p] = (uint32_t)cw;
                val[p] = cu;
            }
            o += __popcll(m);
        }
    }
}
// after the second pass (by source, stable): key = source, val = target
__global__ void k_dag_uniq(int64_t E, const uint32_t* src, const int32_t* dst, int32_t* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < E) flag[i] = (i == 0 || src[i] != src[i - 1] || dst[i] != dst[i - 1]) ? 1 : 0;
}
__global__ void k_dag_compact(int64_t E, const uint32_t* src, const int32_t* dst, const int32_t* pos,
                              const int32_t* flag, int32_t* asrc, int32_t* adst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < E && flag[i]) {
        asrc[pos[i]] = (int32_t)src[i];
        adst[pos[i]] = dst[i];
    }
}

// inclusive scan within runs of equal keys (runs are contiguous lanes)
template <typename T, typename Op>
__device__ __forceinline__ T seg_scan(T v, int32_t key, Op op) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(v, o, 64);
        const int32_t yk = __shfl_up(key, o, 64);
        if (lane_id() >= o && yk == key) v = op(v, y);
    }
    return v;
}
// the last lane of its run of equal keys within the wave (a shuffle: call
// it from every lane, outside divergent branches)
__device__ __forceinline__ bool seg_tail(int32_t key) {
    const int32_t nk = __shfl_down(key, 1, 64);
    return lane_id() == 63 || nk != key;
}

// one relaxation round over the DAG arcs (sorted by source): heights
// (longest path to a sink), "reaches C~" and "reached from C~"
__global__ void k_dag_relax(int32_t U, const int32_t* asrc, const int32_t* adst, int32_t* hgt, int32_t* tob,
                            int32_t* frb, int32_t* changed) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = j < U;
    const int32_t c = ok ? asrc[j] : -1;
    const int32_t d = ok ? adst[j] : 0;
    int32_t h = 0, t = 0;
    bool ch = false;
    if (ok) {
        h = __hip_atomic_load(&hgt[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        t = __hip_atomic_load(&tob[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_load(&frb[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
            !__hip_atomic_load(&frb[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(&frb[d], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ch = true;
        }
    }
    h = seg_scan(h, c, [](int32_t x, int32_t y) { return x > y ? x : y; });
    t = seg_scan(t, c, [](int32_t x, int32_t y) { return x | y; });
    const bool tail = seg_tail(c);   // every lane takes part in the shuffle
    if (ok && tail) {
        if (h > __hip_atomic_load(&hgt[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            atomicMax(&hgt[c], h);
            ch = true;
        }
        if (t && !__hip_atomic_load(&tob[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(&tob[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ch = true;
        }
    }
    if (__ballot(ch) && lane_id() == 0) *changed = 1;
}
// |reach of C~| and the largest height (one atomic per wave each)
__global__ void __launch_bounds__(SB) k_dag_reach_big(int32_t nc, const int32_t* wt, const int32_t* frb,
                                                      const int32_t* hgt, unsigned long long* rb, int32_t* hmax) {
    __shared__ int64_t sh[SB / 64];
    __shared__ unsigned long long shm[SB / 64];
    int64_t w = 0;
    unsigned long long h = 0;
    for (int64_t c = (int64_t)blockIdx.x * SB + threadIdx.x; c < nc; c += (int64_t)gridDim.x * SB) {
        if (frb[c]) w += wt[c];
        h = (unsigned long long)hgt[c] > h ? (unsigned long long)hgt[c] : h;
    }
    w = block_sum_i64(w, sh);
    h = block_max_u64(h, shm);
    if (threadIdx.x == 0) {
        if (w) atomicAdd(rb, (unsigned long long)w);
        atomicMax(hmax, (int32_t)h);
    }
}
// sort keys: components and arcs by decreasing height (of the source)
__global__ void k_comp_hkey(int32_t nc, const int32_t* hgt, int32_t hmax, uint32_t* key, int32_t* val) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    key[c] = (uint32_t)(hmax - hgt[c]);
    val[c] = c;
}
__global__ void k_arc_hkey(int32_t U, const int32_t* asrc, const int32_t* hgt, int32_t hmax, uint32_t* key,
                           int32_t* val) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= U) return;
    key[j] = (uint32_t)(hmax - hgt[asrc[j]]);
    val[j] = j;
}
// first position of every key in a sorted key array (-1 where absent)
__global__ void k_bucket_starts(int32_t cnt, const uint32_t* key, int32_t* start) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt && (i == 0 || key[i] != key[i - 1])) start[key[i]] = i;
}
__global__ void k_topo_of(int32_t nc, const int32_t* byh, int32_t* topo) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) topo[byh[i]] = i;
}
__global__ void k_arc_gather(int32_t U, const int32_t* idx, const int32_t* asrc, const int32_t* adst, int32_t* hsrc,
                             int32_t* hdst) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U) return;
    hsrc[i] = asrc[idx[i]];
    hdst[i] = adst[idx[i]];
}
// Alg. 6 for one height: the successors' contributions (arcs [lo, hi),
// sorted by source), one atomic per run of a source within a wave ...
__global__ void k_dp_arcs(int32_t lo, int32_t hi, const int32_t* hsrc, const int32_t* hdst, const int64_t* ca,
                          const int64_t* co, const int32_t* frb, unsigned long long* accA, unsigned long long* accO,
                          unsigned long long* accO2) {
    const int32_t j = lo + blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = j < hi;
    const int32_t c = ok ? hsrc[j] : -1;
    int64_t a = 0, o = 0, o2 = 0;
    if (ok) {
        const int32_t d = hdst[j];
        a = ca[d];
        o = co[d];
        o2 = frb[d] ? 0 : o;
    }
    a = seg_scan(a, c, [](int64_t x, int64_t y) { return x > y ? x : y; });
    o = seg_scan(o, c, [](int64_t x, int64_t y) { return x + y; });
    o2 = seg_scan(o2, c, [](int64_t x, int64_t y) { return x + y; });
    const bool tail = seg_tail(c);   // every lane takes part in the shuffle
    if (ok && tail) {
        atomicMax(&accA[c], (unsigned long long)a);
        atomicAdd(&accO[c], (unsigned long long)o);
        atomicAdd(&accO2[c], (unsigned long long)o2);
    }
}
// ... then the components of that height (byh[lo, hi))
__global__ void k_dp_fin(int32_t lo, int32_t hi, const int32_t* byh, int32_t big, int64_t n, const int32_t* wt,
                         const int32_t* tob, const unsigned long long* rb, const unsigned long long* accA,
                         const unsigned long long* accO, const unsigned long long* accO2, int64_t* ca, int64_t* co) {
    const int32_t i = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hi) return;
    const int32_t c = byh[i];
    if (c == big) {
        ca[c] = co[c] = (int64_t)*rb;
        return;
    }
    int64_t o = tob[c] ? (int64_t)accO2[c] + (int64_t)*rb : (int64_t)accO[c];
    o += wt[c];
    ca[c] = (int64_t)accA[c] + wt[c];
    co[c] = o > n ? n : o;
}
__global__ void k_scc_out(int32_t n, const int32_t* comp, const int64_t* ca, const int64_t* co, const int32_t* topo,
                          int64_t* alpha, int64_t* omega, int32_t* scc_topo) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t c = comp[v];
    alpha[v] = ca[c];
    omega[v] = co[c];
    scc_topo[v] = topo[c];
}

// ------------------------------------------- one-thread passes for chains
// The parallel steps converge in a number of rounds that grows with the
// length of the longest chain of components (a directed path of 10^4
// vertices needs 10^4 search levels, and colouring can need that many
// rounds per component).  Past their round caps the rest is finished by
// the passes below, one thread each: linear in the vertices and arcs they
// touch, whatever the chain length.

// the unassigned vertices, in id order (flags, then after a scan a scatter)
__global__ void k_unassigned_flag(int32_t n, const int32_t* scc, int32_t* flag) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = scc[v] < 0;
}
__global__ void k_unassigned_scatter(int32_t n, const int32_t* scc, const int32_t* pos, int32_t* out) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && scc[v] < 0) out[pos[v]] = v;
}

// Tarjan's algorithm, iteratively, over the subgraph of unassigned vertices
// (ulist[0, ucnt)), one thread.  Every component gets the id of its root,
// a member, as the parallel steps do.  idx[] must be -1 on every listed
// vertex; low, tstk, cstk and epos hold n entries each.  A vertex whose
// scc[] is set is either assigned by an earlier step or closed by this
// pass; in both cases its arcs lead nowhere new and are skipped.
__global__ void k_seq_scc(const int32_t* ulist, int32_t ucnt, const int32_t* rp, const int32_t* ci, int32_t* scc,
                          int32_t* idx, int32_t* low, int32_t* tstk, int32_t* cstk, int32_t* epos) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int32_t nidx = 0;
    for (int32_t i = 0; i < ucnt; i++) {
        const int32_t s0 = ulist[i];
        if (idx[s0] >= 0) continue;
        int32_t tsp = 0, csp = 0;
        idx[s0] = low[s0] = nidx++;
        epos[s0] = rp[s0];
        tstk[tsp++] = s0;
        cstk[csp++] = s0;
        while (csp > 0) {
            const int32_t u = cstk[csp - 1];
            const int32_t e = epos[u];
            if (e < rp[u + 1]) {
                epos[u] = e + 1;
                const int32_t w = ci[e];
                if (scc[w] >= 0) continue;
                const int32_t iw = idx[w];
                if (iw < 0) {
                    idx[w] = low[w] = nidx++;
                    epos[w] = rp[w];
                    tstk[tsp++] = w;
                    cstk[csp++] = w;
                } else if (iw < low[u]) {
                    low[u] = iw;   // w is open: on the search stack
                }
            } else {
                csp--;
                const int32_t lu = low[u];
                if (csp > 0) {
                    const int32_t p = cstk[csp - 1];
                    if (lu < low[p]) low[p] = lu;
                }
                if (lu == idx[u]) {
                    int32_t w;
                    do {
                        w = tstk[--tsp];
                        scc[w] = u;
                    } while (w != u);
                }
            }
        }
    }
}

// Alg. 6 over a deep component DAG, one thread: arcs asrc/adst (U of them,
// deduplicated, sorted by source), component weights wt, the largest
// component big.  The components are peeled sinks first (Kahn's order on
// the reversed DAG), which puts every component after all of its
// successors; "reaches big" follows in that order, "reached from big" in
// the opposite one, then alpha and omega as in the parallel sweep by
// height.  topo numbers the components in the reverse of the peel order, a
// topological order.  soff, poff: nc + 1 entries; cnt, queue, cur: nc;
// pred: U.
__global__ void k_seq_dag(int32_t nc, int32_t U, const int32_t* asrc, const int32_t* adst, const int32_t* wt,
                          int32_t big, int64_t n, int32_t* soff, int32_t* poff, int32_t* pred, int32_t* cnt,
                          int32_t* queue, int32_t* cur, int32_t* tob, int32_t* frb, int64_t* ca, int64_t* co,
                          int32_t* topo, int32_t* err) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    // successor lists: the arcs are grouped by source
    int32_t j = 0;
    for (int32_t c = 0; c < nc; c++) {
        soff[c] = j;
        while (j < U && asrc[j] == c) j++;
    }
    soff[nc] = U;
    // predecessor lists by counting
    for (int32_t c = 0; c <= nc; c++) poff[c] = 0;
    for (int32_t a = 0; a < U; a++) poff[adst[a] + 1]++;
    for (int32_t c = 0; c < nc; c++) poff[c + 1] += poff[c];
    for (int32_t c = 0; c < nc; c++) cur[c] = poff[c];
    for (int32_t a = 0; a < U; a++) pred[cur[adst[a]]++] = asrc[a];
    // peel: a component joins the queue once all its successors are in it
    int32_t qt = 0;
    for (int32_t c = 0; c < nc; c++) {
        cnt[c] = soff[c + 1] - soff[c];
        if (cnt[c] == 0) queue[qt++] = c;
    }
    for (int32_t qh = 0; qh < qt; qh++) {
        const int32_t c = queue[qh];
        for (int32_t q = poff[c]; q < poff[c + 1]; q++)
            if (--cnt[pred[q]] == 0) queue[qt++] = pred[q];
    }
    if (qt != nc) {   // not acyclic: the components are wrong
        *err = 1;
        return;
    }
    // reaches big: successors first
    for (int32_t i = 0; i < nc; i++) {
        const int32_t c = queue[i];
        int32_t t = c == big;
        for (int32_t q = soff[c]; q < soff[c + 1] && !t; q++) t = tob[adst[q]];
        tob[c] = t;
    }
    // reached from big: predecessors first
    int64_t rb = 0;
    for (int32_t i = nc - 1; i >= 0; i--) {
        const int32_t c = queue[i];
        int32_t f = c == big;
        for (int32_t q = poff[c]; q < poff[c + 1] && !f; q++) f = frb[pred[q]];
        frb[c] = f;
        if (f) rb += wt[c];
    }
    // alpha and omega, successors first
    for (int32_t i = 0; i < nc; i++) {
        const int32_t c = queue[i];
        topo[c] = nc - 1 - i;
        if (c == big) {
            ca[c] = co[c] = rb;
            continue;
        }
        int64_t a = 0, o = 0, o2 = 0;
        for (int32_t q = soff[c]; q < soff[c + 1]; q++) {
            const int32_t d = adst[q];
            a = ca[d] > a ? ca[d] : a;
            o += co[d];
            if (!frb[d]) o2 += co[d];
        }
        if (tob[c]) o = o2 + rb;
        o += wt[c];
        ca[c] = a + wt[c];
        co[c] = o > n ? n : o;
    }
}

// ------------------------------------------------------------------ host
namespace {

struct Scratch {
    void* base = nullptr;
    char* p = nullptr;
    template <typename T>
    T* take(int64_t count) {
        T* r = (T*)p;
        p += ((int64_t)sizeof(T) * (count > 0 ? count : 1) + 255) / 256 * 256;
        return r;
    }
};

int scan(int32_t* a, int64_t n, int32_t* bsum, int32_t* total_dev, hipStream_t s) {
    const int64_t per = SCAN_T * SCAN_I;
    const int nb = (int)((n + per - 1) / per);
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(SCAN_T), 0, s, a, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, s, bsum, nb, total_dev);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(n)), dim3(SB), 0, s, a, n, bsum);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

double wall_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int32_t read_i32(const int32_t* dev, int32_t* pin, hipStream_t s) {
    if (hipMemcpyAsync(pin, dev, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    return *pin;
}

}  // namespace

// Returns 0 on success (*seq_used: a one-thread pass finished a long chain),
// -2 when the scratch arena cannot be allocated, -3 when the caller's arena
// (arena_bytes) is smaller than the *need bytes this graph takes, -1 on a
// device error.  arena NULL: the function allocates its own and frees it.  pinned: at least 256 bytes of pinned host memory.
int tkc_device_alpha_omega(const DevGraph& g, int64_t* alpha, int64_t* omega, int32_t* scc_topo, void* pinned,
                           hipStream_t s, int* seq_used, void* arena, size_t arena_bytes, size_t* need) {
    *seq_used = 0;
    const int32_t n = g.n;
    const int64_t m = g.m;
    if (n <= 0) return 0;
    const int gb = nblk(n);
    const int64_t mx = m > n ? m : n;
    const int64_t words_scan = mx / (SCAN_T * SCAN_I) + 2;
    const int64_t hist_words = tkc_sort_hist_words((int32_t)mx);
    Scratch sc;
    // scratch: vertex arrays, component arrays, arc arrays, scan and sort
    // state; the same sequence of takes sizes it (base null) and lays it out
    int32_t* scc = nullptr;
    int32_t* in_rem = nullptr;
    int32_t* out_rem = nullptr;
    uint32_t* mark = nullptr;
    int32_t* color = nullptr;
    int32_t* list = nullptr;
    int32_t* next = nullptr;
    int32_t* cid = nullptr;
    int32_t* comp = nullptr;
    int32_t* cnt = nullptr;
    int32_t* wt = nullptr;
    int32_t* minid = nullptr;
    int32_t* hgt = nullptr;
    int32_t* tob = nullptr;
    int32_t* frb = nullptr;
    int32_t* topo = nullptr;
    int32_t* cstart = nullptr;
    int32_t* astart = nullptr;
    int64_t* ca = nullptr;
    int64_t* co = nullptr;
    unsigned long long *accA = nullptr, *accO = nullptr, *accO2 = nullptr;
    uint32_t* key = nullptr;
    int32_t* val = nullptr;
    uint32_t* tkey = nullptr;
    int32_t* tval = nullptr;
    int32_t* flag = nullptr;
    int32_t* pos = nullptr;
    int32_t* asrc = nullptr;
    int32_t* adst = nullptr;
    int32_t* hsrc = nullptr;
    int32_t* hdst = nullptr;
    int32_t *ccnt = nullptr, *cfirst = nullptr;   // heavy-vertex chunks
    int32_t* bsum = nullptr;
    int32_t* hist = nullptr;
    int32_t* small = nullptr;
    auto layout = [&](char* base) -> size_t {
        sc.p = base;
        scc = sc.take<int32_t>(n);
        in_rem = sc.take<int32_t>(n);
        out_rem = sc.take<int32_t>(n);
        mark = sc.take<uint32_t>(n);
        color = sc.take<int32_t>(n);
        list = sc.take<int32_t>(n);
        next = sc.take<int32_t>(n);
        cid = sc.take<int32_t>(n);
        comp = sc.take<int32_t>(n);
        cnt = sc.take<int32_t>(n);
        wt = sc.take<int32_t>(n);
        minid = sc.take<int32_t>(n);
        hgt = sc.take<int32_t>(n);
        tob = sc.take<int32_t>(n);
        frb = sc.take<int32_t>(n);
        topo = sc.take<int32_t>(n);
        cstart = sc.take<int32_t>((int64_t)n + 2);
        astart = sc.take<int32_t>((int64_t)n + 2);
        ca = sc.take<int64_t>(n);
        co = sc.take<int64_t>(n);
        accA = sc.take<unsigned long long>(n);
        accO = sc.take<unsigned long long>(n);
        accO2 = sc.take<unsigned long long>(n);
        key = sc.take<uint32_t>(m);
        val = sc.take<int32_t>(m);
        tkey = sc.take<uint32_t>(m);
        tval = sc.take<int32_t>(m);
        flag = sc.take<int32_t>(m);
        pos = sc.take<int32_t>(m);
        asrc = sc.take<int32_t>(m);
        adst = sc.take<int32_t>(m);
        hsrc = sc.take<int32_t>(m);
        hdst = sc.take<int32_t>(m);
        ccnt = sc.take<int32_t>((int64_t)g.nchunks + 1);
        cfirst = sc.take<int32_t>((int64_t)g.nchunks + 1);
        bsum = sc.take<int32_t>(words_scan);
        hist = sc.take<int32_t>(hist_words);
        small = sc.take<int32_t>(256);
        return (size_t)(sc.p - base);
    };
    const size_t bytes = layout(nullptr);
    if (need) *need = bytes;
    const bool own = arena == nullptr;
    if (own) {
        if (hipMalloc(&sc.base, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return -2;
        }
    } else {
        if (bytes > arena_bytes) return -3;
        sc.base = arena;
    }
    layout((char*)sc.base);
    unsigned long long* big_key = (unsigned long long*)(small + 64);
    unsigned long long* rb = (unsigned long long*)(small + 66);
    uint32_t* smask = (uint32_t*)(small + 70);
    int32_t* pin = (int32_t*)pinned;
    uint32_t* pin_mask = (uint32_t*)pinned + 16;
    int rc = 0;
    int32_t pivot = -1;
    auto fail = [&](int code) { rc = code; return code; };
    // TKC_REACH_TRACE: phase times and round counts on stderr
    const bool tr = getenv("TKC_REACH_TRACE") != nullptr;
    double tph = wall_ms();
    auto phase = [&](const char* what, int64_t a, int64_t b) {
        if (!tr) return;
        (void)hipStreamSynchronize(s);
        const double t = wall_ms();
        fprintf(stderr, "reach %-10s %9.3f ms  %lld %lld\n", what, t - tph, (long long)a, (long long)b);
        tph = t;
    };
#define DEV_OK(x) \
    if ((x) != hipSuccess) { fail(-1); goto done; }
#define STEP_OK(x) \
    if ((x) != 0) { fail(-1); goto done; }
    {
        // round caps of the parallel steps; past them the one-thread passes
        // finish the job (long chains of components)
        const int FB_LEVELS = 1024;    // levels of the pivot's forward or backward search
        const int COL_ITERS = 64;      // colouring iterations
        const int COL_ROUNDS = 256;    // propagation or closing rounds in one iteration
        constexpr int DAG_ROUNDS = 64; // relaxation rounds for the heights
        bool seq = false;
        hipLaunchKernelGGL(k_scc_init, dim3(gb), dim3(SB), 0, s, n, g.rp, g.rrp, scc, in_rem, out_rem, mark);
        auto trim = [&](int max_rounds) -> int {
            for (int r = 0; r < max_rounds; r++) {
                if (hipMemsetAsync(small, 0, 4, s) != hipSuccess) return -1;
                hipLaunchKernelGGL(k_scc_trim, dim3(rblk(n)), dim3(SB), 0, s, n, scc, in_rem, out_rem, list, small);
                const int32_t c = read_i32(small, pin, s);
                if (c < 0) return -1;
                if (c == 0) break;
                hipLaunchKernelGGL(k_scc_trim_update, dim3(wblk(c)), dim3(SB), 0, s, list, c, g.rp, g.ci, g.rrp,
                                   g.rci, in_rem, out_rem);
            }
            return hipGetLastError() == hipSuccess ? 0 : -1;
        };
        STEP_OK(trim(32));
        phase("trim", 0, 0);
        // ---- forward / backward search from the pivot
        DEV_OK(hipMemsetAsync(big_key, 0, 8, s));
        hipLaunchKernelGGL(k_scc_pivot, dim3(rblk(n)), dim3(SB), 0, s, n, scc, in_rem, out_rem, big_key);
        DEV_OK(hipMemcpyAsync(pin, big_key, 8, hipMemcpyDeviceToHost, s));
        DEV_OK(hipStreamSynchronize(s));
        if (*(unsigned long long*)pin != 0) {
            pivot = (int32_t)(0xffffffffull - (*(unsigned long long*)pin & 0xffffffffull));
            int32_t* lev = color;   // free until the colouring
            for (int dir = 0; dir < 2 && !seq; dir++) {
                const uint32_t bit = dir == 0 ? 1u : 2u;
                const int32_t* arp = dir == 0 ? g.rp : g.rrp;
                const int32_t* aci = dir == 0 ? g.ci : g.rci;
                DEV_OK(hipMemsetAsync(lev, 0xff, 4 * (size_t)n, s));
                hipLaunchKernelGGL(k_scc_seed, dim3(1), dim3(64), 0, s, list, mark, lev, pivot, bit, small);
                // frontier size (small[0]), its arcs (small[2]) and their
                // prefix by entry (next[]), read back once per level
                auto frontier = [&]() -> int {
                    hipLaunchKernelGGL(k_front_deg, dim3(rblk(n)), dim3(SB), 0, s, n, list, small, arp, next);
                    if (scan(next, n, bsum, small + 2, s)) return -1;
                    if (hipMemcpyAsync(pin, small, 16, hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
                    if (hipStreamSynchronize(s) != hipSuccess) return -1;
                    return 0;
                };
                STEP_OK(frontier());
                int32_t fcnt = pin[0];
                int64_t farcs = pin[2];
                for (int32_t nl = 1; fcnt > 0; nl++) {
                    if (nl > FB_LEVELS) {
                        seq = true;
                        break;
                    }
                    // a frontier holding a large share of the arcs: pull
                    // over the predecessors instead (direction optimising)
                    if ((int64_t)fcnt * 16 > n || farcs * 8 > m)
                        hipLaunchKernelGGL(k_scc_pull, dim3(nblk(n)), dim3(SB), 0, s, n, dir == 0 ? g.rrp : g.rp,
                                           dir == 0 ? g.rci : g.ci, scc, mark, bit, lev, nl);
                    else if (farcs > 0)
                        hipLaunchKernelGGL(k_scc_push, dim3(std::min(nblk(farcs), 8192)), dim3(SB), 0, s, list, next,
                                           fcnt, farcs, arp, aci, scc, mark, bit, lev, nl);
                    hipLaunchKernelGGL(k_lev_flag, dim3(gb), dim3(SB), 0, s, n, lev, nl, cid);
                    STEP_OK(scan(cid, n, bsum, small, s));
                    hipLaunchKernelGGL(k_lev_scatter, dim3(gb), dim3(SB), 0, s, n, lev, nl, cid, list);
                    STEP_OK(frontier());
                    fcnt = pin[0];
                    farcs = pin[2];
                }
            }
            phase("fw-bw", seq, pivot);
            if (seq) {
                // a long search: drop its marks, the one-thread pass takes over
                DEV_OK(hipMemsetAsync(mark, 0, 4 * (size_t)n, s));
            } else {
                hipLaunchKernelGGL(k_scc_assign_fb, dim3(gb), dim3(SB), 0, s, n, scc, mark, pivot);
                hipLaunchKernelGGL(k_scc_recount, dim3(wblk(n)), dim3(SB), 0, s, n, g.rp, g.ci, g.rrp, g.rci, scc,
                                   in_rem, out_rem);
            }
        }
        if (!seq) {
            STEP_OK(trim(32));
            phase("trim2", 0, 0);
        }
        // ---- colouring until every vertex has a component
        for (int it = 0; !seq; it++) {
            DEV_OK(hipMemsetAsync(small + 1, 0, 4, s));
            hipLaunchKernelGGL(k_col_init, dim3(rblk(n)), dim3(SB), 0, s, n, scc, color, small + 1);
            const int32_t un = read_i32(small + 1, pin, s);
            if (un < 0) { fail(-1); goto done; }
            phase("col-init", it, un);
            if (un == 0) break;
            if (it >= COL_ITERS) {
                seq = true;
                break;
            }
            for (int r = 0;; r++) {
                if (r >= COL_ROUNDS) {
                    seq = true;
                    break;
                }
                DEV_OK(hipMemsetAsync(small + 2, 0, 4, s));
                hipLaunchKernelGGL(k_col_prop, dim3(gb), dim3(SB), 0, s, n, g.rrp, g.rci, scc, color, small + 2);
                const int32_t ch = read_i32(small + 2, pin, s);
                if (ch < 0) { fail(-1); goto done; }
                if (!ch) break;
            }
            if (seq) break;
            phase("col-prop", it, 0);
            hipLaunchKernelGGL(k_col_close_init, dim3(gb), dim3(SB), 0, s, n, scc, color, mark);
            for (int r = 0;; r++) {
                if (r >= COL_ROUNDS) {
                    seq = true;
                    break;
                }
                DEV_OK(hipMemsetAsync(small + 2, 0, 4, s));
                hipLaunchKernelGGL(k_col_close, dim3(gb), dim3(SB), 0, s, n, g.rp, g.ci, scc, color, mark, small + 2);
                const int32_t ch = read_i32(small + 2, pin, s);
                if (ch < 0) { fail(-1); goto done; }
                if (!ch) break;
            }
            if (seq) {
                DEV_OK(hipMemsetAsync(mark, 0, 4 * (size_t)n, s));
                break;
            }
            phase("col-close", it, 0);
            hipLaunchKernelGGL(k_col_assign, dim3(gb), dim3(SB), 0, s, n, scc, color, mark);
            hipLaunchKernelGGL(k_scc_recount, dim3(wblk(n)), dim3(SB), 0, s, n, g.rp, g.ci, g.rrp, g.rci, scc, in_rem,
                               out_rem);
            STEP_OK(trim(32));
        }
        if (seq) {
            // ---- the rest, one thread: Tarjan over the unassigned vertices
            hipLaunchKernelGGL(k_unassigned_flag, dim3(gb), dim3(SB), 0, s, n, scc, cid);
            STEP_OK(scan(cid, n, bsum, small + 1, s));
            hipLaunchKernelGGL(k_unassigned_scatter, dim3(gb), dim3(SB), 0, s, n, scc, cid, list);
            const int32_t un = read_i32(small + 1, pin, s);
            if (un < 0) { fail(-1); goto done; }
            if (un > 0) {
                // idx = color, low = next, search stack = cid, call stack = cnt, arc cursor = hgt
                DEV_OK(hipMemsetAsync(color, 0xff, 4 * (size_t)n, s));
                hipLaunchKernelGGL(k_seq_scc, dim3(1), dim3(64), 0, s, list, un, g.rp, g.ci, scc, color, next, cid,
                                   cnt, hgt);
                DEV_OK(hipGetLastError());
            }
            phase("seq-scc", un, 0);
        }
        // ---- dense component ids, sizes, the largest component
        hipLaunchKernelGGL(k_rep_flag, dim3(gb), dim3(SB), 0, s, n, scc, cid);
        STEP_OK(scan(cid, n, bsum, small + 3, s));
        const int32_t nc = read_i32(small + 3, pin, s);
        if (nc <= 0) { fail(-1); goto done; }
        hipLaunchKernelGGL(k_comp_of, dim3(gb), dim3(SB), 0, s, n, scc, cid, comp);
        DEV_OK(hipMemsetAsync(wt, 0, 4 * (size_t)nc, s));
        DEV_OK(hipMemsetAsync(minid, 0x7f, 4 * (size_t)nc, s));
        hipLaunchKernelGGL(k_comp_stats, dim3(rblk(n)), dim3(SB), 0, s, n, comp, pivot, wt, minid, g.oid);
        DEV_OK(hipMemsetAsync(big_key, 0, 8, s));
        hipLaunchKernelGGL(k_comp_big, dim3(rblk(nc)), dim3(SB), 0, s, nc, wt, minid, big_key);
        phase("ids", nc, 0);
        // ---- DAG arcs, sorted by (source, target) and deduplicated
        hipLaunchKernelGGL(k_dag_count, dim3(nblk(n)), dim3(SB), 0, s, n, g.rp, g.ci, comp, cnt);
        if (g.nheavy) {
            hipLaunchKernelGGL(k_dag_chunk_count, dim3(wblk(g.nchunks)), dim3(SB), 0, s, g.nchunks, g.ch_beg, g.ch_end,
                               g.ch_vtx, g.ci, comp, ccnt);
            hipLaunchKernelGGL(k_dag_heavy_sum, dim3(nblk(g.nheavy)), dim3(SB), 0, s, g.nheavy, g.heavy, g.hcb, ccnt,
                               cnt, cfirst);
            STEP_OK(scan(ccnt, g.nchunks, bsum, small + 10, s));
        }
        STEP_OK(scan(cnt, n, bsum, small + 4, s));
        const int32_t E = read_i32(small + 4, pin, s);
        if (E < 0) { fail(-1); goto done; }
        int32_t U = 0;
        if (E > 0) {
            hipLaunchKernelGGL(k_dag_pairs, dim3(nblk(n)), dim3(SB), 0, s, n, g.rp, g.ci, comp, cnt, key, val);
            if (g.nheavy)
                hipLaunchKernelGGL(k_dag_chunk_pairs, dim3(wblk(g.nchunks)), dim3(SB), 0, s, g.nchunks, g.ch_beg,
                                   g.ch_end, g.ch_vtx, g.ci, comp, cnt, ccnt, cfirst, key, val);
            // by target, then (stable) by source
            STEP_OK(tkc_sort_pairs(key, val, tkey, tval, E, hist, smask, pin_mask, s));
            DEV_OK(hipMemcpyAsync(tkey, val, 4 * (size_t)E, hipMemcpyDeviceToDevice, s));
            DEV_OK(hipMemcpyAsync(tval, key, 4 * (size_t)E, hipMemcpyDeviceToDevice, s));
            STEP_OK(tkc_sort_pairs(tkey, tval, key, val, E, hist, smask, pin_mask, s));
            hipLaunchKernelGGL(k_dag_uniq, dim3(nblk(E)), dim3(SB), 0, s, (int64_t)E, tkey, tval, flag);
            DEV_OK(hipMemcpyAsync(pos, flag, 4 * (size_t)E, hipMemcpyDeviceToDevice, s));
            STEP_OK(scan(pos, E, bsum, small + 5, s));
            U = read_i32(small + 5, pin, s);
            if (U < 0) { fail(-1); goto done; }
            hipLaunchKernelGGL(k_dag_compact, dim3(nblk(E)), dim3(SB), 0, s, (int64_t)E, tkey, tval, pos, flag, asrc,
                               adst);
        }
        phase("dag", E, U);
        // ---- heights, "reaches C~", "reached from C~"
        DEV_OK(hipMemcpyAsync(pin, big_key, 8, hipMemcpyDeviceToHost, s));
        DEV_OK(hipStreamSynchronize(s));
        const uint32_t bmin = 0xffffffffu - (uint32_t)(*(unsigned long long*)pin & 0xffffffffull);
        DEV_OK(hipMemsetAsync(hgt, 0, 4 * (size_t)nc, s));
        DEV_OK(hipMemsetAsync(tob, 0, 4 * (size_t)nc, s));
        DEV_OK(hipMemsetAsync(frb, 0, 4 * (size_t)nc, s));
        // the largest component is the one holding the caller's vertex bmin
        hipLaunchKernelGGL(k_set_big, dim3(1), dim3(64), 0, s, comp, (int32_t)bmin, g.nid, tob, frb, small + 9);
        const int32_t big = read_i32(small + 9, pin, s);
        if (big < 0) { fail(-1); goto done; }
        bool deep = false;
        for (int r = 0; U > 0; r++) {
            if (r >= DAG_ROUNDS) {
                deep = true;
                break;
            }
            DEV_OK(hipMemsetAsync(small + 2, 0, 4, s));
            hipLaunchKernelGGL(k_dag_relax, dim3(nblk(U)), dim3(SB), 0, s, U, asrc, adst, hgt, tob, frb, small + 2);
            const int32_t ch = read_i32(small + 2, pin, s);
            if (ch < 0) { fail(-1); goto done; }
            if (!ch) break;
        }
        if (deep) {
            // ---- a deep DAG: Alg. 6 in one thread, in peel order
            // soff = cstart, poff = astart, pred = pos, cnt = hgt, queue = cnt, cursor = minid
            DEV_OK(hipMemsetAsync(small + 8, 0, 4, s));
            hipLaunchKernelGGL(k_seq_dag, dim3(1), dim3(64), 0, s, nc, U, asrc, adst, wt, big, (int64_t)n, cstart,
                               astart, pos, hgt, cnt, minid, tob, frb, ca, co, topo, small + 8);
            const int32_t bad = read_i32(small + 8, pin, s);
            if (bad != 0) { fail(-1); goto done; }
            phase("seq-dag", nc, U);
        } else {
            DEV_OK(hipMemsetAsync(rb, 0, 8, s));
            DEV_OK(hipMemsetAsync(small + 7, 0, 4, s));
            hipLaunchKernelGGL(k_dag_reach_big, dim3(rblk(nc)), dim3(SB), 0, s, nc, wt, frb, hgt, rb, small + 7);
            const int32_t hmax = read_i32(small + 7, pin, s);
            if (hmax < 0 || hmax > DAG_ROUNDS) { fail(-1); goto done; }
            phase("heights", 0, hmax);
            // ---- components and arcs grouped by decreasing height (of the
            // source): a topological numbering, and the sweep order of Alg. 6
            uint32_t* ck = (uint32_t*)in_rem;   // vertex arrays free from here on
            int32_t* byh = out_rem;
            hipLaunchKernelGGL(k_comp_hkey, dim3(nblk(nc)), dim3(SB), 0, s, nc, hgt, hmax, ck, byh);
            STEP_OK(tkc_sort_pairs(ck, byh, (uint32_t*)list, next, nc, hist, smask, pin_mask, s));
            hipLaunchKernelGGL(k_topo_of, dim3(nblk(nc)), dim3(SB), 0, s, nc, byh, topo);
            DEV_OK(hipMemsetAsync(cstart, 0xff, 4 * ((size_t)hmax + 2), s));
            DEV_OK(hipMemsetAsync(astart, 0xff, 4 * ((size_t)hmax + 2), s));
            hipLaunchKernelGGL(k_bucket_starts, dim3(nblk(nc)), dim3(SB), 0, s, nc, ck, cstart);
            if (U > 0) {
                hipLaunchKernelGGL(k_arc_hkey, dim3(nblk(U)), dim3(SB), 0, s, U, asrc, hgt, hmax, tkey, tval);
                STEP_OK(tkc_sort_pairs(tkey, tval, key, val, U, hist, smask, pin_mask, s));
                hipLaunchKernelGGL(k_arc_gather, dim3(nblk(U)), dim3(SB), 0, s, U, tval, asrc, adst, hsrc, hdst);
                hipLaunchKernelGGL(k_bucket_starts, dim3(nblk(U)), dim3(SB), 0, s, U, tkey, astart);
            }
            int32_t cb[DAG_ROUNDS + 2], ab[DAG_ROUNDS + 2];   // hmax <= DAG_ROUNDS
            DEV_OK(hipMemcpyAsync(cb, cstart, 4 * ((size_t)hmax + 2), hipMemcpyDeviceToHost, s));
            DEV_OK(hipMemcpyAsync(ab, astart, 4 * ((size_t)hmax + 2), hipMemcpyDeviceToHost, s));
            DEV_OK(hipStreamSynchronize(s));
            cb[hmax + 1] = nc;
            ab[hmax + 1] = U;
            for (int32_t b = hmax; b >= 0; b--) {
                if (cb[b] < 0) cb[b] = cb[b + 1];
                if (ab[b] < 0) ab[b] = ab[b + 1];
            }
            DEV_OK(hipMemsetAsync(accA, 0, 8 * (size_t)nc, s));
            DEV_OK(hipMemsetAsync(accO, 0, 8 * (size_t)nc, s));
            DEV_OK(hipMemsetAsync(accO2, 0, 8 * (size_t)nc, s));
            // sinks first: height h is bucket hmax - h
            for (int32_t h = 0; h <= hmax; h++) {
                const int32_t bk = hmax - h;
                if (ab[bk + 1] > ab[bk])
                    hipLaunchKernelGGL(k_dp_arcs, dim3(nblk(ab[bk + 1] - ab[bk])), dim3(SB), 0, s, ab[bk], ab[bk + 1],
                                       hsrc, hdst, ca, co, frb, accA, accO, accO2);
                if (cb[bk + 1] > cb[bk])
                    hipLaunchKernelGGL(k_dp_fin, dim3(nblk(cb[bk + 1] - cb[bk])), dim3(SB), 0, s, cb[bk], cb[bk + 1],
                                       byh, big, (int64_t)n, wt, tob, rb, accA, accO, accO2, ca, co);
            }
        }
        *seq_used = (seq || deep) ? 1 : 0;
        hipLaunchKernelGGL(k_scc_out, dim3(gb), dim3(SB), 0, s, n, comp, ca, co, topo, alpha, omega, scc_topo);
        DEV_OK(hipStreamSynchronize(s));
        if (hipGetLastError() != hipSuccess) fail(-1);
        phase("dp+out", 0, 0);
    }
done:
#undef DEV_OK
#undef STEP_OK
    (void)hipStreamSynchronize(s);
    if (own) (void)hipFree(sc.base);
    return rc;
}
