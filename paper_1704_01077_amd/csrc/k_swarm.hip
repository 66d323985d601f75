// Per-workgroup engine: most BFSCut searches of Alg. 1 stop after two or
// three levels (Sect. 6), far too little work to fill the GPU one search at
// a time.  Here every workgroup pulls the next candidate from the order
// with an atomic cursor and runs that search alone: levels are separated by
// workgroup barriers only, the visited set is a private bitmap that stays
// in the XCD's L2, the queue is private, and the current k-th farness x is
// re-read from the shared top-k at every level boundary.  A search whose
// queue outgrows its capacity is handed back (deferred) to the batched
// engine, which is better at large searches.  The stop rule of Alg. 1 is
// applied when a candidate is taken: once one candidate's key proves that
// every later bound exceeds x, the cursor is closed for all workgroups.
//
// Deferred searches do not lower x, so on a graph where most candidates
// reach a large part of the graph quickly the workgroups would walk the
// whole order deferring everything.  After `defer_cap` deferrals the engine
// therefore closes itself: the cursor stops, searches in flight are
// deferred at their next level boundary, and the host hands the deferred
// list and the rest of the order to the batched engine.
//
// stop word bits: 1 = the stop rule fired, 2 = the engine closed itself.
#include "dev_common.hpp"
#include "engine.hpp"

#include <stdlib.h>

// workgroup size: big enough that one search keeps many arcs in flight
// (the searches left after the seed batch are few and large on complex
// networks); TKC_SWARM_SB=256 or 1024 picks one for experiments
#define SB_DEFAULT 1024
static int swarm_sb() {
    static const int v = [] {
        const char* e = getenv("TKC_SWARM_SB");
        const int x = e ? atoi(e) : SB_DEFAULT;
        return x == 256 ? 256 : (x == 1024 ? 1024 : SB_DEFAULT);
    }();
    return v;
}

struct SwarmArgs {
    DevGraph g;
    DevReach rc;
    OrderView ov;
    BoundsView bv;
    DevTopk tk;
    SwarmWork w;
    int64_t* stats;
    int32_t start_pos;
    int32_t words;
    int32_t defer_cap;
};

// exclusive scan of one int per thread over the workgroup; returns the total
template <int SB>
TKC_DEV int32_t block_excl_scan(int32_t v, int32_t* out, int32_t* wsum) {
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane_id() >= o) x += y;
    }
    int wv = threadIdx.x >> 6;
    if (lane_id() == 63) wsum[wv] = x;
    __syncthreads();
    int32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SB / 64; w++) {
        int32_t t = wsum[w];
        if (w < wv) base += t;
        tot += t;
    }
    *out = base + x - v;
    return tot;
}

template <int SB>
__global__ void __launch_bounds__(SB) k_swarm(SwarmArgs a) {
    __shared__ int32_t s_pos;
    __shared__ int32_t s_pre[SB + 1];
    __shared__ int32_t s_beg[SB];
    __shared__ int32_t s_wsum[SB / 64];
    __shared__ int32_t s_tail;
    __shared__ int32_t s_over;
    __shared__ int64_t s_cnt, s_deg;
    __shared__ int64_t s_x[3];
    __shared__ int32_t s_dec;
    __shared__ int32_t s_closed;

    const int tid = threadIdx.x;
    const int32_t* __restrict__ rp = a.g.rp;
    const int32_t* __restrict__ ci = a.g.ci;
    const int32_t* __restrict__ deg = a.g.deg;
    const bool dir = a.g.directed;
    uint32_t* vis = a.w.vis + (int64_t)blockIdx.x * a.words;
    int32_t* q = a.w.queue + (int64_t)blockIdx.x * a.w.qcap;
    const int32_t qcap = a.w.qcap;
    const int32_t count = a.ov.count;
    int64_t st_mvis = 0, st_started = 0, st_exact = 0, st_cut = 0, st_skip = 0, st_def = 0;
    int64_t st_maxl = 0, st_bytes = 0;
    // the preceding batch (same stream, finished) hands over where it stopped
    int32_t start_pos = a.start_pos;
    bool seed_stopped = false;
    if (a.w.seed) {
        start_pos = (int32_t)a.w.seed[ST_CURSOR];
        seed_stopped = a.w.seed[ST_STOP] != 0;
    }

    for (;;) {
        if (tid == 0) {
            int32_t p = -1;
            if (!seed_stopped && ld_rlx(a.w.stop) == 0) p = start_pos + fadd_rlx(a.w.cursor, 1);
            s_pos = p;
            XVal x = read_x(a.tk.st, a.tk.ring);
            s_x[0] = x.num; s_x[1] = x.den; s_x[2] = x.id;
            s_dec = 0;
            if (p >= 0 && p < count) {
                int32_t v = a.ov.ord[p];
                uint32_t key = a.ov.key[p];
                bool stop = a.bv.harm ? key_stops_h(key, x)
                                      : (a.ov.key_is_bound ? key_stops(key, x) : (key == 0xffffffffu && x.den != 0));
                if (stop) { for_rlx(a.w.stop, 1); s_dec = 1; }
                else if (lex_after(a.bv.num[v], a.bv.den[v], TKC_OID(a.g, v), x.num, x.den, x.id)) { s_dec = 2; st_skip++; }
                else if (a.rc.omega[v] <= 1) {
                    s_dec = 3;
                    st_started++; st_exact++;
                    if (a.bv.harm) topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, harm_enc(0.0), 2, TKC_OID(a.g, v));
                    else topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, 0, 1, TKC_OID(a.g, v));
                }
            } else {
                s_dec = 1;
            }
        }
        __syncthreads();
        const int32_t pos = s_pos;
        const int dec = s_dec;
        __syncthreads();
        if (dec == 1) break;
        if (dec != 0) continue;

        const int32_t v = a.ov.ord[pos];
        const int64_t av = a.rc.alpha[v], ov = a.rc.omega[v];
        const int64_t dv = deg[v];
        if (tid == 0) {
            vis[v >> 5] |= 1u << (v & 31);
            q[0] = v;
            s_tail = 1;
            s_over = 0;
        }
        __syncthreads();
        int64_t D = 0, nD = 1, SD = 0, U = dv, nf = 1;
        double H = 0.0;   // harmonic centrality so far (levels 1..D)
        int32_t ls = 0, le = 1;
        int status = 0;   // 1 exact, 2 cut, 3 deferred
        int64_t mvis = 0;
        for (;;) {
            if (nf == 0) { status = 1; break; }
            if (tid == 0) {
                XVal x = read_x(a.tk.st, a.tk.ring);
                s_x[0] = x.num; s_x[1] = x.den; s_x[2] = x.id;
                s_cnt = 0; s_deg = 0;
                s_closed = (ld_rlx(a.w.stop) & 2) != 0;
            }
            __syncthreads();
            {
                int64_t bn, bd;
                if (a.bv.harm) harm_cut_bound(H, nD, U, D, ov, &bn, &bd);
                else cut_bound(SD, nD, U, D, av, ov, &bn, &bd);
                if (lex_after(bn, bd, TKC_OID(a.g, v), s_x[0], s_x[1], (int32_t)s_x[2])) { status = 2; break; }
            }
            if (s_closed) { status = 3; break; }
            // expand level D: frontier q[ls, le), edge-balanced in chunks of SB vertices
            int64_t my_cnt = 0, my_deg = 0;
            for (int32_t c = ls; c < le; c += SB) {
                int32_t i = c + tid;
                int32_t d = 0, b = 0;
                if (i < le) {
                    int32_t u = q[i];
                    b = rp[u];
                    d = rp[u + 1] - b;
                }
                int32_t pre;
                int32_t tot = block_excl_scan<SB>(d, &pre, s_wsum);
                s_pre[tid] = pre;
                s_beg[tid] = b;
                if (tid == 0) s_pre[SB] = tot;
                __syncthreads();
                mvis += tot;
                for (int32_t e = tid; e < tot; e += SB) {
                    // owner: last j with s_pre[j] <= e
                    int32_t lo = 0, hi = SB;
                    while (hi - lo > 1) {
                        int32_t mid = (lo + hi) >> 1;
                        if (s_pre[mid] <= e) lo = mid; else hi = mid;
                    }
                    int32_t w = ci[s_beg[lo] + (e - s_pre[lo])];
                    uint32_t bit = 1u << (w & 31);
                    if (!(vis[w >> 5] & bit)) {
                        uint32_t old = for_wg(&vis[w >> 5], bit);
                        if (!(old & bit)) {
                            int32_t slot = atomicAdd(&s_tail, 1);
                            if (slot < qcap) q[slot] = w;
                            else s_over = 1;
                            my_cnt++;
                            my_deg += deg[w];
                        }
                    }
                }
                __syncthreads();
            }
            my_cnt = wave_sum_i64(my_cnt);
            my_deg = wave_sum_i64(my_deg);
            if (lane_id() == 0 && my_cnt) {
                atomicAdd((unsigned long long*)&s_cnt, (unsigned long long)my_cnt);
                atomicAdd((unsigned long long*)&s_deg, (unsigned long long)my_deg);
            }
            __syncthreads();
            if (s_over) { status = 3; break; }
            int64_t cnt = s_cnt, dsum = s_deg;
            D++;
            nD += cnt;
            SD += D * cnt;
            if (a.bv.harm) H += (double)cnt / (double)D;
            U = dir ? dsum : dsum - cnt;
            nf = cnt;
            ls = le;
            le = s_tail;
            __syncthreads();
        }
        // clear the private bitmap: by the queue, unless it overflowed (then
        // some marked vertices are not in it)
        if (status == 3 && s_over) {
            for (int32_t qw = tid; qw < a.words; qw += SB) vis[qw] = 0;
        } else {
            int32_t tail = s_tail;
            for (int32_t i = tid; i < tail; i += SB) { int32_t w = q[i]; vis[w >> 5] = 0; }
        }
        if (tid == 0) {
            st_started++;
            st_mvis += mvis;
            st_bytes += 8 * mvis + 12 * (int64_t)le + 16 * (nD - 1);
            int64_t md = status == 1 ? D - 1 : D;
            if (md > st_maxl) st_maxl = md;
            if (status == 1) {
                st_exact++;
                if (a.bv.harm) topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, harm_enc(H), 2, TKC_OID(a.g, v));
                else topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, SD, nD, TKC_OID(a.g, v));
            } else if (status == 2) {
                st_cut++;
            } else {
                st_def++;
                st_started--;
                // every candidate is taken once, so slot < n
                int32_t slot = fadd_rlx(a.w.ndeferred, 1);
                a.w.deferred[slot] = v;
                if (slot + 1 >= a.defer_cap) for_rlx(a.w.stop, 2);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        int64_t* s = a.stats;
        if (st_mvis) fadd_rlx(&s[ST_MVIS], st_mvis);
        if (st_started) fadd_rlx(&s[ST_STARTED], st_started);
        if (st_exact) fadd_rlx(&s[ST_EXACT], st_exact);
        if (st_cut) fadd_rlx(&s[ST_CUT], st_cut);
        if (st_skip) fadd_rlx(&s[ST_SKIPPED], st_skip);
        if (st_def) fadd_rlx(&s[ST_DEFERRED], st_def);
        if (st_bytes) fadd_rlx(&s[ST_BYTES], st_bytes);
        __hip_atomic_fetch_max(&s[ST_MAXLEVEL], st_maxl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

int tkc_swarm_max_blocks(int block) {
    (void)block;
    const int cus = tkc_cu_count();
    if (cus < 1) return -1;
    int occ = 0;
    const int sb = swarm_sb();
    if (sb == 1024) {
        occ = tkc_occupancy((const void*)k_swarm<1024>, 1024);
        if (occ < 0) return -1;
        if (occ > 2) occ = 2;
    } else {
        occ = tkc_occupancy((const void*)k_swarm<256>, 256);
        if (occ < 0) return -1;
        if (occ > 8) occ = 8;
    }
    return cus * (occ > 0 ? occ : 1);
}

int tkc_launch_swarm(const DevGraph& g, DevReach rc, OrderView ov, BoundsView bv, DevTopk tk,
                     SwarmWork w, int64_t* stats, int32_t start_pos, const EngineTuning& tune,
                     hipStream_t s) {
    (void)tune;
    SwarmArgs a{};
    a.g = g; a.rc = rc; a.ov = ov; a.bv = bv; a.tk = tk; a.w = w;
    a.stats = stats;
    a.start_pos = start_pos;
    a.words = (int32_t)(((int64_t)g.n + 31) / 32);
    a.defer_cap = w.defer_cap > 0 ? w.defer_cap : 0x7fffffff;
    if (swarm_sb() == 1024)
        hipLaunchKernelGGL(k_swarm<1024>, dim3(w.nblocks), dim3(1024), 0, s, a);
    else
        hipLaunchKernelGGL(k_swarm<256>, dim3(w.nblocks), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
