// Batched engine: W candidates of Alg. 1 searched together, one bit lane
// per source in W-bit words per vertex.  A push step reads each frontier
// vertex's adjacency once for all its lanes and ORs the lanes into its
// neighbours' next-frontier words; a pull step lets every vertex with
// unreached lanes scan its in-arcs for frontier lanes.  Each lane keeps its
// own BFSCut state (Sect. 6): after every level the exact per-lane counts
// give the bound, and a lane whose bound passes the k-th farness x retires
// (its bits are masked out of later steps).  Bound variants run every lane
// to the end and then apply the level-based update (Sect. 7) of all lanes
// at once.
//
// One grid barrier per level.  F_D, the lanes that first reached each
// vertex at level D, lives in one of three rotating word arrays; the
// visited words `vis` hold the levels before D, so "seen" means vis | F_D.
// During level D every frontier vertex's owner folds F_D into vis, the
// expansion writes F_{D+1} and counts each newly reached (vertex, lane) at
// the moment it is set (the atomic OR that sets a bit returns the bits set
// before, so exactly one caller sees each bit as new), and the words of
// F_{D-1} are cleared through the level list L_{D-1}.  Lists rotate over
// four slots and counters over three parities so that no slot is reset or
// rewritten before every workgroup has passed the barrier after its last
// reader.
//
// One cooperative launch processes batch after batch; block 0's first wave
// selects the next candidates from the order (stop and skip rules of
// Alg. 1) and every workgroup replicates the per-lane control so all take
// the same path through the grid barriers.
#include "dev_common.hpp"
#include "engine.hpp"

#define BB 256
#define MAXW 256
#define PUSH_SUB 4   // work items per heavy-vertex chunk in a push

// ctr layout (int64)
#define C_CNT(p, l) ((p) * 2 * MAXW + (l))
#define C_DEG(p, l) ((p) * 2 * MAXW + MAXW + (l))
#define C_BASE (3 * 2 * MAXW)
// per parity p = level % 3, for the vertices first reached in that level's
// expansion: their out-degree sum, and the out-degrees of vertices that
// became seen by every active lane when folded
#define C_UDEG(p) (C_BASE + (p) * 4 + 0)
#define C_DDONE(p) (C_BASE + (p) * 4 + 1)
// vertex list tails per slot s = level % 4: [0] light, [1] heavy
#define C_LT(s, c) (C_BASE + 12 + 2 * (s) + (c))
// heavy-vertex chunk list tail per level % 3
#define C_CT(q) (C_BASE + 20 + (q))
#define C_NSEL (C_BASE + 24)
#define C_POS (C_BASE + 25)
#define C_STOP (C_BASE + 26)
#define C_XDONE (C_BASE + 27)   // until_x: x became finite in this batch
#define C_TOTAL (C_BASE + 32)

struct BatchArgs {
    DevGraph g;
    DevReach rc;
    OrderView ov;
    BoundsView bv;
    DevTopk tk;
    BatchWork w;
    int64_t* stats;
    const int32_t* list;
    int32_t list_count;
    int32_t start_pos;
    int32_t max_batches;
    int32_t lb_mode;
    int32_t no_cut;        // full searches, results to out_S / out_r only
    int32_t until_x;       // stop after the batch in which x becomes finite
    int32_t W;
    int32_t Wsel;          // lanes filled per batch (<= W)
    int32_t alpha_td;
    int32_t beta_bu;
    int64_t* out_S;
    int64_t* out_r;
    int32_t* mark;         // per-vertex level stamp (NW > 1)
    uint32_t* bar;         // grid barrier state
    // packed launch (npreq > 0): the batches' lanes are shared by npreq
    // requests on the members of a union graph; a.ov, a.bv, a.rc and a.tk
    // are then unused, every request brings its own
    const PackReq* preq;
    int32_t npreq;
};

TKC_DEV int64_t shfl64b(int64_t v, int src) {
    int32_t lo = __shfl((int32_t)(v & 0xffffffff), src, 64);
    int32_t hi = __shfl((int32_t)(v >> 32), src, 64);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}
TKC_DEV uint64_t below_mask() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <int NW>
struct Mask {
    uint64_t w[NW];
    TKC_DEV bool any() const {
        uint64_t o = 0;
#pragma unroll
        for (int j = 0; j < NW; j++) o |= w[j];
        return o != 0;
    }
};

// Appends to the next level's vertex lists.  One tail counter per list
// takes every append, and a large level makes tens of thousands of them, so
// light vertices (the vast majority) are first staged in a per-wave LDS
// buffer and reserved in the list once per STAGE entries; heavy vertices
// (rare) are appended directly, together with their arc chunks.
#define STAGE 1024
struct Stage {
    int32_t* buf;   // this wave's LDS slots
    int32_t n;      // filled slots (wave-uniform)
};
struct NextLists {
    int32_t* light;
    int32_t* heavy;
    int64_t* tails;     // [0] light, [1] heavy
    int32_t* cu;        // chunk owners
    int32_t* cb;        // chunk first arcs
    int64_t* ctail;
    const int32_t* rp;
};
TKC_DEV void stage_flush(Stage& st, int32_t* list, int64_t* tail) {
    if (st.n == 0) return;
    int64_t b = 0;
    if (lane_id() == 0) b = fadd_rlx(tail, (int64_t)st.n);
    b = shfl64b(b, 0);
    __builtin_amdgcn_wave_barrier();
    for (int32_t i = lane_id(); i < st.n; i += 64) list[b + i] = st.buf[i];
    __builtin_amdgcn_wave_barrier();
    st.n = 0;
}
// called by all 64 lanes of a wave
TKC_DEV void list_append(bool isnew, int32_t w, int32_t dw, const NextLists& L, Stage& st) {
    const bool heavy = dw > HEAVY_DEG;
    const uint64_t ml = __ballot(isnew && !heavy);
    const uint64_t mh = __ballot(isnew && heavy);
    const uint64_t bm = below_mask();
    if (mh) {
        int64_t b = 0;
        if (lane_id() == 0) b = fadd_rlx(&L.tails[1], (int64_t)__popcll(mh));
        b = shfl64b(b, 0);
        const int32_t nck = (isnew && heavy) ? (dw + CHUNK_ARCS - 1) / CHUNK_ARCS : 0;
        int32_t pre = nck;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int32_t y = __shfl_up(pre, o, 64);
            if (lane_id() >= o) pre += y;
        }
        const int32_t tot = __shfl(pre, 63, 64);
        pre -= nck;
        int64_t c0 = 0;
        if (lane_id() == 0) c0 = fadd_rlx(L.ctail, (int64_t)tot);
        c0 = shfl64b(c0, 0);
        if (isnew && heavy) {
            L.heavy[b + __popcll(mh & bm)] = w;
            const int32_t r0 = L.rp[w];
            for (int32_t j = 0; j < nck; j++) {
                L.cu[c0 + pre + j] = w;
                L.cb[c0 + pre + j] = r0 + j * CHUNK_ARCS;
            }
        }
    }
    if (ml) {
        const int32_t c = __popcll(ml);
        if (st.n + c > STAGE) stage_flush(st, L.light, &L.tails[0]);
        if (isnew && !heavy) st.buf[st.n + __popcll(ml & bm)] = w;
        st.n += c;
    }
}

// Per-lane tallies of newly reached vertices: count and out-degree sum per
// lane, in the workgroup's LDS.
// Sparse masks (push): each thread adds its own bits.
template <int NW>
TKC_DEV void tally_bits(const Mask<NW>& nb, int32_t dw, int32_t* cnt, int64_t* dsum) {
#pragma unroll
    for (int j = 0; j < NW; j++) {
        uint64_t m = nb.w[j];
        while (m) {
            int l = j * 64 + __ffsll((long long)m) - 1;
            m &= m - 1;
            atomicAdd(&cnt[l], 1);
            atomicAdd((unsigned long long*)&dsum[l], (unsigned long long)dw);
        }
    }
}
// Dense masks (pull, one vertex per lane), called by all 64 lanes: the
// wave transposes each word's 64 x 64 bit matrix, so lane l holds the
// vertices that search lane j * 64 + l reached; their count is a popcount
// and their out-degree sum is taken bit slice by bit slice of the degrees
// (one ballot per slice).  One LDS add per lane and word.
template <int NW>
TKC_DEV void tally_dense(const Mask<NW>& nb, int32_t dw, int32_t* cnt, int64_t* dsum) {
    const int lane = lane_id();
    uint64_t col[NW];
    int64_t ds[NW];
#pragma unroll
    for (int j = 0; j < NW; j++) {
        col[j] = __ballot(nb.w[j] != 0) ? wave_transpose64(nb.w[j]) : 0;
        ds[j] = 0;
    }
    const uint32_t d = (uint32_t)dw;
    for (int b = 0; b < 32; b++) {
        const uint64_t slice = __ballot((d >> b) & 1u);
        if (!__ballot((d >> b) != 0u)) break;   // wave-uniform
#pragma unroll
        for (int j = 0; j < NW; j++) ds[j] += (int64_t)__popcll(col[j] & slice) << b;
    }
#pragma unroll
    for (int j = 0; j < NW; j++) {
        const int c = __popcll(col[j]);
        if (c) {
            atomicAdd(&cnt[j * 64 + lane], c);
            atomicAdd((unsigned long long*)&dsum[j * 64 + lane], (unsigned long long)ds[j]);
        }
    }
}
// Called by all 64 lanes: the wave picks the cheaper way from two ballots.
// No new bits -> nothing; a lane with more than four new bits -> the
// transposition (fixed cost); otherwise each thread adds its own bits (at
// most four LDS adds per thread and counter kind).
template <int NW>
TKC_DEV void tally(const Mask<NW>& nb, int32_t dw, int32_t* cnt, int64_t* dsum) {
    int32_t bits = 0;
#pragma unroll
    for (int j = 0; j < NW; j++) bits += __popcll(nb.w[j]);
    if (!__ballot(bits != 0)) return;   // wave-uniform
    if (__ballot(bits > 4)) tally_dense<NW>(nb, dw, cnt, dsum);
    else tally_bits<NW>(nb, dw, cnt, dsum);
}

// level of every newly reached lane (level-based bound of Sect. 7)
template <int NW>
TKC_DEV void record_levels(const Mask<NW>& nb, int32_t w, uint16_t* lvl, int W, int64_t level) {
#pragma unroll
    for (int j = 0; j < NW; j++) {
        uint64_t m = nb.w[j];
        while (m) {
            int l = __ffsll((long long)m) - 1;
            m &= m - 1;
            lvl[(int64_t)w * W + j * 64 + l] = (uint16_t)level;
        }
    }
}

// Edge-balanced pull over up to 64 vertices, one per lane: the lane's
// vertex has in-arcs [eb, eb + len) and misses the lanes in `miss`; *acc
// receives the frontier lanes among its in-neighbours, restricted to miss.
// The wave's lanes share all the arcs: each arc finds its vertex by binary
// search over the prefix sums and ORs into the vertex's LDS accumulator.
// Called by all 64 lanes; the LDS slots belong to the calling wave.
template <int NW>
TKC_DEV void pull_shared(int32_t eb, int32_t len, const Mask<NW>& miss, const uint64_t* Fc,
                         const int32_t* __restrict__ rci, int32_t* c_pre, int32_t* c_beg, uint64_t* c_miss,
                         uint64_t* c_acc, Mask<NW>* acc, int64_t* scanned) {
    const int lane = lane_id();
    int32_t pre = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(pre, o, 64);
        if (lane >= o) pre += y;
    }
    const int32_t tot = __shfl(pre, 63, 64);
    pre -= len;
    c_pre[lane] = pre;
    c_beg[lane] = eb;
#pragma unroll
    for (int j = 0; j < NW; j++) {
        c_miss[lane * NW + j] = miss.w[j];
        c_acc[lane * NW + j] = 0;
    }
    __builtin_amdgcn_wave_barrier();
    // each lane takes four consecutive arcs per pass: one owner search, then
    // four index loads and four frontier loads in flight together
    for (int32_t t0 = lane * 4; t0 < tot; t0 += 256) {
        int32_t lo = 0, hi = 64;   // owner: last vertex whose range starts at or before t0
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (c_pre[mid] <= t0) lo = mid; else hi = mid;
        }
        int32_t own[4], u[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int32_t t = t0 + q;
            own[q] = -1;
            u[q] = 0;
            if (t < tot) {
                while (lo < 63 && c_pre[lo + 1] <= t) lo++;
                own[q] = lo;
                u[q] = rci[c_beg[lo] + (t - c_pre[lo])];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (own[q] < 0) continue;
            (*scanned)++;
#pragma unroll
            for (int j = 0; j < NW; j++) {
                const uint64_t f = Fc[(int64_t)u[q] * NW + j] & c_miss[own[q] * NW + j];
                if (f) atomicOr((unsigned long long*)&c_acc[own[q] * NW + j], (unsigned long long)f);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < NW; j++) acc->w[j] = c_acc[lane * NW + j];
    __builtin_amdgcn_wave_barrier();
}

// OR the lanes nb into w's next-frontier word(s).  *fresh receives the
// lanes this call set first (each (vertex, lane) is fresh for exactly one
// caller); the result is true for exactly one caller per vertex and level,
// the one that appends it to the next list.  A plain read of the word that
// already holds every lane in nb proves other callers set them first: the
// word only gains bits during the expansion.
template <int NW>
TKC_DEV bool discover(uint64_t* Fn, int32_t* mark, int32_t w, const Mask<NW>& nb, int32_t stamp,
                      Mask<NW>* fresh) {
    if (NW == 1) {
        fresh->w[0] = 0;
        const uint64_t seen = Fn[w];
        if ((seen & nb.w[0]) == nb.w[0]) return false;
        const uint64_t old = for_rlx(&Fn[w], nb.w[0]);
        fresh->w[0] = nb.w[0] & ~old;
        return old == 0;
    } else {
#pragma unroll
        for (int j = 0; j < NW; j++) {
            fresh->w[j] = 0;
            if (nb.w[j]) fresh->w[j] = nb.w[j] & ~for_rlx(&Fn[(int64_t)w * NW + j], nb.w[j]);
        }
        const int32_t old = __hip_atomic_fetch_max(&mark[w], stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return old < stamp;
    }
}

// Candidate selection of Alg. 1 from one processing order, by the 64 lanes
// of one wave: positions pos, pos + 1, ... are taken, skipped (the bound
// already passes x) or finished at once (nothing reachable: S = 0, r = 1)
// until cap candidates are selected, the order ends, or the stop rule fires
// (sets *stop).  Selected vertices, plus `off`, go to cand[nsel ...].
struct SelIn {
    const int32_t* ord;      // the order (order mode) or the source list (list mode)
    const uint32_t* key;     // the order's keys; null in list mode
    int32_t count;
    bool key_is_bound;
    const int64_t* num;
    const int64_t* den;
    const int64_t* omega;
    DevTopk tk;
    int32_t harm;
    int32_t no_cut;
    int32_t off;
    const int32_t* oid;      // relabelled graph: the caller's ids (ties), else null
};
TKC_DEV void select_cands(const SelIn& in, int32_t& pos, int32_t cap, int32_t* cand, int32_t& nsel, int32_t& stop,
                          int64_t& skipped, int64_t& r1) {
    const int lane = lane_id();
    const bool order_mode = in.key != nullptr;
    const int32_t count = in.count;
    XVal x = read_x(in.tk.st, in.tk.ring);
    int64_t r1_here = 0;
    while (nsel < cap && pos < count && !stop) {
        int32_t i = pos + lane;
        bool valid = i < count;
        int32_t v = valid ? in.ord[i] : -1;
        bool st = false, sk = false, one = false;
        if (valid && !in.no_cut) {
            if (order_mode) {
                uint32_t key = in.key[i];
                st = in.harm ? key_stops_h(key, x)
                             : (in.key_is_bound ? key_stops(key, x) : (key == 0xffffffffu && x.den != 0));
            }
            if (!st) sk = lex_after(in.num[v], in.den[v], in.oid ? in.oid[v] : v, x.num, x.den, x.id);
        }
        // in list mode without cuts every position gets a lane, sinks included
        if (valid && !st && !sk && !in.no_cut) one = in.omega[v] <= 1;
        uint64_t mst = __ballot(valid && st);
        int lim = mst ? (__ffsll((long long)mst) - 1) : 64;
        bool inwin = valid && lane < lim;
        bool elig = inwin && !st && !sk && !one;
        uint64_t me = __ballot(elig);
        int room = cap - nsel;
        // lanes beyond the room-th eligible one are left for the next batch
        int cut_lane = 64;
        if (__popcll(me) > room) {
            uint64_t m = me;
            for (int q = 0; q < room; q++) m &= m - 1;
            cut_lane = __ffsll((long long)m) - 1;
        }
        bool take = inwin && lane < cut_lane;
        int rank = __popcll(me & below_mask());
        if (take && elig) cand[nsel + rank] = v + in.off;
        uint64_t mone = __ballot(take && one);
        uint64_t msk = __ballot(take && sk);
        // vertices that reach nothing are exact at once: (S, r) = (0, 1)
        if (lane == 0) {
            uint64_t m = mone;
            while (m) {
                int l = __ffsll((long long)m) - 1;
                m &= m - 1;
                int32_t vv = in.ord[pos + l];
                if (in.oid) vv = in.oid[vv];
                if (in.harm) topk_insert(in.tk.st, in.tk.ring, in.tk.S, in.tk.R, in.tk.I, harm_enc(0.0), 2, vv);
                else topk_insert(in.tk.st, in.tk.ring, in.tk.S, in.tk.R, in.tk.I, 0, 1, vv);
            }
        }
        r1_here += __popcll(mone);
        skipped += __popcll(msk);
        int took = __popcll(me & ((cut_lane >= 64) ? ~0ull : ((1ull << cut_lane) - 1)));
        int consumed = lim < cut_lane ? lim : cut_lane;
        if (consumed > count - pos) consumed = count - pos;
        nsel += took;
        pos += consumed;
        if (mst && lim < cut_lane) stop = 1;
        if (r1_here) x = read_x(in.tk.st, in.tk.ring);
    }
    r1 += r1_here;
}

TKC_DEV uint64_t* fsel(const BatchWork& w, int64_t level) {
    const int i = (int)(level % 3);
    return i == 0 ? w.frt0 : (i == 1 ? w.frt1 : w.nxt);
}

// vertex list of class c (0 light, 1 heavy) in slot s (level % 4), and the
// heavy-vertex chunk lists (owner, first arc) in slot q (level % 2)
#define VL(c, s) (a.w.list + (int64_t)(2 * (s) + (c)) * n)
#define CU(q) (a.w.list + 8 * (int64_t)n + (int64_t)(2 * (q)) * a.w.ccap)
#define CB(q) (a.w.list + 8 * (int64_t)n + (int64_t)(2 * (q) + 1) * a.w.ccap)

// TR: per-level phase timing of workgroup 0's waves into the trace (the
// diagnostic TKC_TRACE mode); the untraced kernel carries none of it.
template <int NW, bool TR>
__global__ void __launch_bounds__(BB) k_batch(BatchArgs a) {
    const int32_t n = a.g.n;
    const bool dir = a.g.directed;
    const int W = a.W;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nwaves = nthreads / 64;
    const int64_t gwave = gtid / 64;
    const int lane = lane_id();
    const int tid = threadIdx.x;
    const bool boss = (blockIdx.x == 0 && tid == 0);
    const int32_t* __restrict__ rp = a.g.rp;
    const int32_t* __restrict__ ci = a.g.ci;
    const int32_t* __restrict__ deg = a.g.deg;
    int64_t* ctr = a.w.ctr;
    uint64_t* vis = a.w.vis;
    int64_t* stats = a.stats;
    const bool order_mode = (a.list == nullptr);
    const int32_t count = order_mode ? a.ov.count : a.list_count;

    // replicated per-lane control state
    __shared__ int32_t s_v[MAXW];
    // per lane: the x its cuts compare with (its request's, read at the
    // start of the batch), the union offset of its graph, its request
    __shared__ int64_t s_xn[MAXW], s_xd[MAXW];
    __shared__ int32_t s_xi[MAXW], s_off[MAXW], s_req[MAXW];
    // cursors and stop flags of a pack's requests (block 0's first wave)
    __shared__ int32_t s_pk_pos[TKC_PACK_MAXREQ], s_pk_stop[TKC_PACK_MAXREQ];
    __shared__ int64_t s_a[MAXW], s_o[MAXW], s_nD[MAXW], s_SD[MAXW], s_U[MAXW], s_nf[MAXW], s_mf[MAXW];
    __shared__ double s_H[MAXW];   // harmonic centrality so far (levels 1..D)
    __shared__ int32_t s_st[MAXW];      // 0 unused, 1 active, 2 exact, 3 cut
    __shared__ int32_t s_maxD[MAXW];
    __shared__ uint64_t s_act[NW];
    __shared__ int32_t s_red_cnt[MAXW];
    __shared__ int64_t s_red_deg[MAXW];
    __shared__ int64_t s_scal[8];
    __shared__ int32_t s_stage[BB / 64][STAGE];
    __shared__ int64_t s_blk[4];
    __shared__ int64_t s_ph[BB / 64][6];
    int64_t ph[6] = {0, 0, 0, 0, 0, 0};
    uint64_t tp = 0;
    const bool trb = TR && blockIdx.x == 0;
#define PHASE(i)                                   \
    if (trb) {                                     \
        const uint64_t t_ = wall_clock64();        \
        ph[i] += (int64_t)(t_ - tp);               \
        tp = t_;                                   \
    }
    // edge-balanced pull: per-wave vertex ranges, missing lanes, accumulators
    __shared__ int32_t s_cpre[BB / 64][64];
    __shared__ int32_t s_cbeg[BB / 64][64];
    __shared__ uint64_t s_cmiss[BB / 64][64 * NW];
    __shared__ uint64_t s_cacc[BB / 64][64 * NW];

    int32_t pos = a.start_pos;
    int32_t batches = 0;
    if (tid < TKC_PACK_MAXREQ) {
        s_pk_pos[tid] = 0;
        s_pk_stop[tid] = 0;
    }
    __syncthreads();
    while (batches < a.max_batches) {
        // ---------------------------------------------- candidate selection
        if (blockIdx.x == 0 && tid < 64) {
            int32_t nsel = 0;
            int32_t stop = 0;
            int64_t skipped = 0, r1 = 0;
            if (a.npreq == 0) {
                const SelIn in{order_mode ? a.ov.ord : a.list, order_mode ? a.ov.key : nullptr, count,
                               a.ov.key_is_bound, a.bv.num, a.bv.den, a.rc.omega, a.tk, a.bv.harm, a.no_cut, 0,
                               a.g.oid};
                select_cands(in, pos, a.Wsel, a.w.cand, nsel, stop, skipped, r1);
            } else {
                // the requests of a pack take turns: first up to an even
                // share of the lanes each, then whatever is left over
                const int32_t share = a.Wsel / a.npreq > 0 ? a.Wsel / a.npreq : 1;
                for (int pass = 0; pass < 2 && nsel < a.Wsel; pass++) {
                    for (int32_t r = 0; r < a.npreq && nsel < a.Wsel; r++) {
                        if (s_pk_stop[r] || s_pk_pos[r] >= a.preq[r].n) continue;
                        const PackReq& q = a.preq[r];
                        const SelIn in{q.ov.ord, q.ov.key, q.n, q.ov.key_is_bound, q.bv.num, q.bv.den, q.rc.omega,
                                       q.tk, 0, 0, q.off, nullptr};
                        const int32_t before = nsel;
                        const int32_t cap = pass == 0 ? (nsel + share < a.Wsel ? nsel + share : a.Wsel) : a.Wsel;
                        int32_t rpos = s_pk_pos[r], rstop = s_pk_stop[r];
                        select_cands(in, rpos, cap, a.w.cand, nsel, rstop, skipped, r1);
                        for (int32_t c = before + lane; c < nsel; c += 64) a.w.cand_req[c] = r;
                        __builtin_amdgcn_wave_barrier();
                        if (lane == 0) {
                            s_pk_pos[r] = rpos;
                            s_pk_stop[r] = rstop;
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
            if (lane == 0) {
                ctr[C_NSEL] = nsel;
                ctr[C_POS] = pos;
                ctr[C_STOP] = stop;
                stats[ST_SKIPPED] += skipped;
                stats[ST_STARTED] += r1;
                stats[ST_EXACT] += r1;
                if (stop) stats[ST_STOP] = 1;
            }
        }
        grid_barrier(a.bar, gridDim.x);
        const int32_t nsel = (int32_t)ld_rlx(&ctr[C_NSEL]);
        pos = (int32_t)ld_rlx(&ctr[C_POS]);
        const bool stop_now = ld_rlx(&ctr[C_STOP]) != 0;
        if (nsel == 0) break;

        // ------------------------------------------------------ lane init
        XVal xb{0, 0, 0};
        if (a.npreq == 0) xb = read_x(a.tk.st, a.tk.ring);
        if (tid < MAXW) {
            int l = tid;
            if (l < nsel) {
                int32_t v = a.w.cand[l];
                int32_t off = 0, r = 0;
                const int64_t* al = a.rc.alpha;
                const int64_t* om = a.rc.omega;
                XVal xl = xb;
                if (a.npreq) {
                    r = a.w.cand_req[l];
                    off = a.preq[r].off;
                    al = a.preq[r].rc.alpha;
                    om = a.preq[r].rc.omega;
                    xl = read_x(a.preq[r].tk.st, a.preq[r].tk.ring);
                }
                s_v[l] = v;
                // s_v[l] - s_off[l] is the source's id as the caller numbers
                // it: the member's own id in a pack, the caller's id in a
                // relabelled graph (ties of the exact order break on it)
                s_off[l] = a.g.oid ? v - a.g.oid[v] : off;
                s_req[l] = r;
                s_xn[l] = xl.num;
                s_xd[l] = xl.den;
                s_xi[l] = xl.id;
                s_a[l] = al[v - off];
                s_o[l] = om[v - off];
                s_nD[l] = 1; s_SD[l] = 0; s_H[l] = 0.0;
                s_U[l] = deg[v]; s_nf[l] = 1; s_mf[l] = deg[v];
                s_st[l] = 1;
                s_maxD[l] = 0;
            } else {
                s_st[l] = 0;
            }
        }
        __syncthreads();   // every lane's source is in s_v
        if (blockIdx.x == 0) {
            // level-0 frontier (list slot 0): light sources, heavy sources
            // and the heavy sources' arc chunks.  A source list may name one
            // vertex twice: F_0 takes atomic ORs, the lists take it once.
            if (tid < 3) s_blk[tid] = 0;
            __syncthreads();
            if (tid < nsel) {
                const int l = tid;
                const int32_t v = s_v[l];
                for_rlx(&fsel(a.w, 0)[(int64_t)v * NW + (l >> 6)], (uint64_t)1 << (l & 63));
                if (a.lb_mode) { a.w.lvl[(int64_t)v * W + l] = 0; a.w.hist[l] = 1; }
                bool dup = false;
                for (int q = 0; q < l; q++) dup |= s_v[q] == v;
                if (!dup) {
                    const int32_t dv = deg[v];
                    if (dv > HEAVY_DEG) {
                        const int32_t nck = (dv + CHUNK_ARCS - 1) / CHUNK_ARCS;
                        const int64_t h = (int64_t)atomicAdd((unsigned long long*)&s_blk[1], 1ull);
                        const int64_t c0 = (int64_t)atomicAdd((unsigned long long*)&s_blk[2], (unsigned long long)nck);
                        VL(1, 0)[h] = v;
                        const int32_t r0 = rp[v];
                        for (int32_t j = 0; j < nck; j++) {
                            CU(0)[c0 + j] = v;
                            CB(0)[c0 + j] = r0 + j * CHUNK_ARCS;
                        }
                    } else {
                        const int64_t h = (int64_t)atomicAdd((unsigned long long*)&s_blk[0], 1ull);
                        VL(0, 0)[h] = v;
                    }
                }
            }
            // per-lane counters of every parity (C_CNT, C_DEG)
            for (int i = tid; i < C_BASE; i += BB) ctr[i] = 0;
            __syncthreads();
            if (tid == 0) {
                for (int p = 0; p < 3; p++) { ctr[C_UDEG(p)] = 0; ctr[C_DDONE(p)] = 0; ctr[C_CT(p)] = 0; }
                for (int q = 0; q < 4; q++) { ctr[C_LT(q, 0)] = 0; ctr[C_LT(q, 1)] = 0; }
                ctr[C_LT(0, 0)] = s_blk[0];
                ctr[C_LT(0, 1)] = s_blk[1];
                ctr[C_CT(0)] = s_blk[2];
            }
        }
        grid_barrier(a.bar, gridDim.x);

        int64_t D = 0;
        // lengths of the current level's lists (L_D) and of the previous
        // level's (L_{D-1}, whose frontier words are cleared during level D)
        int64_t fl_len = ld_rlx(&ctr[C_LT(0, 0)]), fh_len = ld_rlx(&ctr[C_LT(0, 1)]);
        int64_t fc_len = ld_rlx(&ctr[C_CT(0)]);
        int64_t ol_len = 0, oh_len = 0;
        int64_t ucnt = fl_len + fh_len, udeg = 0;
        for (int l = 0; l < nsel; l++) udeg += s_mf[l];
        // out-arcs of vertices that every active lane has reached: a pull
        // step never scans their in-arcs again
        int64_t ddone = 0;
        bool bu = false;
        int64_t tslot = -1;
        int64_t mvis = 0, bytes = 0;
        int64_t my_scan = 0;   // in-arcs this thread scanned in pull steps (traffic count)
        for (;;) {
            // ------------------------------------ per-lane control (replicated)
            if (tid < MAXW) {
                int l = tid;
                if (s_st[l] == 1) {
                    if (s_nf[l] == 0) {
                        s_st[l] = 2;
                        s_maxD[l] = (int32_t)(D - 1);
                    } else if (cut_allowed(a.lb_mode, D) && !a.no_cut) {
                        int64_t bn, bd;
                        if (a.bv.harm) harm_cut_bound(s_H[l], s_nD[l], s_U[l], D, s_o[l], &bn, &bd);
                        else cut_bound(s_SD[l], s_nD[l], s_U[l], D, s_a[l], s_o[l], &bn, &bd);
                        if (lex_after(bn, bd, s_v[l] - s_off[l], s_xn[l], s_xd[l], s_xi[l])) {
                            s_st[l] = 3;
                            s_maxD[l] = (int32_t)D;
                        }
                    }
                }
                s_red_cnt[l] = 0;
                s_red_deg[l] = 0;
            }
            if (tid < 4) s_blk[tid] = 0;
            __syncthreads();
            if (tid < 64 * NW) {
                int l = tid;
                uint64_t m = __ballot(s_st[l] == 1);
                if (lane == 0) s_act[l >> 6] = m;
            }
            if (tid >= BB - 64) {   // the last wave: this level's out-degree sum over active lanes
                int64_t mv = 0;
                for (int l = lane; l < nsel; l += 64)
                    if (s_st[l] == 1) mv += s_mf[l];
                mv = wave_sum_i64(mv);
                if (lane == 0) s_scal[0] = mv;
            }
            __syncthreads();
            Mask<NW> act;
            bool any = false;
#pragma unroll
            for (int j = 0; j < NW; j++) { act.w[j] = s_act[j]; any |= act.w[j] != 0; }
            if (!any) break;
            mvis += s_scal[0];
            // direction on the union frontier.  With several lanes a pull
            // rarely stops early (every missing lane must be found), so it
            // pays only once the frontier's arcs rival the arcs still to be
            // scanned.  A pull also needs a frontier of at least n / beta
            // vertices, the size below which a pull returns to push, so the
            // choice cannot flip back and forth between small levels.
            const bool big = ucnt >= (int64_t)n / a.beta_bu;
            bool want_bu = bu ? big : (big && udeg > (a.g.m - ddone) / a.alpha_td);
            bu = want_bu;
            tslot = -1;
            if (boss && a.w.trace) {
                int64_t t = fadd_rlx(&a.w.trace[0], (int64_t)1);
                if (t < a.w.trace_cap) {
                    tslot = t;
                    int64_t* r = a.w.trace + 8 + 16 * t;
                    r[0] = batches; r[1] = D; r[2] = bu; r[3] = ucnt; r[4] = udeg;
                    r[5] = (int64_t)wall_clock64(); r[6] = nsel; r[7] = 0;
                    for (int j = 0; j < NW; j++) r[7] += __popcll(act.w[j]);
                }
            }
            const int p = (int)(D % 3);
            const int sC = (int)(D & 3), sN = (int)((D + 1) & 3), sO = (int)((D + 3) & 3);
            const uint64_t* Fc = fsel(a.w, D);
            uint64_t* Fn = fsel(a.w, D + 1);
            uint64_t* Fo = fsel(a.w, D + 2);   // F_{D-1}
            const int32_t* fl = VL(0, sC);
            const int32_t* fh = VL(1, sC);
            const int32_t* fcu = CU(D & 1);
            const int32_t* fcb = CB(D & 1);
            const NextLists nl{VL(0, sN), VL(1, sN), &ctr[C_LT(sN, 0)], CU((D + 1) & 1), CB((D + 1) & 1),
                               &ctr[C_CT((D + 1) % 3)], rp};
            const int32_t stamp = (int32_t)(D + 1);
            const bool rec_lvl = a.lb_mode && D + 1 < a.w.lcap;
            Stage stg{&s_stage[tid >> 6][0], 0};
            int64_t my_dd = 0, my_ud = 0;
            if (trb) tp = wall_clock64();
            // algorithmic bytes: clearing reads a list entry and writes the
            // old frontier word; push reads each frontier vertex's row and
            // frontier word and folds it into its visited word, then per
            // out-arc the index, the target's visited and frontier words and
            // its next word; pull reads every vertex's row, frontier and
            // visited words, writes the visited words of frontier vertices,
            // and per scanned in-arc reads the index and a frontier word
            // (counted in my_scan)
            bytes += (ol_len + oh_len) * (4 + 8 * NW) +
                     (bu ? (int64_t)n * (8 + 16 * NW) + (fl_len + fh_len) * (8 * NW)
                         : (fl_len + fh_len) * (8 + 24 * NW) + udeg * (4 + 24 * NW));
            // (1) F_{D-1} is no longer read: clear its words through L_{D-1}
            {
                const int32_t* ofl = VL(0, sO);
                const int32_t* ofh = VL(1, sO);
                for (int64_t i = gtid; i < ol_len + oh_len; i += nthreads) {
                    const int32_t u = i < ol_len ? ofl[i] : ofh[i - ol_len];
#pragma unroll
                    for (int j = 0; j < NW; j++) Fo[(int64_t)u * NW + j] = 0;
                }
            }
            PHASE(0);
            if (!bu) {
                if (fl_len <= nwaves) {
                    // small frontier: one wave per light vertex, one out-arc
                    // per lane (light vertices have at most 64)
                    for (int64_t i = gwave; i < fl_len; i += nwaves) {
                        const int32_t u = fl[i];
                        Mask<NW> f;
                        bool done = true;
#pragma unroll
                        for (int j = 0; j < NW; j++) {
                            const uint64_t fw = Fc[(int64_t)u * NW + j];
                            const uint64_t vn = vis[(int64_t)u * NW + j] | fw;
                            f.w[j] = fw & act.w[j];
                            done &= (act.w[j] & ~vn) == 0;
                            if (lane == 0) vis[(int64_t)u * NW + j] = vn;
                        }
                        const int32_t b = rp[u], e1 = rp[u + 1];
                        if (lane == 0 && done) my_dd += e1 - b;
                        if (!f.any()) continue;   // wave-uniform
                        const int32_t e = b + lane;
                        bool isnew = false;
                        int32_t w = 0, dw = 0;
                        Mask<NW> fr;
#pragma unroll
                        for (int j = 0; j < NW; j++) fr.w[j] = 0;
                        if (e < e1) {
                            w = ci[e];
                            Mask<NW> nb;
#pragma unroll
                            for (int j = 0; j < NW; j++)
                                nb.w[j] = f.w[j] & ~(vis[(int64_t)w * NW + j] | Fc[(int64_t)w * NW + j]);
                            if (nb.any()) {
                                isnew = discover<NW>(Fn, a.mark, w, nb, stamp, &fr);
                                if (isnew || fr.any()) dw = deg[w];
                                if (rec_lvl && fr.any()) record_levels<NW>(fr, w, a.w.lvl, W, D + 1);
                            }
                        }
                        tally<NW>(fr, dw, s_red_cnt, s_red_deg);
                        if (isnew) my_ud += dw;
                        list_append(isnew, w, dw, nl, stg);
                    }
                } else {
                    // push, light frontier vertices: one per lane; the owner
                    // folds F_D into the visited word
                    for (int64_t base = gwave * 64; base < fl_len; base += nwaves * 64) {
                        int64_t i = base + lane;
                        int32_t e = 0, end = 0;
                        Mask<NW> f;
#pragma unroll
                        for (int j = 0; j < NW; j++) f.w[j] = 0;
                        if (i < fl_len) {
                            const int32_t u = fl[i];
                            bool done = true;
#pragma unroll
                            for (int j = 0; j < NW; j++) {
                                const uint64_t fw = Fc[(int64_t)u * NW + j];
                                const uint64_t vn = vis[(int64_t)u * NW + j] | fw;
                                vis[(int64_t)u * NW + j] = vn;
                                f.w[j] = fw & act.w[j];
                                done &= (act.w[j] & ~vn) == 0;
                            }
                            e = rp[u];
                            end = rp[u + 1];
                            if (done) my_dd += end - e;
                            if (!f.any()) end = e;
                        }
                        while (__any(e < end)) {
                            bool isnew = false;
                            int32_t w = 0, dw = 0;
                            Mask<NW> fr;
#pragma unroll
                            for (int j = 0; j < NW; j++) fr.w[j] = 0;
                            if (e < end) {
                                w = ci[e];
                                e++;
                                Mask<NW> nb;
#pragma unroll
                                for (int j = 0; j < NW; j++)
                                    nb.w[j] = f.w[j] & ~(vis[(int64_t)w * NW + j] | Fc[(int64_t)w * NW + j]);
                                if (nb.any()) {
                                    isnew = discover<NW>(Fn, a.mark, w, nb, stamp, &fr);
                                    if (isnew || fr.any()) dw = deg[w];
                                    if (rec_lvl && fr.any()) record_levels<NW>(fr, w, a.w.lvl, W, D + 1);
                                }
                            }
                            tally<NW>(fr, dw, s_red_cnt, s_red_deg);
                            if (isnew) my_ud += dw;
                            list_append(isnew, w, dw, nl, stg);
                        }
                    }
                }
                PHASE(2);
                // heavy frontier vertices: the owner folds; their arcs go
                // through the chunk list
                for (int64_t i = gtid; i < fh_len; i += nthreads) {
                    const int32_t u = fh[i];
                    bool done = true;
#pragma unroll
                    for (int j = 0; j < NW; j++) {
                        const uint64_t vn = vis[(int64_t)u * NW + j] | Fc[(int64_t)u * NW + j];
                        vis[(int64_t)u * NW + j] = vn;
                        done &= (act.w[j] & ~vn) == 0;
                    }
                    if (done) my_dd += deg[u];
                }
                PHASE(1);
                // push, heavy frontier vertices: one wave per quarter chunk
                // (a few hubs then still spread over many waves)
                for (int64_t cq = gwave; cq < fc_len * PUSH_SUB; cq += nwaves) {
                    const int64_t c = cq / PUSH_SUB;
                    const int32_t u = fcu[c];
                    Mask<NW> f;
#pragma unroll
                    for (int j = 0; j < NW; j++) f.w[j] = Fc[(int64_t)u * NW + j] & act.w[j];
                    if (!f.any()) continue;   // wave-uniform
                    const int32_t b = fcb[c] + (int32_t)(cq % PUSH_SUB) * (CHUNK_ARCS / PUSH_SUB);
                    const int32_t lim = b + CHUNK_ARCS / PUSH_SUB;
                    const int32_t end = lim < rp[u + 1] ? lim : rp[u + 1];
                    for (int32_t e0 = b; e0 < end; e0 += 64) {
                        const int32_t e = e0 + lane;
                        bool isnew = false;
                        int32_t w = 0, dw = 0;
                        Mask<NW> fr;
#pragma unroll
                        for (int j = 0; j < NW; j++) fr.w[j] = 0;
                        if (e < end) {
                            w = ci[e];
                            Mask<NW> nb;
#pragma unroll
                            for (int j = 0; j < NW; j++)
                                nb.w[j] = f.w[j] & ~(vis[(int64_t)w * NW + j] | Fc[(int64_t)w * NW + j]);
                            if (nb.any()) {
                                isnew = discover<NW>(Fn, a.mark, w, nb, stamp, &fr);
                                if (isnew || fr.any()) dw = deg[w];
                                if (rec_lvl && fr.any()) record_levels<NW>(fr, w, a.w.lvl, W, D + 1);
                            }
                        }
                        tally<NW>(fr, dw, s_red_cnt, s_red_deg);
                        if (isnew) my_ud += dw;
                        list_append(isnew, w, dw, nl, stg);
                    }
                }
            } else {
                // pull: one lane per vertex.  A frontier vertex folds F_D into
                // its visited words here (readers use vis | F_D, so the
                // fold's timing does not matter).  Light vertices (few
                // in-arcs) scan their in-arcs, in groups of four (four
                // independent index loads, then four independent frontier
                // loads), until every missing active lane is found
                PHASE(1);
                // the next pass's frontier and visited words and row
                // pointers are loaded before this pass's dependent loads, so
                // they arrive while this pass waits for its own (only this
                // wave folds these vertices' visited words, and F_D does not
                // change during the level)
                uint64_t pf_f[NW], pf_v[NW];
                int32_t pf_b = 0, pf_e = 0;
                {
                    const int64_t w0 = gwave * 64 + lane;
#pragma unroll
                    for (int j = 0; j < NW; j++) { pf_f[j] = 0; pf_v[j] = 0; }
                    if (w0 < n) {
#pragma unroll
                        for (int j = 0; j < NW; j++) {
                            pf_f[j] = Fc[w0 * NW + j];
                            pf_v[j] = vis[w0 * NW + j];
                        }
                        pf_b = a.g.rrp[w0];
                        pf_e = a.g.rrp[w0 + 1];
                    }
                }
                for (int64_t base = gwave * 64; base < n; base += nwaves * 64) {
                    const int32_t w = (int32_t)(base + lane);
                    uint64_t cur_f[NW], cur_v[NW];
#pragma unroll
                    for (int j = 0; j < NW; j++) { cur_f[j] = pf_f[j]; cur_v[j] = pf_v[j]; }
                    const int32_t cur_b = pf_b, cur_e = pf_e;
                    {
                        const int64_t w2 = base + nwaves * 64 + lane;
                        if (w2 < n) {
#pragma unroll
                            for (int j = 0; j < NW; j++) {
                                pf_f[j] = Fc[w2 * NW + j];
                                pf_v[j] = vis[w2 * NW + j];
                            }
                            pf_b = a.g.rrp[w2];
                            pf_e = a.g.rrp[w2 + 1];
                        }
                    }
                    bool isnew = false;
                    int32_t dw = 0;
                    Mask<NW> acc, miss;
                    int32_t eb = 0, len = 0;
#pragma unroll
                    for (int j = 0; j < NW; j++) { acc.w[j] = 0; miss.w[j] = 0; }
                    if (w < n) {
                        uint64_t vn[NW];
                        bool inF = false;
#pragma unroll
                        for (int j = 0; j < NW; j++) {
                            const uint64_t fw = cur_f[j];
                            vn[j] = cur_v[j] | fw;
                            inF |= fw != 0;
                            miss.w[j] = act.w[j] & ~vn[j];
                        }
                        if (inF) {
#pragma unroll
                            for (int j = 0; j < NW; j++) vis[(int64_t)w * NW + j] = vn[j];
                            if (!miss.any()) my_dd += deg[w];
                        }
                        eb = cur_b;
                        const int32_t d_in = cur_e - eb;
                        if (d_in <= HEAVY_DEG && miss.any()) len = d_in;
                    }
                    int32_t* c_pre = &s_cpre[tid >> 6][0];
                    int32_t* c_beg = &s_cbeg[tid >> 6][0];
                    uint64_t* c_miss = &s_cmiss[tid >> 6][0];
                    uint64_t* c_acc = &s_cacc[tid >> 6][0];
                    if (wave_max_i32(len) > 8) {
                        // skewed in-degrees: the wave's lanes share the arcs
                        pull_shared<NW>(eb, len, miss, Fc, a.g.rci, c_pre, c_beg, c_miss, c_acc, &acc, &my_scan);
                    } else if (len > 0) {
                        {
                            const int32_t ee = eb + len;
                            for (int32_t e = eb; e < ee; e += 4) {
                                my_scan += (ee - e < 4 ? ee - e : 4);
                                int32_t u[4];
#pragma unroll
                                for (int t = 0; t < 4; t++) u[t] = e + t < ee ? a.g.rci[e + t] : -1;
                                bool full = true;
#pragma unroll
                                for (int j = 0; j < NW; j++) {
                                    uint64_t fo = 0;
#pragma unroll
                                    for (int t = 0; t < 4; t++)
                                        if (u[t] >= 0) fo |= Fc[(int64_t)u[t] * NW + j];
                                    acc.w[j] |= fo & miss.w[j];
                                    full &= acc.w[j] == miss.w[j];
                                }
                                if (full) break;
                            }
                        }
                    }
                    if (acc.any()) {
                        // a light vertex has one pulling thread: plain stores
#pragma unroll
                        for (int j = 0; j < NW; j++) Fn[(int64_t)w * NW + j] = acc.w[j];
                        isnew = true;
                        dw = deg[w];
                        if (rec_lvl) record_levels<NW>(acc, w, a.w.lvl, W, D + 1);
                    }
                    tally<NW>(acc, dw, s_red_cnt, s_red_deg);
                    if (isnew) my_ud += dw;
                    list_append(isnew, w, dw, nl, stg);
                }
                PHASE(2);
                // pull, mid in-degree vertices: packed segments of about
                // MID_ARCS in-arcs, one wave each, edge-balanced.  Segments,
                // then hub chunks, are dealt from the last wave down: low
                // vertex ids tend to have high degrees (preferential
                // attachment, R-MAT), so the first waves' light blocks are
                // the heaviest ones
                for (int64_t sg = nwaves - 1 - gwave; sg < a.g.nmseg; sg += nwaves) {
                    const int32_t v0 = a.g.mseg[sg], v1 = a.g.mseg[sg + 1];
                    const int32_t idx = v0 + lane;
                    int32_t w = 0, eb = 0, len = 0;
                    Mask<NW> miss, acc;
#pragma unroll
                    for (int j = 0; j < NW; j++) { miss.w[j] = 0; acc.w[j] = 0; }
                    if (idx < v1) {
                        w = a.g.mid_vtx[idx];
#pragma unroll
                        for (int j = 0; j < NW; j++)
                            miss.w[j] = act.w[j] & ~(vis[(int64_t)w * NW + j] | Fc[(int64_t)w * NW + j]);
                        eb = a.g.rrp[w];
                        if (miss.any()) len = a.g.rrp[w + 1] - eb;
                    }
                    if (wave_max_i32(len) > 0)
                        pull_shared<NW>(eb, len, miss, Fc, a.g.rci, &s_cpre[tid >> 6][0], &s_cbeg[tid >> 6][0],
                                        &s_cmiss[tid >> 6][0], &s_cacc[tid >> 6][0], &acc, &my_scan);
                    bool isnew = false;
                    int32_t dw = 0;
                    if (acc.any()) {
                        // a mid vertex lies in one segment: one pulling wave, plain stores
#pragma unroll
                        for (int j = 0; j < NW; j++) Fn[(int64_t)w * NW + j] = acc.w[j];
                        isnew = true;
                        dw = deg[w];
                        if (rec_lvl) record_levels<NW>(acc, w, a.w.lvl, W, D + 1);
                    }
                    tally<NW>(acc, dw, s_red_cnt, s_red_deg);
                    if (isnew) my_ud += dw;
                    list_append(isnew, w, dw, nl, stg);
                }
                // pull, hubs: one wave per chunk of their in-arcs; chunk c
                // goes to wave nwaves - 1 - (nmseg + c) mod nwaves
                for (int64_t c = ((nwaves - 1 - gwave - a.g.nmseg) % nwaves + nwaves) % nwaves; c < a.g.bnchunks;
                     c += nwaves) {
                    const int32_t w = a.g.bch_vtx[c];
                    Mask<NW> miss, acc;
#pragma unroll
                    for (int j = 0; j < NW; j++) {
                        miss.w[j] = __shfl(act.w[j] & ~(vis[(int64_t)w * NW + j] | Fc[(int64_t)w * NW + j]), 0, 64);
                        acc.w[j] = 0;
                    }
                    if (!miss.any()) continue;   // wave-uniform
                    const int32_t eb = a.g.bch_beg[c], ee = a.g.bch_end[c];
                    for (int32_t e0 = eb; e0 < ee; e0 += 64) {
                        const int32_t e = e0 + lane;
                        my_scan += e < ee ? 1 : 0;
                        if (e < ee) {
                            const int32_t u = a.g.rci[e];
#pragma unroll
                            for (int j = 0; j < NW; j++) acc.w[j] |= Fc[(int64_t)u * NW + j] & miss.w[j];
                        }
                        bool full = true;
#pragma unroll
                        for (int j = 0; j < NW; j++) {
                            acc.w[j] = wave_or_u64(acc.w[j]);
                            full &= acc.w[j] == miss.w[j];
                        }
                        if (full) break;
                    }
                    bool isnew = false;
                    int32_t dw = 0;
                    Mask<NW> fr;
#pragma unroll
                    for (int j = 0; j < NW; j++) fr.w[j] = 0;
                    if (lane == 0 && acc.any()) {
                        isnew = discover<NW>(Fn, a.mark, w, acc, stamp, &fr);
                        if (isnew || fr.any()) dw = deg[w];
                        if (rec_lvl && fr.any()) record_levels<NW>(fr, w, a.w.lvl, W, D + 1);
                    }
                    tally<NW>(fr, dw, s_red_cnt, s_red_deg);
                    if (isnew) my_ud += dw;
                    list_append(isnew, w, dw, nl, stg);
                }
            }
            PHASE(3);
            stage_flush(stg, nl.light, nl.tails);
            // workgroup totals into this level's counters
            my_dd = wave_sum_i64(my_dd);
            my_ud = wave_sum_i64(my_ud);
            if (lane == 0) {
                if (my_ud) atomicAdd((unsigned long long*)&s_blk[0], (unsigned long long)my_ud);
                if (my_dd) atomicAdd((unsigned long long*)&s_blk[1], (unsigned long long)my_dd);
            }
            __syncthreads();
            if (tid < W && s_red_cnt[tid]) {
                fadd_rlx(&ctr[C_CNT(p, tid)], (int64_t)s_red_cnt[tid]);
                fadd_rlx(&ctr[C_DEG(p, tid)], s_red_deg[tid]);
            }
            if (tid == 0) {
                if (s_blk[0]) fadd_rlx(&ctr[C_UDEG(p)], s_blk[0]);
                if (s_blk[1]) fadd_rlx(&ctr[C_DDONE(p)], s_blk[1]);
            }
            PHASE(4);
            grid_barrier(a.bar, gridDim.x);
            PHASE(5);
            if (boss && tslot >= 0) a.w.trace[8 + 16 * tslot + 8] = (int64_t)wall_clock64();
            if (trb) {
                if (lane == 0)
                    for (int i = 0; i < 6; i++) s_ph[tid >> 6][i] = ph[i];
                __syncthreads();
                if (tid == 0 && tslot >= 0)
                    for (int i = 0; i < 6; i++) {
                        int64_t mx = 0;
                        for (int wv = 0; wv < BB / 64; wv++) mx = s_ph[wv][i] > mx ? s_ph[wv][i] : mx;
                        a.w.trace[8 + 16 * tslot + 9 + i] = mx;
                    }
                for (int i = 0; i < 6; i++) ph[i] = 0;
            }
            // --------------------------------------------- advance lane state
            if (tid < MAXW) {
                int l = tid;
                if (s_st[l] == 1) {
                    int64_t c = ld_rlx(&ctr[C_CNT(p, l)]);
                    int64_t d = ld_rlx(&ctr[C_DEG(p, l)]);
                    s_nD[l] += c;
                    s_SD[l] += (D + 1) * c;
                    if (a.bv.harm) s_H[l] += (double)c / (double)(D + 1);
                    s_U[l] = dir ? d : d - c;
                    s_nf[l] = c;
                    s_mf[l] = d;
                    if (a.lb_mode && blockIdx.x == 0) {
                        if (D + 1 < a.w.lcap) a.w.hist[(D + 1) * W + l] = c;
                    }
                }
            }
            ol_len = fl_len;
            oh_len = fh_len;
            fl_len = ld_rlx(&ctr[C_LT(sN, 0)]);
            fh_len = ld_rlx(&ctr[C_LT(sN, 1)]);
            fc_len = ld_rlx(&ctr[C_CT((D + 1) % 3)]);
            ucnt = fl_len + fh_len;
            udeg = ld_rlx(&ctr[C_UDEG(p)]);
            ddone += ld_rlx(&ctr[C_DDONE(p)]);
            bytes += ucnt * (8 * NW + 4);
            if (boss) {
                // Reset what the next barrier's far side reuses: every
                // workgroup read these before the barrier just passed, and
                // none writes them before the next one.  Per-lane and union
                // counters of parity (D+2)%3 were last read after level D-1;
                // slot sO held L_{D-1} (cleared during this level) and is next
                // filled during level D+2; chunk tail D%3 was read after
                // level D-1 and is next filled during level D+2.
                const int q3 = (int)((D + 2) % 3);
                ctr[C_UDEG(q3)] = 0;
                ctr[C_DDONE(q3)] = 0;
                ctr[C_LT(sO, 0)] = 0;
                ctr[C_LT(sO, 1)] = 0;
                ctr[C_CT(D % 3)] = 0;
            }
            if (blockIdx.x == 0 && tid < W) {   // the per-lane counters of that parity
                const int q3 = (int)((D + 2) % 3);
                ctr[C_CNT(q3, tid)] = 0;
                ctr[C_DEG(q3, tid)] = 0;
            }
            D++;
            __syncthreads();
        }
        // pull traffic of the batch: one count per workgroup
        {
            const int64_t t = wave_sum_i64(my_scan);
            if (tid == 0) s_blk[0] = 0;
            __syncthreads();
            if (lane == 0 && t) atomicAdd((unsigned long long*)&s_blk[0], (unsigned long long)t);
            __syncthreads();
            if (tid == 0 && s_blk[0]) fadd_rlx(&stats[ST_BYTES], s_blk[0] * (int64_t)(4 + 8 * NW));
        }
        // ----------------------------------------------------- batch results
        // The exact lanes' results go into their request's top k (Alg. 1).
        // Only the k best of a request's results in this batch can be among
        // its k best overall, so wave 0 of workgroup 0 ranks them per
        // request (by farness, then id, then lane), and one thread inserts
        // the ranks below k best first: an entry that no entry before it
        // follows is placed after one comparison.  In all-ties mode every
        // exact result goes in, in lane order, so the tie buffer sees what
        // the top k refuses.  (The pull's per-wave LDS scratch is free here.)
        if (blockIdx.x == 0 && tid < 64) {
            int32_t* r_rank = &s_cpre[0][0];
            int32_t* r_id = &s_cbeg[0][0];
            int64_t* r_num = (int64_t*)&s_cmiss[0][0];
            int64_t* r_den = (int64_t*)&s_cacc[0][0];
            int64_t ex = 0, cu = 0, md = 0;
            for (int l = lane; l < nsel; l += 64) {
                md = s_maxD[l] > md ? s_maxD[l] : md;
                r_rank[l] = -1;
                if (s_st[l] == 2) {
                    ex++;
                    r_id[l] = s_v[l] - s_off[l];
                    if (a.bv.harm) {
                        r_num[l] = harm_enc(s_H[l]);
                        r_den[l] = 1;
                    } else {
                        r_num[l] = s_SD[l];
                        r_den[l] = s_nD[l] <= 1 ? 0 : sq64(s_nD[l] - 1);
                    }
                } else if (s_st[l] == 3) {
                    cu++;
                }
            }
            ex = wave_sum_i64(ex);
            cu = wave_sum_i64(cu);
            md = wave_max_i64(md);
            __builtin_amdgcn_wave_barrier();
            if (ex > 0 && !a.no_cut) {
                for (int l = lane; l < nsel; l += 64) {
                    if (s_st[l] != 2) continue;
                    const DevTopk& tk = a.npreq ? a.preq[s_req[l]].tk : a.tk;
                    if (ld_rlx(&tk.st->ties)) {
                        r_rank[l] = -2;
                        continue;
                    }
                    int32_t rk = 0;
                    for (int q = 0; q < nsel; q++) {
                        if (q == l || s_st[q] != 2 || s_req[q] != s_req[l]) continue;
                        if (lex_after(r_num[l], r_den[l], r_id[l], r_num[q], r_den[q], r_id[q]) ||
                            (q < l && !lex_after(r_num[q], r_den[q], r_id[q], r_num[l], r_den[l], r_id[l])))
                            rk++;
                    }
                    r_rank[l] = rk < ld_rlx(&tk.st->k) ? rk : -1;
                }
                __builtin_amdgcn_wave_barrier();
                // insertion order: by rank, then lane (each request's own
                // entries arrive in rank order)
                int32_t* r_ord = &s_stage[0][0];
                int32_t nins = 0;
                for (int l = lane; l < nsel; l += 64) {
                    if (r_rank[l] < 0) continue;
                    int32_t g = 0;
                    for (int q = 0; q < nsel; q++)
                        g += r_rank[q] >= 0 && (r_rank[q] < r_rank[l] || (r_rank[q] == r_rank[l] && q < l));
                    r_ord[g] = l;
                    nins++;
                }
                nins = wave_sum_i32(nins);
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) {
                    for (int32_t g = 0; g < nins; g++) {
                        const int l = r_ord[g];
                        const DevTopk& tk = a.npreq ? a.preq[s_req[l]].tk : a.tk;
                        topk_insert(tk.st, tk.ring, tk.S, tk.R, tk.I, r_num[l], a.bv.harm ? 2 : s_nD[l], r_id[l]);
                    }
                    // all-ties mode: every exact result, in lane order
                    for (int l = 0; l < nsel; l++) {
                        if (r_rank[l] != -2) continue;
                        const DevTopk& tk = a.npreq ? a.preq[s_req[l]].tk : a.tk;
                        topk_insert(tk.st, tk.ring, tk.S, tk.R, tk.I, r_num[l], a.bv.harm ? 2 : s_nD[l], r_id[l]);
                    }
                }
            }
            if (lane == 0) {
                // the until_x decision, taken once so every workgroup makes it alike
                if (a.until_x) ctr[C_XDONE] = ld_acq(&a.tk.st->seq) >= 0 ? 1 : 0;
                fadd_rlx(&stats[ST_STARTED], (int64_t)nsel);
                fadd_rlx(&stats[ST_EXACT], ex);
                fadd_rlx(&stats[ST_CUT], cu);
                fadd_rlx(&stats[ST_MVIS], mvis);
                fadd_rlx(&stats[ST_BYTES], bytes);
                __hip_atomic_fetch_max(&stats[ST_MAXLEVEL], md, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (a.no_cut && blockIdx.x == 0 && tid < nsel) {
            a.out_S[pos - nsel + tid] = s_SD[tid];
            a.out_r[pos - nsel + tid] = s_nD[tid];
        }
        if (a.lb_mode) {
            // Lev tables per exact lane (thread per lane), then every vertex
            // takes the best level bound over the lanes that reached it
            // every level's counts and levels fit the tables (same value in
            // every workgroup: D is replicated)
            const bool lbok = D < a.w.lcap;
            if (lbok && a.bv.harm) {
                // harmonic centrality: per exact lane and level l the sum
                // over levels i of n_i / max(2, gap) minus w's own 1/2, in
                // increasing i (entries spread over the whole grid)
                const int64_t L1 = D + 1;
                for (int64_t q = gtid; q < (int64_t)nsel * L1; q += nthreads) {
                    const int l = (int)(q / L1);
                    const int64_t lv = q % L1;
                    if (s_st[l] != 2 || lv > s_maxD[l]) continue;
                    double x = 0.0;
                    for (int64_t i = 0; i <= s_maxD[l]; i++) {
                        const int64_t t = dir ? i - lv : (i > lv ? i - lv : lv - i);
                        x += (double)a.w.hist[i * W + l] / (double)(t < 2 ? 2 : t);
                    }
                    a.w.levtab[lv * W + l] = __double_as_longlong(x - 0.5);
                }
                grid_barrier(a.bar, gridDim.x);
                // every vertex takes the least bound over the lanes that
                // reached it, its out-neighbours at exactly 1
                for (int64_t w = gtid; w < n; w += nthreads) {
                    double best = 0.0;
                    bool any = false;
#pragma unroll
                    for (int j = 0; j < NW; j++) {
                        uint64_t m = vis[w * NW + j];
                        while (m) {
                            int l = j * 64 + __ffsll((long long)m) - 1;
                            m &= m - 1;
                            if (l >= nsel || s_st[l] != 2 || s_v[l] == w) continue;
                            if (dir && a.rc.scc[w] != a.rc.scc[s_v[l]]) continue;
                            const int64_t lv = a.w.lvl[w * W + l];
                            const double b = __longlong_as_double(a.w.levtab[lv * W + l]) + 0.5 * (double)deg[w];
                            if (!any || b < best) { best = b; any = true; }
                        }
                    }
                    if (any) {
                        const int64_t f = harm_enc(best * (1.0 + HARM_MARGIN));
                        if (rat_cmp(f, 1, a.bv.num[w], a.bv.den[w]) > 0) { a.bv.num[w] = f; a.bv.den[w] = 1; }
                    }
                }
            } else if (lbok) {
                if (blockIdx.x == 0 && tid < nsel && s_st[tid] == 2) {
                    int l = tid;
                    int64_t maxD = s_maxD[l];
                    int64_t r = s_nD[l];
                    int64_t* lev = a.w.levtab;
                    const int64_t* gam = a.w.hist;
                    int64_t L = -2;
                    for (int64_t j = 0; j <= maxD; j++) {
                        int64_t t = j > 1 ? j - 1 : 1 - j;
                        L += (t <= 1 ? 2 : t) * gam[j * W + l];
                    }
                    lev[1 * W + l] = L;
                    int64_t pre = 0, low = 0;
                    for (int64_t j = 0; j <= 2 && j <= maxD; j++) pre += gam[j * W + l];
                    for (int64_t i = 2; i <= maxD; i++) {
                        if (i + 1 <= maxD) pre += gam[(i + 1) * W + l];
                        if (i - 3 >= 0) low += gam[(i - 3) * W + l];
                        lev[i * W + l] = lev[(i - 1) * W + l] + (dir ? 0 : low) - (r - pre);
                    }
                }
                grid_barrier(a.bar, gridDim.x);
                for (int64_t w = gtid; w < n; w += nthreads) {
                    int64_t best = -1;
                    int64_t bden = 0;
#pragma unroll
                    for (int j = 0; j < NW; j++) {
                        uint64_t m = vis[w * NW + j];
                        while (m) {
                            int l = j * 64 + __ffsll((long long)m) - 1;
                            m &= m - 1;
                            if (l >= nsel || s_st[l] != 2 || s_v[l] == w) continue;
                            if (dir && a.rc.scc[w] != a.rc.scc[s_v[l]]) continue;
                            int64_t lv = a.w.lvl[w * W + l];
                            int64_t b = a.w.levtab[lv * W + l];
                            if (b > best) { best = b; bden = sq64(s_nD[l] - 1); }
                        }
                    }
                    if (best >= 0) {
                        int64_t b = best - deg[w];
                        if (b < 0) b = 0;
                        int64_t on = a.bv.num[w], od = a.bv.den[w];
                        if (od != 0 && rat_cmp(b, bden, on, od) > 0) { a.bv.num[w] = b; a.bv.den[w] = bden; }
                    }
                }
            }
        }
        // Clear the batch's words for the next batch.  Nothing reads them
        // after the last level's barrier except the level-based update, so
        // only that (and the until_x decision) needs a barrier first; the
        // next batch's selection barrier orders the clear before its level 0
        // (and the kernel's end before the host reads anything)
        if (a.lb_mode || a.until_x) grid_barrier(a.bar, gridDim.x);
        {
            int64_t tot = (int64_t)n * NW;
            for (int64_t q = gtid; q < tot; q += nthreads) {
                vis[q] = 0;
                a.w.frt0[q] = 0;
                a.w.frt1[q] = 0;
                a.w.nxt[q] = 0;
            }
            if (NW > 1)
                for (int64_t q = gtid; q < n; q += nthreads) a.mark[q] = 0;
        }
        batches++;
        if (stop_now) break;
        if (a.until_x && ld_rlx(&ctr[C_XDONE]) != 0) break;
    }
    if (boss) stats[ST_CURSOR] = pos;
}

int tkc_launch_batch(const DevGraph& g, DevReach rc, OrderView ov, BoundsView bv, DevTopk tk,
                     BatchWork w, int64_t* stats, const int32_t* list, int32_t list_count,
                     int32_t start_pos, int32_t max_batches, int lb_mode, bool no_cut,
                     int64_t* out_S, int64_t* out_r, const EngineTuning& tune, hipStream_t s,
                     int* grid_out, const PackReq* preq, int32_t npreq) {
    int W = tune.batch_width;
    if (W != 32 && W != 64 && W != 128 && W != 256) return -2;
    // a packed launch: requests of a union graph, BFSCut only, from their orders
    if (npreq < 0 || npreq > TKC_PACK_MAXREQ) return -2;
    if (npreq > 0 && (!preq || !w.cand_req || lb_mode || no_cut || list || max_batches != 0)) return -2;
    if (!w.bar || !w.vis || !w.frt0 || !w.frt1 || !w.nxt || !w.list || !w.ctr || !w.cand || !stats) return -2;
    if (lb_mode && (!w.lvl || !w.hist || !w.levtab)) return -2;
    int NW = W <= 64 ? 1 : W / 64;
    const int cus = tkc_cu_count();
    if (cus < 1) return -1;
    const bool tr = w.trace != nullptr;
    const void* fn = NW == 1 ? (tr ? (const void*)k_batch<1, true> : (const void*)k_batch<1, false>)
                   : NW == 2 ? (tr ? (const void*)k_batch<2, true> : (const void*)k_batch<2, false>)
                             : (tr ? (const void*)k_batch<4, true> : (const void*)k_batch<4, false>);
    hipError_t e;
    const int occ = tkc_occupancy(fn, BB);
    if (occ < 1) return -1;
    const int want = tune.blocks_per_cu > 0 ? tune.blocks_per_cu : 2;
    int per = occ < want ? occ : want;
    const int grid = tkc_grid_for(cus, per, g.n);
    if (grid_out) *grid_out = grid;
    BatchArgs a{};
    a.g = g; a.rc = rc; a.ov = ov; a.bv = bv; a.tk = tk; a.w = w;
    a.stats = stats; a.list = list; a.list_count = list_count;
    a.start_pos = start_pos;
    a.max_batches = max_batches > 0 ? max_batches : 0x7fffffff;
    a.lb_mode = lb_mode;
    a.no_cut = no_cut ? 1 : 0;
    a.until_x = (max_batches == -1) ? 1 : 0;
    if (max_batches == -1) a.max_batches = 0x7fffffff;
    a.W = W;
    a.Wsel = (tune.lanes_cap > 0 && tune.lanes_cap < W) ? tune.lanes_cap : W;
    a.alpha_td = tune.batch_alpha > 0 ? tune.batch_alpha : 14;
    a.beta_bu = tune.bu_td_beta > 0 ? tune.bu_td_beta : 24;
    a.out_S = out_S;
    a.out_r = out_r;
    a.mark = (int32_t*)w.touched;
    a.bar = w.bar;
    a.preq = preq;
    a.npreq = npreq;
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(BB), args, 0, s);
    return e == hipSuccess ? 0 : -1;
}
