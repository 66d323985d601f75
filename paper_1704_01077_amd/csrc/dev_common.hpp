// Device-side helpers shared by the HIP kernels of the top-k closeness path.
// gfx950 (CDNA4): 64-lane wavefronts, per-XCD L2, agent-scope atomics for
// anything another workgroup may read before the kernel ends.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TKC_DEV __device__ __forceinline__

typedef unsigned __int128 tkc_u128;

// ---------------------------------------------------------------- atomics
template <typename T>
TKC_DEV T ld_acq(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
TKC_DEV T ld_rlx(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
TKC_DEV void st_rel(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
TKC_DEV void st_rlx(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
TKC_DEV T fadd_rlx(T* p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
TKC_DEV T for_rlx(T* p, T v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// or into a word only this workgroup touches
template <typename T>
TKC_DEV T for_wg(T* p, T v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------------ grid barrier
// Barrier of a cooperative (all workgroups resident) launch.  Same-address
// atomics serialize at the memory side (~75 ns each on MI355X), so a flat
// counter costs ~75 ns per workgroup; here arrivals go up a tree of
// counters with fan-in 16, each counter on its own 128-byte line, and only
// the last arriver of a group climbs.  The overall last arriver bumps the
// generation word that everyone else polls.  Counters return to zero after
// every use (the last arriver of a group resets it before climbing; nobody
// re-arrives before the generation changes).  Layout of `bar`: word 0 is
// the generation, counter slot s lives at word (s + 1) * TKC_BAR_PAD.
// Publication: a workgroup barrier does not wait for a wave's outstanding
// global stores, so every wave first waits for its own (vmcnt(0)); once all
// of them sit in the XCD's L2, one agent-scope release fence by thread 0
// (an L2 write-back) publishes the whole workgroup's stores before its
// relaxed arrival.  The last arriver of a group takes an acquire-release
// fence before it climbs, and thread 0 of every workgroup takes an
// agent-scope acquire fence (L1/L2 invalidate, shared by the workgroup's
// waves on one CU) before the closing workgroup barrier.  Per-wave fences
// instead of thread-0 fences cost about three times as much (43 us against
// 13 us per barrier at 512 workgroups).
#define TKC_BAR_FAN 16
#define TKC_BAR_PAD 32
// Which searches the BFSCut bound may stop (lb_mode as the engines take
// it).  Cut variants: any.  Level-based variants: none, since only complete
// searches give level-based updates.  The combination: only shallow ones
// (level <= CUTLB_DEPTH).  A search that the bound stops early costs little
// and its update would be worth little; one that runs deep (high-diameter
// graphs, where the cut bound fires late) is completed and feeds the
// level-based update instead.
#define CUTLB_DEPTH 8
TKC_DEV bool cut_allowed(int32_t lb_mode, int64_t level) {
    return lb_mode == 0 || (lb_mode == 2 && level <= CUTLB_DEPTH);
}

TKC_DEV void grid_barrier(uint32_t* bar, uint32_t nblocks) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's stores done
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* gen = bar;
        uint32_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        uint32_t idx = blockIdx.x, width = nblocks, base = 0;
        for (;;) {
            uint32_t grp = idx / TKC_BAR_FAN;
            uint32_t ngroups = (width + TKC_BAR_FAN - 1) / TKC_BAR_FAN;
            uint32_t gsize = width - grp * TKC_BAR_FAN;
            if (gsize > TKC_BAR_FAN) gsize = TKC_BAR_FAN;
            uint32_t* c = bar + (size_t)(base + grp + 1) * TKC_BAR_PAD;
            uint32_t old = __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old + 1 != gsize) {
                while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g)
                    __builtin_amdgcn_s_sleep(1);
                break;
            }
            __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            if (ngroups == 1) {
                __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            base += ngroups;
            idx = grp;
            width = ngroups;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}
// words of barrier state for up to `nblocks` workgroups
static inline size_t tkc_bar_words(uint32_t nblocks) { return (size_t)(nblocks + 2) * TKC_BAR_PAD; }

// ------------------------------------------------------------ wave helpers
TKC_DEV int lane_id() { return (int)__lane_id(); }

// Wave reductions.  With every lane of the wave active they run on DPP
// moves inside each row of 16 lanes (quad permutations, then the half-row
// and row mirrors), join the four rows with the row broadcasts of lanes 15
// and 31, and read the total from lane 63: VALU work, no trip through the
// LDS crossbar.  In divergent code they fall back to butterfly shuffles.
#define TKC_DPP_XOR1 0xB1        // quad_perm [1,0,3,2]
#define TKC_DPP_XOR2 0x4E        // quad_perm [2,3,0,1]
#define TKC_DPP_QREV 0x1B        // quad_perm [3,2,1,0]
#define TKC_DPP_HMIRROR 0x141    // lane i of each 8 reads lane 7 - i
#define TKC_DPP_MIRROR 0x140     // lane i of each row reads lane 15 - i
#define TKC_DPP_ROR8 0x128       // lane i of each row reads lane i ^ 8
#define TKC_DPP_BCAST15 0x142    // lane 15 of each row into the next row
#define TKC_DPP_BCAST31 0x143    // lane 31 into rows 2 and 3
TKC_DEV bool wave_full() { return __builtin_amdgcn_read_exec() == ~0ull; }
template <int CTRL>
TKC_DEV uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
// the value of lane 15 (rows 1, 3) or 31 (rows 2, 3); `idv` elsewhere
template <int CTRL, int ROWS>
TKC_DEV uint32_t dpp_bcast_u32(uint32_t idv, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)idv, (int)v, CTRL, ROWS, 0xF, false);
}
TKC_DEV uint32_t readlane63(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }

TKC_DEV int64_t wave_sum_i64(int64_t v) {
    if (wave_full()) {
        uint64_t x = (uint64_t)v;
#define TKC_STEP64(MOVE)                                                              \
        {                                                                             \
            const uint64_t y = (uint64_t)MOVE((uint32_t)x) | ((uint64_t)MOVE((uint32_t)(x >> 32)) << 32); \
            x += y;                                                                   \
        }
        TKC_STEP64(dpp_u32<TKC_DPP_XOR1>)
        TKC_STEP64(dpp_u32<TKC_DPP_XOR2>)
        TKC_STEP64(dpp_u32<TKC_DPP_HMIRROR>)
        TKC_STEP64(dpp_u32<TKC_DPP_MIRROR>)
#undef TKC_STEP64
        {
            const uint64_t y = (uint64_t)dpp_bcast_u32<TKC_DPP_BCAST15, 0xA>(0u, (uint32_t)x) |
                               ((uint64_t)dpp_bcast_u32<TKC_DPP_BCAST15, 0xA>(0u, (uint32_t)(x >> 32)) << 32);
            x += y;
        }
        {
            const uint64_t y = (uint64_t)dpp_bcast_u32<TKC_DPP_BCAST31, 0xC>(0u, (uint32_t)x) |
                               ((uint64_t)dpp_bcast_u32<TKC_DPP_BCAST31, 0xC>(0u, (uint32_t)(x >> 32)) << 32);
            x += y;
        }
        return (int64_t)((uint64_t)readlane63((uint32_t)x) | ((uint64_t)readlane63((uint32_t)(x >> 32)) << 32));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
TKC_DEV int32_t wave_sum_i32(int32_t v) {
    if (wave_full()) {
        uint32_t x = (uint32_t)v;
        x += dpp_u32<TKC_DPP_XOR1>(x);
        x += dpp_u32<TKC_DPP_XOR2>(x);
        x += dpp_u32<TKC_DPP_HMIRROR>(x);
        x += dpp_u32<TKC_DPP_MIRROR>(x);
        x += dpp_bcast_u32<TKC_DPP_BCAST15, 0xA>(0u, x);
        x += dpp_bcast_u32<TKC_DPP_BCAST31, 0xC>(0u, x);
        return (int32_t)readlane63(x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
TKC_DEV int32_t wave_max_i32(int32_t v) {
    if (wave_full()) {
        int32_t x = v, y;
        y = (int32_t)dpp_u32<TKC_DPP_XOR1>((uint32_t)x); x = y > x ? y : x;
        y = (int32_t)dpp_u32<TKC_DPP_XOR2>((uint32_t)x); x = y > x ? y : x;
        y = (int32_t)dpp_u32<TKC_DPP_HMIRROR>((uint32_t)x); x = y > x ? y : x;
        y = (int32_t)dpp_u32<TKC_DPP_MIRROR>((uint32_t)x); x = y > x ? y : x;
        y = (int32_t)dpp_bcast_u32<TKC_DPP_BCAST15, 0xA>(0x80000000u, (uint32_t)x); x = y > x ? y : x;
        y = (int32_t)dpp_bcast_u32<TKC_DPP_BCAST31, 0xC>(0x80000000u, (uint32_t)x); x = y > x ? y : x;
        return (int32_t)readlane63((uint32_t)x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        int32_t y = __shfl_xor(v, o, 64);
        v = y > v ? y : v;
    }
    return v;
}
TKC_DEV int64_t wave_max_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t y = __shfl_xor(v, o, 64);
        v = y > v ? y : v;
    }
    return v;
}
TKC_DEV uint64_t wave_or_u64(uint64_t v) {
    if (wave_full()) {
        uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
        lo |= dpp_u32<TKC_DPP_XOR1>(lo);    hi |= dpp_u32<TKC_DPP_XOR1>(hi);
        lo |= dpp_u32<TKC_DPP_XOR2>(lo);    hi |= dpp_u32<TKC_DPP_XOR2>(hi);
        lo |= dpp_u32<TKC_DPP_HMIRROR>(lo); hi |= dpp_u32<TKC_DPP_HMIRROR>(hi);
        lo |= dpp_u32<TKC_DPP_MIRROR>(lo);  hi |= dpp_u32<TKC_DPP_MIRROR>(hi);
        lo |= dpp_bcast_u32<TKC_DPP_BCAST15, 0xA>(0u, lo); hi |= dpp_bcast_u32<TKC_DPP_BCAST15, 0xA>(0u, hi);
        lo |= dpp_bcast_u32<TKC_DPP_BCAST31, 0xC>(0u, lo); hi |= dpp_bcast_u32<TKC_DPP_BCAST31, 0xC>(0u, hi);
        return (uint64_t)readlane63(lo) | ((uint64_t)readlane63(hi) << 32);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}
// 64 x 64 bit-matrix transpose across the wave, called by all 64 lanes: on
// entry lane r holds row r, on return lane c holds column c (bit r of the
// result is bit c of row r).  Stage s exchanges, between lanes r and r ^ s,
// the bits whose column index differs from the row index in bit s; the six
// stages commute.  Stages 32 and 16 cross rows of 16 lanes and take one
// 32-bit shuffle each (a lane sends exactly the half of its bits the
// partner keeps); stages 8, 4, 2 and 1 use DPP moves.
TKC_DEV uint64_t wave_transpose64(uint64_t x) {
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {   // s = 32: columns 32-63 of rows 0-31 trade with columns 0-31 of rows 32-63
        const bool up = lane & 32u;
        const uint32_t got = (uint32_t)__shfl_xor((int)(up ? lo : hi), 32, 64);
        if (up) lo = got; else hi = got;
    }
    {   // s = 16, in both 32-bit halves at once: a lower lane keeps the low
        // 16 bits of each half and takes the partner's low 16 bits into its
        // high 16; an upper lane the other way round
        const bool up = lane & 16u;
        const uint32_t send = up ? ((lo & 0xFFFFu) | (hi << 16)) : ((lo >> 16) | (hi & 0xFFFF0000u));
        const uint32_t got = (uint32_t)__shfl_xor((int)send, 16, 64);
        if (up) {
            lo = (lo & 0xFFFF0000u) | (got & 0xFFFFu);
            hi = (hi & 0xFFFF0000u) | (got >> 16);
        } else {
            lo = (lo & 0xFFFFu) | (got << 16);
            hi = (hi & 0xFFFFu) | (got & 0xFFFF0000u);
        }
    }
#define TKC_TSTAGE(S, M, YLO, YHI)                                                 \
    {                                                                              \
        const uint32_t ylo = YLO, yhi = YHI;                                       \
        if (lane & (S)) {                                                          \
            lo = (lo & ~(M)) | ((ylo >> (S)) & (M));                               \
            hi = (hi & ~(M)) | ((yhi >> (S)) & (M));                               \
        } else {                                                                   \
            lo = (lo & (M)) | ((ylo << (S)) & ~(M));                               \
            hi = (hi & (M)) | ((yhi << (S)) & ~(M));                               \
        }                                                                          \
    }
    TKC_TSTAGE(8u, 0x00FF00FFu, dpp_u32<TKC_DPP_ROR8>(lo), dpp_u32<TKC_DPP_ROR8>(hi))
    // lane i ^ 4: the half-row mirror (7 - i) after the quad reversal (3 - i)
    TKC_TSTAGE(4u, 0x0F0F0F0Fu, dpp_u32<TKC_DPP_HMIRROR>(dpp_u32<TKC_DPP_QREV>(lo)),
               dpp_u32<TKC_DPP_HMIRROR>(dpp_u32<TKC_DPP_QREV>(hi)))
    TKC_TSTAGE(2u, 0x33333333u, dpp_u32<TKC_DPP_XOR2>(lo), dpp_u32<TKC_DPP_XOR2>(hi))
    TKC_TSTAGE(1u, 0x55555555u, dpp_u32<TKC_DPP_XOR1>(lo), dpp_u32<TKC_DPP_XOR1>(hi))
#undef TKC_TSTAGE
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
// exclusive prefix of a 0/1 predicate within the wave, plus the wave total
TKC_DEV int wave_rank(bool pred, int* total) {
    uint64_t m = __ballot(pred);
    *total = __popcll(m);
    uint64_t below = (lane_id() == 0) ? 0ull : (m & (~0ull >> (64 - lane_id())));
    return __popcll(below);
}

// --------------------------------------------------- exact farness algebra
// A farness value in units of (n-1): num / den with den = (r-1)^2 > 0, or
// +inf encoded as den == 0.  Comparisons are exact (128-bit products: num
// stays below 2^40 and den below 2^62 on every supported graph).
TKC_DEV int rat_cmp(int64_t na, int64_t da, int64_t nb, int64_t db) {
    bool ia = (da == 0), ib = (db == 0);
    if (ia || ib) return (int)ia - (int)ib;
    tkc_u128 x = (tkc_u128)(uint64_t)na * (uint64_t)db;
    tkc_u128 y = (tkc_u128)(uint64_t)nb * (uint64_t)da;
    return x < y ? -1 : (x > y ? 1 : 0);
}
// signed numerators (the raw Lemma 6.1 form can go negative)
TKC_DEV int rat_cmp_signed(int64_t na, int64_t da, int64_t nb, int64_t db) {
    __int128 x = (__int128)na * (__int128)db;
    __int128 y = (__int128)nb * (__int128)da;
    return x < y ? -1 : (x > y ? 1 : 0);
}
TKC_DEV int64_t sq64(int64_t a) { return a * a; }

// exact (farness, id) order: true when (na/da, ia) comes strictly after (nb/db, ib)
TKC_DEV bool lex_after(int64_t na, int64_t da, int32_t ia, int64_t nb, int64_t db, int32_t ib) {
    int c = rat_cmp(na, da, nb, db);
    return c > 0 || (c == 0 && ia > ib);
}

// -------------------------------------------------------------- k-th value
// The current k-th best result x = (S, r, id).  Published through a ring of
// records and a sequence counter so readers never mix two records: a reader
// takes seq, the record, then seq again, and retries unless fewer than RING
// newer records were published meanwhile.  seq < 0 means "fewer than k
// results so far" (x = +inf).
#define TKC_XRING 256
struct XRec {
    int64_t S;
    int64_t r;
    int64_t id;
};
struct TopkState {
    int32_t lock;
    int32_t cnt;
    int64_t seq;      // number of published records - 1
    int32_t k;
    int32_t ties;     // all-ties mode: x is published with id +inf
    int64_t n_inserts;
    // all-ties mode: every entry pushed out of the top k or rejected there
    int32_t tcnt;
    int32_t tcap;
    int64_t* tieS;
    int64_t* tieR;
    int32_t* tieI;
};
struct XVal {
    int64_t num;      // S
    int64_t den;      // (r-1)^2, 0 = +inf
    int32_t id;
};

TKC_DEV XVal read_x(TopkState* st, const XRec* ring) {
    XVal x;
    for (;;) {
        int64_t s1 = ld_acq(&st->seq);
        if (s1 < 0) { x.num = 0; x.den = 0; x.id = 0x7fffffff; return x; }
        const XRec* rc = ring + (s1 % TKC_XRING);
        int64_t S = ld_rlx(&rc->S), r = ld_rlx(&rc->r), id = ld_rlx(&rc->id);
        int64_t s2 = ld_acq(&st->seq);
        if (s2 - s1 < TKC_XRING - 1) {
            x.num = S;
            x.den = r <= 1 ? 0 : sq64(r - 1);
            x.id = (int32_t)id;
            return x;
        }
    }
}

TKC_DEV void tie_keep(TopkState* st, int64_t S, int64_t r, int32_t id) {
    const int32_t t = ld_rlx(&st->tcnt);
    if (t < st->tcap) {
        st_rlx(&st->tieS[t], S);
        st_rlx(&st->tieR[t], r);
        st_rlx(&st->tieI[t], id);
    }
    st_rlx(&st->tcnt, t + 1);
}
// Insert an exact result; the caller is one thread.  topk arrays hold the
// min(k, inserted) best (S, r, id) in exact order.  Spins on st->lock.  In
// all-ties mode every entry that leaves the top k, or is refused by it, is
// kept for the final tie filter, and x carries id +inf, which turns every
// lexicographic cut, skip and stop test into a strict "farness above x".
TKC_DEV void topk_insert(TopkState* st, XRec* ring, int64_t* tS, int64_t* tR, int32_t* tI,
                         int64_t S, int64_t r, int32_t id) {
    while (__hip_atomic_exchange(&st->lock, 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0)
        __builtin_amdgcn_s_sleep(2);
    int32_t k = ld_rlx(&st->k);
    int32_t cnt = ld_rlx(&st->cnt);
    int64_t den = r <= 1 ? 0 : sq64(r - 1);
    // position = number of entries that precede (S, r, id)
    int32_t p = cnt;
    while (p > 0) {
        int64_t pr = ld_rlx(&tR[p - 1]);
        int64_t pd = pr <= 1 ? 0 : sq64(pr - 1);
        if (lex_after(ld_rlx(&tS[p - 1]), pd, ld_rlx(&tI[p - 1]), S, den, id)) p--;
        else break;
    }
    if (st->ties) {
        if (p >= k) tie_keep(st, S, r, id);
        else if (cnt == k) tie_keep(st, ld_rlx(&tS[k - 1]), ld_rlx(&tR[k - 1]), ld_rlx(&tI[k - 1]));
    }
    if (p < k) {
        int32_t last = cnt < k ? cnt : k - 1;
        for (int32_t q = last; q > p; q--) {
            st_rlx(&tS[q], ld_rlx(&tS[q - 1]));
            st_rlx(&tR[q], ld_rlx(&tR[q - 1]));
            st_rlx(&tI[q], ld_rlx(&tI[q - 1]));
        }
        st_rlx(&tS[p], S); st_rlx(&tR[p], r); st_rlx(&tI[p], id);
        if (cnt < k) { cnt++; st_rlx(&st->cnt, cnt); }
        if (cnt == k) {
            int64_t s = ld_rlx(&st->seq) + 1;
            XRec* rc = ring + (s % TKC_XRING);
            st_rlx(&rc->S, ld_rlx(&tS[k - 1]));
            st_rlx(&rc->r, ld_rlx(&tR[k - 1]));
            st_rlx(&rc->id, st->ties ? (int64_t)0x7fffffff : (int64_t)ld_rlx(&tI[k - 1]));
            st_rel(&st->seq, s);
        }
    }
    fadd_rlx(&st->n_inserts, (int64_t)1);
    __hip_atomic_store(&st->lock, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------- BFSCut bound (Sect. 6)
// After levels 0..D are fully known (nD vertices, distance sum SD) and U
// bounds the size of level D+1, the least S(v) consistent with r(v) = r is
//   S_D + (D+1) rem + max(0, rem - U),   rem = r - nD
// (Lemma 6.1 tightened: every unseen vertex sits at distance >= D+1 and at
// most U of them at D+1).  With only alpha <= r <= omega known (Sect. 8.2)
// the farness bound is minimised over r in [a', o'] with a' = max(alpha, nD),
// o' = max(omega, a'); as a function of r the bound is convex piecewise
// linear with one kink at r = nD + U, so the ends and the clamped kink are
// the only candidates (Lemma 8.1).  Returns the bound as num/den.
TKC_DEV void cut_bound(int64_t SD, int64_t nD, int64_t U, int64_t D, int64_t alpha, int64_t omega,
                       int64_t* bnum, int64_t* bden) {
    int64_t a1 = alpha > nD ? alpha : nD;
    int64_t o1 = omega > a1 ? omega : a1;
    int64_t kink = nD + U;
    kink = kink < a1 ? a1 : (kink > o1 ? o1 : kink);
    int64_t cand[3] = {a1, o1, kink};
    int64_t bn = 0, bd = 0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        int64_t r = cand[c];
        if (r <= 1) continue;
        int64_t rem = r - nD;
        int64_t extra = rem - U;
        int64_t s = SD + (D + 1) * rem + (extra > 0 ? extra : 0);
        int64_t d = sq64(r - 1);
        if (bd == 0 || rat_cmp(s, d, bn, bd) < 0) { bn = s; bd = d; }
    }
    *bnum = bn;
    *bden = bd;
}

// ------------------------------------------- harmonic centrality (Sect. 2)
// h(v) = sum of 1/d(v,w) over the vertices v reaches, evaluated in binary64
// as the terms n_d / d added in increasing d.  Larger is better, so the
// engines, the top k and the order keys carry it as the farness-like
// integer F = HARM_TOP - bits(h) with denominator 1: the bit pattern of a
// non-negative double grows with its value, so F orders vertices exactly as
// h does, reversed, and every (value, id) comparison above applies as is.
#define HARM_TOP ((int64_t)0x7FF0000000000000LL)
TKC_DEV int64_t harm_enc(double h) { return HARM_TOP - (int64_t)__double_as_longlong(h); }
// Relative margin on every upper bound: covers the rounding of the bound's
// own binary64 terms and that of the final value (ecc terms, far below it).
#define HARM_MARGIN 1e-9
// BFSCut bound for harmonic centrality: after levels 0..D (nD vertices,
// partial value H) with at most U vertices at level D+1 and at most omega
// reachable, h(v) <= H + a/(D+1) + b/(D+2), a = min(U, rem), b = rem - a,
// rem = omega - nD: the unseen vertices placed as close as allowed.
TKC_DEV void harm_cut_bound(double H, int64_t nD, int64_t U, int64_t D, int64_t omega, int64_t* bnum,
                            int64_t* bden) {
    const int64_t rem = omega > nD ? omega - nD : 0;
    const int64_t a = U < rem ? U : rem;
    const double ub = H + (double)a / (double)(D + 1) + (double)(rem - a) / (double)(D + 2);
    *bnum = harm_enc(ub * (1.0 + HARM_MARGIN));
    *bden = 1;
}

// key of a lower bound for the processing order: the top 32 bits of the
// IEEE double num/den (monotone in the value; +inf sorts last).  Its value
// read back never exceeds the true bound by more than the double rounding.
TKC_DEV uint32_t order_key(int64_t num, int64_t den) {
    if (den == 0) return 0xffffffffu;
    double d = (double)num / (double)den;
    uint64_t b = (uint64_t)__double_as_longlong(d);
    return (uint32_t)(b >> 32);
}
TKC_DEV double key_value(uint32_t key) {
    if (key == 0xffffffffu) return __builtin_inf();
    return __longlong_as_double((long long)((uint64_t)key << 32));
}
// Stop test of Alg. 1 on a key: every vertex at or after this key position
// has a bound strictly above x (1e-9 relative margin covers the two double
// roundings of the key and of x).
TKC_DEV bool key_stops(uint32_t key, XVal x) {
    if (x.den == 0) return false;
    double kv = key_value(key);
    if (kv == __builtin_inf()) return true;
    double xv = (double)x.num / (double)x.den;
    return kv > xv * (1.0 + 1e-9);
}
// Harmonic order keys: the complement of the top 32 bits of the (margined)
// upper bound's bit pattern, so ascending keys run from the largest bound
// down at 2^-20 relative resolution.
TKC_DEV uint32_t harm_key(double ub) {
    return ~(uint32_t)((uint64_t)__double_as_longlong(ub) >> 32);
}
// Stop test on a harmonic key: the largest bound the key can stand for
// (the top of its bucket) is already below x, and so is every later one.
TKC_DEV bool key_stops_h(uint32_t key, XVal x) {
    if (x.den == 0) return false;
    const uint64_t top = ((uint64_t)(uint32_t)(~key) + 1) << 32;
    const double ub_hi = __longlong_as_double((long long)top);
    const double xh = __longlong_as_double((long long)(HARM_TOP - x.num));
    return ub_hi < xh;
}
