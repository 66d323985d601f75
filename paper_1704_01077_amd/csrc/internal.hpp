// Library-private host structures: context, device graph, query workspace.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/tkc.h"
#include "engine.hpp"

struct WsShape {
    int32_t n = 0, W = 64, nw = 1, kcap = 1, lcap = 0, qcap = 0, swarm_blocks = 0, nchunks = 0;
    bool lb = false;
    bool ties = false;   // all-ties buffers
    bool covers(const WsShape& o) const {
        return n >= o.n && nw >= o.nw && W >= o.W && kcap >= o.kcap && lcap >= o.lcap && qcap >= o.qcap &&
               swarm_blocks >= o.swarm_blocks && nchunks >= o.nchunks && (lb || !o.lb) && (ties || !o.ties);
    }
};

// Every device buffer one query may touch; one allocation, grown on demand.
struct Workspace {
    char* base = nullptr;
    size_t bytes = 0;
    // pinned host copy of the span from `stats` to the end of `tI` (the
    // query's results and counters, read back with one copy)
    char* pin = nullptr;
    size_t pin_bytes = 0;
    WsShape shape;
    int64_t *alpha, *omega;
    int32_t* scc;
    int64_t *lnum, *lden;
    uint32_t *key, *tkey;
    int32_t *ord, *tval;
    int32_t* hist;
    void* mask;
    int32_t* parent;
    int64_t* csize;
    int64_t *gbuf, *nbsum, *nbvis;
    double* nbhub;
    uint64_t* nbpart;
    uint8_t* nbflags;
    void* small;
    void* tstate;
    void* ring;
    int64_t *tS, *tR;
    int32_t* tI;
    int64_t *tieS, *tieR;
    int32_t* tieI;
    int64_t* stats;
    uint32_t* bar;
    // plain engine
    uint32_t *p_vis, *p_fb;
    int32_t *p_ql, *p_qh, *p_qg, *p_lvl;
    int64_t *p_ctr, *p_levcnt, *p_levtab;
    // batched engine
    uint64_t *b_vis, *b_frt0, *b_frt1, *b_nxt;
    int32_t *b_list, *b_mark, *b_cand;
    int64_t *b_ctr, *b_hist, *b_levtab, *b_outS, *b_outR;
    uint16_t* b_lvl;
    // per-workgroup engine
    uint32_t* s_vis;
    int32_t *s_queue, *s_deferred;
    int64_t* trace = nullptr;   // optional level trace (separate allocation)
};

struct tkc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    EngineTuning tune;
    Workspace ws;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // query phase marks on the stream: start, reachability done, bounds and
    // top-k set-up done, searches done (phase times without host waits)
    hipEvent_t evq[4] = {nullptr, nullptr, nullptr, nullptr};
    // between two launches timed as one span (the seed batch and the swarm)
    hipEvent_t evm = nullptr;
    void* pinned = nullptr;   // 4 KiB of pinned host memory for small readbacks
};

struct tkc_graph {
    tkc_ctx* ctx = nullptr;
    int32_t n = 0;
    int64_t m = 0;
    bool directed = false;
    void* dbase = nullptr;
    int32_t *rp = nullptr, *ci = nullptr, *rrp = nullptr, *rci = nullptr;
    int32_t* deg = nullptr;
    int32_t* heavy = nullptr;
    int32_t nheavy = 0;
    int32_t *hcb = nullptr, *ch_beg = nullptr, *ch_end = nullptr, *ch_vtx = nullptr;
    int32_t *rch_beg = nullptr, *rch_end = nullptr, *rch_vtx = nullptr;
    int32_t nchunks = 0, rnchunks = 0;
    int32_t *bch_beg = nullptr, *bch_end = nullptr, *bch_vtx = nullptr;
    int32_t bnchunks = 0;
    int32_t *mid_vtx = nullptr, *mseg = nullptr;
    int32_t nmseg = 0;
    // TKC_RELABEL: vertex v is the caller's vertex oid[v]; nid is the inverse
    bool relabeled = false;
    int32_t *d_oid = nullptr, *d_nid = nullptr;
    std::vector<int32_t> h_nid;
    int32_t server_refs = 0;
    std::atomic<int32_t> auto_variant{0};   // read by server workers without the graph lock
    // reachability bounds of a directed graph, computed once per graph:
    // alpha, omega (n int64 each) and topological SCC ids (n int32)
    void* reach_base = nullptr;
    int64_t *d_alpha = nullptr, *d_omega = nullptr;
    int32_t* d_scc = nullptr;
    int32_t reach_path = 0;     // 0 not yet, 1 parallel steps, 2 a one-thread pass finished chains
    double reach_ms = 0;        // time of that computation
    std::mutex mu;
    // cached preprocessing (serving): [0] Deg, [1] NB
    struct Prep {
        void* base = nullptr;
        int32_t rounds = 0;
        bool ready = false;
    } prep[2];
    bool cache_prep = false;
    // autotuned knobs (TKC_MODE_AUTO)
    bool tuned = false;
    EngineTuning tune;
    DevGraph view() const {
        DevGraph g;
        g.n = n; g.m = m; g.directed = directed;
        g.rp = rp; g.ci = ci; g.rrp = rrp; g.rci = rci; g.deg = deg;
        g.heavy = heavy; g.nheavy = nheavy; g.hcb = hcb; g.ch_beg = ch_beg; g.ch_end = ch_end; g.ch_vtx = ch_vtx;
        g.nchunks = nchunks;
        g.rch_vtx = rch_vtx; g.rch_beg = rch_beg; g.rch_end = rch_end; g.rnchunks = rnchunks;
        g.bch_vtx = bch_vtx; g.bch_beg = bch_beg; g.bch_end = bch_end; g.bnchunks = bnchunks;
        g.mid_vtx = mid_vtx; g.mseg = mseg; g.nmseg = nmseg;
        g.oid = relabeled ? d_oid : nullptr;
        g.nid = relabeled ? d_nid : nullptr;
        return g;
    }
};

int tkc_fail(int code, const char* fmt, ...);
// milliseconds on the host's steady clock
double tkc_now_ms();
// the batched engine's buffers in a workspace
BatchWork tkc_batch_view(Workspace& ws);

// A pack: the disjoint union of member graphs, whose top-k requests share the
// lanes of one batched launch (pack.cpp)
struct tkc_pack {
    tkc_ctx* ctx = nullptr;
    std::vector<tkc_graph*> members;
    std::vector<int32_t> off;   // union id of each member's vertex 0
    tkc_graph* ug = nullptr;    // the union graph
    void* dev = nullptr;        // per-request top-k states and the request table
    size_t dev_bytes = 0;
    std::mutex mu;              // one packed call at a time
};
// tkc_pack_topk on context c's stream and workspace (the server's slots)
int tkc_pack_topk_on(tkc_ctx* c, tkc_pack* p, int32_t nreq, const int32_t* member, const int32_t* k,
                     int32_t variant, int32_t* ids, int64_t* sum_dist, int64_t* reach, double* farness,
                     int32_t* n_out, tkc_stats* stats);

// noalloc.hip: the per-device address of the no-allocation scratch array
int tkc_noalloc_init(int device);
// level-based updates of a variant: 0 none (Cut), 1 only (Bound), 2 with cuts
static inline int tkc_lb_level(int32_t variant) {
    if (variant == TKC_DEG_BOUND || variant == TKC_NB_BOUND) return 1;
    if (variant == TKC_DEG_CUTLB || variant == TKC_NB_CUTLB) return 2;
    return 0;
}
static inline bool tkc_is_nb(int32_t variant) {
    return variant == TKC_NB_CUT || variant == TKC_NB_BOUND || variant == TKC_NB_CUTLB;
}
int tkc_ws_reserve(tkc_ctx* ctx, Workspace& ws, const WsShape& sh);
// ties_cap > 0: all-ties mode, output arrays of ties_cap entries
// harm: harmonic centrality; farness then receives the values h
int tkc_run_query(tkc_ctx* c, tkc_graph* g, int32_t k, int32_t variant, int32_t mode, int32_t* ids,
                  int64_t* sum_dist, int64_t* reach, double* farness, int32_t* n_out, tkc_stats* stats,
                  int32_t ties_cap = 0, bool harm = false, int64_t max_searches = 0);
int tkc_sums_impl(tkc_ctx* c, tkc_graph* g, const int32_t* sources, int32_t count, int64_t* S, int64_t* R,
                  tkc_stats* st);
int32_t tkc_auto_variant(tkc_ctx* c, tkc_graph* g);
int tkc_step_reach(tkc_ctx* c, tkc_graph* g, Workspace& ws);
int tkc_step_bounds(tkc_ctx* c, tkc_graph* g, Workspace& ws, bool nb, int32_t* rounds, bool harm = false);
// copy a graph's cached reachability/bounds/order into c's workspace; false
// when the graph has no cache for this bound kind
bool tkc_prep_cached(tkc_ctx* c, tkc_graph* g, bool nb, int32_t* rounds);
// build that cache from c's workspace after a query computed it
int tkc_prep_store(tkc_ctx* c, tkc_graph* g, bool nb, int32_t rounds);
WsShape tkc_shape_for(const EngineTuning& t, tkc_graph* g, int32_t k, bool lb);
// the knobs a TKC_MODE_AUTO query on g runs with, given the context's own
EngineTuning tkc_effective_tuning(const EngineTuning& ctx_tune, tkc_graph* g);
size_t tkc_ws_bytes(const WsShape& sh);
// one cooperative kernel at a time on the device
std::mutex& tkc_coop_mutex();
