// Serving loop: graphs stay resident on the device and top-k requests are
// admitted as they arrive.  The server owns `max_inflight` slots; each slot
// is a worker thread with its own HIP stream and query workspace, so the
// device work of requests in different slots overlaps (continuous batching:
// a request that arrives while others run starts as soon as a slot and
// memory are free, it does not wait for the running ones to finish).
//   - Admission: a request needs its slot's workspace grown to the request's
//     shape; the sum of all slot workspaces must stay within the HBM budget.
//     A request that could never fit is refused at submission (TKC_EBUSY).
//   - Per-graph preprocessing (reachability, initial bounds, order) is
//     computed by the first request on a graph and reused by later ones.
//   - Cooperative (grid-barrier) kernels of different slots never overlap:
//     they take a process-wide lock, while ordinary kernels run freely.
//   - Packing (tkc_server_enable_packing): the small graphs are grouped into
//     packs (disjoint unions, pack.cpp).  A slot that takes a request on a
//     packed graph also takes the queued requests on the pack's other
//     members (distinct graphs, the same BFSCut variant) and serves them
//     all with one batched launch, so requests that arrived together share
//     the GPU's lanes instead of queuing for the cooperative lock one by one.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/tkc.h"
#include "internal.hpp"

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    int32_t graph_id = 0;
    int32_t k = 1;
    int32_t variant = TKC_AUTO;
    double t_submit = 0, t_done = 0;
    int state = 0;          // 0 queued, 1 running, 2 done
    bool cancelled = false;
    int status = TKC_OK;
    std::string err;
    std::vector<int32_t> ids;
    std::vector<int64_t> S, R;
    std::vector<double> F;
    size_t need = 0;        // workspace bytes this request needs
};

}  // namespace

struct tkc_server {
    tkc_ctx* ctx = nullptr;
    size_t budget = 0;
    int32_t slots_n = 0;
    std::vector<tkc_graph*> graphs;
    std::vector<tkc_ctx*> slot_ctx;
    std::vector<size_t> slot_bytes;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1;
    bool stopping = false;
    // packing
    bool packing = false;
    std::vector<tkc_pack*> packs;
    std::vector<int32_t> pack_of, member_of;   // per graph id (-1: not packed)
    std::vector<size_t> pack_need;             // workspace bytes of a packed call
    int64_t n_served = 0, n_packed = 0, n_pack_calls = 0;

    // fills request rq's answer from a packed call's concatenated results
    static void take(Request& rq, const std::vector<int32_t>& ids, const std::vector<int64_t>& S,
                     const std::vector<int64_t>& R, const std::vector<double>& F, int32_t o, int32_t c) {
        rq.ids.assign(ids.begin() + o, ids.begin() + o + c);
        rq.S.assign(S.begin() + o, S.begin() + o + c);
        rq.R.assign(R.begin() + o, R.begin() + o + c);
        rq.F.assign(F.begin() + o, F.begin() + o + c);
    }

    size_t committed_except(int slot) {
        size_t t = 0;
        for (int i = 0; i < slots_n; i++)
            if (i != slot) t += slot_bytes[i];
        return t;
    }

    void worker(int slot) {
        tkc_ctx* c = slot_ctx[slot];
        hipSetDevice(c->device);
        for (;;) {
            std::shared_ptr<Request> rq;
            tkc_graph* g = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (stopping) return;
                    // first queued request whose workspace fits next to the others
                    for (auto it = queue.begin(); it != queue.end(); ++it) {
                        size_t need = std::max((*it)->need, slot_bytes[slot]);
                        if (committed_except(slot) + need <= budget) {
                            rq = *it;
                            queue.erase(it);
                            slot_bytes[slot] = need;
                            break;
                        }
                    }
                    if (rq) break;
                    if (!queue.empty() && slot_bytes[slot] > 0) {
                        // nothing fits next to the other slots: give this idle
                        // slot's workspace back so a waiting request can run
                        if (c->ws.base) {
                            hipStreamSynchronize(c->stream);
                            hipFree(c->ws.base);
                            c->ws.base = nullptr;
                            c->ws.bytes = 0;
                            c->ws.shape = WsShape();
                        }
                        slot_bytes[slot] = 0;
                        cv_work.notify_all();
                        continue;
                    }
                    cv_work.wait(lk);
                }
                rq->state = 1;
                // the graph table may grow while requests run
                // (tkc_server_add_graph): read it under the lock only
                g = graphs[rq->graph_id];
            }
            // packing: queued requests on the pack's other members join this one
            std::vector<std::shared_ptr<Request>> group;
            std::vector<int32_t> mem, ks;   // the group's members and k
            int32_t tot = 0;                // and its result count
            int32_t pk = -1, pv = 0;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (packing && !rq->cancelled) pk = pack_of[rq->graph_id];
            }
            if (pk >= 0) {
                pv = rq->variant == TKC_AUTO ? tkc_auto_variant(c, g) : rq->variant;
                if (pv != TKC_NB_CUT && pv != TKC_DEG_CUT) pk = -1;
            }
            if (pk >= 0) {
                std::lock_guard<std::mutex> lk(mu);
                const size_t need = std::max(slot_bytes[slot], pack_need[pk]);
                if (committed_except(slot) + need <= budget) {
                    slot_bytes[slot] = need;
                    group.push_back(rq);
                    std::vector<char> used(packs[pk]->members.size(), 0);
                    used[member_of[rq->graph_id]] = 1;
                    for (auto it = queue.begin(); it != queue.end() && group.size() < TKC_PACK_MAXREQ;) {
                        const std::shared_ptr<Request>& q = *it;
                        const int32_t gid = q->graph_id;
                        // an AUTO request joins once its graph's variant is known
                        const int32_t qv = q->variant == TKC_AUTO ? graphs[gid]->auto_variant.load() : q->variant;
                        if (pack_of[gid] == pk && !used[member_of[gid]] && qv == pv && !q->cancelled) {
                            used[member_of[gid]] = 1;
                            q->state = 1;
                            group.push_back(q);
                            it = queue.erase(it);
                        } else {
                            ++it;
                        }
                    }
                    for (const std::shared_ptr<Request>& q : group) {
                        mem.push_back(member_of[q->graph_id]);
                        ks.push_back(q->k);
                        tot += std::min(q->k, graphs[q->graph_id]->n);
                    }
                }
            }
            if (group.size() >= 2) {
                const int32_t nr = (int32_t)group.size();
                std::vector<int32_t> nout(nr);
                std::vector<int32_t> ids(tot);
                std::vector<int64_t> S(tot), R(tot);
                std::vector<double> F(tot);
                const int st = tkc_pack_topk_on(c, packs[pk], nr, mem.data(), ks.data(), pv, ids.data(), S.data(),
                                                R.data(), F.data(), nout.data(), nullptr);
                {
                    std::lock_guard<std::mutex> lk(mu);
                    int32_t o = 0;
                    for (int32_t i = 0; i < nr; i++) {
                        Request& q = *group[i];
                        if (st == TKC_OK) take(q, ids, S, R, F, o, nout[i]);
                        else q.err = tkc_last_error();
                        o += st == TKC_OK ? nout[i] : 0;
                        q.status = q.cancelled ? TKC_ECANCELED : st;
                        q.t_done = now_ms();
                        q.state = 2;
                    }
                    n_served += nr;
                    n_packed += nr;
                    n_pack_calls++;
                    slot_bytes[slot] = std::max(slot_bytes[slot], c->ws.bytes);
                }
                cv_done.notify_all();
                cv_work.notify_all();
                continue;
            }
            int32_t k = std::min(rq->k, g->n);
            rq->ids.resize(k);
            rq->S.resize(k);
            rq->R.resize(k);
            rq->F.resize(k);
            int32_t got = 0;
            int st = TKC_OK;
            bool skip;
            {
                std::lock_guard<std::mutex> lk(mu);
                skip = rq->cancelled;
            }
            if (!skip)
                st = tkc_run_query(c, g, k, rq->variant, TKC_MODE_AUTO, rq->ids.data(), rq->S.data(), rq->R.data(),
                                   rq->F.data(), &got, nullptr);
            {
                std::lock_guard<std::mutex> lk(mu);
                rq->status = rq->cancelled ? TKC_ECANCELED : st;
                if (st != TKC_OK) rq->err = tkc_last_error();
                rq->t_done = now_ms();
                rq->state = 2;
                slot_bytes[slot] = c->ws.bytes;
                n_served++;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

extern "C" int tkc_server_create(tkc_ctx* ctx, size_t hbm_budget_bytes, int32_t max_inflight, tkc_server** out) {
    if (!ctx || !out) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (max_inflight < 1 || max_inflight > 64) return tkc_fail(TKC_EINVAL, "max_inflight must be in [1, 64]");
    if (hbm_budget_bytes == 0) return tkc_fail(TKC_EINVAL, "hbm budget must be > 0");
    tkc_server* s = new tkc_server();
    s->ctx = ctx;
    s->budget = hbm_budget_bytes;
    s->slots_n = max_inflight;
    for (int i = 0; i < max_inflight; i++) {
        tkc_ctx* c = nullptr;
        int rc = tkc_ctx_create(ctx->device, nullptr, &c);
        if (rc) {
            for (auto* cc : s->slot_ctx) tkc_ctx_destroy(cc);
            delete s;
            return rc;
        }
        c->tune = ctx->tune;
        // long batched queries run a few batches per launch, so requests in
        // other slots interleave instead of waiting for the whole query
        c->tune.slice_batches = 2;
        s->slot_ctx.push_back(c);
        s->slot_bytes.push_back(0);
    }
    for (int i = 0; i < max_inflight; i++) s->workers.emplace_back(&tkc_server::worker, s, i);
    *out = s;
    return TKC_OK;
}

extern "C" int tkc_server_add_graph(tkc_server* s, tkc_graph* g, int32_t* graph_id) {
    if (!s || !g || !graph_id) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (g->ctx->device != s->ctx->device) return tkc_fail(TKC_EINVAL, "graph lives on another device");
    std::lock_guard<std::mutex> lk(s->mu);
    {
        std::lock_guard<std::mutex> gl(g->mu);
        g->server_refs++;
        g->cache_prep = true;
    }
    s->graphs.push_back(g);
    *graph_id = (int32_t)s->graphs.size() - 1;
    return TKC_OK;
}

extern "C" int tkc_server_submit(tkc_server* s, int32_t graph_id, int32_t k, int32_t variant, uint64_t* ticket) {
    if (!s || !ticket) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (k < 1) return tkc_fail(TKC_EINVAL, "k must be >= 1");
    if (variant < TKC_AUTO || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "unknown variant");
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return tkc_fail(TKC_EINVAL, "unknown graph id");
    tkc_graph* g = s->graphs[graph_id];
    auto rq = std::make_shared<Request>();
    rq->ticket = s->next_ticket++;
    rq->graph_id = graph_id;
    rq->k = k;
    rq->variant = variant;
    rq->t_submit = now_ms();
    bool lb = tkc_lb_level(variant) != 0 || variant == TKC_AUTO;
    rq->need = tkc_ws_bytes(tkc_shape_for(tkc_effective_tuning(s->ctx->tune, g), g, std::min(k, g->n), lb));
    if (rq->need > s->budget) return tkc_fail(TKC_EBUSY, "request needs %zu bytes, budget is %zu", rq->need, s->budget);
    s->queue.push_back(rq);
    s->all[rq->ticket] = rq;
    *ticket = rq->ticket;
    s->cv_work.notify_all();
    return TKC_OK;
}

extern "C" int tkc_server_poll(tkc_server* s, uint64_t ticket, int32_t* done) {
    if (!s || !done) return tkc_fail(TKC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return tkc_fail(TKC_EINVAL, "unknown ticket");
    *done = it->second->state == 2 ? 1 : 0;
    return TKC_OK;
}

extern "C" int tkc_server_result(tkc_server* s, uint64_t ticket, int32_t* ids, int64_t* sum_dist, int64_t* reach,
                                 double* farness, int32_t* n_out, double* latency_ms) {
    if (!s || !ids || !n_out) return tkc_fail(TKC_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return tkc_fail(TKC_EINVAL, "unknown ticket");
    std::shared_ptr<Request> rq = it->second;
    s->cv_done.wait(lk, [&] { return rq->state == 2; });
    s->all.erase(it);
    if (rq->status != TKC_OK) {
        if (rq->status == TKC_ECANCELED) return tkc_fail(TKC_ECANCELED, "request cancelled");
        return tkc_fail(rq->status, "%s", rq->err.c_str());
    }
    int32_t c = (int32_t)rq->ids.size();
    memcpy(ids, rq->ids.data(), 4 * (size_t)c);
    if (sum_dist) memcpy(sum_dist, rq->S.data(), 8 * (size_t)c);
    if (reach) memcpy(reach, rq->R.data(), 8 * (size_t)c);
    if (farness) memcpy(farness, rq->F.data(), 8 * (size_t)c);
    *n_out = c;
    if (latency_ms) *latency_ms = rq->t_done - rq->t_submit;
    return TKC_OK;
}

extern "C" int tkc_server_cancel(tkc_server* s, uint64_t ticket) {
    if (!s) return tkc_fail(TKC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return tkc_fail(TKC_EINVAL, "unknown ticket");
    std::shared_ptr<Request> rq = it->second;
    rq->cancelled = true;
    if (rq->state == 0) {
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (*q == rq) { s->queue.erase(q); break; }
        rq->state = 2;
        rq->status = TKC_ECANCELED;
        rq->t_done = now_ms();
        s->cv_done.notify_all();
    }
    return TKC_OK;
}

extern "C" int tkc_server_enable_packing(tkc_server* s, int32_t max_vertices) {
    if (!s) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (max_vertices < 0) return tkc_fail(TKC_EINVAL, "max_vertices must be >= 0");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->queue.empty()) return tkc_fail(TKC_EBUSY, "requests are queued");
    for (auto& kv : s->all)
        if (kv.second->state == 1) return tkc_fail(TKC_EBUSY, "requests are running");
    s->packing = false;
    for (tkc_pack* p : s->packs) tkc_pack_free(p);
    s->packs.clear();
    s->pack_need.clear();
    const int32_t ng = (int32_t)s->graphs.size();
    s->pack_of.assign(ng, -1);
    s->member_of.assign(ng, -1);
    if (max_vertices == 0) return TKC_OK;
    // members of at most max_vertices vertices, one kind of graph per pack,
    // up to TKC_PACK_MAXREQ members and 2^28 arcs per union
    for (int dir = 0; dir < 2; dir++) {
        std::vector<int32_t> cur;
        int64_t arcs = 0;
        auto flush = [&]() -> int {
            if (cur.size() >= 2) {
                std::vector<tkc_graph*> mg;
                for (int32_t gid : cur) mg.push_back(s->graphs[gid]);
                tkc_pack* p = nullptr;
                int rc = tkc_pack_create(s->ctx, mg.data(), (int32_t)mg.size(), &p);
                if (rc) return rc;
                const int32_t pi = (int32_t)s->packs.size();
                s->packs.push_back(p);
                s->pack_need.push_back(tkc_ws_bytes(tkc_shape_for(s->ctx->tune, p->ug, 1024, false)));
                for (int32_t i = 0; i < (int32_t)cur.size(); i++) {
                    s->pack_of[cur[i]] = pi;
                    s->member_of[cur[i]] = i;
                }
            }
            cur.clear();
            arcs = 0;
            return TKC_OK;
        };
        for (int32_t gid = 0; gid < ng; gid++) {
            tkc_graph* g = s->graphs[gid];
            if (g->directed != (dir == 1) || g->n > max_vertices || g->relabeled) continue;
            if ((int32_t)cur.size() == TKC_PACK_MAXREQ || arcs + g->m > (int64_t(1) << 28))
                if (int rc = flush()) return rc;
            cur.push_back(gid);
            arcs += g->m;
        }
        if (int rc = flush()) return rc;
    }
    s->packing = !s->packs.empty();
    return TKC_OK;
}

extern "C" int tkc_server_info(tkc_server* s, int64_t* served, int64_t* packed, int64_t* pack_calls,
                               int32_t* packs) {
    if (!s) return tkc_fail(TKC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (served) *served = s->n_served;
    if (packed) *packed = s->n_packed;
    if (pack_calls) *pack_calls = s->n_pack_calls;
    if (packs) *packs = (int32_t)s->packs.size();
    return TKC_OK;
}

extern "C" int tkc_server_destroy(tkc_server* s) {
    if (!s) return TKC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (tkc_pack* p : s->packs) tkc_pack_free(p);
    s->packs.clear();
    for (auto* c : s->slot_ctx) tkc_ctx_destroy(c);
    for (auto* g : s->graphs) {
        std::lock_guard<std::mutex> gl(g->mu);
        g->server_refs--;
    }
    delete s;
    return TKC_OK;
}
