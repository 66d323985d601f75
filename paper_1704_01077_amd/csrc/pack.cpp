// Packed queries: top-k requests on several graphs in one batched launch.
//
// A pack is the disjoint union of member graphs (the same context, all
// directed or all undirected), member i's vertices renumbered by adding
// off[i].  No arc joins two members, so a batch whose lanes start in
// different members is still one multi-source search of the union: each
// lane stays inside its own member.  The requests of a packed call share
// the batches' lanes; each lane carries its request's processing order,
// initial bounds, reachability and top k (its own member's, from the
// member's cached preprocessing), and compares with its request's current
// k-th farness (Alg. 1 and BFSCut, Sect. 6, per request).  Every answer is
// the one a query on the member alone returns.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/tkc.h"
#include "dev_common.hpp"
#include "engine.hpp"
#include "internal.hpp"

#define PCHK(call)                                                                    \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return tkc_fail(TKC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace {
size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }
// per request in the pack's device buffer: top-k state, x ring, S, R, ids
size_t req_bytes(int32_t kcap) {
    return up256(sizeof(TopkState)) + up256(sizeof(XRec) * TKC_XRING) + up256(8 * (size_t)kcap) * 2 +
           up256(4 * (size_t)kcap);
}
}  // namespace

extern "C" int tkc_pack_create(tkc_ctx* ctx, tkc_graph* const* graphs, int32_t count, tkc_pack** out) {
    if (!ctx || !graphs || !out) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (count < 1) return tkc_fail(TKC_EINVAL, "a pack needs at least one graph");
    const bool directed = graphs[0] && graphs[0]->directed;
    int64_t N = 0, M = 0;
    for (int32_t i = 0; i < count; i++) {
        tkc_graph* g = graphs[i];
        if (!g) return tkc_fail(TKC_EINVAL, "graph %d is NULL", i);
        if (g->ctx != ctx) return tkc_fail(TKC_EINVAL, "graph %d belongs to another context", i);
        if (g->directed != directed) return tkc_fail(TKC_EINVAL, "members must be all directed or all undirected");
        if (g->relabeled) return tkc_fail(TKC_EINVAL, "graph %d was uploaded with TKC_RELABEL", i);
        for (int32_t j = 0; j < i; j++)
            if (graphs[j] == g) return tkc_fail(TKC_EINVAL, "graph %d is listed twice", i);
        N += g->n;
        M += g->m;
    }
    if (N > 0x7fffffffLL - 1 || M > 0x7fffffffLL - 1)
        return tkc_fail(TKC_EINVAL, "the union of the members exceeds int32 vertex or arc ids");
    PCHK(hipSetDevice(ctx->device));
    PCHK(hipStreamSynchronize(ctx->stream));
    // the union CSR, on the host, from the members' device copies
    std::vector<int32_t> rp((size_t)N + 1), ci((size_t)M), rrp, rci;
    if (directed) {
        rrp.resize((size_t)N + 1);
        rci.resize((size_t)M);
    }
    std::vector<int32_t> off(count);
    int64_t vo = 0, ao = 0;
    std::vector<int32_t> tmp;
    for (int32_t i = 0; i < count; i++) {
        tkc_graph* g = graphs[i];
        off[i] = (int32_t)vo;
        for (int dir = 0; dir < (directed ? 2 : 1); dir++) {
            const int32_t* drp = dir ? g->rrp : g->rp;
            const int32_t* dci = dir ? g->rci : g->ci;
            std::vector<int32_t>& urp = dir ? rrp : rp;
            std::vector<int32_t>& uci = dir ? rci : ci;
            tmp.resize((size_t)g->n + 1);
            PCHK(hipMemcpy(tmp.data(), drp, 4 * ((size_t)g->n + 1), hipMemcpyDeviceToHost));
            for (int32_t v = 0; v < g->n; v++) urp[(size_t)(vo + v)] = (int32_t)(ao + tmp[v]);
            if (g->m) PCHK(hipMemcpy(uci.data() + ao, dci, 4 * (size_t)g->m, hipMemcpyDeviceToHost));
            for (int64_t e = 0; e < g->m; e++) uci[(size_t)(ao + e)] += (int32_t)vo;
        }
        vo += g->n;
        ao += g->m;
    }
    rp[(size_t)N] = (int32_t)M;
    if (directed) rrp[(size_t)N] = (int32_t)M;
    tkc_graph* ug = nullptr;
    int rc = tkc_graph_upload(ctx, (int32_t)N, M, rp.data(), ci.data(), directed ? rrp.data() : nullptr,
                              directed ? rci.data() : nullptr, directed ? TKC_DIRECTED : 0u, &ug);
    if (rc) return rc;
    tkc_pack* p = new tkc_pack();
    p->ctx = ctx;
    p->members.assign(graphs, graphs + count);
    p->off = off;
    p->ug = ug;
    for (tkc_graph* g : p->members) {
        std::lock_guard<std::mutex> lk(g->mu);
        g->server_refs++;      // held: tkc_graph_free returns TKC_EBUSY meanwhile
        g->cache_prep = true;  // requests read the members' cached bounds and order
    }
    *out = p;
    return TKC_OK;
}

extern "C" int tkc_pack_free(tkc_pack* p) {
    if (!p) return TKC_OK;
    hipSetDevice(p->ctx->device);
    hipStreamSynchronize(p->ctx->stream);
    for (tkc_graph* g : p->members) {
        std::lock_guard<std::mutex> lk(g->mu);
        g->server_refs--;
    }
    tkc_graph_free(p->ug);
    if (p->dev) hipFree(p->dev);
    delete p;
    return TKC_OK;
}

// the member's reachability, bounds and order in its preprocessing cache
static int ensure_prep(tkc_ctx* c, tkc_graph* g, bool nb) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->prep[nb ? 1 : 0].ready) return TKC_OK;
    }
    int rc = tkc_ws_reserve(c, c->ws, tkc_shape_for(c->tune, g, 1, false));
    if (rc) return rc;
    if ((rc = tkc_step_reach(c, g, c->ws))) return rc;
    int32_t rounds = 0;
    if ((rc = tkc_step_bounds(c, g, c->ws, nb, &rounds, false))) return rc;
    if ((rc = tkc_prep_store(c, g, nb, rounds))) return rc;
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->prep[nb ? 1 : 0].ready) return tkc_fail(TKC_ENOMEM, "no device memory for a member's preprocessing");
    return TKC_OK;
}

extern "C" int tkc_pack_topk(tkc_pack* p, int32_t nreq, const int32_t* member, const int32_t* k, int32_t variant,
                             int32_t* ids, int64_t* sum_dist, int64_t* reach, double* farness, int32_t* n_out,
                             tkc_stats* stats) {
    if (!p) return tkc_fail(TKC_EINVAL, "NULL argument");
    return tkc_pack_topk_on(p->ctx, p, nreq, member, k, variant, ids, sum_dist, reach, farness, n_out, stats);
}

int tkc_pack_topk_on(tkc_ctx* c, tkc_pack* p, int32_t nreq, const int32_t* member, const int32_t* k,
                     int32_t variant, int32_t* ids, int64_t* sum_dist, int64_t* reach, double* farness,
                     int32_t* n_out, tkc_stats* stats) {
    if (!c || !p || !member || !k || !ids || !n_out) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (c->device != p->ctx->device) return tkc_fail(TKC_EINVAL, "the context lives on another device");
    if (nreq < 1 || nreq > TKC_PACK_MAXREQ)
        return tkc_fail(TKC_EINVAL, "a packed call takes 1 to %d requests", TKC_PACK_MAXREQ);
    if (variant == TKC_AUTO) variant = TKC_NB_CUT;
    if (variant != TKC_NB_CUT && variant != TKC_DEG_CUT)
        return tkc_fail(TKC_EINVAL, "packed requests run the BFSCut variants (TKC_NB_CUT, TKC_DEG_CUT)");
    const int32_t nm = (int32_t)p->members.size();
    int32_t kmax = 1;
    for (int32_t r = 0; r < nreq; r++) {
        if (member[r] < 0 || member[r] >= nm) return tkc_fail(TKC_EINVAL, "request %d: no member %d", r, member[r]);
        if (k[r] < 1) return tkc_fail(TKC_EINVAL, "request %d: k must be >= 1", r);
        for (int32_t q = 0; q < r; q++)
            if (member[q] == member[r])
                return tkc_fail(TKC_EINVAL, "requests %d and %d name the same member (its searches would share "
                                            "the member's vertices)", q, r);
        kmax = std::max(kmax, std::min(k[r], p->members[member[r]]->n));
    }
    PCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const bool nb = variant == TKC_NB_CUT;
    // one packed call at a time per pack: its request states are shared
    std::lock_guard<std::mutex> plk(p->mu);
    const double t0 = tkc_now_ms();
    int rc;
    for (int32_t r = 0; r < nreq; r++)
        if ((rc = ensure_prep(c, p->members[member[r]], nb))) return rc;
    // the union graph's batched-engine buffers
    if ((rc = tkc_ws_reserve(c, c->ws, tkc_shape_for(c->tune, p->ug, kmax, false)))) return rc;
    // per-request top-k states and the request table
    const size_t per = req_bytes(kmax);
    const size_t need = per * (size_t)nreq + up256(sizeof(PackReq) * (size_t)nreq);
    if (p->dev_bytes < need) {
        PCHK(hipDeviceSynchronize());
        if (p->dev) hipFree(p->dev);
        p->dev = nullptr;
        p->dev_bytes = 0;
        if (hipMalloc(&p->dev, need) != hipSuccess) {
            hipGetLastError();
            return tkc_fail(TKC_ENOMEM, "device allocation of %zu bytes failed", need);
        }
        p->dev_bytes = need;
    }
    std::vector<PackReq> tab(nreq);
    std::vector<int32_t> kk(nreq);
    for (int32_t r = 0; r < nreq; r++) {
        tkc_graph* g = p->members[member[r]];
        kk[r] = std::min(k[r], g->n);
        char* b = (char*)p->dev + per * (size_t)r;
        DevTopk tk;
        tk.st = (TopkState*)b;
        b += up256(sizeof(TopkState));
        tk.ring = (XRec*)b;
        b += up256(sizeof(XRec) * TKC_XRING);
        tk.S = (int64_t*)b;
        b += up256(8 * (size_t)kmax);
        tk.R = (int64_t*)b;
        b += up256(8 * (size_t)kmax);
        tk.I = (int32_t*)b;
        if (tkc_launch_topk_init(tk, kk[r], s)) return tkc_fail(TKC_EDEVICE, "top-k init failed");
        // the member's cached preprocessing: alpha, omega, num, den, order, keys
        const size_t n = (size_t)g->n;
        char* pb = (char*)g->prep[nb ? 1 : 0].base;
        PackReq q{};
        q.off = p->off[member[r]];
        q.n = g->n;
        q.rc = DevReach{(const int64_t*)pb, (const int64_t*)(pb + 8 * n), nullptr};
        q.bv.num = (int64_t*)(pb + 16 * n);
        q.bv.den = (int64_t*)(pb + 24 * n);
        q.bv.harm = 0;
        q.ov = OrderView{(const int32_t*)(pb + 32 * n), (const uint32_t*)(pb + 36 * n), g->n, nb};
        q.tk = tk;
        tab[r] = q;
    }
    PackReq* dtab = (PackReq*)((char*)p->dev + per * (size_t)nreq);
    PCHK(hipMemcpyAsync(dtab, tab.data(), sizeof(PackReq) * (size_t)nreq, hipMemcpyHostToDevice, s));
    int64_t* st_dev = c->ws.stats;
    PCHK(hipMemsetAsync(st_dev, 0, 8 * ST_COUNT, s));
    DevGraph dg = p->ug->view();
    const DevReach rc0{nullptr, nullptr, nullptr};
    const OrderView ov0{nullptr, nullptr, 0, false};
    const BoundsView bv0{nullptr, nullptr};
    const DevTopk tk0{nullptr, nullptr, nullptr, nullptr, nullptr};
    double ms_launch = 0;
    {
        std::lock_guard<std::mutex> lk(tkc_coop_mutex());
        PCHK(hipEventRecord(c->ev0, s));
        int grid = 0;
        if (tkc_launch_batch(dg, rc0, ov0, bv0, tk0, tkc_batch_view(c->ws), st_dev, nullptr, 0, 0, 0, 0, false,
                             nullptr, nullptr, c->tune, s, &grid, dtab, nreq))
            return tkc_fail(TKC_EDEVICE, "packed batched launch failed: %s", hipGetErrorString(hipGetLastError()));
        PCHK(hipEventRecord(c->ev1, s));
        PCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        PCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        ms_launch = ms;
    }
    // results, request by request
    int32_t o = 0;
    std::vector<int64_t> hS(kmax), hR(kmax);
    std::vector<int32_t> hI(kmax);
    for (int32_t r = 0; r < nreq; r++) {
        tkc_graph* g = p->members[member[r]];
        TopkState hst;
        PCHK(hipMemcpy(&hst, tab[r].tk.st, sizeof(TopkState), hipMemcpyDeviceToHost));
        if (hst.cnt < kk[r]) return tkc_fail(TKC_EDEVICE, "internal error: request %d has %d of %d results", r,
                                             hst.cnt, kk[r]);
        PCHK(hipMemcpy(hS.data(), tab[r].tk.S, 8 * (size_t)kk[r], hipMemcpyDeviceToHost));
        PCHK(hipMemcpy(hR.data(), tab[r].tk.R, 8 * (size_t)kk[r], hipMemcpyDeviceToHost));
        PCHK(hipMemcpy(hI.data(), tab[r].tk.I, 4 * (size_t)kk[r], hipMemcpyDeviceToHost));
        for (int32_t i = 0; i < kk[r]; i++) {
            ids[o + i] = hI[i];
            if (sum_dist) sum_dist[o + i] = hS[i];
            if (reach) reach[o + i] = hR[i];
            if (farness)
                farness[o + i] = hR[i] <= 1 ? INFINITY
                                            : ((double)(g->n - 1) * (double)hS[i]) /
                                                  ((double)(hR[i] - 1) * (double)(hR[i] - 1));
        }
        n_out[r] = kk[r];
        o += kk[r];
    }
    if (stats) {
        int64_t h[ST_COUNT];
        PCHK(hipMemcpy(h, st_dev, sizeof(h), hipMemcpyDeviceToHost));
        tkc_stats st;
        memset(&st, 0, sizeof(st));
        st.m_vis = h[ST_MVIS];
        st.bfs_started = h[ST_STARTED];
        st.bfs_exact = h[ST_EXACT];
        st.bfs_cut = h[ST_CUT];
        st.skipped = h[ST_SKIPPED];
        st.max_level = (int32_t)h[ST_MAXLEVEL];
        st.batch_width = c->tune.batch_width;
        st.variant_used = variant;
        st.mode_used = TKC_BATCHED;
        st.ms_traverse = ms_launch;
        st.ms_kernel_main = ms_launch;
        st.main_launches = 1;
        st.main_kernel = 1;
        st.bytes_main = h[ST_BYTES];
        st.ms_total = tkc_now_ms() - t0;
        *stats = st;
    }
    return TKC_OK;
}
