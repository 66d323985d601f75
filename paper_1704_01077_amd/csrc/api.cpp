// C ABI of the top-k closeness library and the host driver of Alg. 1.
//
// A query runs these steps on the context's stream:
//   1. reachability: r(v) by connected components (undirected), or the
//      alpha/omega bounds of Alg. 6 (directed), on the device -- Sect. 4
//      and Sect. 8.4;
//   2. initial bounds (computeBounds): Deg (L = 0, order by degree) or NB
//      (walk-count bound of Sect. 5 / 8.1, order by the bound);
//   3. processing order: one stable radix sort of the order keys;
//   4. searches (updateBounds): plain, batched or hybrid engine, BFSCut or
//      level-based updates;
//   5. readback of the k results (ids, S, r) and the farness doubles.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tkc.h"
#include "dev_common.hpp"
#include "engine.hpp"
#include "internal.hpp"

static thread_local std::string g_err;

int tkc_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return tkc_fail(TKC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

double tkc_now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ arena
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsItem {
    void** p;
    size_t bytes;
    bool zero;
};
// layout of every buffer a query may use
static size_t ws_items(Workspace& ws, const WsShape& sh, std::vector<WsItem>& items) {
    size_t n = (size_t)sh.n, nw = (size_t)sh.nw, W = (size_t)sh.W;
    size_t words = (n + 31) / 32;
    size_t lcap = (size_t)sh.lcap;
    items = {
        {(void**)&ws.alpha, 8 * n, false}, {(void**)&ws.omega, 8 * n, false},
        {(void**)&ws.scc, 4 * n, false}, {(void**)&ws.lnum, 8 * n, false},
        {(void**)&ws.lden, 8 * n, false}, {(void**)&ws.key, 4 * n, false},
        {(void**)&ws.ord, 4 * n, false}, {(void**)&ws.tkey, 4 * n, false},
        {(void**)&ws.tval, 4 * n, false},
        {(void**)&ws.hist, 4 * (size_t)tkc_sort8_hist_words(sh.n), false},
        {(void**)&ws.mask, 64, false}, {(void**)&ws.parent, 4 * n, false},
        {(void**)&ws.csize, 8 * n + 16, false}, {(void**)&ws.gbuf, 32 * n, false},
        {(void**)&ws.nbsum, 8 * n, false}, {(void**)&ws.nbvis, 8 * n, false},
        {(void**)&ws.nbhub, 8 * n, false},
        {(void**)&ws.nbflags, n, false}, {(void**)&ws.small, 8192, false},
        // NB: heavy chunks' partial sums, or the tail rounds' list (n / 64 int32)
        {(void**)&ws.nbpart, std::max(8 * (size_t)sh.nchunks, 4 * (n / 64)) + 8, false},
        // read back together: keep stats .. tI adjacent and in this order
        {(void**)&ws.stats, 8 * 4 * ST_COUNT, false}, {(void**)&ws.tstate, 4096, false},
        {(void**)&ws.tS, 8 * (size_t)sh.kcap, false}, {(void**)&ws.tR, 8 * (size_t)sh.kcap, false},
        {(void**)&ws.tI, 4 * (size_t)sh.kcap, false},
        {(void**)&ws.ring, sizeof(XRec) * TKC_XRING, false},
        {(void**)&ws.tieS, sh.ties ? 8 * n : 8, false}, {(void**)&ws.tieR, sh.ties ? 8 * n : 8, false},
        {(void**)&ws.tieI, sh.ties ? 4 * n : 4, false},
        {(void**)&ws.bar, 4 * tkc_bar_words(4096), true},
        // plain engine
        {(void**)&ws.p_vis, 4 * words, true}, {(void**)&ws.p_fb, 12 * words, true},
        {(void**)&ws.p_ql, 4 * n, false}, {(void**)&ws.p_qh, 4 * n, false},
        {(void**)&ws.p_qg, 8 * ((size_t)sh.nchunks + 64), false}, {(void**)&ws.p_ctr, 8 * 32, true}, {(void**)&ws.p_lvl, 4 * n, false},
        {(void**)&ws.p_levcnt, 8 * (n + 2), false}, {(void**)&ws.p_levtab, 8 * (n + 2), false},
        // batched engine
        {(void**)&ws.b_vis, 8 * n * nw, true}, {(void**)&ws.b_frt0, 8 * n * nw, true},
        {(void**)&ws.b_frt1, 8 * n * nw, true}, {(void**)&ws.b_nxt, 8 * n * nw, true},
        {(void**)&ws.b_list, 32 * n + 16 * ((size_t)sh.nchunks + 64), false}, {(void**)&ws.b_mark, 4 * n, true},
        {(void**)&ws.b_ctr, 8 * 2048, true}, {(void**)&ws.b_cand, 8 * 256, false},
        {(void**)&ws.b_hist, sh.lb ? 8 * lcap * W : 8, false},
        {(void**)&ws.b_levtab, sh.lb ? 8 * lcap * W : 8, false},
        {(void**)&ws.b_lvl, sh.lb ? 2 * n * W : 8, false},
        {(void**)&ws.b_outS, 8 * n, false}, {(void**)&ws.b_outR, 8 * n, false},
        // per-workgroup engine
        {(void**)&ws.s_vis, 4 * words * (size_t)sh.swarm_blocks, true},
        {(void**)&ws.s_queue, 4 * (size_t)sh.qcap * (size_t)sh.swarm_blocks, false},
        {(void**)&ws.s_deferred, 4 * n, false},
    };
    size_t total = 0;
    for (auto& it : items) total += align_up(it.bytes);
    return total;
}

size_t tkc_ws_bytes(const WsShape& sh) {
    Workspace tmp;
    std::vector<WsItem> items;
    return ws_items(tmp, sh, items);
}

std::mutex& tkc_coop_mutex() {
    static std::mutex m;
    return m;
}

int tkc_ws_reserve(tkc_ctx* ctx, Workspace& ws, const WsShape& sh) {
    std::vector<WsItem> items;
    size_t total = ws_items(ws, sh, items);
    if (ws.base && total <= ws.bytes && ws.shape.covers(sh)) return TKC_OK;
    if (ws.base) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        hipFree(ws.base);
        ws.base = nullptr;
        ws.bytes = 0;
    }
    void* base = nullptr;
    if (hipMalloc(&base, total) != hipSuccess) {
        hipGetLastError();
        return tkc_fail(TKC_ENOMEM, "device allocation of %zu bytes failed", total);
    }
    ws.base = (char*)base;
    ws.bytes = total;
    ws.shape = sh;
    size_t off = 0;
    for (auto& it : items) {
        *it.p = ws.base + off;
        if (it.zero) HIPCHK(hipMemsetAsync(ws.base + off, 0, it.bytes, ctx->stream));
        off += align_up(it.bytes);
    }
    const size_t span = (size_t)(((char*)ws.tI + 4 * (size_t)sh.kcap) - (char*)ws.stats);
    if (ws.pin_bytes < span) {
        if (ws.pin) hipHostFree(ws.pin);
        ws.pin = nullptr;
        ws.pin_bytes = 0;
        if (hipHostMalloc((void**)&ws.pin, span, hipHostMallocDefault) != hipSuccess) {
            hipGetLastError();
            ws.pin = nullptr;
            // give the device arena back too, so that the next call starts
            // over instead of finding a workspace without its readback buffer
            hipStreamSynchronize(ctx->stream);
            hipFree(ws.base);
            ws.base = nullptr;
            ws.bytes = 0;
            return tkc_fail(TKC_ENOMEM, "pinned host allocation of %zu bytes failed", span);
        }
        ws.pin_bytes = span;
    }
    if (getenv("TKC_TRACE") && !ws.trace) {
        if (hipMalloc((void**)&ws.trace, 8 * (8 + 16 * 4096)) != hipSuccess) ws.trace = nullptr;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return TKC_OK;
}

// ---------------------------------------------------------------- context
extern "C" int tkc_ctx_create(int device, void* hip_stream, tkc_ctx** out) {
    if (!out) return tkc_fail(TKC_EINVAL, "out is NULL");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return tkc_fail(TKC_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return tkc_fail(TKC_EINVAL, "device %d out of range", device);
    HIPCHK(hipSetDevice(device));
    if (int rc = tkc_noalloc_init(device)) return rc;
    tkc_ctx* c = new tkc_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return tkc_fail(TKC_EDEVICE, "stream creation failed");
        }
        c->own_stream = true;
    }
    bool ok = hipEventCreate(&c->ev0) == hipSuccess && hipEventCreate(&c->ev1) == hipSuccess &&
              hipEventCreate(&c->evm) == hipSuccess;
    for (auto& e : c->evq) ok = ok && hipEventCreate(&e) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&c->pinned, 4096, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        tkc_ctx_destroy(c);
        return tkc_fail(TKC_EDEVICE, "event or pinned buffer creation failed");
    }
    *out = c;
    return TKC_OK;
}

extern "C" int tkc_ctx_destroy(tkc_ctx* c) {
    if (!c) return TKC_OK;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    if (c->ws.base) hipFree(c->ws.base);
    if (c->ws.trace) hipFree(c->ws.trace);
    if (c->ws.pin) hipHostFree(c->ws.pin);
    if (c->pinned) hipHostFree(c->pinned);
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    for (auto& e : c->evq)
        if (e) hipEventDestroy(e);
    if (c->evm) hipEventDestroy(c->evm);
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return TKC_OK;
}

static void tuning_out(const EngineTuning& e, tkc_tuning* t) {
    t->batch_width = e.batch_width;
    t->td_bu_alpha = e.td_bu_alpha;
    t->bu_td_beta = e.bu_td_beta;
    t->batch_alpha = e.batch_alpha;
    t->swarm_qcap = e.swarm_qcap;
    t->seed_lanes = e.seed_lanes;
    t->blocks_per_cu = e.blocks_per_cu;
    t->mode = e.mode;
}

static int tuning_in(const tkc_tuning* t, EngineTuning* e) {
    const int32_t bw = t->batch_width;
    if (bw != 32 && bw != 64 && bw != 128 && bw != 256)
        return tkc_fail(TKC_EINVAL, "batch_width must be 32, 64, 128 or 256");
    if (t->td_bu_alpha < 1 || t->bu_td_beta < 1 || t->batch_alpha < 1)
        return tkc_fail(TKC_EINVAL, "direction thresholds must be >= 1");
    if (t->swarm_qcap < 64) return tkc_fail(TKC_EINVAL, "swarm_qcap must be >= 64");
    if (t->seed_lanes < 0 || t->seed_lanes > bw) return tkc_fail(TKC_EINVAL, "seed_lanes must be in [0, batch_width]");
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 8) return tkc_fail(TKC_EINVAL, "blocks_per_cu must be in [1, 8]");
    if (t->mode < TKC_PLAIN || t->mode > TKC_HYBRID) return tkc_fail(TKC_EINVAL, "mode must be plain, batched or hybrid");
    EngineTuning x = *e;
    x.batch_width = bw;
    x.td_bu_alpha = t->td_bu_alpha;
    x.bu_td_beta = t->bu_td_beta;
    x.batch_alpha = t->batch_alpha;
    x.swarm_qcap = t->swarm_qcap;
    x.seed_lanes = t->seed_lanes;
    x.blocks_per_cu = t->blocks_per_cu;
    x.mode = t->mode;
    *e = x;
    return TKC_OK;
}

extern "C" int tkc_ctx_get_tuning(tkc_ctx* c, tkc_tuning* out) {
    if (!c || !out) return tkc_fail(TKC_EINVAL, "NULL argument");
    tuning_out(c->tune, out);
    return TKC_OK;
}

extern "C" int tkc_ctx_set_tuning(tkc_ctx* c, const tkc_tuning* t) {
    if (!c || !t) return tkc_fail(TKC_EINVAL, "NULL argument");
    return tuning_in(t, &c->tune);
}

// ------------------------------------------------------------------ graphs
static int validate_csr(int32_t n, int64_t m, const int32_t* rp, const int32_t* ci, const char* what) {
    if (rp[0] != 0) return tkc_fail(TKC_EINVAL, "%s: row_ptr[0] must be 0", what);
    if ((int64_t)rp[n] != m) return tkc_fail(TKC_EINVAL, "%s: row_ptr[n] != m_arcs", what);
    std::vector<int32_t> row;
    for (int32_t u = 0; u < n; u++) {
        if (rp[u + 1] < rp[u]) return tkc_fail(TKC_EINVAL, "%s: row_ptr not monotone at %d", what, u);
        row.assign(ci + rp[u], ci + rp[u + 1]);
        for (int32_t w : row) {
            if (w < 0 || w >= n) return tkc_fail(TKC_EINVAL, "%s: vertex id %d out of range", what, w);
            if (w == u) return tkc_fail(TKC_EINVAL, "%s: self-loop at %d", what, u);
        }
        std::sort(row.begin(), row.end());
        for (size_t q = 1; q < row.size(); q++)
            if (row[q] == row[q - 1]) return tkc_fail(TKC_EINVAL, "%s: repeated arc %d->%d", what, u, row[q]);
    }
    return TKC_OK;
}

// the checks every upload runs (memory safety of the kernels): row_ptr starts
// at 0, never decreases and ends at m; every vertex id is in [0, n)
static int check_csr_bounds(int32_t n, int64_t m, const int32_t* rp, const int32_t* ci, const char* what) {
    if (rp[0] != 0) return tkc_fail(TKC_EINVAL, "%s: row_ptr[0] must be 0", what);
    if ((int64_t)rp[n] != m) return tkc_fail(TKC_EINVAL, "%s: row_ptr[n] != m_arcs", what);
    for (int32_t u = 0; u < n; u++)
        if (rp[u + 1] < rp[u]) return tkc_fail(TKC_EINVAL, "%s: row_ptr not monotone at %d", what, u);
    bool bad = false;
    for (int64_t e = 0; e < m; e++) bad |= (uint32_t)ci[e] >= (uint32_t)n;
    if (bad) return tkc_fail(TKC_EINVAL, "%s: vertex id out of range", what);
    return TKC_OK;
}

// true when (rp2, ci2) is the transpose of (rp, ci)
static bool is_transpose(int32_t n, int64_t m, const int32_t* rp, const int32_t* ci, const int32_t* rp2,
                         const int32_t* ci2) {
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t e = 0; e < m; e++) cnt[ci[e] + 1]++;
    for (int32_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    for (int32_t i = 0; i <= n; i++)
        if (cnt[i] != rp2[i]) return false;
    std::vector<int32_t> t(m);
    std::vector<int64_t> fill(cnt.begin(), cnt.end());
    for (int32_t u = 0; u < n; u++)
        for (int32_t e = rp[u]; e < rp[u + 1]; e++) t[fill[ci[e]]++] = u;
    std::vector<int32_t> a, b;
    for (int32_t v = 0; v < n; v++) {
        a.assign(t.begin() + cnt[v], t.begin() + cnt[v + 1]);
        b.assign(ci2 + rp2[v], ci2 + rp2[v + 1]);
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        if (a != b) return false;
    }
    return true;
}

extern "C" int tkc_graph_upload(tkc_ctx* c, int32_t n, int64_t m, const int32_t* row_ptr,
                                const int32_t* col_idx, const int32_t* rrow_ptr, const int32_t* rcol_idx,
                                uint32_t flags, tkc_graph** out) {
    if (!c || !out || !row_ptr || (!col_idx && m > 0)) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (n < 1) return tkc_fail(TKC_EINVAL, "n must be >= 1");
    if (m < 0 || m > 0x7fffffffLL) return tkc_fail(TKC_EINVAL, "m_arcs must be in [0, 2^31)");
    const bool directed = (flags & TKC_DIRECTED) != 0;
    if (directed && (flags & TKC_REVERSE)) {
        // in-closeness: the reversed graph's out-arcs are the in-arcs
        std::swap(row_ptr, rrow_ptr);
        std::swap(col_idx, rcol_idx);
    }
    if (directed && (!rrow_ptr || (!rcol_idx && m > 0)))
        return tkc_fail(TKC_EINVAL, "directed graph needs the reverse CSR");
    if (!directed && (rrow_ptr || rcol_idx))
        return tkc_fail(TKC_EINVAL, "reverse CSR given for an undirected graph");
    HIPCHK(hipSetDevice(c->device));
    // host copies: the checks below, the heavy-vertex tables, and (directed)
    // the host fallback of the reachability bounds
    std::vector<int32_t> hrp(n + 1), hci(m), hrrp, hrci;
    const hipMemcpyKind k = (flags & TKC_DEVICE_PTRS) ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HIPCHK(hipMemcpy(hrp.data(), row_ptr, 4 * (size_t)(n + 1), k));
    if (m) HIPCHK(hipMemcpy(hci.data(), col_idx, 4 * (size_t)m, k));
    if (directed) {
        hrrp.resize(n + 1);
        hrci.resize(m);
        HIPCHK(hipMemcpy(hrrp.data(), rrow_ptr, 4 * (size_t)(n + 1), k));
        if (m) HIPCHK(hipMemcpy(hrci.data(), rcol_idx, 4 * (size_t)m, k));
    }
    {
        int rc = check_csr_bounds(n, m, hrp.data(), hci.data(), "out-arcs");
        if (!rc && directed) rc = check_csr_bounds(n, m, hrrp.data(), hrci.data(), "in-arcs");
        if (rc) return rc;
    }
    if (flags & TKC_VALIDATE) {
        int rc = validate_csr(n, m, hrp.data(), hci.data(), "out-arcs");
        if (rc) return rc;
        if (directed) {
            rc = validate_csr(n, m, hrrp.data(), hrci.data(), "in-arcs");
            if (rc) return rc;
            if (!is_transpose(n, m, hrp.data(), hci.data(), hrrp.data(), hrci.data()))
                return tkc_fail(TKC_EINVAL, "reverse CSR is not the transpose of the CSR");
        } else if (!is_transpose(n, m, hrp.data(), hci.data(), hrp.data(), hci.data())) {
            return tkc_fail(TKC_EINVAL, "undirected CSR is not symmetric");
        }
    }
    // TKC_RELABEL: vertices renumbered by decreasing out-degree (ties by id),
    // rows sorted; oid[new] = caller's id, nid[caller's id] = new
    std::vector<int32_t> oid, nid;
    if (flags & TKC_RELABEL) {
        oid.resize(n);
        nid.resize(n);
        for (int32_t v = 0; v < n; v++) oid[v] = v;
        std::stable_sort(oid.begin(), oid.end(), [&](int32_t a, int32_t b) {
            return hrp[a + 1] - hrp[a] > hrp[b + 1] - hrp[b];
        });
        for (int32_t v = 0; v < n; v++) nid[oid[v]] = v;
        auto permute = [&](std::vector<int32_t>& rp, std::vector<int32_t>& ci) {
            std::vector<int32_t> rp2(n + 1), ci2(m);
            rp2[0] = 0;
            for (int32_t v = 0; v < n; v++) {
                const int32_t o = oid[v];
                int32_t at = rp2[v];
                for (int32_t e = rp[o]; e < rp[o + 1]; e++) ci2[at++] = nid[ci[e]];
                std::sort(ci2.begin() + rp2[v], ci2.begin() + at);
                rp2[v + 1] = at;
            }
            rp.swap(rp2);
            ci.swap(ci2);
        };
        permute(hrp, hci);
        if (directed) permute(hrrp, hrci);
    }
    tkc_graph* g = new tkc_graph();
    g->ctx = c;
    g->n = n;
    g->m = m;
    g->directed = directed;
    g->relabeled = (flags & TKC_RELABEL) != 0;
    // heavy vertices and their arc chunks (ascending ids: deterministic), for
    // the out-arcs and (directed) the in-arcs
    std::vector<int32_t> hv, hcb(1, 0), cb, ce, cv, rcb, rce, rcv;
    for (int32_t u = 0; u < n; u++) {
        int32_t d = hrp[u + 1] - hrp[u];
        if (d <= HEAVY_DEG) continue;
        hv.push_back(u);
        for (int32_t b = hrp[u]; b < hrp[u + 1]; b += CHUNK_ARCS) {
            cb.push_back(b);
            ce.push_back(std::min(b + CHUNK_ARCS, hrp[u + 1]));
            cv.push_back(u);
        }
        hcb.push_back((int32_t)cb.size());
    }
    if (directed) {
        for (int32_t u = 0; u < n; u++) {
            if (hrrp[u + 1] - hrrp[u] <= HEAVY_DEG) continue;
            for (int32_t b = hrrp[u]; b < hrrp[u + 1]; b += CHUNK_ARCS) {
                rcb.push_back(b);
                rce.push_back(std::min(b + CHUNK_ARCS, hrrp[u + 1]));
                rcv.push_back(u);
            }
        }
    }
    // in-arc chunks of the hubs (in-degree above HUB_IN_DEG)
    std::vector<int32_t> bcb, bce, bcv;
    {
        const int32_t* irp = directed ? hrrp.data() : hrp.data();
        for (int32_t u = 0; u < n; u++) {
            if (irp[u + 1] - irp[u] <= HUB_IN_DEG) continue;
            for (int32_t b = irp[u]; b < irp[u + 1]; b += CHUNK_ARCS) {
                bcb.push_back(b);
                bce.push_back(std::min(b + CHUNK_ARCS, irp[u + 1]));
                bcv.push_back(u);
            }
        }
    }
    g->bnchunks = (int32_t)bcb.size();
    // mid in-degree vertices packed into segments (edge-balanced pulls)
    std::vector<int32_t> mvtx, mseg(1, 0);
    {
        const int32_t* irp = directed ? hrrp.data() : hrp.data();
        int64_t arcs = 0;
        for (int32_t u = 0; u < n; u++) {
            const int32_t d = irp[u + 1] - irp[u];
            if (d <= HEAVY_DEG || d > HUB_IN_DEG) continue;
            const int32_t cnt = (int32_t)mvtx.size() - mseg.back();
            if (cnt > 0 && (cnt == 64 || arcs + d > MID_ARCS)) {
                mseg.push_back((int32_t)mvtx.size());
                arcs = 0;
            }
            mvtx.push_back(u);
            arcs += d;
        }
        if ((int32_t)mvtx.size() > mseg.back()) mseg.push_back((int32_t)mvtx.size());
    }
    g->nmseg = (int32_t)mseg.size() - 1;
    g->nheavy = (int32_t)hv.size();
    g->nchunks = (int32_t)cb.size();
    g->rnchunks = directed ? (int32_t)rcb.size() : g->nchunks;
    size_t bytes = 4 * (size_t)(n + 1) + 4 * (size_t)(m ? m : 1) + 4 * (size_t)n + 4 * (hv.size() + 1) +
                   4 * hcb.size() + 12 * (cb.size() + 1) + 12 * (rcb.size() + 1) + 12 * (bcb.size() + 1) +
                   4 * (mvtx.size() + 1) + 4 * mseg.size() + 16 * 256;
    if (directed) bytes += 4 * (size_t)(n + 1) + 4 * (size_t)(m ? m : 1);
    if (g->relabeled) bytes += 8 * (size_t)n + 512;
    if (hipMalloc(&g->dbase, bytes + 1024) != hipSuccess) {
        hipGetLastError();
        delete g;
        return tkc_fail(TKC_ENOMEM, "graph allocation failed");
    }
    char* p = (char*)g->dbase;
    auto take = [&](size_t b) { char* r = p; p += align_up(b); return r; };
    g->rp = (int32_t*)take(4 * (size_t)(n + 1));
    g->ci = (int32_t*)take(4 * (size_t)(m ? m : 1));
    g->deg = (int32_t*)take(4 * (size_t)n);
    g->heavy = (int32_t*)take(4 * (hv.size() + 1));
    g->hcb = (int32_t*)take(4 * hcb.size());
    g->ch_beg = (int32_t*)take(4 * (cb.size() + 1));
    g->ch_end = (int32_t*)take(4 * (cb.size() + 1));
    g->ch_vtx = (int32_t*)take(4 * (cb.size() + 1));
    if (directed) {
        g->rch_beg = (int32_t*)take(4 * (rcb.size() + 1));
        g->rch_end = (int32_t*)take(4 * (rcb.size() + 1));
        g->rch_vtx = (int32_t*)take(4 * (rcb.size() + 1));
    } else {
        g->rch_beg = g->ch_beg;
        g->rch_end = g->ch_end;
        g->rch_vtx = g->ch_vtx;
    }
    g->bch_beg = (int32_t*)take(4 * (bcb.size() + 1));
    g->bch_end = (int32_t*)take(4 * (bcb.size() + 1));
    g->bch_vtx = (int32_t*)take(4 * (bcb.size() + 1));
    g->mid_vtx = (int32_t*)take(4 * (mvtx.size() + 1));
    g->mseg = (int32_t*)take(4 * mseg.size());
    if (directed) {
        g->rrp = (int32_t*)take(4 * (size_t)(n + 1));
        g->rci = (int32_t*)take(4 * (size_t)(m ? m : 1));
    } else {
        g->rrp = g->rp;
        g->rci = g->ci;
    }
    if (g->relabeled) {
        g->d_oid = (int32_t*)take(4 * (size_t)n);
        g->d_nid = (int32_t*)take(4 * (size_t)n);
    }
    hipStream_t s = c->stream;
    int rc = TKC_OK;
    if (g->relabeled &&
        (hipMemcpyAsync(g->d_oid, oid.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(g->d_nid, nid.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess))
        rc = tkc_fail(TKC_EDEVICE, "vertex map copy failed");
    if (g->relabeled) g->h_nid = nid;
    if (hipMemcpyAsync(g->rp, hrp.data(), 4 * (size_t)(n + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        (m && hipMemcpyAsync(g->ci, hci.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s) != hipSuccess))
        rc = tkc_fail(TKC_EDEVICE, "graph copy failed");
    if (!rc && directed &&
        (hipMemcpyAsync(g->rrp, hrrp.data(), 4 * (size_t)(n + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
         (m && hipMemcpyAsync(g->rci, hrci.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s) != hipSuccess)))
        rc = tkc_fail(TKC_EDEVICE, "reverse graph copy failed");
    if (!rc && ((hv.size() && hipMemcpyAsync(g->heavy, hv.data(), 4 * hv.size(), hipMemcpyHostToDevice, s)) ||
                hipMemcpyAsync(g->hcb, hcb.data(), 4 * hcb.size(), hipMemcpyHostToDevice, s) ||
                (cb.size() && (hipMemcpyAsync(g->ch_beg, cb.data(), 4 * cb.size(), hipMemcpyHostToDevice, s) ||
                               hipMemcpyAsync(g->ch_end, ce.data(), 4 * ce.size(), hipMemcpyHostToDevice, s) ||
                               hipMemcpyAsync(g->ch_vtx, cv.data(), 4 * cv.size(), hipMemcpyHostToDevice, s))) ||
                (rcb.size() && (hipMemcpyAsync(g->rch_beg, rcb.data(), 4 * rcb.size(), hipMemcpyHostToDevice, s) ||
                                hipMemcpyAsync(g->rch_end, rce.data(), 4 * rce.size(), hipMemcpyHostToDevice, s) ||
                                hipMemcpyAsync(g->rch_vtx, rcv.data(), 4 * rcv.size(), hipMemcpyHostToDevice, s))) ||
                (bcb.size() && (hipMemcpyAsync(g->bch_beg, bcb.data(), 4 * bcb.size(), hipMemcpyHostToDevice, s) ||
                                hipMemcpyAsync(g->bch_end, bce.data(), 4 * bce.size(), hipMemcpyHostToDevice, s) ||
                                hipMemcpyAsync(g->bch_vtx, bcv.data(), 4 * bcv.size(), hipMemcpyHostToDevice, s))) ||
                (mvtx.size() && hipMemcpyAsync(g->mid_vtx, mvtx.data(), 4 * mvtx.size(), hipMemcpyHostToDevice, s)) ||
                hipMemcpyAsync(g->mseg, mseg.data(), 4 * mseg.size(), hipMemcpyHostToDevice, s)))
        rc = tkc_fail(TKC_EDEVICE, "heavy-vertex table copy failed");
    if (!rc) {
        DevGraph dg = g->view();
        if (tkc_launch_degrees(dg, s) || hipStreamSynchronize(s) != hipSuccess)
            rc = tkc_fail(TKC_EDEVICE, "degree kernel failed");
    }
    if (rc) {
        hipStreamSynchronize(s);
        hipFree(g->dbase);
        delete g;
        return rc;
    }
    *out = g;
    return TKC_OK;
}

extern "C" int tkc_graph_free(tkc_graph* g) {
    if (!g) return TKC_OK;
    if (g->server_refs > 0) return tkc_fail(TKC_EBUSY, "graph is held by a server");
    hipSetDevice(g->ctx->device);
    hipStreamSynchronize(g->ctx->stream);
    hipFree(g->dbase);
    if (g->reach_base) hipFree(g->reach_base);
    for (auto& p : g->prep)
        if (p.base) hipFree(p.base);
    delete g;
    return TKC_OK;
}

// ------------------------------------------------------------ query steps
EngineTuning tkc_effective_tuning(const EngineTuning& ctx_tune, tkc_graph* g) {
    std::lock_guard<std::mutex> lk(g->mu);
    return g->tuned ? g->tune : ctx_tune;
}

WsShape tkc_shape_for(const EngineTuning& t, tkc_graph* g, int32_t k, bool lb) {
    WsShape sh;
    sh.n = g->n;
    sh.W = t.batch_width;
    sh.nw = sh.W <= 64 ? 1 : sh.W / 64;
    sh.kcap = std::max(k, 1);
    sh.lb = lb;
    sh.lcap = (int32_t)std::min<int64_t>((int64_t)g->n + 2, 65000);
    sh.nchunks = std::max(g->nchunks, g->rnchunks);
    sh.qcap = std::max(64, std::min(t.swarm_qcap, g->n));
    sh.swarm_blocks = std::max(1, tkc_swarm_max_blocks(256));
    // the private bitmaps of the per-workgroup engine cost blocks * n/8 bytes;
    // keep them under 2 GiB
    while (sh.swarm_blocks > 64 && (int64_t)sh.swarm_blocks * ((g->n + 31) / 32) * 4 > (2ll << 30))
        sh.swarm_blocks /= 2;
    return sh;
}

// step 1: reachability into ws.alpha / ws.omega (/ ws.scc)
int tkc_step_reach(tkc_ctx* c, tkc_graph* g, Workspace& ws) {
    hipStream_t s = c->stream;
    DevGraph dg = g->view();
    if (!g->directed) {
        if (tkc_launch_cc(dg, ws.parent, ws.csize, ws.alpha, ws.omega, ws.nbflags, (int32_t*)c->pinned, s))
            return tkc_fail(TKC_EDEVICE, "components kernel failed");
        return TKC_OK;
    }
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (!g->reach_path) {
            const size_t n = g->n;
            if (!g->reach_base) {
                HIPCHK(hipMalloc(&g->reach_base, 16 * n + 4 * n + 256));
                g->d_alpha = (int64_t*)g->reach_base;
                g->d_omega = g->d_alpha + n;
                g->d_scc = (int32_t*)(g->d_omega + n);
            }
            const double t0 = now_ms();
            int seq = 0;
            const int r = tkc_device_alpha_omega(dg, g->d_alpha, g->d_omega, g->d_scc, c->pinned, s, &seq);
            if (r == -2) return tkc_fail(TKC_ENOMEM, "no device memory for the reachability scratch");
            if (r < 0) return tkc_fail(TKC_EDEVICE, "reachability kernels failed");
            g->reach_ms = now_ms() - t0;
            g->reach_path = seq ? 2 : 1;
        }
    }
    HIPCHK(hipMemcpyAsync(ws.alpha, g->d_alpha, 8 * (size_t)g->n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ws.omega, g->d_omega, 8 * (size_t)g->n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ws.scc, g->d_scc, 4 * (size_t)g->n, hipMemcpyDeviceToDevice, s));
    return TKC_OK;
}

extern "C" int tkc_graph_reach_info(const tkc_graph* g, int32_t* path, double* ms) {
    if (!g) return tkc_fail(TKC_EINVAL, "null graph");
    if (path) *path = g->directed ? g->reach_path : 1;
    if (ms) *ms = g->reach_ms;
    return TKC_OK;
}

// step 2 + 3: bounds into ws.lnum / ws.lden, order into ws.ord / ws.key
int tkc_step_bounds(tkc_ctx* c, tkc_graph* g, Workspace& ws, bool nb, int32_t* rounds, bool harm) {
    hipStream_t s = c->stream;
    DevGraph dg = g->view();
    int32_t n = g->n;
    if (rounds) *rounds = 0;
    // the sort's key mask, staged apart from the NB finish count in pinned memory
    uint32_t* mask_pin = (uint32_t*)c->pinned + 64;
    bool keyed = false;
    if (nb) {
        int32_t* nfin_dev = (int32_t*)ws.small;
        // order keys and their mask, queued by the NB rounds before their
        // last host wait
        const std::function<int()> fin = [&]() -> int {
            if (harm) {
                if (tkc_launch_harm_bounds(dg, ws.omega, ws.nbhub, ws.lnum, ws.lden, ws.key, ws.ord, s)) return -1;
            } else if (tkc_launch_nb_keys(n, ws.lnum, ws.lden, ws.key, ws.ord, s)) {
                return -1;
            }
            return tkc_sort_mask(ws.key, n, (uint32_t*)ws.mask, mask_pin, s);
        };
        int r = tkc_launch_nb(dg, ws.alpha, ws.omega, ws.gbuf, ws.nbsum, ws.nbvis, ws.nbflags, ws.lnum, ws.lden,
                              ws.nbpart, nfin_dev, (int32_t*)c->pinned, s, harm ? ws.nbhub : nullptr, &fin, &keyed);
        if (r < 0) return tkc_fail(TKC_EDEVICE, "NB bound kernels failed");
        if (rounds) *rounds = r;
        if (!keyed) {
            if (harm) {
                if (tkc_launch_harm_bounds(dg, ws.omega, ws.nbhub, ws.lnum, ws.lden, ws.key, ws.ord, s))
                    return tkc_fail(TKC_EDEVICE, "harmonic bound kernel failed");
            } else if (tkc_launch_nb_keys(n, ws.lnum, ws.lden, ws.key, ws.ord, s)) {
                return tkc_fail(TKC_EDEVICE, "key kernel failed");
            }
        }
    } else if (harm) {
        if (tkc_launch_harm_bounds(dg, ws.omega, nullptr, ws.lnum, ws.lden, ws.key, ws.ord, s))
            return tkc_fail(TKC_EDEVICE, "harmonic bound kernel failed");
    } else {
        if (tkc_launch_deg_bounds(dg, ws.omega, ws.lnum, ws.lden, ws.key, ws.ord, s))
            return tkc_fail(TKC_EDEVICE, "degree bound kernel failed");
    }
    if (tkc_sort_pairs8(ws.key, ws.ord, ws.tkey, ws.tval, n, ws.hist, (uint32_t*)ws.mask,
                        (uint32_t*)c->pinned, s, keyed ? mask_pin : nullptr))
        return tkc_fail(TKC_EDEVICE, "sort failed");
    return TKC_OK;
}

static DevTopk topk_view(Workspace& ws) {
    DevTopk t;
    t.st = (TopkState*)ws.tstate;
    t.ring = (XRec*)ws.ring;
    t.S = ws.tS;
    t.R = ws.tR;
    t.I = ws.tI;
    return t;
}

static PlainWork plain_view(Workspace& ws) {
    PlainWork w{};
    w.vis = ws.p_vis; w.fb = ws.p_fb; w.ql = ws.p_ql; w.qh = ws.p_qh; w.qg = ws.p_qg; w.ctr = ws.p_ctr;
    w.ccap = (int64_t)ws.shape.nchunks + 64;
    w.lvl = ws.p_lvl; w.levcnt = ws.p_levcnt; w.levtab = ws.p_levtab;
    w.bar = ws.bar;
    return w;
}
BatchWork tkc_batch_view(Workspace& ws) {
    BatchWork w{};
    w.vis = ws.b_vis; w.frt0 = ws.b_frt0; w.frt1 = ws.b_frt1; w.nxt = ws.b_nxt;
    w.list = ws.b_list; w.touched = ws.b_mark; w.ctr = ws.b_ctr; w.lanes = nullptr;
    w.ccap = (int64_t)ws.shape.nchunks + 64;
    w.lvl = ws.b_lvl; w.hist = ws.b_hist; w.levtab = ws.b_levtab; w.lcap = ws.shape.lcap;
    w.cand = ws.b_cand;
    w.cand_req = ws.b_cand + 256;
    w.trace = ws.trace;
    w.trace_cap = ws.trace ? 4096 : 0;
    w.bar = ws.bar;
    return w;
}

// optional per-level trace of the batched engine (environment TKC_TRACE=1):
// one line per level on stderr, timestamps from the device wall clock
static void trace_reset(tkc_ctx* c) {
    if (c->ws.trace) hipMemsetAsync(c->ws.trace, 0, 8 * 8, c->stream);
}
static void trace_dump(tkc_ctx* c, const char* tag) {
    if (!c->ws.trace) return;
    std::vector<int64_t> h(8 + 16 * 4096);
    hipMemcpyAsync(h.data(), c->ws.trace, 8 * h.size(), hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    int64_t cnt = std::min<int64_t>(h[0], 4096);
    int rate = 0;
    hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, c->device);
    double khz = rate > 0 ? rate : 100000.0;
    for (int64_t i = 0; i < cnt; i++) {
        const int64_t* r = h.data() + 8 + 16 * i;
        double dt = i + 1 < cnt ? (h[8 + 16 * (i + 1) + 5] - r[5]) / khz * 1e3 : 0.0;
        double te = r[8] ? (r[8] - r[5]) / khz * 1e3 : 0.0;
        const double us = 1e3 / khz;
        fprintf(stderr,
                "trace %s batch %lld level %lld %s frontier %lld arcs %lld lanes %lld/%lld  %.1f us"
                " (to barrier exit %.1f; slowest wave of workgroup 0: clear %.1f fold %.1f vertices %.1f"
                " chunks %.1f flush %.1f barrier %.1f)\n",
                tag, (long long)r[0], (long long)r[1], r[2] ? "pull" : "push", (long long)r[3], (long long)r[4],
                (long long)r[7], (long long)r[6], dt, te, r[9] * us, r[10] * us, r[11] * us, r[12] * us,
                r[13] * us, r[14] * us);
    }
}

// time one engine launch with events on the context stream
struct EngineTimer {
    tkc_ctx* c;
    double* acc;
    int32_t* launches;
    std::lock_guard<std::mutex> lk;
    EngineTimer(tkc_ctx* c_, double* a, int32_t* l) : c(c_), acc(a), launches(l), lk(tkc_coop_mutex()) {
        hipEventRecord(c->ev0, c->stream);
    }
    // ends the timed launch; `more` queues copies to pinned memory that the
    // same host wait completes
    template <typename F>
    int done(F more) {
        hipEventRecord(c->ev1, c->stream);
        const int rc = more();
        if (hipStreamSynchronize(c->stream) != hipSuccess)
            return tkc_fail(TKC_EDEVICE, "engine launch failed: %s", hipGetErrorString(hipGetLastError()));
        float ms = 0.f;
        hipEventElapsedTime(&ms, c->ev0, c->ev1);
        *acc += ms;
        (*launches)++;
        return rc;
    }
    int done() {
        return done([] { return (int)TKC_OK; });
    }
};

// where a device address inside the read-back span sits in the pinned copy
template <typename T>
static T* pin_at(Workspace& ws, const void* dev) {
    return (T*)(ws.pin + ((const char*)dev - (const char*)ws.stats));
}
// queue the copy of one engine's counters into the pinned span
static int queue_stats(tkc_ctx* c, const int64_t* dev) {
    HIPCHK(hipMemcpyAsync(pin_at<int64_t>(c->ws, dev), dev, 8 * ST_COUNT, hipMemcpyDeviceToHost, c->stream));
    return TKC_OK;
}
// queue the copy of the whole result span (counters, top-k state, the k
// results): one copy while the capacity is modest, else one per part
static int queue_readback(tkc_ctx* c, int32_t k) {
    Workspace& ws = c->ws;
    hipStream_t s = c->stream;
    if (ws.shape.kcap <= 4096) {
        const size_t span = (size_t)(((char*)ws.tI + 4 * (size_t)k) - (char*)ws.stats);
        HIPCHK(hipMemcpyAsync(ws.pin, ws.stats, span, hipMemcpyDeviceToHost, s));
        return TKC_OK;
    }
    const size_t head = (size_t)(((char*)ws.tstate + sizeof(TopkState)) - (char*)ws.stats);
    HIPCHK(hipMemcpyAsync(ws.pin, ws.stats, head, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(pin_at<int64_t>(ws, ws.tS), ws.tS, 8 * (size_t)k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(pin_at<int64_t>(ws, ws.tR), ws.tR, 8 * (size_t)k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(pin_at<int32_t>(ws, ws.tI), ws.tI, 4 * (size_t)k, hipMemcpyDeviceToHost, s));
    return TKC_OK;
}

extern "C" int tkc_topk_closeness(tkc_graph* g, int32_t k, int32_t variant, int32_t mode, int32_t* ids,
                                  int64_t* sum_dist, int64_t* reach, double* farness, int32_t* n_out,
                                  tkc_stats* stats) {
    if (!g || !ids || !n_out) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (k < 1) return tkc_fail(TKC_EINVAL, "k must be >= 1");
    if (variant < TKC_AUTO || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "unknown variant %d", variant);
    if (mode < TKC_PLAIN || mode > TKC_MODE_AUTO) return tkc_fail(TKC_EINVAL, "unknown mode %d", mode);
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    return tkc_run_query(c, g, k, variant, mode, ids, sum_dist, reach, farness, n_out, stats);
}

extern "C" int tkc_topk_closeness_ties(tkc_graph* g, int32_t k, int32_t variant, int32_t mode, int32_t cap,
                                       int32_t* ids, int64_t* sum_dist, int64_t* reach, double* farness,
                                       int32_t* n_out, tkc_stats* stats) {
    if (!g || !ids || !n_out) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (k < 1) return tkc_fail(TKC_EINVAL, "k must be >= 1");
    if (variant < TKC_AUTO || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "unknown variant %d", variant);
    if (mode < TKC_PLAIN || mode > TKC_MODE_AUTO) return tkc_fail(TKC_EINVAL, "unknown mode %d", mode);
    if (cap < std::min(k, g->n)) return tkc_fail(TKC_EINVAL, "cap must be >= min(k, n)");
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    return tkc_run_query(c, g, k, variant, mode, ids, sum_dist, reach, farness, n_out, stats, cap);
}

extern "C" int tkc_topk_closeness_budget(tkc_graph* g, int32_t k, int32_t variant, int64_t max_searches,
                                         int32_t* ids, int64_t* sum_dist, int64_t* reach, double* farness,
                                         int32_t* n_out, tkc_stats* stats) {
    if (!g || !ids || !n_out) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (k < 1) return tkc_fail(TKC_EINVAL, "k must be >= 1");
    if (max_searches < 1) return tkc_fail(TKC_EINVAL, "max_searches must be >= 1");
    if (variant < TKC_AUTO || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "unknown variant %d", variant);
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    return tkc_run_query(c, g, k, variant, TKC_PLAIN, ids, sum_dist, reach, farness, n_out, stats, 0, false,
                         max_searches);
}

extern "C" int tkc_topk_harmonic(tkc_graph* g, int32_t k, int32_t variant, int32_t mode, int32_t* ids,
                                 double* harmonic, int32_t* n_out, tkc_stats* stats) {
    if (!g || !ids || !n_out) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (k < 1) return tkc_fail(TKC_EINVAL, "k must be >= 1");
    if (variant < TKC_AUTO || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "unknown variant %d", variant);
    if (mode < TKC_PLAIN || mode > TKC_MODE_AUTO) return tkc_fail(TKC_EINVAL, "unknown mode %d", mode);
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    return tkc_run_query(c, g, k, variant, mode, ids, nullptr, nullptr, harmonic, n_out, stats, 0, true);
}

// Runs one query under knobs t (on the graph's context, whose own knobs are
// restored afterwards) and returns its wall time.
static int autotune_trial(tkc_graph* g, int32_t k, int32_t variant, const EngineTuning& t,
                          std::vector<int32_t>& ids, double* ms) {
    tkc_ctx* c = g->ctx;
    const EngineTuning keep = c->tune;
    c->tune = t;
    int32_t nout = 0;
    double best = 1e300;
    int rc = TKC_OK;
    // short queries are repeated (best of three) so that noise does not pick
    for (int rep = 0; rep < 3 && rc == TKC_OK; rep++) {
        double t0 = now_ms();
        rc = tkc_run_query(c, g, k, variant, t.mode, ids.data(), nullptr, nullptr, nullptr, &nout, nullptr);
        double dt = now_ms() - t0;
        best = std::min(best, dt);
        if (dt > 20.0) break;
    }
    c->tune = keep;
    *ms = best;
    return rc;
}

extern "C" int tkc_autotune(tkc_graph* g, int32_t k, int32_t variant, double budget_ms, tkc_tuning* best,
                            double* best_ms) {
    if (!g) return tkc_fail(TKC_EINVAL, "graph is NULL");
    if (k < 1) return tkc_fail(TKC_EINVAL, "k must be >= 1");
    if (variant < TKC_AUTO || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "unknown variant %d", variant);
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    if (variant == TKC_AUTO) variant = tkc_auto_variant(c, g);
    const bool lb = tkc_lb_level(variant) != 0;
    const int32_t kk = std::min(k, g->n);
    std::vector<int32_t> ref(kk), ids(kk);
    EngineTuning cur = c->tune;
    if (cur.mode == TKC_PLAIN) cur.mode = TKC_BATCHED;
    double cur_ms = 0, spent = 0;
    // the first trial also warms up (workspace, preprocessing)
    int rc = autotune_trial(g, k, variant, cur, ref, &cur_ms);
    if (rc) return rc;
    rc = autotune_trial(g, k, variant, cur, ref, &cur_ms);
    if (rc) return rc;
    spent += cur_ms;
    // one knob at a time, most influential first
    struct Axis {
        int32_t EngineTuning::*field;
        std::vector<int32_t> values;
    };
    std::vector<Axis> axes = {
        {&EngineTuning::batch_width, {64, 128, 256, 32}},
        {&EngineTuning::mode, lb ? std::vector<int32_t>{TKC_BATCHED} : std::vector<int32_t>{TKC_BATCHED, TKC_HYBRID}},
        {&EngineTuning::blocks_per_cu, {1, 2, 3, 4}},
        {&EngineTuning::bu_td_beta, {24, 4, 1}},
        {&EngineTuning::batch_alpha, {4, 14, 40}},
    };
    for (const Axis& ax : axes) {
        for (int32_t v : ax.values) {
            if (spent >= budget_ms) break;
            if (cur.*(ax.field) == v) continue;
            EngineTuning t = cur;
            t.*(ax.field) = v;
            double ms = 0;
            rc = autotune_trial(g, k, variant, t, ids, &ms);
            if (rc) return rc;
            spent += ms;
            if (ids != ref) return tkc_fail(TKC_EDEVICE, "internal error: autotune trials disagree");
            if (ms < cur_ms) { cur = t; cur_ms = ms; }
        }
    }
    {
        std::lock_guard<std::mutex> lk(g->mu);
        g->tune = cur;
        g->tuned = true;
    }
    if (best) tuning_out(cur, best);
    if (best_ms) *best_ms = cur_ms;
    return TKC_OK;
}

int tkc_run_query(tkc_ctx* c, tkc_graph* g, int32_t k, int32_t variant, int32_t mode, int32_t* ids,
                  int64_t* sum_dist, int64_t* reach, double* farness, int32_t* n_out, tkc_stats* stats,
                  int32_t ties_cap, bool harm, int64_t max_searches) {
    const bool ties = ties_cap > 0;
    Workspace& ws = c->ws;
    hipStream_t s = c->stream;
    const int32_t n = g->n;
    if (k > n) k = n;
    double t0 = now_ms();
    tkc_stats st;
    memset(&st, 0, sizeof(st));
    int rc;
    // AUTO mode: the graph's autotuned knobs for this query, else the
    // context's preferred mode
    if (mode == TKC_MODE_AUTO) {
        const EngineTuning keep = c->tune;
        c->tune = tkc_effective_tuning(keep, g);
        c->tune.slice_batches = keep.slice_batches;
        rc = tkc_run_query(c, g, k, variant, c->tune.mode, ids, sum_dist, reach, farness, n_out, stats, ties_cap,
                           harm, max_searches);
        c->tune = keep;
        return rc;
    }
    // AUTO: high-diameter graphs favour level-based updates (Sect. 9.1)
    if (variant == TKC_AUTO) variant = tkc_auto_variant(c, g);
    const int lbl = tkc_lb_level(variant);
    const bool lb = lbl != 0;
    const bool nb = tkc_is_nb(variant);
    {
        WsShape sh = tkc_shape_for(c->tune, g, k, lb);
        sh.ties = ties;
        rc = tkc_ws_reserve(c, ws, sh);
    }
    if (rc) return rc;
    int32_t rounds = 0;
    HIPCHK(hipEventRecord(c->evq[0], s));
    if (!harm && tkc_prep_cached(c, g, nb, &rounds)) {
        HIPCHK(hipEventRecord(c->evq[1], s));
    } else {
        rc = tkc_step_reach(c, g, ws);
        if (rc) return rc;
        HIPCHK(hipEventRecord(c->evq[1], s));
        rc = tkc_step_bounds(c, g, ws, nb, &rounds, harm);
        if (rc) return rc;
        if (g->cache_prep && !harm) {
            rc = tkc_prep_store(c, g, nb, rounds);
            if (rc) return rc;
        }
    }
    DevTopk tk = topk_view(ws);
    const TieBuf tb{ws.tieS, ws.tieR, ws.tieI, n};
    if (tkc_launch_topk_init(tk, k, s, ties ? &tb : nullptr)) return tkc_fail(TKC_EDEVICE, "top-k init failed");
    HIPCHK(hipMemsetAsync(ws.stats, 0, 8 * 4 * ST_COUNT, s));
    HIPCHK(hipMemsetAsync(ws.p_vis, 0, 4 * (((size_t)n + 31) / 32), s));
    HIPCHK(hipEventRecord(c->evq[2], s));

    DevGraph dg = g->view();
    DevReach rcv{ws.alpha, ws.omega, g->directed ? ws.scc : nullptr};
    // harmonic bounds order from the largest down for both variants, so the
    // keys bound the value and the stop rule applies
    OrderView ov{ws.ord, ws.key, n, nb || harm};
    BoundsView bv{ws.lnum, ws.lden};
    bv.harm = harm ? 1 : 0;
    // the results' copy, queued inside the last engine's host wait
    bool rb_ready = false;
    auto readback = [&] { return queue_readback(c, k); };
    int64_t* st_plain = ws.stats;
    int64_t* st_batch = ws.stats + ST_COUNT;
    int64_t* st_swarm = ws.stats + 2 * ST_COUNT;
    int64_t* st_tail = ws.stats + 3 * ST_COUNT;
    double ms_eng[3] = {0, 0, 0};
    int32_t nl_eng[3] = {0, 0, 0};
    int grid = 0;
    // the per-workgroup engine has no level-based path
    if (lb && mode == TKC_HYBRID) mode = TKC_BATCHED;
    if (mode == TKC_PLAIN) {
        EngineTimer tm(c, &ms_eng[0], &nl_eng[0]);
        if (tkc_launch_plain(dg, rcv, ov, bv, tk, plain_view(ws), st_plain, nullptr, 0, lbl, c->tune, s, &grid,
                             max_searches))
            return tkc_fail(TKC_EDEVICE, "plain engine launch failed: %s", hipGetErrorString(hipGetLastError()));
        if ((rc = tm.done(readback))) return rc;
        rb_ready = true;
    } else if (mode == TKC_BATCHED) {
        trace_reset(c);
        // one launch, or slices of slice_batches batches (the cursor, stop
        // flag, top k and bounds live in device memory between them)
        const int32_t slice = c->tune.slice_batches > 0 ? c->tune.slice_batches : 0;
        int32_t pos = 0;
        for (;;) {
            {
                EngineTimer tm(c, &ms_eng[1], &nl_eng[1]);
                int e = tkc_launch_batch(dg, rcv, ov, bv, tk, tkc_batch_view(ws), st_batch, nullptr, 0, pos, slice, lbl,
                                         false, nullptr, nullptr, c->tune, s, &grid);
                if (e)
                    return tkc_fail(TKC_EDEVICE, "batched engine launch failed: %s", hipGetErrorString(hipGetLastError()));
                if (!slice) {
                    if ((rc = tm.done(readback))) return rc;
                    rb_ready = true;
                } else if ((rc = tm.done([&] { return queue_stats(c, st_batch); }))) {
                    return rc;
                }
            }
            if (!slice) break;
            int64_t hs[ST_COUNT];
            memcpy(hs, pin_at<int64_t>(ws, st_batch), sizeof(hs));
            if (hs[ST_STOP] || hs[ST_CURSOR] >= n) break;
            pos = (int32_t)hs[ST_CURSOR];
        }
        trace_dump(c, "batched");
    } else {
        // hybrid: batched seed until x is known, then one search per workgroup,
        // then the deferred (large) searches batched; if the per-workgroup
        // engine closed itself (too many deferrals), the rest of the order
        // continues batched from its cursor
        int64_t hs[ST_COUNT];
        trace_reset(c);
        int32_t* small = (int32_t*)ws.small;
        int32_t* pin = (int32_t*)c->pinned;
        SwarmWork sw{};
        sw.vis = ws.s_vis;
        sw.queue = ws.s_queue;
        sw.deferred = ws.s_deferred;
        sw.ndeferred = small + 4;
        sw.cursor = small + 5;
        sw.stop = small + 6;
        sw.nblocks = ws.shape.swarm_blocks;
        sw.qcap = ws.shape.qcap;
        sw.defer_cap = c->tune.batch_width;
        // the seed's cursor and stop flag reach the swarm on the device: no
        // host wait between the two launches
        sw.seed = st_batch;
        {
            const double before = ms_eng[1];
            EngineTimer tm(c, &ms_eng[1], &nl_eng[1]);
            EngineTuning seed = c->tune;
            seed.lanes_cap = seed.seed_lanes;
            if (tkc_launch_batch(dg, rcv, ov, bv, tk, tkc_batch_view(ws), st_batch, nullptr, 0, 0, -1, false,
                                 false, nullptr, nullptr, seed, s, &grid))
                return tkc_fail(TKC_EDEVICE, "batched seed launch failed: %s", hipGetErrorString(hipGetLastError()));
            HIPCHK(hipEventRecord(c->evm, s));
            HIPCHK(hipMemsetAsync(small + 4, 0, 3 * sizeof(int32_t), s));
            if (tkc_launch_swarm(dg, rcv, ov, bv, tk, sw, st_swarm, 0, c->tune, s))
                return tkc_fail(TKC_EDEVICE, "per-workgroup engine launch failed");
            // the seed's counters, the swarm's exit state, and the results in
            // case nothing follows
            if ((rc = tm.done([&] {
                     HIPCHK(hipMemcpyAsync(pin, small + 4, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                     if (int r = queue_stats(c, st_batch)) return r;
                     return readback();
                 })))
                return rc;
            rb_ready = true;
            // split the timed span at the mark between the launches
            float seed_ms = 0.f;
            HIPCHK(hipEventElapsedTime(&seed_ms, c->ev0, c->evm));
            const double span = ms_eng[1] - before;
            const double seed_part = std::min(span, (double)seed_ms);
            ms_eng[1] = before + seed_part;
            ms_eng[2] += span - seed_part;
            nl_eng[2]++;
        }
        memcpy(hs, pin_at<int64_t>(ws, st_batch), sizeof(hs));
        trace_dump(c, "seed");
        const int32_t cursor = (int32_t)hs[ST_CURSOR];
        const bool stopped = hs[ST_STOP] != 0;
        if (!stopped && cursor < n) {
            const int32_t ndef = pin[0], fetched = pin[1], sw_stop = pin[2];
            if (c->ws.trace)
                fprintf(stderr, "trace hybrid: seed cursor %d, swarm deferred %d, fetched %d, stop bits %d\n",
                        cursor, ndef, fetched, sw_stop);
            if (ndef > 0) {
                trace_reset(c);
                EngineTimer tm(c, &ms_eng[1], &nl_eng[1]);
                if (tkc_launch_batch(dg, rcv, ov, bv, tk, tkc_batch_view(ws), st_tail, ws.s_deferred, ndef, 0, 0,
                                     false, false, nullptr, nullptr, c->tune, s, &grid))
                    return tkc_fail(TKC_EDEVICE, "batched tail launch failed");
                if ((rc = tm.done(readback))) return rc;
                trace_dump(c, "tail");
            }
            // every position the cursor handed out was searched, skipped or
            // deferred; without a stop rule firing, the order resumes there
            const int32_t resume = cursor + std::min(fetched, n - cursor);
            if (!(sw_stop & 1) && (sw_stop & 2) && resume < n) {
                trace_reset(c);
                EngineTimer tm(c, &ms_eng[1], &nl_eng[1]);
                if (tkc_launch_batch(dg, rcv, ov, bv, tk, tkc_batch_view(ws), st_batch, nullptr, 0, resume, 0, false,
                                     false, nullptr, nullptr, c->tune, s, &grid))
                    return tkc_fail(TKC_EDEVICE, "batched continuation launch failed");
                if ((rc = tm.done(readback))) return rc;
                trace_dump(c, "rest");
            }
        }
    }
    // the searches end with the last engine's end mark when its host wait
    // already took the results, else here
    hipEvent_t trav_end = c->ev1;
    if (!rb_ready) {
        trav_end = c->evq[3];
        HIPCHK(hipEventRecord(trav_end, s));
    }
    // readback (already in pinned memory when the last engine's wait copied it)
    if (!rb_ready) {
        if ((rc = readback())) return rc;
        HIPCHK(hipStreamSynchronize(s));
    }
    int64_t hstat[4][ST_COUNT];
    memcpy(hstat, pin_at<int64_t>(ws, ws.stats), sizeof(hstat));
    TopkState hst;
    memcpy(&hst, pin_at<TopkState>(ws, ws.tstate), sizeof(hst));
    const int64_t* pS = pin_at<int64_t>(ws, ws.tS);
    const int64_t* pR = pin_at<int64_t>(ws, ws.tR);
    const int32_t* pI = pin_at<int32_t>(ws, ws.tI);
    auto fill_stats = [&]() -> int {
        if (!stats) return TKC_OK;
        for (int e = 0; e < 4; e++) {
            st.m_vis += hstat[e][ST_MVIS];
            st.bfs_started += hstat[e][ST_STARTED];
            st.bfs_exact += hstat[e][ST_EXACT];
            st.bfs_cut += hstat[e][ST_CUT];
            st.skipped += hstat[e][ST_SKIPPED];
            st.deferred += hstat[e][ST_DEFERRED];
            st.max_level = (int32_t)std::max<int64_t>(st.max_level, hstat[e][ST_MAXLEVEL]);
        }
        st.batch_width = c->tune.batch_width;
        st.variant_used = variant;
        st.mode_used = mode;
        st.nb_rounds = rounds;
        // phases from the stream's marks (the readback synchronised it)
        float ph[3] = {0.f, 0.f, 0.f};
        for (int i = 0; i < 3; i++)
            HIPCHK(hipEventElapsedTime(&ph[i], c->evq[i], i < 2 ? c->evq[i + 1] : trav_end));
        st.ms_reach = ph[0];
        st.ms_bounds = ph[1];
        st.ms_traverse = ph[2];
        st.ms_total = now_ms() - t0;
        int best = 0;
        for (int e = 1; e < 3; e++)
            if (ms_eng[e] > ms_eng[best]) best = e;
        st.main_kernel = best;
        st.ms_kernel_main = ms_eng[best];
        st.main_launches = nl_eng[best];
        st.bytes_main = best == 0 ? hstat[0][ST_BYTES]
                                  : (best == 1 ? hstat[1][ST_BYTES] + hstat[3][ST_BYTES] : hstat[2][ST_BYTES]);
        *stats = st;
        return TKC_OK;
    };
    if (hstat[0][ST_CAPPED]) {
        // the plain engine met its search cap: counters only, no answer
        *n_out = 0;
        if ((rc = fill_stats())) return rc;
        return tkc_fail(TKC_ECANCELED, "search cap of %lld searches reached", (long long)max_searches);
    }
    std::vector<int64_t> hS(pS, pS + k), hR(pR, pR + k);
    std::vector<int32_t> hI(pI, pI + k);
    int32_t cnt = std::min(hst.cnt, k);
    if (cnt != k)
        return tkc_fail(TKC_EDEVICE, "internal error: %d results for k = %d", cnt, k);
    if (ties) {
        // entries that left or were refused by the top k and tie with the
        // final k-th farness, by increasing id (all of them have ids above
        // the k-th's: a tied smaller id would precede it)
        if (hst.tcnt > n) return tkc_fail(TKC_EDEVICE, "internal error: tie buffer overflow");
        const int32_t tc = hst.tcnt;
        std::vector<int64_t> tS(tc), tR(tc);
        std::vector<int32_t> tI(tc);
        if (tc) {
            HIPCHK(hipMemcpyAsync(tS.data(), ws.tieS, 8 * (size_t)tc, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(tR.data(), ws.tieR, 8 * (size_t)tc, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(tI.data(), ws.tieI, 4 * (size_t)tc, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        const int64_t Sk = hS[k - 1], Rk = hR[k - 1];
        auto same_farness = [&](int64_t S2, int64_t R2) {
            if (R2 <= 1 || Rk <= 1) return R2 <= 1 && Rk <= 1;
            const unsigned __int128 a = (unsigned __int128)S2 * (unsigned __int128)((Rk - 1) * (Rk - 1));
            const unsigned __int128 b = (unsigned __int128)Sk * (unsigned __int128)((R2 - 1) * (R2 - 1));
            return a == b;
        };
        std::vector<int32_t> extra;
        for (int32_t i = 0; i < tc; i++)
            if (same_farness(tS[i], tR[i])) extra.push_back(i);
        std::sort(extra.begin(), extra.end(), [&](int32_t a, int32_t b) { return tI[a] < tI[b]; });
        const int32_t total = k + (int32_t)extra.size();
        if (total > ties_cap) {
            *n_out = total;
            return tkc_fail(TKC_EINVAL, "%d results (with ties) do not fit cap %d", total, ties_cap);
        }
        for (int32_t i : extra) {
            hS.push_back(tS[i]);
            hR.push_back(tR[i]);
            hI.push_back(tI[i]);
        }
        cnt = total;
    }
    for (int32_t i = 0; i < cnt; i++) {
        ids[i] = hI[i];
        if (harm) {
            // decode harm_enc: the value's bit pattern is HARM_TOP - S
            const int64_t bits = (int64_t)0x7FF0000000000000LL - hS[i];
            double h;
            memcpy(&h, &bits, 8);
            if (farness) farness[i] = h;
            continue;
        }
        if (sum_dist) sum_dist[i] = hS[i];
        if (reach) reach[i] = hR[i];
        if (farness)
            farness[i] = hR[i] <= 1 ? INFINITY
                                    : ((double)(n - 1) * (double)hS[i]) / ((double)(hR[i] - 1) * (double)(hR[i] - 1));
    }
    *n_out = cnt;
    return fill_stats();
}

// AUTO variant: one full search from the highest-degree vertex measures its
// eccentricity; a deep graph (road-like) gets NB + level-based updates,
// a shallow one NB + BFSCut.
int32_t tkc_auto_variant(tkc_ctx* c, tkc_graph* g) {
    if (g->auto_variant) return g->auto_variant;
    std::vector<int32_t> deg(g->n);
    if (hipMemcpy(deg.data(), g->deg, 4 * (size_t)g->n, hipMemcpyDeviceToHost) != hipSuccess)
        return TKC_NB_CUT;
    int32_t src = (int32_t)(std::max_element(deg.begin(), deg.end()) - deg.begin());
    int64_t S = 0, r = 0;
    tkc_stats st;
    int rc = tkc_sums_impl(c, g, &src, 1, &S, &r, &st);
    int32_t v = TKC_NB_CUT;
    if (rc == TKC_OK) {
        double lg = std::log2((double)std::max<int32_t>(g->n, 2));
        if (st.max_level > 64 && st.max_level > 4 * lg) v = TKC_NB_BOUND;
    }
    g->auto_variant = v;
    return v;
}

// ------------------------------------------------------------ inspection
extern "C" int tkc_graph_reach(tkc_graph* g, int64_t* alpha, int64_t* omega, int32_t* scc) {
    if (!g || !alpha || !omega) return tkc_fail(TKC_EINVAL, "NULL argument");
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    int rc = tkc_ws_reserve(c, c->ws, tkc_shape_for(c->tune, g, 1, false));
    if (rc) return rc;
    rc = tkc_step_reach(c, g, c->ws);
    if (rc) return rc;
    if (g->relabeled) {
        // device arrays by stored vertex, outputs by the caller's id
        const size_t n = (size_t)g->n;
        std::vector<int64_t> ha(n), ho(n);
        std::vector<int32_t> hs(g->directed && scc ? n : 0);
        HIPCHK(hipMemcpyAsync(ha.data(), c->ws.alpha, 8 * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(ho.data(), c->ws.omega, 8 * n, hipMemcpyDeviceToHost, c->stream));
        if (hs.size()) HIPCHK(hipMemcpyAsync(hs.data(), c->ws.scc, 4 * n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (size_t v = 0; v < n; v++) {
            const int32_t u = g->h_nid[v];
            alpha[v] = ha[u];
            omega[v] = ho[u];
            if (hs.size()) scc[v] = hs[u];
        }
        return TKC_OK;
    }
    HIPCHK(hipMemcpyAsync(alpha, c->ws.alpha, 8 * (size_t)g->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(omega, c->ws.omega, 8 * (size_t)g->n, hipMemcpyDeviceToHost, c->stream));
    if (scc && g->directed)
        HIPCHK(hipMemcpyAsync(scc, c->ws.scc, 4 * (size_t)g->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TKC_OK;
}

extern "C" int tkc_graph_harmonic_bounds(tkc_graph* g, int32_t variant, double* ub, int32_t* order) {
    if (!g || !ub) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (g->relabeled) return tkc_fail(TKC_EINVAL, "not available for a graph uploaded with TKC_RELABEL");
    if (variant < TKC_DEG_CUT || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "bad variant");
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    int rc = tkc_ws_reserve(c, c->ws, tkc_shape_for(c->tune, g, 1, false));
    if (rc) return rc;
    rc = tkc_step_reach(c, g, c->ws);
    if (rc) return rc;
    rc = tkc_step_bounds(c, g, c->ws, tkc_is_nb(variant), nullptr, true);
    if (rc) return rc;
    const size_t n = g->n;
    std::vector<int64_t> f(n);
    HIPCHK(hipMemcpyAsync(f.data(), c->ws.lnum, 8 * n, hipMemcpyDeviceToHost, c->stream));
    if (order) HIPCHK(hipMemcpyAsync(order, c->ws.ord, 4 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t v = 0; v < n; v++) {
        const int64_t bits = (int64_t)0x7FF0000000000000LL - f[v];
        memcpy(&ub[v], &bits, 8);
    }
    return TKC_OK;
}

extern "C" int tkc_graph_bounds(tkc_graph* g, int32_t variant, int64_t* num, int64_t* den, int32_t* order) {
    if (!g || !num || !den) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (g->relabeled) return tkc_fail(TKC_EINVAL, "not available for a graph uploaded with TKC_RELABEL");
    if (variant < TKC_DEG_CUT || variant > TKC_NB_CUTLB) return tkc_fail(TKC_EINVAL, "bad variant");
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    int rc = tkc_ws_reserve(c, c->ws, tkc_shape_for(c->tune, g, 1, false));
    if (rc) return rc;
    rc = tkc_step_reach(c, g, c->ws);
    if (rc) return rc;
    bool nb = tkc_is_nb(variant);
    rc = tkc_step_bounds(c, g, c->ws, nb, nullptr);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(num, c->ws.lnum, 8 * (size_t)g->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(den, c->ws.lden, 8 * (size_t)g->n, hipMemcpyDeviceToHost, c->stream));
    if (order) HIPCHK(hipMemcpyAsync(order, c->ws.ord, 4 * (size_t)g->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TKC_OK;
}

int tkc_sums_impl(tkc_ctx* c, tkc_graph* g, const int32_t* sources, int32_t count, int64_t* S, int64_t* R,
                  tkc_stats* stout) {
    Workspace& ws = c->ws;
    hipStream_t s = c->stream;
    int rc = tkc_ws_reserve(c, ws, tkc_shape_for(c->tune, g, std::max(1, ws.shape.kcap), ws.shape.lb));
    if (rc) return rc;
    rc = tkc_step_reach(c, g, ws);
    if (rc) return rc;
    int32_t* dsrc = ws.s_deferred;
    HIPCHK(hipMemcpyAsync(dsrc, sources, 4 * (size_t)count, hipMemcpyHostToDevice, s));
    DevTopk tk = topk_view(ws);
    if (tkc_launch_topk_init(tk, 1, s)) return tkc_fail(TKC_EDEVICE, "top-k init failed");
    HIPCHK(hipMemsetAsync(ws.stats, 0, 8 * ST_COUNT, s));
    DevReach rcv{ws.alpha, ws.omega, g->directed ? ws.scc : nullptr};
    OrderView ov{ws.ord, ws.key, 0, false};
    BoundsView bv{ws.lnum, ws.lden};
    int grid = 0;
    std::lock_guard<std::mutex> lk(tkc_coop_mutex());
    if (tkc_launch_batch(g->view(), rcv, ov, bv, tk, tkc_batch_view(ws), ws.stats, dsrc, count, 0, 0, false, true,
                         ws.b_outS, ws.b_outR, c->tune, s, &grid))
        return tkc_fail(TKC_EDEVICE, "batched engine launch failed");
    HIPCHK(hipMemcpyAsync(S, ws.b_outS, 8 * (size_t)count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(R, ws.b_outR, 8 * (size_t)count, hipMemcpyDeviceToHost, s));
    int64_t hs[ST_COUNT];
    HIPCHK(hipMemcpyAsync(hs, ws.stats, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (stout) {
        memset(stout, 0, sizeof(*stout));
        stout->m_vis = hs[ST_MVIS];
        stout->max_level = (int32_t)hs[ST_MAXLEVEL];
        stout->bfs_started = hs[ST_STARTED];
        stout->bfs_exact = hs[ST_EXACT];
    }
    return TKC_OK;
}

extern "C" int tkc_graph_sums(tkc_graph* g, const int32_t* sources, int32_t count, int64_t* S, int64_t* R) {
    if (!g || !sources || !S || !R || count < 0) return tkc_fail(TKC_EINVAL, "bad argument");
    if (g->relabeled) return tkc_fail(TKC_EINVAL, "not available for a graph uploaded with TKC_RELABEL");
    for (int32_t i = 0; i < count; i++)
        if (sources[i] < 0 || sources[i] >= g->n) return tkc_fail(TKC_EINVAL, "source %d out of range", sources[i]);
    HIPCHK(hipSetDevice(g->ctx->device));
    // the source list shares n-sized buffers: chunks of at most n
    for (int64_t off = 0; off < count; off += g->n) {
        const int32_t c = (int32_t)std::min<int64_t>(count - off, g->n);
        int rc = tkc_sums_impl(g->ctx, g, sources + off, c, S + off, R + off, nullptr);
        if (rc) return rc;
    }
    return TKC_OK;
}

extern "C" int tkc_graph_lb_update(tkc_graph* g, const int32_t* sources, int32_t count, int64_t* num,
                                   int64_t* den) {
    if (!g || !sources || !num || !den || count < 0) return tkc_fail(TKC_EINVAL, "bad argument");
    if (g->relabeled) return tkc_fail(TKC_EINVAL, "not available for a graph uploaded with TKC_RELABEL");
    for (int32_t i = 0; i < count; i++)
        if (sources[i] < 0 || sources[i] >= g->n) return tkc_fail(TKC_EINVAL, "source %d out of range", sources[i]);
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    Workspace& ws = c->ws;
    int rc = tkc_ws_reserve(c, ws, tkc_shape_for(c->tune, g, 1, true));
    if (rc) return rc;
    rc = tkc_step_reach(c, g, ws);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(ws.lnum, num, 8 * (size_t)g->n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws.lden, den, 8 * (size_t)g->n, hipMemcpyHostToDevice, s));
    DevTopk tk = topk_view(ws);
    if (tkc_launch_topk_init(tk, 1, s)) return tkc_fail(TKC_EDEVICE, "top-k init failed");
    HIPCHK(hipMemsetAsync(ws.stats, 0, 8 * ST_COUNT, s));
    DevReach rcv{ws.alpha, ws.omega, g->directed ? ws.scc : nullptr};
    OrderView ov{ws.ord, ws.key, 0, false};
    BoundsView bv{ws.lnum, ws.lden};
    int grid = 0;
    for (int64_t off = 0; off < count; off += g->n) {
        const int32_t cnt = (int32_t)std::min<int64_t>(count - off, g->n);
        HIPCHK(hipMemcpyAsync(ws.s_deferred, sources + off, 4 * (size_t)cnt, hipMemcpyHostToDevice, s));
        std::lock_guard<std::mutex> lk(tkc_coop_mutex());
        if (tkc_launch_batch(g->view(), rcv, ov, bv, tk, tkc_batch_view(ws), ws.stats, ws.s_deferred, cnt, 0, 0,
                             true, true, ws.b_outS, ws.b_outR, c->tune, s, &grid))
            return tkc_fail(TKC_EDEVICE, "batched engine launch failed");
        HIPCHK(hipStreamSynchronize(s));
    }
    HIPCHK(hipMemcpyAsync(num, ws.lnum, 8 * (size_t)g->n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(den, ws.lden, 8 * (size_t)g->n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return TKC_OK;
}

extern "C" int tkc_graph_harmonic_lb_update(tkc_graph* g, const int32_t* sources, int32_t count, double* ub) {
    if (!g || !sources || !ub || count < 0) return tkc_fail(TKC_EINVAL, "bad argument");
    if (g->relabeled) return tkc_fail(TKC_EINVAL, "not available for a graph uploaded with TKC_RELABEL");
    for (int32_t i = 0; i < count; i++)
        if (sources[i] < 0 || sources[i] >= g->n) return tkc_fail(TKC_EINVAL, "source %d out of range", sources[i]);
    for (int32_t v = 0; v < g->n; v++)
        if (!(ub[v] >= 0.0) || ub[v] == INFINITY) return tkc_fail(TKC_EINVAL, "bound %d is not finite and >= 0", v);
    tkc_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    Workspace& ws = c->ws;
    int rc = tkc_ws_reserve(c, ws, tkc_shape_for(c->tune, g, 1, true));
    if (rc) return rc;
    rc = tkc_step_reach(c, g, ws);
    if (rc) return rc;
    const size_t n = g->n;
    std::vector<int64_t> f(n), one(n, 1);
    for (size_t v = 0; v < n; v++) {
        int64_t bits;
        memcpy(&bits, &ub[v], 8);
        f[v] = (int64_t)0x7FF0000000000000LL - bits;
    }
    HIPCHK(hipMemcpyAsync(ws.lnum, f.data(), 8 * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ws.lden, one.data(), 8 * n, hipMemcpyHostToDevice, s));
    DevTopk tk = topk_view(ws);
    if (tkc_launch_topk_init(tk, 1, s)) return tkc_fail(TKC_EDEVICE, "top-k init failed");
    HIPCHK(hipMemsetAsync(ws.stats, 0, 8 * ST_COUNT, s));
    DevReach rcv{ws.alpha, ws.omega, g->directed ? ws.scc : nullptr};
    OrderView ov{ws.ord, ws.key, 0, false};
    BoundsView bv{ws.lnum, ws.lden};
    bv.harm = 1;
    int grid = 0;
    for (int64_t off = 0; off < count; off += g->n) {
        const int32_t cnt = (int32_t)std::min<int64_t>(count - off, g->n);
        HIPCHK(hipMemcpyAsync(ws.s_deferred, sources + off, 4 * (size_t)cnt, hipMemcpyHostToDevice, s));
        std::lock_guard<std::mutex> lk(tkc_coop_mutex());
        if (tkc_launch_batch(g->view(), rcv, ov, bv, tk, tkc_batch_view(ws), ws.stats, ws.s_deferred, cnt, 0, 0,
                             1, true, ws.b_outS, ws.b_outR, c->tune, s, &grid))
            return tkc_fail(TKC_EDEVICE, "batched engine launch failed");
        HIPCHK(hipStreamSynchronize(s));
    }
    HIPCHK(hipMemcpyAsync(f.data(), ws.lnum, 8 * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t v = 0; v < n; v++) {
        const int64_t bits = (int64_t)0x7FF0000000000000LL - f[v];
        memcpy(&ub[v], &bits, 8);
    }
    return TKC_OK;
}

// ------------------------------------------- cached preprocessing (serving)
static size_t prep_bytes(int32_t n) { return (size_t)n * 44 + 8 * 256; }

bool tkc_prep_cached(tkc_ctx* c, tkc_graph* g, bool nb, int32_t* rounds) {
    tkc_graph::Prep* p;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        p = &g->prep[nb ? 1 : 0];
        if (!g->cache_prep || !p->ready) return false;
    }
    size_t n = (size_t)g->n;
    char* b = (char*)p->base;
    Workspace& ws = c->ws;
    hipStream_t s = c->stream;
    bool ok = hipMemcpyAsync(ws.alpha, b, 8 * n, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(ws.omega, b + 8 * n, 8 * n, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(ws.lnum, b + 16 * n, 8 * n, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(ws.lden, b + 24 * n, 8 * n, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(ws.ord, b + 32 * n, 4 * n, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              hipMemcpyAsync(ws.key, b + 36 * n, 4 * n, hipMemcpyDeviceToDevice, s) == hipSuccess &&
              (!g->directed || hipMemcpyAsync(ws.scc, b + 40 * n, 4 * n, hipMemcpyDeviceToDevice, s) == hipSuccess);
    if (!ok) return false;
    *rounds = p->rounds;
    return true;
}

int tkc_prep_store(tkc_ctx* c, tkc_graph* g, bool nb, int32_t rounds) {
    std::lock_guard<std::mutex> lk(g->mu);
    tkc_graph::Prep& p = g->prep[nb ? 1 : 0];
    if (p.ready) return TKC_OK;
    size_t n = (size_t)g->n;
    if (!p.base && hipMalloc(&p.base, prep_bytes(g->n)) != hipSuccess) {
        hipGetLastError();
        p.base = nullptr;
        return TKC_OK;   // no cache: queries recompute
    }
    char* b = (char*)p.base;
    Workspace& ws = c->ws;
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(b, ws.alpha, 8 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b + 8 * n, ws.omega, 8 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b + 16 * n, ws.lnum, 8 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b + 24 * n, ws.lden, 8 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b + 32 * n, ws.ord, 4 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b + 36 * n, ws.key, 4 * n, hipMemcpyDeviceToDevice, s));
    if (g->directed) HIPCHK(hipMemcpyAsync(b + 40 * n, ws.scc, 4 * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    p.rounds = rounds;
    p.ready = true;
    return TKC_OK;
}

extern "C" const char* tkc_last_error(void) { return g_err.c_str(); }
extern "C" const char* tkc_version(void) { return "tkc 0.1 gfx950"; }
