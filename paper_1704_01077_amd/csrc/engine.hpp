// Host-side view of the device data used by the kernels, and the launch
// entry points each .hip file provides to the driver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

struct TopkState;
struct XRec;

struct DevGraph {
    int32_t n;
    int64_t m;            // arcs
    bool directed;
    const int32_t* rp;    // out-arcs CSR
    const int32_t* ci;
    const int32_t* rrp;   // in-arcs CSR (== rp/ci when undirected)
    const int32_t* rci;
    int32_t* deg;         // out-degree
    // vertices with more than HEAVY_DEG out-arcs, ascending, and their arcs cut
    // into chunks of CHUNK_ARCS: heavy vertex i owns chunks [hcb[i], hcb[i+1])
    const int32_t* heavy;
    int32_t nheavy;
    const int32_t* hcb;
    const int32_t* ch_beg;
    const int32_t* ch_end;
    const int32_t* ch_vtx;   // owner of each chunk
    int32_t nchunks;
    // in-arc chunks of the vertices with more than HEAVY_DEG in-arcs (pull
    // steps; the same table as above for undirected graphs)
    const int32_t* rch_vtx;
    const int32_t* rch_beg;
    const int32_t* rch_end;
    int32_t rnchunks;
    // in-arc chunks of the hubs only (more than HUB_IN_DEG in-arcs): the
    // batched engine's pull sends every other vertex through its
    // edge-balanced path, which shares a wave's in-arcs over all its lanes
    const int32_t* bch_vtx;
    const int32_t* bch_beg;
    const int32_t* bch_end;
    int32_t bnchunks;
    // vertices with HEAVY_DEG < in-degree <= HUB_IN_DEG, ascending, packed
    // into segments of at most 64 vertices and MID_ARCS in-arcs (a segment
    // of one vertex may exceed it); segment s is mid_vtx[mseg[s] .. mseg[s+1])
    const int32_t* mid_vtx;
    const int32_t* mseg;
    int32_t nmseg;
    // relabelled graphs (TKC_RELABEL): the caller's id of each vertex and
    // the vertex of each caller id; null otherwise (ids are the caller's)
    const int32_t* oid = nullptr;
    const int32_t* nid = nullptr;
};
// the caller's id of vertex v (ties of the exact order break on it)
#define TKC_OID(g, v) ((g).oid ? (g).oid[v] : (v))
#define HEAVY_DEG 64
#define CHUNK_ARCS 512
#define HUB_IN_DEG 1024
#define MID_ARCS 1024

// reachability and bounds of one query
struct DevReach {
    const int64_t* alpha;   // alpha = omega = r when known
    const int64_t* omega;
    const int32_t* scc;     // directed only (same-SCC rule of the LB update)
};

struct DevTopk {
    TopkState* st;
    XRec* ring;
    int64_t* S;
    int64_t* R;
    int32_t* I;
};

// counters the engines add to (device, int64 each)
enum {
    ST_MVIS = 0, ST_STARTED, ST_EXACT, ST_CUT, ST_SKIPPED, ST_DEFERRED, ST_MAXLEVEL, ST_CURSOR,
    ST_STOP, ST_BYTES, ST_CAPPED, ST_COUNT
};

struct OrderView {
    const int32_t* ord;      // vertex per position
    const uint32_t* key;     // sorted key per position
    int32_t count;           // positions available
    bool key_is_bound;       // NB keys bound the farness; Deg keys only order
};

struct BoundsView {
    int64_t* num;            // current lower bound num/den (den 0 = +inf)
    int64_t* den;
    int32_t harm = 0;        // harmonic centrality: bounds, cuts and results
                             // carry harm_enc of an upper bound / value
};

struct EngineTuning {
    int32_t td_bu_alpha = 14;    // push -> pull when frontier arcs > unexplored arcs / alpha
    int32_t bu_td_beta = 24;     // pull -> push when frontier vertices < n / beta
    int32_t batch_alpha = 14;    // the same push -> pull rule for batched searches
    int32_t batch_width = 64;
    int32_t swarm_qcap = 65536;
    int32_t seed_lanes = 0;      // lanes of the hybrid mode's seed batch (0: batch_width)
    int32_t lanes_cap = 0;       // lanes used per batch in one launch (0: batch_width)
    int32_t blocks_per_cu = 2;   // workgroups per CU of the persistent kernels
    int32_t mode = 1;            // preferred mode (TKC_BATCHED) for TKC_MODE_AUTO
    int32_t slice_batches = 0;   // batched searches per launch (0: all in one); servers
                                 // slice long queries so other requests interleave
};
// workgroups of a persistent grid for a graph of n vertices: the whole GPU
// for big graphs, fewer (cheaper grid barriers) for small ones
static inline int tkc_grid_for(int cus, int per, int32_t n) {
    int64_t want = ((int64_t)n + 2047) / 2048;
    if (want < 64) want = 64;
    const int64_t full = (int64_t)cus * per;
    return (int)(want < full ? want : full);
}

// k_topk.hip: the current device's compute units, and how many workgroups
// of `block` threads of kernel fn fit on one of them (both asked of the
// runtime once per device and kernel, then cached); -1 on error
int tkc_cu_count();
int tkc_occupancy(const void* fn, int block);

// k_prep.hip
int tkc_launch_degrees(const DevGraph& g, hipStream_t s);
// size holds n+2 int64; in_giant n bytes; sample_host is unused (the
// dominant component is found on the device)
int tkc_launch_cc(const DevGraph& g, int32_t* parent, int64_t* size, int64_t* alpha, int64_t* omega,
                  uint8_t* in_giant, int32_t* sample_host, hipStream_t s);
// gbuf holds 3n int64 and then 2n int32; partial holds nchunks uint64 and
// at least n/64 int32; nfin_dev the finish counters (1,057 int32).  Returns
// the number of rounds, -1 on error.  hub (n doubles, may be null): also
// the walk-count upper bound on the harmonic centrality
// fin (may be null): the caller's work on the final bounds (order keys and
// the like), queued before the check that follows a tail round so that one
// host wait covers both; *fin_done says whether the rounds ended at such a
// check (else the bounds changed after fin ran, and the caller runs it again)
int tkc_launch_nb(const DevGraph& g, const int64_t* alpha, const int64_t* omega, int64_t* gbuf, int64_t* sum,
                  int64_t* vis, uint8_t* flags, int64_t* num, int64_t* den, uint64_t* partial,
                  int32_t* nfin_dev, int32_t* nfin_host, hipStream_t s, double* hub = nullptr,
                  const std::function<int()>* fin = nullptr, bool* fin_done = nullptr);
// harmonic centrality bounds and order keys: from hub (walk counts) when
// given, else the degree bound
int tkc_launch_harm_bounds(const DevGraph& g, const int64_t* omega, const double* hub, int64_t* num,
                           int64_t* den, uint32_t* key, int32_t* val, hipStream_t s);
int tkc_launch_deg_bounds(const DevGraph& g, const int64_t* omega, int64_t* num, int64_t* den,
                          uint32_t* key, int32_t* val, hipStream_t s);
int tkc_launch_nb_keys(int32_t n, const int64_t* num, const int64_t* den, uint32_t* key,
                       int32_t* val, hipStream_t s);

// k_scc.hip: alpha / omega / topological SCC ids of a directed graph.
// 0 on success (*seq_used = 1 when a one-thread pass finished long chains),
// -2 when its scratch arena cannot be allocated, -3 when the caller's arena
// is too small (*need: the bytes it takes), -1 on a device error.  arena
// NULL: it allocates its scratch and frees it before returning.
// pinned: 256 bytes of pinned host memory.
int tkc_device_alpha_omega(const DevGraph& g, int64_t* alpha, int64_t* omega, int32_t* scc_topo, void* pinned,
                           hipStream_t s, int* seq_used, void* arena = nullptr, size_t arena_bytes = 0,
                           size_t* need = nullptr);

// k_sort.hip: stable ascending sort of (key, val) pairs; the result ends in
// keys/vals.  tmp_* hold n items, hist holds sort_hist_words(n) int32.
int64_t tkc_sort_hist_words(int32_t n);
int tkc_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* tmp_keys, int32_t* tmp_vals,
                   int32_t n, int32_t* hist, uint32_t* mask_dev, uint32_t* mask_host,
                   hipStream_t s);
// the same with 8-bit digits (the processing order): hist holds
// tkc_sort8_hist_words(n) int32
int64_t tkc_sort8_hist_words(int32_t n);
// known_mask: the OR and AND of the keys already in host memory (from
// tkc_sort_mask and a host wait), else null: the sort finds them itself
int tkc_sort_pairs8(uint32_t* keys, int32_t* vals, uint32_t* tmp_keys, int32_t* tmp_vals,
                    int32_t n, int32_t* hist, uint32_t* mask_dev, uint32_t* mask_host,
                    hipStream_t s, const uint32_t* known_mask = nullptr);
// queue the OR and AND of n keys into mask_dev[0..1] and their copy to the
// pinned mask_host[0..1] (no wait)
int tkc_sort_mask(const uint32_t* keys, int32_t n, uint32_t* mask_dev, uint32_t* mask_host, hipStream_t s);

// k_topk.hip
// all-ties mode: buffers for the entries that leave or are refused by the top k
struct TieBuf {
    int64_t* S;
    int64_t* R;
    int32_t* I;
    int32_t cap;
};
int tkc_launch_topk_init(DevTopk t, int32_t k, hipStream_t s, const TieBuf* tb = nullptr);

// k_plain.hip: one source at a time on the whole GPU (cooperative kernel).
struct PlainWork {
    uint32_t* vis;       // n bits
    uint32_t* fb;        // 3 x n bits (frontier bitmaps of pull steps)
    int32_t* ql;         // queue of light vertices (n)
    int32_t* qh;         // queue of heavy vertices (n)
    int32_t* qg;         // chunk queue: owners [0, ccap), first arcs [ccap, 2 ccap)
    int64_t ccap;
    int64_t* ctr;        // 3 x 8 level counters
    int32_t* lvl;        // distance from the source (level-based updates)
    int64_t* levcnt;     // vertices per level (n + 2)
    int64_t* levtab;     // Lev(i) table (n + 2)
    uint32_t* bar;       // grid barrier state (zeroed once)
};
// lb_mode: 0 cut searches (Cut variants), 1 complete searches feeding
// level-based updates (Bound variants), 2 both: shallow searches may be cut
// (cut_allowed), and the complete ones feed level-based updates
// max_searches > 0: stop before the search that would exceed it and set
// stats[ST_CAPPED] (the top k is then incomplete)
int tkc_launch_plain(const DevGraph& g, DevReach rc, OrderView ov, BoundsView bv, DevTopk tk,
                     PlainWork w, int64_t* stats, const int32_t* list, int32_t list_count,
                     int lb_mode, const EngineTuning& tune, hipStream_t s, int* grid_out,
                     int64_t max_searches = 0);

// k_batch.hip: W sources per launch, one bit lane each (cooperative kernel).
struct BatchWork {
    uint64_t* vis;       // n * nw words
    uint64_t* frt0;      // n * nw
    uint64_t* frt1;      // n * nw
    uint64_t* nxt;       // n * nw
    int32_t* list;       // level lists: 8 n vertex entries (4 slots x light/heavy) + 4 ccap chunk entries
    int64_t ccap;        // chunk entries per list
    int32_t* touched;    // every vertex touched in the batch (for clearing), cap n
    int64_t* ctr;        // per-lane level counters, 3 * 2 * 256 + misc
    int64_t* lanes;      // per-lane state
    uint16_t* lvl;       // n * W levels (level-based updates), may be null
    int64_t* hist;       // LCAP * W vertices per level per lane
    int64_t* levtab;     // LCAP * W Lev tables
    int32_t lcap;
    int32_t* cand;       // selected candidates of a batch (W)
    int32_t* cand_req;   // the request of each candidate (W; packed launches)
    int64_t* trace;      // optional per-level records (16 int64 from word 8), [0] = count
    int64_t trace_cap;
    uint32_t* bar;       // grid barrier state (zeroed once)
};
// One request of a packed launch: a top-k query on one member of a union
// graph (the members' vertices renumbered by adding `off`).  The views are
// the member's own, in its own vertex ids; the top k is the request's.
struct PackReq {
    int32_t off;             // union id of the member's vertex 0
    int32_t n;               // the member's vertex count (its order's length)
    OrderView ov;
    BoundsView bv;
    DevReach rc;
    DevTopk tk;
};
#define TKC_PACK_MAXREQ 64

int tkc_launch_batch(const DevGraph& g, DevReach rc, OrderView ov, BoundsView bv, DevTopk tk,
                     BatchWork w, int64_t* stats, const int32_t* list, int32_t list_count,
                     int32_t start_pos, int32_t max_batches, int lb_mode, bool no_cut,
                     int64_t* out_S, int64_t* out_r, const EngineTuning& tune, hipStream_t s,
                     int* grid_out, const PackReq* preq = nullptr, int32_t npreq = 0);

// k_swarm.hip: one search per workgroup for short cut searches.
struct SwarmWork {
    uint32_t* vis;       // nblocks * words_per_block
    int32_t* queue;      // nblocks * qcap
    int32_t* deferred;   // n
    int32_t* ndeferred;  // 1
    int32_t* cursor;     // 1
    int32_t* stop;       // 1: bit 0 stop rule fired, bit 1 engine closed
    int32_t nblocks;
    int32_t qcap;
    int32_t defer_cap;   // deferrals after which the engine closes itself
    // counters of the batch launched just before (its cursor is the start
    // position, its stop flag ends the engine at once), or null: start_pos
    const int64_t* seed;
};
int tkc_launch_swarm(const DevGraph& g, DevReach rc, OrderView ov, BoundsView bv, DevTopk tk,
                     SwarmWork w, int64_t* stats, int32_t start_pos, const EngineTuning& tune,
                     hipStream_t s);
int tkc_swarm_max_blocks(int block);
