// Plain engine: the candidates of Alg. 1 are searched one at a time, each
// search spread over the whole GPU.  One cooperative (persistent) launch
// walks the candidate order; every level of a search is one grid-wide phase
// followed by a grid barrier, so there is no host round trip per level.
//
// Per search (updateBoundsBFSCut, Sect. 6, or updateBoundsLB, Sect. 7):
//   - level-synchronous BFS; push steps expand the frontier queue (light
//     vertices one per lane, heavy vertices one per wave), pull steps scan
//     the unvisited vertices' in-arcs against a frontier bitmap (Beamer's
//     direction switch);
//   - after each level the exact counts n_D, S_D and the out-degree sum U of
//     the level give the BFSCut bound, checked against the current k-th
//     farness x in the exact (farness, id) order;
//   - Bound variants search to the end and then raise the bounds of every
//     reached vertex with the level-based bound (Eq. 4 / Eq. 5).
// Control decisions are computed redundantly by every thread from values
// read after a barrier, so all workgroups take the same path.
#include "dev_common.hpp"
#include "engine.hpp"

#define PB 256
#define CS 8   // counters per level parity: found, degree sum, light/heavy/chunk appends

struct PlainArgs {
    DevGraph g;
    DevReach rc;
    OrderView ov;
    BoundsView bv;
    DevTopk tk;
    PlainWork w;
    int64_t* stats;
    const int32_t* list;
    int32_t list_count;
    int32_t lb_mode;
    int32_t alpha_td;
    int32_t beta_bu;
    int64_t max_searches;   // 0: no cap
    uint32_t* bar;
};

TKC_DEV int64_t shfl64(int64_t v, int src) {
    int32_t lo = __shfl((int32_t)(v & 0xffffffff), src, 64);
    int32_t hi = __shfl((int32_t)(v >> 32), src, 64);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}
TKC_DEV uint64_t lanes_below() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// wave-aggregated append of newly found vertices: light ones to ql, heavy
// ones to qh and their arc chunks (owner, first arc) to qcu/qcb.  The
// level's appends count from zero in its own counters cnts[0..2] on top of
// the segment ends base[0..2], so the queue ends every workgroup reads after
// the barrier never move under it.
TKC_DEV void q_append(bool isnew, int32_t w, int32_t dw, int32_t* ql, int32_t* qh, int32_t* qcu,
                      int32_t* qcb, const int32_t* rp, int64_t* cnts, const int64_t* base) {
    bool hv = isnew && dw > HEAVY_DEG;
    bool lt = isnew && !hv;
    uint64_t ml = __ballot(lt), mh = __ballot(hv);
    if ((ml | mh) == 0) return;
    int32_t nck = hv ? (dw + CHUNK_ARCS - 1) / CHUNK_ARCS : 0;
    int32_t pre = nck;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(pre, o, 64);
        if (lane_id() >= o) pre += y;
    }
    int leader = __ffsll((long long)__ballot(1)) - 1;
    int32_t tot = __shfl(pre, 63, 64);
    pre -= nck;
    int64_t bl = 0, bh = 0, bc = 0;
    if (lane_id() == leader) {
        if (ml) bl = fadd_rlx(&cnts[0], (int64_t)__popcll(ml));
        if (mh) {
            bh = fadd_rlx(&cnts[1], (int64_t)__popcll(mh));
            bc = fadd_rlx(&cnts[2], (int64_t)tot);
        }
    }
    uint64_t below = lanes_below();
    bl = shfl64(bl, leader) + base[0];
    bh = shfl64(bh, leader) + base[1];
    bc = shfl64(bc, leader) + base[2];
    if (lt) ql[bl + __popcll(ml & below)] = w;
    if (hv) {
        qh[bh + __popcll(mh & below)] = w;
        int32_t b0 = rp[w];
        for (int32_t j = 0; j < nck; j++) {
            qcu[bc + pre + j] = w;
            qcb[bc + pre + j] = b0 + j * CHUNK_ARCS;
        }
    }
}

// test-and-set of a visited bit; true for the single caller that sets it
// (the plain pre-read may be stale, but bits only turn on during a search,
// so a set bit seen there is really set)
TKC_DEV bool visit(uint32_t* vis, int32_t w) {
    uint32_t bit = 1u << (w & 31);
    if (vis[w >> 5] & bit) return false;
    uint32_t old = for_rlx(&vis[w >> 5], bit);
    return !(old & bit);
}

// level table of the level-based bound from per-level counts gamma_0..maxD
// (gamma_0 = 1 counts the source): Lev(1) from the definition, then the
// recurrence of Lemma 7.2 (undirected) or its one-sided form for Eq. 5.
TKC_DEV void lev_table(const int64_t* gam, int64_t maxD, int64_t r, bool directed, int64_t* lev) {
    int64_t L = -2;
    for (int64_t j = 0; j <= maxD; j++) {
        int64_t t = j > 1 ? j - 1 : 1 - j;
        L += (t <= 1 ? 2 : t) * gam[j];
    }
    lev[1] = L;
    int64_t pre = 0;   // sum of gamma_j for j <= i+1, maintained incrementally
    for (int64_t j = 0; j <= 2 && j <= maxD; j++) pre += gam[j];
    int64_t low = 0;   // sum of gamma_j for j < i-2
    for (int64_t i = 2; i <= maxD; i++) {
        if (i + 1 <= maxD) pre += gam[i + 1];
        if (i - 3 >= 0) low += gam[i - 3];
        int64_t high = r - pre;   // sum_{j > i+1} gamma_j
        lev[i] = lev[i - 1] + (directed ? 0 : low) - high;
    }
}

__global__ void __launch_bounds__(PB) k_plain(PlainArgs a) {
    const int32_t n = a.g.n;
    const bool dir = a.g.directed;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nwaves = nthreads / 64;
    const int64_t gwave = gtid / 64;
    const int lane = lane_id();
    const bool boss = (blockIdx.x == 0 && threadIdx.x == 0);
    const int32_t* __restrict__ rp = a.g.rp;
    const int32_t* __restrict__ ci = a.g.ci;
    const int32_t* __restrict__ deg = a.g.deg;
    // ctr[p*CS + 0..4], p = level % 3: vertices found, their degree sum,
    // light, heavy and chunk queue appends of that level
    int64_t* ctr = a.w.ctr;
    int32_t* const qcu = a.w.qg;
    int32_t* const qcb = a.w.qg + a.w.ccap;
    uint32_t* vis = a.w.vis;
    const int64_t words = ((int64_t)n + 31) / 32;
    const int32_t count = a.list ? a.list_count : a.ov.count;
    int64_t* stats = a.stats;

    int32_t pos;
    int64_t searches = 0;   // replicated: every workgroup takes the same path
    for (pos = 0; pos < count; pos++) {
        const int32_t v = a.list ? a.list[pos] : a.ov.ord[pos];
        const XVal x = read_x(a.tk.st, a.tk.ring);
        if (!a.list) {
            uint32_t key = a.ov.key[pos];
            bool stop = a.bv.harm ? key_stops_h(key, x)
                                  : (a.ov.key_is_bound ? key_stops(key, x) : (key == 0xffffffffu && x.den != 0));
            if (stop) {
                if (boss) stats[ST_STOP] = 1;
                break;
            }
        }
        if (lex_after(a.bv.num[v], a.bv.den[v], TKC_OID(a.g, v), x.num, x.den, x.id)) {
            if (boss) stats[ST_SKIPPED]++;
            continue;
        }
        const int64_t av = a.rc.alpha[v], ov = a.rc.omega[v];
        if (ov <= 1) {   // reaches nothing: S = 0, r = 1, farness +inf
            if (boss) {
                stats[ST_STARTED]++;
                stats[ST_EXACT]++;
                if (a.bv.harm) topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, harm_enc(0.0), 2, TKC_OID(a.g, v));
                else topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, 0, 1, TKC_OID(a.g, v));
            }
            grid_barrier(a.bar, gridDim.x);
            continue;
        }
        if (a.max_searches > 0 && searches >= a.max_searches) {
            if (boss) stats[ST_CAPPED] = 1;
            break;
        }
        searches++;
        const int64_t dv = deg[v];
        if (boss) {
            for (int q = 0; q < 3 * CS; q++) ctr[q] = 0;
            for_rlx(&vis[v >> 5], 1u << (v & 31));
            if (dv > HEAVY_DEG) {
                a.w.qh[0] = v;
                int32_t j = 0;
                for (int32_t b = rp[v]; b < rp[v + 1]; b += CHUNK_ARCS, j++) { qcu[j] = v; qcb[j] = b; }
            } else {
                a.w.ql[0] = v;
            }
            if (a.lb_mode) { a.w.lvl[v] = 0; a.w.levcnt[0] = 1; }
        }
        grid_barrier(a.bar, gridDim.x);

        int64_t D = 0, nD = 1, SD = 0;
        double H = 0.0;   // harmonic centrality so far (levels 1..D)
        int64_t U = dv, mf = dv, nf = 1, mdisc = dv;
        // frontier segments [st[c], en[c]) of the light, heavy and chunk queues
        int64_t st[3] = {0, 0, 0}, en[3] = {0, 0, 0};
        if (dv > HEAVY_DEG) { en[1] = 1; en[2] = (dv + CHUNK_ARCS - 1) / CHUNK_ARCS; }
        else en[0] = 1;
        bool bu = false, used_bu = false;
        int status = 0;   // 1 exact, 2 cut
        int64_t mvis = 0, bytes = 0;
        for (;;) {
            if (nf == 0) { status = 1; break; }
            if (cut_allowed(a.lb_mode, D)) {
                int64_t bn, bd;
                if (a.bv.harm) harm_cut_bound(H, nD, U, D, ov, &bn, &bd);
                else cut_bound(SD, nD, U, D, av, ov, &bn, &bd);
                if (lex_after(bn, bd, TKC_OID(a.g, v), x.num, x.den, x.id)) { status = 2; break; }
            }
            // direction (Beamer): pull when the frontier's arcs outweigh the
            // unexplored ones, push again once the frontier is small
            bool want_bu = bu ? (nf >= (int64_t)n / a.beta_bu)
                              : (mf > (a.g.m - mdisc) / a.alpha_td && nf > 64);
            if (want_bu && !bu) {
                // frontier bitmap of level D from the queue segments
                for (int64_t q = gtid; q < 3 * words; q += nthreads) a.w.fb[q] = 0;
                grid_barrier(a.bar, gridDim.x);
                uint32_t* fcur = a.w.fb + (D % 3) * words;
                for (int64_t i = gtid; i < en[0] - st[0]; i += nthreads) {
                    int32_t u = a.w.ql[st[0] + i];
                    for_rlx(&fcur[u >> 5], 1u << (u & 31));
                }
                for (int64_t i = gtid; i < en[1] - st[1]; i += nthreads) {
                    int32_t u = a.w.qh[st[1] + i];
                    for_rlx(&fcur[u >> 5], 1u << (u & 31));
                }
                grid_barrier(a.bar, gridDim.x);
                used_bu = true;
            }
            bu = want_bu;
            mvis += mf;
            bytes += 8 * mf + 12 * nf;
            const int p = (int)(D % 3);
            int64_t my_cnt = 0, my_deg = 0;
            if (!bu) {
                // push: light frontier vertices, one per lane
                for (int64_t base = gwave * 64; base < en[0] - st[0]; base += nwaves * 64) {
                    int64_t i = base + lane;
                    int32_t e = 0, end = 0;
                    if (i < en[0] - st[0]) {
                        int32_t u = a.w.ql[st[0] + i];
                        e = rp[u]; end = rp[u + 1];
                    }
                    while (__any(e < end)) {
                        bool isnew = false;
                        int32_t w = 0, dw = 0;
                        if (e < end) {
                            w = ci[e]; e++;
                            if (visit(vis, w)) { isnew = true; dw = deg[w]; }
                        }
                        if (isnew) {
                            my_cnt++; my_deg += dw;
                            if (a.lb_mode) a.w.lvl[w] = (int32_t)(D + 1);
                        }
                        q_append(isnew, w, dw, a.w.ql, a.w.qh, qcu, qcb, rp, &ctr[p * CS + 2], en);
                    }
                }
                // push: heavy frontier vertices, one wave per chunk of arcs
                for (int64_t c = gwave; c < en[2] - st[2]; c += nwaves) {
                    int32_t u = qcu[st[2] + c];
                    int32_t b = qcb[st[2] + c];
                    int32_t end = b + CHUNK_ARCS < rp[u + 1] ? b + CHUNK_ARCS : rp[u + 1];
                    for (int32_t e0 = b; e0 < end; e0 += 64) {
                        int32_t e = e0 + lane;
                        bool isnew = false;
                        int32_t w = 0, dw = 0;
                        if (e < end) {
                            w = ci[e];
                            if (visit(vis, w)) { isnew = true; dw = deg[w]; }
                        }
                        if (isnew) {
                            my_cnt++; my_deg += dw;
                            if (a.lb_mode) a.w.lvl[w] = (int32_t)(D + 1);
                        }
                        q_append(isnew, w, dw, a.w.ql, a.w.qh, qcu, qcb, rp, &ctr[p * CS + 2], en);
                    }
                }
            } else {
                // pull: every unvisited vertex looks for an in-neighbour in the frontier
                const uint32_t* fcur = a.w.fb + (D % 3) * words;
                uint32_t* fnxt = a.w.fb + ((D + 1) % 3) * words;
                uint32_t* fold = a.w.fb + ((D + 2) % 3) * words;
                for (int64_t q = gtid; q < words; q += nthreads) fold[q] = 0;
                // light vertices (few in-arcs): one per lane
                for (int64_t base = gwave * 64; base < n; base += nwaves * 64) {
                    int32_t w = (int32_t)(base + lane);
                    bool isnew = false;
                    int32_t dw = 0;
                    if (w < n && a.g.rrp[w + 1] - a.g.rrp[w] <= HEAVY_DEG &&
                        !(ld_rlx(&vis[w >> 5]) & (1u << (w & 31)))) {
                        for (int32_t e = a.g.rrp[w]; e < a.g.rrp[w + 1]; e++) {
                            int32_t u = a.g.rci[e];
                            if (fcur[u >> 5] & (1u << (u & 31))) { isnew = true; break; }
                        }
                        if (isnew) {
                            for_rlx(&vis[w >> 5], 1u << (w & 31));
                            for_rlx(&fnxt[w >> 5], 1u << (w & 31));
                            dw = deg[w];
                            my_cnt++; my_deg += dw;
                            if (a.lb_mode) a.w.lvl[w] = (int32_t)(D + 1);
                        }
                    }
                    q_append(isnew, w, dw, a.w.ql, a.w.qh, qcu, qcb, rp, &ctr[p * CS + 2], en);
                }
                // heavy vertices: one wave per chunk of their in-arcs; the
                // visited bit decides which chunk's wave reports the vertex
                for (int64_t c = gwave; c < a.g.rnchunks; c += nwaves) {
                    int32_t w = a.g.rch_vtx[c];
                    int vw = (int)(ld_rlx(&vis[w >> 5]) >> (w & 31)) & 1;
                    if (__shfl(vw, 0, 64)) continue;   // wave-uniform
                    int32_t eb = a.g.rch_beg[c], ee = a.g.rch_end[c];
                    bool found = false;
                    for (int32_t e0 = eb; e0 < ee && !found; e0 += 64) {
                        int32_t e = e0 + lane;
                        bool hit = false;
                        if (e < ee) {
                            int32_t u = a.g.rci[e];
                            hit = (fcur[u >> 5] & (1u << (u & 31))) != 0;
                        }
                        found = __any(hit);
                    }
                    bool isnew = false;
                    int32_t dw = 0;
                    if (found && lane == 0 && visit(vis, w)) {
                        for_rlx(&fnxt[w >> 5], 1u << (w & 31));
                        isnew = true;
                        dw = deg[w];
                        my_cnt++; my_deg += dw;
                        if (a.lb_mode) a.w.lvl[w] = (int32_t)(D + 1);
                    }
                    q_append(isnew, w, dw, a.w.ql, a.w.qh, qcu, qcb, rp, &ctr[p * CS + 2], en);
                }
            }
            my_cnt = wave_sum_i64(my_cnt);
            my_deg = wave_sum_i64(my_deg);
            if (lane == 0 && (my_cnt | my_deg)) {
                fadd_rlx(&ctr[p * CS + 0], my_cnt);
                fadd_rlx(&ctr[p * CS + 1], my_deg);
            }
            grid_barrier(a.bar, gridDim.x);
            const int64_t cnt = ld_rlx(&ctr[p * CS + 0]);
            const int64_t dsum = ld_rlx(&ctr[p * CS + 1]);
            int64_t tails[3];
            for (int c = 0; c < 3; c++) tails[c] = en[c] + ld_rlx(&ctr[p * CS + 2 + c]);
            if (boss) {
                int q = (int)((D + 2) % 3);
                for (int j = 0; j < CS; j++) ctr[q * CS + j] = 0;
            }
            D++;
            nD += cnt;
            SD += D * cnt;
            if (a.bv.harm) H += (double)cnt / (double)D;
            U = dir ? dsum : dsum - cnt;
            mf = dsum;
            nf = cnt;
            mdisc += dsum;
            bytes += 16 * cnt;
            for (int c = 0; c < 3; c++) { st[c] = en[c]; en[c] = tails[c]; }
            if (a.lb_mode && boss) a.w.levcnt[D] = cnt;
        }
        const int64_t maxD = D - (status == 1 ? 1 : 0);
        if (a.lb_mode && status == 1 && a.bv.harm) {
            // harmonic centrality: per level l the sum over levels i of
            // n_i / max(2, gap) minus w's own 1/2, in increasing i; then
            // every reached vertex adds its out-neighbours' 1/2 each
            for (int64_t lv = gtid; lv <= maxD; lv += nthreads) {
                double xs = 0.0;
                for (int64_t i = 0; i <= maxD; i++) {
                    const int64_t t = dir ? i - lv : (i > lv ? i - lv : lv - i);
                    xs += (double)a.w.levcnt[i] / (double)(t < 2 ? 2 : t);
                }
                a.w.levtab[lv] = __double_as_longlong(xs - 0.5);
            }
            grid_barrier(a.bar, gridDim.x);
            const int32_t sc = dir ? a.rc.scc[v] : 0;
            for (int64_t i = gtid; i < en[0] + en[1]; i += nthreads) {
                int32_t w = i < en[0] ? a.w.ql[i] : a.w.qh[i - en[0]];
                if (w == v) continue;
                if (dir && a.rc.scc[w] != sc) continue;
                const double b = __longlong_as_double(a.w.levtab[a.w.lvl[w]]) + 0.5 * (double)deg[w];
                const int64_t f = harm_enc(b * (1.0 + HARM_MARGIN));
                if (rat_cmp(f, 1, a.bv.num[w], a.bv.den[w]) > 0) { a.bv.num[w] = f; a.bv.den[w] = 1; }
            }
        } else if (a.lb_mode && status == 1) {
            // level-based update of every reached vertex (Sect. 7)
            if (boss) {
                a.w.levcnt[D] = 0;
                lev_table(a.w.levcnt, maxD, nD, dir, a.w.levtab);
            }
            grid_barrier(a.bar, gridDim.x);
            const int64_t den = sq64(nD - 1);
            const int32_t sc = dir ? a.rc.scc[v] : 0;
            for (int64_t i = gtid; i < en[0] + en[1]; i += nthreads) {
                int32_t w = i < en[0] ? a.w.ql[i] : a.w.qh[i - en[0]];
                if (w == v) continue;
                if (dir && a.rc.scc[w] != sc) continue;
                int64_t b = a.w.levtab[a.w.lvl[w]] - deg[w];
                if (b < 0) b = 0;
                int64_t on = a.bv.num[w], od = a.bv.den[w];
                if (od != 0 && rat_cmp(b, den, on, od) > 0) { a.bv.num[w] = b; a.bv.den[w] = den; }
            }
        }
        // clear the visited bits of every reached vertex
        for (int64_t i = gtid; i < en[0] + en[1]; i += nthreads) {
            int32_t w = i < en[0] ? a.w.ql[i] : a.w.qh[i - en[0]];
            vis[w >> 5] = 0;
        }
        if (used_bu)
            for (int64_t q = gtid; q < 3 * words; q += nthreads) a.w.fb[q] = 0;
        if (boss) {
            stats[ST_STARTED]++;
            stats[ST_MVIS] += mvis;
            stats[ST_BYTES] += bytes;
            if (maxD > stats[ST_MAXLEVEL]) stats[ST_MAXLEVEL] = maxD;
            if (status == 1) {
                stats[ST_EXACT]++;
                if (a.bv.harm) topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, harm_enc(H), 2, TKC_OID(a.g, v));
                else topk_insert(a.tk.st, a.tk.ring, a.tk.S, a.tk.R, a.tk.I, SD, nD, TKC_OID(a.g, v));
            } else {
                stats[ST_CUT]++;
            }
        }
        grid_barrier(a.bar, gridDim.x);
    }
    if (boss) stats[ST_CURSOR] = pos;
}

int tkc_launch_plain(const DevGraph& g, DevReach rc, OrderView ov, BoundsView bv, DevTopk tk,
                     PlainWork w, int64_t* stats, const int32_t* list, int32_t list_count,
                     int lb_mode, const EngineTuning& tune, hipStream_t s, int* grid_out,
                     int64_t max_searches) {
    if (!w.bar || !w.vis || !w.fb || !w.ql || !w.qh || !w.qg || !w.ctr || !stats) return -2;
    const int cus = tkc_cu_count();
    if (cus < 1) return -1;
    const int occ = tkc_occupancy((const void*)k_plain, PB);
    if (occ < 1) return -1;
    const int want = tune.blocks_per_cu > 0 ? tune.blocks_per_cu : 2;
    int per = occ < want ? occ : want;
    const int grid = tkc_grid_for(cus, per, g.n);
    if (grid_out) *grid_out = grid;
    PlainArgs a{};
    a.g = g; a.rc = rc; a.ov = ov; a.bv = bv; a.tk = tk; a.w = w;
    a.stats = stats; a.list = list; a.list_count = list_count;
    a.lb_mode = lb_mode;
    a.alpha_td = tune.td_bu_alpha > 0 ? tune.td_bu_alpha : 14;
    a.beta_bu = tune.bu_td_beta > 0 ? tune.bu_td_beta : 24;
    a.max_searches = max_searches > 0 ? max_searches : 0;
    a.bar = w.bar;
    void* args[] = {&a};
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_plain, dim3(grid), dim3(PB), args, 0, s);
    return e == hipSuccess ? 0 : -1;
}
