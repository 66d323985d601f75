// Preprocessing kernels: out-degrees, connected components (r(v) of an
// undirected graph), the neighbourhood-based lower bound of Sect. 5 and the
// keys of the processing order (Sect. 4, computeBounds).
#include "dev_common.hpp"
#include "engine.hpp"

#define NB_INF ((int64_t)1 << 62)
#define HEAVY_DEG 64

// --------------------------------------------------------------- degrees
__global__ void k_degrees(int32_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ deg) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) deg[v] = rp[v + 1] - rp[v];
}

// list of vertices with more than HEAVY_DEG arcs (wave-per-vertex work)
__global__ void k_heavy_list(int32_t n, const int32_t* __restrict__ deg, int32_t* heavy,
                             int32_t* nheavy) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    bool h = v < n && deg[v] > HEAVY_DEG;
    int tot;
    int rank = wave_rank(h, &tot);
    int leader = __ffsll((long long)__ballot(1)) - 1;
    int base = 0;
    if (lane_id() == leader && tot) base = fadd_rlx(nheavy, tot);
    base = __shfl(base, leader, 64);
    if (h) heavy[base + rank] = v;
}

// ----------------------------------------------- connected components
// Lock-free union-find: roots only ever point to smaller ids, so every
// component ends rooted at its smallest vertex and every chain of parents
// strictly decreases (no cycles even under races).  Parent reads go
// through agent-scope atomics so a retry never sees a stale cached line.
TKC_DEV int32_t uf_find(int32_t* parent, int32_t x) {
    for (;;) {
        int32_t p = ld_rlx(&parent[x]);
        if (p == x) return x;
        int32_t gp = ld_rlx(&parent[p]);
        if (gp != p) st_rlx(&parent[x], gp);   // path halving (gp is still an ancestor)
        x = gp;
    }
}
TKC_DEV void uf_union(int32_t* parent, int32_t a, int32_t b) {
    for (;;) {
        int32_t ra = uf_find(parent, a), rb = uf_find(parent, b);
        if (ra == rb) return;
        int32_t hi = ra > rb ? ra : rb, lo = ra > rb ? rb : ra;
        int32_t exp = hi;
        if (__hip_atomic_compare_exchange_strong(&parent[hi], &exp, lo, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}
__global__ void k_cc_init(int32_t n, int32_t* parent, int64_t* size) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) { parent[v] = v; size[v] = 0; }
}
// light vertices: one thread each; heavy vertices: one wave each
__global__ void k_cc_hook(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const int32_t* __restrict__ deg, const int32_t* __restrict__ heavy,
                          int32_t nheavy, int32_t nlight_blocks, int32_t* parent) {
    if ((int32_t)blockIdx.x < nlight_blocks) {
        int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
        if (u >= n || deg[u] > HEAVY_DEG) return;
        for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
            int32_t w = ci[e];
            if (w > u) uf_union(parent, u, w);
        }
    } else {
        int32_t wv = ((blockIdx.x - nlight_blocks) * blockDim.x + threadIdx.x) >> 6;
        if (wv >= nheavy) return;
        int32_t u = heavy[wv];
        for (int32_t e = rp[u] + lane_id(); e < rp[u + 1]; e += 64) {
            int32_t w = ci[e];
            if (w > u) uf_union(parent, u, w);
        }
    }
}
__global__ void k_cc_finish(int32_t n, int32_t* parent, int64_t* size) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t root = uf_find(parent, v);
    parent[v] = root;
    fadd_rlx(&size[root], (int64_t)1);
}
__global__ void k_cc_assign(int32_t n, const int32_t* parent, const int64_t* size, int64_t* alpha,
                            int64_t* omega) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int64_t s = size[parent[v]];
    alpha[v] = s;
    omega[v] = s;
}

// ------------------------------------------- NB bound (Sect. 5, Alg. 3)
// gamma_k(s) bounds the number of vertices at distance k.  Undirected: the
// non-backtracking walk recurrence of Eq. 2; directed: plain walk counts
// (Eq. 3).  Three rotating buffers hold gamma_{k-2}, gamma_{k-1}, gamma_k so
// one kernel per round both gathers the new counts and advances each
// vertex's sum (Prop. 5.1) -- a vertex only ever writes its own state.
// Counts saturate at 2^62 ("at least that many").  A finished vertex keeps
// updating its counts because its neighbours still read them.
// Disconnected directed graphs (Sect. 8.1): with alpha <= r <= omega the
// bound is the least value over r in {alpha, omega} and the cumulative
// counts strictly between them; with r known alpha = omega = r.
struct NBState {
    int64_t* sum;
    int64_t* vis;
    uint8_t* flags;   // bit0 finished, bit1 alpha reached
    int64_t* num;
    int64_t* den;
};
TKC_DEV void rat_keep_min(int64_t* num, int64_t* den, int64_t cn, int64_t cd) {
    if (*den == 0 || rat_cmp(cn, cd, *num, *den) < 0) { *num = cn; *den = cd; }
}
// advance vertex s by one level (level k, count gk); returns true when s finishes now
TKC_DEV bool nb_advance(int64_t k, int64_t gk, int64_t a, int64_t o, int64_t& pv, int64_t& ps,
                        uint8_t& fl, int64_t& num, int64_t& den) {
    if (gk == 0) {
        // nothing at distance >= k: r <= pv and alpha was already reached
        if (!(fl & 2)) rat_keep_min(&num, &den, ps, sq64(pv - 1));
        fl |= 1;
        return true;
    }
    int64_t nv = pv + gk;
    if (nv > NB_INF) nv = NB_INF;
    if (nv < a) {
        ps += k * gk; pv = nv;
        return false;
    }
    if (nv < o) {
        if (!(fl & 2)) { rat_keep_min(&num, &den, ps + k * (a - pv), sq64(a - 1)); fl |= 2; }
        ps += k * gk; pv = nv;
        rat_keep_min(&num, &den, ps, sq64(nv - 1));
        return false;
    }
    if (!(fl & 2)) rat_keep_min(&num, &den, ps + k * (a - pv), sq64(a - 1));
    rat_keep_min(&num, &den, ps + k * (o - pv), sq64(o - 1));
    fl |= 1;
    return true;
}

__global__ void k_nb_init(int32_t n, const int32_t* __restrict__ deg, const int64_t* __restrict__ alpha,
                          const int64_t* __restrict__ omega, int64_t* g0, int64_t* g1, NBState st,
                          int32_t* nfin) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    bool fin = false;
    if (s < n) {
        int64_t d = deg[s];
        g0[s] = 1;
        g1[s] = d;
        int64_t a = alpha[s], o = omega[s];
        int64_t pv = 1, ps = 0, num = 0, den = 0;
        uint8_t fl = 0;
        if (o <= 1) { fl = 1; fin = true; }
        else fin = nb_advance(1, d, a, o, pv, ps, fl, num, den);
        st.sum[s] = ps; st.vis[s] = pv; st.flags[s] = fl; st.num[s] = num; st.den[s] = den;
    }
    int tot;
    wave_rank(fin, &tot);
    if (lane_id() == 0 && tot) fadd_rlx(nfin, tot);
}

template <bool DIRECTED>
TKC_DEV void nb_finish_vertex(int32_t s, uint64_t acc, int64_t k, int32_t d, const int64_t* g2,
                              int64_t* gk, const int64_t* alpha, const int64_t* omega, NBState st,
                              bool* fin_now) {
    int64_t val;
    if (acc >= (uint64_t)NB_INF) val = NB_INF;
    else {
        val = (int64_t)acc;
        if (!DIRECTED) {
            // exact counts: the subtracted walks never exceed the sum
            tkc_u128 sub = (k == 2) ? (tkc_u128)d : (tkc_u128)(uint64_t)(d - 1) * (uint64_t)g2[s];
            val = ((tkc_u128)(uint64_t)val >= sub) ? (int64_t)((tkc_u128)(uint64_t)val - sub) : 0;
        }
    }
    gk[s] = val;
    uint8_t fl = st.flags[s];
    *fin_now = false;
    if (fl & 1) return;
    int64_t pv = st.vis[s], ps = st.sum[s], num = st.num[s], den = st.den[s];
    *fin_now = nb_advance(k, val, alpha[s], omega[s], pv, ps, fl, num, den);
    st.vis[s] = pv; st.sum[s] = ps; st.flags[s] = fl; st.num[s] = num; st.den[s] = den;
}

template <bool DIRECTED>
__global__ void k_nb_round(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const int32_t* __restrict__ deg, const int32_t* __restrict__ heavy,
                           int32_t nheavy, int32_t nlight_blocks, int64_t k,
                           const int64_t* __restrict__ g1, const int64_t* __restrict__ g2,
                           int64_t* __restrict__ gk, const int64_t* __restrict__ alpha,
                           const int64_t* __restrict__ omega, NBState st, int32_t* nfin) {
    bool fin = false;
    if ((int32_t)blockIdx.x < nlight_blocks) {
        int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
        if (s < n && deg[s] <= HEAVY_DEG) {
            uint64_t acc = 0;
            int32_t e = rp[s], end = rp[s + 1];
            for (; e + 4 <= end; e += 4) {
                uint64_t a0 = g1[ci[e]], a1 = g1[ci[e + 1]], a2 = g1[ci[e + 2]], a3 = g1[ci[e + 3]];
                acc += a0 + a1 + a2 + a3;           // 4 x 2^62 fits in 64 unsigned bits
                if (acc > (uint64_t)NB_INF) acc = NB_INF;
            }
            for (; e < end; e++) {
                acc += (uint64_t)g1[ci[e]];
                if (acc > (uint64_t)NB_INF) acc = NB_INF;
            }
            nb_finish_vertex<DIRECTED>(s, acc, k, deg[s], g2, gk, alpha, omega, st, &fin);
        }
        int tot;
        wave_rank(fin, &tot);
        if (lane_id() == 0 && tot) fadd_rlx(nfin, tot);
    } else {
        int32_t wv = ((blockIdx.x - nlight_blocks) * blockDim.x + threadIdx.x) >> 6;
        if (wv >= nheavy) return;   // wave-uniform
        int32_t s = heavy[wv];
        uint64_t acc = 0;
        for (int32_t e = rp[s] + lane_id(); e < rp[s + 1]; e += 64) {
            acc += (uint64_t)g1[ci[e]];
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            acc += __shfl_xor(acc, o, 64);
            if (acc > (uint64_t)NB_INF) acc = NB_INF;
        }
        if (lane_id() == 0) {
            nb_finish_vertex<DIRECTED>(s, acc, k, deg[s], g2, gk, alpha, omega, st, &fin);
            if (fin) fadd_rlx(nfin, 1);
        }
    }
}

// ------------------------------------------------------ order keys (Sect. 4)
// Deg: L = 0 (the bound is the trivial one) and the key is the degree,
// largest first; NB: the key is the bound itself.  Vertices that reach
// nothing get L = +inf and the last key.
__global__ void k_deg_bounds(int32_t n, const int32_t* __restrict__ deg, const int64_t* __restrict__ omega,
                             int64_t* num, int64_t* den, uint32_t* key, int32_t* val) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    bool inf = omega[v] <= 1;
    num[v] = 0;
    den[v] = inf ? 0 : 1;
    key[v] = inf ? 0xffffffffu : (uint32_t)(0x7fffffff - deg[v]);
    val[v] = v;
}
__global__ void k_nb_keys(int32_t n, const int64_t* __restrict__ num, const int64_t* __restrict__ den,
                          uint32_t* key, int32_t* val) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    key[v] = order_key(num[v], den[v]);
    val[v] = v;
}

// ------------------------------------------------------------ host side
static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

int tkc_launch_degrees(const DevGraph& g, int32_t* heavy, int32_t* nheavy, hipStream_t s) {
    int32_t n = g.n;
    hipLaunchKernelGGL(k_degrees, dim3(nblk(n, 256)), dim3(256), 0, s, n, g.rp, g.deg);
    hipMemsetAsync(nheavy, 0, sizeof(int32_t), s);
    hipLaunchKernelGGL(k_heavy_list, dim3(nblk(n, 256)), dim3(256), 0, s, n, g.deg, heavy, nheavy);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int tkc_launch_cc(const DevGraph& g, const int32_t* heavy, int32_t nheavy, int32_t* parent,
                  int64_t* size, int64_t* alpha, int64_t* omega, hipStream_t s) {
    int32_t n = g.n;
    int nl = nblk(n, 256);
    hipLaunchKernelGGL(k_cc_init, dim3(nl), dim3(256), 0, s, n, parent, size);
    int nh = nblk((int64_t)nheavy * 64, 256);
    hipLaunchKernelGGL(k_cc_hook, dim3(nl + nh), dim3(256), 0, s, n, g.rp, g.ci, g.deg, heavy,
                       nheavy, nl, parent);
    hipLaunchKernelGGL(k_cc_finish, dim3(nl), dim3(256), 0, s, n, parent, size);
    hipLaunchKernelGGL(k_cc_assign, dim3(nl), dim3(256), 0, s, n, parent, size, alpha, omega);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// NB bound: returns the number of rounds, -1 on error.  gbuf holds 3*n int64.
int tkc_launch_nb(const DevGraph& g, const int32_t* heavy, int32_t nheavy, const int64_t* alpha,
                  const int64_t* omega, int64_t* gbuf, int64_t* sum, int64_t* vis, uint8_t* flags,
                  int64_t* num, int64_t* den, int32_t* nfin_dev, int32_t* nfin_host, hipStream_t s) {
    int32_t n = g.n;
    int nl = nblk(n, 256);
    int nh = nblk((int64_t)nheavy * 64, 256);
    NBState st{sum, vis, flags, num, den};
    int64_t* buf[3] = {gbuf, gbuf + n, gbuf + 2 * (int64_t)n};
    hipMemsetAsync(nfin_dev, 0, sizeof(int32_t), s);
    // gamma_0 -> buf[0], gamma_1 -> buf[1]
    hipLaunchKernelGGL(k_nb_init, dim3(nl), dim3(256), 0, s, n, g.deg, alpha, omega, buf[0], buf[1],
                       st, nfin_dev);
    if (hipGetLastError() != hipSuccess) return -1;
    int32_t done = 0;
    int64_t k = 2;
    const int64_t kmax = (int64_t)n + 2;
    for (;;) {
        if (hipMemcpyAsync(nfin_host, nfin_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
            return -1;
        if (hipStreamSynchronize(s) != hipSuccess) return -1;
        done = *nfin_host;
        if (done >= n || k > kmax) break;
        // several rounds per host check: a finished graph makes extra rounds no-ops
        for (int rep = 0; rep < 2 && k <= kmax; rep++, k++) {
            int64_t* g1 = buf[(k - 1) % 3];
            int64_t* g2 = buf[(k - 2) % 3];
            int64_t* gk = buf[k % 3];
            if (g.directed)
                hipLaunchKernelGGL(k_nb_round<true>, dim3(nl + nh), dim3(256), 0, s, n, g.rp, g.ci,
                                   g.deg, heavy, nheavy, nl, k, g1, g2, gk, alpha, omega, st, nfin_dev);
            else
                hipLaunchKernelGGL(k_nb_round<false>, dim3(nl + nh), dim3(256), 0, s, n, g.rp, g.ci,
                                   g.deg, heavy, nheavy, nl, k, g1, g2, gk, alpha, omega, st, nfin_dev);
        }
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return (int)(k - 2);
}

int tkc_launch_deg_bounds(const DevGraph& g, const int64_t* omega, int64_t* num, int64_t* den,
                          uint32_t* key, int32_t* val, hipStream_t s) {
    hipLaunchKernelGGL(k_deg_bounds, dim3(nblk(g.n, 256)), dim3(256), 0, s, g.n, g.deg, omega, num,
                       den, key, val);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
int tkc_launch_nb_keys(int32_t n, const int64_t* num, const int64_t* den, uint32_t* key, int32_t* val,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_nb_keys, dim3(nblk(n, 256)), dim3(256), 0, s, n, num, den, key, val);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
