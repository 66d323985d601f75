// Reachability bounds of a directed graph (Sect. 8.4, Alg. 6), host side.
//
// Strongly connected components by Tarjan's algorithm (iterative), which
// emits components sinks-first, i.e. in reverse topological order of the
// component DAG -- exactly the order in which Alg. 6 sweeps them:
//   alpha(C) = w(C) + max over successors D of alpha(D)
//   omega(C) = w(C) + sum over successors D of omega(D)
// with the refinement through the largest component C~: its reach is
// counted exactly, and for a component X that reaches C~ the successors
// that C~ does not reach are summed with omega(C~) added once.  Readings:
// the largest component's ties go to the one holding the smallest vertex
// id; every omega is capped at n (r <= n always holds).
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "reach_host.hpp"

int tkc_host_alpha_omega(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<int64_t>& alpha,
                         std::vector<int64_t>& omega, std::vector<int32_t>& scc_topo) {
    // ---- Tarjan, iterative
    std::vector<int32_t> index(n, -1), low(n, 0), comp(n, -1), stack, call;
    std::vector<int32_t> edge_pos(n, 0);
    std::vector<char> on_stack(n, 0);
    stack.reserve(n);
    call.reserve(n);
    int32_t next_index = 0, nc = 0;
    for (int32_t s = 0; s < n; s++) {
        if (index[s] >= 0) continue;
        call.push_back(s);
        index[s] = low[s] = next_index++;
        edge_pos[s] = rp[s];
        stack.push_back(s);
        on_stack[s] = 1;
        while (!call.empty()) {
            int32_t u = call.back();
            if (edge_pos[u] < rp[u + 1]) {
                int32_t w = ci[edge_pos[u]++];
                if (index[w] < 0) {
                    index[w] = low[w] = next_index++;
                    edge_pos[w] = rp[w];
                    stack.push_back(w);
                    on_stack[w] = 1;
                    call.push_back(w);
                } else if (on_stack[w]) {
                    low[u] = std::min(low[u], index[w]);
                }
            } else {
                call.pop_back();
                if (!call.empty()) {
                    int32_t p = call.back();
                    low[p] = std::min(low[p], low[u]);
                }
                if (low[u] == index[u]) {
                    int32_t w;
                    do {
                        w = stack.back();
                        stack.pop_back();
                        on_stack[w] = 0;
                        comp[w] = nc;
                    } while (w != u);
                    nc++;
                }
            }
        }
    }
    // comp ids: 0 = first emitted (a sink component); reverse topological
    std::vector<int64_t> wt(nc, 0);
    std::vector<int32_t> minid(nc, n);
    for (int32_t v = 0; v < n; v++) {
        wt[comp[v]]++;
        minid[comp[v]] = std::min(minid[comp[v]], v);
    }
    int32_t big = 0;
    for (int32_t c = 1; c < nc; c++)
        if (wt[c] > wt[big] || (wt[c] == wt[big] && minid[c] < minid[big])) big = c;
    // component DAG successor lists (deduplicated)
    std::vector<std::vector<int32_t>> succ(nc);
    for (int32_t u = 0; u < n; u++)
        for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
            int32_t cu = comp[u], cw = comp[ci[e]];
            if (cu != cw) succ[cu].push_back(cw);
        }
    for (auto& s : succ) {
        std::sort(s.begin(), s.end());
        s.erase(std::unique(s.begin(), s.end()), s.end());
    }
    // reachable from C~: successors have smaller ids (reverse topological)
    std::vector<char> from_big(nc, 0), to_big(nc, 0);
    from_big[big] = 1;
    for (int32_t c = big; c >= 0; c--)
        if (from_big[c])
            for (int32_t d : succ[c]) from_big[d] = 1;
    to_big[big] = 1;
    for (int32_t c = big + 1; c < nc; c++)
        for (int32_t d : succ[c])
            if (to_big[d]) { to_big[c] = 1; break; }
    int64_t reach_big = 0;
    for (int32_t c = 0; c < nc; c++)
        if (from_big[c]) reach_big += wt[c];
    std::vector<int64_t> aS(nc, 0), oS(nc, 0);
    aS[big] = oS[big] = reach_big;
    for (int32_t c = 0; c < nc; c++) {   // sinks first
        if (c == big) continue;
        int64_t a = 0, o = 0, o2 = 0;
        for (int32_t d : succ[c]) {
            a = std::max(a, aS[d]);
            o += oS[d];
            if (!from_big[d]) o2 += oS[d];
        }
        if (to_big[c]) o = o2 + oS[big];
        a += wt[c];
        o += wt[c];
        if (o > n) o = n;
        aS[c] = a;
        oS[c] = o;
    }
    alpha.resize(n);
    omega.resize(n);
    scc_topo.resize(n);
    for (int32_t v = 0; v < n; v++) {
        alpha[v] = aS[comp[v]];
        omega[v] = oS[comp[v]];
        scc_topo[v] = nc - 1 - comp[v];   // topological numbering
    }
    return nc;
}
