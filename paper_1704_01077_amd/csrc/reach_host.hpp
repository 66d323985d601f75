// Host-side reachability bounds of directed graphs (Sect. 8.4, Alg. 6).
#pragma once
#include <stdint.h>

#include <vector>

// Returns the number of strongly connected components; scc_topo numbers the
// components in a topological order of the component DAG.
int tkc_host_alpha_omega(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<int64_t>& alpha,
                         std::vector<int64_t>& omega, std::vector<int32_t>& scc_topo);
