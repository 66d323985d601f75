// Top-k state (Alg. 1: the list Top and Farn[Top[k]]) reset for a query.
#include "dev_common.hpp"
#include "engine.hpp"

__global__ void k_topk_init(TopkState* st, int32_t k, int32_t ties, int32_t tcap, int64_t* tieS, int64_t* tieR,
                            int32_t* tieI) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->lock = 0;
        st->cnt = 0;
        st->seq = -1;
        st->k = k;
        st->ties = ties;
        st->n_inserts = 0;
        st->tcnt = 0;
        st->tcap = ties ? tcap : 0;
        st->tieS = tieS;
        st->tieR = tieR;
        st->tieI = tieI;
    }
}

int tkc_launch_topk_init(DevTopk t, int32_t k, hipStream_t s, const TieBuf* tb) {
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(64), 0, s, t.st, k, tb ? 1 : 0, tb ? tb->cap : 0,
                       tb ? tb->S : nullptr, tb ? tb->R : nullptr, tb ? tb->I : nullptr);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

#include <map>
#include <mutex>
#include <tuple>

static std::mutex& launch_cache_mutex() {
    static std::mutex m;
    return m;
}
int tkc_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return -1;
    static std::map<int, int> cus;
    std::lock_guard<std::mutex> lk(launch_cache_mutex());
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) return -1;
    cus[dev] = v;
    return v;
}
int tkc_occupancy(const void* fn, int block) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return -1;
    static std::map<std::tuple<const void*, int, int>, int> occ;
    std::lock_guard<std::mutex> lk(launch_cache_mutex());
    const auto key = std::make_tuple(fn, block, dev);
    auto it = occ.find(key);
    if (it != occ.end()) return it->second;
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, fn, block, 0) != hipSuccess) return -1;
    occ[key] = v;
    return v;
}
