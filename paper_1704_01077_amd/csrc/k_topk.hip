// Top-k state (Alg. 1: the list Top and Farn[Top[k]]) reset for a query.
#include "dev_common.hpp"
#include "engine.hpp"

__global__ void k_topk_init(TopkState* st, int32_t k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->lock = 0;
        st->cnt = 0;
        st->seq = -1;
        st->k = k;
        st->pad = 0;
        st->n_inserts = 0;
    }
}

int tkc_launch_topk_init(DevTopk t, int32_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(64), 0, s, t.st, k);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
