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
