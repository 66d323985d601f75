// The reachability bounds of tkc_graph_reach (Sect. 4 and Sect. 8.4,
// Alg. 6) for callers that cannot allocate: every buffer the kernels need
// beyond the graph and the caller's outputs comes from one static device
// array per GPU, `scratch`, held until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (at
// context creation, with that device current) and only that address is
// ever passed to kernels or copies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/tkc.h"
#include "engine.hpp"
#include "internal.hpp"

static __device__ __align__(256) unsigned char scratch[TKC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_init_mu;
void* g_scratch_dev[kMaxDevices];      // device address of `scratch` on each device
std::mutex g_call_mu[kMaxDevices];     // calls in this process that share a device's array
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

// Called by tkc_ctx_create with `device` current: looks the array's device
// address up once per device.
int tkc_noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return tkc_fail(TKC_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_scratch_dev[device]) return TKC_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return tkc_fail(TKC_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_dev[device] = p;
    return TKC_OK;
}

extern "C" int tkc_graph_reach_noalloc(tkc_graph* g, int64_t* alpha, int64_t* omega, int32_t* scc) {
    if (!g || !alpha || !omega) return tkc_fail(TKC_EINVAL, "NULL argument");
    if (g->relabeled) return tkc_fail(TKC_EINVAL, "not available for a graph uploaded with TKC_RELABEL");
    tkc_ctx* c = g->ctx;
    if (c->device < 0 || c->device >= kMaxDevices) return tkc_fail(TKC_EINVAL, "device out of range");
    if (hipSetDevice(c->device) != hipSuccess) return tkc_fail(TKC_EDEVICE, "hipSetDevice failed");
    void* base = g_scratch_dev[c->device];
    if (!base) return tkc_fail(TKC_EDEVICE, "no-allocation scratch not set up on device %d", c->device);
    const size_t cap = TKC_NOALLOC_SCRATCH_BYTES;
    const size_t n = (size_t)g->n;
    hipStream_t s = c->stream;
    DevGraph dg = g->view();
    std::lock_guard<std::mutex> lk(g_call_mu[c->device]);
    if (!g->directed) {
        // union-find: parents int32[n], component counts int64[n + 2], giant flags uint8[n]
        const size_t need = align256(4 * n) + align256(8 * (n + 2)) + align256(n);
        if (need > cap)
            return tkc_fail(TKC_EINVAL, "graph needs %zu bytes of scratch; the no-allocation limit is %zu", need,
                            cap);
        char* p = (char*)base;
        int32_t* parent = (int32_t*)p;
        int64_t* size = (int64_t*)(p + align256(4 * n));
        uint8_t* in_giant = (uint8_t*)(p + align256(4 * n) + align256(8 * (n + 2)));
        if (tkc_launch_cc(dg, parent, size, alpha, omega, in_giant, (int32_t*)c->pinned, s))
            return tkc_fail(TKC_EDEVICE, "components kernel failed");
        if (hipStreamSynchronize(s) != hipSuccess) return tkc_fail(TKC_EDEVICE, "components kernel failed");
        return TKC_OK;
    }
    // directed: the topological SCC ids go to the caller's scc, or to the
    // top of the scratch when scc is NULL
    size_t arena_cap = cap;
    int32_t* sc_out = scc;
    if (!sc_out) {
        if (align256(4 * n) > cap)
            return tkc_fail(TKC_EINVAL, "graph needs more than the %zu bytes of no-allocation scratch", cap);
        arena_cap = cap - align256(4 * n);
        sc_out = (int32_t*)((char*)base + arena_cap);
    }
    int seq = 0;
    size_t need = 0;
    const int r = tkc_device_alpha_omega(dg, alpha, omega, sc_out, c->pinned, s, &seq, base, arena_cap, &need);
    if (r == -3)
        return tkc_fail(TKC_EINVAL, "graph needs %zu bytes of scratch; the no-allocation limit is %zu",
                        need + (scc ? 0 : align256(4 * n)), cap);
    if (r < 0) return tkc_fail(TKC_EDEVICE, "reachability kernels failed");
    return TKC_OK;
}
