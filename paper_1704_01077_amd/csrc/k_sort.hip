// Stable LSD radix sort of (uint32 key, int32 value) pairs, 4-bit digits.
// Used once per query to lay out the processing order of Alg. 1 (values
// start as vertex ids, so equal keys keep ascending ids).  Digits on which
// all keys agree are skipped.
#include "dev_common.hpp"
#include "engine.hpp"

#define RS_THREADS 256
#define RS_ITEMS 8
#define RS_TILE (RS_THREADS * RS_ITEMS)
#define RS_DIG 16

static inline int rs_tiles(int32_t n) { return (n + RS_TILE - 1) / RS_TILE; }

__global__ void k_rs_mask(const uint32_t* __restrict__ keys, int32_t n, uint32_t* mask) {
    // mask[0] = OR of keys, mask[1] = AND of keys
    uint32_t o = 0, a = 0xffffffffu;
    const int32_t t0 = blockIdx.x * blockDim.x + threadIdx.x, step = gridDim.x * blockDim.x;
    int32_t head = 0;
    if (((uintptr_t)keys & 15u) == 0) {
        // 16-byte loads, independent across the loop
        const uint4* k4 = (const uint4*)keys;
        head = n & ~3;
        for (int32_t i = t0; i < head / 4; i += step) {
            const uint4 q = k4[i];
            o |= q.x | q.y | q.z | q.w;
            a &= q.x & q.y & q.z & q.w;
        }
    }
    for (int32_t i = head + t0; i < n; i += step) {
        const uint32_t k = keys[i];
        o |= k; a &= k;
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        o |= __shfl_xor(o, s, 64);
        a &= __shfl_xor(a, s, 64);
    }
    __shared__ uint32_t so[4], sa[4];
    if (lane_id() == 0) { so[threadIdx.x >> 6] = o; sa[threadIdx.x >> 6] = a; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) { o |= so[w]; a &= sa[w]; }
        __hip_atomic_fetch_or(&mask[0], o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_and(&mask[1], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// per-tile digit counts, stored digit-major: cnt[d * tiles + tile]
__global__ void __launch_bounds__(RS_THREADS) k_rs_count(const uint32_t* __restrict__ keys, int32_t n,
                                                          int shift, int32_t* cnt, int32_t tiles) {
    __shared__ int32_t part[RS_THREADS / 64][RS_DIG];
    int32_t base = blockIdx.x * RS_TILE + threadIdx.x * RS_ITEMS;
    int32_t c[RS_DIG];
#pragma unroll
    for (int d = 0; d < RS_DIG; d++) c[d] = 0;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; j++) {
        int32_t i = base + j;
        if (i < n) {
            uint32_t dg = (keys[i] >> shift) & 15u;
#pragma unroll
            for (int d = 0; d < RS_DIG; d++) c[d] += (dg == (uint32_t)d);
        }
    }
    int wv = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < RS_DIG; d++) {
        int32_t s = wave_sum_i32(c[d]);
        if (lane_id() == 0) part[wv][d] = s;
    }
    __syncthreads();
    if (threadIdx.x < RS_DIG) {
        int32_t s = 0;
        for (int w = 0; w < RS_THREADS / 64; w++) s += part[w][threadIdx.x];
        cnt[threadIdx.x * tiles + blockIdx.x] = s;
    }
}

// exclusive scan of `len` int32 in place, one workgroup of 1024 threads
__global__ void __launch_bounds__(1024) k_rs_scan(int32_t* a, int32_t len) {
    __shared__ int32_t wsum[16];
    int32_t per = (len + 1023) / 1024;
    int32_t lo = threadIdx.x * per;
    int32_t hi = lo + per < len ? lo + per : len;
    int32_t s = 0;
    for (int32_t i = lo; i < hi; i++) s += a[i];
    // block exclusive scan of s
    int32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane_id() >= o) x += y;
    }
    int wv = threadIdx.x >> 6;
    if (lane_id() == 63) wsum[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int w = 0; w < 16; w++) { int32_t t = wsum[w]; wsum[w] = run; run += t; }
    }
    __syncthreads();
    int32_t run = wsum[wv] + x - s;
    for (int32_t i = lo; i < hi; i++) { int32_t t = a[i]; a[i] = run; run += t; }
}

// Up to RS_FUSE_TILES tiles, each scatter workgroup finds its own 16 offsets
// in the count table (thread t sums digit t / 16 over the t % 16-th
// sixteenth of the tiles: the counts of earlier tiles and of all tiles),
// which saves the scan launch; above that, off holds the scanned table.
#define RS_FUSE_TILES 512
static_assert(RS_THREADS == RS_DIG * 16, "one digit per 16 threads");
static_assert(RS_DIG * RS_THREADS >= 2 * RS_TILE, "the count table's LDS holds a staged tile");
template <bool FUSED>
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint32_t* __restrict__ keys,
                                                            const int32_t* __restrict__ vals, int32_t n,
                                                            int shift, const int32_t* __restrict__ off,
                                                            int32_t tiles, uint32_t* __restrict__ okeys,
                                                            int32_t* __restrict__ ovals) {
    __shared__ int32_t cs[RS_DIG * RS_THREADS];   // [digit][thread]
    __shared__ int32_t wtot[RS_THREADS / 64];
    __shared__ int32_t dstart[RS_DIG];
    __shared__ int32_t s_off[RS_DIG], s_bef[RS_DIG], s_all[RS_DIG];
    if (FUSED) {
        const int d = threadIdx.x >> 4, r = threadIdx.x & 15;
        const int32_t per = (tiles + 15) / 16;
        const int32_t t0 = r * per, t1 = t0 + per < tiles ? t0 + per : tiles;
        const int32_t* row = off + (int64_t)d * tiles;
        int32_t bef = 0, all = 0;
#pragma unroll 8
        for (int32_t t = t0; t < t1; t++) {
            const int32_t c = row[t];
            all += c;
            bef += t < (int32_t)blockIdx.x ? c : 0;
        }
        // the 16 threads of a digit are 16 consecutive lanes of one wave
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            bef += __shfl_xor(bef, o, 64);
            all += __shfl_xor(all, o, 64);
        }
        if (r == 0) { s_bef[d] = bef; s_all[d] = all; }
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t run = 0;
            for (int q = 0; q < RS_DIG; q++) { s_off[q] = run + s_bef[q]; run += s_all[q]; }
        }
        __syncthreads();
    }
    int32_t base = blockIdx.x * RS_TILE + threadIdx.x * RS_ITEMS;
    uint32_t k[RS_ITEMS];
    int32_t v[RS_ITEMS];
    uint32_t dg[RS_ITEMS];
    int32_t c[RS_DIG];
#pragma unroll
    for (int d = 0; d < RS_DIG; d++) c[d] = 0;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; j++) {
        int32_t i = base + j;
        if (i < n) {
            k[j] = keys[i]; v[j] = vals[i];
            dg[j] = (k[j] >> shift) & 15u;
        } else {
            dg[j] = RS_DIG;
        }
#pragma unroll
        for (int d = 0; d < RS_DIG; d++) c[d] += (dg[j] == (uint32_t)d);
    }
#pragma unroll
    for (int d = 0; d < RS_DIG; d++) cs[d * RS_THREADS + threadIdx.x] = c[d];
    __syncthreads();
    // exclusive scan over the 4096 entries in digit-major order: thread t
    // owns 16 consecutive entries
    int32_t loc[16];
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < 16; q++) { loc[q] = cs[threadIdx.x * 16 + q]; s += loc[q]; }
    int32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane_id() >= o) x += y;
    }
    int wv = threadIdx.x >> 6;
    if (lane_id() == 63) wtot[wv] = x;
    __syncthreads();
    int32_t run = x - s;
    for (int w = 0; w < wv; w++) run += wtot[w];
#pragma unroll
    for (int q = 0; q < 16; q++) { int32_t t = loc[q]; cs[threadIdx.x * 16 + q] = run; run += t; }
    __syncthreads();
    if (threadIdx.x < RS_DIG) dstart[threadIdx.x] = cs[threadIdx.x * RS_THREADS];
    __syncthreads();
    if (!FUSED && threadIdx.x < RS_DIG) s_off[threadIdx.x] = off[threadIdx.x * tiles + blockIdx.x];
    // each item's place in the tile's stable order by digit
    int32_t seen[RS_DIG];
#pragma unroll
    for (int d = 0; d < RS_DIG; d++) seen[d] = 0;
    int32_t lp[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; j++) {
        uint32_t d = dg[j];
        lp[j] = -1;
        if (d < RS_DIG) {
            int32_t rank = 0;
#pragma unroll
            for (int e = 0; e < RS_DIG; e++) {
                if ((uint32_t)e == d) { rank = seen[e]; seen[e]++; }
            }
            lp[j] = cs[d * RS_THREADS + threadIdx.x] + rank;
        }
    }
    // the tile in that order in LDS (cs is free once every place is read),
    // then written out in order: consecutive threads store consecutive
    // positions of a digit's run
    __syncthreads();
    uint32_t* sk = (uint32_t*)cs;
    int32_t* sv = cs + RS_TILE;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; j++) {
        if (lp[j] >= 0) { sk[lp[j]] = k[j]; sv[lp[j]] = v[j]; }
    }
    __syncthreads();
    const int32_t rem = n - (int32_t)blockIdx.x * RS_TILE;
    const int32_t cnt = rem < RS_TILE ? rem : RS_TILE;
    for (int32_t q = threadIdx.x; q < cnt; q += RS_THREADS) {
        const uint32_t key = sk[q];
        const uint32_t d = (key >> shift) & 15u;
        const int32_t pos = s_off[d] + (q - dstart[d]);
        okeys[pos] = key;
        ovals[pos] = sv[q];
    }
}

int64_t tkc_sort_hist_words(int32_t n) { return (int64_t)RS_DIG * rs_tiles(n > 0 ? n : 1) + 16; }

int tkc_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* tmp_keys, int32_t* tmp_vals, int32_t n,
                   int32_t* hist, uint32_t* mask_dev, uint32_t* mask_host, hipStream_t s) {
    if (n <= 1) return 0;
    // OR of all keys from 0, AND from all ones (fills: no host staging)
    if (hipMemsetD32Async((hipDeviceptr_t)mask_dev, 0u, 1, s) != hipSuccess) return -1;
    if (hipMemsetD32Async((hipDeviceptr_t)(mask_dev + 1), 0xffffffffu, 1, s) != hipSuccess) return -1;
    int gb = rs_tiles(n);
    if (gb > 256) gb = 256;   // one pair of adds to the mask per workgroup
    hipLaunchKernelGGL(k_rs_mask, dim3(gb), dim3(256), 0, s, keys, n, mask_dev);
    if (hipMemcpyAsync(mask_host, mask_dev, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    uint32_t vary = mask_host[0] ^ mask_host[1];
    int tiles = rs_tiles(n);
    uint32_t* ka = keys; int32_t* va = vals;
    uint32_t* kb = tmp_keys; int32_t* vb = tmp_vals;
    for (int shift = 0; shift < 32; shift += 4) {
        if (((vary >> shift) & 15u) == 0) continue;
        hipLaunchKernelGGL(k_rs_count, dim3(tiles), dim3(RS_THREADS), 0, s, ka, n, shift, hist, tiles);
        if (tiles <= RS_FUSE_TILES) {
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3(tiles), dim3(RS_THREADS), 0, s, ka, va, n, shift,
                               (const int32_t*)hist, tiles, kb, vb);
        } else {
            hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, s, hist, RS_DIG * tiles);
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3(tiles), dim3(RS_THREADS), 0, s, ka, va, n, shift,
                               (const int32_t*)hist, tiles, kb, vb);
        }
        uint32_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        hipMemcpyAsync(keys, ka, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(vals, va, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort with 8-bit digits, for the processing order: half
// the passes of the 4-bit sort on keys whose varying bits span two bytes.
// A tile is RS8_TILE items taken round-robin (item j * 256 + t is thread t's
// j-th), so rounds in order and lanes in order visit the tile in order.
// Per pass: per-tile digit counts; per digit, the exclusive prefix over
// tiles and the total; the scatter, which ranks each round's items by
// digit within each wave (a match over the digit's eight bits) and keeps
// running per-digit counts in LDS.
#define RS8_THREADS 256
#define RS8_ROUNDS 8
#define RS8_TILE (RS8_THREADS * RS8_ROUNDS)

static inline int rs8_tiles(int32_t n) { return (n + RS8_TILE - 1) / RS8_TILE; }

TKC_DEV uint64_t below_lanes() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// lanes of the wave whose (valid) digit equals this lane's; all 64 lanes call
TKC_DEV uint64_t rs8_match(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

// cnt[d * tiles + tile] = items of digit d in the tile
__global__ void __launch_bounds__(RS8_THREADS) k_rs8_count(const uint32_t* __restrict__ keys, int32_t n, int shift,
                                                            int32_t* cnt, int32_t tiles) {
    __shared__ int32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS8_TILE;
#pragma unroll
    for (int j = 0; j < RS8_ROUNDS; j++) {
        const int64_t i = base + j * RS8_THREADS + t;
        const bool valid = i < n;
        const uint32_t d = valid ? (keys[i] >> shift) & 255u : 0u;
        const uint64_t m = rs8_match(d, valid);
        if (valid && __ffsll((long long)m) - 1 == lane_id()) atomicAdd(&h[d], __popcll(m));
    }
    __syncthreads();
    cnt[(int64_t)t * tiles + blockIdx.x] = h[t];
}

// workgroup d: the exclusive prefix of digit d's counts over the tiles, in
// place, and the digit's total
__global__ void __launch_bounds__(RS8_THREADS) k_rs8_scan(int32_t* cnt, int32_t tiles, int32_t* total) {
    __shared__ int32_t wsum[RS8_THREADS / 64];
    int32_t* row = cnt + (int64_t)blockIdx.x * tiles;
    const int t = threadIdx.x;
    const int32_t per = (tiles + RS8_THREADS - 1) / RS8_THREADS;
    const int32_t lo = t * per, hi = lo + per < tiles ? lo + per : tiles;
    int32_t s = 0;
    for (int32_t q = lo; q < hi; q++) s += row[q];
    int32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane_id() >= o) x += y;
    }
    if (lane_id() == 63) wsum[t >> 6] = x;
    __syncthreads();
    int32_t run = x - s;
    for (int w = 0; w < (t >> 6); w++) run += wsum[w];
    for (int32_t q = lo; q < hi; q++) {
        const int32_t c = row[q];
        row[q] = run;
        run += c;
    }
    if (t == RS8_THREADS - 1) total[blockIdx.x] = run;
}

__global__ void __launch_bounds__(RS8_THREADS) k_rs8_scatter(const uint32_t* __restrict__ keys,
                                                              const int32_t* __restrict__ vals, int32_t n, int shift,
                                                              const int32_t* __restrict__ pre, int32_t tiles,
                                                              const int32_t* __restrict__ total,
                                                              uint32_t* __restrict__ okeys, int32_t* __restrict__ ovals) {
    __shared__ int32_t start[256];   // where digit d's items of this tile go
    __shared__ int32_t run[256];     // of which this many are placed
    __shared__ int32_t wc[RS8_THREADS / 64][256];
    __shared__ int32_t wsum[RS8_THREADS / 64];
    const int t = threadIdx.x, wv = t >> 6, lane = lane_id();
    {   // digits before d over the whole input, then this tile's prefix in d
        const int32_t tot = total[t];
        int32_t x = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int32_t below = x - tot;
        for (int w = 0; w < wv; w++) below += wsum[w];
        start[t] = below + pre[(int64_t)t * tiles + blockIdx.x];
        run[t] = 0;
    }
    const int64_t base = (int64_t)blockIdx.x * RS8_TILE;
    for (int j = 0; j < RS8_ROUNDS; j++) {
        const int64_t i = base + j * RS8_THREADS + t;
        const bool valid = i < n;
        uint32_t k = 0;
        int32_t v = 0;
        if (valid) {
            k = keys[i];
            v = vals[i];
        }
        const uint32_t d = (k >> shift) & 255u;
#pragma unroll
        for (int w = 0; w < RS8_THREADS / 64; w++) wc[w][t] = 0;
        __syncthreads();
        const uint64_t m = rs8_match(d, valid);
        if (valid && __ffsll((long long)m) - 1 == lane) wc[wv][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int32_t pos = start[d] + run[d] + __popcll(m & below_lanes());
            for (int w = 0; w < wv; w++) pos += wc[w][d];
            okeys[pos] = k;
            ovals[pos] = v;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < RS8_THREADS / 64; w++) add += wc[w][t];
        run[t] += add;
    }
}

int64_t tkc_sort8_hist_words(int32_t n) { return 256LL * rs8_tiles(n > 0 ? n : 1) + 256 + 16; }

int tkc_sort_mask(const uint32_t* keys, int32_t n, uint32_t* mask_dev, uint32_t* mask_host, hipStream_t s) {
    if (hipMemsetD32Async((hipDeviceptr_t)mask_dev, 0u, 1, s) != hipSuccess) return -1;
    if (hipMemsetD32Async((hipDeviceptr_t)(mask_dev + 1), 0xffffffffu, 1, s) != hipSuccess) return -1;
    int gb = rs_tiles(n > 0 ? n : 1);
    if (gb > 256) gb = 256;
    hipLaunchKernelGGL(k_rs_mask, dim3(gb), dim3(256), 0, s, keys, n, mask_dev);
    if (hipMemcpyAsync(mask_host, mask_dev, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int tkc_sort_pairs8(uint32_t* keys, int32_t* vals, uint32_t* tmp_keys, int32_t* tmp_vals, int32_t n, int32_t* hist,
                    uint32_t* mask_dev, uint32_t* mask_host, hipStream_t s, const uint32_t* known_mask) {
    if (n <= 1) return 0;
    if (!known_mask) {
        if (tkc_sort_mask(keys, n, mask_dev, mask_host, s)) return -1;
        if (hipStreamSynchronize(s) != hipSuccess) return -1;
        known_mask = mask_host;
    }
    const uint32_t vary = known_mask[0] ^ known_mask[1];
    const int tiles = rs8_tiles(n);
    int32_t* total = hist + 256LL * tiles;
    uint32_t* ka = keys; int32_t* va = vals;
    uint32_t* kb = tmp_keys; int32_t* vb = tmp_vals;
    for (int shift = 0; shift < 32; shift += 8) {
        if (((vary >> shift) & 255u) == 0) continue;
        hipLaunchKernelGGL(k_rs8_count, dim3(tiles), dim3(RS8_THREADS), 0, s, ka, n, shift, hist, tiles);
        hipLaunchKernelGGL(k_rs8_scan, dim3(256), dim3(RS8_THREADS), 0, s, hist, tiles, total);
        hipLaunchKernelGGL(k_rs8_scatter, dim3(tiles), dim3(RS8_THREADS), 0, s, ka, va, n, shift,
                           (const int32_t*)hist, tiles, (const int32_t*)total, kb, vb);
        uint32_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        hipMemcpyAsync(keys, ka, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(vals, va, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
