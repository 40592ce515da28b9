// Device-wide exclusive prefix sum (reduce-then-scan).
//
// Tiles of TILE = BLOCK*ITEMS elements: one kernel reduces every tile, the
// tile totals are scanned recursively, and a second kernel rescans each
// tile in LDS and adds its tile offset.  Loads and stores are coalesced
// (striped through LDS); each thread scans ITEMS consecutive elements.
#include "tc_internal.h"

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;
constexpr int SCAN_WAVES = SCAN_BLOCK / TC_WAVE;

template <typename T>
__device__ T block_sum(T x, T *red) {
    x = tc_wave_sum(x);
    int w = threadIdx.x / TC_WAVE;
    if (__lane_id() == 0) red[w] = x;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int i = 0; i < SCAN_WAVES; ++i) t += red[i];
    return t;
}

template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_reduce(const T *__restrict__ in, int64_t n,
                                                            T *__restrict__ partial) {
    __shared__ T red[SCAN_WAVES];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        int64_t i = base + it * SCAN_BLOCK + threadIdx.x;
        if (i < n) acc += in[i];
    }
    T t = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Exclusive scan of one tile; tile_off (may be null) holds scanned tile
// offsets.  The block that owns the last element writes the grand total.
template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan(const T *in, T *out, int64_t n,
                                                          const T *__restrict__ tile_off,
                                                          T *total) {
    __shared__ T buf[SCAN_TILE];
    __shared__ T wsum[SCAN_WAVES];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        int j = it * SCAN_BLOCK + tid;
        int64_t i = base + j;
        buf[j] = (i < n) ? in[i] : (T)0;
    }
    __syncthreads();
    T v[SCAN_ITEMS];
    T run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = run;
        run += buf[tid * SCAN_ITEMS + k];
    }
    T incl = tc_wave_incl_scan(run);
    int w = tid / TC_WAVE;
    if (__lane_id() == TC_WAVE - 1) wsum[w] = incl;
    __syncthreads();
    T before = incl - run;
    for (int i = 0; i < w; ++i) before += wsum[i];
    T off = tile_off ? tile_off[blockIdx.x] : (T)0;
    before += off;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) buf[tid * SCAN_ITEMS + k] = v[k] + before;
    if (total != nullptr && tid == SCAN_BLOCK - 1 && base + SCAN_TILE >= n) {
        *total = before + run;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; ++it) {
        int j = it * SCAN_BLOCK + tid;
        int64_t i = base + j;
        if (i < n) out[i] = buf[j];
    }
}

template <typename T>
__global__ void k_set_zero(T *p) { *p = 0; }

template <typename T>
tc_status scan_impl(const T *in, T *out, int64_t n, T *total, hipStream_t s) {
    if (n < 0) return TC_ERR_INVALID_ARG;
    if (n == 0) {
        if (total) {
            k_set_zero<T><<<1, 1, 0, s>>>(total);
            TC_LAUNCHED();
        }
        return TC_OK;
    }
    int64_t tiles = tc_div_up(n, SCAN_TILE);
    if (tiles == 1) {
        k_tile_scan<T><<<1, SCAN_BLOCK, 0, s>>>(in, out, n, nullptr, total);
        TC_LAUNCHED();
        return TC_OK;
    }
    if (tiles > 0x7FFFFFFF) return TC_ERR_UNSUPPORTED;
    tc_scratch tmp(s);
    T *partial = nullptr;
    TC_TRY(tmp.get(&partial, tiles));
    k_tile_reduce<T><<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(in, n, partial);
    TC_LAUNCHED();
    TC_TRY(scan_impl<T>(partial, partial, tiles, (T *)nullptr, s));
    k_tile_scan<T><<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(in, out, n, partial, total);
    TC_LAUNCHED();
    return TC_OK;
}

}  // namespace

tc_status tc_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                      hipStream_t s) {
    return scan_impl<uint32_t>(in, out, n, total, s);
}

tc_status tc_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total,
                      hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, total, s);
}
