// Stable LSD radix sort, 8-bit digits, for the graph build.
//
// Per digit pass (reduce-then-scan form):
//   k_radix_hist    each tile of TILE keys counts its 256 digits in LDS and
//                   writes them digit-major: counts[d * tiles + tile];
//   tc_scan_u32     exclusive scan of the counts gives, for every (digit,
//                   tile), the first output position of that tile's keys
//                   with that digit (smaller digits first, then earlier
//                   tiles: this is what makes the pass stable);
//   k_radix_scatter every wavefront ranks its keys with 8 ballots per item
//                   (lanes holding the same digit form a 64-bit peer mask;
//                   the rank is the popcount of lower peers plus the
//                   wavefront's running count of that digit), wavefronts
//                   are combined by a per-digit prefix over the block, and
//                   keys (and values) are written to their final place.
// Tile element order is (wavefront, item, lane), which equals memory order,
// so equal digits keep their input order.
#include "tc_internal.h"

namespace {

constexpr int RB = 8;
constexpr int RADIX = 1 << RB;
constexpr int SORT_BLOCK = 256;
constexpr int SORT_WAVES = SORT_BLOCK / TC_WAVE;
// Keys per thread: tiles of 8192 elements for elements (key and value) of
// up to 8 bytes; bigger tiles mean longer runs per digit in the scatter's
// stores.  Wider elements take tiles of 4096, since their registers would
// otherwise leave one wavefront per SIMD, and are staged in two rounds
// (keys, then values, through the same LDS buffer), which keeps their LDS
// near 36 KB.
template <typename K, typename V, bool HAS_VAL>
constexpr int sort_items() {
    return (sizeof(K) + (HAS_VAL ? sizeof(V) : 0)) <= 8 ? 32 : 16;
}
// Below this many elements the big tiles would leave CUs idle: 8 keys per
// thread (tiles of 2048) instead.
constexpr int64_t SORT_BIG_TILES_MIN = (int64_t)1 << 22;
constexpr int SORT_SMALL_ITEMS = 8;

static_assert(SORT_BLOCK == RADIX, "one digit per thread in the scatter's digit scans");

struct NoVal {};

template <typename K, int SORT_ITEMS>
__global__ __launch_bounds__(SORT_BLOCK) void k_radix_hist(const K *__restrict__ keys, int64_t n,
                                                           int shift, uint32_t *__restrict__ counts,
                                                           int64_t tiles) {
    constexpr int SORT_TILE = SORT_BLOCK * SORT_ITEMS;
    __shared__ uint32_t hist[SORT_WAVES][RADIX];
    for (int i = threadIdx.x; i < SORT_WAVES * RADIX; i += SORT_BLOCK) (&hist[0][0])[i] = 0;
    __syncthreads();
    int w = threadIdx.x / TC_WAVE;
    int64_t base = (int64_t)blockIdx.x * SORT_TILE;
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it) {
        int64_t i = base + it * SORT_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&hist[w][(uint32_t)(keys[i] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RADIX; d += SORT_BLOCK) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < SORT_WAVES; ++q) c += hist[q][d];
        counts[(int64_t)d * tiles + blockIdx.x] = c;
    }
}

template <typename K, typename V, bool HAS_VAL, int SORT_ITEMS>
__global__ __launch_bounds__(SORT_BLOCK) void k_radix_scatter(
    const K *__restrict__ kin, const V *__restrict__ vin, K *__restrict__ kout,
    V *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offsets,
    int64_t tiles, const uint32_t *__restrict__ vhi) {
    constexpr int SORT_TILE = SORT_BLOCK * SORT_ITEMS;
    // The tile is first put in digit order in LDS, then written out by
    // consecutive threads to consecutive positions of each digit's run, so
    // the global stores coalesce.
    __shared__ uint32_t wcnt[SORT_WAVES][RADIX];
    __shared__ uint32_t gbase[RADIX];   // global start of the tile's keys of each digit
    __shared__ uint32_t lbase[RADIX];   // start of each digit within the tile
    constexpr int KB = sizeof(K), VB = HAS_VAL ? sizeof(V) : 0;
    constexpr bool SPLIT = HAS_VAL && KB + VB > 8;  // keys and values staged in turn
    constexpr int STAGE = SORT_TILE * (SPLIT ? (KB > VB ? KB : VB) : KB + VB);
    __shared__ __align__(16) unsigned char sraw[STAGE];
    __shared__ uint8_t sdig[SPLIT ? SORT_TILE : 1];  // digit of each staged position
    K *skey = reinterpret_cast<K *>(sraw);
    V *sval = reinterpret_cast<V *>(SPLIT ? sraw : sraw + (size_t)SORT_TILE * KB);
    for (int i = threadIdx.x; i < SORT_WAVES * RADIX; i += SORT_BLOCK) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const int w = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    const uint64_t lt = tc_lanemask_lt();
    const int64_t tbase = (int64_t)blockIdx.x * SORT_TILE;
    const int64_t wbase = tbase + (int64_t)w * (TC_WAVE * SORT_ITEMS);
    const int tn = (int)((n - tbase) < SORT_TILE ? (n - tbase) : SORT_TILE);

    K key[SORT_ITEMS];
    V val[SORT_ITEMS];
    uint32_t rnk[SORT_ITEMS];
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it) {
        int64_t i = wbase + it * TC_WAVE + lane;
        bool valid = i < n;
        key[it] = valid ? kin[i] : (K)0;
        // no value array: the value is the element's index, with vhi[i] in
        // the high half for 64-bit values when vhi is given
        if constexpr (HAS_VAL) {
            V v = 0;
            if (valid) {
                if (vin) {
                    v = vin[i];
                } else {
                    v = (V)i;
                    if constexpr (sizeof(V) == 8)
                        if (vhi) v |= (V)vhi[i] << 32;
                }
            }
            val[it] = v;
        }
    }
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it) {
        int64_t i = wbase + it * TC_WAVE + lane;
        bool valid = i < n;
        uint32_t d = (uint32_t)(key[it] >> shift) & (RADIX - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t prior = 0;
        if (valid) prior = wcnt[w][d];
        rnk[it] = prior + (uint32_t)__popcll(peers & lt);
        // the highest peer publishes the new running count of this digit
        bool last = valid && ((peers >> lane) == 1ull);
        if (last) wcnt[w][d] = prior + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: offsets of the waves, the tile total, and the global base
    uint32_t tot = 0;
    {
        const int d = threadIdx.x;  // SORT_BLOCK == RADIX
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < SORT_WAVES; ++q) {
            uint32_t c = wcnt[q][d];
            wcnt[q][d] = run;
            run += c;
        }
        tot = run;
        gbase[d] = offsets[(int64_t)d * tiles + blockIdx.x];
    }
    // exclusive scan of the digit totals over the workgroup (one digit per thread)
    {
        const uint32_t incl = tc_wave_incl_scan(tot);
        __shared__ uint32_t wsum[SORT_WAVES];
        if (lane == TC_WAVE - 1) wsum[w] = incl;
        __syncthreads();
        uint32_t before = incl - tot;
        for (int q = 0; q < w; ++q) before += wsum[q];
        lbase[threadIdx.x] = before;
    }
    __syncthreads();
    // place of each item in the tile's digit order
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it) {
        int64_t i = wbase + it * TC_WAVE + lane;
        if (i < n) {
            uint32_t d = (uint32_t)(key[it] >> shift) & (RADIX - 1);
            rnk[it] += lbase[d] + wcnt[w][d];
            skey[rnk[it]] = key[it];
            if constexpr (SPLIT) sdig[rnk[it]] = (uint8_t)d;
            else if constexpr (HAS_VAL) sval[rnk[it]] = val[it];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < tn; j += SORT_BLOCK) {
        const K k = skey[j];
        const uint32_t d = (uint32_t)(k >> shift) & (RADIX - 1);
        const uint32_t pos = gbase[d] + (uint32_t)j - lbase[d];
        kout[pos] = k;
        if constexpr (HAS_VAL && !SPLIT) vout[pos] = sval[j];
    }
    if constexpr (SPLIT) {
        __syncthreads();
#pragma unroll
        for (int it = 0; it < SORT_ITEMS; ++it) {
            int64_t i = wbase + it * TC_WAVE + lane;
            if (i < n) sval[rnk[it]] = val[it];
        }
        __syncthreads();
        for (int j = threadIdx.x; j < tn; j += SORT_BLOCK) {
            const uint32_t d = sdig[j];
            vout[gbase[d] + (uint32_t)j - lbase[d]] = sval[j];
        }
    }
}

template <typename K, typename V, bool HAS_VAL, int ITEMS>
tc_status radix_pass(const K *in, const V *vin, K *kout, V *vout, int64_t n, int shift,
                     uint32_t *counts, int64_t tiles, const uint32_t *vhi, hipStream_t s) {
    k_radix_hist<K, ITEMS><<<(unsigned)tiles, SORT_BLOCK, 0, s>>>(in, n, shift, counts, tiles);
    TC_LAUNCHED();
    TC_TRY(tc_scan_u32(counts, counts, tiles * RADIX, nullptr, s));
    k_radix_scatter<K, V, HAS_VAL, ITEMS><<<(unsigned)tiles, SORT_BLOCK, 0, s>>>(
        in, vin, kout, vout, n, shift, counts, tiles, vhi);
    TC_LAUNCHED();
    return TC_OK;
}

// src, when given, is read by the first pass in place of *keys (which then
// needs no contents); with iota the first pass takes each element's index as
// its value in place of *vals.  *keys and *tkeys are ping-pong buffers as
// usual.  With either, at least one pass runs, so the result is always
// written to the buffers.
template <typename K, typename V, bool HAS_VAL>
tc_status radix_sort(K **keys, V **vals, K **tkeys, V **tvals, int64_t n, int bits, hipStream_t s,
                     const K *src = nullptr, bool iota = false, const uint32_t *vhi = nullptr) {
    if (n < 0 || bits < 0 || bits > (int)(8 * sizeof(K))) return TC_ERR_INVALID_ARG;
    const bool fresh = src != nullptr || iota;
    if (n == 0 || (!fresh && (n <= 1 || bits == 0))) return TC_OK;
    if (fresh && bits == 0) bits = 1;  // keys below 2^0 are all zero: one pass keeps the order
    if (n >= (int64_t)0xFFFFFFFFll) return TC_ERR_UNSUPPORTED;
    constexpr int ITEMS = sort_items<K, V, HAS_VAL>();
    const bool big = n >= SORT_BIG_TILES_MIN;
    int64_t tiles = tc_div_up(n, (int64_t)SORT_BLOCK * (big ? ITEMS : SORT_SMALL_ITEMS));
    tc_scratch tmp(s);
    uint32_t *counts = nullptr;
    TC_TRY(tmp.get(&counts, tiles * RADIX));
    for (int shift = 0; shift < bits; shift += RB) {
        const K *in = (src && shift == 0) ? src : *keys;
        const V *vin = (HAS_VAL && !(iota && shift == 0)) ? *vals : nullptr;
        V *vout = HAS_VAL ? *tvals : nullptr;
        const uint32_t *vh = shift == 0 ? vhi : nullptr;
        if (big)
            TC_TRY((radix_pass<K, V, HAS_VAL, ITEMS>(in, vin, *tkeys, vout, n, shift, counts, tiles,
                                                     vh, s)));
        else
            TC_TRY((radix_pass<K, V, HAS_VAL, SORT_SMALL_ITEMS>(in, vin, *tkeys, vout, n, shift,
                                                                counts, tiles, vh, s)));
        TC_LAUNCHED();
        K *tk = *keys;
        *keys = *tkeys;
        *tkeys = tk;
        if constexpr (HAS_VAL) {
            V *tv = *vals;
            *vals = *tvals;
            *tvals = tv;
        }
    }
    return TC_OK;
}

}  // namespace

tc_status tc_sort_u64(uint64_t **keys, uint64_t **tmp_keys, int64_t n, int bits, hipStream_t s) {
    uint32_t *nv = nullptr, *ntv = nullptr;
    return radix_sort<uint64_t, uint32_t, false>(keys, &nv, tmp_keys, &ntv, n, bits, s);
}


tc_status tc_sort_u32_index(const uint32_t *src, uint32_t **keys, uint32_t **vals,
                            uint32_t **tmp_keys, uint32_t **tmp_vals, int64_t n, int bits,
                            hipStream_t s) {
    return radix_sort<uint32_t, uint32_t, true>(keys, vals, tmp_keys, tmp_vals, n, bits, s, src,
                                                true);
}

tc_status tc_sort_u32_index_hi(const uint32_t *src, const uint32_t *hi, uint32_t **keys,
                               uint64_t **vals, uint32_t **tmp_keys, uint64_t **tmp_vals,
                               int64_t n, int bits, hipStream_t s) {
    return radix_sort<uint32_t, uint64_t, true>(keys, vals, tmp_keys, tmp_vals, n, bits, s, src,
                                                true, hi);
}

tc_status tc_sort_u64_u32(uint64_t **keys, uint32_t **vals, uint64_t **tmp_keys,
                          uint32_t **tmp_vals, int64_t n, int bits, hipStream_t s) {
    return radix_sort<uint64_t, uint32_t, true>(keys, vals, tmp_keys, tmp_vals, n, bits, s);
}

tc_status tc_partition_u32_u32(const uint32_t *keys, const uint32_t *vals, uint32_t *keys_out,
                               uint32_t *vals_out, int64_t n, int shift, hipStream_t s) {
    if (n < 0 || shift < 0 || shift > 24) return TC_ERR_INVALID_ARG;
    if (n == 0) return TC_OK;
    if (n >= (int64_t)0xFFFFFFFFll) return TC_ERR_UNSUPPORTED;
    constexpr int ITEMS = sort_items<uint32_t, uint32_t, true>();
    const bool big = n >= SORT_BIG_TILES_MIN;
    const int64_t tiles = tc_div_up(n, (int64_t)SORT_BLOCK * (big ? ITEMS : SORT_SMALL_ITEMS));
    tc_scratch tmp(s);
    uint32_t *counts = nullptr;
    TC_TRY(tmp.get(&counts, tiles * RADIX));
    if (big)
        return radix_pass<uint32_t, uint32_t, true, ITEMS>(keys, vals, keys_out, vals_out, n, shift,
                                                           counts, tiles, nullptr, s);
    return radix_pass<uint32_t, uint32_t, true, SORT_SMALL_ITEMS>(keys, vals, keys_out, vals_out, n,
                                                                  shift, counts, tiles, nullptr, s);
}

tc_status tc_sort_u32_u32(uint32_t **keys, uint32_t **vals, uint32_t **tmp_keys,
                          uint32_t **tmp_vals, int64_t n, int bits, hipStream_t s) {
    return radix_sort<uint32_t, uint32_t, true>(keys, vals, tmp_keys, tmp_vals, n, bits, s);
}

