// Per-row LDS hash tables shared by the counting kernels (both the
// low-pivot and the middle-pivot forms).
#pragma once

#include "tc_internal.h"

namespace tc_tab {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;

// Buckets needed for d keys at load factor <= 1/2: 2^bb >= d/2.
__host__ __device__ __forceinline__ int bucket_bits(int d) {
    int bb = 0;
    while ((1 << bb) * 2 < d) ++bb;
    return bb;
}

// LDS hash table of one row: 2^bb buckets of 4 keys, so a probe is one
// 16-byte LDS read; the index of each key in N_H(v) sits in a parallel
// 16-bit array.  Keys are ranks (< 2^31), EMPTY marks a free slot.
// Buckets fill in slot order, so a bucket whose last slot is free ends a
// search; otherwise the search moves on to the next bucket.
struct RowTable {
    uint32_t *keys;  // 4 << bb words, 16-byte aligned
    uint16_t *pos;   // 4 << bb halfwords
    int bb;
};

// Bucket of a key: a multiplicative hash with the full-rate 24-bit
// multiplier (the key's bits above 20 are folded in first).
__device__ __forceinline__ uint32_t bucket_of(uint32_t key, int bb) {
    const uint32_t h = __umul24(key ^ (key >> 20), 0x9E3779u);
    return bb == 0 ? 0u : h >> (32 - bb);
}

__device__ __forceinline__ void table_insert(const RowTable &t, uint32_t key, uint32_t p) {
    const uint32_t mask = (1u << t.bb) - 1;
    uint32_t b = bucket_of(key, t.bb);
    while (true) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (atomicCAS(&t.keys[4 * b + q], EMPTY, key) == EMPTY) {
                t.pos[4 * b + q] = (uint16_t)p;
                return;
            }
        }
        b = (b + 1) & mask;
    }
}

// Index in N_H(v) of key, or -1.  The first bucket is probed without
// branches (one 16-byte LDS read, selects); only a full bucket without the
// key continues to the next one, which at load factor <= 1/2 is rare.
__device__ __forceinline__ int slot_in(const uint4 &k, uint32_t key) {
    int s = k.w == key ? 3 : -1;
    s = k.z == key ? 2 : s;
    s = k.y == key ? 1 : s;
    s = k.x == key ? 0 : s;
    return s;
}

__device__ __forceinline__ int table_find(const RowTable &t, uint32_t key) {
    const uint32_t mask = (1u << t.bb) - 1;
    const uint4 *kb = reinterpret_cast<const uint4 *>(__builtin_assume_aligned(t.keys, 16));
    uint32_t b = bucket_of(key, t.bb);
    uint4 k = kb[b];
    int s = slot_in(k, key);
    while (s < 0 && k.w != EMPTY) {
        b = (b + 1) & mask;
        k = kb[b];
        s = slot_in(k, key);
    }
    return s < 0 ? -1 : (int)t.pos[4 * b + s];
}

// Probes N keys at once: the N first-bucket reads are all issued before
// any result is used, so their LDS latencies overlap.  Keys above limit
// (EMPTY included) are not members and give -1.  Everything on the common
// path is branch-free; a full bucket without the key (rare at load factor
// <= 1/2) is followed up behind one wave-uniform test per batch.
template <int N>
__device__ __forceinline__ void table_find_n(const RowTable &t, const uint32_t (&key)[N],
                                             uint32_t limit, int (&q)[N]) {
    const uint32_t mask = (1u << t.bb) - 1;
    const uint4 *kb = reinterpret_cast<const uint4 *>(__builtin_assume_aligned(t.keys, 16));
    uint32_t b[N];
    uint4 k[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        b[e] = bucket_of(key[e], t.bb);
        k[e] = kb[b[e]];
    }
    int s[N];
    uint32_t more = 0;
#pragma unroll
    for (int e = 0; e < N; ++e) {
        s[e] = slot_in(k[e], key[e]);
        const bool m = (key[e] <= limit) & (s[e] < 0) & (k[e].w != EMPTY);
        more |= (uint32_t)m << e;
    }
    if (__builtin_expect(__ballot(more != 0) != 0ull, 0)) {
#pragma unroll
        for (int e = 0; e < N; ++e) {
            if ((more >> e) & 1u) {
                uint32_t bb = b[e];
                uint4 kk = k[e];
                int ss = -1;
                while (ss < 0 && kk.w != EMPTY) {
                    bb = (bb + 1) & mask;
                    kk = kb[bb];
                    ss = slot_in(kk, key[e]);
                }
                b[e] = bb;
                s[e] = ss;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const int p = (int)t.pos[4 * b[e] + (s[e] < 0 ? 0 : s[e])];
        q[e] = (key[e] <= limit && s[e] >= 0) ? p : -1;
    }
}

// Position of w in the sorted row ocol[vstart, vstart + dv), or -1.
__device__ __forceinline__ int row_search(const int32_t *__restrict__ ocol, int64_t vstart, int dv,
                                          uint32_t w) {
    int lo = 0, hi = dv;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((uint32_t)ocol[vstart + mid] < w) lo = mid + 1; else hi = mid;
    }
    return (lo < dv && (uint32_t)ocol[vstart + lo] == w) ? lo : -1;
}

// LDS bytes of one table with its 16-bit positions for rows of up to d
// entries (16-byte multiple).
__host__ __device__ __forceinline__ size_t table_bytes(int d) {
    const size_t nb = (size_t)1 << bucket_bits(d);
    return 16 * nb + 8 * nb;
}

}  // namespace tc_tab
