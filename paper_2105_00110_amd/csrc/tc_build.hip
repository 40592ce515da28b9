// Graph build on the device: normalisation into the canonical edge list
// and the symmetric CSR, the degree ordering, and the degree-ordered
// orientation.
//
//  1. Pack every pair as the 64-bit key (min << bits) | max (self-loops
//     become a sentinel above every real key), radix sort, keep first
//     occurrences: canonical edges (u < v) in lexicographic order.
//  2. Symmetric CSR in original ids.  Row x is [smaller neighbours] then
//     [larger neighbours]; the larger ones are the run of canonical edges
//     with eu = x (already sorted), the smaller ones come from a stable
//     sort of (ev, e) -- the transpose -- which lists them by increasing eu.
//  3. Degree ordering π (Sec. "Notation"): position in the order by
//     (degree, id), from a stable sort of degrees over ids in id order.
//  4. Orientation: each canonical edge becomes (π(low), π(high)); a sort of
//     these packed keys yields the oriented CSR whose row r lists the
//     higher-ordered neighbours N_H of the rank-r vertex, ascending.  This
//     is the paper's split of N(v) into N_L(v) | N_H(v) (Lemma 1's proof),
//     stored as its own compact array for the counting kernels.
#include <stdlib.h>

#include "tc_internal.h"

namespace {

constexpr int BK = 256;

static inline unsigned grid_for(int64_t n, int block = BK) {
    int64_t g = tc_div_up(n, block);
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (unsigned)g;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// Pair -> packed canonical key.  For a batch, pair i belongs to the graph g
// with pair_off[g] <= i < pair_off[g+1]; its ids are local and get the
// graph's first global vertex id added.
__global__ void k_make_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                            int64_t P, int32_t n, int bits, const int64_t *__restrict__ pair_off,
                            const int64_t *__restrict__ vtx_off, int32_t G,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ err) {
    const uint64_t sentinel = (bits >= 32) ? ~0ull : ((1ull << (2 * bits)) - 1);
    GRID_STRIDE(i, P) {
        int64_t a = src[i], b = dst[i];
        int64_t lim = n, base = 0;
        if (pair_off != nullptr) {
            int32_t lo = 0, hi = G - 1;  // last g with pair_off[g] <= i
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (pair_off[mid] <= i) lo = mid; else hi = mid - 1;
            }
            base = vtx_off[lo];
            lim = vtx_off[lo + 1] - base;
        }
        uint64_t key;
        if (a < 0 || a >= lim || b < 0 || b >= lim) {
            atomicOr(err, 1u);
            key = sentinel;
        } else if (a == b) {
            key = sentinel;
        } else {
            uint64_t lo = (uint64_t)((a < b ? a : b) + base), hi = (uint64_t)((a < b ? b : a) + base);
            key = (lo << bits) | hi;
        }
        keys[i] = key;
    }
}

// Deduplication as a two-pass compaction over tiles of UQ_TILE sorted keys:
// k_unique_count counts each tile's canonical edges (the first key of every
// run of equal keys, sentinels excluded), the tile counts are scanned, and
// k_unique_emit recomputes the flags, places them by a workgroup scan and
// stores the tile's edges side by side.  Every key is read twice and every
// edge written once; no per-key flag or position array goes to memory.
constexpr int UQ_BLOCK = 256;
constexpr int UQ_ITEMS = 16;
constexpr int UQ_TILE = UQ_BLOCK * UQ_ITEMS;

__device__ __forceinline__ bool first_of_run(const uint64_t *__restrict__ keys, int64_t i,
                                             uint64_t k, uint64_t sentinel) {
    return k != sentinel && (i == 0 || keys[i - 1] != k);
}

__global__ __launch_bounds__(UQ_BLOCK) void k_unique_count(const uint64_t *__restrict__ keys,
                                                           int64_t P, uint64_t sentinel,
                                                           uint32_t *__restrict__ cnt) {
    __shared__ uint32_t red[UQ_BLOCK / TC_WAVE];
    const int64_t base = (int64_t)blockIdx.x * UQ_TILE;
    uint32_t c = 0;
#pragma unroll
    for (int it = 0; it < UQ_ITEMS; ++it) {
        const int64_t i = base + it * UQ_BLOCK + threadIdx.x;
        if (i < P) c += first_of_run(keys, i, keys[i], sentinel) ? 1u : 0u;
    }
    c = tc_wave_sum(c);
    if (__lane_id() == 0) red[threadIdx.x / TC_WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < UQ_BLOCK / TC_WAVE; ++w) t += red[w];
        cnt[blockIdx.x] = t;
    }
}

// Writes the canonical edges of each tile at tile_off[tile] and, in the same
// pass, the run [us[u], ue[u]) of the edges whose smaller end is u (edges
// come sorted by it).  us and ue start zeroed; the end of the last run is set
// by k_last_run.
__global__ __launch_bounds__(UQ_BLOCK) void k_unique_emit(const uint64_t *__restrict__ keys,
                                                          int64_t P, uint64_t sentinel, int bits,
                                                          const uint32_t *__restrict__ tile_off,
                                                          int32_t *__restrict__ eu,
                                                          int32_t *__restrict__ ev,
                                                          uint32_t *__restrict__ us,
                                                          uint32_t *__restrict__ ue) {
    constexpr int W = UQ_BLOCK / TC_WAVE;
    __shared__ int32_t su[UQ_TILE], sv[UQ_TILE];
    __shared__ uint32_t cnt[UQ_ITEMS * W];  // flags per (item, wavefront), then their prefix
    __shared__ uint32_t total;
    const uint64_t mask = (1ull << bits) - 1;
    const int64_t base = (int64_t)blockIdx.x * UQ_TILE;
    const int w = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    const uint64_t lt = tc_lanemask_lt();
    // element it * UQ_BLOCK + threadIdx.x of the tile: a wavefront holds 64
    // consecutive elements per item, and tile order is (item, wavefront, lane)
    uint64_t k[UQ_ITEMS], prev[UQ_ITEMS], fl[UQ_ITEMS];
#pragma unroll
    for (int it = 0; it < UQ_ITEMS; ++it) {
        const int64_t i = base + it * UQ_BLOCK + threadIdx.x;
        k[it] = i < P ? keys[i] : sentinel;
        prev[it] = (i > 0 && i < P) ? keys[i - 1] : sentinel;
        fl[it] = __ballot(k[it] != sentinel && (i == 0 || prev[it] != k[it]));
        if (lane == 0) cnt[it * W + w] = (uint32_t)__popcll(fl[it]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int q = 0; q < UQ_ITEMS * W; ++q) {
            const uint32_t c = cnt[q];
            cnt[q] = run;
            run += c;
        }
        total = run;
    }
    __syncthreads();
    const uint32_t p0 = tile_off[blockIdx.x];
#pragma unroll
    for (int it = 0; it < UQ_ITEMS; ++it) {
        if ((fl[it] >> lane) & 1ull) {
            const uint32_t lp = cnt[it * W + w] + (uint32_t)__popcll(fl[it] & lt);
            const uint32_t u = (uint32_t)(k[it] >> bits), v = (uint32_t)(k[it] & mask);
            su[lp] = (int32_t)u;
            sv[lp] = (int32_t)v;
            // prev is the previous distinct key (sentinels sort last)
            const uint32_t pu = (uint32_t)(prev[it] >> bits);
            if (base + it * UQ_BLOCK + threadIdx.x == 0) {
                us[u] = 0;
            } else if (pu != u) {
                us[u] = p0 + lp;
                ue[pu] = p0 + lp;
            }
        }
    }
    __syncthreads();
    const uint32_t tot = total;
    for (uint32_t j = threadIdx.x; j < tot; j += UQ_BLOCK) {
        eu[p0 + j] = su[j];
        ev[p0 + j] = sv[j];
    }
}

// A CSR given as simple and sorted: each row strictly increasing, ids in
// [0, n), no self-loop (checked: a violation sets err).  Its entries above
// the diagonal, row by row, are the canonical edges in order; cnt[v] counts
// row v's.
__global__ void k_csr_upper_count(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                  int32_t n, uint32_t *__restrict__ cnt,
                                  uint32_t *__restrict__ err) {
    GRID_STRIDE(v, n) {
        const int64_t a = rp[v], b = rp[v + 1];
        bool bad = b < a;
        uint32_t c = 0;
        for (int64_t j = a; j < b && !bad; ++j) {
            const int32_t x = col[j];
            bad = x < 0 || x >= n || x == (int32_t)v || (j > a && col[j - 1] >= x);
            c += x > (int32_t)v ? 1u : 0u;
        }
        if (bad) atomicOr(err, 1u);
        cnt[v] = bad ? 0u : c;
    }
}

// Writes row v's upper entries as canonical edges off[v] .. off[v] + cnt[v]
// - 1 and their run [us[v], ue[v]) (left zero for an empty run).
__global__ void k_csr_upper_emit(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                 int32_t n, const uint32_t *__restrict__ cnt,
                                 const uint32_t *__restrict__ off, int32_t *__restrict__ eu,
                                 int32_t *__restrict__ ev, uint32_t *__restrict__ us,
                                 uint32_t *__restrict__ ue) {
    GRID_STRIDE(v, n) {
        const uint32_t c = cnt[v];
        if (c == 0) continue;
        const int64_t b = rp[v + 1], first = b - c;
        const uint32_t o = off[v];
        for (int64_t j = first; j < b; ++j) {
            eu[o + (j - first)] = (int32_t)v;
            ev[o + (j - first)] = col[j];
        }
        us[v] = o;
        ue[v] = o + c;
    }
}

__global__ void k_last_run(int64_t m, const int32_t *__restrict__ eu, uint32_t *__restrict__ ue) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ue[eu[m - 1]] = (uint32_t)m;
}

// Run boundaries of a sorted id sequence: start/end of each present id.
// start and end must be zeroed first.
template <typename Get>
__global__ void k_runs(Get get, int64_t len, uint32_t *__restrict__ start,
                       uint32_t *__restrict__ end) {
    GRID_STRIDE(i, len) {
        uint32_t x = get(i);
        if (i == 0 || get(i - 1) != x) start[x] = (uint32_t)i;
        if (i == len - 1 || get(i + 1) != x) end[x] = (uint32_t)(i + 1);
    }
}

struct GetU32 {
    const uint32_t *a;
    __device__ uint32_t operator()(int64_t i) const { return a[i]; }
};
struct GetHigh {
    const uint64_t *a;
    int bits;
    __device__ uint32_t operator()(int64_t i) const { return (uint32_t)(a[i] >> bits); }
};

__global__ void k_degree(int32_t n, const uint32_t *__restrict__ us, const uint32_t *__restrict__ ue,
                         const uint32_t *__restrict__ ls, const uint32_t *__restrict__ le,
                         int64_t *__restrict__ deg64, uint32_t *__restrict__ deg32) {
    GRID_STRIDE(x, n) {
        uint32_t d = (ue[x] - us[x]) + (le[x] - ls[x]);
        deg64[x] = d;
        deg32[x] = d;
    }
}

// Smaller neighbours: transposed entry j = (ev, e) sorted by ev.
__global__ void k_fill_lower(int64_t m, const uint32_t *__restrict__ tkey,
                             const uint32_t *__restrict__ tval, const uint32_t *__restrict__ lstart,
                             const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ eu,
                             int32_t *__restrict__ col, uint32_t *__restrict__ sym2e) {
    GRID_STRIDE(j, m) {
        uint32_t x = tkey[j], e = tval[j];
        int64_t p = row_ptr[x] + (j - (int64_t)lstart[x]);
        col[p] = eu[e];
        sym2e[p] = e;
    }
}

// Larger neighbours: canonical edge e = (x, v) is the (e - ustart[x])-th.
__global__ void k_fill_upper(int64_t m, const int32_t *__restrict__ eu,
                             const int32_t *__restrict__ ev, const uint32_t *__restrict__ ustart,
                             const uint32_t *__restrict__ lstart, const uint32_t *__restrict__ lend,
                             const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                             uint32_t *__restrict__ sym2e) {
    GRID_STRIDE(e, m) {
        uint32_t x = (uint32_t)eu[e];
        int64_t p = row_ptr[x] + (lend[x] - lstart[x]) + (e - (int64_t)ustart[x]);
        col[p] = ev[e];
        sym2e[p] = (uint32_t)e;
    }
}

__global__ void k_iota(uint32_t *a, int64_t n) {
    GRID_STRIDE(i, n) a[i] = (uint32_t)i;
}

__global__ void k_invert(const uint32_t *__restrict__ perm, int32_t n, int32_t *__restrict__ perm_out,
                         int32_t *__restrict__ rank) {
    GRID_STRIDE(r, n) {
        uint32_t v = perm[r];
        perm_out[r] = (int32_t)v;
        rank[v] = (int32_t)r;
    }
}

__global__ void k_orient_keys(int64_t m, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                              const int32_t *__restrict__ rank, int bits, uint64_t *__restrict__ okey,
                              uint32_t *__restrict__ oval) {
    GRID_STRIDE(e, m) {
        uint64_t a = (uint32_t)rank[eu[e]], b = (uint32_t)rank[ev[e]];
        uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        okey[e] = (lo << bits) | hi;
        oval[e] = (uint32_t)e;
    }
}

__global__ void k_orient_split(int64_t m, const uint64_t *__restrict__ okey, int bits,
                               int32_t *__restrict__ ocol, int32_t *__restrict__ orow) {
    const uint64_t mask = (1ull << bits) - 1;
    GRID_STRIDE(k, m) {
        ocol[k] = (int32_t)(okey[k] & mask);
        orow[k] = (int32_t)(okey[k] >> bits);
    }
}

__global__ void k_run_len64(int32_t n, const uint32_t *__restrict__ s, const uint32_t *__restrict__ e,
                            int64_t *__restrict__ len, uint32_t *__restrict__ maxlen) {
    // one atomic per wavefront: a single word hit by every thread serialises
    uint32_t mx = 0;
    GRID_STRIDE(x, n) {
        uint32_t d = e[x] - s[x];
        len[x] = d;
        mx = d > mx ? d : mx;
    }
    mx = tc_wave_max(mx);
    if (__lane_id() == 0 && mx) atomicMax(maxlen, mx);
}

// ---------------------------------------------------------------------------
// Orientation without a global sort (every row at most SEG_MAX entries):
//   pass A  each canonical edge is written once, into the bucket of its
//           lower-ordered endpoint x: (rank of the other end, edge id) at
//           tmp[row_ptr[x] + slot] (a bucket never outgrows x's symmetric
//           row).  The edges are visited twice, in canonical order (runs of
//           the smaller id u) taking those with x = u, and ordered by the
//           larger id (runs of v) taking those with x = v, so a wavefront's
//           entries for one bucket are neighbours and take their slots with
//           one atomic on x's cursor, and are stored side by side;
//   pass B  d+ = the cursors, scanned into the offsets of the rank rows;
//           each bucket is put in order by rank in LDS and written to
//           ocol/o2e, with the row of every slot in orow.
// ---------------------------------------------------------------------------
constexpr int SEG_MAX = 4096;
constexpr int SEG_WAVE = 64;    // buckets up to this many entries: a group of lanes each
constexpr int SEG_SMALL = 256;  // up to this many: k_orient_small; above: bitonic sorts

// Lanes hold consecutive elements of a sequence sorted by x (x is the same
// for neighbouring lanes of one run); the active ones store their entry in
// x's bucket, each run's active lanes taking consecutive slots with one
// atomic.
__device__ __forceinline__ void place_runs(bool valid, int32_t x, bool active, uint64_t entry,
                                           const int64_t *__restrict__ row_ptr,
                                           uint32_t *__restrict__ cursor,
                                           uint64_t *__restrict__ tbuf) {
    const int lane = __lane_id();
    const int32_t prev = __shfl_up(x, 1, TC_WAVE);
    const bool head = valid && (lane == 0 || prev != x);
    const uint64_t heads = __ballot(head);
    const uint64_t acts = __ballot(valid && active);
    const uint64_t upto = (2ull << lane) - 1;             // lanes 0..lane
    const uint64_t below = (1ull << lane) - 1;            // lanes 0..lane-1
    const uint64_t mine = heads & upto;
    const int hl = mine ? 63 - __clzll((long long)mine) : 0;  // head of this lane's run
    uint32_t base = 0;
    if (head) {
        const uint64_t later = heads & ~upto;
        const uint64_t run = (later ? ((later & (0 - later)) - 1) : ~0ull) & ~below;
        const uint32_t cnt = (uint32_t)__popcll(acts & run);
        if (cnt) base = atomicAdd(&cursor[x], cnt);
    }
    base = __shfl(base, hl, TC_WAVE);
    if (valid && active) {
        const uint64_t before = acts & below & ~((1ull << hl) - 1);  // active lanes in [hl, lane)
        tbuf[row_ptr[x] + base + (uint32_t)__popcll(before)] = entry;
    }
}

// Canonical order: edge e = (u, v), u < v; x = u when u is ordered first.
// Also records the rank of u per edge for the second pass.
__global__ void k_place_by_smaller(int64_t m, const int32_t *__restrict__ eu,
                                   const int32_t *__restrict__ ev, const int32_t *__restrict__ rank,
                                   const int64_t *__restrict__ row_ptr,
                                   uint32_t *__restrict__ cursor, uint64_t *__restrict__ tbuf,
                                   uint32_t *__restrict__ rank_u) {
    const int lane = __lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; e0 < m; e0 += stride) {
        const int64_t e = e0 + lane;
        const bool valid = e < m;
        int32_t u = -1;
        bool active = false;
        uint64_t entry = 0;
        if (valid) {
            u = eu[e];
            const uint32_t a = (uint32_t)rank[u], b = (uint32_t)rank[ev[e]];
            rank_u[e] = a;
            active = a < b;
            entry = ((uint64_t)b << 32) | (uint32_t)e;
        }
        place_runs(valid, u, active, entry, row_ptr, cursor, tbuf);
    }
}

// Edges ordered by the larger id v (key v, value e): x = v when v is
// ordered first.
__global__ void k_place_by_larger(int64_t m, const uint32_t *__restrict__ lt_key,
                                  const uint32_t *__restrict__ lt_val,
                                  const int32_t *__restrict__ rank,
                                  const uint32_t *__restrict__ rank_u,
                                  const int64_t *__restrict__ row_ptr,
                                  uint32_t *__restrict__ cursor, uint64_t *__restrict__ tbuf) {
    const int lane = __lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; j0 < m; j0 += stride) {
        const int64_t j = j0 + lane;
        const bool valid = j < m;
        int32_t v = -1;
        bool active = false;
        uint64_t entry = 0;
        if (valid) {
            v = (int32_t)lt_key[j];
            const uint32_t e = lt_val[j];
            const uint32_t a = rank_u[e], b = (uint32_t)rank[v];
            active = b < a;
            entry = ((uint64_t)a << 32) | e;
        }
        place_runs(valid, v, active, entry, row_ptr, cursor, tbuf);
    }
}

// d+ by rank row, and its maximum.
__global__ void k_dplus_by_rank(int32_t n, const uint32_t *__restrict__ cursor,
                                const int32_t *__restrict__ rank, int64_t *__restrict__ dplus,
                                uint32_t *__restrict__ dmax) {
    uint32_t mx = 0;
    GRID_STRIDE(x, n) {
        const uint32_t d = cursor[x];
        dplus[rank[x]] = d;
        mx = d > mx ? d : mx;
    }
    mx = tc_wave_max(mx);
    if (__lane_id() == 0 && mx) atomicMax(dmax, mx);
}

// Buckets of 1..SEG_SMALL entries.  Every wavefront reads the sizes of 64
// consecutive vertices and sorts their buckets by size class (lo, GL],
// GL = 8, 16, 32, 64: GL lanes per bucket, 64 / GL buckets at a time, taken
// from the ballot of the class (classes (64, 128] and (128, 256]: the whole
// wavefront, orient_class_wide).  Each lane places its entry by the number of
// smaller keys in its group (keys of a bucket are distinct ranks).  The grid
// strides over the vertices, so there is no wavefront per vertex to
// dispatch.
template <int GL>
__device__ __forceinline__ void orient_class(int64_t x0, uint32_t dl, uint32_t lo, uint32_t *wsk,
                                             int64_t bl, int32_t rl, int64_t ol,
                                             const uint64_t *__restrict__ tbuf,
                                             int32_t *__restrict__ ocol, uint32_t *__restrict__ o2e,
                                             int32_t *__restrict__ orow) {
    static_assert(GL <= SEG_WAVE && TC_WAVE % GL == 0, "group size");
    constexpr int GPW = TC_WAVE / GL;
    const int lane = __lane_id();
    const int grp = lane / GL, sl = lane % GL;
    uint32_t *gsk = wsk + grp * GL;
    uint64_t mask = __ballot(dl > lo && dl <= (uint32_t)GL);
    while (mask) {
        // this group's vertex: the grp-th set bit of the mask, if any
        uint64_t mm = mask;
        for (int q = 0; q < grp && mm; ++q) mm &= mm - 1;
        const bool has = mm != 0;
        const int j = has ? __ffsll((long long)mm) - 1 : 0;
        for (int q = 0; q < GPW && mask; ++q) mask &= mask - 1;
        const int d = (int)__shfl(dl, j, TC_WAVE);
        // the row's bucket start, rank and oriented start, loaded once per
        // chunk by the lane of the vertex
        const int64_t bx = __shfl(bl, j, TC_WAVE);
        const int32_t rx = __shfl(rl, j, TC_WAVE);
        const int64_t ob = __shfl(ol, j, TC_WAVE);
        const bool mine = has && sl < d;
        uint32_t key = 0xFFFFFFFFu, val = 0;
        if (mine) {
            const uint64_t w = tbuf[bx + sl];
            key = (uint32_t)(w >> 32);
            val = (uint32_t)w;
        }
        gsk[sl] = key;
        __builtin_amdgcn_wave_barrier();
        if (mine) {
            int pos = 0;
            for (int t = 0; t < d; ++t) pos += gsk[t] < key ? 1 : 0;
            const int64_t k = ob + pos;
            ocol[k] = (int32_t)key;
            o2e[k] = val;
            orow[k] = rx;
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Buckets of lo < d <= 64 E entries: the whole wavefront, E entries per
// lane, each placed by counting the smaller keys (the keys are read back from
// LDS one at a time, the same word for every lane).
template <int E>
__device__ __forceinline__ void orient_class_wide(int64_t x0, uint32_t dl, uint32_t lo,
                                                  uint32_t *wsk, int64_t bl, int32_t rl,
                                                  int64_t ol, const uint64_t *__restrict__ tbuf,
                                                  int32_t *__restrict__ ocol,
                                                  uint32_t *__restrict__ o2e,
                                                  int32_t *__restrict__ orow) {
    const int lane = __lane_id();
    uint64_t mask = __ballot(dl > lo && dl <= (uint32_t)(TC_WAVE * E));
    while (mask) {
        const int j = __ffsll((long long)mask) - 1;
        mask &= mask - 1;
        const int d = (int)__shfl(dl, j, TC_WAVE);
        const int64_t b = __shfl(bl, j, TC_WAVE);
        const int32_t rx = __shfl(rl, j, TC_WAVE);
        const int64_t ob = __shfl(ol, j, TC_WAVE);
        uint32_t key[E], val[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = lane + TC_WAVE * e;
            key[e] = 0xFFFFFFFFu;
            val[e] = 0;
            if (i < d) {
                const uint64_t w = tbuf[b + i];
                key[e] = (uint32_t)(w >> 32);
                val[e] = (uint32_t)w;
            }
            wsk[i] = key[e];
        }
        __builtin_amdgcn_wave_barrier();
        int pos[E];
#pragma unroll
        for (int e = 0; e < E; ++e) pos[e] = 0;
        for (int t = 0; t < d; ++t) {
            const uint32_t kt = wsk[t];
#pragma unroll
            for (int e = 0; e < E; ++e) pos[e] += kt < key[e] ? 1 : 0;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (lane + TC_WAVE * e < d) {
                ocol[ob + pos[e]] = (int32_t)key[e];
                o2e[ob + pos[e]] = val[e];
                orow[ob + pos[e]] = rx;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ __launch_bounds__(256) void k_orient_small(
    int32_t n, const int64_t *__restrict__ row_ptr, const uint32_t *__restrict__ cursor,
    const int32_t *__restrict__ rank, const int64_t *__restrict__ orp,
    const uint64_t *__restrict__ tbuf, int32_t *__restrict__ ocol, uint32_t *__restrict__ o2e,
    int32_t *__restrict__ orow) {
    __shared__ uint32_t sk[4][SEG_SMALL];
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t x0 = ((int64_t)blockIdx.x * 4 + wv) * TC_WAVE; x0 < n; x0 += nwaves * TC_WAVE) {
        const int64_t xl = x0 + lane;
        const uint32_t dl = xl < n ? cursor[xl] : 0u;
        // each lane's vertex: bucket start, rank, oriented row start (the
        // rows of every class in this chunk read them from here)
        int64_t bl = 0, ol = 0;
        int32_t rl = 0;
        if (dl > 0) {
            bl = row_ptr[xl];
            rl = rank[xl];
            ol = orp[rl];
        }
        orient_class<8>(x0, dl, 0, sk[wv], bl, rl, ol, tbuf, ocol, o2e, orow);
        orient_class<16>(x0, dl, 8, sk[wv], bl, rl, ol, tbuf, ocol, o2e, orow);
        orient_class<32>(x0, dl, 16, sk[wv], bl, rl, ol, tbuf, ocol, o2e, orow);
        orient_class<64>(x0, dl, 32, sk[wv], bl, rl, ol, tbuf, ocol, o2e, orow);
        orient_class_wide<2>(x0, dl, 64, sk[wv], bl, rl, ol, tbuf, ocol, o2e, orow);
        orient_class_wide<4>(x0, dl, 128, sk[wv], bl, rl, ol, tbuf, ocol, o2e, orow);
    }
}

// One workgroup per listed vertex (more than SEG_MID entries): the bucket
// as packed (rank << 32 | edge) words, padded with all-ones words to a power
// of two, is put in order by a bitonic sort in LDS.
__global__ __launch_bounds__(256) void k_orient_block(
    const int32_t *__restrict__ list, int64_t nlist, const int64_t *__restrict__ row_ptr,
    const uint32_t *__restrict__ cursor, const int32_t *__restrict__ rank,
    const int64_t *__restrict__ orp, const uint64_t *__restrict__ tbuf,
    int32_t *__restrict__ ocol, uint32_t *__restrict__ o2e, int32_t *__restrict__ orow) {
    __shared__ uint64_t sk[SEG_MAX];
    const int tid = threadIdx.x;
    for (int64_t i = blockIdx.x; i < nlist; i += gridDim.x) {
        const int32_t x = list[i];
        const int32_t rx = rank[x];
        const int64_t ob = orp[rx];
        const int d = (int)cursor[x];
        const int64_t b = row_ptr[x];
        int P = 1;
        while (P < d) P <<= 1;
        for (int j = tid; j < P; j += 256)
            sk[j] = j < d ? tbuf[b + j] : ~0ull;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = tid; t < (P >> 1); t += 256) {
                    // t-th pair of this round: lower index a, partner a + j
                    const int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                    const uint64_t va = sk[a], vb = sk[a + j];
                    const bool up = (a & k) == 0;
                    if ((va > vb) == up) {
                        sk[a] = vb;
                        sk[a + j] = va;
                    }
                }
                __syncthreads();
            }
        }
        for (int t = tid; t < d; t += 256) {
            const uint64_t w = sk[t];
            ocol[ob + t] = (int32_t)(w >> 32);
            o2e[ob + t] = (uint32_t)w;
            orow[ob + t] = rx;
        }
        __syncthreads();
    }
}

// One wavefront per listed vertex with SEG_SMALL < entries <= SEG_MID: a
// bitonic sort over an LDS buffer of the wavefront's own, so its rounds need
// no workgroup barrier (a wavefront's LDS operations stay in order).
constexpr int SEG_MID = 1024;

// Bitonic compare-exchange of stage (k, J) on a lane's E consecutive
// elements (global index base + i), for partners inside the lane (J < E).
template <int E, int J>
__device__ __forceinline__ void bitonic_in_lane(uint64_t (&r)[E], int base, int k) {
    if constexpr (J < E) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            if ((i & J) == 0) {
                const bool up = ((base + i) & k) == 0;
                const uint64_t va = r[i], vb = r[i + J];
                const bool sw = (va > vb) == up;
                r[i] = sw ? vb : va;
                r[i + J] = sw ? va : vb;
            }
        }
    }
}

// One bucket of E * 64 slots (its d entries, padded with all-ones words),
// sorted by one wavefront: each lane keeps E consecutive elements in
// registers, the stages whose partners lie E or more apart go through LDS
// (one store and one load per merge size k), the others stay in registers.
// Slot i sits at LDS word i + i / E, so the lanes' runs of E start in
// different banks.
template <int E>
__device__ __forceinline__ void orient_mid_row(uint64_t *sk, int d, int64_t b, int32_t rx,
                                               int64_t ob, const uint64_t *__restrict__ tbuf,
                                               int32_t *__restrict__ ocol,
                                               uint32_t *__restrict__ o2e,
                                               int32_t *__restrict__ orow) {
    constexpr int P = E * TC_WAVE;
    const int lane = __lane_id();
    const int base = E * lane;
    auto px = [](int i) { return i + i / E; };
    for (int j = lane; j < P; j += TC_WAVE) sk[px(j)] = j < d ? tbuf[b + j] : ~0ull;
    __builtin_amdgcn_wave_barrier();
    uint64_t r[E];
#pragma unroll
    for (int i = 0; i < E; ++i) r[i] = sk[px(base) + i];
    for (int k = 2; k <= P; k <<= 1) {
        if (k > E) {
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int i = 0; i < E; ++i) sk[px(base) + i] = r[i];
            __builtin_amdgcn_wave_barrier();
            for (int j = k >> 1; j >= E; j >>= 1) {
                for (int t = lane; t < (P >> 1); t += TC_WAVE) {
                    const int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                    const uint64_t va = sk[px(a)], vb = sk[px(a + j)];
                    const bool up = (a & k) == 0;
                    if ((va > vb) == up) {
                        sk[px(a)] = vb;
                        sk[px(a + j)] = va;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int i = 0; i < E; ++i) r[i] = sk[px(base) + i];
        }
        // partners inside the lane: J from min(k / 2, E / 2) down to 1
        const int jtop = (k >> 1) < E ? (k >> 1) : (E >> 1);
        if (jtop >= 8) bitonic_in_lane<E, 8>(r, base, k);
        if (jtop >= 4) bitonic_in_lane<E, 4>(r, base, k);
        if (jtop >= 2) bitonic_in_lane<E, 2>(r, base, k);
        bitonic_in_lane<E, 1>(r, base, k);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < E; ++i) sk[px(base) + i] = r[i];
    __builtin_amdgcn_wave_barrier();
    for (int t = lane; t < d; t += TC_WAVE) {
        const uint64_t w = sk[px(t)];
        ocol[ob + t] = (int32_t)(w >> 32);
        o2e[ob + t] = (uint32_t)w;
        orow[ob + t] = rx;
    }
    __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(256) void k_orient_mid(
    const int32_t *__restrict__ list, int64_t nlist, const int64_t *__restrict__ row_ptr,
    const uint32_t *__restrict__ cursor, const int32_t *__restrict__ rank,
    const int64_t *__restrict__ orp, const uint64_t *__restrict__ tbuf,
    int32_t *__restrict__ ocol, uint32_t *__restrict__ o2e, int32_t *__restrict__ orow) {
    static_assert(SEG_SMALL == 256 && SEG_MID == 1024, "rows of 257..1024 entries: 512 or 1024 slots");
    __shared__ uint64_t sk_all[4][SEG_MID + SEG_MID / 8];
    const int wv = threadIdx.x / TC_WAVE;
    uint64_t *sk = sk_all[wv];
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wv; i < nlist; i += waves) {
        const int32_t x = list[i];
        const int32_t rx = rank[x];
        const int64_t ob = orp[rx];
        const int d = (int)cursor[x];
        const int64_t b = row_ptr[x];
        if (d <= SEG_MID / 2)
            orient_mid_row<SEG_MID / 2 / TC_WAVE>(sk, d, b, rx, ob, tbuf, ocol, o2e, orow);
        else
            orient_mid_row<SEG_MID / TC_WAVE>(sk, d, b, rx, ob, tbuf, ocol, o2e, orow);
    }
}

__global__ void k_size_flags(int32_t n, const uint32_t *__restrict__ cursor, uint32_t lo,
                             uint32_t hi, uint32_t *__restrict__ f) {
    GRID_STRIDE(x, n) f[x] = (cursor[x] > lo && cursor[x] <= hi) ? 1u : 0u;
}

__global__ void k_compact_flags(int32_t n, const uint32_t *__restrict__ f,
                                const uint32_t *__restrict__ pos, int32_t *__restrict__ out) {
    GRID_STRIDE(x, n) if (f[x]) out[pos[x]] = (int32_t)x;
}

}  // namespace

static tc_status orient_sorted(tc_graph *g, hipStream_t s);

// Lists the vertices whose flag is set (flags in f, n entries); the count
// goes to the device word *count (read back by the caller with others).
static tc_status compact_vertices(int32_t n, uint32_t *f, int32_t *out, uint32_t *count,
                                  hipStream_t s) {
    tc_scratch tmp(s);
    uint32_t *pos = nullptr;
    TC_TRY(tmp.get(&pos, n));
    TC_TRY(tc_scan_u32(f, pos, n, count, s));
    k_compact_flags<<<grid_for(n), BK, 0, s>>>(n, f, pos, out);
    TC_LAUNCHED();
    return TC_OK;
}

void tc_release_transposition(tc_graph *g, hipStream_t s) {
    if (!g->lt_key) return;
    tc_dev_free(g->lt_key, s);
    tc_dev_free(g->lt_val, s);
    g->lt_key = nullptr;
    g->lt_val = nullptr;
    g->bytes -= 2 * sizeof(uint32_t) * (size_t)g->m;
}

tc_status tc_orient(tc_graph *g, hipStream_t s) {
    const int32_t n = g->n;
    const int64_t m = g->m;
    int64_t nn = n > 0 ? n : 1;
    TC_TRY(tc_graph_alloc(g, &g->orp, nn + 1, s));
    // TC_OCOL_PAD trailing entries let the counting kernels load whole
    // 32-entry runs without bounds tests (entries past a run are masked)
    TC_TRY(tc_graph_alloc(g, &g->ocol, m + TC_OCOL_PAD, s));
    TC_TRY(tc_graph_alloc(g, &g->o2e, m, s));
    TC_TRY(tc_graph_alloc(g, &g->orow, m, s));
    g->max_dplus = 0;
    if (m == 0) {
        TC_HIP(hipMemsetAsync(g->orp, 0, sizeof(int64_t) * (nn + 1), s));
        tc_prof_mark(g, 3, s);
        return TC_OK;
    }
    tc_scratch tmp(s);
    int64_t *dplus = nullptr;
    uint32_t *info = nullptr, *flags = nullptr, *flags2 = nullptr, *cursor = nullptr;
    uint64_t *tbuf = nullptr;
    int32_t *list_mid = nullptr, *list_big = nullptr;
    TC_TRY(tmp.get(&cursor, nn));
    TC_TRY(tmp.get(&tbuf, 2 * m));
    TC_TRY(tmp.get(&dplus, nn));
    TC_TRY(tmp.get(&info, 4));  // max d+, mid-list count, big-list count
    TC_TRY(tmp.get(&flags, nn));
    TC_TRY(tmp.get(&flags2, nn));
    TC_TRY(tmp.get(&list_mid, nn));
    TC_TRY(tmp.get(&list_big, nn));
    TC_HIP(hipMemsetAsync(info, 0, 16, s));
    TC_HIP(hipMemsetAsync(cursor, 0, sizeof(uint32_t) * nn, s));
    // pass A: buckets of the lower-ordered endpoints
    {
        uint32_t *rank_u = nullptr;
        TC_TRY(tmp.get(&rank_u, m));
        k_place_by_smaller<<<grid_for(m), BK, 0, s>>>(m, g->eu, g->ev, g->rank, g->row_ptr, cursor,
                                                      tbuf, rank_u);
        TC_LAUNCHED();
        k_place_by_larger<<<grid_for(m), BK, 0, s>>>(m, g->lt_key, g->lt_val, g->rank, rank_u,
                                                     g->row_ptr, cursor, tbuf);
        TC_LAUNCHED();
    }
    k_dplus_by_rank<<<grid_for(n) < 4096 ? grid_for(n) : 4096, BK, 0, s>>>(n, cursor, g->rank, dplus,
                                                                          info);
    TC_LAUNCHED();
    // the buckets sorted by a wavefront and by a workgroup, listed now so that
    // one read-back brings their counts with the largest d+
    k_size_flags<<<grid_for(n), BK, 0, s>>>(n, cursor, SEG_SMALL, SEG_MID, flags);
    TC_LAUNCHED();
    TC_TRY(compact_vertices(n, flags, list_mid, info + 1, s));
    k_size_flags<<<grid_for(n), BK, 0, s>>>(n, cursor, SEG_MID, 0xFFFFFFFFu, flags2);
    TC_LAUNCHED();
    TC_TRY(compact_vertices(n, flags2, list_big, info + 2, s));
    uint32_t h_info[4] = {0, 0, 0, 0};
    TC_HIP(hipMemcpyAsync(h_info, info, 16, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    const uint32_t h_max = h_info[0];
    const int64_t nmid = h_info[1], nblk = h_info[2];
    g->max_dplus = (int32_t)h_max;
    // TC_ORIENT_SEG_MAX (environment) lowers the LDS-sort limit, so that the
    // sort-based path can be exercised on small graphs
    uint32_t seg_max = SEG_MAX;
    if (const char *ev = getenv("TC_ORIENT_SEG_MAX")) {
        const long v = strtol(ev, nullptr, 10);
        if (v >= 0 && v < SEG_MAX) seg_max = (uint32_t)v;
    }
    if (h_max > seg_max) {
        TC_TRY(orient_sorted(g, s));
        tc_prof_mark(g, 3, s);
        return TC_OK;
    }
    TC_TRY(tc_scan_i64(dplus, g->orp, n, g->orp + n, s));
    // pass B: each bucket in rank order
    {
        const int64_t want = tc_div_up(n, 4 * TC_WAVE);
        const unsigned grid = (unsigned)(want < 2048 ? (want > 0 ? want : 1) : 2048);
        k_orient_small<<<grid, BK, 0, s>>>(n, g->row_ptr, cursor, g->rank, g->orp, tbuf, g->ocol,
                                           g->o2e, g->orow);
        TC_LAUNCHED();
    }
    if (nmid > 0) {
        const int64_t blocks = tc_div_up(nmid, 4);
        k_orient_mid<<<(unsigned)(blocks < 1048576 ? blocks : 1048576), BK, 0, s>>>(
            list_mid, nmid, g->row_ptr, cursor, g->rank, g->orp, tbuf, g->ocol, g->o2e, g->orow);
        TC_LAUNCHED();
    }
    if (nblk > 0) {
        k_orient_block<<<(unsigned)(nblk < 1048576 ? nblk : 1048576), BK, 0, s>>>(
            list_big, nblk, g->row_ptr, cursor, g->rank, g->orp, tbuf, g->ocol, g->o2e, g->orow);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 3, s);
    return TC_OK;
}

// ---------------------------------------------------------------------------
tc_status tc_build_from_pairs(tc_graph *g, const int32_t *d_src, const int32_t *d_dst, int64_t P,
                              const int64_t *d_vtx_off, const int64_t *d_pair_off,
                              int32_t num_graphs, hipStream_t s, const int64_t *simple_rp,
                              const int32_t *simple_col) {
    const int32_t n = g->n;
    const int bits = g->bits;
    const uint64_t sentinel = (bits >= 32) ? ~0ull : ((1ull << (2 * bits)) - 1);
    tc_scratch tmp(s);

    TC_TRY(tc_graph_alloc(g, &g->err, 4, s));
    TC_HIP(hipMemsetAsync(g->err, 0, 16, s));

    // runs of the edges by smaller end, filled while the canonical edges are
    // written
    int64_t nn = n > 0 ? n : 1;
    uint32_t *ue = nullptr;
    TC_TRY(tc_graph_alloc(g, &g->run_us, nn, s));
    uint32_t *us = g->run_us;
    TC_TRY(tmp.get(&ue, nn));
    TC_HIP(hipMemsetAsync(us, 0, sizeof(uint32_t) * nn, s));
    TC_HIP(hipMemsetAsync(ue, 0, sizeof(uint32_t) * nn, s));

    // -- 1. canonical edges ---------------------------------------------------
    int64_t m = 0;
    if (simple_rp && n > 0) {
        // a simple sorted CSR: the upper triangle, no sort and no dedup
        uint32_t *cnt = nullptr, *off = nullptr, *d_m = nullptr;
        TC_TRY(tmp.get(&cnt, nn));
        TC_TRY(tmp.get(&off, nn));
        TC_TRY(tmp.get(&d_m, 1));
        k_csr_upper_count<<<grid_for(n), BK, 0, s>>>(simple_rp, simple_col, n, cnt, g->err);
        TC_LAUNCHED();
        TC_TRY(tc_scan_u32(cnt, off, n, d_m, s));
        uint32_t h_m = 0, h_err = 0;
        TC_HIP(hipMemcpyAsync(&h_err, g->err, 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipMemcpyAsync(&h_m, d_m, 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        if (h_err) return TC_ERR_INVALID_ARG;
        m = h_m;
        TC_TRY(tc_graph_alloc(g, &g->eu, m, s));
        TC_TRY(tc_graph_alloc(g, &g->ev, m, s));
        if (m > 0) {
            k_csr_upper_emit<<<grid_for(n), BK, 0, s>>>(simple_rp, simple_col, n, cnt, off, g->eu,
                                                        g->ev, us, ue);
            TC_LAUNCHED();
        }
    } else if (simple_rp) {
        TC_TRY(tc_graph_alloc(g, &g->eu, 0, s));
        TC_TRY(tc_graph_alloc(g, &g->ev, 0, s));
    } else if (P > 0) {
        uint64_t *keys = nullptr, *keys2 = nullptr;
        TC_TRY(tmp.get(&keys, P));
        TC_TRY(tmp.get(&keys2, P));
        // an id out of range makes a sentinel key (dropped like a self
        // loop) and sets err, which is read back with the edge count
        k_make_keys<<<grid_for(P), BK, 0, s>>>(d_src, d_dst, P, n, bits, d_pair_off, d_vtx_off,
                                               num_graphs, keys, g->err);
        TC_LAUNCHED();
        TC_TRY(tc_sort_u64(&keys, &keys2, P, 2 * bits, s));
        const int64_t tiles = tc_div_up(P, UQ_TILE);
        uint32_t *tcnt = nullptr, *d_m = nullptr;
        TC_TRY(tmp.get(&tcnt, tiles));
        TC_TRY(tmp.get(&d_m, 1));
        k_unique_count<<<(unsigned)tiles, UQ_BLOCK, 0, s>>>(keys, P, sentinel, tcnt);
        TC_LAUNCHED();
        TC_TRY(tc_scan_u32(tcnt, tcnt, tiles, d_m, s));
        uint32_t h_m = 0, h_err = 0;
        TC_HIP(hipMemcpyAsync(&h_err, g->err, 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipMemcpyAsync(&h_m, d_m, 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        if (h_err) return TC_ERR_VERTEX_RANGE;
        m = h_m;
        TC_TRY(tc_graph_alloc(g, &g->eu, m, s));
        TC_TRY(tc_graph_alloc(g, &g->ev, m, s));
        if (m > 0) {
            k_unique_emit<<<(unsigned)tiles, UQ_BLOCK, 0, s>>>(keys, P, sentinel, bits, tcnt, g->eu,
                                                               g->ev, us, ue);
            TC_LAUNCHED();
            k_last_run<<<1, 64, 0, s>>>(m, g->eu, ue);
            TC_LAUNCHED();
        }
    } else {
        TC_TRY(tc_graph_alloc(g, &g->eu, 0, s));
        TC_TRY(tc_graph_alloc(g, &g->ev, 0, s));
    }
    g->m = m;

    // -- 2. degrees and the symmetric row offsets ------------------------------
    // The adjacency itself (col / sym2e) is filled only when a consumer
    // needs it (tc_ensure_symmetric).
    TC_TRY(tc_graph_alloc(g, &g->row_ptr, (int64_t)n + 1, s));
    // the canonical edges ordered by their larger end (kept for the
    // orientation), whose runs count the edges by larger end
    uint32_t *deg32 = nullptr, *ls = nullptr, *le = nullptr;
    int64_t *deg64 = nullptr;
    TC_TRY(tmp.get(&deg32, nn));
    TC_TRY(tmp.get(&deg64, nn));
    TC_TRY(tmp.get(&ls, nn));
    TC_TRY(tmp.get(&le, nn));
    TC_HIP(hipMemsetAsync(ls, 0, sizeof(uint32_t) * nn, s));
    TC_HIP(hipMemsetAsync(le, 0, sizeof(uint32_t) * nn, s));
    if (m > 0) {
        uint32_t *lk2 = nullptr, *lv2 = nullptr;
        TC_TRY(tc_graph_alloc(g, &g->lt_key, m, s));
        TC_TRY(tc_graph_alloc(g, &g->lt_val, m, s));
        TC_TRY(tmp.get(&lk2, m));
        TC_TRY(tmp.get(&lv2, m));
        uint32_t *lk = g->lt_key, *lv = g->lt_val;
        TC_TRY(tc_sort_u32_index((const uint32_t *)g->ev, &lk, &lv, &lk2, &lv2, m, bits, s));
        if (lk != g->lt_key) {  // the result is in the scratch pair: swap ownership
            tmp.exchange(lk, g->lt_key);
            tmp.exchange(lv, g->lt_val);
            g->lt_key = lk;
            g->lt_val = lv;
        }
        k_runs<<<grid_for(m), BK, 0, s>>>(GetU32{g->lt_key}, m, ls, le);
        TC_LAUNCHED();
    }
    if (n > 0) {
        k_degree<<<grid_for(n), BK, 0, s>>>(n, us, ue, ls, le, deg64, deg32);
        TC_LAUNCHED();
        TC_TRY(tc_scan_i64(deg64, g->row_ptr, n, g->row_ptr + n, s));
    } else {
        TC_HIP(hipMemsetAsync(g->row_ptr, 0, sizeof(int64_t), s));
    }

    tc_prof_mark(g, 1, s);

    // -- 3. degree ordering -------------------------------------------------------
    TC_TRY(tc_graph_alloc(g, &g->rank, nn, s));
    TC_TRY(tc_graph_alloc(g, &g->perm, nn, s));
    if (n > 0) {
        uint32_t *pv = nullptr, *pv2 = nullptr, *dk2 = nullptr;
        TC_TRY(tmp.get(&pv, nn));
        TC_TRY(tmp.get(&pv2, nn));
        TC_TRY(tmp.get(&dk2, nn));
        k_iota<<<grid_for(n), BK, 0, s>>>(pv, n);
        TC_LAUNCHED();
        // degrees are below n, so `bits` bits hold them
        TC_TRY(tc_sort_u32_u32(&deg32, &pv, &dk2, &pv2, n, bits, s));
        k_invert<<<grid_for(n), BK, 0, s>>>(pv, n, g->perm, g->rank);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 2, s);
    return TC_OK;
}

// Orientation by one global sort of the packed (π(low), π(high)) keys; used
// when some row has more than SEG_MAX higher-ordered neighbours.
static tc_status orient_sorted(tc_graph *g, hipStream_t s) {
    const int32_t n = g->n;
    const int64_t m = g->m;
    const int bits = g->bits;
    tc_scratch tmp(s);
    int64_t nn = n > 0 ? n : 1;
    uint64_t *okey = nullptr, *okey2 = nullptr;
    uint32_t *oval2 = nullptr;
    TC_TRY(tmp.get(&okey, m));
    TC_TRY(tmp.get(&okey2, m));
    TC_TRY(tmp.get(&oval2, m));
    uint32_t *oval = g->o2e;
    uint32_t *oval_swap = oval2;
    k_orient_keys<<<grid_for(m), BK, 0, s>>>(m, g->eu, g->ev, g->rank, bits, okey, oval);
    TC_LAUNCHED();
    TC_TRY(tc_sort_u64_u32(&okey, &oval, &okey2, &oval_swap, m, 2 * bits, s));
    if (oval != g->o2e) {
        TC_HIP(hipMemcpyAsync(g->o2e, oval, sizeof(uint32_t) * m, hipMemcpyDeviceToDevice, s));
    }
    k_orient_split<<<grid_for(m), BK, 0, s>>>(m, okey, bits, g->ocol, g->orow);
    TC_LAUNCHED();
    uint32_t *rs = nullptr, *re = nullptr, *d_max = nullptr;
    int64_t *dplus = nullptr;
    TC_TRY(tmp.get(&rs, nn));
    TC_TRY(tmp.get(&re, nn));
    TC_TRY(tmp.get(&dplus, nn));
    TC_TRY(tmp.get(&d_max, 1));
    TC_HIP(hipMemsetAsync(rs, 0, sizeof(uint32_t) * nn, s));
    TC_HIP(hipMemsetAsync(re, 0, sizeof(uint32_t) * nn, s));
    TC_HIP(hipMemsetAsync(d_max, 0, sizeof(uint32_t), s));
    k_runs<<<grid_for(m), BK, 0, s>>>(GetHigh{okey, bits}, m, rs, re);
    TC_LAUNCHED();
    k_run_len64<<<grid_for(n), BK, 0, s>>>(n, rs, re, dplus, d_max);
    TC_LAUNCHED();
    TC_TRY(tc_scan_i64(dplus, g->orp, n, g->orp + n, s));
    return TC_OK;
}

// ---------------------------------------------------------------------------
tc_status tc_ensure_symmetric(tc_graph *g, hipStream_t s) {
    if (g->col) return TC_OK;
    const int32_t n = g->n;
    const int64_t m = g->m;
    const int64_t nn = n > 0 ? n : 1;
    TC_TRY(tc_graph_alloc(g, &g->col, 2 * m, s));
    TC_TRY(tc_graph_alloc(g, &g->sym2e, 2 * m, s));
    if (m == 0) return TC_OK;
    // the transposition: canonical edges sorted by their larger end (kept
    // from the build unless the middle-pivot count released it), and the
    // run of every vertex in that order
    tc_scratch tmp(s);
    uint32_t *tkey = g->lt_key, *tval = g->lt_val;
    uint32_t *ls = nullptr, *le = nullptr;
    if (!tkey) {
        uint32_t *tkey2 = nullptr, *tval2 = nullptr;
        TC_TRY(tmp.get(&tkey, m));
        TC_TRY(tmp.get(&tval, m));
        TC_TRY(tmp.get(&tkey2, m));
        TC_TRY(tmp.get(&tval2, m));
        TC_TRY(tc_sort_u32_index((const uint32_t *)g->ev, &tkey, &tval, &tkey2, &tval2, m, g->bits,
                                 s));
    }
    TC_TRY(tmp.get(&ls, nn));
    TC_TRY(tmp.get(&le, nn));
    TC_HIP(hipMemsetAsync(ls, 0, sizeof(uint32_t) * nn, s));
    TC_HIP(hipMemsetAsync(le, 0, sizeof(uint32_t) * nn, s));
    k_runs<<<grid_for(m), BK, 0, s>>>(GetU32{tkey}, m, ls, le);
    TC_LAUNCHED();
    k_fill_lower<<<grid_for(m), BK, 0, s>>>(m, tkey, tval, ls, g->row_ptr, g->eu, g->col, g->sym2e);
    TC_LAUNCHED();
    k_fill_upper<<<grid_for(m), BK, 0, s>>>(m, g->eu, g->ev, g->run_us, ls, le, g->row_ptr, g->col,
                                            g->sym2e);
    TC_LAUNCHED();
    tc_release_transposition(g, s);
    return TC_OK;
}
