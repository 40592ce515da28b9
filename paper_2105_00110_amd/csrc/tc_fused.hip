// Batched small graphs in one persistent launch.
//
// Every workgroup of k_fused_graphs pulls graph indices from a device
// counter and runs the whole path on one graph with workgroup-local steps:
//
//   keys      each pair as lo * n + hi (lo < hi, ids local to the graph),
//             self-loops as the sentinel n * n;
//   sort      LSD radix sort of the keys, 8-bit digits, in the graph's
//             workspace (one digit histogram read for all passes; ranks by
//             8 ballots per key inside a wavefront, then wavefront offsets);
//   unique    distinct keys below the sentinel: the canonical edges
//             (u < v, lexicographic), m of them;
//   degree    d(v) by atomics on the canonical edges;
//   rank      sort of d(v) * n + v: the order (degree, id) of Sec.
//             "Notation", ties by smaller id; rank[v] and perm[r];
//   orient    each edge as rank(low) * n + rank(high) with its canonical
//             index as value, sorted: rows of N_H in rank space, ascending,
//             and their offsets;
//   count     one thread per oriented slot (r -> c) merges the tail of
//             N_H(r) after c with N_H(c), both sorted (the appendix's
//             Procedure 2 with counts in place of marks): every common w is
//             the triangle (r, c, w), found once from its lowest rank, and
//             adds 1 to the support of (r, w) and (c, w); the slot's own
//             support gains the number found;
//   tri       tri(v) = 1/2 Σ_{u ∈ N(v)} sup(v, u) and triG = 1/3 Σ_e sup(e)
//             (the quoted theorem of Sec. "Formulation");
//   aggregate num(v) = tri(v) + Σ_{u ∈ N(v)} (sup(v,u) > 0 ? 1 : 3) tri(u),
//             Definition 1's numerator times 3 with N△(v) read as the
//             neighbours sharing a triangle with v (Algorithm 2 in integer
//             form);
//   quotient  tc(v) = double(num) / double(3 triG), one IEEE division.
//
// Graphs of at most FUSED_MAX_N vertices qualify (keys stay below 2^32).
// Nothing is read back to the host and no memory is allocated, so the two
// launches can be captured in a graph and replayed.  tc_batch_fused takes
// its workspace from the caller; tc_batch_fused_noalloc uses a fixed device
// array of this file instead.
#include <mutex>

#include "tc_internal.h"

namespace {

constexpr int64_t FUSED_MAX_N = 65535;
constexpr int FUSED_MW = 8;  // entries of each list per round of the count's merge
constexpr int FUSED_RB = 8;
constexpr int FUSED_RADIX = 1 << FUSED_RB;
constexpr int FUSED_ITEMS = 8;          // keys per thread in a scatter tile
constexpr int64_t FUSED_HEADER = 256;   // queue head and flags
// Workspace: a header, then 5 uint32 arrays per pair (the pair region,
// rounded up to 256 bytes), then per graph and vertex two uint64 and five
// uint32 arrays (40 bytes per vertex, 8 per graph for the extra row offset
// and alignment).
constexpr int64_t FUSED_PAIR_BYTES = 20;
constexpr int64_t FUSED_VTX_BYTES = 40;
constexpr int64_t FUSED_GRAPH_BYTES = 8;

__host__ __device__ inline int64_t pair_region(int64_t P) {
    return (FUSED_PAIR_BYTES * P + 255) / 256 * 256;
}

struct FusedArgs {
    const int32_t *src, *dst;
    const int64_t *pair_off, *vtx_off;
    const int32_t *order;
    int32_t G;
    int64_t P, N;
    int32_t *eu, *ev;
    uint64_t *sup;
    int64_t *num_edges;
    uint64_t *tri, *num;
    double *tc;
    uint64_t *triG;
    int32_t *status;
    unsigned char *ws;  // workspace (header first)
};

template <int BLOCK>
struct FusedLds {
    static constexpr int WAVES = BLOCK / TC_WAVE;
    uint32_t hist[4][FUSED_RADIX];  // digit counts of up to 4 passes, then running bases
    uint32_t wcnt[WAVES][FUSED_RADIX];
    uint32_t tot[FUSED_RADIX];
    uint32_t wsum[WAVES];
    uint64_t wsum64[WAVES];
    uint32_t bcast;
};

// Atomic add ordered for the workgroup.  Every array these touch belongs to
// one graph and is read back only by the workgroup that owns it, after a
// barrier; device scope would make each fence write back and invalidate the
// L2, and the barriers' workgroup-scope release and acquire suffice.
template <typename T>
__device__ __forceinline__ void wg_add(T *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Sum of x over each run of equal keys among a wavefront's valid lanes, the
// keys non-decreasing in lane order: the run's last lane gets the run's sum
// and tail = true.
__device__ __forceinline__ uint64_t run_sum(uint32_t key, uint64_t x, bool valid, bool &tail) {
    const int lane = __lane_id();
    const uint32_t prev = __shfl_up(key, 1, TC_WAVE);
    const bool head = valid && (lane == 0 || prev != key);
    const uint64_t heads = __ballot(head);
    const uint64_t upto = heads & ((2ull << lane) - 1ull);  // heads at or below this lane
    const int start = upto ? 63 - __clzll(upto) : 0;
#pragma unroll
    for (int off = 1; off < TC_WAVE; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, TC_WAVE);
        if (lane - off >= start) x += y;
    }
    const uint32_t next = __shfl_down(key, 1, TC_WAVE);
    const uint64_t live = __ballot(valid);
    const bool next_live = lane < TC_WAVE - 1 && ((live >> (lane + 1)) & 1ull);
    tail = valid && (!next_live || next != key);
    return x;
}

__device__ __forceinline__ int fused_bits(uint32_t max_value) {
    return max_value == 0 ? 0 : 32 - __clz(max_value);
}

// Sum over the workgroup (every thread returns it).
template <int BLOCK>
__device__ uint64_t block_sum64(uint64_t x, FusedLds<BLOCK> &sh) {
    x = tc_wave_sum(x);
    if (__lane_id() == 0) sh.wsum64[threadIdx.x / TC_WAVE] = x;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int q = 0; q < FusedLds<BLOCK>::WAVES; ++q) t += sh.wsum64[q];
    __syncthreads();
    return t;
}

template <int BLOCK>
__device__ uint32_t block_max32(uint32_t x, FusedLds<BLOCK> &sh) {
    x = tc_wave_max(x);
    if (__lane_id() == 0) sh.wsum[threadIdx.x / TC_WAVE] = x;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int q = 0; q < FusedLds<BLOCK>::WAVES; ++q) t = sh.wsum[q] > t ? sh.wsum[q] : t;
    __syncthreads();
    return t;
}

// Exclusive prefix of v[0..256) in place; threads below 256 hold one digit.
template <int BLOCK>
__device__ void scan256(uint32_t *v, FusedLds<BLOCK> &sh) {
    static_assert(BLOCK >= FUSED_RADIX, "one digit per thread");
    const int tid = threadIdx.x;
    const uint32_t x = tid < FUSED_RADIX ? v[tid] : 0u;
    const uint32_t incl = tc_wave_incl_scan(x);
    if (tid < FUSED_RADIX && __lane_id() == TC_WAVE - 1) sh.wsum[tid / TC_WAVE] = incl;
    __syncthreads();
    if (tid < FUSED_RADIX) {
        uint32_t before = 0;
        for (int q = 0; q < tid / TC_WAVE; ++q) before += sh.wsum[q];
        v[tid] = before + incl - x;
    }
    __syncthreads();
}

// Stable LSD radix sort of n keys (and values) held in device memory, by
// the whole workgroup.  The sorted data ends in *k / *v; the other buffers
// are ping-pong space.  One read of the keys counts the digits of every
// pass (the multiset of keys is the same before each pass).
template <int BLOCK, bool VAL>
__device__ void block_sort(uint32_t *&k, uint32_t *&kt, uint32_t *&v, uint32_t *&vt, uint32_t n,
                           int bits, FusedLds<BLOCK> &sh) {
    constexpr int WAVES = FusedLds<BLOCK>::WAVES;
    constexpr int TILE = BLOCK * FUSED_ITEMS;
    const int passes = (bits + FUSED_RB - 1) / FUSED_RB;
    if (n <= 1 || passes == 0) return;
    const int tid = threadIdx.x, w = tid / TC_WAVE, lane = __lane_id();
    const uint64_t lt = tc_lanemask_lt();
    for (int i = tid; i < 4 * FUSED_RADIX; i += BLOCK) (&sh.hist[0][0])[i] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += BLOCK) {
        const uint32_t key = k[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&sh.hist[p][(key >> (FUSED_RB * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p) scan256(sh.hist[p], sh);
    for (int p = 0; p < passes; ++p) {
        const int shift = FUSED_RB * p;
        uint32_t *base = sh.hist[p];
        for (uint32_t t0 = 0; t0 < n; t0 += TILE) {
            for (int i = tid; i < WAVES * FUSED_RADIX; i += BLOCK) (&sh.wcnt[0][0])[i] = 0;
            __syncthreads();
            uint32_t key[FUSED_ITEMS], val[FUSED_ITEMS], rnk[FUSED_ITEMS];
            const uint32_t wb = t0 + (uint32_t)w * (TC_WAVE * FUSED_ITEMS);
#pragma unroll
            for (int it = 0; it < FUSED_ITEMS; ++it) {
                const uint32_t i = wb + it * TC_WAVE + lane;
                const bool valid = i < n;
                key[it] = valid ? k[i] : 0u;
                if constexpr (VAL) val[it] = valid ? v[i] : 0u;
            }
            // rank among equal digits: earlier items of the wavefront, then
            // lower lanes of the same item (memory order)
#pragma unroll
            for (int it = 0; it < FUSED_ITEMS; ++it) {
                const uint32_t i = wb + it * TC_WAVE + lane;
                const bool valid = i < n;
                const uint32_t d = (key[it] >> shift) & 255u;
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int b = 0; b < FUSED_RB; ++b) {
                    const bool bit = (d >> b) & 1u;
                    const uint64_t bal = __ballot(bit);
                    peers &= bit ? bal : ~bal;
                }
                uint32_t prior = 0;
                if (valid) prior = sh.wcnt[w][d];
                rnk[it] = prior + (uint32_t)__popcll(peers & lt);
                // every lane has read the count before the highest peer
                // replaces it (a wavefront's LDS operations run in order)
                __builtin_amdgcn_wave_barrier();
                if (valid && (peers >> lane) == 1ull) sh.wcnt[w][d] = prior + (uint32_t)__popcll(peers);
            }
            __syncthreads();
            if (tid < FUSED_RADIX) {
                uint32_t run = 0;
                for (int q = 0; q < WAVES; ++q) {
                    const uint32_t c = sh.wcnt[q][tid];
                    sh.wcnt[q][tid] = run;
                    run += c;
                }
                sh.tot[tid] = run;
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < FUSED_ITEMS; ++it) {
                const uint32_t i = wb + it * TC_WAVE + lane;
                if (i < n) {
                    const uint32_t d = (key[it] >> shift) & 255u;
                    const uint32_t pos = base[d] + sh.wcnt[w][d] + rnk[it];
                    kt[pos] = key[it];
                    if constexpr (VAL) vt[pos] = val[it];
                }
            }
            __syncthreads();
            if (tid < FUSED_RADIX) base[tid] += sh.tot[tid];
            __syncthreads();
        }
        uint32_t *t = k;
        k = kt;
        kt = t;
        if constexpr (VAL) {
            t = v;
            v = vt;
            vt = t;
        }
    }
}

// The distinct keys of the sorted a[0..n) that lie below `limit`, in order,
// written to out; returns their count.
template <int BLOCK>
__device__ uint32_t block_unique(const uint32_t *a, uint32_t n, uint32_t limit, uint32_t *out,
                                 FusedLds<BLOCK> &sh) {
    constexpr int WAVES = FusedLds<BLOCK>::WAVES;
    const int w = threadIdx.x / TC_WAVE;
    uint32_t count = 0;
    for (uint32_t t0 = 0; t0 < n; t0 += BLOCK) {
        const uint32_t i = t0 + threadIdx.x;
        bool keep = false;
        uint32_t key = 0;
        if (i < n) {
            key = a[i];
            keep = key < limit && (i == 0 || a[i - 1] != key);
        }
        const uint64_t bal = __ballot(keep);
        if (__lane_id() == 0) sh.wsum[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < WAVES; ++q) {
            const uint32_t c = sh.wsum[q];
            before += q < w ? c : 0u;
            all += c;
        }
        if (keep) out[count + before + (uint32_t)__popcll(bal & tc_lanemask_lt())] = key;
        count += all;
        __syncthreads();
    }
    return count;
}

// Writes the outputs of a graph that is not computed (status < 0): no
// edges, zero counts and quotients for its vertices.
template <int BLOCK>
__device__ void fused_fail(const FusedArgs &a, int32_t g, int64_t va, int64_t n, int32_t st) {
    for (int64_t v = threadIdx.x; v < n; v += BLOCK) {
        if (a.tri) a.tri[va + v] = 0;
        if (a.num) a.num[va + v] = 0;
        if (a.tc) a.tc[va + v] = 0.0;
    }
    if (threadIdx.x == 0) {
        a.num_edges[g] = 0;
        if (a.triG) a.triG[g] = 0;
        a.status[g] = st;
    }
}

template <int BLOCK>
__device__ void fused_one_graph(const FusedArgs &a, int32_t g, FusedLds<BLOCK> &sh) {
    const int tid = threadIdx.x;
    const int64_t pa = a.pair_off[g], pb = a.pair_off[g + 1];
    const int64_t va = a.vtx_off[g], vb = a.vtx_off[g + 1];
    // offsets outside the arrays, or decreasing: nothing of this graph is
    // touched but its status
    if (pa < 0 || pb < pa || pb > a.P || va < 0 || vb < va || vb > a.N) {
        if (tid == 0) {
            a.num_edges[g] = 0;
            a.status[g] = TC_ERR_INVALID_ARG;
        }
        return;
    }
    if (vb - va > FUSED_MAX_N || pb - pa > 0x7FFFFFFFll) {
        fused_fail<BLOCK>(a, g, va, vb - va, TC_ERR_UNSUPPORTED);
        return;
    }
    const uint32_t n = (uint32_t)(vb - va), P = (uint32_t)(pb - pa);
    const uint32_t sentinel = n * n;  // n <= 65535: below 2^32

    // workspace of this graph: 5 pair arrays, then the vertex arrays
    uint32_t *A = reinterpret_cast<uint32_t *>(a.ws + FUSED_HEADER) + 5 * pa;
    uint32_t *B = A + P, *C = B + P, *D = C + P, *E = D + P;
    unsigned char *vbase = a.ws + FUSED_HEADER + pair_region(a.P) + FUSED_VTX_BYTES * va +
                           FUSED_GRAPH_BYTES * (int64_t)g;
    uint64_t *triR = reinterpret_cast<uint64_t *>(vbase);
    uint64_t *numR = triR + n;
    uint32_t *deg = reinterpret_cast<uint32_t *>(numR + n);
    uint32_t *rank = deg + n, *perm = rank + n, *vtmp = perm + n, *orp = vtmp + n;  // orp[n+1]

    // keys, with the id range check
    bool bad = false;
    for (uint32_t i = tid; i < P; i += BLOCK) {
        const int32_t x = a.src[pa + i], y = a.dst[pa + i];
        uint32_t key = sentinel;
        if ((uint32_t)x >= n || (uint32_t)y >= n) {
            bad = true;
        } else if (x != y) {
            const uint32_t lo = (uint32_t)(x < y ? x : y), hi = (uint32_t)(x < y ? y : x);
            key = lo * n + hi;
        }
        A[i] = key;
    }
    if (__syncthreads_or(bad)) {
        fused_fail<BLOCK>(a, g, va, n, TC_ERR_VERTEX_RANGE);
        __syncthreads();
        return;
    }
    // canonical edges
    uint32_t *k = A, *kt = B, *nv = nullptr, *nvt = nullptr;
    block_sort<BLOCK, false>(k, kt, nv, nvt, P, fused_bits(sentinel), sh);
    const uint32_t m = block_unique<BLOCK>(k, P, sentinel, C, sh);
    if (a.eu || a.ev) {
        for (uint32_t e = tid; e < m; e += BLOCK) {
            const uint32_t key = C[e], lo = key / n, hi = key - lo * n;
            if (a.eu) a.eu[pa + e] = (int32_t)lo;
            if (a.ev) a.ev[pa + e] = (int32_t)hi;
        }
    }

    // degrees
    for (uint32_t v = tid; v < n; v += BLOCK) deg[v] = 0;
    __syncthreads();
    // canonical edges come sorted by their smaller end: a wavefront's lanes
    // with the same smaller end form a run, whose first lane adds its length
    for (uint32_t e0 = 0; e0 < m; e0 += BLOCK) {
        const uint32_t e = e0 + tid;
        const bool valid = e < m;
        uint32_t lo = 0, hi = 0;
        if (valid) {
            const uint32_t key = C[e];
            lo = key / n;
            hi = key - lo * n;
        }
        const int lane = __lane_id();
        const uint32_t prev = __shfl_up(lo, 1, TC_WAVE);
        const bool head = valid && (lane == 0 || prev != lo);
        const uint64_t heads = __ballot(head);
        const uint64_t live = __ballot(valid);
        if (head) {
            const uint64_t after = lane == TC_WAVE - 1 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
            const uint32_t end = after ? (uint32_t)(__ffsll((unsigned long long)after) - 1)
                                       : (uint32_t)(64 - __clzll(live));
            wg_add(&deg[lo], end - (uint32_t)lane);
        }
        if (valid) wg_add(&deg[hi], 1u);
    }
    __syncthreads();
    // order (degree, id): keys d * n + v, sorted; the key gives v back
    uint32_t dmax = 0;
    for (uint32_t v = tid; v < n; v += BLOCK) {
        const uint32_t d = deg[v];
        dmax = d > dmax ? d : dmax;
        deg[v] = d * n + v;
    }
    dmax = block_max32<BLOCK>(dmax, sh);
    k = deg;
    kt = vtmp;
    block_sort<BLOCK, false>(k, kt, nv, nvt, n, n ? fused_bits(dmax * n + (n - 1)) : 0, sh);
    for (uint32_t r = tid; r < n; r += BLOCK) {
        const uint32_t key = k[r], v = key - (key / n) * n;
        perm[r] = v;
        rank[v] = r;
    }
    __syncthreads();

    // orientation: keys rank(low) * n + rank(high), values canonical edge
    for (uint32_t e = tid; e < m; e += BLOCK) {
        const uint32_t key = C[e], lo = key / n, hi = key - lo * n;
        const uint32_t ra = rank[lo], rb = rank[hi];
        A[e] = ra < rb ? ra * n + rb : rb * n + ra;
        D[e] = e;
    }
    for (uint32_t r = tid; r < n; r += BLOCK) {
        triR[r] = 0;
        numR[r] = 0;
    }
    __syncthreads();
    k = A;
    kt = B;
    uint32_t *o2e = D, *vt = E;
    block_sort<BLOCK, true>(k, kt, o2e, vt, m, n ? fused_bits(n * n - 1) : 0, sh);
    uint32_t *ocol = k, *orow = kt, *osup = vt;
    for (uint32_t s = tid; s < m; s += BLOCK) {
        const uint32_t key = ocol[s], r = key / n;
        orow[s] = r;
        ocol[s] = key - r * n;
        osup[s] = 0;
    }
    __syncthreads();
    // row offsets: every entry of orp[0..n] is written once
    for (uint32_t s = tid; s < m; s += BLOCK) {
        const uint32_t r = orow[s];
        const uint32_t from = s == 0 ? 0u : orow[s - 1] + 1u;
        for (uint32_t q = from; q <= r; ++q) orp[q] = s;
        if (s == m - 1)
            for (uint32_t q = r + 1; q <= n; ++q) orp[q] = m;
    }
    if (m == 0)
        for (uint32_t q = tid; q <= n; q += BLOCK) orp[q] = 0;
    __syncthreads();

    // count: the tail of N_H(r) after c against N_H(c), merged four entries
    // of each list at a time: the eight loads of a round are independent
    // (one memory latency per round instead of one per step), all sixteen
    // pairs are compared, and every entry up to the smaller of the two
    // windows' last entries is then settled (an entry above it can equal
    // nothing in the other window)
    for (uint32_t s = tid; s < m; s += BLOCK) {
        const uint32_t r = orow[s], c = ocol[s];
        uint32_t i = s + 1, j = orp[c];
        const uint32_t ie = orp[r + 1], je = orp[c + 1];
        uint32_t t = 0;
        while (i < ie && j < je) {
            uint32_t x[FUSED_MW], y[FUSED_MW];
#pragma unroll
            for (int e = 0; e < FUSED_MW; ++e) x[e] = i + e < ie ? ocol[i + e] : 0xFFFFFFFFu;
#pragma unroll
            for (int e = 0; e < FUSED_MW; ++e) y[e] = j + e < je ? ocol[j + e] : 0xFFFFFFFEu;
            const uint32_t lim = x[FUSED_MW - 1] < y[FUSED_MW - 1] ? x[FUSED_MW - 1] : y[FUSED_MW - 1];
            uint32_t na = 0, nb = 0;
#pragma unroll
            for (int e = 0; e < FUSED_MW; ++e) {
                na += x[e] <= lim ? 1u : 0u;
                nb += y[e] <= lim ? 1u : 0u;
            }
#pragma unroll
            for (int e = 0; e < FUSED_MW; ++e) {
                int f = -1;  // the other window's entry equal to x[e], if any
#pragma unroll
                for (int q = 0; q < FUSED_MW; ++q) f = x[e] == y[q] ? q : f;
                if (f >= 0) {
                    wg_add(&osup[i + e], 1u);
                    wg_add(&osup[j + f], 1u);
                    ++t;
                }
            }
            i += na;
            j += nb;
        }
        if (t) wg_add(&osup[s], t);
    }
    __syncthreads();

    // tri(v) = 1/2 Σ sup over v's edges; 3 triG = Σ_e sup(e)
    // (slots are sorted by row: a wavefront's slots of one row form a run)
    uint64_t local = 0;
    for (uint32_t s0 = 0; s0 < m; s0 += BLOCK) {
        const uint32_t s = s0 + tid;
        const bool valid = s < m;
        const uint32_t x = valid ? osup[s] : 0u, r = valid ? orow[s] : 0u;
        bool tail;
        const uint64_t rs = run_sum(r, (uint64_t)x, valid, tail);
        if (tail && rs) wg_add(&triR[r], rs);
        if (x) wg_add(&triR[ocol[s]], (uint64_t)x);
        local += x;
    }
    const uint64_t three_t = block_sum64<BLOCK>(local, sh);
    bool odd = (three_t % 3) != 0;
    for (uint32_t r = tid; r < n; r += BLOCK) {
        const uint64_t t2 = triR[r];
        odd |= (t2 & 1) != 0;
        triR[r] = t2 >> 1;
    }
    odd = __syncthreads_or(odd);
    const uint64_t tg = three_t / 3;

    // numerator: weight 1 for triangle neighbours (sup > 0), 3 for the others
    for (uint32_t s0 = 0; s0 < m; s0 += BLOCK) {
        const uint32_t s = s0 + tid;
        const bool valid = s < m;
        uint32_t r = 0, c = 0;
        uint64_t f = 0;
        if (valid) {
            r = orow[s];
            c = ocol[s];
            f = osup[s] ? 1 : 3;
        }
        bool tail;
        const uint64_t rs = run_sum(r, valid ? f * triR[c] : 0ull, valid, tail);
        if (tail && rs) wg_add(&numR[r], rs);
        if (valid) {
            const uint64_t y = f * triR[r];
            if (y) wg_add(&numR[c], y);
        }
    }
    __syncthreads();

    // outputs in the graph's own vertex ids and canonical edge order
    for (uint32_t r = tid; r < n; r += BLOCK) {
        const uint32_t v = perm[r];
        const uint64_t t = triR[r], x = numR[r] + t;
        if (a.tri) a.tri[va + v] = t;
        if (a.num) a.num[va + v] = x;
        if (a.tc) a.tc[va + v] = tg == 0 ? 0.0 : __ddiv_rn((double)x, (double)(3 * tg));
    }
    if (a.sup)
        for (uint32_t s = tid; s < m; s += BLOCK) a.sup[pa + o2e[s]] = osup[s];
    if (tid == 0) {
        a.num_edges[g] = m;
        if (a.triG) a.triG[g] = tg;
        a.status[g] = odd ? TC_ERR_DEVICE : (tg == 0 ? TC_TRIANGLE_FREE : TC_OK);
    }
    __syncthreads();
}

__global__ void k_fused_init(unsigned char *ws) {
    if (threadIdx.x == 0) reinterpret_cast<uint32_t *>(ws)[0] = 0;
}

// 512-thread workgroups ask for 4 wavefronts per SIMD (at most 128 VGPRs),
// so that two of them fit on a compute unit
template <int BLOCK>
__global__ __launch_bounds__(BLOCK, BLOCK == 512 ? 4 : 1) void k_fused_graphs(FusedArgs a) {
    __shared__ FusedLds<BLOCK> sh;
    uint32_t *head = reinterpret_cast<uint32_t *>(a.ws);
    for (;;) {
        if (threadIdx.x == 0) sh.bcast = atomicAdd(head, 1u);
        __syncthreads();
        // the same value in every lane: keep it (and what derives from it) in
        // scalar registers
        const uint32_t slot = __builtin_amdgcn_readfirstlane(sh.bcast);
        __syncthreads();
        if (slot >= (uint32_t)a.G) break;
        const int32_t g = a.order ? __builtin_amdgcn_readfirstlane(a.order[slot]) : (int32_t)slot;
        if (g < 0 || g >= a.G) continue;  // not a permutation: skip the entry
        fused_one_graph<BLOCK>(a, g, sh);
    }
}

int cu_count() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

template <int BLOCK>
tc_status launch(const FusedArgs &a, int wg_per_cu, hipStream_t s) {
    int64_t grid = (int64_t)cu_count() * wg_per_cu;
    if (grid > a.G) grid = a.G;
    if (grid < 1) grid = 1;
    k_fused_graphs<BLOCK><<<(unsigned)grid, BLOCK, 0, s>>>(a);
    TC_LAUNCHED();
    return TC_OK;
}

// Workspace of the allocation-free entry point: one array per GPU, held from
// the library's load to the end of the process and shared by every call on
// that GPU.  Host code never uses the array's name as an address (it is a
// host-side stand-in): the device address comes from hipGetSymbolAddress,
// taken once per device on the first call there, with that device current.
constexpr int64_t FUSED_SCRATCH_BYTES = (int64_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[FUSED_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {nullptr};

tc_status scratch_address(void **out) {
    int dev = 0;
    TC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        TC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return TC_ERR_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TC_OK;
}

tc_status check_args(const int32_t *src, const int32_t *dst, const int64_t *pair_off,
                     const int64_t *vtx_off, int32_t G, int64_t P, int64_t N, const int64_t *num_edges,
                     const int32_t *status, const tc_fused_tuning *t) {
    if (G < 0 || P < 0 || N < 0) return TC_ERR_INVALID_ARG;
    if (G > 0 && (!pair_off || !vtx_off || !num_edges || !status)) return TC_ERR_INVALID_ARG;
    if (P > 0 && (!src || !dst)) return TC_ERR_INVALID_ARG;
    if (P >= (int64_t)1 << 40 || N >= (int64_t)1 << 40) return TC_ERR_UNSUPPORTED;
    if (t) {
        if (t->block != 256 && t->block != 512 && t->block != 1024) return TC_ERR_INVALID_ARG;
        if (t->wg_per_cu < 1 || t->wg_per_cu > 16) return TC_ERR_INVALID_ARG;
    }
    return TC_OK;
}

tc_status run(const int32_t *src, const int32_t *dst, const int64_t *pair_off,
              const int64_t *vtx_off, const int32_t *order, int32_t G, int64_t P, int64_t N,
              int32_t *eu, int32_t *ev, uint64_t *support, int64_t *num_edges, uint64_t *tri,
              uint64_t *triG, uint64_t *num, double *tc, int32_t *status, void *ws,
              const tc_fused_tuning *t, hipStream_t s) {
    if (G == 0) return TC_OK;
    FusedArgs a;
    a.src = src;
    a.dst = dst;
    a.pair_off = pair_off;
    a.vtx_off = vtx_off;
    a.order = order;
    a.G = G;
    a.P = P;
    a.N = N;
    a.eu = eu;
    a.ev = ev;
    a.sup = support;
    a.num_edges = num_edges;
    a.tri = tri;
    a.num = num;
    a.tc = tc;
    a.triG = triG;
    a.status = status;
    a.ws = static_cast<unsigned char *>(ws);
    tc_fused_tuning d;
    tc_fused_tuning_default(&d);
    const tc_fused_tuning &u = t ? *t : d;
    k_fused_init<<<1, 64, 0, s>>>(a.ws);
    TC_LAUNCHED();
    switch (u.block) {
        case 256: return launch<256>(a, u.wg_per_cu, s);
        case 512: return launch<512>(a, u.wg_per_cu, s);
        default: return launch<1024>(a, u.wg_per_cu, s);
    }
}

}  // namespace

extern "C" {

tc_status tc_fused_tuning_default(tc_fused_tuning *t) {
    if (!t) return TC_ERR_INVALID_ARG;
    // measured on MI355X: 1024-thread workgroups, one per compute unit
    // (the 4096-graph BA batch 29.7 ms against 39.2 ms at 512 x 4)
    t->block = 1024;
    t->wg_per_cu = 1;
    return TC_OK;
}

int64_t tc_batch_fused_workspace_bytes(int64_t num_pairs, int64_t num_vertices, int32_t num_graphs) {
    if (num_pairs < 0 || num_vertices < 0 || num_graphs < 0) return -1;
    return FUSED_HEADER + pair_region(num_pairs) + FUSED_VTX_BYTES * num_vertices +
           FUSED_GRAPH_BYTES * (int64_t)num_graphs;
}

tc_status tc_batch_fused(const int32_t *src, const int32_t *dst, const int64_t *graph_pair_off,
                         const int64_t *graph_vtx_off, const int32_t *order, int32_t num_graphs,
                         int64_t num_pairs, int64_t num_vertices, int32_t *eu, int32_t *ev,
                         uint64_t *support, int64_t *num_edges, uint64_t *tri, uint64_t *triG,
                         uint64_t *num, double *tc, int32_t *status, void *workspace,
                         int64_t workspace_bytes, const tc_fused_tuning *tuning, void *stream) {
    TC_TRY(check_args(src, dst, graph_pair_off, graph_vtx_off, num_graphs, num_pairs, num_vertices,
                      num_edges, status, tuning));
    if (num_graphs == 0) return TC_OK;
    const int64_t need = tc_batch_fused_workspace_bytes(num_pairs, num_vertices, num_graphs);
    if (!workspace || workspace_bytes < need) return TC_ERR_INVALID_ARG;
    if (((uintptr_t)workspace & 255) != 0) return TC_ERR_INVALID_ARG;
    return run(src, dst, graph_pair_off, graph_vtx_off, order, num_graphs, num_pairs, num_vertices,
               eu, ev, support, num_edges, tri, triG, num, tc, status, workspace, tuning,
               (hipStream_t)stream);
}

int64_t tc_batch_fused_noalloc_max_bytes(void) { return FUSED_SCRATCH_BYTES; }

tc_status tc_batch_fused_noalloc(const int32_t *src, const int32_t *dst,
                                 const int64_t *graph_pair_off, const int64_t *graph_vtx_off,
                                 const int32_t *order, int32_t num_graphs, int64_t num_pairs,
                                 int64_t num_vertices, int32_t *eu, int32_t *ev, uint64_t *support,
                                 int64_t *num_edges, uint64_t *tri, uint64_t *triG, uint64_t *num,
                                 double *tc, int32_t *status, const tc_fused_tuning *tuning,
                                 void *stream) {
    TC_TRY(check_args(src, dst, graph_pair_off, graph_vtx_off, num_graphs, num_pairs, num_vertices,
                      num_edges, status, tuning));
    if (num_graphs == 0) return TC_OK;
    const int64_t need = tc_batch_fused_workspace_bytes(num_pairs, num_vertices, num_graphs);
    if (need > FUSED_SCRATCH_BYTES) return TC_ERR_BUDGET;
    void *ws = nullptr;
    TC_TRY(scratch_address(&ws));
    return run(src, dst, graph_pair_off, graph_vtx_off, order, num_graphs, num_pairs, num_vertices,
               eu, ev, support, num_edges, tri, triG, num, tc, status, ws, tuning,
               (hipStream_t)stream);
}

}  // extern "C"
