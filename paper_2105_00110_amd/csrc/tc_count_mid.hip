// Triangle counting with per-edge support, middle-pivot form.
//
// This is the paper's Procedure 1 (TriangleNeighbor, Sec. "Algorithm") on
// the degree-ordered orientation: for a pivot v, mark N_H(v) (the array T
// of the procedure, here an LDS hash table); for every lower neighbour u of
// v (u ∈ N_L(v)) scan N_H(u) for marked entries.  Reading the procedure's
// test as "T(w) is 1" for w ∈ N_H(u), each hit w is a triangle u < v < w
// (u low, v middle, w high), found exactly once.  Since w must lie above v
// in N_H(u) (which is sorted), only the part of N_H(u) after v's own slot is
// scanned: the streamed work is Σ_u C(|N_H(u)|, 2), the number of oriented
// wedges, instead of Σ_{v→u} |N_H(u)| for the low-pivot form.
//
// Support updates per triangle (u, v, w):
//   sup(v,w) += 1   LDS counter of the pivot's slot, flushed once per slot;
//   sup(u,v), sup(u,w): both lie in u's row.  Every scanned pair (u, v)
//   records its hits as a bit row over u's tail after v (bit b <-> the
//   entry b+1 places after v's slot), written with plain 32-bit stores; u's
//   rows form a triangular bit matrix B_u (row i = pair (u, N_H(u)[i])).
//   A second kernel folds each B_u: the popcount of row i is the number of
//   triangles on (u, N_H(u)[i]) as its (low, middle) edge, the sum of
//   column j is the number on (u, N_H(u)[j]) as its (low, high) edge.  So no
//   support update of the scan goes to device memory by atomic.
//
// Data: the transposed orientation in_pair, grouped by pivot: entry i of
// pivot v holds (u << 32) | k where k is the slot of v in N_H(u); the scan
// runs over ocol[k+1, orp[u+1]).  B_u starts at word rowbase[u]; its row i
// holds ceil((d-1-i)/32) words (d = |N_H(u)|), so row i starts at word
// S(d) - S(d-i) with S(d) = Σ_{t<d} ceil(t/32).
//
// 16-bit candidates.  Every entry scanned for a pivot v is a rank above v,
// so for the pivots among the top 2^16 ranks it fits in 16 bits once
// n - 2^16 is taken off.  Those pivots scan ocol16, a 16-bit copy of ocol,
// and key their lookup structure the same way: half the bytes of the scan
// for most of its candidates on skewed graphs.
//
// Work mapping.  A work item is a pivot with a slice of its pairs.  A
// wavefront takes 64 pairs at a time and flattens their bit rows: a prefix
// sum of the row lengths in words places word x of the group, and the lane
// that owns word x scans its 32 candidates and stores the word, so short
// and long scans both keep all 64 lanes busy.  Pivots with small |N_H(v)|
// are one wavefront per item with a private table; larger ones share a
// workgroup table; pivots whose table does not fit LDS probe N_H(v) by
// binary search in device memory.
#include "tc_internal.h"
#include <stdlib.h>
#include "tc_table.h"

namespace {

using namespace tc_tab;

constexpr int BK = 256;
constexpr size_t GROUP_BYTES = 64 * 8 * 3 + 64 * 4;  // gx, gs, gb (int64), gt (int32)
constexpr int GROUP_LANES = 16;  // lanes per short pivot (k_mid_groups)
constexpr int GROUP_DMAX = 128;  // rows up to this many entries go to k_mid_groups
constexpr int GROUP_PAIRS = 64;  // pairs per k_mid_groups item

// Words of the bit rows of a row with d entries: Σ_{t=1}^{d-1} ceil(t/32).
__host__ __device__ __forceinline__ int64_t bit_words(int64_t d) {
    if (d < 2) return 0;
    const int64_t q = (d - 1) >> 5, r = (d - 1) & 31;
    return 32 * (q * (q + 1) / 2) + (q + 1) * r;
}

// bit_words in the index type I of the fold: 32-bit for rows below
// FOLD_I32_MAX entries (every offset inside such a B_u fits), 64-bit
// otherwise.  With 32-bit indices x < 2^15, so q < 2^10 and both products
// are exact in the full-rate 24-bit multiply.
template <typename I>
__device__ __forceinline__ I bit_words_t(I x) {
    if (x < 2) return 0;
    const I q = (x - 1) >> 5, r = (x - 1) & 31;
    if constexpr (sizeof(I) == 4)
        return (I)(32u * (__umul24((uint32_t)q, (uint32_t)q + 1u) >> 1) +
                   __umul24((uint32_t)q + 1u, (uint32_t)r));
    else
        return 32 * (q * (q + 1) / 2) + (q + 1) * r;
}
constexpr int64_t FOLD_I32_MAX = 32768;

static inline unsigned grid_for(int64_t n, int block = BK) {
    int64_t g = tc_div_up(n, block);
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (unsigned)g;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ---------------------------------------------------------------------------
// 16-bit copy of ocol: two entries per thread, r - base for ranks at or
// above base, 0 for the others and for the padding.
// ---------------------------------------------------------------------------
__global__ void k_ocol16(int64_t pairs, int64_t m, const int32_t *__restrict__ ocol, int32_t base,
                         uint32_t *__restrict__ o16) {
    GRID_STRIDE(i, pairs) {
        uint32_t h[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t k = 2 * i + e;
            const int32_t r = k < m ? ocol[k] : 0;
            h[e] = r >= base ? (uint32_t)(r - base) : 0u;
        }
        o16[i] = h[0] | h[1] << 16;
    }
}

// ---------------------------------------------------------------------------
// Transposed orientation
// ---------------------------------------------------------------------------
// Number of lower-ordered neighbours of rank r: its degree less d+(r).
__global__ void k_in_len(int32_t n, const int32_t *__restrict__ perm,
                         const int64_t *__restrict__ row_ptr, const int64_t *__restrict__ orp,
                         int64_t *__restrict__ len) {
    GRID_STRIDE(r, n) {
        const int32_t v = perm[r];
        len[r] = (row_ptr[v + 1] - row_ptr[v]) - (orp[r + 1] - orp[r]);
    }
}

// ---------------------------------------------------------------------------
// Work items: pivot v with |N_H(v)| in [lo, hi] and at least one lower
// neighbour, cut into slices of at most S pairs.
// ---------------------------------------------------------------------------
// Items of the pivots with lo <= |N_H(v)| <= hi.  A pivot "fits the bitmap"
// when its rank span is at most span_max and it has at least pairs_min
// pairs; sel 1 keeps only such pivots, sel 2 only the others, sel 0 all.
__global__ void k_item_count(int32_t n, const int64_t *__restrict__ orp,
                             const int32_t *__restrict__ ocol, const int64_t *__restrict__ in_ptr,
                             int lo, int hi, int S, int sel, int64_t span_max, int64_t pairs_min,
                             int32_t rlo, int32_t rhi, uint32_t *__restrict__ cnt) {
    GRID_STRIDE(v, n) {
        const int64_t d = orp[v + 1] - orp[v];
        const int64_t in = in_ptr[v + 1] - in_ptr[v];
        bool ok = d >= lo && d <= hi && in > 0 && v >= rlo && v < rhi;
        if (ok && sel != 0) {
            const int64_t span = (int64_t)ocol[orp[v + 1] - 1] - ocol[orp[v]] + 1;
            const bool fits = span <= span_max && in >= pairs_min;
            ok = sel == 1 ? fits : !fits;
        }
        cnt[v] = ok ? (uint32_t)tc_div_up(in, S) : 0u;
    }
}

__global__ void k_item_write(int32_t n, const uint32_t *__restrict__ cnt,
                             const uint32_t *__restrict__ off, const int64_t *__restrict__ in_ptr,
                             int S, int32_t *__restrict__ item_v, uint32_t *__restrict__ item_first) {
    GRID_STRIDE(v, n) {
        const uint32_t c = cnt[v];
        for (uint32_t t = 0; t < c; ++t) {
            item_v[off[v] + t] = (int32_t)v;
            item_first[off[v] + t] = (uint32_t)(in_ptr[v] + (int64_t)t * S);
        }
    }
}

// ---------------------------------------------------------------------------
// Lookups of a pivot's row N_H(v) (position of a rank in the row, or -1).
//   LK_HASH    the LDS hash table (tc_table.h);
//   LK_GLOBAL  binary search in device memory (rows too long for LDS);
//   LK_BITMAP  a bitmap over the row's rank span [lo, lo + span) in LDS:
//              word x holds bits (rank - lo) in [32x, 32x + 32) and the
//              number of row entries before them; a probe is one 8-byte
//              read, a bit test and a popcount.
//   LK_BITMAP16  for pivots v among the top 2^16 ranks, whose candidates
//              are 16-bit entries (rank less rank16_base): the bitmap has
//              2048 words indexed by the 16-bit value itself, so every
//              value indexes inside it with no subtraction and no range
//              test, and the bit-field reads take their offset and width
//              from the value's low 5 bits.  Values at or below v's own
//              hold no bits.  A probe reads the packed pairs of entries as
//              loaded; only hits add to the counters.
// ---------------------------------------------------------------------------
constexpr int LK_HASH = 0, LK_GLOBAL = 1, LK_BITMAP = 2, LK_BITMAP16 = 3;
constexpr int BITMAP16_WORDS = 2048;

struct BitmapRow {
    const uint2 *bm;  // {bits, entries before this word}
    uint32_t lo, span;
};

template <int N>
__device__ __forceinline__ void bitmap_find_n(const BitmapRow &b, const uint32_t (&key)[N],
                                              int (&q)[N]) {
    uint32_t idx[N];
    uint2 w[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        idx[e] = key[e] - b.lo;  // keys below lo wrap above span
        const bool in = idx[e] < b.span;
        w[e] = b.bm[in ? idx[e] >> 5 : 0];
        idx[e] = in ? idx[e] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const uint32_t sh = idx[e] & 31;
        const bool hit = idx[e] != 0xFFFFFFFFu && ((w[e].x >> sh) & 1u);
        const uint32_t below = w[e].x & ((1u << sh) - 1u);
        q[e] = hit ? (int)(w[e].y + (uint32_t)__popc(below)) : -1;
    }
}

// The same probe, as a counter index that is always in bounds and a hit bit:
// q = entries of the row before the key's place (spare, this lane's spare
// counter, for a key outside the span), hit = 1 if the key is in the row.
template <int N>
__device__ __forceinline__ void bitmap_probe_n(const BitmapRow &b, const uint32_t (&key)[N],
                                               int spare, int (&q)[N], uint32_t (&hit)[N]) {
    uint32_t idx[N];
    uint2 w[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        idx[e] = key[e] - b.lo;  // keys below lo wrap above span
        w[e] = b.bm[idx[e] < b.span ? idx[e] >> 5 : 0];
    }
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const uint32_t sh = idx[e] & 31;
        const uint32_t in = idx[e] < b.span ? 1u : 0u;
        hit[e] = ((w[e].x >> sh) & 1u) & in;
        const int pos = (int)(w[e].y + (uint32_t)__popc(w[e].x & ((1u << sh) - 1u)));
        q[e] = in ? pos : spare;
    }
}

// Builds the bitmap of row ocol[vstart, vstart + d) (sorted ranks) with the
// threads of a workgroup; words beyond the span are not touched.
__device__ void bitmap_build(uint2 *bm, uint32_t *scan, const int32_t *__restrict__ ocol,
                             int64_t vstart, int d, uint32_t lo, uint32_t span) {
    const int nw = (int)((span + 31) >> 5);
    for (int x = threadIdx.x; x < nw; x += blockDim.x) bm[x] = make_uint2(0u, 0u);
    __syncthreads();
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        const uint32_t r = (uint32_t)ocol[vstart + j] - lo;
        atomicOr(&bm[r >> 5].x, 1u << (r & 31));
    }
    __syncthreads();
    // exclusive prefix of the word popcounts: each thread a contiguous run
    const int per = (nw + (int)blockDim.x - 1) / (int)blockDim.x;
    const int x0 = threadIdx.x * per;
    uint32_t c = 0;
    for (int x = x0; x < x0 + per && x < nw; ++x) c += (uint32_t)__popc(bm[x].x);
    const uint32_t incl = tc_wave_incl_scan(c);
    const int wv = threadIdx.x / TC_WAVE;
    if (__lane_id() == TC_WAVE - 1) scan[wv] = incl;
    __syncthreads();
    uint32_t before = incl - c;
    for (int q = 0; q < wv; ++q) before += scan[q];
    for (int x = x0; x < x0 + per && x < nw; ++x) {
        bm[x].y = before;
        before += (uint32_t)__popc(bm[x].x);
    }
    __syncthreads();
}

// One lane's 32-entry run of a pair's tail for an LK_BITMAP16 pivot: the
// hit mask of entries c0 .. c0 + cnt - 1 (bit j for entry c0 + j).  17
// aligned words hold the 32 entries from c0 (an odd c0 starts in the upper
// half of the first); each aligned pair is probed as loaded: the lower entry
// is the word's low 16 bits, whose low 5 bits the bit-field reads take as
// they are, the upper entry its high 16 bits.  Every hit inside the tail
// adds 1 to the counter of its place in the pivot's row: only those lanes
// take part in the LDS add (a lane mask, not a select of a spare counter:
// the select cost a VALU instruction per entry).
__device__ __forceinline__ uint32_t bitmap16_run(const uint16_t *__restrict__ ocol16, int64_t c0,
                                                 int cnt, const uint2 *bm, uint32_t *lsup) {
    const uint32_t *o32 = reinterpret_cast<const uint32_t *>(ocol16);
    const int64_t q = c0 >> 1;
    const uint32_t sh = (uint32_t)(c0 & 1) << 4;
    uint32_t dw[17];
#pragma unroll
    for (int j = 0; j < 17; ++j) dw[j] = o32[q + j];
    uint32_t pk[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) pk[j] = __builtin_amdgcn_alignbit(dw[j + 1], dw[j], sh);
    uint32_t mask = 0;
#pragma unroll
    for (int c = 0; c < 16; c += 4) {
        uint32_t key[8];
        uint2 w[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            key[2 * e] = pk[c + e];
            key[2 * e + 1] = pk[c + e] >> 16;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = bm[__builtin_amdgcn_ubfe(key[e], 5u, 11u)];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 2 * c + e;  // the entry's place in the run
            const uint32_t bit = __builtin_amdgcn_ubfe(w[e].x, key[e], 1u);
            const uint32_t at =
                w[e].y + (uint32_t)__popc(__builtin_amdgcn_ubfe(w[e].x, 0u, key[e]));
            if (bit != 0u && k < cnt) atomicAdd(&lsup[at], 1u);
            mask |= bit << k;
        }
    }
    if (cnt < 32) mask &= (1u << cnt) - 1u;
    return mask;
}

// ---------------------------------------------------------------------------
// One 64-pair group of pivot v (wave-level).  Pairs g0 .. gend-1 (at most
// 64).  gx/gs/gb/gt: this wavefront's LDS arrays (exclusive scan of word
// counts, scan starts, bit-row bases, tail lengths).
// ---------------------------------------------------------------------------
// GL lanes take the group (a whole wavefront for GL = 64, or one of its
// 64 / GL groups, each with its own arrays and counters); at most GL pairs.
template <int LK, int GL = TC_WAVE, bool N16 = false>
__device__ __forceinline__ void mid_group(const int32_t *__restrict__ ocol,
                                          const uint16_t *__restrict__ ocol16,
                                          const uint64_t *__restrict__ in_pair,
                                          const uint4 *__restrict__ rowinfo, int64_t g0,
                                          int64_t gend, const RowTable &t, const BitmapRow &bmr,
                                          uint32_t hmax,
                                          uint32_t *lsup, int64_t vstart, int dv, int64_t *gx,
                                          int64_t *gs, int64_t *gb, int32_t *gt,
                                          uint32_t *__restrict__ bits, uint32_t *__restrict__ osup,
                                          unsigned long long &found) {
    static_assert(GL <= TC_WAVE && TC_WAVE % GL == 0, "group width");
    static_assert(LK != LK_BITMAP16 || N16, "the 2048-word bitmap takes 16-bit keys");
    const int lane = __lane_id() % GL;
    const int64_t i = g0 + lane;
    int64_t words = 0;
    if (i < gend) {
        const uint64_t pr = in_pair[i];
        const int64_t k = (int64_t)(uint32_t)pr;
        const int32_t u = (int32_t)(pr >> 32);
        // the row's start and end in ocol and its bit matrix's first
        // word, in one 16-byte record
        const uint4 ri = rowinfo[u];
        const int64_t rs = ri.z;
        const int64_t d = (int64_t)ri.w - rs;
        const int64_t ii = k - rs;
        const int64_t tail = d - 1 - ii;
        words = (tail + 31) >> 5;
        gs[lane] = k + 1;
        gb[lane] = (int64_t)(((uint64_t)ri.y << 32) | ri.x) + bit_words(d) - bit_words(d - ii);
        gt[lane] = (int32_t)tail;
    }
    int64_t incl = words;
    if constexpr (GL == TC_WAVE) {
        incl = tc_wave_incl_scan(words);
    } else {
#pragma unroll
        for (int off = 1; off < GL; off <<= 1) {
            const int64_t t = __shfl_up(incl, off, GL);
            if (lane >= off) incl += t;
        }
    }
    const int64_t total = __shfl(incl, GL - 1, GL);
    gx[lane] = incl - words;
    for (int64_t base = 0; base < total; base += GL) {
        const int64_t x = base + lane;
        if (x < total) {
            int lo = 0, hi = GL - 1;  // last pair p with gx[p] <= x
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (gx[mid] <= x) lo = mid; else hi = mid - 1;
            }
            const int p = lo;
            const int64_t kw = x - gx[p];
            const int64_t c0 = gs[p] + 32 * kw;
            const int cnt = min(32, gt[p] - 32 * (int)kw);
            // whole 32-entry run (the arrays are padded past their end);
            // entries past the tail are masked to EMPTY
            uint32_t ww[32];
            if constexpr (N16) {
                // 17 aligned words hold the 32 entries from c0; an odd c0
                // starts in the upper half of the first
                const uint32_t *o32 = reinterpret_cast<const uint32_t *>(ocol16);
                const int64_t q = c0 >> 1;
                const uint32_t sh = (uint32_t)(c0 & 1) << 4;
                uint32_t dw[17];
#pragma unroll
                for (int j = 0; j < 17; ++j) dw[j] = o32[q + j];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const uint32_t a = __builtin_amdgcn_alignbit(dw[j + 1], dw[j], sh);
                    ww[2 * j] = 2 * j < cnt ? (a & 0xFFFFu) : EMPTY;
                    ww[2 * j + 1] = 2 * j + 1 < cnt ? (a >> 16) : EMPTY;
                }
            } else {
#pragma unroll
                for (int b = 0; b < 32; ++b) {
                    const uint32_t v = (uint32_t)ocol[c0 + b];
                    ww[b] = b < cnt ? v : EMPTY;
                }
            }
            // probe in batches of 8 (EMPTY, past the tail, is above every
            // rank and is never looked up); apply each batch's hits at once
            uint32_t mask = 0;
#pragma unroll
            for (int c = 0; c < 32; c += 8) {
                uint32_t kk[8];
                int qc[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) kk[e] = ww[c + e];
                if constexpr (LK == LK_GLOBAL) {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        qc[e] = kk[e] <= hmax ? row_search(ocol, vstart, dv, kk[e]) : -1;
                } else if constexpr (LK == LK_BITMAP) {
                    // the counter index is always valid (the key's place in
                    // the row, or this lane's spare counter outside the
                    // span), and the add is the hit bit itself
                    uint32_t hb[8];
                    bitmap_probe_n<8>(bmr, kk, dv + lane, qc, hb);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        mask |= hb[e] << (c + e);
                        atomicAdd(&lsup[qc[e]], hb[e]);
                    }
                    continue;
                } else {
                    table_find_n<8>(t, kk, hmax, qc);
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const bool hit = qc[e] >= 0;
                    mask |= (hit ? 1u : 0u) << (c + e);
                    if constexpr (LK == LK_GLOBAL) {
                        if (hit) atomicAdd(&osup[vstart + qc[e]], 1u);
                    } else {
                        // a miss adds 0 to this lane's spare counter: no branch
                        atomicAdd(&lsup[hit ? qc[e] : dv + lane], hit ? 1u : 0u);
                    }
                }
            }
            bits[gb[p] + kw] = mask;
            found += (unsigned long long)__popc(mask);
        }
    }
}

// Counter slots rounded up to keep the int64 group arrays 16-byte aligned.
// (plus one spare slot per lane that branch-free misses add 0 to)
__host__ __device__ __forceinline__ size_t counter_bytes(int d) {
    return 4 * ((((size_t)d + 3) & ~(size_t)3) + TC_WAVE);
}

__host__ __device__ __forceinline__ size_t mid_wave_bytes(int dcap) {
    return table_bytes(dcap) + counter_bytes(dcap) + GROUP_BYTES;
}

// One wavefront per item; pivots with |N_H(v)| <= dcap.
__global__ __launch_bounds__(1024) void k_mid_wave(const int64_t *__restrict__ orp,
                                                   const int32_t *__restrict__ ocol,
                                                   const int64_t *__restrict__ in_ptr,
                                                   const uint64_t *__restrict__ in_pair,
                                                   const uint4 *__restrict__ rowinfo,
                                                   uint32_t *__restrict__ bits,
                                                   const int32_t *__restrict__ item_v,
                                                   const uint32_t *__restrict__ item_first,
                                                   int64_t nitems, int dcap, int item_pairs,
                                                   const uint16_t *__restrict__ ocol16, int32_t r16,
                                                   uint32_t *__restrict__ osup,
                                                   unsigned long long *__restrict__ tri_total) {
    extern __shared__ uint4 lds4[];
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    char *base = reinterpret_cast<char *>(lds4) + (size_t)wv * mid_wave_bytes(dcap);
    const size_t tb = table_bytes(dcap);
    const size_t nbmax = (size_t)1 << bucket_bits(dcap);
    uint32_t *keys = reinterpret_cast<uint32_t *>(base);
    uint16_t *pos = reinterpret_cast<uint16_t *>(base + 16 * nbmax);
    uint32_t *lsup = reinterpret_cast<uint32_t *>(base + tb);
    char *grp = base + tb + counter_bytes(dcap);
    int64_t *gx = reinterpret_cast<int64_t *>(grp);
    int64_t *gs = gx + 64;
    int64_t *gb = gs + 64;
    int32_t *gt = reinterpret_cast<int32_t *>(gb + 64);
    unsigned long long found = 0;
    for (int64_t it = (int64_t)blockIdx.x * wpb + wv; it < nitems; it += (int64_t)gridDim.x * wpb) {
        const int32_t v = item_v[it];
        const int64_t first = item_first[it];
        const int64_t pend = min(first + (int64_t)item_pairs, in_ptr[v + 1]);
        const int64_t vstart = orp[v];
        const int d = (int)(orp[v + 1] - vstart);
        const RowTable t{keys, pos, bucket_bits(d)};
        // pivots among the top 2^16 ranks scan 16-bit entries; their table
        // holds ranks less r16 to match
        const bool n16 = v >= r16;
        const uint32_t rel = n16 ? (uint32_t)r16 : 0u;
        for (int j = lane; j < (4 << t.bb); j += TC_WAVE) keys[j] = EMPTY;
        for (int j = lane; j < d; j += TC_WAVE) lsup[j] = 0;
        for (int j = lane; j < d; j += TC_WAVE)
            table_insert(t, (uint32_t)ocol[vstart + j] - rel, j);
        const uint32_t hmax = (uint32_t)ocol[vstart + d - 1] - rel;
        for (int64_t g0 = first; g0 < pend; g0 += TC_WAVE) {
            if (n16)
                mid_group<LK_HASH, TC_WAVE, true>(ocol, ocol16, in_pair, rowinfo, g0,
                                                  min(g0 + TC_WAVE, pend), t,
                                                  BitmapRow{nullptr, 0, 0}, hmax, lsup, vstart, d,
                                                  gx, gs, gb, gt, bits, osup, found);
            else
                mid_group<LK_HASH>(ocol, nullptr, in_pair, rowinfo, g0,
                                   min(g0 + TC_WAVE, pend), t, BitmapRow{nullptr, 0, 0}, hmax,
                                   lsup, vstart, d, gx, gs, gb, gt, bits, osup, found);
        }
        for (int j = lane; j < d; j += TC_WAVE) {
            const uint32_t c = lsup[j];
            if (c) atomicAdd(&osup[vstart + j], c);
        }
    }
    found = tc_wave_sum(found);
    if (lane == 0 && found) atomicAdd(tri_total, found);
}

static inline size_t mid_block_bytes(int dmax, int wpb, int lk, int bitmap_words) {
    size_t t = 0;
    if (lk == LK_HASH) t = table_bytes(dmax) + counter_bytes(dmax);
    if (lk == LK_BITMAP) t = 8 * (size_t)bitmap_words + counter_bytes(dmax) + 64;
    return t + (size_t)wpb * GROUP_BYTES;
}

// Several short pivots per wavefront: groups of GL lanes each take one item
// (pivot rows of at most dcap entries, items of a few pairs), with their own
// LDS table, counters and pair arrays; mid_group runs on the group.  Short
// pivots have a few words of candidates per item, so a whole wavefront per
// item would leave most lanes idle.
__host__ __device__ __forceinline__ size_t mid_group_bytes(int dcap, int gl) {
    return table_bytes(dcap) + counter_bytes(dcap) + (size_t)gl * (8 * 3 + 4);
}

template <int GL>
__global__ __launch_bounds__(256, 4) void k_mid_groups(const int64_t *__restrict__ orp,
                                                    const int32_t *__restrict__ ocol,
                                                    const int64_t *__restrict__ in_ptr,
                                                    const uint64_t *__restrict__ in_pair,
                                                    const uint4 *__restrict__ rowinfo,
                                                    uint32_t *__restrict__ bits,
                                                    const int32_t *__restrict__ item_v,
                                                    const uint32_t *__restrict__ item_first,
                                                    int64_t nitems, int dcap, int item_pairs,
                                                    uint32_t *__restrict__ osup,
                                                    unsigned long long *__restrict__ tri_total) {
    extern __shared__ uint4 lds4[];
    const int gpb = blockDim.x / GL;
    const int gi = threadIdx.x / GL;
    const int lane = threadIdx.x % GL;
    char *base = reinterpret_cast<char *>(lds4) + (size_t)gi * mid_group_bytes(dcap, GL);
    const size_t tb = table_bytes(dcap);
    const size_t nbmax = (size_t)1 << bucket_bits(dcap);
    uint32_t *keys = reinterpret_cast<uint32_t *>(base);
    uint16_t *pos = reinterpret_cast<uint16_t *>(base + 16 * nbmax);
    uint32_t *lsup = reinterpret_cast<uint32_t *>(base + tb);
    char *grp = base + tb + counter_bytes(dcap);
    int64_t *gx = reinterpret_cast<int64_t *>(grp);
    int64_t *gs = gx + GL;
    int64_t *gb = gs + GL;
    int32_t *gt = reinterpret_cast<int32_t *>(gb + GL);
    unsigned long long found = 0;
    for (int64_t it = (int64_t)blockIdx.x * gpb + gi; it < nitems; it += (int64_t)gridDim.x * gpb) {
        const int32_t v = item_v[it];
        const int64_t first = item_first[it];
        const int64_t pend = min(first + (int64_t)item_pairs, in_ptr[v + 1]);
        const int64_t vstart = orp[v];
        const int d = (int)(orp[v + 1] - vstart);
        const RowTable t{keys, pos, bucket_bits(d)};
        for (int j = lane; j < (4 << t.bb); j += GL) keys[j] = EMPTY;
        for (int j = lane; j < d; j += GL) lsup[j] = 0;
        for (int j = lane; j < d; j += GL) table_insert(t, (uint32_t)ocol[vstart + j], j);
        const uint32_t hmax = (uint32_t)ocol[vstart + d - 1];
        for (int64_t g0 = first; g0 < pend; g0 += GL)
            mid_group<LK_HASH, GL>(ocol, nullptr, in_pair, rowinfo, g0, min(g0 + GL, pend), t,
                                   BitmapRow{nullptr, 0, 0}, hmax, lsup, vstart, d, gx, gs, gb, gt,
                                   bits, osup, found);
        for (int j = lane; j < d; j += GL) {
            const uint32_t c = lsup[j];
            if (c) atomicAdd(&osup[vstart + j], c);
        }
    }
    found = tc_wave_sum(found);
    if (__lane_id() == 0 && found) atomicAdd(tri_total, found);
}

// One workgroup per item; its wavefronts share the pivot's lookup structure
// and take the item's 64-pair groups in turn.  Pivots among the top 2^16
// ranks scan 16-bit entries; short items (the wavefront pivots moved to
// LK_BITMAP) take the bitmap over their row's span, which is cheaper to
// build than the 2048-word one of k_mid_block16.
template <int LK>
__global__ __launch_bounds__(1024) void k_mid_block(const int64_t *__restrict__ orp,
                                                    const int32_t *__restrict__ ocol,
                                                    const int64_t *__restrict__ in_ptr,
                                                    const uint64_t *__restrict__ in_pair,
                                                    const uint4 *__restrict__ rowinfo,
                                                    uint32_t *__restrict__ bits,
                                                    const int32_t *__restrict__ item_v,
                                                    const uint32_t *__restrict__ item_first,
                                                    int64_t nitems, int dmax, int item_pairs,
                                                    int bitmap_words,
                                                    const uint16_t *__restrict__ ocol16, int32_t r16,
                                                    uint32_t *__restrict__ osup,
                                                    unsigned long long *__restrict__ tri_total) {
    extern __shared__ uint4 lds4[];
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    char *base = reinterpret_cast<char *>(lds4);
    size_t tpart = 0;
    uint32_t *keys = nullptr, *lsup = nullptr, *scan = nullptr;
    uint16_t *pos = nullptr;
    uint2 *bm = nullptr;
    if constexpr (LK == LK_HASH) {
        const size_t nbmax = (size_t)1 << bucket_bits(dmax);
        keys = reinterpret_cast<uint32_t *>(base);
        pos = reinterpret_cast<uint16_t *>(base + 16 * nbmax);
        lsup = reinterpret_cast<uint32_t *>(base + table_bytes(dmax));
        tpart = table_bytes(dmax) + counter_bytes(dmax);
    } else if constexpr (LK == LK_BITMAP) {
        bm = reinterpret_cast<uint2 *>(base);
        lsup = reinterpret_cast<uint32_t *>(base + 8 * (size_t)bitmap_words);
        scan = reinterpret_cast<uint32_t *>(base + 8 * (size_t)bitmap_words + counter_bytes(dmax));
        tpart = 8 * (size_t)bitmap_words + counter_bytes(dmax) + 64;
    }
    char *grp = base + tpart + (size_t)wv * GROUP_BYTES;
    int64_t *gx = reinterpret_cast<int64_t *>(grp);
    int64_t *gs = gx + 64;
    int64_t *gb = gs + 64;
    int32_t *gt = reinterpret_cast<int32_t *>(gb + 64);
    unsigned long long found = 0;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int32_t v = item_v[it];
        const int64_t first = item_first[it];
        const int64_t pend = min(first + (int64_t)item_pairs, in_ptr[v + 1]);
        const int64_t vstart = orp[v];
        const int d = (int)(orp[v + 1] - vstart);
        RowTable t{keys, pos, 0};
        BitmapRow bmr{bm, 0, 0};
        // pivots among the top 2^16 ranks scan 16-bit entries (ranks less
        // r16); the lookup structure takes keys on the same footing
        const bool n16 = LK != LK_GLOBAL && v >= r16;
        const uint32_t rel = n16 ? (uint32_t)r16 : 0u;
        if constexpr (LK == LK_HASH) {
            t.bb = bucket_bits(d);
            for (int j = threadIdx.x; j < (4 << t.bb); j += blockDim.x) keys[j] = EMPTY;
            for (int j = threadIdx.x; j < d; j += blockDim.x) lsup[j] = 0;
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += blockDim.x)
                table_insert(t, (uint32_t)ocol[vstart + j] - rel, j);
            __syncthreads();
        } else if constexpr (LK == LK_BITMAP) {
            for (int j = threadIdx.x; j < d; j += blockDim.x) lsup[j] = 0;
            const uint32_t lo = (uint32_t)ocol[vstart];
            bmr.span = (uint32_t)ocol[vstart + d - 1] - lo + 1;
            bitmap_build(bm, scan, ocol, vstart, d, lo, bmr.span);
            bmr.lo = lo - rel;
        }
        const uint32_t hmax = (uint32_t)ocol[vstart + d - 1] - rel;
        for (int64_t g0 = first + (int64_t)wv * TC_WAVE; g0 < pend; g0 += (int64_t)wpb * TC_WAVE) {
            if constexpr (LK != LK_GLOBAL) {
                if (n16) {
                    mid_group<LK, TC_WAVE, true>(ocol, ocol16, in_pair, rowinfo, g0,
                                                 min(g0 + TC_WAVE, pend), t, bmr, hmax, lsup,
                                                 vstart, d, gx, gs, gb, gt, bits, osup, found);
                    continue;
                }
            }
            mid_group<LK>(ocol, nullptr, in_pair, rowinfo, g0, min(g0 + TC_WAVE, pend), t, bmr,
                          hmax, lsup, vstart, d, gx, gs, gb, gt, bits, osup, found);
        }
        if constexpr (LK != LK_GLOBAL) {
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += blockDim.x) {
                const uint32_t c = lsup[j];
                if (c) atomicAdd(&osup[vstart + j], c);
            }
            __syncthreads();
        }
    }
    found = tc_wave_sum(found);
    if (lane == 0 && found) atomicAdd(tri_total, found);
}

// Dynamic LDS bytes of k_mid_block16: the pivot's counters and the bitmap
// build's per-wavefront sums (the 2048-word bitmap is a static array, whose
// address the compiler folds into each read's offset).
__host__ __device__ __forceinline__ size_t mid_block16_bytes(int dmax) {
    return counter_bytes(dmax) + 64;
}

// Workgroup pivots among the top 2^16 ranks (LK_BITMAP16).  One workgroup
// per item as in k_mid_block, but a wavefront keeps its 64 pairs' word
// offsets, scan starts, tails and bit-row bases in registers and finds a
// word's pair by a search over lane shuffles, so the workgroup's LDS is the
// bitmap and the counters alone; with at most 80 VGPRs, six wavefronts per
// SIMD stay resident to cover the latency of the candidate loads.
__global__ __launch_bounds__(1024, 6) void k_mid_block16(
    const int64_t *__restrict__ orp, const int32_t *__restrict__ ocol,
    const int64_t *__restrict__ in_ptr, const uint64_t *__restrict__ in_pair,
    const uint4 *__restrict__ rowinfo, uint32_t *__restrict__ bits,
    const int32_t *__restrict__ item_v, const uint32_t *__restrict__ item_first, int64_t nitems,
    int dmax, int item_pairs, const uint16_t *__restrict__ ocol16, int32_t r16,
    uint32_t *__restrict__ osup, unsigned long long *__restrict__ tri_total) {
    __shared__ uint2 bm[BITMAP16_WORDS];
    extern __shared__ uint4 lds4[];
    char *base = reinterpret_cast<char *>(lds4);
    uint32_t *lsup = reinterpret_cast<uint32_t *>(base);
    uint32_t *scan = reinterpret_cast<uint32_t *>(base + counter_bytes(dmax));
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    unsigned long long found = 0;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int32_t v = item_v[it];
        const int64_t first = item_first[it];
        const int64_t pend = min(first + (int64_t)item_pairs, in_ptr[v + 1]);
        const int64_t vstart = orp[v];
        const int d = (int)(orp[v + 1] - vstart);
        // 2048 words over the 16-bit values, that is ranks r16 .. r16 + 2^16 - 1
        for (int j = threadIdx.x; j < d; j += blockDim.x) lsup[j] = 0;
        bitmap_build(bm, scan, ocol, vstart, d, (uint32_t)r16, 32u * BITMAP16_WORDS);
        for (int64_t g0 = first + (int64_t)wv * TC_WAVE; g0 < pend; g0 += (int64_t)wpb * TC_WAVE) {
            // this lane's pair: scan start, tail length, bit-row base and
            // word count (a row below 2^16 entries has fewer than 2^11
            // words per pair, so the group's word offsets fit 32 bits)
            const int64_t i = g0 + lane;
            int words = 0, tail = 0;
            uint32_t start = 0;
            int64_t gbase = 0;
            if (i < pend) {
                const uint64_t pr = in_pair[i];
                const int64_t k = (int64_t)(uint32_t)pr;
                const uint4 ri = rowinfo[(int32_t)(pr >> 32)];
                const int64_t rs = ri.z;
                const int64_t du = (int64_t)ri.w - rs;
                const int64_t ii = k - rs;
                tail = (int)(du - 1 - ii);
                words = (tail + 31) >> 5;
                start = (uint32_t)(k + 1);
                gbase = (int64_t)(((uint64_t)ri.y << 32) | ri.x) + bit_words(du) - bit_words(du - ii);
            }
            const int incl = tc_wave_incl_scan(words);
            const int excl = incl - words;
            const int total = __shfl(incl, TC_WAVE - 1, TC_WAVE);
            for (int wb = 0; wb < total; wb += TC_WAVE) {
                const int x = wb + lane;
                // the last pair p with excl(p) <= x: six steps, every lane
                int p = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1) {
                    const int e = __shfl(excl, p + step, TC_WAVE);
                    if (e <= x) p += step;
                }
                const int kw = x - __shfl(excl, p, TC_WAVE);
                const uint32_t st = __shfl(start, p, TC_WAVE);
                const int tl = __shfl(tail, p, TC_WAVE);
                const int64_t gb = __shfl(gbase, p, TC_WAVE);
                if (x < total) {
                    const int cnt = min(32, tl - 32 * kw);
                    const uint32_t mask =
                        bitmap16_run(ocol16, (int64_t)st + 32 * kw, cnt, bm, lsup);
                    bits[gb + kw] = mask;
                    found += (unsigned long long)__popc(mask);
                }
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < d; j += blockDim.x) {
            const uint32_t c = lsup[j];
            if (c) atomicAdd(&osup[vstart + j], c);
        }
        __syncthreads();
    }
    found = tc_wave_sum(found);
    if (lane == 0 && found) atomicAdd(tri_total, found);
}

// ---------------------------------------------------------------------------
// Fold of the bit matrices: a group of GL lanes per row u (|N_H(u)| >= 2).
//   row sums:    sup(u, N_H(u)[i]) += popcount(B_u row i)
//   column sums: sup(u, N_H(u)[j]) += Σ_{i<j} B_u[i][j]
// Column sums run over stripes of 32 columns; lane (stripe c, group g)
// takes every row i ≡ g (mod G) that reaches the stripe, extracts that
// row's 32 bits at the stripe's columns (row i's bit b is column i + 1 + b)
// and adds them into 6 bit-sliced counter planes (a carry-save adder, up to
// 63 rows), which are emptied into 32 integer counters every 63 rows.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void planes_flush(uint32_t (&pl)[6], uint32_t (&cnt)[32]) {
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) v |= ((pl[k] >> b) & 1u) << k;
        cnt[b] += v;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) pl[k] = 0;
}

// Phase boundary of one wavefront's LDS counters: the lanes run in
// lockstep, so a lane's LDS access after it sees every lane's access before
// it; the fences and the wave barrier keep the compiler from moving LDS
// accesses across it (no instruction is emitted).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Carry-save add of three bit vectors: s = a ^ b ^ c, cy = majority(a, b, c).
__device__ __forceinline__ void csa(uint32_t a, uint32_t b, uint32_t c, uint32_t &s,
                                    uint32_t &cy) {
    const uint32_t u = a ^ b;
    s = u ^ c;
    cy = (a & b) | (u & c);
}

// The 32 bits of row i of B_u at the columns of stripe c (row i's bit b
// is column i + 1 + b; bits outside the row read as 0).  lo/hi are the two
// row words the stripe can touch, already loaded.
__device__ __forceinline__ uint32_t stripe_bits(int o, uint32_t lo, uint32_t hi) {
    if (o < 0) return lo << (int)(-o);
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)o & 31u);  // (hi:lo) >> (o mod 32)
}

// Rows of at most 64 entries, GL lanes each (GL a power of two, 16).
// Row sums go to the group's LDS counters; for the column sums lane
// (stripe c, row group g) walks rows g, g + G, ... of its stripe and adds
// each row's 32 bits to byte counters: word s holds columns s, s + 8,
// s + 16, s + 24 in its bytes (a column of such a row counts at most 63).
// A butterfly over the G lanes of a stripe sums them, and one lane per
// stripe adds the 32 counts to the LDS counters (each counter has one
// writer), which are added to the support once per slot: no device-memory
// atomics.  The GL lanes of a group sit in one wavefront and take the same
// path up to the butterfly.
template <int GL>
__global__ __launch_bounds__(256) void k_fold(const int32_t *__restrict__ rows, int64_t nrows,
                                              const int64_t *__restrict__ orp,
                                              const int64_t *__restrict__ rowbase,
                                              const uint32_t *__restrict__ bits,
                                              uint32_t *__restrict__ osup) {
    static_assert(GL >= 2 && GL <= TC_WAVE && (GL & (GL - 1)) == 0, "GL: a power of two");
    __shared__ uint32_t acc_all[256 / GL][64];
    const int sub = threadIdx.x % GL;
    uint32_t *acc = acc_all[threadIdx.x / GL];
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / GL);
    for (int64_t gi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GL; gi < nrows; gi += groups) {
        const int32_t r = rows[gi];
        const int64_t rs = orp[r];
        const int d = (int)(orp[r + 1] - rs);  // 2 <= d <= 64
        const uint32_t *rb = bits + rowbase[r];  // B_u; offsets inside it fit 32 bits
        const int sd = bit_words_t<int>(d);
        for (int i = sub; i < d; i += GL) {
            uint32_t c = 0;
            if (i < d - 1) {
                const int off = sd - bit_words_t<int>(d - i);
                const int nw = (d - 1 - i + 31) >> 5;
                for (int q = 0; q < nw; ++q) c += __popc(rb[off + q]);
            }
            acc[i] = c;
        }
        wave_lds_sync();
        const int nst = (d + 31) >> 5;  // 1 or 2 (a power of two)
        const int G = GL / nst;
        const int c = sub % nst, g = sub / nst;
        uint32_t b8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int imax = min(d - 2, 32 * c + 30);
        for (int i = g; i <= imax; i += G) {
            const int off = sd - bit_words_t<int>(d - i);
            const int nw = (d - 1 - i + 31) >> 5;
            const int o = 32 * c - (i + 1);  // row-i bit of the stripe's first column
            uint32_t w;
            if (o >= 0) {
                const int q = o >> 5;
                const uint32_t lo = q < nw ? rb[off + q] : 0u;
                const uint32_t hi = q + 1 < nw ? rb[off + q + 1] : 0u;
                w = stripe_bits(o, lo, hi);
            } else {
                w = nw > 0 ? rb[off] << (-o) : 0u;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) b8[t] += (w >> t) & 0x01010101u;
        }
        // lanes sub ^ m share the stripe for m = nst, 2 nst, ...; every
        // group takes the same steps (m < nst: another stripe, not added)
#pragma unroll
        for (int m = 1; m < GL; m <<= 1)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t y = __shfl_xor(b8[t], m, GL);
                if (m >= nst) b8[t] += y;
            }
        if (g == 0) {
#pragma unroll
            for (int b = 0; b < 32; ++b) {
                const int j = 32 * c + b;
                const uint32_t v = (b8[b & 7] >> (8 * (b >> 3))) & 0xFFu;
                if (j < d && v) acc[j] += v;  // this lane is the column's only writer
            }
        }
        wave_lds_sync();
        for (int j = sub; j < d; j += GL) {
            const uint32_t v = acc[j];
            if (v) osup[rs + j] += v;  // the group owns row u's slots here
        }
        wave_lds_sync();  // before the next row's counters
    }
}

// Big rows (|N_H(u)| > 64): one wavefront per row u.
//   row sums:    lane i takes rows i, i + 64, ... (its row's words in order);
//   column sums: lane c owns stripe c (columns 32c .. 32c + 31) of a group
//                of 64 stripes and walks the rows in order, so at every row
//                the wavefront reads consecutive words (coalesced) and each
//                word is fetched about once; the stripe's 32 columns sum in
//                6 bit-sliced planes flushed to counters every 63 rows.
// Both sums land in the wavefront's LDS counters and are added to the
// support once.  Rows longer than the LDS counters add to device memory
// with atomics instead.
constexpr int FOLD_RC = 63;  // rows per flush: 6 counter planes hold up to 63

// Rows of up to FOLD_PRIV_D entries (at most 32 stripes, so 64 / stripes
// >= 2 lanes share each stripe) combine the lanes of a stripe through
// private LDS partials: every lane stores its 16 counter words at
// 17 lane + q (17 is odd: the 64 lanes of one store hit 64 banks), then
// each column is summed by the one lane that owns it.  Until the column walk
// is over, the same words hold the first word of each row of B_u (written
// with the row sums), which the walk reads in place of the closed form.
constexpr int FOLD_PRIV_D = 1024;
constexpr int FOLD_PRIV_WORDS = TC_WAVE * 17;
static_assert(FOLD_PRIV_WORDS >= FOLD_PRIV_D, "the row offsets of such a row fit the same words");

// The 6 counter planes of a stripe (counts <= 63) added to 16 words of
// 16-bit counters: word q holds column q (low half) and q + 16 (high
// half).  Each plane is spread to bytes with one shift and one mask per
// plane and byte offset s: byte t of v collects bit s + 8t of every plane
// (bit k of the byte from plane k).
__device__ __forceinline__ void planes_flush16(uint32_t (&pl)[6], uint32_t (&acc)[16]) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const uint32_t x = k >= s ? pl[k] << (k - s) : pl[k] >> (s - k);
            v |= x & (0x01010101u << k);
        }
        acc[s] += v & 0x00FF00FFu;             // columns s, s + 16
        acc[s + 8] += (v >> 8) & 0x00FF00FFu;  // columns s + 8, s + 24
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) pl[k] = 0;
}

// The column walk of one lane: rows g, g + G, ... up to ilast of stripe c,
// 8 rows per step into the planes pl, flush(pl) every 63 rows or fewer and
// once at the end.
template <typename I, bool TAB, typename Flush>
__device__ __forceinline__ void stripe_walk(const uint32_t *__restrict__ rb, I d, I sd, I c,
                                            I g, I G, bool active, I ilast,
                                            const uint32_t *__restrict__ rowoff,
                                            uint32_t (&pl)[6], Flush flush) {
    const I steps = (ilast + G) / G;  // rows per group, rounded up
    int fill = 0;
    for (I tb = 0; tb < steps; tb += 8) {
        uint32_t lo[8], hi[8];
        I oo[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const I i = g + G * (tb + e);
            const I o = 32 * c - (i + 1);  // row bit of the stripe's column 0
            lo[e] = 0u;
            hi[e] = 0u;
            oo[e] = -32;
            if (active && i <= ilast && o > -32) {
                I off;
                if constexpr (TAB) off = (I)rowoff[i];
                else off = sd - bit_words_t<I>(d - i);
                const I nw = (d - 1 - i + 31) >> 5;
                const I q = o < 0 ? 0 : (o >> 5);
                oo[e] = o;
                if (q < nw) lo[e] = rb[off + q];
                if (o >= 0 && q + 1 < nw) hi[e] = rb[off + q + 1];
            }
        }
        uint32_t w[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = oo[e] > -32 ? stripe_bits((int)oo[e], lo[e], hi[e]) : 0u;
        // the 8 rows into the planes by a carry-save tree: pl[0..2] are
        // the ones, twos and fours of every column, and the one eights
        // word of the step ripples into pl[3..5]
        uint32_t t2a, t2b, t4a, t4b, e8;
        csa(pl[0], w[0], w[1], pl[0], t2a);
        csa(pl[0], w[2], w[3], pl[0], t2b);
        csa(pl[1], t2a, t2b, pl[1], t4a);
        csa(pl[0], w[4], w[5], pl[0], t2a);
        csa(pl[0], w[6], w[7], pl[0], t2b);
        csa(pl[1], t2a, t2b, pl[1], t4b);
        csa(pl[2], t4a, t4b, pl[2], e8);
#pragma unroll
        for (int k = 3; k < 6; ++k) {
            const uint32_t tk = pl[k] & e8;
            pl[k] ^= e8;
            e8 = tk;
        }
        fill += 8;
        if (fill > FOLD_RC - 8) {
            flush(pl);
            fill = 0;
        }
    }
    flush(pl);
}

// Row sums of B_u: lane i takes rows i, i + 64, ...; each lands in the LDS
// counter of its slot (or in the support by atomic when not in LDS).  The
// last slot has no row: it starts at 0.
template <typename I>
__device__ __forceinline__ void fold_row_sums(const uint32_t *__restrict__ rb, I d, I sd,
                                              bool in_lds, uint32_t *__restrict__ colc,
                                              uint32_t *__restrict__ rowoff,
                                              uint32_t *__restrict__ sup) {
    for (I i = __lane_id(); i < d; i += TC_WAVE) {
        uint32_t c = 0;
        if (i < d - 1) {
            const I off = sd - bit_words_t<I>(d - i);
            if (rowoff) rowoff[i] = (uint32_t)off;
            const I nw = (d - 1 - i + 31) >> 5;
            // aligned 16-byte loads from the row's first word rounded down:
            // the up to 3 words before the row (inside the buffer, whose
            // base is 16-byte aligned) and after it (inside its padding)
            // are masked
            const uint32_t *p = rb + off;
            const I mis = (I)(((uintptr_t)p >> 2) & 3u);
            const uint4 *pa = reinterpret_cast<const uint4 *>(p - mis);
            const I tot = nw + mis;
            for (I q0 = 0; q0 < tot; q0 += 8) {
                const uint4 v0 = pa[q0 >> 2];
                const uint4 v1 = q0 + 4 < tot ? pa[(q0 >> 2) + 1] : make_uint4(0u, 0u, 0u, 0u);
                const uint32_t x[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    c += q0 + e >= mis && q0 + e < tot ? __popc(x[e]) : 0u;
            }
        }
        if (in_lds) colc[i + (i >> 5)] = c;
        else if (c) atomicAdd(&sup[i], c);
    }
}

// One row u of the big-row fold; rb = B_u's first word, sup = u's supports.
// The LDS counter of column j sits at j + j / 32 (one pad word per 32), so
// lanes that own neighbouring stripes hit different banks.
//
// Column sums: lane (stripe c, row group g) of a group of up to 64 stripes;
// with fewer stripes than lanes the rows are dealt to G = 64 / stripes
// groups (row i to group i mod G), and the lanes of one group read
// consecutive words of one row at every step.
//
// Rows below FOLD_I32_MAX entries (I = int32_t) keep 16-bit counters (no
// column of such a row reaches 2^15) and combine the G lanes of a stripe
// through the private partials; longer rows keep 32 counters per lane and
// add them by atomic.
template <typename I>
__device__ __forceinline__ void fold_big_row(const uint32_t *__restrict__ rb, I d, bool in_lds,
                                             uint32_t *__restrict__ colc,
                                             uint32_t *__restrict__ priv,
                                             uint32_t *__restrict__ sup) {
    const int lane = __lane_id();
    const I sd = bit_words_t<I>(d);
    // rows that combine through the private partials keep their first
    // word's offset in the same LDS words until the walk is over
    uint32_t *rowoff = nullptr;
    if constexpr (sizeof(I) == 4)
        if (in_lds && d <= FOLD_PRIV_D) rowoff = priv;
    fold_row_sums<I>(rb, d, sd, in_lds, colc, rowoff, sup);
    wave_lds_sync();
    const I nst = (d + 31) >> 5;
    for (I sg = 0; sg < nst; sg += TC_WAVE) {
        const I ns = min((I)TC_WAVE, nst - sg);
        const I G = TC_WAVE / ns;
        const I c = sg + lane % ns;
        const I g = lane / ns;
        const bool active = g < G;
        // rows that reach some stripe of the group: i + 1 <= 32 (sg + ns - 1) + 31
        const I ilast = min(d - 2, 32 * (sg + ns) - 2);
        uint32_t pl[6] = {0, 0, 0, 0, 0, 0};
        if constexpr (sizeof(I) == 4) {
            uint32_t acc[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = 0;
            const auto flush16 = [&](uint32_t (&p)[6]) { planes_flush16(p, acc); };
            if (rowoff)
                stripe_walk<I, true>(rb, d, sd, c, g, G, active, ilast, rowoff, pl, flush16);
            else
                stripe_walk<I, false>(rb, d, sd, c, g, G, active, ilast, nullptr, pl, flush16);
            if (in_lds && d <= FOLD_PRIV_D) {
                // one group (sg = 0): partials (over the row offsets, read by
                // every lane before this point), then one owner per column
                wave_lds_sync();
#pragma unroll
                for (int q = 0; q < 16; ++q) priv[17 * lane + q] = acc[q];
                wave_lds_sync();
                for (int u = lane; u < ns * 16; u += TC_WAVE) {
                    const int cl = u >> 4, q = u & 15;
                    uint32_t t = 0;
                    for (int gg = 0; gg < G; ++gg) t += priv[17 * (gg * ns + cl) + q];
                    const int j0 = 32 * cl + q, j1 = j0 + 16;
                    if (j0 < d) colc[j0 + (j0 >> 5)] += t & 0xFFFFu;
                    if (j1 < d) colc[j1 + (j1 >> 5)] += t >> 16;
                }
            } else if (active) {
#pragma unroll
                for (int h = 0; h < 32; ++h) {
                    const I j = 32 * c + h;
                    const uint32_t v = h < 16 ? acc[h] & 0xFFFFu : acc[h - 16] >> 16;
                    if (j < d && v) {
                        if (!in_lds) atomicAdd(&sup[j], v);
                        else if (G == 1) colc[j + (j >> 5)] += v;  // its only owner
                        else atomicAdd(&colc[j + (j >> 5)], v);
                    }
                }
            }
        } else {
            uint32_t cnt[32];
#pragma unroll
            for (int b = 0; b < 32; ++b) cnt[b] = 0;
            stripe_walk<I, false>(rb, d, sd, c, g, G, active, ilast, nullptr, pl,
                                  [&](uint32_t (&p)[6]) { planes_flush(p, cnt); });
            if (active) {
#pragma unroll
                for (int b = 0; b < 32; ++b) {
                    const I j = 32 * c + b;
                    if (j < d && cnt[b]) {
                        if (in_lds) atomicAdd(&colc[j + (j >> 5)], cnt[b]);
                        else atomicAdd(&sup[j], cnt[b]);
                    }
                }
            }
        }
        wave_lds_sync();  // also: the next group's partials overwrite these
    }
    if (in_lds)
        for (I j = lane; j < d; j += TC_WAVE) {
            const uint32_t v = colc[j + (j >> 5)];
            if (v) sup[j] += v;  // the wavefront owns row u's slots here
        }
    wave_lds_sync();  // before the next row's counters
}

// LDS words of one wavefront's column counters for rows up to dcap entries.
__host__ __device__ __forceinline__ size_t fold_colc_words(int dcap) {
    return (size_t)dcap + ((size_t)dcap >> 5) + 1;
}

// Offset of the private partials in a wavefront's LDS words (after the
// counters of the longest row that uses them), and the words per wavefront.
__host__ __device__ __forceinline__ size_t fold_priv_off(int dcap) {
    return fold_colc_words(dcap < FOLD_PRIV_D ? dcap : FOLD_PRIV_D);
}
__host__ __device__ __forceinline__ size_t fold_wave_words(int dcap) {
    const size_t a = fold_colc_words(dcap), b = fold_priv_off(dcap) + FOLD_PRIV_WORDS;
    return a > b ? a : b;
}

// One kernel per index type: rows below i32_max entries (I = int32_t; at
// most FOLD_I32_MAX) or from it up (int64_t); each skips the other's rows of
// the list.
template <typename I>
__global__ __launch_bounds__(256, 4) void k_fold_big(const int32_t *__restrict__ rows, int64_t nrows,
                                                  const int64_t *__restrict__ orp,
                                                  const int64_t *__restrict__ rowbase,
                                                  const uint32_t *__restrict__ bits,
                                                  uint32_t *__restrict__ osup, int dcap,
                                                  int64_t i32_max) {
    extern __shared__ uint32_t colc_all[];
    const int wv = threadIdx.x / TC_WAVE;
    uint32_t *colc = colc_all + (size_t)wv * fold_wave_words(dcap);
    uint32_t *priv = colc + fold_priv_off(dcap);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / TC_WAVE);
    for (int64_t gi = (int64_t)blockIdx.x * (blockDim.x / TC_WAVE) + wv; gi < nrows; gi += waves) {
        // the list is in rank order and the longest rows rank highest: take
        // it from the end so they start first instead of forming the tail
        const int32_t r = rows[nrows - 1 - gi];
        const int64_t rs = orp[r];
        const int64_t d = orp[r + 1] - rs;
        if ((d < i32_max) != (sizeof(I) == 4)) continue;
        fold_big_row<I>(bits + rowbase[r], (I)d, d <= dcap, colc, priv, osup + rs);
    }
}

__global__ void k_dplus_flags(int32_t n, const int64_t *__restrict__ orp, int lo, int hi,
                              uint32_t *__restrict__ f) {
    GRID_STRIDE(r, n) {
        const int64_t d = orp[r + 1] - orp[r];
        f[r] = (d >= lo && d <= hi) ? 1u : 0u;
    }
}

__global__ void k_dplus_write(int32_t n, const int64_t *__restrict__ orp, int lo, int hi,
                              const uint32_t *__restrict__ pos, int32_t *__restrict__ out) {
    GRID_STRIDE(r, n) {
        const int64_t d = orp[r + 1] - orp[r];
        if (d >= lo && d <= hi) out[pos[r]] = (int32_t)r;
    }
}

// Rows with lo <= |N_H| <= hi for the fold, in the same two phases.
struct RowPlan {
    int lo = 2, hi = 0;
    uint32_t *pos = nullptr;
    int64_t count = 0;
    int32_t *rows = nullptr;
};

tc_status rows_count(const tc_graph *g, RowPlan &p, uint32_t *tot, tc_scratch &keep,
                     hipStream_t s) {
    const int32_t n = g->n;
    TC_TRY(keep.get(&p.pos, n));
    k_dplus_flags<<<grid_for(n), BK, 0, s>>>(n, g->orp, p.lo, p.hi, p.pos);
    TC_LAUNCHED();
    return tc_scan_u32(p.pos, p.pos, n, tot, s);
}

tc_status rows_write(const tc_graph *g, RowPlan &p, tc_scratch &keep, hipStream_t s) {
    TC_TRY(keep.get(&p.rows, p.count));
    if (p.count > 0) {
        k_dplus_write<<<grid_for(g->n), BK, 0, s>>>(g->n, g->orp, p.lo, p.hi, p.pos, p.rows);
        TC_LAUNCHED();
    }
    return TC_OK;
}

// The bit rows of the pairs whose pivot has no higher neighbours: no count
// kernel scans them (nothing can close), so they are cleared here.  Every
// other pair's row is written whole by the kernel that scans it, so no
// other word needs clearing.  One wavefront per item, a lane per pair.
__global__ void k_zero_rows(const uint4 *__restrict__ rowinfo, const uint64_t *__restrict__ in_pair,
                            const int64_t *__restrict__ in_ptr, const int32_t *__restrict__ item_v,
                            const uint32_t *__restrict__ item_first, int64_t nitems, int S,
                            uint32_t *__restrict__ bits) {
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    for (int64_t it = (int64_t)blockIdx.x * wpb + wv; it < nitems; it += (int64_t)gridDim.x * wpb) {
        const int32_t v = item_v[it];
        const int64_t first = item_first[it];
        const int64_t pend = min(first + (int64_t)S, in_ptr[v + 1]);
        for (int64_t i = first + lane; i < pend; i += TC_WAVE) {
            const uint64_t pr = in_pair[i];
            const int64_t k = (int64_t)(uint32_t)pr;
            const uint4 ri = rowinfo[(int32_t)(pr >> 32)];
            const int64_t d = (int64_t)ri.w - ri.z;
            const int64_t ii = k - ri.z;
            const int64_t words = (d - 1 - ii + 31) >> 5;
            const int64_t gb = (int64_t)(((uint64_t)ri.y << 32) | ri.x) + bit_words(d) -
                               bit_words(d - ii);
            for (int64_t w = 0; w < words; ++w) bits[gb + w] = 0u;
        }
    }
}

__global__ void k_row_words(int32_t n, const int64_t *__restrict__ orp, int64_t *__restrict__ out) {
    GRID_STRIDE(r, n) out[r] = bit_words(orp[r + 1] - orp[r]);
}

// Σ_r bit_words(|N_H(r)|): the words of every row's bit matrix.
__global__ void k_row_words_total(int32_t n, const int64_t *__restrict__ orp,
                                  unsigned long long *__restrict__ total) {
    unsigned long long acc = 0;
    GRID_STRIDE(r, n) acc += (unsigned long long)bit_words(orp[r + 1] - orp[r]);
    acc = tc_wave_sum(acc);
    if (__lane_id() == 0 && acc) atomicAdd(total, acc);
}

// Work per bin for the statistics: scan lengths of every pair, binned by
// the pivot's |N_H|.
__global__ void k_mid_stats(int64_t m, const int64_t *__restrict__ orp,
                            const int32_t *__restrict__ ocol, const uint64_t *__restrict__ in_pair,
                            int light_max, int huge_min, int32_t r16,
                            unsigned long long *__restrict__ acc) {
    // cand per bin, pairs per bin, heavy cand and pairs of pivots among the
    // top 2^16 ranks
    unsigned long long sums[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_STRIDE(i, m) {
        const uint64_t pr = in_pair[i];
        const uint32_t k = (uint32_t)pr;
        const int32_t u = (int32_t)(pr >> 32);
        const int32_t v = ocol[k];
        const int64_t d = orp[v + 1] - orp[v];
        const int64_t len = orp[u + 1] - (int64_t)k - 1;
        if (d < 1) continue;
        const int bin = d <= light_max ? 0 : (d < huge_min ? 1 : 2);
        sums[bin] += (unsigned long long)len;
        sums[3 + bin] += 1ull;
        if (bin == 1 && v >= r16) {
            sums[6] += (unsigned long long)len;
            sums[7] += 1ull;
        }
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const unsigned long long v = tc_wave_sum(sums[b]);
        if (__lane_id() == 0 && v) atomicAdd(&acc[b < 3 ? 3 + b : (b < 6 ? 5 + b : 6 + b)], v);
    }
}

__global__ void k_mid_pivots(int32_t n, const int64_t *__restrict__ orp,
                             const int64_t *__restrict__ in_ptr, int light_max, int huge_min,
                             int32_t r16, unsigned long long *__restrict__ acc) {
    // per-thread bin counts (and heavy pivots among the top 2^16 ranks),
    // summed over the wavefront: four atomics per wavefront instead of one
    // per pivot on the same four words
    unsigned long long c[4] = {0, 0, 0, 0};
    GRID_STRIDE(v, n) {
        const int64_t d = orp[v + 1] - orp[v];
        if (d < 1 || in_ptr[v + 1] == in_ptr[v]) continue;
        const int bin = d <= light_max ? 0 : (d < huge_min ? 1 : 2);
        c[0] += bin == 0;
        c[1] += bin == 1;
        c[2] += bin == 2;
        c[3] += bin == 1 && v >= r16;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const unsigned long long t = tc_wave_sum(c[b]);
        if (__lane_id() == 0 && t) atomicAdd(&acc[b < 3 ? b : 14], t);
    }
}

// Work-item lists are built in two phases so that one read-back serves all
// of them: count (per-pivot item counts and their scan; the total stays on
// the device), then, with the totals on the host, allocate and write.
struct ItemPlan {
    int lo = 1, hi = 0, S = 64, sel = 0;
    int64_t span_max = 0, pairs_min = 0;
    int32_t rlo = 0, rhi = 0x7FFFFFFF;  // pivot ranks [rlo, rhi)
    uint32_t *cnt = nullptr, *off = nullptr;
    int64_t count = 0;
    int32_t *item_v = nullptr;
    uint32_t *item_first = nullptr;
};

tc_status plan_count(const tc_graph *g, ItemPlan &p, uint32_t *tot, tc_scratch &keep,
                     hipStream_t s) {
    const int32_t n = g->n;
    TC_TRY(keep.get(&p.cnt, n));
    TC_TRY(keep.get(&p.off, n));
    k_item_count<<<grid_for(n), BK, 0, s>>>(n, g->orp, g->ocol, g->in_ptr, p.lo, p.hi, p.S, p.sel,
                                            p.span_max, p.pairs_min, p.rlo, p.rhi, p.cnt);
    TC_LAUNCHED();
    return tc_scan_u32(p.cnt, p.off, n, tot, s);
}

tc_status plan_write(const tc_graph *g, ItemPlan &p, tc_scratch &keep, hipStream_t s) {
    TC_TRY(keep.get(&p.item_v, p.count));
    TC_TRY(keep.get(&p.item_first, p.count));
    if (p.count > 0) {
        k_item_write<<<grid_for(g->n), BK, 0, s>>>(g->n, p.cnt, p.off, g->in_ptr, p.S, p.item_v,
                                                  p.item_first);
        TC_LAUNCHED();
    }
    return TC_OK;
}

}  // namespace

// Builds in_ptr / in_pair (the transposed orientation) once per handle.
static tc_status bit_rows_prepare(tc_graph *g, hipStream_t s);

tc_status tc_mid_prepare(tc_graph *g, hipStream_t s) {
    // the order by larger id is not needed from here on (the symmetric
    // fill sorts again if it is ever asked for)
    tc_release_transposition(g, s);
    if (g->in_pair) return bit_rows_prepare(g, s);
    const int32_t n = g->n;
    const int64_t m = g->m;
    const int64_t nn = n > 0 ? n : 1;
    TC_TRY(tc_graph_alloc(g, &g->in_ptr, nn + 1, s));
    TC_TRY(tc_graph_alloc(g, &g->in_pair, m, s));
    tc_scratch tmp(s);
    int64_t *len = nullptr;
    TC_TRY(tmp.get(&len, nn));
    if (m > 0) {
        // (row << 32 | slot) of every slot, in order of the pivot (stable:
        // by row within a pivot)
        uint32_t *key = nullptr, *key2 = nullptr;
        uint64_t *val2 = nullptr;
        TC_TRY(tmp.get(&key, m));
        TC_TRY(tmp.get(&key2, m));
        TC_TRY(tmp.get(&val2, m));
        uint64_t *val = g->in_pair;
        TC_TRY(tc_sort_u32_index_hi((const uint32_t *)g->ocol, (const uint32_t *)g->orow, &key, &val,
                                    &key2, &val2, m, g->bits, s));
        if (val != g->in_pair) {  // the result is in the scratch buffer: swap ownership
            tmp.exchange(val, g->in_pair);
            g->in_pair = val;
        }
    }
    if (n > 0) {
        k_in_len<<<grid_for(n), BK, 0, s>>>(n, g->perm, g->row_ptr, g->orp, len);
        TC_LAUNCHED();
        TC_TRY(tc_scan_i64(len, g->in_ptr, n, g->in_ptr + n, s));
    } else {
        TC_HIP(hipMemsetAsync(g->in_ptr, 0, sizeof(int64_t), s));
    }
    return bit_rows_prepare(g, s);
}

// Per row: its bit matrix's first word (low, high), its start and end in
// ocol (below 2^32: the slots number m).
__global__ void k_row_info(int32_t n, const int64_t *__restrict__ orp,
                           const int64_t *__restrict__ rowbase, uint4 *__restrict__ ri) {
    GRID_STRIDE(r, n) {
        const uint64_t b = (uint64_t)rowbase[r];
        ri[r] = make_uint4((uint32_t)b, (uint32_t)(b >> 32), (uint32_t)orp[r], (uint32_t)orp[r + 1]);
    }
}

// Bit matrices: rowbase = exclusive scan of each row's word count.
static tc_status bit_rows_prepare(tc_graph *g, hipStream_t s) {
    if (g->rowbase) return TC_OK;
    const int32_t n = g->n;
    const int64_t nn = n > 0 ? n : 1;
    tc_scratch tmp(s);
    int64_t *len = nullptr;
    TC_TRY(tmp.get(&len, nn));
    TC_TRY(tc_graph_alloc(g, &g->rowbase, nn + 1, s));
    k_row_words<<<grid_for(n), BK, 0, s>>>(n, g->orp, len);
    TC_LAUNCHED();
    TC_TRY(tc_scan_i64(len, g->rowbase, n, g->rowbase + n, s));
    int64_t words = 0;
    TC_HIP(hipMemcpyAsync(&words, g->rowbase + n, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    g->bit_words = words;
    // 4 words of padding: the fold's row sums read up to 3 words past a
    // row's end
    TC_TRY(tc_graph_alloc(g, &g->hitbits, words + 4, s));
    TC_TRY(tc_graph_alloc(g, &g->rowinfo, nn, s));
    if (n > 0) {
        k_row_info<<<grid_for(n), BK, 0, s>>>(n, g->orp, g->rowbase, g->rowinfo);
        TC_LAUNCHED();
    }
    return TC_OK;
}

// The 16-bit copy of ocol for the pivots among the top 2^16 ranks (once per
// handle): every entry after such a pivot in a row is a rank in
// [rank16_base, n), below 2^16 once rank16_base is taken off.
static tc_status ocol16_prepare(tc_graph *g, hipStream_t s) {
    if (g->ocol16) return TC_OK;
    g->rank16_base = g->n > 65536 ? g->n - 65536 : 0;
    const int64_t total = (g->m + TC_OCOL_PAD + 1) & ~(int64_t)1;
    TC_TRY(tc_graph_alloc(g, &g->ocol16, total, s));
    k_ocol16<<<grid_for(total / 2), BK, 0, s>>>(total / 2, g->m, g->ocol, g->rank16_base,
                                               reinterpret_cast<uint32_t *>(g->ocol16));
    TC_LAUNCHED();
    return TC_OK;
}

tc_status tc_count_mid(tc_graph *g, const tc_tuning &t, int lds_limit, int max_entries,
                       unsigned long long *found, hipStream_t s) {
    TC_TRY(tc_mid_prepare(g, s));
    TC_TRY(ocol16_prepare(g, s));
    const int light_max = t.light_max_dplus;
    int huge_min = max_entries / 2 + 1;
    if (huge_min <= light_max) huge_min = light_max + 1;
    g->light_max = light_max;
    g->huge_min = huge_min;

    int wpb_block = t.heavy_block / TC_WAVE;
    const int wave_pairs = t.item_pairs;
    const int block_pairs = t.item_pairs * wpb_block;
    tc_scratch items(s);
    // workgroup pivots whose rank span fits the LDS bitmap use it; the
    // others hash (or, above huge_min, search device memory).  Wavefront
    // pivots with at least light_bitmap_pairs pairs and a span that fits go
    // to the bitmap kernel too (enough pairs to pay for building it).
    const int bw = t.bitmap_words;
    const int64_t span_max = 32 * (int64_t)bw;
    const int split = bw > 0 ? 1 : 0;
    const int lsplit = (bw > 0 && t.light_bitmap_pairs > 0) ? 1 : 0;
    // wavefront pivots with rows of at most GROUP_DMAX entries run
    // 64 / GROUP_LANES to a wavefront, in items of at most GROUP_PAIRS pairs
    const int gmax = light_max < GROUP_DMAX ? light_max : GROUP_DMAX;
    const int group_pairs = wave_pairs < GROUP_PAIRS ? wave_pairs : GROUP_PAIRS;
    enum { P_GROUP, P_WAVE, P_LBITMAP, P_BITMAP16, P_BITMAP, P_BLOCK, P_HUGE, P_ZERO, NPLANS };
    ItemPlan pl[NPLANS];
    pl[P_GROUP] = {1, gmax, group_pairs, 2 * lsplit, span_max, t.light_bitmap_pairs};
    pl[P_WAVE] = {gmax + 1, light_max, wave_pairs, 2 * lsplit, span_max, t.light_bitmap_pairs};
    pl[P_LBITMAP] = {1, lsplit ? light_max : 0, block_pairs, 1, span_max, t.light_bitmap_pairs};
    // workgroup pivots among the top 2^16 ranks take the 2048-word bitmap
    // over 16-bit values whatever their span (when the tuning allows that
    // many words), in a launch of their own whose smaller LDS footprint
    // keeps more wavefronts resident; the others take the span bitmap or
    // hash
    const int32_t r16s = bw >= BITMAP16_WORDS ? g->rank16_base : 0x7FFFFFFF;
    pl[P_BITMAP16] = {light_max + 1, huge_min - 1, block_pairs, 0, 0, 0, r16s, 0x7FFFFFFF};
    pl[P_BITMAP] = {light_max + 1, split ? huge_min - 1 : light_max, block_pairs, 1, span_max, 0,
                    0, r16s};
    pl[P_BLOCK] = {light_max + 1, huge_min - 1, block_pairs, 2 * split, span_max, 0, 0, r16s};
    pl[P_HUGE] = {huge_min, 0x7FFFFFFF, block_pairs, 0, 0, 0};
    // pivots with an empty row: their pairs' bit rows are only cleared
    pl[P_ZERO] = {0, 0, wave_pairs, 0, 0, 0};
    RowPlan rp[2];
    rp[0].lo = 2;
    rp[0].hi = 64;
    rp[1].lo = 65;
    rp[1].hi = 0x7FFFFFFF;
    uint32_t *tots = nullptr;
    TC_TRY(items.get(&tots, NPLANS + 2));
    for (int i = 0; i < NPLANS; ++i) TC_TRY(plan_count(g, pl[i], tots + i, items, s));
    if (g->bit_words > 0)
        for (int i = 0; i < 2; ++i) TC_TRY(rows_count(g, rp[i], tots + NPLANS + i, items, s));
    uint32_t h_tots[NPLANS + 2] = {};
    TC_HIP(hipMemcpyAsync(h_tots, tots, sizeof(h_tots), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < NPLANS; ++i) {
        pl[i].count = h_tots[i];
        TC_TRY(plan_write(g, pl[i], items, s));
    }
    if (g->bit_words > 0)
        for (int i = 0; i < 2; ++i) {
            rp[i].count = h_tots[NPLANS + i];
            TC_TRY(rows_write(g, rp[i], items, s));
        }
    const int64_t n_group = pl[P_GROUP].count;
    const int64_t n_wave = pl[P_WAVE].count, n_lbitmap = pl[P_LBITMAP].count;
    const int64_t n_bitmap = pl[P_BITMAP].count, n_block = pl[P_BLOCK].count;
    const int64_t n_bitmap16 = pl[P_BITMAP16].count;
    const int64_t n_huge = pl[P_HUGE].count;
    int32_t *wv_v = pl[P_WAVE].item_v, *lb_v = pl[P_LBITMAP].item_v, *bm_v = pl[P_BITMAP].item_v;
    int32_t *bl_v = pl[P_BLOCK].item_v, *hu_v = pl[P_HUGE].item_v;
    uint32_t *wv_f = pl[P_WAVE].item_first, *lb_f = pl[P_LBITMAP].item_first;
    uint32_t *bm_f = pl[P_BITMAP].item_first, *bl_f = pl[P_BLOCK].item_first;
    uint32_t *hu_f = pl[P_HUGE].item_first;
    g->n_light = n_group + n_wave + n_lbitmap;
    g->n_heavy = n_block + n_bitmap + n_bitmap16;
    g->n_huge = n_huge;
    // pairs whose pivot closes nothing are never scanned: their rows are
    // cleared, and every other word is written by the count
    if (pl[P_ZERO].count > 0) {
        int64_t zb = tc_div_up(pl[P_ZERO].count, BK / TC_WAVE);
        k_zero_rows<<<(unsigned)(zb < 262144 ? zb : 262144), BK, 0, s>>>(
            g->rowinfo, g->in_pair, g->in_ptr, pl[P_ZERO].item_v, pl[P_ZERO].item_first,
            pl[P_ZERO].count, wave_pairs, g->hitbits);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 5, s);

    if (n_group > 0) {
        const int gpb = 256 / GROUP_LANES;
        int64_t blocks = tc_div_up(n_group, gpb);
        if (blocks > 262144) blocks = 262144;
        k_mid_groups<GROUP_LANES><<<(unsigned)blocks, 256, (size_t)gpb * mid_group_bytes(gmax, GROUP_LANES), s>>>(
            g->orp, g->ocol, g->in_ptr, g->in_pair, g->rowinfo, g->hitbits, pl[P_GROUP].item_v,
            pl[P_GROUP].item_first, n_group, gmax, group_pairs, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 12, s);
    if (n_wave > 0) {
        const size_t per_wave = mid_wave_bytes(light_max);
        int wpb = t.light_block / TC_WAVE;
        while (wpb > 1 && (size_t)wpb * per_wave > (size_t)lds_limit) --wpb;
        int64_t blocks = tc_div_up(n_wave, wpb);
        if (blocks > 262144) blocks = 262144;
        k_mid_wave<<<(unsigned)blocks, wpb * TC_WAVE, (size_t)wpb * per_wave, s>>>(
            g->orp, g->ocol, g->in_ptr, g->in_pair, g->rowinfo, g->hitbits, wv_v, wv_f, n_wave,
            light_max, wave_pairs, g->ocol16, g->rank16_base, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 13, s);
    if (n_lbitmap > 0) {
        const size_t lds = mid_block_bytes(light_max, wpb_block, LK_BITMAP, bw);
        int64_t blocks = n_lbitmap < 1048576 ? n_lbitmap : 1048576;
        k_mid_block<LK_BITMAP><<<(unsigned)blocks, wpb_block * TC_WAVE, lds, s>>>(
            g->orp, g->ocol, g->in_ptr, g->in_pair, g->rowinfo, g->hitbits, lb_v, lb_f, n_lbitmap,
            light_max, block_pairs, bw, g->ocol16, g->rank16_base, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 6, s);
    if (n_bitmap16 > 0) {
        const int hmax = g->max_dplus < huge_min - 1 ? g->max_dplus : huge_min - 1;
        const size_t lds = mid_block16_bytes(hmax);
        int64_t blocks = n_bitmap16 < 1048576 ? n_bitmap16 : 1048576;
        k_mid_block16<<<(unsigned)blocks, wpb_block * TC_WAVE, lds, s>>>(
            g->orp, g->ocol, g->in_ptr, g->in_pair, g->rowinfo, g->hitbits, pl[P_BITMAP16].item_v,
            pl[P_BITMAP16].item_first, n_bitmap16, hmax, block_pairs, g->ocol16, g->rank16_base,
            g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 14, s);
    if (n_bitmap > 0) {
        const int hmax = g->max_dplus < huge_min - 1 ? g->max_dplus : huge_min - 1;
        const size_t lds = mid_block_bytes(hmax, wpb_block, LK_BITMAP, bw);
        int64_t blocks = n_bitmap < 1048576 ? n_bitmap : 1048576;
        k_mid_block<LK_BITMAP><<<(unsigned)blocks, wpb_block * TC_WAVE, lds, s>>>(
            g->orp, g->ocol, g->in_ptr, g->in_pair, g->rowinfo, g->hitbits, bm_v, bm_f, n_bitmap,
            hmax, block_pairs, bw, g->ocol16, g->rank16_base, g->osup, found);
        TC_LAUNCHED();
    }
    if (n_block > 0) {
        const int hmax = g->max_dplus < huge_min - 1 ? g->max_dplus : huge_min - 1;
        const size_t lds = mid_block_bytes(hmax, wpb_block, LK_HASH, 0);
        int64_t blocks = n_block < 1048576 ? n_block : 1048576;
        k_mid_block<LK_HASH><<<(unsigned)blocks, wpb_block * TC_WAVE, lds, s>>>(
            g->orp, g->ocol, g->in_ptr, g->in_pair, g->rowinfo, g->hitbits, bl_v, bl_f, n_block, hmax,
            block_pairs, 0, g->ocol16, g->rank16_base, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 7, s);
    if (n_huge > 0) {
        const size_t lds = mid_block_bytes(0, wpb_block, LK_GLOBAL, 0);
        int64_t blocks = n_huge < 1048576 ? n_huge : 1048576;
        k_mid_block<LK_GLOBAL><<<(unsigned)blocks, wpb_block * TC_WAVE, lds, s>>>(
            g->orp, g->ocol, g->in_ptr, g->in_pair, g->rowinfo, g->hitbits, hu_v, hu_f, n_huge, 0,
            block_pairs, 0, g->ocol16, g->rank16_base, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 8, s);
    if (g->bit_words > 0) {
        int32_t *small = rp[0].rows, *big = rp[1].rows;
        const int64_t ns = rp[0].count, nb = rp[1].count;
        if (ns > 0) {
            int64_t fb = tc_div_up(ns, BK / 16);
            k_fold<16><<<(unsigned)(fb < 1048576 ? fb : 1048576), BK, 0, s>>>(
                small, ns, g->orp, g->rowbase, g->hitbits, g->osup);
            TC_LAUNCHED();
        }
        if (nb > 0) {
            int64_t fb = tc_div_up(nb, BK / TC_WAVE);
            // LDS counters for rows up to 7936 entries: 4 wavefronts x
            // fold_wave_words(7936) words stay within 128 KB
            int dcap = g->max_dplus < 7936 ? g->max_dplus : 7936;
            dcap = (dcap + 3) & ~3;
            // TC_FOLD_I32_MAX (environment) lowers the row length from which
            // the 64-bit kernel folds, so that its path can be exercised on
            // small graphs
            int64_t i32_max = FOLD_I32_MAX;
            if (const char *ev = getenv("TC_FOLD_I32_MAX")) {
                const long v = strtol(ev, nullptr, 10);
                if (v >= 0 && v < FOLD_I32_MAX) i32_max = v;
            }
            const size_t lds = (size_t)(BK / TC_WAVE) * fold_wave_words(dcap) * sizeof(uint32_t);
            k_fold_big<int32_t><<<(unsigned)(fb < 1048576 ? fb : 1048576), BK, lds, s>>>(
                big, nb, g->orp, g->rowbase, g->hitbits, g->osup, dcap, i32_max);
            TC_LAUNCHED();
            if (g->max_dplus >= i32_max) {
                k_fold_big<int64_t><<<(unsigned)(fb < 1048576 ? fb : 1048576), BK, lds, s>>>(
                    big, nb, g->orp, g->rowbase, g->hitbits, g->osup, dcap, i32_max);
                TC_LAUNCHED();
            }
        }
    }
    tc_prof_mark(g, 9, s);
    return TC_OK;
}

tc_status tc_mid_stats(tc_graph *g, unsigned long long *acc, hipStream_t s) {
    TC_TRY(tc_mid_prepare(g, s));
    const int light_max = g->light_max > 0 ? g->light_max : 64;
    const int huge_min = g->huge_min > 0 ? g->huge_min : 0x7FFFFFFF;
    const int32_t r16 = g->n > 65536 ? g->n - 65536 : 0;  // as the count's 16-bit copy
    // a bounded grid: each wavefront adds its sums to the same few words
    const unsigned sg = grid_for(g->m) < 4096u ? grid_for(g->m) : 4096u;
    k_mid_stats<<<sg, BK, 0, s>>>(g->m, g->orp, g->ocol, g->in_pair, light_max,
                                             huge_min, r16, acc);
    TC_LAUNCHED();
    const unsigned pg = grid_for(g->n) < 4096u ? grid_for(g->n) : 4096u;
    k_mid_pivots<<<pg, BK, 0, s>>>(g->n, g->orp, g->in_ptr, light_max, huge_min, r16, acc);
    TC_LAUNCHED();
    return TC_OK;
}

tc_status tc_mid_bit_words(const tc_graph *g, int64_t *words, hipStream_t s) {
    if (g->rowbase) {
        *words = g->bit_words;
        return TC_OK;
    }
    tc_scratch tmp(s);
    unsigned long long *d = nullptr;
    TC_TRY(tmp.get(&d, 1));
    TC_HIP(hipMemsetAsync(d, 0, 8, s));
    if (g->n > 0) {
        k_row_words_total<<<grid_for(g->n), BK, 0, s>>>(g->n, g->orp, d);
        TC_LAUNCHED();
    }
    unsigned long long h = 0;
    TC_HIP(hipMemcpyAsync(&h, d, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    *words = (int64_t)h;
    return TC_OK;
}
