// Triangle counting with per-edge support on the degree-ordered orientation.
//
// In rank space every triangle is v < u < w with u, w ∈ N_H(v) and
// w ∈ N_H(u); it is found exactly once, from row v, while intersecting
// N_H(v) with N_H(u) (the appendix's alternative TriangleNeighbor
// procedure: only the low and middle vertices' higher-ordered sets are
// intersected, only the high vertex is ever returned).  For each common w
// at index l of N_H(v) and index r of N_H(u), the procedure marks L_v(l)
// and L_u(r), and marks L_v(i) for u's own index i if anything was found;
// here each mark is a count instead, so the slot ends holding the number
// of triangles on its edge (the value of T = A² ∘ A there):
//     sup(v,w) += 1,   sup(u,w) += 1,   sup(v,u) += |N_H(v) ∩ N_H(u)|.
//
// MI355X mapping.  Row v's set N_H(v) is put into an LDS hash table (key =
// rank, value = index in the row); the wavefront streams N_H(u) for each u
// of the row with coalesced 64-wide loads and probes the table, so the
// candidate stream is Σ_{u ∈ N_H(v)} |N_H(u)| reads.  sup(v,·) accumulates
// in LDS and is flushed once per slot; sup(u,w) is one global atomic per
// triangle; sup(v,u) is a ballot/popcount reduction.  Streaming of N_H(u)
// stops at the first entry above max N_H(v), since both lists are sorted.
//
// Rows are binned by d+ = |N_H(v)|: rows with d+ < 2 close no triangle;
// "light" rows (d+ <= light_max_dplus) get one wavefront each; "heavy"
// rows a workgroup sharing one table; "huge" rows (table larger than the
// LDS budget) probe by binary search in device memory.  The schedule never
// changes a result: every count is an integer sum.
#include "tc_internal.h"
#include "tc_table.h"

namespace {

constexpr int BK = 256;
constexpr int UNROLL = 4;  // independent candidate loads in flight per lane
// TC_ALGO_AUTO takes the middle pivot from AUTO_MID_MIN_EDGES edges when
// the orientation has a row of AUTO_MID_MIN_DPLUS entries or more (degree
// skew), and from AUTO_MID_MIN_EDGES_FLAT edges otherwise
constexpr int64_t AUTO_MID_MIN_EDGES = 600000;
constexpr int64_t AUTO_MID_MIN_EDGES_FLAT = 3000000;
constexpr int AUTO_MID_MIN_DPLUS = 32;
using namespace tc_tab;

static inline unsigned grid_for(int64_t n, int block = BK) {
    int64_t g = tc_div_up(n, block);
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (unsigned)g;
}

// Streams N_H(u) = ocol[ub, ue) against row v and applies the support
// updates; returns |N_H(v) ∩ N_H(u)| (wave-uniform).  Each lane keeps
// UNROLL loads in flight; the stream stops once it passes vmax = max N_H(v).
template <bool GLOBAL_LOOKUP>
__device__ __forceinline__ uint32_t stream_u(const int32_t *__restrict__ ocol, int64_t ub,
                                             int64_t ue, uint32_t vmax, const RowTable &t,
                                             uint32_t *lsup, int64_t vstart, int dv,
                                             uint32_t *__restrict__ osup) {
    const int lane = __lane_id();
    uint32_t c = 0;
    for (int64_t jb = ub; jb < ue; jb += TC_WAVE * UNROLL) {
        uint32_t w[UNROLL];
#pragma unroll
        for (int q = 0; q < UNROLL; ++q) {
            const int64_t j = jb + q * TC_WAVE + lane;
            w[q] = j < ue ? (uint32_t)ocol[j] : EMPTY;
        }
        // lane 0's first load is the smallest candidate of the chunk
        if ((uint32_t)__shfl(w[0], 0, TC_WAVE) > vmax) break;
        // EMPTY (past the row end) is above every rank: never looked up
        int pq[UNROLL];
        if constexpr (GLOBAL_LOOKUP) {
#pragma unroll
            for (int q = 0; q < UNROLL; ++q)
                pq[q] = w[q] <= vmax ? row_search(ocol, vstart, dv, w[q]) : -1;
        } else {
            table_find_n<UNROLL>(t, w, vmax, pq);
        }
#pragma unroll
        for (int q = 0; q < UNROLL; ++q) {
            const int p = pq[q];
            const bool hit = p >= 0;
            if (hit) {
                if constexpr (GLOBAL_LOOKUP) atomicAdd(&osup[vstart + p], 1u);
                else atomicAdd(&lsup[p], 1u);
                atomicAdd(&osup[jb + q * TC_WAVE + lane], 1u);
            }
            c += (uint32_t)__popcll(__ballot(hit));
        }
        if ((uint32_t)__shfl(w[UNROLL - 1], TC_WAVE - 1, TC_WAVE) > vmax) break;
    }
    return c;
}

// Per-wave LDS footprint of the light kernel (bytes, 16-aligned).
__host__ __device__ __forceinline__ size_t light_wave_bytes(int dcap) {
    const size_t nb = (size_t)1 << bucket_bits(dcap);
    return (16 * nb + 2 * 4 * nb + 4 * (size_t)dcap + 15) & ~(size_t)15;
}

// One wavefront per light row.
__global__ __launch_bounds__(1024) void k_count_light(const int64_t *__restrict__ orp,
                                                      const int32_t *__restrict__ ocol,
                                                      const int32_t *__restrict__ rows,
                                                      int64_t nrows, int dcap,
                                                      uint32_t *__restrict__ osup,
                                                      unsigned long long *__restrict__ tri_total) {
    extern __shared__ uint4 lds4[];
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    const int nbmax = 1 << bucket_bits(dcap);
    char *base = reinterpret_cast<char *>(lds4) + (size_t)wv * light_wave_bytes(dcap);
    uint32_t *keys = reinterpret_cast<uint32_t *>(base);
    uint16_t *pos = reinterpret_cast<uint16_t *>(base + 16 * (size_t)nbmax);
    uint32_t *lsup = reinterpret_cast<uint32_t *>(base + 24 * (size_t)nbmax);
    unsigned long long found = 0;
    for (int64_t ri = (int64_t)blockIdx.x * wpb + wv; ri < nrows; ri += (int64_t)gridDim.x * wpb) {
        const int32_t r = rows[ri];
        const int64_t start = orp[r];
        const int d = (int)(orp[r + 1] - start);
        const RowTable t{keys, pos, bucket_bits(d)};
        for (int j = lane; j < (4 << t.bb); j += TC_WAVE) keys[j] = EMPTY;
        for (int j = lane; j < d; j += TC_WAVE) lsup[j] = 0;
        for (int j = lane; j < d; j += TC_WAVE) table_insert(t, (uint32_t)ocol[start + j], j);
        const uint32_t vmax = (uint32_t)ocol[start + d - 1];
        for (int i0 = 0; i0 < d - 1; i0 += TC_WAVE) {
            const int ii = i0 + lane;
            int64_t ub_l = 0, ue_l = 0;
            if (ii < d - 1) {
                const int32_t u = ocol[start + ii];
                ub_l = orp[u];
                ue_l = orp[u + 1];
            }
            const int cnt = min(TC_WAVE, d - 1 - i0);
            for (int k = 0; k < cnt; ++k) {
                const int64_t ub = __shfl(ub_l, k, TC_WAVE), ue = __shfl(ue_l, k, TC_WAVE);
                const uint32_t c = stream_u<false>(ocol, ub, ue, vmax, t, lsup, start, d, osup);
                if (c != 0 && lane == 0) atomicAdd(&lsup[i0 + k], c);
                found += c;
            }
        }
        for (int j = lane; j < d; j += TC_WAVE) {
            const uint32_t x = lsup[j];
            if (x) atomicAdd(&osup[start + j], x);
        }
    }
    if (lane == 0 && found) atomicAdd(tri_total, found);
}

// LDS footprint of the heavy kernel for rows of at most dmax entries.
static inline size_t heavy_bytes(int dmax) {
    const size_t nb = (size_t)1 << bucket_bits(dmax);
    return 16 * nb + 8 * nb + 4 * (size_t)dmax;
}

// One workgroup per heavy row (GLOBAL_LOOKUP: no table, binary search in
// device memory, for rows whose table would not fit).  Wavefront wv takes
// the row's u at indices wv, wv + wpb, wv + 2·wpb, ...; rows are taken from
// the end of the list (highest rank, typically the most work) first.
template <bool GLOBAL_LOOKUP>
__global__ __launch_bounds__(1024) void k_count_heavy(const int64_t *__restrict__ orp,
                                                      const int32_t *__restrict__ ocol,
                                                      const int32_t *__restrict__ rows,
                                                      int64_t nrows, int dmax,
                                                      uint32_t *__restrict__ osup,
                                                      unsigned long long *__restrict__ tri_total) {
    extern __shared__ uint4 lds4[];
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    const int nbmax = GLOBAL_LOOKUP ? 0 : (1 << bucket_bits(dmax));
    char *base = reinterpret_cast<char *>(lds4);
    uint32_t *keys = reinterpret_cast<uint32_t *>(base);
    uint16_t *pos = reinterpret_cast<uint16_t *>(base + 16 * (size_t)nbmax);
    uint32_t *lsup = reinterpret_cast<uint32_t *>(base + 24 * (size_t)nbmax);
    unsigned long long found = 0;
    for (int64_t bi = blockIdx.x; bi < nrows; bi += gridDim.x) {
        const int32_t r = rows[nrows - 1 - bi];
        const int64_t start = orp[r];
        const int d = (int)(orp[r + 1] - start);
        RowTable t{keys, pos, 0};
        if constexpr (!GLOBAL_LOOKUP) {
            t.bb = bucket_bits(d);
            for (int j = threadIdx.x; j < (4 << t.bb); j += blockDim.x) keys[j] = EMPTY;
            for (int j = threadIdx.x; j < d; j += blockDim.x) lsup[j] = 0;
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += blockDim.x)
                table_insert(t, (uint32_t)ocol[start + j], j);
            __syncthreads();
        }
        const uint32_t vmax = (uint32_t)ocol[start + d - 1];
        const int nu = d - 1;  // the last entry closes no triangle in this row
        for (int k0 = 0; wv + wpb * k0 < nu; k0 += TC_WAVE) {
            const int ii = wv + wpb * (k0 + lane);
            int64_t ub_l = 0, ue_l = 0;
            if (ii < nu) {
                const int32_t u = ocol[start + ii];
                ub_l = orp[u];
                ue_l = orp[u + 1];
            }
            for (int k = 0; k < TC_WAVE; ++k) {
                const int i = wv + wpb * (k0 + k);
                if (i >= nu) break;
                const int64_t ub = __shfl(ub_l, k, TC_WAVE), ue = __shfl(ue_l, k, TC_WAVE);
                const uint32_t c =
                    stream_u<GLOBAL_LOOKUP>(ocol, ub, ue, vmax, t, lsup, start, d, osup);
                if (c != 0 && lane == 0) {
                    if constexpr (GLOBAL_LOOKUP) atomicAdd(&osup[start + i], c);
                    else atomicAdd(&lsup[i], c);
                }
                found += c;
            }
        }
        if constexpr (!GLOBAL_LOOKUP) {
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += blockDim.x) {
                const uint32_t x = lsup[j];
                if (x) atomicAdd(&osup[start + j], x);
            }
            __syncthreads();
        }
    }
    if (lane == 0 && found) atomicAdd(tri_total, found);
}

__global__ void k_bin_flags(int32_t n, const int64_t *__restrict__ orp, int lo, int hi,
                            uint32_t *__restrict__ flags) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = orp[r + 1] - orp[r];
        flags[r] = (d >= lo && d <= hi) ? 1u : 0u;
    }
}

__global__ void k_bin_write(int32_t n, const int64_t *__restrict__ orp, int lo, int hi,
                            const uint32_t *__restrict__ pos, int32_t *__restrict__ out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = orp[r + 1] - orp[r];
        if (d >= lo && d <= hi) out[pos[r]] = (int32_t)r;
    }
}

// Rows with lo <= d+ <= hi, in rank order; their count goes to the device
// word *count (the caller reads the counts of all bins back at once).
tc_status select_rows(const tc_graph *g, int lo, int hi, int32_t *out, uint32_t *count,
                      hipStream_t s) {
    tc_scratch tmp(s);
    uint32_t *pos = nullptr;
    TC_TRY(tmp.get(&pos, g->n));
    k_bin_flags<<<grid_for(g->n), BK, 0, s>>>(g->n, g->orp, lo, hi, pos);
    TC_LAUNCHED();
    TC_TRY(tc_scan_u32(pos, pos, g->n, count, s));
    k_bin_write<<<grid_for(g->n), BK, 0, s>>>(g->n, g->orp, lo, hi, pos, out);
    TC_LAUNCHED();
    return TC_OK;
}

}  // namespace

tc_status tc_tuning_default(tc_tuning *t) {
    if (!t) return TC_ERR_INVALID_ARG;
    t->light_max_dplus = 512;
    t->heavy_block = 256;
    t->light_block = 256;
    t->lds_max_entries = 4096;
    t->algorithm = TC_ALGO_AUTO;
    t->item_pairs = 512;
    t->bitmap_words = 4096;
    t->light_bitmap_pairs = 64;
    return TC_OK;
}

static bool tuning_valid(const tc_tuning *t) {
    auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
    return t->light_max_dplus >= 2 && t->light_max_dplus <= 1024 && t->heavy_block >= 64 &&
           t->heavy_block <= 1024 && t->heavy_block % 64 == 0 && t->light_block >= 64 &&
           t->light_block <= 1024 && t->light_block % 64 == 0 && pow2(t->lds_max_entries) &&
           t->lds_max_entries >= 1024 && t->lds_max_entries <= 16384 && t->algorithm >= 0 &&
           t->algorithm <= 2 && t->item_pairs >= 64 && t->item_pairs <= 65536 &&
           t->item_pairs % 64 == 0 &&
           (t->bitmap_words == 0 ||
            (pow2(t->bitmap_words) && t->bitmap_words >= 256 && t->bitmap_words <= 8192)) &&
           t->light_bitmap_pairs >= 0;
}

// The pivot form AUTO (or the tuning) takes for this graph.
static int choose_algo(const tc_graph *g, const tc_tuning &t) {
    if (t.algorithm != TC_ALGO_AUTO) return t.algorithm;
    const int64_t m = g->m;
    const bool mid = m >= AUTO_MID_MIN_EDGES_FLAT ||
                     (m >= AUTO_MID_MIN_EDGES && g->max_dplus >= AUTO_MID_MIN_DPLUS);
    return mid ? TC_ALGO_MID_PIVOT : TC_ALGO_LOW_PIVOT;
}

tc_status tc_count_bytes(tc_graph *g, const tc_tuning *tin, hipStream_t s, int64_t *bytes) {
    tc_tuning t;
    if (tin) t = *tin; else tc_tuning_default(&t);
    if (!tuning_valid(&t)) return TC_ERR_INVALID_ARG;
    const int64_t m = g->m, nn = g->n > 0 ? g->n : 1, G = g->num_graphs;
    // both forms: support per oriented slot and per edge, tri, num, tc, triG
    int64_t b = 8 * m + 24 * nn + 8 * (G + 1);
    if (m > 0 && g->max_dplus >= 2 && choose_algo(g, t) == TC_ALGO_MID_PIVOT) {
        int64_t words = 0;
        TC_TRY(tc_mid_bit_words(g, &words, s));
        // transposition (pair lists and offsets), bit matrices with their
        // row records and offsets, the 16-bit columns; temporaries of the
        // transposition sort, work-item lists, support reordering and
        // aggregation, all counted at once
        b += 8 * m + 8 * (nn + 1) + 4 * (words + 4) + 16 * nn + 8 * (nn + 1) + 2 * (m + 66) +
             30 * m + 96 * nn;
    } else {
        // flags, symmetric adjacency with its slot map; temporaries of the
        // bins and the aggregation
        b += 2 * m + 16 * m + 16 * m + 40 * nn;
    }
    // the caching allocator rounds each block up: by under 512 bytes below
    // 1 MiB, by under 2 MiB above; at most 64 blocks, each above 1 MiB
    // taking at least 1 MiB of b
    const int64_t big = (b >> 20) < 64 ? (b >> 20) : 64;
    *bytes = b + 64 * 512 + big * ((int64_t)2 << 20);
    return TC_OK;
}

tc_status tc_count(tc_graph *g, const tc_tuning *tin, hipStream_t s) {
    tc_tuning t;
    if (tin) t = *tin; else tc_tuning_default(&t);
    if (!tuning_valid(&t)) return TC_ERR_INVALID_ARG;
    const int64_t m = g->m;
    if (!g->osup) TC_TRY(tc_graph_alloc(g, &g->osup, m, s));
    if (!g->triG) TC_TRY(tc_graph_alloc(g, &g->triG, g->num_graphs + 1, s));
    TC_HIP(hipMemsetAsync(g->osup, 0, sizeof(uint32_t) * (m > 0 ? m : 1), s));
    // triG[num_graphs] is the scratch total of triangles found by the count
    unsigned long long *found = (unsigned long long *)(g->triG + g->num_graphs);
    TC_HIP(hipMemsetAsync(found, 0, sizeof(uint64_t), s));
    if (m == 0 || g->max_dplus < 2) {
        g->n_light = g->n_heavy = g->n_huge = 0;
        g->light_max = t.light_max_dplus;
        g->huge_min = 0x7FFFFFFF;
        for (int k = 5; k <= 9; ++k) tc_prof_mark(g, k, s);
        for (int k = 12; k <= 14; ++k) tc_prof_mark(g, k, s);
        return TC_OK;
    }

    // The heavy kernel's table and counters must fit one workgroup's LDS:
    // clamp the table size to what this device allows.
    int dev = 0, lds_limit = 65536;
    TC_HIP(hipGetDevice(&dev));
    TC_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    int max_entries = t.lds_max_entries;
    while (max_entries > 1024 && heavy_bytes(max_entries / 2) > (size_t)lds_limit) max_entries >>= 1;
    // AUTO: the middle pivot streams fewer candidates (the oriented wedges),
    // but its transposition, work items and fold cost a fixed number of
    // launches and host round trips.  On this device the low pivot finishes
    // first below about 0.6 M edges, and, on graphs whose oriented rows all
    // stay short (no degree skew, e.g. ER at average degree 16), up to a few
    // million.
    const int algo = choose_algo(g, t);
    g->algo_used = algo;
    if (algo == TC_ALGO_MID_PIVOT) return tc_count_mid(g, t, lds_limit, max_entries, found, s);
    const int light_max = t.light_max_dplus;
    // heavy rows: light_max < d+ < huge_min (table at most half full); the
    // three bins must not overlap, whatever the knobs
    int huge_min = max_entries / 2 + 1;
    if (huge_min <= light_max) huge_min = light_max + 1;
    tc_scratch tmp(s);
    int32_t *rows = nullptr, *heavy = nullptr, *huge = nullptr;
    uint32_t *cnt = nullptr;
    TC_TRY(tmp.get(&rows, g->n));
    TC_TRY(tmp.get(&heavy, g->n));
    TC_TRY(tmp.get(&huge, g->n));
    TC_TRY(tmp.get(&cnt, 4));
    TC_TRY(select_rows(g, 2, light_max, rows, cnt, s));
    TC_TRY(select_rows(g, light_max + 1, huge_min - 1, heavy, cnt + 1, s));
    TC_TRY(select_rows(g, huge_min, 0x7FFFFFFF, huge, cnt + 2, s));
    uint32_t hc[4] = {0, 0, 0, 0};
    TC_HIP(hipMemcpyAsync(hc, cnt, 12, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    const int64_t nl = hc[0], nh = hc[1], nz = hc[2];
    g->n_light = nl;
    g->n_heavy = nh;
    g->n_huge = nz;
    g->light_max = light_max;
    g->huge_min = huge_min;
    tc_prof_mark(g, 5, s);

    if (nl > 0) {
        const int dcap = light_max;
        const size_t per_wave = light_wave_bytes(dcap);
        int wpb = t.light_block / TC_WAVE;
        while (wpb > 1 && (size_t)wpb * per_wave > (size_t)lds_limit) --wpb;
        const int block = wpb * TC_WAVE;
        const size_t lds = (size_t)wpb * per_wave;
        int64_t blocks = tc_div_up(nl, wpb);
        if (blocks > 65536) blocks = 65536;
        k_count_light<<<(unsigned)blocks, block, lds, s>>>(g->orp, g->ocol, rows, nl, dcap, g->osup,
                                                         found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 6, s);
    if (nh > 0) {
        // every heavy row has light_max < d+ < huge_min and d+ <= max d+
        const int hmax = g->max_dplus < huge_min - 1 ? g->max_dplus : huge_min - 1;
        const size_t lds = heavy_bytes(hmax);
        int64_t blocks = nh < 1048576 ? nh : 1048576;
        k_count_heavy<false><<<(unsigned)blocks, t.heavy_block, lds, s>>>(
            g->orp, g->ocol, heavy, nh, hmax, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 7, s);
    if (nz > 0) {
        int64_t blocks = nz < 65536 ? nz : 65536;
        k_count_heavy<true><<<(unsigned)blocks, t.heavy_block, 0, s>>>(g->orp, g->ocol, huge, nz, 0,
                                                                      g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 8, s);
    tc_prof_mark(g, 9, s);  // the low-pivot form has no fold step
    return TC_OK;
}

// ---------------------------------------------------------------------------
// Work measures of the orientation (instrumentation).
// ---------------------------------------------------------------------------
namespace {

__global__ void k_work_stats(int32_t n, const int64_t *__restrict__ orp,
                             const int32_t *__restrict__ ocol, int light_max, int huge_min,
                             bool low_bins, unsigned long long *__restrict__ acc) {
    // per-thread sums of the 12 words, added once per wavefront: the words
    // are shared by every row
    unsigned long long sums[12] = {};
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = orp[r], e = orp[r + 1];
        const int64_t d = e - b;
        if (d == 0) continue;
        unsigned long long cand = 0, merge = 0;
        for (int64_t k = b; k < e; ++k) {
            const int32_t u = ocol[k];
            const int64_t du = orp[u + 1] - orp[u];
            cand += du;
            merge += d + du;
        }
        const int bin = d < 2 ? -1 : (d <= light_max ? 0 : (d < huge_min ? 1 : 2));
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (bin == q && low_bins) {
                sums[q] += 1ull;
                sums[3 + q] += cand;
                sums[8 + q] += (unsigned long long)d;
            }
        }
        sums[6] += merge;
        sums[7] += (unsigned long long)(d * (d - 1) / 2);
        sums[11] += cand;
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const unsigned long long t = tc_wave_sum(sums[q]);
        if (__lane_id() == 0 && t) atomicAdd(&acc[q], t);
    }
}

}  // namespace

tc_status tc_work_stats(tc_graph *g, int64_t *stats, hipStream_t s) {
    for (int i = 0; i < TC_NUM_WORK_STATS; ++i) stats[i] = 0;
    stats[TC_STAT_N] = g->n;
    stats[TC_STAT_M] = g->m;
    stats[TC_STAT_MAX_DPLUS] = g->max_dplus;
    if (g->n == 0 || g->m == 0) return TC_OK;
    tc_scratch tmp(s);
    unsigned long long *acc = nullptr;
    TC_TRY(tmp.get(&acc, 15));
    TC_HIP(hipMemsetAsync(acc, 0, 15 * sizeof(unsigned long long), s));
    int light_max = g->light_max > 0 ? g->light_max : 64;
    int huge_min = g->huge_min > 0 ? g->huge_min : 0x7FFFFFFF;
    const bool mid = g->algo_used != TC_ALGO_LOW_PIVOT;
    const unsigned wg = grid_for(g->n) < 4096u ? grid_for(g->n) : 4096u;
    k_work_stats<<<wg, BK, 0, s>>>(g->n, g->orp, g->ocol, light_max, huge_min, !mid,
                                               acc);
    TC_LAUNCHED();
    if (mid) TC_TRY(tc_mid_stats(g, acc, s));
    unsigned long long h[15];
    uint64_t tri = 0;
    TC_HIP(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    if (g->triG) TC_HIP(hipMemcpyAsync(&tri, g->triG + g->num_graphs, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    stats[TC_STAT_ROWS_LIGHT] = (int64_t)h[0];
    stats[TC_STAT_ROWS_HEAVY] = (int64_t)h[1];
    stats[TC_STAT_ROWS_HUGE] = (int64_t)h[2];
    stats[TC_STAT_CAND_LIGHT] = (int64_t)h[3];
    stats[TC_STAT_CAND_HEAVY] = (int64_t)h[4];
    stats[TC_STAT_CAND_HUGE] = (int64_t)h[5];
    stats[TC_STAT_MERGE_WORK] = (int64_t)h[6];
    stats[TC_STAT_WEDGES] = (int64_t)h[7];
    stats[TC_STAT_TRIANGLES] = (int64_t)tri;
    stats[TC_STAT_EDGES_LIGHT] = (int64_t)h[8];
    stats[TC_STAT_EDGES_HEAVY] = (int64_t)h[9];
    stats[TC_STAT_EDGES_HUGE] = (int64_t)h[10];
    stats[TC_STAT_W_HASH] = (int64_t)h[11];
    stats[TC_STAT_ALGORITHM] = mid ? TC_ALGO_MID_PIVOT : TC_ALGO_LOW_PIVOT;
    stats[TC_STAT_CAND_HEAVY_16] = (int64_t)h[12];
    stats[TC_STAT_EDGES_HEAVY_16] = (int64_t)h[13];
    stats[TC_STAT_ROWS_HEAVY_16] = (int64_t)h[14];
    return TC_OK;
}
