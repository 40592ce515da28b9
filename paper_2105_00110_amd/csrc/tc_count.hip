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

namespace {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;
constexpr int BK = 256;

static inline unsigned grid_for(int64_t n, int block = BK) {
    int64_t g = tc_div_up(n, block);
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (unsigned)g;
}

static inline int ceil_log2(int64_t x) {
    int b = 0;
    while ((1ll << b) < x) ++b;
    return b;
}

__device__ __forceinline__ int ceil_log2_dev(int x) {
    return x <= 1 ? 0 : 32 - __clz(x - 1);
}

__device__ __forceinline__ uint32_t hash_slot(uint32_t key, int cb) {
    return (key * 0x9E3779B1u) >> (32 - cb);
}

__device__ __forceinline__ void hash_insert(uint32_t *hkey, uint32_t *hpos, int cb, uint32_t key,
                                            uint32_t pos) {
    const uint32_t mask = (1u << cb) - 1;
    uint32_t h = hash_slot(key, cb);
    while (true) {
        uint32_t prev = atomicCAS(&hkey[h], EMPTY, key);
        if (prev == EMPTY) {
            hpos[h] = pos;
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ int hash_find(const uint32_t *hkey, const uint32_t *hpos, int cb,
                                         uint32_t key) {
    const uint32_t mask = (1u << cb) - 1;
    uint32_t h = hash_slot(key, cb);
    while (true) {
        uint32_t k = hkey[h];
        if (k == key) return (int)hpos[h];
        if (k == EMPTY) return -1;
        h = (h + 1) & mask;
    }
}

// Streams N_H(u) = ocol[ub, ue) against the table of row v and applies the
// support updates.  Returns |N_H(v) ∩ N_H(u)| (wave-uniform).
template <bool GLOBAL_LOOKUP>
__device__ __forceinline__ uint32_t stream_u(const int32_t *__restrict__ ocol, int64_t ub,
                                             int64_t ue, uint32_t vmax, const uint32_t *hkey,
                                             const uint32_t *hpos, int cb, uint32_t *lsup,
                                             int64_t vstart, int dv, uint32_t *__restrict__ osup) {
    const int lane = __lane_id();
    uint32_t c = 0;
    for (int64_t jb = ub; jb < ue; jb += TC_WAVE) {
        int64_t j = jb + lane;
        bool in = j < ue;
        uint32_t w = in ? (uint32_t)ocol[j] : EMPTY;
        if ((uint32_t)__shfl(w, 0, TC_WAVE) > vmax) break;
        int p = -1;
        if (in && w <= vmax) {
            if constexpr (GLOBAL_LOOKUP) {
                int lo = 0, hi = dv;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if ((uint32_t)ocol[vstart + mid] < w) lo = mid + 1; else hi = mid;
                }
                if (lo < dv && (uint32_t)ocol[vstart + lo] == w) p = lo;
            } else {
                p = hash_find(hkey, hpos, cb, w);
            }
        }
        bool hit = p >= 0;
        if (hit) {
            if constexpr (GLOBAL_LOOKUP) atomicAdd(&osup[vstart + p], 1u);
            else atomicAdd(&lsup[p], 1u);
            atomicAdd(&osup[j], 1u);
        }
        c += (uint32_t)__popcll(__ballot(hit));
    }
    return c;
}

// One wavefront per light row.  LDS per wavefront: table (2·cap words) and
// the row's support counters (dcap words).
__global__ __launch_bounds__(1024) void k_count_light(const int64_t *__restrict__ orp,
                                                      const int32_t *__restrict__ ocol,
                                                      const int32_t *__restrict__ rows,
                                                      int64_t nrows, int cbmax, int dcap,
                                                      uint32_t *__restrict__ osup,
                                                      unsigned long long *__restrict__ tri_total) {
    extern __shared__ uint32_t lds[];
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    const int capmax = 1 << cbmax;
    uint32_t *hkey = lds + wv * (2 * capmax + dcap);
    uint32_t *hpos = hkey + capmax;
    uint32_t *lsup = hpos + capmax;
    unsigned long long found = 0;
    for (int64_t ri = (int64_t)blockIdx.x * wpb + wv; ri < nrows; ri += (int64_t)gridDim.x * wpb) {
        const int32_t r = rows[ri];
        const int64_t start = orp[r];
        const int d = (int)(orp[r + 1] - start);
        int cb = ceil_log2_dev(2 * d);
        if (cb < 1) cb = 1;
        const int cap = 1 << cb;
        for (int j = lane; j < cap; j += TC_WAVE) hkey[j] = EMPTY;
        for (int j = lane; j < d; j += TC_WAVE) lsup[j] = 0;
        for (int j = lane; j < d; j += TC_WAVE) hash_insert(hkey, hpos, cb, (uint32_t)ocol[start + j], j);
        const uint32_t vmax = (uint32_t)ocol[start + d - 1];
        for (int i0 = 0; i0 < d - 1; i0 += TC_WAVE) {
            const int ii = i0 + lane;
            int64_t ub_l = 0, ue_l = 0;
            if (ii < d - 1) {
                int32_t u = ocol[start + ii];
                ub_l = orp[u];
                ue_l = orp[u + 1];
            }
            const int cnt = min(TC_WAVE, d - 1 - i0);
            for (int k = 0; k < cnt; ++k) {
                int64_t ub = __shfl(ub_l, k, TC_WAVE), ue = __shfl(ue_l, k, TC_WAVE);
                uint32_t c = stream_u<false>(ocol, ub, ue, vmax, hkey, hpos, cb, lsup, start, d, osup);
                if (c != 0 && lane == 0) atomicAdd(&lsup[i0 + k], c);
                found += c;
            }
        }
        for (int j = lane; j < d; j += TC_WAVE) {
            uint32_t x = lsup[j];
            if (x) atomicAdd(&osup[start + j], x);
        }
    }
    if (lane == 0 && found) atomicAdd(tri_total, found);
}

// One workgroup per heavy row; the workgroup's wavefronts share the table
// and take the row's u in chunks of 64.  Rows are taken from the end of
// the list (highest rank, typically the most work) first.
template <bool GLOBAL_LOOKUP>
__global__ __launch_bounds__(1024) void k_count_heavy(const int64_t *__restrict__ orp,
                                                      const int32_t *__restrict__ ocol,
                                                      const int32_t *__restrict__ rows,
                                                      int64_t nrows, int cbmax, int dcap,
                                                      uint32_t *__restrict__ osup,
                                                      unsigned long long *__restrict__ tri_total) {
    extern __shared__ uint32_t lds[];
    const int wpb = blockDim.x / TC_WAVE;
    const int wv = threadIdx.x / TC_WAVE;
    const int lane = __lane_id();
    const int capmax = GLOBAL_LOOKUP ? 0 : (1 << cbmax);
    uint32_t *hkey = lds;
    uint32_t *hpos = hkey + capmax;
    uint32_t *lsup = hpos + capmax;
    unsigned long long found = 0;
    for (int64_t bi = blockIdx.x; bi < nrows; bi += gridDim.x) {
        const int32_t r = rows[nrows - 1 - bi];
        const int64_t start = orp[r];
        const int d = (int)(orp[r + 1] - start);
        int cb = 1;
        if constexpr (!GLOBAL_LOOKUP) {
            cb = ceil_log2_dev(2 * d);
            if (cb < 1) cb = 1;
            const int cap = 1 << cb;
            for (int j = threadIdx.x; j < cap; j += blockDim.x) hkey[j] = EMPTY;
            for (int j = threadIdx.x; j < d; j += blockDim.x) lsup[j] = 0;
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += blockDim.x)
                hash_insert(hkey, hpos, cb, (uint32_t)ocol[start + j], j);
            __syncthreads();
        }
        const uint32_t vmax = (uint32_t)ocol[start + d - 1];
        for (int i0 = wv * TC_WAVE; i0 < d - 1; i0 += wpb * TC_WAVE) {
            const int ii = i0 + lane;
            int64_t ub_l = 0, ue_l = 0;
            if (ii < d - 1) {
                int32_t u = ocol[start + ii];
                ub_l = orp[u];
                ue_l = orp[u + 1];
            }
            const int cnt = min(TC_WAVE, d - 1 - i0);
            for (int k = 0; k < cnt; ++k) {
                int64_t ub = __shfl(ub_l, k, TC_WAVE), ue = __shfl(ue_l, k, TC_WAVE);
                uint32_t c = stream_u<GLOBAL_LOOKUP>(ocol, ub, ue, vmax, hkey, hpos, cb, lsup, start,
                                                     d, osup);
                if (c != 0 && lane == 0) {
                    if constexpr (GLOBAL_LOOKUP) atomicAdd(&osup[start + i0 + k], c);
                    else atomicAdd(&lsup[i0 + k], c);
                }
                found += c;
            }
        }
        if constexpr (!GLOBAL_LOOKUP) {
            __syncthreads();
            for (int j = threadIdx.x; j < d; j += blockDim.x) {
                uint32_t x = lsup[j];
                if (x) atomicAdd(&osup[start + j], x);
            }
            __syncthreads();
        }
    }
    (void)dcap;
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

__global__ void k_max_in_list(const int64_t *__restrict__ orp, const int32_t *__restrict__ rows,
                              int64_t nrows, uint32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = rows[i];
        atomicMax(out, (uint32_t)(orp[r + 1] - orp[r]));
    }
}

// Rows with lo <= d+ <= hi, in rank order; returns their count.
tc_status select_rows(const tc_graph *g, int lo, int hi, int32_t *out, int64_t *count,
                      hipStream_t s) {
    tc_scratch tmp(s);
    uint32_t *pos = nullptr, *tot = nullptr;
    TC_TRY(tmp.get(&pos, g->n));
    TC_TRY(tmp.get(&tot, 1));
    k_bin_flags<<<grid_for(g->n), BK, 0, s>>>(g->n, g->orp, lo, hi, pos);
    TC_LAUNCHED();
    TC_TRY(tc_scan_u32(pos, pos, g->n, tot, s));
    k_bin_write<<<grid_for(g->n), BK, 0, s>>>(g->n, g->orp, lo, hi, pos, out);
    TC_LAUNCHED();
    uint32_t h = 0;
    TC_HIP(hipMemcpyAsync(&h, tot, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    *count = h;
    return TC_OK;
}

}  // namespace

tc_status tc_tuning_default(tc_tuning *t) {
    if (!t) return TC_ERR_INVALID_ARG;
    t->light_max_dplus = 64;
    t->heavy_block = 256;
    t->light_block = 256;
    t->lds_max_entries = 4096;
    return TC_OK;
}

static bool tuning_valid(const tc_tuning *t) {
    auto pow2 = [](int x) { return x > 0 && (x & (x - 1)) == 0; };
    return t->light_max_dplus >= 2 && t->light_max_dplus <= 1024 && t->heavy_block >= 64 &&
           t->heavy_block <= 1024 && t->heavy_block % 64 == 0 && t->light_block >= 64 &&
           t->light_block <= 1024 && t->light_block % 64 == 0 && pow2(t->lds_max_entries) &&
           t->lds_max_entries >= 1024 && t->lds_max_entries <= 16384;
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
        for (int k = 5; k <= 8; ++k) tc_prof_mark(g, k, s);
        return TC_OK;
    }

    // The heavy kernel needs 8 bytes per table entry plus 4 per row entry
    // (at most half the table) in LDS: clamp the table to what one
    // workgroup may allocate on this device.
    int dev = 0, lds_limit = 65536;
    TC_HIP(hipGetDevice(&dev));
    TC_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    int max_entries = t.lds_max_entries;
    while (max_entries > 1024 && (size_t)max_entries * 10 > (size_t)lds_limit) max_entries >>= 1;
    const int light_max = t.light_max_dplus;
    // heavy rows: light_max < d+ < huge_min (table at most half full); the
    // three bins must not overlap, whatever the knobs
    int huge_min = max_entries / 2 + 1;
    if (huge_min <= light_max) huge_min = light_max + 1;
    tc_scratch tmp(s);
    int32_t *rows = nullptr;
    TC_TRY(tmp.get(&rows, g->n));
    int64_t nl = 0, nh = 0, nz = 0;
    TC_TRY(select_rows(g, 2, light_max, rows, &nl, s));
    int32_t *heavy = rows + nl;
    TC_TRY(select_rows(g, light_max + 1, huge_min - 1, heavy, &nh, s));
    int32_t *huge = heavy + nh;
    TC_TRY(select_rows(g, huge_min, 0x7FFFFFFF, huge, &nz, s));
    g->n_light = nl;
    g->n_heavy = nh;
    g->n_huge = nz;
    g->light_max = light_max;
    g->huge_min = huge_min;
    tc_prof_mark(g, 5, s);

    if (nl > 0) {
        const int dcap = light_max;
        const int cbmax = ceil_log2(2 * (int64_t)light_max);
        const size_t per_wave = (2 * ((size_t)1 << cbmax) + dcap) * sizeof(uint32_t);
        int wpb = t.light_block / TC_WAVE;
        while (wpb > 1 && (size_t)wpb * per_wave > (size_t)lds_limit) --wpb;
        const int block = wpb * TC_WAVE;
        const size_t lds = (size_t)wpb * per_wave;
        int64_t blocks = tc_div_up(nl, wpb);
        if (blocks > 65536) blocks = 65536;
        k_count_light<<<(unsigned)blocks, block, lds, s>>>(g->orp, g->ocol, rows, nl, cbmax, dcap,
                                                         g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 6, s);
    if (nh > 0) {
        uint32_t *dmax = nullptr;
        TC_TRY(tmp.get(&dmax, 1));
        TC_HIP(hipMemsetAsync(dmax, 0, 4, s));
        k_max_in_list<<<grid_for(nh), BK, 0, s>>>(g->orp, heavy, nh, dmax);
        TC_LAUNCHED();
        uint32_t hmax = 0;
        TC_HIP(hipMemcpyAsync(&hmax, dmax, 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        const int cbmax = ceil_log2(2 * (int64_t)hmax);
        const size_t lds = (2 * ((size_t)1 << cbmax) + hmax) * sizeof(uint32_t);
        int64_t blocks = nh < 1048576 ? nh : 1048576;
        tc_prof_mark(g, 6, s);  // after the host round trip for the table size
        k_count_heavy<false><<<(unsigned)blocks, t.heavy_block, lds, s>>>(
            g->orp, g->ocol, heavy, nh, cbmax, (int)hmax, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 7, s);
    if (nz > 0) {
        int64_t blocks = nz < 65536 ? nz : 65536;
        k_count_heavy<true><<<(unsigned)blocks, t.heavy_block, 0, s>>>(g->orp, g->ocol, huge, nz, 0,
                                                                      0, g->osup, found);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 8, s);
    return TC_OK;
}

// ---------------------------------------------------------------------------
// Work measures of the orientation (instrumentation).
// ---------------------------------------------------------------------------
namespace {

__global__ void k_work_stats(int32_t n, const int64_t *__restrict__ orp,
                             const int32_t *__restrict__ ocol, int light_max, int huge_min,
                             unsigned long long *__restrict__ acc) {
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
        int bin = d < 2 ? -1 : (d <= light_max ? 0 : (d < huge_min ? 1 : 2));
        if (bin >= 0) {
            atomicAdd(&acc[bin], 1ull);
            atomicAdd(&acc[3 + bin], cand);
            atomicAdd(&acc[8 + bin], (unsigned long long)d);
        }
        atomicAdd(&acc[6], merge);
        atomicAdd(&acc[7], (unsigned long long)(d * (d - 1) / 2));
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
    TC_TRY(tmp.get(&acc, 11));
    TC_HIP(hipMemsetAsync(acc, 0, 11 * sizeof(unsigned long long), s));
    int light_max = g->light_max > 0 ? g->light_max : 64;
    int huge_min = g->huge_min > 0 ? g->huge_min : 0x7FFFFFFF;
    k_work_stats<<<grid_for(g->n), BK, 0, s>>>(g->n, g->orp, g->ocol, light_max, huge_min, acc);
    TC_LAUNCHED();
    unsigned long long h[11];
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
    return TC_OK;
}
