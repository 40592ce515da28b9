// Triangle counts per vertex, Algorithm 2's aggregation and the quotient.
//
//  * support moves from oriented slots to canonical edges (its output order);
//  * tri(v) = 1/2 Σ_{u ∈ N(v)} sup(v,u), the quoted theorem of the "Algebraic
//    Form" section (each triangle at v puts 1 on two of v's edges); the same
//    pass records, per symmetric slot, whether the edge has support: that is
//    u ∈ N△(v), since N△(v) = supp T_v (Proposition 2's proof);
//  * triG = 1/3 Σ_v tri(v) per graph;
//  * Algorithm 2 over each row: x = tri(v) + Σ_{u ∈ N△(v)} tri(u),
//    s = Σ_{u ∈ N(v)} tri(u), y = s - x + tri(v), and Definition 1 times
//    3·triG is num = x + 3y = tri(v) + Σ_u tri(u)·(1 if u ∈ N△(v) else 3),
//    accumulated in that last form so every term is non-negative;
//  * tc = (double)num / (double)(3·triG), one IEEE division (0 if triG = 0).
//
// Rows are processed by 16-lane groups (four per wavefront) so that short
// rows do not idle a whole wavefront; rows longer than BIG_DEG go to a
// second kernel with a workgroup per row.
#include "tc_internal.h"

namespace {

constexpr int BK = 256;
constexpr int GS = 16;            // lanes per row in the small-row kernels
constexpr int64_t BIG_DEG = 4096;  // rows above this use a workgroup

static inline unsigned grid_for(int64_t n, int block = BK) {
    int64_t g = tc_div_up(n, block);
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (unsigned)g;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
    for (int off = GS / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, TC_WAVE);
    return x;
}

template <typename T>
__device__ T block_sum(T x, T *red) {
    x = tc_wave_sum(x);
    const int w = threadIdx.x / TC_WAVE;
    if (__lane_id() == 0) red[w] = x;
    __syncthreads();
    T t = 0;
    for (int i = 0; i < (int)(blockDim.x / TC_WAVE); ++i) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ int32_t graph_of(const int64_t *__restrict__ vtx_off, int32_t G,
                                            int64_t v) {
    int32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (vtx_off[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// esup[e[i]] = sup[i] for pairs already grouped by the top bits of e, so
// that the stores of neighbouring blocks fall in a few narrow windows.
__global__ void k_store_pairs(int64_t m, const uint32_t *__restrict__ e,
                              const uint32_t *__restrict__ sup, uint32_t *__restrict__ esup) {
    GRID_STRIDE(i, m) esup[e[i]] = sup[i];
}

__global__ void k_scatter_sup(int64_t m, const uint32_t *__restrict__ o2e,
                              const uint32_t *__restrict__ osup, uint32_t *__restrict__ esup) {
    GRID_STRIDE(k, m) esup[o2e[k]] = osup[k];
}

// tri(v) and the triangle-neighbour flag of each slot, small rows.
__global__ void k_tri_small(int32_t n, const int64_t *__restrict__ row_ptr,
                            const uint32_t *__restrict__ sym2e, const uint32_t *__restrict__ esup,
                            uint8_t *__restrict__ flag, uint64_t *__restrict__ tri,
                            uint32_t *__restrict__ err) {
    const int sub = threadIdx.x % GS;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / GS);
    for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GS; v < n; v += groups) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        if (e - b > BIG_DEG) continue;
        uint64_t acc = 0;
        for (int64_t p = b + sub; p < e; p += GS) {
            uint32_t sp = esup[sym2e[p]];
            flag[p] = sp != 0;
            acc += sp;
        }
        acc = group_sum(acc);
        if (sub == 0) {
            if (acc & 1) atomicOr(err, 2u);
            tri[v] = acc >> 1;
        }
    }
}

__global__ void k_tri_big(const int32_t *__restrict__ big, int64_t nbig,
                          const int64_t *__restrict__ row_ptr, const uint32_t *__restrict__ sym2e,
                          const uint32_t *__restrict__ esup, uint8_t *__restrict__ flag,
                          uint64_t *__restrict__ tri, uint32_t *__restrict__ err) {
    __shared__ uint64_t red[16];
    for (int64_t i = blockIdx.x; i < nbig; i += gridDim.x) {
        const int32_t v = big[i];
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        uint64_t acc = 0;
        for (int64_t p = b + threadIdx.x; p < e; p += blockDim.x) {
            uint32_t sp = esup[sym2e[p]];
            flag[p] = sp != 0;
            acc += sp;
        }
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) {
            if (acc & 1) atomicOr(err, 2u);
            tri[v] = acc >> 1;
        }
    }
}

// Σ tri over each graph's vertex range (block-level pre-reduction when the
// block's vertices lie in one graph).
__global__ void k_tri_sum(int32_t n, const uint64_t *__restrict__ tri,
                          const int64_t *__restrict__ vtx_off, int32_t G,
                          unsigned long long *__restrict__ sums) {
    __shared__ uint64_t red[16];
    const int64_t per_block = (int64_t)blockDim.x * 8;
    for (int64_t base = (int64_t)blockIdx.x * per_block; base < n; base += (int64_t)gridDim.x * per_block) {
        int64_t last = base + per_block - 1;
        if (last >= n) last = n - 1;
        const int32_t g0 = vtx_off ? graph_of(vtx_off, G, base) : 0;
        const int32_t g1 = vtx_off ? graph_of(vtx_off, G, last) : 0;
        if (g0 == g1) {
            uint64_t acc = 0;
            for (int64_t v = base + threadIdx.x; v <= last; v += blockDim.x) acc += tri[v];
            acc = block_sum(acc, red);
            if (threadIdx.x == 0 && acc) atomicAdd(&sums[g0], (unsigned long long)acc);
        } else {
            for (int64_t v = base + threadIdx.x; v <= last; v += blockDim.x) {
                uint64_t t = tri[v];
                if (t) atomicAdd(&sums[graph_of(vtx_off, G, v)], (unsigned long long)t);
            }
        }
    }
}

__global__ void k_tri_finish(int32_t G, uint64_t *__restrict__ triG, uint32_t *__restrict__ err) {
    GRID_STRIDE(g, G) {
        uint64_t s = triG[g];
        if (s % 3) atomicOr(err, 4u);
        uint64_t t = s / 3;
        if (t > ~0ull / 3) atomicOr(err, 8u);
        triG[g] = t;
    }
}

__device__ __forceinline__ double quotient(uint64_t num, uint64_t tg) {
    // one correctly rounded binary64 division of two exactly converted
    // integers (both below 2^53 in practice; the conversion rounds to
    // nearest even otherwise, as it does on the host)
    return tg == 0 ? 0.0 : __ddiv_rn((double)num, (double)(3 * tg));
}

__global__ void k_num_small(int32_t n, const int64_t *__restrict__ row_ptr,
                            const int32_t *__restrict__ col, const uint8_t *__restrict__ flag,
                            const uint64_t *__restrict__ tri, const uint64_t *__restrict__ triG,
                            const int64_t *__restrict__ vtx_off, int32_t G,
                            uint64_t *__restrict__ num, double *__restrict__ tcv) {
    const int sub = threadIdx.x % GS;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / GS);
    for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GS; v < n; v += groups) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        if (e - b > BIG_DEG) continue;
        uint64_t acc = 0;
        for (int64_t p = b + sub; p < e; p += GS) {
            uint64_t t = tri[col[p]];
            acc += flag[p] ? t : 3 * t;
        }
        acc = group_sum(acc);
        if (sub == 0) {
            uint64_t x = acc + tri[v];
            num[v] = x;
            uint64_t tg = triG[vtx_off ? graph_of(vtx_off, G, v) : 0];
            tcv[v] = quotient(x, tg);
        }
    }
}

__global__ void k_num_big(const int32_t *__restrict__ big, int64_t nbig,
                          const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                          const uint8_t *__restrict__ flag, const uint64_t *__restrict__ tri,
                          const uint64_t *__restrict__ triG, const int64_t *__restrict__ vtx_off,
                          int32_t G, uint64_t *__restrict__ num, double *__restrict__ tcv) {
    __shared__ uint64_t red[16];
    for (int64_t i = blockIdx.x; i < nbig; i += gridDim.x) {
        const int32_t v = big[i];
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        uint64_t acc = 0;
        for (int64_t p = b + threadIdx.x; p < e; p += blockDim.x) {
            uint64_t t = tri[col[p]];
            acc += flag[p] ? t : 3 * t;
        }
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) {
            uint64_t x = acc + tri[v];
            num[v] = x;
            uint64_t tg = triG[vtx_off ? graph_of(vtx_off, G, v) : 0];
            tcv[v] = quotient(x, tg);
        }
    }
}

// ---------------------------------------------------------------------------
// The same aggregation in rank space, from the orientation and its
// transposition (available once the middle-pivot count has run): the
// neighbours of rank row r are its out-slots k (N_H(r), ocol[k]) and its
// in-pairs (u, k) (N_L(r)), and every edge's support sits at its oriented
// slot, so the symmetric adjacency is not needed.  A row's entries are its
// out-slots followed by its in-pairs.  Rows of up to RANK_SMALL entries go
// to 16-lane groups; longer ones are cut into chunks of RANK_CHUNK entries,
// one workgroup each, whose partial sums the row's first chunk adds up in a
// second kernel (no atomics, and a hub no longer holds one workgroup for the
// whole of its row).
// ---------------------------------------------------------------------------
constexpr int64_t RANK_SMALL = 256;
constexpr int64_t RANK_CHUNK = 2048;

__device__ __forceinline__ int64_t rank_row_len(const int64_t *__restrict__ orp,
                                                const int64_t *__restrict__ in_ptr, int64_t r) {
    return (orp[r + 1] - orp[r]) + (in_ptr[r + 1] - in_ptr[r]);
}

// Σ over entries [a, b) of row r of sup (PASS 1) or of tri(other end)
// weighted 1 if the edge has support, 3 if not (PASS 2), over the lanes
// tid, tid + L, ...  PASS 1 also packs each in-pair as its lower end with
// bit 31 set when the edge has no support (in_uw, in in_pair's order), so
// PASS 2 reads one coalesced word per in-pair instead of gathering the
// support again.
template <int PASS>
__device__ __forceinline__ uint64_t rank_range_sum(int64_t r, int64_t a, int64_t b, int tid, int L,
                                                   const int64_t *__restrict__ orp,
                                                   const int32_t *__restrict__ ocol,
                                                   const int64_t *__restrict__ in_ptr,
                                                   const uint64_t *__restrict__ in_pair,
                                                   const uint32_t *__restrict__ osup,
                                                   uint32_t *__restrict__ in_uw,
                                                   const uint64_t *__restrict__ tri_r) {
    const int64_t ob = orp[r], olen = orp[r + 1] - ob, ib = in_ptr[r];
    uint64_t acc = 0;
    for (int64_t t = a + tid; t < (b < olen ? b : olen); t += L) {
        const int64_t k = ob + t;
        const uint32_t sp = osup[k];
        if constexpr (PASS == 1) {
            acc += sp;
        } else {
            const uint64_t x = tri_r[ocol[k]];
            acc += sp ? x : 3 * x;
        }
    }
    for (int64_t t = (a > olen ? a : olen) + tid; t < b; t += L) {
        const int64_t i = ib + (t - olen);
        if constexpr (PASS == 1) {
            const uint64_t pr = in_pair[i];
            const uint32_t sp = osup[(uint32_t)pr];
            acc += sp;
            in_uw[i] = (uint32_t)(pr >> 32) | (sp ? 0u : 0x80000000u);
        } else {
            const uint32_t w = in_uw[i];
            const uint64_t x = tri_r[w & 0x7FFFFFFFu];
            acc += (w >> 31) ? 3 * x : x;
        }
    }
    return acc;
}

// PASS 1: tri in rank order (tri_r) and in vertex order (tri).
// PASS 2: num and tc in vertex order.
template <int PASS>
__device__ __forceinline__ void rank_row_finish(int64_t r, uint64_t acc,
                                                const int32_t *__restrict__ perm,
                                                uint64_t *__restrict__ tri_r,
                                                uint64_t *__restrict__ tri,
                                                const uint64_t *__restrict__ triG,
                                                const int64_t *__restrict__ vtx_off, int32_t G,
                                                uint64_t *__restrict__ num,
                                                double *__restrict__ tcv, uint32_t *__restrict__ err) {
    const int32_t v = perm[r];
    if constexpr (PASS == 1) {
        if (acc & 1) atomicOr(err, 2u);
        tri_r[r] = acc >> 1;
        tri[v] = acc >> 1;
    } else {
        const uint64_t x = acc + tri_r[r];
        num[v] = x;
        tcv[v] = quotient(x, triG[vtx_off ? graph_of(vtx_off, G, v) : 0]);
    }
}

struct RankArgs {
    const int64_t *orp;
    const int32_t *ocol;
    const int64_t *in_ptr;
    const uint64_t *in_pair;
    const uint32_t *osup;
    uint32_t *in_uw;
    const int32_t *perm;
    uint64_t *tri_r;
    uint64_t *tri;
    const uint64_t *triG;
    const int64_t *vtx_off;
    int32_t G;
    uint64_t *num;
    double *tcv;
    uint32_t *err;
};

template <int PASS>
__global__ void k_rank_rows(int32_t n, RankArgs q) {
    const int sub = threadIdx.x % GS;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / GS);
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GS; r < n; r += groups) {
        const int64_t len = rank_row_len(q.orp, q.in_ptr, r);
        if (len > RANK_SMALL) continue;
        uint64_t acc = rank_range_sum<PASS>(r, 0, len, sub, GS, q.orp, q.ocol, q.in_ptr, q.in_pair,
                                            q.osup, q.in_uw, q.tri_r);
        acc = group_sum(acc);
        if (sub == 0)
            rank_row_finish<PASS>(r, acc, q.perm, q.tri_r, q.tri, q.triG, q.vtx_off, q.G, q.num,
                                  q.tcv, q.err);
    }
}

// chunk[c] = (row << 32) | index of the chunk within its row
template <int PASS>
__global__ __launch_bounds__(256) void k_rank_chunks(const uint64_t *__restrict__ chunk,
                                                     int64_t nchunk, RankArgs q,
                                                     uint64_t *__restrict__ part) {
    __shared__ uint64_t red[4];
    for (int64_t c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const uint64_t w = chunk[c];
        const int64_t r = (int64_t)(w >> 32);
        const int64_t a = (int64_t)(uint32_t)w * RANK_CHUNK;
        const int64_t len = rank_row_len(q.orp, q.in_ptr, r);
        const int64_t b = a + RANK_CHUNK < len ? a + RANK_CHUNK : len;
        uint64_t acc = rank_range_sum<PASS>(r, a, b, threadIdx.x, blockDim.x, q.orp, q.ocol,
                                            q.in_ptr, q.in_pair, q.osup, q.in_uw, q.tri_r);
        acc = block_sum(acc, red);
        if (threadIdx.x == 0) part[c] = acc;
    }
}

// The first chunk of each row adds the row's partial sums and finishes it.
template <int PASS>
__global__ void k_rank_chunks_finish(const uint64_t *__restrict__ chunk, int64_t nchunk,
                                     const uint64_t *__restrict__ part, RankArgs q) {
    GRID_STRIDE(c, nchunk) {
        const uint64_t w = chunk[c];
        if ((uint32_t)w != 0) continue;
        const int64_t r = (int64_t)(w >> 32);
        const int64_t nc = tc_div_up(rank_row_len(q.orp, q.in_ptr, r), RANK_CHUNK);
        uint64_t acc = 0;
        for (int64_t j = 0; j < nc; ++j) acc += part[c + j];
        rank_row_finish<PASS>(r, acc, q.perm, q.tri_r, q.tri, q.triG, q.vtx_off, q.G, q.num, q.tcv,
                              q.err);
    }
}

__global__ void k_rank_chunk_count(int32_t n, const int64_t *__restrict__ orp,
                                   const int64_t *__restrict__ in_ptr, uint32_t *__restrict__ cnt) {
    GRID_STRIDE(r, n) {
        const int64_t len = rank_row_len(orp, in_ptr, r);
        cnt[r] = len > RANK_SMALL ? (uint32_t)tc_div_up(len, RANK_CHUNK) : 0u;
    }
}

__global__ void k_rank_chunk_write(int32_t n, const uint32_t *__restrict__ cnt,
                                   const uint32_t *__restrict__ off, uint64_t *__restrict__ chunk) {
    GRID_STRIDE(r, n) {
        const uint32_t c = cnt[r];
        for (uint32_t j = 0; j < c; ++j) chunk[off[r] + j] = ((uint64_t)r << 32) | j;
    }
}

__global__ void k_big_flags(int32_t n, const int64_t *__restrict__ row_ptr, uint32_t *__restrict__ f) {
    GRID_STRIDE(v, n) f[v] = (row_ptr[v + 1] - row_ptr[v]) > BIG_DEG ? 1u : 0u;
}

__global__ void k_big_write(int32_t n, const int64_t *__restrict__ row_ptr,
                            const uint32_t *__restrict__ pos, int32_t *__restrict__ out) {
    GRID_STRIDE(v, n) if ((row_ptr[v + 1] - row_ptr[v]) > BIG_DEG) out[pos[v]] = (int32_t)v;
}

}  // namespace

static tc_status aggregate_rank_space(tc_graph *g, hipStream_t s);

// esup (canonical edge order) from osup (oriented slot order).  Large
// graphs first group the (edge, support) pairs by the top 8 bits of the
// edge id with one stable radix pass, so the stores then land in windows of
// about m / 256 edges instead of all over esup.
static tc_status support_to_edge_order(tc_graph *g, hipStream_t s) {
    const int64_t m = g->m;
    if (m == 0) return TC_OK;
    if (m < ((int64_t)1 << 22)) {
        k_scatter_sup<<<grid_for(m), BK, 0, s>>>(m, g->o2e, g->osup, g->esup);
        TC_LAUNCHED();
        return TC_OK;
    }
    int ebits = 0;
    while (((int64_t)1 << ebits) < m) ++ebits;
    tc_scratch tmp(s);
    uint32_t *e2 = nullptr, *s2 = nullptr;
    TC_TRY(tmp.get(&e2, m));
    TC_TRY(tmp.get(&s2, m));
    TC_TRY(tc_partition_u32_u32(g->o2e, g->osup, e2, s2, m, ebits - 8, s));
    k_store_pairs<<<grid_for(m), BK, 0, s>>>(m, e2, s2, g->esup);
    TC_LAUNCHED();
    return TC_OK;
}

tc_status tc_aggregate(tc_graph *g, hipStream_t s) {
    // with the transposed orientation at hand, aggregate in rank space; the
    // symmetric adjacency is then never filled
    if (g->in_pair) return aggregate_rank_space(g, s);
    const int32_t n = g->n;
    const int64_t m = g->m;
    const int32_t G = g->num_graphs;
    const int64_t nn = n > 0 ? n : 1;
    TC_TRY(tc_ensure_symmetric(g, s));
    if (!g->esup) TC_TRY(tc_graph_alloc(g, &g->esup, m, s));
    if (!g->flag) TC_TRY(tc_graph_alloc(g, &g->flag, 2 * m, s));
    if (!g->tri) TC_TRY(tc_graph_alloc(g, &g->tri, nn, s));
    if (!g->num) TC_TRY(tc_graph_alloc(g, &g->num, nn, s));
    if (!g->tcv) TC_TRY(tc_graph_alloc(g, &g->tcv, nn, s));
    const int64_t *voff = G > 1 ? g->vtx_off : nullptr;
    TC_HIP(hipMemsetAsync(g->triG, 0, sizeof(uint64_t) * G, s));
    if (n == 0) {
        tc_prof_mark(g, 10, s);
        tc_prof_mark(g, 11, s);
        return TC_OK;
    }

    tc_scratch tmp(s);
    uint32_t *pos = nullptr, *tot = nullptr;
    int32_t *big = nullptr;
    TC_TRY(tmp.get(&pos, nn));
    TC_TRY(tmp.get(&tot, 1));
    TC_TRY(tmp.get(&big, nn));
    k_big_flags<<<grid_for(n), BK, 0, s>>>(n, g->row_ptr, pos);
    TC_LAUNCHED();
    TC_TRY(tc_scan_u32(pos, pos, n, tot, s));
    k_big_write<<<grid_for(n), BK, 0, s>>>(n, g->row_ptr, pos, big);
    TC_LAUNCHED();
    uint32_t hbig = 0;
    TC_HIP(hipMemcpyAsync(&hbig, tot, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    const int64_t nbig = hbig;

    if (m > 0) {
        k_scatter_sup<<<grid_for(m), BK, 0, s>>>(m, g->o2e, g->osup, g->esup);
        TC_LAUNCHED();
    }
    const unsigned small_grid = grid_for((int64_t)n * GS);
    k_tri_small<<<small_grid, BK, 0, s>>>(n, g->row_ptr, g->sym2e, g->esup, g->flag, g->tri, g->err);
    TC_LAUNCHED();
    if (nbig > 0) {
        k_tri_big<<<(unsigned)(nbig < 65536 ? nbig : 65536), 1024, 0, s>>>(
            big, nbig, g->row_ptr, g->sym2e, g->esup, g->flag, g->tri, g->err);
        TC_LAUNCHED();
    }
    k_tri_sum<<<grid_for(n, BK * 8), BK, 0, s>>>(n, g->tri, voff, G, (unsigned long long *)g->triG);
    TC_LAUNCHED();
    k_tri_finish<<<grid_for(G), BK, 0, s>>>(G, g->triG, g->err);
    TC_LAUNCHED();
    tc_prof_mark(g, 10, s);
    k_num_small<<<small_grid, BK, 0, s>>>(n, g->row_ptr, g->col, g->flag, g->tri, g->triG, voff, G,
                                          g->num, g->tcv);
    TC_LAUNCHED();
    if (nbig > 0) {
        k_num_big<<<(unsigned)(nbig < 65536 ? nbig : 65536), 1024, 0, s>>>(
            big, nbig, g->row_ptr, g->col, g->flag, g->tri, g->triG, voff, G, g->num, g->tcv);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 11, s);
    return TC_OK;
}

static tc_status aggregate_rank_space(tc_graph *g, hipStream_t s) {
    const int32_t n = g->n;
    const int64_t m = g->m;
    const int32_t G = g->num_graphs;
    const int64_t nn = n > 0 ? n : 1;
    if (!g->esup) TC_TRY(tc_graph_alloc(g, &g->esup, m, s));
    if (!g->tri) TC_TRY(tc_graph_alloc(g, &g->tri, nn, s));
    if (!g->num) TC_TRY(tc_graph_alloc(g, &g->num, nn, s));
    if (!g->tcv) TC_TRY(tc_graph_alloc(g, &g->tcv, nn, s));
    const int64_t *voff = G > 1 ? g->vtx_off : nullptr;
    TC_HIP(hipMemsetAsync(g->triG, 0, sizeof(uint64_t) * G, s));
    if (n == 0) {
        tc_prof_mark(g, 10, s);
        tc_prof_mark(g, 11, s);
        return TC_OK;
    }
    tc_scratch tmp(s);
    uint32_t *cnt = nullptr, *off = nullptr, *tot = nullptr, *in_uw = nullptr;
    uint64_t *tri_r = nullptr;
    TC_TRY(tmp.get(&in_uw, m > 0 ? m : 1));
    TC_TRY(tmp.get(&cnt, nn));
    TC_TRY(tmp.get(&off, nn));
    TC_TRY(tmp.get(&tot, 1));
    TC_TRY(tmp.get(&tri_r, nn));
    k_rank_chunk_count<<<grid_for(n), BK, 0, s>>>(n, g->orp, g->in_ptr, cnt);
    TC_LAUNCHED();
    TC_TRY(tc_scan_u32(cnt, off, n, tot, s));
    TC_TRY(support_to_edge_order(g, s));
    uint32_t hch = 0;
    TC_HIP(hipMemcpyAsync(&hch, tot, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    const int64_t nchunk = hch;
    uint64_t *chunk = nullptr, *part = nullptr;
    TC_TRY(tmp.get(&chunk, nchunk > 0 ? nchunk : 1));
    TC_TRY(tmp.get(&part, nchunk > 0 ? nchunk : 1));
    if (nchunk > 0) {
        k_rank_chunk_write<<<grid_for(n), BK, 0, s>>>(n, cnt, off, chunk);
        TC_LAUNCHED();
    }
    RankArgs q{g->orp, g->ocol, g->in_ptr, g->in_pair, g->osup, in_uw, g->perm, tri_r,
               g->tri, nullptr, voff, G, nullptr, nullptr, g->err};
    const unsigned small_grid = grid_for((int64_t)n * GS);
    const unsigned chunk_grid = (unsigned)(nchunk < 1048576 ? (nchunk > 0 ? nchunk : 1) : 1048576);
    k_rank_rows<1><<<small_grid, BK, 0, s>>>(n, q);
    TC_LAUNCHED();
    if (nchunk > 0) {
        k_rank_chunks<1><<<chunk_grid, 256, 0, s>>>(chunk, nchunk, q, part);
        TC_LAUNCHED();
        k_rank_chunks_finish<1><<<grid_for(nchunk), BK, 0, s>>>(chunk, nchunk, part, q);
        TC_LAUNCHED();
    }
    k_tri_sum<<<grid_for(n, BK * 8), BK, 0, s>>>(n, g->tri, voff, G, (unsigned long long *)g->triG);
    TC_LAUNCHED();
    k_tri_finish<<<grid_for(G), BK, 0, s>>>(G, g->triG, g->err);
    TC_LAUNCHED();
    tc_prof_mark(g, 10, s);
    q.triG = g->triG;
    q.num = g->num;
    q.tcv = g->tcv;
    k_rank_rows<2><<<small_grid, BK, 0, s>>>(n, q);
    TC_LAUNCHED();
    if (nchunk > 0) {
        k_rank_chunks<2><<<chunk_grid, 256, 0, s>>>(chunk, nchunk, q, part);
        TC_LAUNCHED();
        k_rank_chunks_finish<2><<<grid_for(nchunk), BK, 0, s>>>(chunk, nchunk, part, q);
        TC_LAUNCHED();
    }
    tc_prof_mark(g, 11, s);
    return TC_OK;
}
