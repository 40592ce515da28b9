// The numerator by the algebraic form (Sec. "Algebraic Algorithm",
// Algorithm 3; Proposition 2): with T = A²∘A and T̆ its 0/1 pattern,
//     3·triG·TC = num = ½ (3A − 2T̆ + I)(T·1).
// Written as two sparse matrix-vector products over the symmetric CSR that
// carries T's values (T_vu = sup(v,u) on every edge, 0 elsewhere):
//     pass 1   t = T·1                      (t(v) = 2·tri(v));
//     pass 2   z = (3A − 2T̆ + I)·t, num = z/2, where on an edge the
//              coefficient is 3 − 2 = 1 if T_vu > 0 and 3 otherwise, and
//              the diagonal contributes t(v).
// This path shares no kernel with Algorithm 2's aggregation: it reads the
// support per canonical edge and nothing else of the count, so agreement of
// the two numerators is a cross-check of the whole aggregation.
#include "tc_internal.h"

namespace {

constexpr int BK = 256;
constexpr int GS = 16;             // lanes per row for rows up to BIG
constexpr int64_t BIG = 2048;      // longer rows: one workgroup each

static inline unsigned grid_for(int64_t n, int block = BK) {
    int64_t g = tc_div_up(n, block);
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (unsigned)g;
}

// T's values in CSR order: tv[p] = sup of the edge of symmetric slot p.
__global__ void k_alg_values(int64_t nnz, const uint32_t *__restrict__ sym2e,
                             const uint32_t *__restrict__ esup, uint32_t *__restrict__ tv) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        tv[p] = esup[sym2e[p]];
}

// Contribution of slot p to row v's product.
//   PASS 1: T_vu · 1
//   PASS 2: (3 − 2·[T_vu > 0]) · t(u)
template <int PASS>
__device__ __forceinline__ uint64_t term(int64_t p, const int32_t *__restrict__ col,
                                         const uint32_t *__restrict__ tv,
                                         const uint64_t *__restrict__ t) {
    if constexpr (PASS == 1) {
        return tv[p];
    } else {
        const uint64_t x = t[col[p]];
        return tv[p] != 0 ? x : 3 * x;
    }
}

template <int PASS>
__device__ __forceinline__ void finish(int64_t v, uint64_t acc, const uint64_t *__restrict__ t,
                                       uint64_t *__restrict__ out, uint32_t *__restrict__ err) {
    if constexpr (PASS == 1) {
        out[v] = acc;
    } else {
        const uint64_t z = acc + t[v];
        if (z & 1) atomicOr(err, 1u);  // (3A − 2T̆ + I)·T1 is even by Proposition 2
        out[v] = z >> 1;
    }
}

template <int PASS>
__global__ void k_alg_rows(int32_t n, const int64_t *__restrict__ row_ptr,
                           const int32_t *__restrict__ col, const uint32_t *__restrict__ tv,
                           const uint64_t *__restrict__ t, uint64_t *__restrict__ out,
                           uint32_t *__restrict__ err) {
    const int sub = threadIdx.x % GS;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / GS);
    for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GS; v < n; v += groups) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        if (e - b > BIG) continue;
        uint64_t acc = 0;
        for (int64_t p = b + sub; p < e; p += GS) acc += term<PASS>(p, col, tv, t);
#pragma unroll
        for (int off = GS / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, TC_WAVE);
        if (sub == 0) finish<PASS>(v, acc, t, out, err);
    }
}

template <int PASS>
__global__ void k_alg_rows_big(const int32_t *__restrict__ big, int64_t nbig,
                               const int64_t *__restrict__ row_ptr,
                               const int32_t *__restrict__ col, const uint32_t *__restrict__ tv,
                               const uint64_t *__restrict__ t, uint64_t *__restrict__ out,
                               uint32_t *__restrict__ err) {
    __shared__ uint64_t red[16];
    for (int64_t i = blockIdx.x; i < nbig; i += gridDim.x) {
        const int32_t v = big[i];
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        uint64_t acc = 0;
        for (int64_t p = b + threadIdx.x; p < e; p += blockDim.x) acc += term<PASS>(p, col, tv, t);
        acc = tc_wave_sum(acc);
        if (__lane_id() == 0) red[threadIdx.x / TC_WAVE] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t s = 0;
            for (int w = 0; w < (int)(blockDim.x / TC_WAVE); ++w) s += red[w];
            finish<PASS>(v, s, t, out, err);
        }
        __syncthreads();
    }
}

__global__ void k_alg_big_flags(int32_t n, const int64_t *__restrict__ row_ptr,
                                uint32_t *__restrict__ f) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        f[v] = (row_ptr[v + 1] - row_ptr[v]) > BIG ? 1u : 0u;
}

__global__ void k_alg_big_write(int32_t n, const uint32_t *__restrict__ f,
                                const uint32_t *__restrict__ pos, int32_t *__restrict__ out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        if (f[v]) out[pos[v]] = (int32_t)v;
}

}  // namespace

tc_status tc_alg_numerator(const tc_graph *g, uint64_t *d_num, hipStream_t s) {
    const int32_t n = g->n;
    const int64_t nnz = 2 * g->m;
    if (n == 0) return TC_OK;
    // the symmetric adjacency is a cache of the handle: filling it does not
    // change any result the handle reports
    TC_TRY(tc_ensure_symmetric(const_cast<tc_graph *>(g), s));
    tc_scratch tmp(s);
    uint32_t *tv = nullptr, *f = nullptr, *pos = nullptr, *tot = nullptr, *err = nullptr;
    uint64_t *t = nullptr;
    int32_t *big = nullptr;
    TC_TRY(tmp.get(&tv, nnz > 0 ? nnz : 1));
    TC_TRY(tmp.get(&t, n));
    TC_TRY(tmp.get(&f, n));
    TC_TRY(tmp.get(&pos, n));
    TC_TRY(tmp.get(&tot, 1));
    TC_TRY(tmp.get(&err, 1));
    TC_TRY(tmp.get(&big, n));
    TC_HIP(hipMemsetAsync(err, 0, 4, s));
    if (nnz > 0) {
        k_alg_values<<<grid_for(nnz), BK, 0, s>>>(nnz, g->sym2e, g->esup, tv);
        TC_LAUNCHED();
    }
    k_alg_big_flags<<<grid_for(n), BK, 0, s>>>(n, g->row_ptr, f);
    TC_LAUNCHED();
    TC_TRY(tc_scan_u32(f, pos, n, tot, s));
    k_alg_big_write<<<grid_for(n), BK, 0, s>>>(n, f, pos, big);
    TC_LAUNCHED();
    uint32_t hbig = 0;
    TC_HIP(hipMemcpyAsync(&hbig, tot, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    const unsigned grid = grid_for((int64_t)n * GS);
    const unsigned bgrid = hbig < 65536 ? (hbig > 0 ? hbig : 1) : 65536;
    k_alg_rows<1><<<grid, BK, 0, s>>>(n, g->row_ptr, g->col, tv, nullptr, t, err);
    TC_LAUNCHED();
    if (hbig) {
        k_alg_rows_big<1><<<bgrid, 1024, 0, s>>>(big, hbig, g->row_ptr, g->col, tv, nullptr, t, err);
        TC_LAUNCHED();
    }
    k_alg_rows<2><<<grid, BK, 0, s>>>(n, g->row_ptr, g->col, tv, t, d_num, err);
    TC_LAUNCHED();
    if (hbig) {
        k_alg_rows_big<2><<<bgrid, 1024, 0, s>>>(big, hbig, g->row_ptr, g->col, tv, t, d_num, err);
        TC_LAUNCHED();
    }
    uint32_t herr = 0;
    TC_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    return herr ? TC_ERR_DEVICE : TC_OK;
}
