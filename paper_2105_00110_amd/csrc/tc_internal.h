// Internal declarations of libtc: device helpers, primitive launchers and
// the graph handle.  Not part of the public ABI (include/tc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tc.h"

#define TC_WAVE 64
#define TC_PROF_MARKS 15
#define TC_OCOL_PAD 64

// ---------------------------------------------------------------------------
// Error plumbing: internal functions return tc_status; HIP failures map to
// TC_ERR_DEVICE (or TC_ERR_OOM for allocation failures).
// ---------------------------------------------------------------------------
#define TC_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return tc_map_hip_error(e_);   \
    } while (0)

#define TC_TRY(call)                                         \
    do {                                                     \
        tc_status s_ = (call);                               \
        if (s_ < 0) return s_;                               \
    } while (0)

tc_status tc_map_hip_error(hipError_t e);

// Launch check: kernel launch errors surface through hipGetLastError().
#define TC_LAUNCHED() TC_HIP(hipGetLastError())

__host__ __device__ static inline int64_t tc_div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

static inline int tc_bits_for(uint64_t max_value) {
    int b = 0;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

// ---------------------------------------------------------------------------
// Device memory: the library's caching allocator (tc_api.hip).  A block
// freed on one stream is handed to another stream only after the freeing
// stream's prior work, so temporaries never race with queued kernels.  With
// a limit set (tc_set_memory_limit), an allocation that would push the
// device bytes the library holds past it fails with TC_ERR_BUDGET.
// ---------------------------------------------------------------------------
tc_status tc_dev_alloc(void **p, size_t bytes, hipStream_t s);
void tc_dev_free(void *p, hipStream_t s);

template <typename T>
static inline tc_status tc_alloc(T **p, int64_t count, hipStream_t s) {
    size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    return tc_dev_alloc((void **)p, bytes, s);
}

// Temporaries of one host function, released (stream-ordered) on exit.
struct tc_scratch {
    static constexpr int MAX = 64;
    hipStream_t s;
    void *ptrs[MAX];
    int n = 0;
    explicit tc_scratch(hipStream_t st) : s(st) {}
    template <typename T>
    tc_status get(T **p, int64_t count) {
        if (n >= MAX) return TC_ERR_INVALID_ARG;
        tc_status r = tc_alloc(p, count, s);
        if (r == TC_OK) ptrs[n++] = (void *)*p;
        return r;
    }
    // p, allocated here, passes to the caller; q (same size) is freed in its place
    void exchange(void *p, void *q) {
        for (int i = 0; i < n; ++i)
            if (ptrs[i] == p) {
                ptrs[i] = q;
                return;
            }
    }
    ~tc_scratch() {
        for (int i = n - 1; i >= 0; --i) tc_dev_free(ptrs[i], s);
    }
};

// ---------------------------------------------------------------------------
// Primitives (tc_scan.hip, tc_sort.hip)
// ---------------------------------------------------------------------------
// Exclusive prefix sum of in[0..n) into out[0..n); if total != nullptr the
// sum of all n inputs is written to *total (device pointer).  in == out is
// allowed.
tc_status tc_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                      hipStream_t s);
tc_status tc_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, hipStream_t s);

// Stable LSD radix sort on the low `bits` bits of the keys (8-bit digits).
// The sorted data ends in *keys / *vals: the pointers are swapped with the
// tmp pointers when the pass count is odd, so callers free both buffers.
tc_status tc_sort_u64(uint64_t **keys, uint64_t **tmp_keys, int64_t n, int bits, hipStream_t s);
// keys from src (left unchanged), values the input positions 0..n-1: the
// stable sorting permutation of src; the result is in *keys / *vals
tc_status tc_sort_u32_index(const uint32_t *src, uint32_t **keys, uint32_t **vals,
                            uint32_t **tmp_keys, uint32_t **tmp_vals, int64_t n, int bits,
                            hipStream_t s);
// One stable pass: the (key, value) pairs ordered by the 8-bit digit
// (key >> shift) & 255, written to keys_out / vals_out (inputs unchanged).
tc_status tc_partition_u32_u32(const uint32_t *keys, const uint32_t *vals, uint32_t *keys_out,
                               uint32_t *vals_out, int64_t n, int shift, hipStream_t s);
// the same with 64-bit values (hi[i] << 32) | i
tc_status tc_sort_u32_index_hi(const uint32_t *src, const uint32_t *hi, uint32_t **keys,
                               uint64_t **vals, uint32_t **tmp_keys, uint64_t **tmp_vals,
                               int64_t n, int bits, hipStream_t s);
tc_status tc_sort_u64_u32(uint64_t **keys, uint32_t **vals, uint64_t **tmp_keys,
                          uint32_t **tmp_vals, int64_t n, int bits, hipStream_t s);
tc_status tc_sort_u32_u32(uint32_t **keys, uint32_t **vals, uint32_t **tmp_keys,
                          uint32_t **tmp_vals, int64_t n, int bits, hipStream_t s);

// ---------------------------------------------------------------------------
// The graph handle.
// ---------------------------------------------------------------------------
struct tc_graph {
    int device = 0;
    int32_t n = 0;           // vertices (sum over a batch)
    int64_t m = 0;           // canonical edges after normalisation
    int32_t num_graphs = 1;  // 1 unless built by tc_batch_create
    int bits = 1;            // bits per vertex id in packed keys
    hipStream_t last_stream = nullptr;
    bool computed = false;
    int32_t status = TC_OK;

    // canonical edges, lexicographic
    int32_t *eu = nullptr, *ev = nullptr;           // [m]
    // symmetric CSR in original ids, rows sorted by id
    int64_t *row_ptr = nullptr;                     // [n+1]
    int32_t *col = nullptr;                         // [2m] (filled on demand)
    uint32_t *sym2e = nullptr;                      // [2m] canonical edge of each slot
    // kept from the build so that col / sym2e can be filled on demand: the
    // first canonical edge whose smaller end is v
    uint32_t *run_us = nullptr;                     // [n]
    // the canonical edges ordered by their larger end (key = ev, val =
    // edge): from the build to the orientation, and on to the symmetric
    // fill unless the middle-pivot count releases them first
    uint32_t *lt_key = nullptr, *lt_val = nullptr;  // [m]
    // degree order: perm[r] = vertex of rank r, rank[v]
    int32_t *rank = nullptr, *perm = nullptr;       // [n]
    // oriented CSR over ranks: row r holds the ranks above r, ascending
    int64_t *orp = nullptr;                         // [n+1]
    int32_t *ocol = nullptr;                        // [m]
    // ocol for the pivots among the top 2^16 ranks: entries at or above
    // rank16_base, less rank16_base (16 bits); other entries read 0
    uint16_t *ocol16 = nullptr;                     // [m + TC_OCOL_PAD, rounded up to even]
    int32_t rank16_base = 0;
    uint32_t *o2e = nullptr;                        // [m] canonical edge of each oriented slot
    int32_t *orow = nullptr;                        // [m] row (rank) of each oriented slot
    // transposed orientation (middle-pivot counting): pairs grouped by the
    // higher end v, entry = (u << 32) | slot of v in N_H(u)
    int64_t *in_ptr = nullptr;                      // [n+1]
    uint64_t *in_pair = nullptr;                    // [m]
    // per-row triangular bit matrices of the middle-pivot scan
    int64_t *rowbase = nullptr;                     // [n+1] first word of each row's matrix
    uint32_t *hitbits = nullptr;                    // [bit_words]
    uint4 *rowinfo = nullptr;                       // [n] rowbase (low, high), row start, row end
    int64_t bit_words = 0;
    // results
    uint32_t *osup = nullptr;                       // [m] support per oriented slot
    uint32_t *esup = nullptr;                       // [m] support per canonical edge
    uint8_t *flag = nullptr;                        // [2m] slot edge has support > 0
    uint64_t *tri = nullptr, *num = nullptr;        // [n]
    double *tcv = nullptr;                          // [n]
    uint64_t *triG = nullptr;                       // [num_graphs]
    // batch bookkeeping (device copies + host copies)
    int64_t *vtx_off = nullptr;                     // device [G+1]
    int64_t *h_vtx_off = nullptr;                   // host [G+1]
    int64_t *h_edge_off = nullptr;                  // host [G+1]
    int32_t max_dplus = 0;
    int32_t *bin_rows = nullptr;                    // [n] rows with d+ >= 2, light then heavy
    int64_t n_light = 0, n_heavy = 0, n_huge = 0;
    uint32_t *err = nullptr;                        // device error word

    size_t bytes = 0;  // device bytes held

    // bins of the last count: light 2..light_max, heavy ..huge_min-1, huge
    int32_t light_max = 0, huge_min = 0;
    int32_t algo_used = 0;

    // profiling marks (see tc_prof_mark)
    bool prof = false;
    bool prof_build = false, prof_compute = false;
    hipEvent_t prof_ev[TC_PROF_MARKS] = {};
};

// Profiling marks: 0 build start, 1 CSR built, 2 ranked, 3 oriented,
// 4 compute start, 5 binned, 6 light counted, 7 heavy counted,
// 8 huge counted, 9 folded, 10 tri/triG done, 11 aggregated.
bool tc_profiling_on();
void tc_prof_mark(tc_graph *g, int idx, hipStream_t s);

// Pipeline stages (tc_build.hip, tc_count.hip, tc_aggregate.hip).
// Canonical edges from pairs (sorted and deduplicated), or, with simple_rp
// given, from a simple sorted CSR (simple_rp / simple_col, device): the
// entries above the diagonal, taken in order.
tc_status tc_build_from_pairs(tc_graph *g, const int32_t *d_src, const int32_t *d_dst,
                              int64_t P, const int64_t *d_pair_vtx_base,
                              const int64_t *d_pair_off, int32_t num_graphs, hipStream_t s,
                              const int64_t *simple_rp = nullptr,
                              const int32_t *simple_col = nullptr);
tc_status tc_orient(tc_graph *g, hipStream_t s);
tc_status tc_count(tc_graph *g, const tc_tuning *t, hipStream_t s);
tc_status tc_aggregate(tc_graph *g, hipStream_t s);
// Fills the symmetric adjacency col / sym2e from what the build kept
// (once per handle; no-op when filled).  tc_build.hip.
tc_status tc_ensure_symmetric(tc_graph *g, hipStream_t s);
// Frees lt_key / lt_val (no-op when gone).  tc_build.hip.
void tc_release_transposition(tc_graph *g, hipStream_t s);
tc_status tc_alg_numerator(const tc_graph *g, uint64_t *d_num, hipStream_t s);  // tc_algebraic.hip
tc_status tc_work_stats(tc_graph *g, int64_t *stats, hipStream_t s);
tc_status tc_mid_prepare(tc_graph *g, hipStream_t s);
tc_status tc_count_mid(tc_graph *g, const tc_tuning &t, int lds_limit, int max_entries,
                       unsigned long long *found, hipStream_t s);
tc_status tc_mid_stats(tc_graph *g, unsigned long long *acc, hipStream_t s);
// Words of the middle pivot's bit matrices, Σ_r Σ_{t<|N_H(r)|} ceil(t/32)
// (device reduction and one read-back; the stored total once they exist).
tc_status tc_mid_bit_words(const tc_graph *g, int64_t *words, hipStream_t s);
// Upper bound of the device bytes tc_count + tc_aggregate allocate beyond
// what g holds, for the pivot form the tuning (or AUTO) picks.
tc_status tc_count_bytes(tc_graph *g, const tc_tuning *tuning, hipStream_t s, int64_t *bytes);

template <typename T>
tc_status tc_graph_alloc(tc_graph *g, T **p, int64_t count, hipStream_t s) {
    tc_status st = tc_alloc(p, count, s);
    if (st == TC_OK) g->bytes += (size_t)(count > 0 ? count : 1) * sizeof(T);
    return st;
}

// ---------------------------------------------------------------------------
// Device-side helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tc_lane() { return __lane_id(); }

__device__ __forceinline__ uint64_t tc_lanemask_lt() {
    int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T tc_wave_sum(T x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, TC_WAVE);
    return x;
}

// Maximum across the 64 lanes of a wavefront.
template <typename T>
__device__ __forceinline__ T tc_wave_max(T x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T y = __shfl_xor(x, off, TC_WAVE);
        x = y > x ? y : x;
    }
    return x;
}

// Inclusive scan across the 64 lanes of a wavefront.
template <typename T>
__device__ __forceinline__ T tc_wave_incl_scan(T x) {
    int l = __lane_id();
#pragma unroll
    for (int off = 1; off < TC_WAVE; off <<= 1) {
        T y = __shfl_up(x, off, TC_WAVE);
        if (l >= off) x += y;
    }
    return x;
}
