// The extern "C" boundary of libtc (declared in include/tc.h): argument
// checks, host/device staging, handle lifetime, and the order of stages.
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>

#include "tc_internal.h"

#define TC_VERSION 10000

// ---------------------------------------------------------------------------
// Memory
// ---------------------------------------------------------------------------
tc_status tc_map_hip_error(hipError_t e) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return TC_ERR_OOM;
    return TC_ERR_DEVICE;
}

// read by compute calls that may run on several host threads at once
static std::atomic<bool> g_profiling{false};

bool tc_profiling_on() { return g_profiling.load(std::memory_order_relaxed); }

void tc_prof_mark(tc_graph *g, int idx, hipStream_t s) {
    if (!g->prof || idx < 0 || idx >= TC_PROF_MARKS) return;
    if (!g->prof_ev[idx] && hipEventCreate(&g->prof_ev[idx]) != hipSuccess) {
        g->prof_ev[idx] = nullptr;
        return;
    }
    (void)hipEventRecord(g->prof_ev[idx], s);
    if (idx == 3) g->prof_build = true;
    if (idx == 11) g->prof_compute = true;
}

// ---------------------------------------------------------------------------
// Device memory: a caching allocator of the library's own.
//
// Blocks come from hipMalloc and, once freed, stay cached per device in a
// best-fit free list (sizes rounded to 512 B below 1 MiB and to 2 MiB
// above; a block is reused for requests of at least half its size).  A free
// records an event on the freeing stream; a reuse on the same stream needs
// nothing (stream order), a reuse on another stream waits for that event.
// So repeated builds of similar graphs allocate nothing new, without the
// trimming and regrowth of the runtime's stream-ordered pool, whose regrowth
// stalled builds by seconds.  tc_trim_memory() returns cached blocks.
// ---------------------------------------------------------------------------
namespace {

struct Block {
    size_t size = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    int device = 0;
};

constexpr int MAX_DEV = 64;
std::mutex g_alloc_mu;
std::multimap<size_t, std::pair<void *, Block>> g_free[MAX_DEV];
std::unordered_map<void *, Block> g_used;
// bytes per device: held (in use + cached), in use, their peaks, and the
// caller's limit on held bytes (0: none)
int64_t g_held[MAX_DEV], g_in_use[MAX_DEV], g_peak_held[MAX_DEV], g_peak_in_use[MAX_DEV];
int64_t g_limit = 0;

size_t round_size(size_t b) {
    if (b < ((size_t)1 << 20)) return (b + 511) & ~(size_t)511;
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

// Frees the cached blocks of one device (caller holds the lock).
void release_cached(int dev) {
    for (auto &kv : g_free[dev]) {
        Block &b = kv.second.second;
        if (b.ev) {
            (void)hipEventSynchronize(b.ev);
            (void)hipEventDestroy(b.ev);
        }
        (void)hipFree(kv.second.first);
        g_held[dev] -= (int64_t)b.size;
    }
    g_free[dev].clear();
}

void note_in_use(int dev, int64_t delta) {
    g_in_use[dev] += delta;
    if (g_in_use[dev] > g_peak_in_use[dev]) g_peak_in_use[dev] = g_in_use[dev];
}

}  // namespace

tc_status tc_dev_alloc(void **p, size_t bytes, hipStream_t s) {
    int dev = 0;
    TC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEV) return TC_ERR_DEVICE;
    *p = nullptr;
    const size_t size = round_size(bytes > 0 ? bytes : 1);
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto &fl = g_free[dev];
    auto it = fl.lower_bound(size);
    // a cached block up to twice the size is reused; under a limit only up
    // to 1/16 more, so that held blocks track the sizes callers budget for
    const size_t reuse_max = g_limit > 0 ? size + size / 16 : 2 * size;
    if (it != fl.end() && it->first <= reuse_max) {
        void *ptr = it->second.first;
        Block b = it->second.second;
        fl.erase(it);
        if (b.stream != s && b.ev) TC_HIP(hipStreamWaitEvent(s, b.ev, 0));
        b.stream = s;
        g_used[ptr] = b;
        note_in_use(dev, (int64_t)b.size);
        *p = ptr;
        return TC_OK;
    }
    if (g_limit > 0 && g_held[dev] + (int64_t)size > g_limit) {
        release_cached(dev);  // cached blocks count against the limit: give them back first
        if (g_held[dev] + (int64_t)size > g_limit) return TC_ERR_BUDGET;
    }
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, size);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_cached(dev);  // give the cache back and try once more
        e = hipMalloc(&ptr, size);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return tc_map_hip_error(e);
        }
    }
    Block b;
    b.size = size;
    b.stream = s;
    b.device = dev;
    g_used[ptr] = b;
    g_held[dev] += (int64_t)size;
    if (g_held[dev] > g_peak_held[dev]) g_peak_held[dev] = g_held[dev];
    note_in_use(dev, (int64_t)size);
    *p = ptr;
    return TC_OK;
}

void tc_dev_free(void *p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_used.find(p);
    if (it == g_used.end()) return;
    Block b = it->second;
    g_used.erase(it);
    if (!b.ev && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) b.ev = nullptr;
    if (b.ev) (void)hipEventRecord(b.ev, s);
    b.stream = s;
    note_in_use(b.device, -(int64_t)b.size);
    g_free[b.device].emplace(b.size, std::make_pair(p, b));
}

// ---------------------------------------------------------------------------
// Small kernels of the boundary
// ---------------------------------------------------------------------------
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

__global__ void k_widen(const uint32_t *__restrict__ a, int64_t n, uint64_t *__restrict__ out) {
    GRID_STRIDE(i, n) out[i] = a[i];
}

// CSR -> pairs: entry k belongs to the last row v with row_ptr[v] <= k.
__global__ void k_csr_check(const int64_t *__restrict__ rp, int32_t n, uint32_t *__restrict__ err) {
    GRID_STRIDE(v, n) {
        if (rp[v + 1] < rp[v]) atomicOr(err, 1u);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && rp[0] != 0) atomicOr(err, 1u);
}

__global__ void k_csr_expand(const int64_t *__restrict__ rp, int32_t n, int64_t nnz,
                             int32_t *__restrict__ src) {
    GRID_STRIDE(k, nnz) {
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            int32_t mid = (int32_t)(((int64_t)lo + hi + 1) >> 1);
            if (rp[mid] <= k) lo = mid; else hi = mid - 1;
        }
        src[k] = lo;
    }
}

// tc ≥ 0, so the bit pattern orders like the value; the complement sorts
// descending, and a stable sort over id order breaks ties by smaller id.
__global__ void k_topk_keys(const double *__restrict__ tcv, int32_t n, uint64_t *__restrict__ key,
                            uint32_t *__restrict__ id) {
    GRID_STRIDE(v, n) {
        key[v] = ~(uint64_t)__double_as_longlong(tcv[v]);
        id[v] = (uint32_t)v;
    }
}

__global__ void k_topk_out(const uint32_t *__restrict__ id, const double *__restrict__ tcv,
                           int32_t k, int32_t *__restrict__ verts, double *__restrict__ vals) {
    GRID_STRIDE(i, k) {
        uint32_t v = id[i];
        verts[i] = (int32_t)v;
        if (vals) vals[i] = tcv[v];
    }
}

__global__ void k_edge_offsets(const int32_t *__restrict__ eu, int64_t m,
                               const int64_t *__restrict__ vtx_off, int32_t G,
                               int64_t *__restrict__ eoff) {
    GRID_STRIDE(gi, (int64_t)G + 1) {
        const int64_t first = vtx_off[gi];
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (eu[mid] < first) lo = mid + 1; else hi = mid;
        }
        eoff[gi] = lo;
    }
}

tc_status copy_out(void *dst, const void *src, size_t bytes, int32_t mem_kind, hipStream_t s) {
    if (bytes == 0) return TC_OK;
    TC_HIP(hipMemcpyAsync(dst, src, bytes,
                          mem_kind == TC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                          s));
    return TC_OK;
}

void free_graph_arrays(tc_graph *g, hipStream_t s) {
    void *arrs[] = {g->eu,   g->ev,   g->row_ptr, g->col,  g->sym2e, g->rank, g->perm,
                    g->orp,  g->ocol, g->o2e,     g->osup, g->esup,  g->flag, g->tri,
                    g->num,  g->tcv,  g->triG,    g->vtx_off, g->err, g->bin_rows,
                    g->in_ptr, g->in_pair, g->rowbase, g->hitbits, g->orow,
                    g->run_us, g->lt_key, g->lt_val, g->ocol16, g->rowinfo};
    for (void *p : arrs) tc_dev_free(p, s);
}

tc_status new_graph(int32_t n, int32_t num_graphs, tc_graph **out) {
    tc_graph *g = new (std::nothrow) tc_graph();
    if (!g) return TC_ERR_OOM;
    TC_HIP(hipGetDevice(&g->device));
    g->n = n;
    g->num_graphs = num_graphs;
    g->prof = tc_profiling_on();
    int b = tc_bits_for(n > 1 ? (uint64_t)(n - 1) : 1);
    g->bits = b < 1 ? 1 : b;
    *out = g;
    return TC_OK;
}

tc_status finish_build(tc_graph *g, hipStream_t s) {
    TC_TRY(tc_orient(g, s));
    return TC_OK;
}

tc_status build_common(tc_graph *g, const int32_t *src, const int32_t *dst, int64_t P,
                       int32_t mem_kind, const int64_t *h_pair_off, hipStream_t s) {
    tc_scratch tmp(s);
    tc_prof_mark(g, 0, s);
    const int32_t *d_src = src, *d_dst = dst;
    if (mem_kind == TC_MEM_HOST && P > 0) {
        int32_t *a = nullptr, *b = nullptr;
        TC_TRY(tmp.get(&a, P));
        TC_TRY(tmp.get(&b, P));
        TC_HIP(hipMemcpyAsync(a, src, sizeof(int32_t) * P, hipMemcpyHostToDevice, s));
        TC_HIP(hipMemcpyAsync(b, dst, sizeof(int32_t) * P, hipMemcpyHostToDevice, s));
        d_src = a;
        d_dst = b;
    }
    int64_t *d_pair_off = nullptr;
    if (h_pair_off) {
        TC_TRY(tmp.get(&d_pair_off, g->num_graphs + 1));
        TC_HIP(hipMemcpyAsync(d_pair_off, h_pair_off, sizeof(int64_t) * (g->num_graphs + 1),
                              hipMemcpyHostToDevice, s));
    }
    TC_TRY(tc_build_from_pairs(g, d_src, d_dst, P, g->vtx_off, d_pair_off, g->num_graphs, s));
    TC_TRY(finish_build(g, s));
    return TC_OK;
}

bool valid_kind(int32_t k) { return k == TC_MEM_HOST || k == TC_MEM_DEVICE; }

}  // namespace

// ---------------------------------------------------------------------------
// Public entry points
// ---------------------------------------------------------------------------
extern "C" {

int32_t tc_version(void) { return TC_VERSION; }

const char *tc_status_string(int32_t s) {
    switch (s) {
        case TC_OK: return "ok";
        case TC_TRIANGLE_FREE: return "triangle-free graph: TC is 0 everywhere";
        case TC_ERR_INVALID_ARG: return "invalid argument";
        case TC_ERR_VERTEX_RANGE: return "vertex id outside [0, n)";
        case TC_ERR_OOM: return "device out of memory";
        case TC_ERR_DEVICE: return "HIP runtime error";
        case TC_ERR_OVERFLOW: return "result does not fit its integer type";
        case TC_ERR_BUDGET: return "request exceeds the memory budget";
        case TC_ERR_NOT_COMPUTED: return "results requested before tc_compute";
        case TC_ERR_UNSUPPORTED: return "size beyond the library's index types";
        case TC_ERR_IO: return "file cannot be opened, mapped or read";
        default: return "unknown status";
    }
}

tc_status tc_graph_from_edges(const int32_t *src, const int32_t *dst, int64_t num_pairs, int32_t n,
                              int32_t mem_kind, void *stream, tc_graph **out) {
    if (!out) return TC_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 0 || num_pairs < 0 || !valid_kind(mem_kind)) return TC_ERR_INVALID_ARG;
    if (num_pairs > 0 && (!src || !dst)) return TC_ERR_INVALID_ARG;
    if (num_pairs >= (int64_t)0xFFFFFFFFll) return TC_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    tc_graph *g = nullptr;
    TC_TRY(new_graph(n, 1, &g));
    g->last_stream = s;
    tc_status st = build_common(g, src, dst, num_pairs, mem_kind, nullptr, s);
    if (st < 0) {
        tc_graph_destroy(g);
        return st;
    }
    *out = g;
    return TC_OK;
}

tc_status tc_graph_from_csr(const int64_t *row_ptr, const int32_t *col, int32_t n,
                            int32_t mem_kind, int32_t assume_simple_sorted, void *stream,
                            tc_graph **out) {
    if (!out) return TC_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 0 || !row_ptr || !valid_kind(mem_kind)) return TC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    tc_scratch tmp(s);
    const int64_t *d_rp = row_ptr;
    int64_t nnz = 0;
    if (mem_kind == TC_MEM_HOST) {
        if (row_ptr[0] != 0) return TC_ERR_INVALID_ARG;
        for (int32_t v = 0; v < n; ++v)
            if (row_ptr[v + 1] < row_ptr[v]) return TC_ERR_INVALID_ARG;
        nnz = row_ptr[n];
        int64_t *a = nullptr;
        TC_TRY(tmp.get(&a, (int64_t)n + 1));
        TC_HIP(hipMemcpyAsync(a, row_ptr, sizeof(int64_t) * ((int64_t)n + 1), hipMemcpyHostToDevice, s));
        d_rp = a;
    } else {
        uint32_t *err = nullptr;
        TC_TRY(tmp.get(&err, 1));
        TC_HIP(hipMemsetAsync(err, 0, 4, s));
        k_csr_check<<<grid_for(n > 0 ? n : 1), BK, 0, s>>>(d_rp, n, err);
        TC_LAUNCHED();
        uint32_t h_err = 0;
        TC_HIP(hipMemcpyAsync(&h_err, err, 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipMemcpyAsync(&nnz, d_rp + n, 8, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        if (h_err) return TC_ERR_INVALID_ARG;
    }
    if (nnz < 0) return TC_ERR_INVALID_ARG;
    if (nnz > 0 && !col) return TC_ERR_INVALID_ARG;
    if (nnz >= (int64_t)0xFFFFFFFFll) return TC_ERR_UNSUPPORTED;
    const int32_t *d_col = col;
    if (mem_kind == TC_MEM_HOST && nnz > 0) {
        int32_t *c = nullptr;
        TC_TRY(tmp.get(&c, nnz));
        TC_HIP(hipMemcpyAsync(c, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
        d_col = c;
    }
    int32_t *d_src = nullptr;
    if (nnz > 0 && !assume_simple_sorted) {
        TC_TRY(tmp.get(&d_src, nnz));
        k_csr_expand<<<grid_for(nnz), BK, 0, s>>>(d_rp, n, nnz, d_src);
        TC_LAUNCHED();
    }
    tc_graph *g = nullptr;
    TC_TRY(new_graph(n, 1, &g));
    g->last_stream = s;
    tc_prof_mark(g, 0, s);
    tc_status st = assume_simple_sorted
                       ? tc_build_from_pairs(g, nullptr, nullptr, 0, nullptr, nullptr, 1, s, d_rp,
                                             d_col)
                       : tc_build_from_pairs(g, d_src, d_col, nnz, nullptr, nullptr, 1, s);
    if (st >= 0) st = finish_build(g, s);
    if (st < 0) {
        tc_graph_destroy(g);
        return st;
    }
    *out = g;
    return TC_OK;
}

tc_status tc_batch_create(const int32_t *src, const int32_t *dst, const int64_t *graph_pair_off,
                          const int64_t *graph_vtx_off, int32_t num_graphs, int32_t mem_kind,
                          void *stream, tc_graph **out) {
    if (!out) return TC_ERR_INVALID_ARG;
    *out = nullptr;
    if (num_graphs < 1 || !graph_pair_off || !graph_vtx_off || !valid_kind(mem_kind))
        return TC_ERR_INVALID_ARG;
    if (graph_pair_off[0] != 0 || graph_vtx_off[0] != 0) return TC_ERR_INVALID_ARG;
    for (int32_t i = 0; i < num_graphs; ++i)
        if (graph_pair_off[i + 1] < graph_pair_off[i] || graph_vtx_off[i + 1] < graph_vtx_off[i])
            return TC_ERR_INVALID_ARG;
    const int64_t P = graph_pair_off[num_graphs];
    const int64_t N = graph_vtx_off[num_graphs];
    if (N > 0x7FFFFFFFll - 1) return TC_ERR_UNSUPPORTED;
    if (P >= (int64_t)0xFFFFFFFFll) return TC_ERR_UNSUPPORTED;
    if (P > 0 && (!src || !dst)) return TC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    tc_graph *g = nullptr;
    TC_TRY(new_graph((int32_t)N, num_graphs, &g));
    g->last_stream = s;
    tc_status st = TC_OK;
    g->h_vtx_off = (int64_t *)malloc(sizeof(int64_t) * (num_graphs + 1));
    g->h_edge_off = (int64_t *)calloc(num_graphs + 1, sizeof(int64_t));
    if (!g->h_vtx_off || !g->h_edge_off) st = TC_ERR_OOM;
    if (st == TC_OK) {
        memcpy(g->h_vtx_off, graph_vtx_off, sizeof(int64_t) * (num_graphs + 1));
        st = tc_graph_alloc(g, &g->vtx_off, num_graphs + 1, s);
    }
    if (st == TC_OK) {
        hipError_t e = hipMemcpyAsync(g->vtx_off, graph_vtx_off, sizeof(int64_t) * (num_graphs + 1),
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) st = tc_map_hip_error(e);
    }
    if (st == TC_OK) st = build_common(g, src, dst, P, mem_kind, graph_pair_off, s);
    if (st == TC_OK) {
        // canonical edges are sorted by their smaller (global) end, so graph
        // gi's edges start at the first edge whose smaller end is >= its
        // first vertex
        tc_scratch tmp(s);
        int64_t *d_eoff = nullptr;
        st = tmp.get(&d_eoff, num_graphs + 1);
        if (st == TC_OK) {
            k_edge_offsets<<<grid_for(num_graphs + 1), BK, 0, s>>>(g->eu, g->m, g->vtx_off,
                                                                   num_graphs, d_eoff);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess)
                e = hipMemcpyAsync(g->h_edge_off, d_eoff, sizeof(int64_t) * (num_graphs + 1),
                                   hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = tc_map_hip_error(e);
        }
    }
    if (st < 0) {
        tc_graph_destroy(g);
        return st;
    }
    *out = g;
    return TC_OK;
}

int32_t tc_num_graphs(const tc_graph *g) { return g ? g->num_graphs : -1; }

tc_status tc_batch_edge_offsets(const tc_graph *g, int64_t *edge_off) {
    if (!g || !edge_off) return TC_ERR_INVALID_ARG;
    if (g->num_graphs == 1 && !g->h_edge_off) {
        edge_off[0] = 0;
        edge_off[1] = g->m;
        return TC_OK;
    }
    memcpy(edge_off, g->h_edge_off, sizeof(int64_t) * (g->num_graphs + 1));
    return TC_OK;
}

tc_status tc_compute_tuned(tc_graph *g, const tc_tuning *tuning, void *stream) {
    if (!g) return TC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    g->last_stream = s;
    g->computed = false;
    g->prof_compute = false;
    g->prof = tc_profiling_on();  // the switch as it stands when this compute starts
    tc_prof_mark(g, 4, s);
    TC_TRY(tc_count(g, tuning, s));
    TC_TRY(tc_aggregate(g, s));
    uint32_t h_err = 0;
    uint64_t tg = 0;
    TC_HIP(hipMemcpyAsync(&h_err, g->err, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(&tg, g->triG, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h_err & 8u) return TC_ERR_OVERFLOW;
    if (h_err) return TC_ERR_DEVICE;  // an internal parity check failed
    g->computed = true;
    g->status = (g->num_graphs == 1 && tg == 0) ? TC_TRIANGLE_FREE : TC_OK;
    return (tc_status)g->status;
}

tc_status tc_compute(tc_graph *g, void *stream) { return tc_compute_tuned(g, nullptr, stream); }

int64_t tc_num_vertices(const tc_graph *g) { return g ? g->n : -1; }
int64_t tc_num_edges(const tc_graph *g) { return g ? g->m : -1; }

tc_status tc_get_edges(const tc_graph *g, int32_t *u, int32_t *v, int32_t mem_kind, void *stream) {
    if (!g || !valid_kind(mem_kind)) return TC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (u) TC_TRY(copy_out(u, g->eu, sizeof(int32_t) * g->m, mem_kind, s));
    if (v) TC_TRY(copy_out(v, g->ev, sizeof(int32_t) * g->m, mem_kind, s));
    if (mem_kind == TC_MEM_HOST) TC_HIP(hipStreamSynchronize(s));
    return TC_OK;
}

tc_status tc_numerator_algebraic(const tc_graph *g, uint64_t *num, int32_t mem_kind, void *stream) {
    if (!g || !num || !valid_kind(mem_kind)) return TC_ERR_INVALID_ARG;
    if (!g->computed) return TC_ERR_NOT_COMPUTED;
    hipStream_t s = (hipStream_t)stream;
    if (g->n == 0) return TC_OK;
    tc_scratch tmp(s);
    uint64_t *dst = num;
    if (mem_kind == TC_MEM_HOST) TC_TRY(tmp.get(&dst, g->n));
    TC_TRY(tc_alg_numerator(g, dst, s));
    if (mem_kind == TC_MEM_HOST) {
        TC_TRY(copy_out(num, dst, sizeof(uint64_t) * g->n, mem_kind, s));
        TC_HIP(hipStreamSynchronize(s));
    }
    return TC_OK;
}

tc_status tc_get_results(const tc_graph *g, uint64_t *tri, uint64_t *support, uint64_t *triG,
                         uint64_t *num, double *tc, int32_t mem_kind, void *stream) {
    if (!g || !valid_kind(mem_kind)) return TC_ERR_INVALID_ARG;
    if (!g->computed) return TC_ERR_NOT_COMPUTED;
    hipStream_t s = (hipStream_t)stream;
    tc_scratch tmp(s);
    if (tri) TC_TRY(copy_out(tri, g->tri, sizeof(uint64_t) * g->n, mem_kind, s));
    if (num) TC_TRY(copy_out(num, g->num, sizeof(uint64_t) * g->n, mem_kind, s));
    if (tc) TC_TRY(copy_out(tc, g->tcv, sizeof(double) * g->n, mem_kind, s));
    if (triG) TC_TRY(copy_out(triG, g->triG, sizeof(uint64_t) * g->num_graphs, mem_kind, s));
    if (support && g->m > 0) {
        uint64_t *dst = support;
        if (mem_kind == TC_MEM_HOST) TC_TRY(tmp.get(&dst, g->m));
        k_widen<<<grid_for(g->m), BK, 0, s>>>(g->esup, g->m, dst);
        TC_LAUNCHED();
        if (mem_kind == TC_MEM_HOST) TC_TRY(copy_out(support, dst, sizeof(uint64_t) * g->m, mem_kind, s));
    }
    if (mem_kind == TC_MEM_HOST) TC_HIP(hipStreamSynchronize(s));
    return TC_OK;
}

tc_status tc_batch_get_results(const tc_graph *b, uint64_t *tri, uint64_t *support, uint64_t *triG,
                               uint64_t *num, double *tc, int32_t mem_kind, void *stream) {
    return tc_get_results(b, tri, support, triG, num, tc, mem_kind, stream);
}

tc_status tc_graph_device_bytes(const tc_graph *g, int64_t *bytes) {
    if (!g || !bytes) return TC_ERR_INVALID_ARG;
    *bytes = (int64_t)g->bytes;
    return TC_OK;
}

int64_t tc_estimate_device_bytes(int64_t P, int32_t n) {
    if (P < 0 || n < 0) return -1;
    // resident: edges 8m, sym CSR 8(n+1) + 16m (filled on demand), ranks
    // 8n, oriented 8(n+1) + 8m (+ 2m for its 16-bit copy, 16n for the
    // per-row records of the middle pivot), supports 8m,
    // flags 2m, results 24n; peak temporaries of the build: pair keys 16P +
    // flags 4P (+ staged host pairs 8P).  The middle pivot's transposition
    // (8m) and bit matrices (one bit per oriented wedge) reuse the build's
    // temporaries; denser graphs need more for the bits (see the header).
    const int64_t m = P;
    return 8 * m + 8 * (int64_t)n + 16 * m + 8 * (int64_t)n + 8 * (int64_t)n + 8 * m + 2 * m +
           8 * m + 2 * m + 24 * (int64_t)n + 16 * (int64_t)n + 28 * P + (64ll << 20);
}

void tc_graph_destroy(tc_graph *g) {
    if (!g) return;
    hipStream_t s = g->last_stream;
    free_graph_arrays(g, s);
    (void)hipStreamSynchronize(s);
    for (int i = 0; i < TC_PROF_MARKS; ++i)
        if (g->prof_ev[i]) (void)hipEventDestroy(g->prof_ev[i]);
    free(g->h_vtx_off);
    free(g->h_edge_off);
    delete g;
}

tc_status tc_top_k(const tc_graph *g, int32_t k, int32_t *vertices, double *values, int32_t *k_out,
                   int32_t mem_kind, void *stream) {
    if (!g || k < 0 || !vertices || !valid_kind(mem_kind)) return TC_ERR_INVALID_ARG;
    if (!g->computed) return TC_ERR_NOT_COMPUTED;
    hipStream_t s = (hipStream_t)stream;
    const int32_t n = g->n;
    if (k > n) k = n;
    if (k_out) *k_out = k;
    if (k == 0) return TC_OK;
    tc_scratch tmp(s);
    uint64_t *key = nullptr, *key2 = nullptr;
    uint32_t *id = nullptr, *id2 = nullptr;
    TC_TRY(tmp.get(&key, n));
    TC_TRY(tmp.get(&key2, n));
    TC_TRY(tmp.get(&id, n));
    TC_TRY(tmp.get(&id2, n));
    k_topk_keys<<<grid_for(n), BK, 0, s>>>(g->tcv, n, key, id);
    TC_LAUNCHED();
    TC_TRY(tc_sort_u64_u32(&key, &id, &key2, &id2, n, 64, s));
    int32_t *dv = vertices;
    double *dval = values;
    if (mem_kind == TC_MEM_HOST) {
        TC_TRY(tmp.get(&dv, k));
        if (values) TC_TRY(tmp.get(&dval, k));
    }
    k_topk_out<<<grid_for(k), BK, 0, s>>>(id, g->tcv, k, dv, dval);
    TC_LAUNCHED();
    if (mem_kind == TC_MEM_HOST) {
        TC_TRY(copy_out(vertices, dv, sizeof(int32_t) * k, mem_kind, s));
        if (values) TC_TRY(copy_out(values, dval, sizeof(double) * k, mem_kind, s));
        TC_HIP(hipStreamSynchronize(s));
    }
    return TC_OK;
}

tc_status tc_trim_memory(void) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    int cur = 0;
    TC_HIP(hipGetDevice(&cur));
    for (int d = 0; d < MAX_DEV; ++d) {
        if (g_free[d].empty()) continue;
        if (d != cur) TC_HIP(hipSetDevice(d));
        release_cached(d);
    }
    TC_HIP(hipSetDevice(cur));
    return TC_OK;
}

tc_status tc_set_memory_limit(int64_t bytes) {
    if (bytes < 0) return TC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_limit = bytes;
    return TC_OK;
}

tc_status tc_memory_stats(int64_t *held, int64_t *in_use, int64_t *peak_held, int64_t *peak_in_use,
                          int32_t reset_peaks) {
    int dev = 0;
    TC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEV) return TC_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (held) *held = g_held[dev];
    if (in_use) *in_use = g_in_use[dev];
    if (peak_held) *peak_held = g_peak_held[dev];
    if (peak_in_use) *peak_in_use = g_peak_in_use[dev];
    if (reset_peaks) {
        g_peak_held[dev] = g_held[dev];
        g_peak_in_use[dev] = g_in_use[dev];
    }
    return TC_OK;
}

tc_status tc_compute_bytes(tc_graph *g, const tc_tuning *tuning, void *stream, int64_t *bytes) {
    if (!g || !bytes) return TC_ERR_INVALID_ARG;
    return tc_count_bytes(g, tuning, (hipStream_t)stream, bytes);
}

tc_status tc_set_profiling(int32_t on) {
    g_profiling = on != 0;
    return TC_OK;
}

tc_status tc_get_stage_ms(const tc_graph *g, double *ms) {
    if (!g || !ms) return TC_ERR_INVALID_ARG;
    if (!g->prof_build && !g->prof_compute) return TC_ERR_NOT_COMPUTED;
    static const int from[TC_NUM_STAGES] = {0, 1, 2, 4, 5, 6, 7, 8, 9, 10, 5, 12, 13, 6};
    static const int to[TC_NUM_STAGES] = {1, 2, 3, 5, 6, 7, 8, 9, 10, 11, 12, 13, 6, 14};
    for (int i = 0; i < TC_NUM_STAGES; ++i) {
        ms[i] = 0.0;
        bool build = to[i] <= 3;
        if ((build && !g->prof_build) || (!build && !g->prof_compute)) continue;
        // launches of the middle pivot's count: none after the low pivot
        if (i >= TC_STAGE_COUNT_LIGHT_GROUPS && g->algo_used == TC_ALGO_LOW_PIVOT) continue;
        hipEvent_t a = g->prof_ev[from[i]], b = g->prof_ev[to[i]];
        if (!a || !b) continue;
        TC_HIP(hipEventSynchronize(b));
        float t = 0.f;
        TC_HIP(hipEventElapsedTime(&t, a, b));
        ms[i] = t;
    }
    return TC_OK;
}

tc_status tc_get_work_stats(tc_graph *g, int64_t *stats, void *stream) {
    if (!g || !stats) return TC_ERR_INVALID_ARG;
    return tc_work_stats(g, stats, (hipStream_t)stream);
}

}  // extern "C"
