// Ingest of graphs given as text edge lists with arbitrary vertex ids.
//
// The paper's inputs are SNAP graphs stored as text, one "u v" pair per
// line, with the vertices relabelled to 1..n without gaps (Sec.
// "Comparison"; Table 6).  Two steps bring such a file to the form the
// rest of the library takes (int32 ids 0..n-1, n explicit):
//
//  * tc_edge_text_read (host): the file is mapped and split into one chunk
//    per thread at line boundaries.  Every thread counts its pair lines,
//    a prefix over the counts places each chunk, and every thread then
//    parses its chunk into the caller's int64 arrays.  Lines that are empty
//    or start with '#' or '%' are skipped; further columns on a line are
//    ignored.
//  * tc_relabel_ids (device): the 2P ids are radix-sorted (on the bits the
//    largest id needs) and deduplicated; each id is replaced by its rank
//    among the distinct ids, found by binary search.  The map preserves
//    order, so the relabelled graph lists its vertices in the order of
//    their original ids, and the sorted distinct ids translate back.
#include <fcntl.h>
#include <string.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <thread>
#include <vector>

#include "tc_internal.h"

namespace {

constexpr int BK = 256;

static inline unsigned grid_for(int64_t n, int block = BK) {
    int64_t g = tc_div_up(n, block);
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Text parsing (host)
// ---------------------------------------------------------------------------
inline bool is_space(char c) { return c == ' ' || c == '\t' || c == '\r' || c == '\f' || c == '\v'; }

// Parses one unsigned decimal integer at p (p < e).  Returns false if there
// is no digit or the value does not fit 63 bits.
inline bool parse_id(const char *&p, const char *e, int64_t *out) {
    if (p >= e || *p < '0' || *p > '9') return false;
    uint64_t v = 0;
    while (p < e && *p >= '0' && *p <= '9') {
        v = v * 10 + (uint64_t)(*p - '0');
        if (v > (uint64_t)INT64_MAX) return false;
        ++p;
    }
    *out = (int64_t)v;
    return true;
}

// Result of one line: 0 = skipped (blank or comment), 1 = a pair, -1 = malformed.
inline int parse_line(const char *p, const char *e, int64_t *u, int64_t *v) {
    while (p < e && is_space(*p)) ++p;
    if (p == e || *p == '#' || *p == '%') return 0;
    if (!parse_id(p, e, u)) return -1;
    if (p == e || !is_space(*p)) return -1;
    while (p < e && is_space(*p)) ++p;
    if (!parse_id(p, e, v)) return -1;
    if (p < e && !is_space(*p)) return -1;
    return 1;
}

struct Chunk {
    const char *b, *e;
    int64_t pairs = 0, lines = 0, bad_line = -1;
};

// Walks the lines of a chunk; with out arrays, writes the pairs from `at`.
void walk(Chunk &c, int64_t *src, int64_t *dst, int64_t at) {
    const char *p = c.b;
    int64_t line = 0;
    while (p < c.e) {
        const char *q = static_cast<const char *>(memchr(p, '\n', (size_t)(c.e - p)));
        const char *le = q ? q : c.e;
        int64_t u = 0, v = 0;
        const int r = parse_line(p, le, &u, &v);
        if (r < 0) {
            if (c.bad_line < 0) c.bad_line = line;
        } else if (r == 1) {
            if (src) {
                src[at + c.pairs] = u;
                dst[at + c.pairs] = v;
            }
            ++c.pairs;
        }
        ++line;
        p = q ? q + 1 : c.e;
    }
    c.lines = line;
}

// ---------------------------------------------------------------------------
// Relabelling (device)
// ---------------------------------------------------------------------------
__global__ void k_ids_concat(const int64_t *__restrict__ src, const int64_t *__restrict__ dst,
                             int64_t P, uint64_t *__restrict__ keys,
                             unsigned long long *__restrict__ maxv, uint32_t *__restrict__ err) {
    unsigned long long mx = 0;
    bool neg = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = src[i], b = dst[i];
        neg |= (a < 0) | (b < 0);
        keys[i] = (uint64_t)a;
        keys[P + i] = (uint64_t)b;
        const unsigned long long h = (unsigned long long)(a > b ? a : b);
        mx = h > mx ? h : mx;
    }
    mx = tc_wave_max(mx);
    if (__lane_id() == 0 && mx) atomicMax(maxv, mx);
    if (neg) atomicOr(err, 1u);
}

__global__ void k_first_flags(const uint64_t *__restrict__ keys, int64_t n,
                              uint32_t *__restrict__ f) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        f[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_first_write(const uint64_t *__restrict__ keys, int64_t n,
                              const uint32_t *__restrict__ f, const uint32_t *__restrict__ pos,
                              int64_t *__restrict__ uniq) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (f[i]) uniq[pos[i]] = (int64_t)keys[i];
}

__global__ void k_ids_map(const int64_t *__restrict__ src, const int64_t *__restrict__ dst,
                          int64_t P, const int64_t *__restrict__ uniq, int64_t nu,
                          int32_t *__restrict__ s32, int32_t *__restrict__ d32) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * P;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i < P ? src[i] : dst[i - P];
        int64_t lo = 0, hi = nu - 1;  // x is present: the first uniq[k] >= x is x
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (uniq[mid] < x) lo = mid + 1; else hi = mid;
        }
        if (i < P) s32[i] = (int32_t)lo; else d32[i - P] = (int32_t)lo;
    }
}

tc_status copy(void *dst, const void *src, size_t bytes, hipMemcpyKind k, hipStream_t s) {
    if (bytes == 0) return TC_OK;
    TC_HIP(hipMemcpyAsync(dst, src, bytes, k, s));
    return TC_OK;
}

}  // namespace

extern "C" {

tc_status tc_edge_text_read(const char *path, int64_t *src, int64_t *dst, int64_t capacity,
                            int64_t *num_pairs, int64_t *bad_line, int32_t nthreads) {
    if (!path || !num_pairs || capacity < 0 || ((src == nullptr) != (dst == nullptr)))
        return TC_ERR_INVALID_ARG;
    *num_pairs = 0;
    if (bad_line) *bad_line = -1;
    const int fd = open(path, O_RDONLY);
    if (fd < 0) return TC_ERR_IO;
    struct stat st;
    if (fstat(fd, &st) != 0) {
        close(fd);
        return TC_ERR_IO;
    }
    const size_t size = (size_t)st.st_size;
    if (size == 0) {
        close(fd);
        return TC_OK;
    }
    void *map = mmap(nullptr, size, PROT_READ, MAP_PRIVATE, fd, 0);
    close(fd);
    if (map == MAP_FAILED) return TC_ERR_IO;
    const char *base = static_cast<const char *>(map);
    const char *end = base + size;

    int T = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
    if (T < 1) T = 1;
    if (T > 256) T = 256;
    if ((size_t)T > size / 4096 + 1) T = (int)(size / 4096 + 1);
    // chunk boundaries just after a newline
    std::vector<Chunk> ch(T);
    const char *cur = base;
    for (int t = 0; t < T; ++t) {
        ch[t].b = cur;
        const char *cut = t == T - 1 ? end : base + (size * (size_t)(t + 1)) / (size_t)T;
        if (cut < cur) cut = cur;
        if (cut < end) {
            const char *q = static_cast<const char *>(memchr(cut, '\n', (size_t)(end - cut)));
            cut = q ? q + 1 : end;
        }
        ch[t].e = cut;
        cur = cut;
    }
    auto run = [&](int64_t *s, int64_t *d, const std::vector<int64_t> &at) {
        std::vector<std::thread> th;
        for (int t = 1; t < T; ++t) th.emplace_back([&, t] { ch[t].pairs = 0; walk(ch[t], s, d, at[t]); });
        ch[0].pairs = 0;
        walk(ch[0], s, d, at[0]);
        for (auto &x : th) x.join();
    };
    std::vector<int64_t> at(T, 0);
    run(nullptr, nullptr, at);
    int64_t total = 0, lines_before = 0;
    int64_t first_bad = -1;
    for (int t = 0; t < T; ++t) {
        at[t] = total;
        total += ch[t].pairs;
        if (first_bad < 0 && ch[t].bad_line >= 0) first_bad = lines_before + ch[t].bad_line;
        lines_before += ch[t].lines;
    }
    tc_status r = TC_OK;
    *num_pairs = total;
    if (first_bad >= 0) {
        if (bad_line) *bad_line = first_bad + 1;  // 1-based line number
        r = TC_ERR_INVALID_ARG;
    } else if (src) {
        if (capacity < total) r = TC_ERR_INVALID_ARG;
        else run(src, dst, at);
    }
    munmap(map, size);
    return r;
}

tc_status tc_relabel_ids(const int64_t *src, const int64_t *dst, int64_t num_pairs, int32_t *src32,
                         int32_t *dst32, int64_t *ids, int64_t *n_out, int32_t mem_kind,
                         void *stream) {
    if (num_pairs < 0 || !n_out || (num_pairs > 0 && (!src || !dst || !src32 || !dst32)) ||
        (mem_kind != TC_MEM_HOST && mem_kind != TC_MEM_DEVICE))
        return TC_ERR_INVALID_ARG;
    *n_out = 0;
    if (num_pairs == 0) return TC_OK;
    if (2 * num_pairs >= (int64_t)0xFFFFFFFFll) return TC_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const bool host = mem_kind == TC_MEM_HOST;
    const int64_t P = num_pairs, N2 = 2 * num_pairs;
    tc_scratch tmp(s);
    const int64_t *d_src = src, *d_dst = dst;
    if (host) {
        int64_t *a = nullptr, *b = nullptr;
        TC_TRY(tmp.get(&a, P));
        TC_TRY(tmp.get(&b, P));
        TC_TRY(copy(a, src, sizeof(int64_t) * P, hipMemcpyHostToDevice, s));
        TC_TRY(copy(b, dst, sizeof(int64_t) * P, hipMemcpyHostToDevice, s));
        d_src = a;
        d_dst = b;
    }
    uint64_t *keys = nullptr, *keys2 = nullptr;
    uint32_t *f = nullptr, *pos = nullptr, *tot = nullptr, *err = nullptr;
    unsigned long long *maxv = nullptr;
    int64_t *uniq = nullptr;
    TC_TRY(tmp.get(&keys, N2));
    TC_TRY(tmp.get(&keys2, N2));
    TC_TRY(tmp.get(&maxv, 1));
    TC_TRY(tmp.get(&err, 1));
    TC_HIP(hipMemsetAsync(maxv, 0, 8, s));
    TC_HIP(hipMemsetAsync(err, 0, 4, s));
    k_ids_concat<<<grid_for(P) < 65536 ? grid_for(P) : 65536, BK, 0, s>>>(d_src, d_dst, P, keys,
                                                                          maxv, err);
    TC_LAUNCHED();
    unsigned long long hmax = 0;
    uint32_t herr = 0;
    TC_HIP(hipMemcpyAsync(&hmax, maxv, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (herr) return TC_ERR_VERTEX_RANGE;  // negative ids
    int bits = 0;
    while (bits < 64 && (hmax >> bits) != 0) ++bits;
    TC_TRY(tc_sort_u64(&keys, &keys2, N2, bits, s));
    TC_TRY(tmp.get(&f, N2));
    TC_TRY(tmp.get(&pos, N2));
    TC_TRY(tmp.get(&tot, 1));
    k_first_flags<<<grid_for(N2), BK, 0, s>>>(keys, N2, f);
    TC_LAUNCHED();
    TC_TRY(tc_scan_u32(f, pos, N2, tot, s));
    uint32_t hn = 0;
    TC_HIP(hipMemcpyAsync(&hn, tot, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (hn > (uint32_t)INT32_MAX) return TC_ERR_UNSUPPORTED;
    TC_TRY(tmp.get(&uniq, hn));
    k_first_write<<<grid_for(N2), BK, 0, s>>>(keys, N2, f, pos, uniq);
    TC_LAUNCHED();
    int32_t *o_s = src32, *o_d = dst32;
    if (host) {
        TC_TRY(tmp.get(&o_s, P));
        TC_TRY(tmp.get(&o_d, P));
    }
    k_ids_map<<<grid_for(N2), BK, 0, s>>>(d_src, d_dst, P, uniq, hn, o_s, o_d);
    TC_LAUNCHED();
    const hipMemcpyKind out_kind = host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (host) {
        TC_TRY(copy(src32, o_s, sizeof(int32_t) * P, out_kind, s));
        TC_TRY(copy(dst32, o_d, sizeof(int32_t) * P, out_kind, s));
    }
    if (ids) TC_TRY(copy(ids, uniq, sizeof(int64_t) * hn, out_kind, s));
    TC_HIP(hipStreamSynchronize(s));
    *n_out = hn;
    return TC_OK;
}

}  // extern "C"
