/*
 * Seeded synthetic graph generators (host C, no device code).
 *
 * These produce raw undirected pair lists (src[i], dst[i]) that may contain
 * self-loops and duplicate pairs; normalisation into a simple graph is the
 * consumer's job.  Nothing here computes anything about triangles: the
 * module only draws random numbers and writes vertex ids, so that the HIP
 * library and the CPU oracle can be fed identical inputs.
 *
 * Random numbers come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used as a counter-based
 * generator: every logical stream (one R-MAT edge, one ER row, one BA graph)
 * starts from a state derived by hashing (seed, stream index), so output is
 * independent of the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t sm_next(uint64_t *s) {
    *s += 0x9E3779B97F4A7C15ULL;
    return sm_mix(*s);
}

static inline uint64_t stream_state(uint64_t seed, uint64_t stream, uint64_t salt) {
    return sm_mix(sm_mix(seed ^ (salt * 0xD1B54A32D192ED03ULL)) + stream * 0x9E3779B97F4A7C15ULL);
}

/* Uniform double in [0,1) with 53 random bits. */
static inline double sm_unit(uint64_t *s) {
    return (double)(sm_next(s) >> 11) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, bound) by Lemire's multiply-shift with rejection. */
static inline uint64_t sm_below(uint64_t *s, uint64_t bound) {
    uint64_t x = sm_next(s);
    __uint128_t mres = (__uint128_t)x * bound;
    uint64_t lo = (uint64_t)mres;
    if (lo < bound) {
        uint64_t thr = (0 - bound) % bound;
        while (lo < thr) {
            x = sm_next(s);
            mres = (__uint128_t)x * bound;
            lo = (uint64_t)mres;
        }
    }
    return (uint64_t)(mres >> 64);
}

/* ------------------------------------------------------------------------
 * Vertex scramble: a keyed bijection of [0, 2^bits).  Each round is a
 * bijection on bits-wide words (odd multiply mod 2^bits, add, xor-shift),
 * so the composition is one too.
 * ---------------------------------------------------------------------- */
typedef struct { uint64_t mask, k1, k2, k3, k4; int sh1, sh2; } scramble_t;

static void scramble_init(scramble_t *sc, int bits, uint64_t seed) {
    uint64_t s = stream_state(seed, 0, 0x5C4A3B1EULL);
    sc->mask = (bits >= 64) ? ~0ULL : ((1ULL << bits) - 1);
    sc->k1 = sm_next(&s) | 1ULL;
    sc->k2 = sm_next(&s);
    sc->k3 = sm_next(&s) | 1ULL;
    sc->k4 = sm_next(&s);
    sc->sh1 = bits / 2 + 1;
    sc->sh2 = bits / 3 + 1;
}

static inline uint64_t scramble_apply(const scramble_t *sc, uint64_t x) {
    x = (x * sc->k1 + sc->k2) & sc->mask;
    x ^= x >> sc->sh1;
    x = (x * sc->k3 + sc->k4) & sc->mask;
    x ^= x >> sc->sh2;
    x = (x * sc->k1) & sc->mask;
    return x;
}

/* ------------------------------------------------------------------------
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): every pair independently
 * descends `scale` levels of the adjacency matrix, choosing quadrant
 * (0,0),(0,1),(1,0),(1,1) with probabilities a, b, c, 1-a-b-c.  No noise.
 * Pair i uses its own SplitMix64 stream.  With `scramble` set, ids are
 * relabelled through the keyed bijection above.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t *src, *dst;
    int64_t lo, hi;
    int scale, scramble;
    uint64_t ta, tab, tabc, seed;
    const scramble_t *sc;
} rmat_job;

static void *rmat_worker(void *arg) {
    rmat_job *j = (rmat_job *)arg;
    for (int64_t i = j->lo; i < j->hi; ++i) {
        uint64_t s = stream_state(j->seed, (uint64_t)i, 0x524D4154ULL);
        uint64_t u = 0, v = 0, bits = 0;
        int have = 0;
        for (int l = 0; l < j->scale; ++l) {
            if (!have) { bits = sm_next(&s); have = 2; }
            uint64_t r = bits & 0xFFFFFFFFULL;
            bits >>= 32;
            --have;
            uint64_t rb = (r >= j->tab);
            uint64_t cb = ((r >= j->ta) && (r < j->tab)) || (r >= j->tabc);
            u = (u << 1) | rb;
            v = (v << 1) | cb;
        }
        if (j->scramble) {
            u = scramble_apply(j->sc, u);
            v = scramble_apply(j->sc, v);
        }
        j->src[i] = (int32_t)u;
        j->dst[i] = (int32_t)v;
    }
    return NULL;
}

int tcgen_rmat(int32_t *src, int32_t *dst, int64_t num_pairs, int scale,
               double a, double b, double c, uint64_t seed, int scramble,
               int nthreads) {
    if (scale < 1 || scale > 31 || num_pairs < 0) return -1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    const double two32 = 4294967296.0;
    scramble_t sc;
    scramble_init(&sc, scale, seed);
    rmat_job jobs[256];
    pthread_t th[256];
    int64_t chunk = (num_pairs + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        rmat_job *j = &jobs[t];
        j->src = src; j->dst = dst;
        j->lo = (int64_t)t * chunk;
        j->hi = j->lo + chunk < num_pairs ? j->lo + chunk : num_pairs;
        if (j->lo > j->hi) j->lo = j->hi;
        j->scale = scale; j->scramble = scramble;
        j->ta = (uint64_t)(a * two32);
        j->tab = (uint64_t)((a + b) * two32);
        j->tabc = (uint64_t)((a + b + c) * two32);
        j->seed = seed; j->sc = &sc;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, rmat_worker, &jobs[t]);
    rmat_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------------
 * Erdos-Renyi G(n, p): each unordered pair {i, j}, i < j, independently
 * with probability p.  Row i walks j = i+1.. with geometric skips
 * (Batagelj and Brandes, Phys. Rev. E 71, 2005), using its own stream.
 * Returns the number of pairs, or -(needed) if cap is too small (then the
 * output arrays hold a prefix only).  Passing cap = 0 counts.
 * ---------------------------------------------------------------------- */
int64_t tcgen_er(int32_t *src, int32_t *dst, int64_t cap, int32_t n, double p,
                 uint64_t seed) {
    if (n < 0 || p < 0 || p > 1) return -1;
    int64_t k = 0;
    if (p <= 0 || n < 2) return 0;
    const double lq = (p < 1.0) ? log1p(-p) : 0.0;
    for (int64_t i = 0; i + 1 < n; ++i) {
        uint64_t s = stream_state(seed, (uint64_t)i, 0x45520000ULL);
        int64_t j = i;
        for (;;) {
            if (p >= 1.0) {
                j += 1;
            } else {
                double r = sm_unit(&s);
                double skip = floor(log1p(-r) / lq);
                if (skip > (double)n) break;
                j += 1 + (int64_t)skip;
            }
            if (j >= n) break;
            if (k < cap) { src[k] = (int32_t)i; dst[k] = (int32_t)j; }
            ++k;
        }
    }
    return (cap > 0 && k > cap) ? -k : k;
}

/* ------------------------------------------------------------------------
 * Barabasi-Albert preferential attachment (Barabasi and Albert, Science
 * 1999) with planted cliques.
 *   - Seed graph K_{m+1} on vertices 0..m.
 *   - Each new vertex v = m+1..n-1 picks m distinct earlier targets, each
 *     draw proportional to current degree (uniform over the endpoint list).
 *   - Planted cliques: a seeded shuffle of the vertices is cut into
 *     consecutive disjoint groups of size U{kmin..kmax}; every group becomes
 *     a clique, until at least `cover` * n vertices are covered.
 * Pairs may repeat (a clique edge that BA already drew); normalisation
 * removes them.  Returns the pair count, or -(needed) if cap is too small.
 * ---------------------------------------------------------------------- */
int64_t tcgen_ba(int32_t *src, int32_t *dst, int64_t cap, int32_t n, int32_t m,
                 double cover, int32_t kmin, int32_t kmax, uint64_t seed) {
    if (n < 1 || m < 1 || kmin < 2 || kmax < kmin || cover < 0) return -1;
    if (m + 1 > n) m = n - 1;
    if (m < 1) return 0;
    uint64_t s = stream_state(seed, 0, 0x42410000ULL);
    int64_t seed_edges = (int64_t)(m + 1) * m / 2;
    int64_t ba_edges = seed_edges + (int64_t)(n - m - 1) * m;
    int64_t endp_cap = 2 * ba_edges;
    int32_t *endp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(endp_cap > 0 ? endp_cap : 1));
    int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    if (!endp || !pick) { free(endp); free(pick); return -2; }
    int64_t ne = 0, k = 0;
#define EMIT(a, b)                                          \
    do {                                                    \
        if (k < cap) { src[k] = (a); dst[k] = (b); }        \
        ++k;                                                \
    } while (0)
    for (int32_t i = 0; i <= m; ++i)
        for (int32_t j = i + 1; j <= m; ++j) {
            EMIT(i, j);
            endp[ne++] = i;
            endp[ne++] = j;
        }
    for (int32_t v = m + 1; v < n; ++v) {
        int32_t got = 0;
        while (got < m) {
            int32_t t = endp[sm_below(&s, (uint64_t)ne)];
            int dup = 0;
            for (int32_t q = 0; q < got; ++q)
                if (pick[q] == t) { dup = 1; break; }
            if (!dup) pick[got++] = t;
        }
        for (int32_t q = 0; q < m; ++q) {
            EMIT(v, pick[q]);
            endp[ne++] = v;
            endp[ne++] = pick[q];
        }
    }
    free(endp);
    free(pick);
    if (cover > 0) {
        int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!perm) return -2;
        for (int32_t i = 0; i < n; ++i) perm[i] = i;
        for (int32_t i = n - 1; i > 0; --i) {
            int32_t j = (int32_t)sm_below(&s, (uint64_t)i + 1);
            int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
        int64_t need = (int64_t)ceil(cover * (double)n);
        int64_t pos = 0;
        while (pos < need) {
            int32_t size = kmin + (int32_t)sm_below(&s, (uint64_t)(kmax - kmin + 1));
            if (pos + size > n) break;
            for (int32_t x = 0; x < size; ++x)
                for (int32_t y = x + 1; y < size; ++y)
                    EMIT(perm[pos + x], perm[pos + y]);
            pos += size;
        }
        free(perm);
    }
#undef EMIT
    return (cap > 0 && k > cap) ? -k : k;
}

/* Batched BA: graph g gets n[g], m[g] and stream seed (seed, g); its pairs
 * are written at pair_off[g] with vertex ids local to the graph.  pair_off
 * must come from a previous call with count_only = 1, which fills
 * counts[g] instead of writing pairs. */
typedef struct {
    const int32_t *n, *m;
    const int64_t *off;
    int64_t *counts;
    int32_t *src, *dst;
    int32_t g0, g1;
    double cover;
    int32_t kmin, kmax;
    uint64_t seed;
    int count_only;
    int err;
} ba_job;

static void *ba_worker(void *arg) {
    ba_job *j = (ba_job *)arg;
    for (int32_t g = j->g0; g < j->g1; ++g) {
        uint64_t gs = stream_state(j->seed, (uint64_t)g, 0x42415443ULL);
        if (j->count_only) {
            int64_t c = tcgen_ba(NULL, NULL, 0, j->n[g], j->m[g], j->cover, j->kmin, j->kmax, gs);
            if (c < 0) { j->err = 1; return NULL; }
            j->counts[g] = c;
        } else {
            int64_t cap = j->off[g + 1] - j->off[g];
            int64_t c = tcgen_ba(j->src + j->off[g], j->dst + j->off[g], cap, j->n[g], j->m[g],
                                 j->cover, j->kmin, j->kmax, gs);
            if (c != cap) { j->err = 1; return NULL; }
        }
    }
    return NULL;
}

int tcgen_ba_batch(int32_t num_graphs, const int32_t *n, const int32_t *m, double cover,
                   int32_t kmin, int32_t kmax, uint64_t seed, int count_only,
                   int64_t *counts, const int64_t *pair_off, int32_t *src, int32_t *dst,
                   int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    ba_job jobs[256];
    pthread_t th[256];
    int32_t chunk = (num_graphs + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        ba_job *j = &jobs[t];
        memset(j, 0, sizeof(*j));
        j->n = n; j->m = m; j->off = pair_off; j->counts = counts;
        j->src = src; j->dst = dst;
        j->g0 = t * chunk;
        j->g1 = j->g0 + chunk < num_graphs ? j->g0 + chunk : num_graphs;
        if (j->g0 > j->g1) j->g0 = j->g1;
        j->cover = cover; j->kmin = kmin; j->kmax = kmax; j->seed = seed;
        j->count_only = count_only;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, ba_worker, &jobs[t]);
    ba_worker(&jobs[0]);
    int err = 0;
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < nthreads; ++t) err |= jobs[t].err;
    return err ? -1 : 0;
}

/* Uniform draws for workload recipes (log-uniform sizes etc.): fills out[k]
 * with U[0,1) from stream (seed, k). */
void tcgen_uniform(double *out, int64_t count, uint64_t seed, uint64_t salt) {
    for (int64_t k = 0; k < count; ++k) {
        uint64_t s = stream_state(seed, (uint64_t)k, salt);
        out[k] = sm_unit(&s);
    }
}

/* Writes pairs as a text edge list, "u v\n" per line in decimal, after a
 * comment header line.  Returns 0, or -1 if the file cannot be written. */
int tcgen_write_text(const char *path, const int64_t *src, const int64_t *dst, int64_t num_pairs) {
    FILE *f = fopen(path, "wb");
    if (!f) return -1;
    enum { BUF = 1 << 20 };
    char *buf = (char *)malloc(BUF + 64);
    if (!buf) {
        fclose(f);
        return -1;
    }
    size_t len = (size_t)snprintf(buf, 64, "# %lld pairs\n", (long long)num_pairs);
    for (int64_t i = 0; i < num_pairs; ++i) {
        uint64_t x[2] = {(uint64_t)src[i], (uint64_t)dst[i]};
        for (int k = 0; k < 2; ++k) {
            char tmp[24];
            int t = 0;
            uint64_t v = x[k];
            do {
                tmp[t++] = (char)('0' + v % 10);
                v /= 10;
            } while (v);
            while (t) buf[len++] = tmp[--t];
            buf[len++] = k == 0 ? ' ' : '\n';
        }
        if (len > BUF) {
            if (fwrite(buf, 1, len, f) != len) {
                free(buf);
                fclose(f);
                return -1;
            }
            len = 0;
        }
    }
    int r = (len && fwrite(buf, 1, len, f) != len) ? -1 : 0;
    free(buf);
    if (fclose(f) != 0) r = -1;
    return r;
}
