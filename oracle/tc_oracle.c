/*
 * CPU oracle for triangle centrality -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no code with the HIP library: it has
 * its own normalisation, its own orderings and its own loops, written for a
 * reader to check against the paper by eye, not for speed.
 *
 * Two independent formulations of the same exact integer result:
 *
 *   O1 "definition" -- per edge {x,y}: sup(x,y) = |N(x) ∩ N(y)|, the value of
 *      the graph triangle matrix T = A^2 ∘ A at (x,y) (Sec. "Algebraic Form");
 *      tri(v) = 1/2 Σ_u sup(u,v) and triG = 1/3 Σ_v tri(v) (the quoted
 *      theorem there); then Definition 1 multiplied by 3·triG:
 *        num(v) = tri(v) + Σ_{u ∈ N△(v)} tri(u) + 3 Σ_{w ∈ N(v)\N△(v)} tri(w)
 *      with N△(v) = {u ∈ N(v) : sup(u,v) > 0} (Sec. "Notation").
 *
 *   O2 "paper algorithm" -- the appendix Procedure 2 (alternative
 *      TriangleNeighbor) on sorted higher-ordered neighbourhoods N_H under
 *      the degree ordering π of Sec. "Notation", with per-slot counts in
 *      place of the 0/1 marks L_v, followed by Algorithm 2's aggregation
 *      (core sum x, neighbour sum s, non-core sum y = s - x + tri(v)) in
 *      integers: num = x + 3y.
 *
 * Both end with one IEEE-754 binary64 division
 *      tc(v) = (double)num(v) / (double)(3·triG),
 * i.e. Definition 1 with numerator and denominator scaled by 3, and
 * tc ≡ 0 when triG = 0 (the measure is undefined on triangle-free graphs).
 *
 * Status codes: 0 ok, 1 triangle-free, -1 bad argument, -2 vertex id out of
 * range, -3 out of memory, -5 arithmetic overflow, -7 internal check failed.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define OR_OK 0
#define OR_TRIANGLE_FREE 1
#define OR_ERR_ARG (-1)
#define OR_ERR_RANGE (-2)
#define OR_ERR_OOM (-3)
#define OR_ERR_OVERFLOW (-5)
#define OR_ERR_CHECK (-7)

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------------
 * Normalised simple graph: canonical edges (eu[e] < ev[e]) in lexicographic
 * order, and the symmetric adjacency with every row sorted by vertex id.
 * slot_edge[p] is the canonical edge index of adjacency slot p.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    int64_t m;
    int32_t *eu, *ev;
    int64_t *rp;        /* [n+1] */
    int32_t *adj;       /* [2m]  */
    int64_t *slot_edge; /* [2m]  */
} ograph;

static void ograph_free(ograph *g) {
    free(g->eu); free(g->ev); free(g->rp); free(g->adj); free(g->slot_edge);
    memset(g, 0, sizeof(*g));
}

/* Plain LSD radix sort of 64-bit keys, 16-bit digits. */
static int sort_u64(uint64_t *a, int64_t len) {
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(len > 0 ? len : 1));
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * 65536);
    if (!tmp || !cnt) { free(tmp); free(cnt); return OR_ERR_OOM; }
    uint64_t *from = a, *to = tmp;
    for (int shift = 0; shift < 64; shift += 16) {
        memset(cnt, 0, sizeof(int64_t) * 65536);
        for (int64_t i = 0; i < len; ++i) cnt[(from[i] >> shift) & 0xFFFF]++;
        if (cnt[(from[0] >> shift) & 0xFFFF] == len && len > 0) continue; /* digit constant */
        int64_t sum = 0;
        for (int d = 0; d < 65536; ++d) { int64_t c = cnt[d]; cnt[d] = sum; sum += c; }
        for (int64_t i = 0; i < len; ++i) to[cnt[(from[i] >> shift) & 0xFFFF]++] = from[i];
        uint64_t *t = from; from = to; to = t;
    }
    if (from != a) memcpy(a, from, sizeof(uint64_t) * (size_t)len);
    free(tmp);
    free(cnt);
    return OR_OK;
}

/* Drop self-loops, treat (u,v) and (v,u) as one edge, remove duplicates
 * (the paper's test graphs are "symmetrized, weights and loops removed",
 * Sec. "Comparison"). */
static int normalise(const int32_t *src, const int32_t *dst, int64_t P, int32_t n, ograph *g) {
    memset(g, 0, sizeof(*g));
    if (n < 0 || P < 0) return OR_ERR_ARG;
    for (int64_t i = 0; i < P; ++i)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return OR_ERR_RANGE;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(P > 0 ? P : 1));
    if (!keys) return OR_ERR_OOM;
    int64_t k = 0;
    for (int64_t i = 0; i < P; ++i) {
        uint32_t a = (uint32_t)src[i], b = (uint32_t)dst[i];
        if (a == b) continue;
        uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        keys[k++] = ((uint64_t)lo << 32) | hi;
    }
    int st = sort_u64(keys, k);
    if (st) { free(keys); return st; }
    int64_t m = 0;
    for (int64_t i = 0; i < k; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
    g->n = n;
    g->m = m;
    g->eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    g->ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    g->rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m > 0 ? 2 * m : 1));
    g->slot_edge = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m > 0 ? 2 * m : 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!g->eu || !g->ev || !g->rp || !g->adj || !g->slot_edge || !cur) {
        free(keys); free(cur); ograph_free(g); return OR_ERR_OOM;
    }
    for (int64_t e = 0; e < m; ++e) {
        g->eu[e] = (int32_t)(keys[e] >> 32);
        g->ev[e] = (int32_t)(keys[e] & 0xFFFFFFFFULL);
    }
    free(keys);
    for (int64_t e = 0; e < m; ++e) { g->rp[g->eu[e] + 1]++; g->rp[g->ev[e] + 1]++; }
    for (int32_t v = 0; v < n; ++v) g->rp[v + 1] += g->rp[v];
    for (int32_t v = 0; v < n; ++v) cur[v] = g->rp[v];
    /* Edges arrive sorted by (eu, ev): every row first receives its smaller
     * neighbours in increasing order, then its larger ones, so rows end up
     * sorted without a further sort. */
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = g->eu[e], b = g->ev[e];
        g->slot_edge[cur[a]] = e; g->adj[cur[a]++] = b;
        g->slot_edge[cur[b]] = e; g->adj[cur[b]++] = a;
    }
    free(cur);
    return OR_OK;
}

static int64_t find_slot(const ograph *g, int32_t row, int32_t target) {
    int64_t lo = g->rp[row], hi = g->rp[row + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->adj[mid] < target) lo = mid + 1; else hi = mid;
    }
    return (lo < g->rp[row + 1] && g->adj[lo] == target) ? lo : -1;
}

/* ------------------------------------------------------------------------
 * Thread pool helper: workers pull vertex chunks from a shared counter.
 * ---------------------------------------------------------------------- */
typedef struct work_s work_t;
typedef void (*row_fn)(work_t *w, int tid, int32_t v);
struct work_s {
    int32_t n;
    int64_t next; /* atomic */
    int32_t chunk;
    int32_t stride; /* rows v with v % stride == 0 only (1 = all rows) */
    row_fn fn;
    void *ctx;
};
typedef struct { work_t *w; int tid; } worker_arg;

static void *pool_worker(void *p) {
    worker_arg *a = (worker_arg *)p;
    work_t *w = a->w;
    for (;;) {
        int64_t lo = __atomic_fetch_add(&w->next, w->chunk, __ATOMIC_RELAXED);
        if (lo >= w->n) break;
        int64_t hi = lo + w->chunk < w->n ? lo + w->chunk : w->n;
        for (int64_t v = lo; v < hi; ++v)
            if (w->stride <= 1 || v % w->stride == 0) w->fn(w, a->tid, (int32_t)v);
    }
    return NULL;
}

static void run_pool(work_t *w, int nthreads) {
    pthread_t th[256];
    worker_arg args[256];
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    w->next = 0;
    if (w->chunk < 1) w->chunk = 64;
    for (int t = 0; t < nthreads; ++t) { args[t].w = w; args[t].tid = t; }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, pool_worker, &args[t]);
    pool_worker(&args[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------
 * Shared tail: given tri[], triG and the triangle-neighbour relation,
 * Definition 1's numerator and the quotient.
 * ---------------------------------------------------------------------- */
static int finish_quotient(int32_t n, const uint64_t *num, uint64_t triG, double *tc) {
    if (triG > UINT64_MAX / 3) return OR_ERR_OVERFLOW;
    uint64_t den = 3 * triG;
    for (int32_t v = 0; v < n; ++v)
        tc[v] = (triG == 0) ? 0.0 : (double)num[v] / (double)den;
    return triG == 0 ? OR_TRIANGLE_FREE : OR_OK;
}

/* ========================================================================
 * O1: definition.  Each edge {x, y} is handled once, at the endpoint x that
 * is later in the (degree, id) order; N(x) is marked in a per-thread byte
 * array and N(y) (the cheaper side) is scanned against the marks.
 * ====================================================================== */
typedef struct {
    const ograph *g;
    uint64_t *slot_sup; /* [2m] support of the edge at each adjacency slot */
    uint8_t **mark;     /* per thread, [n] */
} o1_ctx;

static int before(const ograph *g, int32_t a, int32_t b) {
    int64_t da = g->rp[a + 1] - g->rp[a], db = g->rp[b + 1] - g->rp[b];
    return da < db || (da == db && a < b);
}

static void o1_row(work_t *w, int tid, int32_t x) {
    o1_ctx *c = (o1_ctx *)w->ctx;
    const ograph *g = c->g;
    uint8_t *mk = c->mark[tid];
    for (int64_t p = g->rp[x]; p < g->rp[x + 1]; ++p) mk[g->adj[p]] = 1;
    for (int64_t p = g->rp[x]; p < g->rp[x + 1]; ++p) {
        int32_t y = g->adj[p];
        if (!before(g, y, x)) continue;
        uint64_t common = 0;
        for (int64_t q = g->rp[y]; q < g->rp[y + 1]; ++q) common += mk[g->adj[q]];
        c->slot_sup[p] = common;
        c->slot_sup[find_slot(g, y, x)] = common;
    }
    for (int64_t p = g->rp[x]; p < g->rp[x + 1]; ++p) mk[g->adj[p]] = 0;
}

int oracle_o1(const int32_t *src, const int32_t *dst, int64_t P, int32_t n, int nthreads,
              int64_t *m_out, int32_t *eu_out, int32_t *ev_out, uint64_t *sup_out,
              uint64_t *tri_out, uint64_t *triG_out, uint64_t *num_out, double *tc_out) {
    ograph g;
    int st = normalise(src, dst, P, n, &g);
    if (st) return st;
    *m_out = g.m;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    o1_ctx c;
    c.g = &g;
    c.slot_sup = (uint64_t *)calloc((size_t)(2 * g.m > 0 ? 2 * g.m : 1), sizeof(uint64_t));
    c.mark = (uint8_t **)calloc((size_t)nthreads, sizeof(uint8_t *));
    int oom = !c.slot_sup || !c.mark;
    for (int t = 0; !oom && t < nthreads; ++t) {
        c.mark[t] = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
        oom |= !c.mark[t];
    }
    if (!oom) {
        work_t w = {n, 0, 256, 1, o1_row, &c};
        run_pool(&w, nthreads);
    }
    if (c.mark)
        for (int t = 0; t < nthreads; ++t) free(c.mark[t]);
    free(c.mark);
    if (oom) { free(c.slot_sup); ograph_free(&g); return OR_ERR_OOM; }

    /* tri(v) = 1/2 Σ_{u ∈ N(v)} sup(u,v); triG = 1/3 Σ_v tri(v). */
    uint64_t total = 0;
    for (int32_t v = 0; v < n; ++v) {
        uint64_t s = 0;
        for (int64_t p = g.rp[v]; p < g.rp[v + 1]; ++p) s += c.slot_sup[p];
        if (s & 1) st = OR_ERR_CHECK;
        tri_out[v] = s / 2;
        total += tri_out[v];
    }
    if (total % 3) st = OR_ERR_CHECK;
    uint64_t triG = total / 3;
    *triG_out = triG;
    for (int64_t p = 0; p < 2 * g.m; ++p) {
        /* canonical order: slot of ev in row eu */
        int64_t e = g.slot_edge[p];
        if (g.adj[p] == g.ev[e]) sup_out[e] = c.slot_sup[p];
    }
    for (int64_t e = 0; e < g.m; ++e) { eu_out[e] = g.eu[e]; ev_out[e] = g.ev[e]; }
    /* num(v) = tri(v) + Σ_{u ∈ N△(v)} tri(u) + 3 Σ_{w ∈ N(v) \ N△(v)} tri(w) */
    for (int32_t v = 0; v < n; ++v) {
        uint64_t acc = tri_out[v];
        for (int64_t p = g.rp[v]; p < g.rp[v + 1]; ++p) {
            uint64_t t = tri_out[g.adj[p]];
            acc += (c.slot_sup[p] > 0) ? t : 3 * t;
        }
        num_out[v] = acc;
    }
    free(c.slot_sup);
    ograph_free(&g);
    if (st) return st;
    return finish_quotient(n, num_out, triG, tc_out);
}

/* ========================================================================
 * O2: the paper's algorithm.
 *
 * pi: position in the order (degree, id)  (Sec. "Notation").
 * N_H(v): neighbours u with pi(u) > pi(v), kept sorted by vertex id.
 * For every v and every u in N_H(v) (at index i), the sorted lists N_H(v)
 * and N_H(u) are scanned with two pointers; every common w (index l in
 * N_H(v), r in N_H(u)) is a triangle with low v, middle u, high w.  Where
 * Procedure 2 sets L_v(l) = L_u(r) = 1 and, if any w was found, L_v(i) = 1,
 * this oracle adds 1 to each of the first two slots and the number of
 * common w to the third, so that each slot ends holding the support of its
 * edge and the marks are recovered as "count > 0".  Every triangle also
 * increments tri of its three vertices and triG.
 * ====================================================================== */
typedef struct {
    const ograph *g;
    int32_t *pi;      /* [n] */
    int64_t *hp;      /* [n+1] */
    int32_t *hadj;    /* [m] */
    int64_t *hedge;   /* [m] canonical edge of each N_H slot */
    uint64_t *hsup;   /* [m] per-slot counts (atomic adds) */
    uint64_t **tri_t; /* per-thread tri deltas, [n] each */
    uint64_t *triG_t; /* per-thread triangle totals */
    uint64_t **lv_t;  /* per-thread scratch of size max |N_H| */
    uint64_t *X;      /* [n] core sums (atomic adds) */
    const uint64_t *tri;
} o2_ctx;

static void o2_count_row(work_t *w, int tid, int32_t v) {
    o2_ctx *c = (o2_ctx *)w->ctx;
    int64_t vb = c->hp[v], ve = c->hp[v + 1];
    int64_t dv = ve - vb;
    if (dv < 2) return;
    uint64_t *Lv = c->lv_t[tid];
    uint64_t *tri = c->tri_t[tid];
    for (int64_t i = 0; i < dv; ++i) Lv[i] = 0;
    for (int64_t i = 0; i < dv; ++i) {
        int32_t u = c->hadj[vb + i];
        int64_t ub = c->hp[u], ue = c->hp[u + 1];
        uint64_t t = 0;
        int64_t l = 0, r = 0;
        while (l < dv && ub + r < ue) {
            int32_t a = c->hadj[vb + l], b = c->hadj[ub + r];
            if (a < b) { ++l; continue; }
            if (b < a) { ++r; continue; }
            /* common w = a = b: triangle {v, u, w} */
            t += 1;
            Lv[l] += 1;
            __atomic_fetch_add(&c->hsup[ub + r], 1, __ATOMIC_RELAXED);
            tri[v] += 1; tri[u] += 1; tri[a] += 1;
            ++l; ++r;
        }
        if (t != 0) Lv[i] += t;
        c->triG_t[tid] += t;
    }
    for (int64_t i = 0; i < dv; ++i)
        if (Lv[i]) __atomic_fetch_add(&c->hsup[vb + i], Lv[i], __ATOMIC_RELAXED);
}

/* Marks -> triangle neighbour sums: every marked slot (v, u) makes u a
 * triangle neighbour of v and v one of u. */
static void o2_core_row(work_t *w, int tid, int32_t v) {
    (void)tid;
    o2_ctx *c = (o2_ctx *)w->ctx;
    uint64_t own = 0;
    for (int64_t k = c->hp[v]; k < c->hp[v + 1]; ++k) {
        if (c->hsup[k] == 0) continue;
        int32_t u = c->hadj[k];
        own += c->tri[u];
        __atomic_fetch_add(&c->X[u], c->tri[v], __ATOMIC_RELAXED);
    }
    if (own) __atomic_fetch_add(&c->X[v], own, __ATOMIC_RELAXED);
}

int oracle_o2(const int32_t *src, const int32_t *dst, int64_t P, int32_t n, int nthreads,
              int32_t row_stride, int64_t *m_out, int32_t *eu_out, int32_t *ev_out,
              uint64_t *sup_out, uint64_t *tri_out, uint64_t *triG_out, uint64_t *num_out,
              double *tc_out, double *phase_s) {
    double t0 = now_s();
    ograph g;
    int st = normalise(src, dst, P, n, &g);
    if (st) return st;
    double t1 = now_s();
    *m_out = g.m;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (row_stride < 1) row_stride = 1;
    o2_ctx c;
    memset(&c, 0, sizeof(c));
    c.g = &g;
    size_t nn = (size_t)(n > 0 ? n : 1), mm = (size_t)(g.m > 0 ? g.m : 1);
    c.pi = (int32_t *)malloc(sizeof(int32_t) * nn);
    c.hp = (int64_t *)calloc(nn + 1, sizeof(int64_t));
    c.hadj = (int32_t *)malloc(sizeof(int32_t) * mm);
    c.hedge = (int64_t *)malloc(sizeof(int64_t) * mm);
    c.hsup = (uint64_t *)calloc(mm, sizeof(uint64_t));
    c.X = (uint64_t *)calloc(nn, sizeof(uint64_t));
    c.tri_t = (uint64_t **)calloc((size_t)nthreads, sizeof(uint64_t *));
    c.lv_t = (uint64_t **)calloc((size_t)nthreads, sizeof(uint64_t *));
    c.triG_t = (uint64_t *)calloc((size_t)nthreads, sizeof(uint64_t));
    int64_t *by_deg = (int64_t *)calloc(nn + 1, sizeof(int64_t));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * nn);
    int oom = !c.pi || !c.hp || !c.hadj || !c.hedge || !c.hsup || !c.X || !c.tri_t ||
              !c.lv_t || !c.triG_t || !by_deg || !order;
    if (!oom) {
        /* pi by a counting sort on degree, stable in vertex id. */
        for (int32_t v = 0; v < n; ++v) by_deg[g.rp[v + 1] - g.rp[v]]++;
        int64_t s = 0;
        for (int32_t d = 0; d <= n; ++d) { int64_t k = by_deg[d]; by_deg[d] = s; s += k; }
        for (int32_t v = 0; v < n; ++v) order[by_deg[g.rp[v + 1] - g.rp[v]]++] = v;
        for (int32_t r = 0; r < n; ++r) c.pi[order[r]] = r;
        /* N_H(v): filter of the id-sorted row, so it stays id-sorted. */
        int64_t maxh = 0;
        for (int32_t v = 0; v < n; ++v) {
            int64_t h = 0;
            for (int64_t p = g.rp[v]; p < g.rp[v + 1]; ++p) h += c.pi[g.adj[p]] > c.pi[v];
            c.hp[v + 1] = c.hp[v] + h;
            if (h > maxh) maxh = h;
        }
        for (int32_t v = 0; v < n; ++v) {
            int64_t k = c.hp[v];
            for (int64_t p = g.rp[v]; p < g.rp[v + 1]; ++p)
                if (c.pi[g.adj[p]] > c.pi[v]) { c.hadj[k] = g.adj[p]; c.hedge[k] = g.slot_edge[p]; ++k; }
        }
        for (int t = 0; !oom && t < nthreads; ++t) {
            c.tri_t[t] = (uint64_t *)calloc(nn, sizeof(uint64_t));
            c.lv_t[t] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(maxh > 0 ? maxh : 1));
            oom |= !c.tri_t[t] || !c.lv_t[t];
        }
    }
    free(by_deg);
    free(order);
    double t2 = now_s(), t3 = t2, t4 = t2;
    if (!oom) {
        work_t w = {n, 0, 64, row_stride, o2_count_row, &c};
        run_pool(&w, nthreads);
        t3 = now_s();
        uint64_t triG = 0;
        for (int t = 0; t < nthreads; ++t) triG += c.triG_t[t];
        for (int32_t v = 0; v < n; ++v) {
            uint64_t s = 0;
            for (int t = 0; t < nthreads; ++t) s += c.tri_t[t][v];
            tri_out[v] = s;
        }
        *triG_out = triG;
        c.tri = tri_out;
        work_t w2 = {n, 0, 256, 1, o2_core_row, &c};
        run_pool(&w2, nthreads);
        /* Algorithm 2: x = X(v) + tri(v); s = Σ_{N(v)} tri; y = s - x + tri(v); num = x + 3y */
        for (int32_t v = 0; v < n; ++v) {
            uint64_t x = c.X[v] + tri_out[v];
            uint64_t sum = 0;
            for (int64_t p = g.rp[v]; p < g.rp[v + 1]; ++p) sum += tri_out[g.adj[p]];
            uint64_t y = sum - x + tri_out[v];
            num_out[v] = x + 3 * y;
        }
        for (int64_t k = 0; k < g.m; ++k) sup_out[c.hedge[k]] = c.hsup[k];
        for (int64_t e = 0; e < g.m; ++e) { eu_out[e] = g.eu[e]; ev_out[e] = g.ev[e]; }
        st = finish_quotient(n, num_out, triG, tc_out);
        t4 = now_s();
    }
    if (phase_s) {
        phase_s[0] = t1 - t0; /* normalisation */
        phase_s[1] = t2 - t1; /* ordering + N_H */
        phase_s[2] = t3 - t2; /* Procedure 2 counting */
        phase_s[3] = t4 - t3; /* aggregation + quotient */
    }
    if (c.tri_t)
        for (int t = 0; t < nthreads; ++t) free(c.tri_t[t]);
    if (c.lv_t)
        for (int t = 0; t < nthreads; ++t) free(c.lv_t[t]);
    free(c.tri_t); free(c.lv_t); free(c.triG_t);
    free(c.pi); free(c.hp); free(c.hadj); free(c.hedge); free(c.hsup); free(c.X);
    ograph_free(&g);
    return oom ? OR_ERR_OOM : st;
}

/* ========================================================================
 * Point queries on the normalised graph, for graphs too large to run O1/O2
 * in a test: support of chosen edges and tri of chosen vertices, each from
 * its definition (common neighbours by marking).
 * ====================================================================== */
typedef struct {
    ograph g;
    uint8_t *mark;
} oquery;

int oracle_query_open(const int32_t *src, const int32_t *dst, int64_t P, int32_t n,
                      void **handle, int64_t *m_out) {
    oquery *q = (oquery *)calloc(1, sizeof(oquery));
    if (!q) return OR_ERR_OOM;
    int st = normalise(src, dst, P, n, &q->g);
    if (st) { free(q); return st; }
    q->mark = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!q->mark) { ograph_free(&q->g); free(q); return OR_ERR_OOM; }
    *handle = q;
    *m_out = q->g.m;
    return OR_OK;
}

void oracle_query_close(void *handle) {
    oquery *q = (oquery *)handle;
    if (!q) return;
    ograph_free(&q->g);
    free(q->mark);
    free(q);
}

int oracle_query_edges(void *handle, int32_t *eu, int32_t *ev) {
    oquery *q = (oquery *)handle;
    memcpy(eu, q->g.eu, sizeof(int32_t) * (size_t)q->g.m);
    memcpy(ev, q->g.ev, sizeof(int32_t) * (size_t)q->g.m);
    return OR_OK;
}

int oracle_query_degree(void *handle, int64_t *deg) {
    oquery *q = (oquery *)handle;
    for (int32_t v = 0; v < q->g.n; ++v) deg[v] = q->g.rp[v + 1] - q->g.rp[v];
    return OR_OK;
}

/* sup(e) = |N(eu) ∩ N(ev)| for the canonical edge indices given. */
int oracle_query_support(void *handle, const int64_t *edges, int64_t k, uint64_t *out) {
    oquery *q = (oquery *)handle;
    const ograph *g = &q->g;
    for (int64_t i = 0; i < k; ++i) {
        if (edges[i] < 0 || edges[i] >= g->m) return OR_ERR_ARG;
        int32_t a = g->eu[edges[i]], b = g->ev[edges[i]];
        for (int64_t p = g->rp[a]; p < g->rp[a + 1]; ++p) q->mark[g->adj[p]] = 1;
        uint64_t c = 0;
        for (int64_t p = g->rp[b]; p < g->rp[b + 1]; ++p) c += q->mark[g->adj[p]];
        for (int64_t p = g->rp[a]; p < g->rp[a + 1]; ++p) q->mark[g->adj[p]] = 0;
        out[i] = c;
    }
    return OR_OK;
}

/* tri(v) = number of edges among N(v) = 1/2 Σ_{u ∈ N(v)} |N(u) ∩ N(v)|. */
int oracle_query_tri(void *handle, const int32_t *verts, int64_t k, uint64_t *out) {
    oquery *q = (oquery *)handle;
    const ograph *g = &q->g;
    for (int64_t i = 0; i < k; ++i) {
        int32_t v = verts[i];
        if (v < 0 || v >= g->n) return OR_ERR_ARG;
        for (int64_t p = g->rp[v]; p < g->rp[v + 1]; ++p) q->mark[g->adj[p]] = 1;
        uint64_t c = 0;
        for (int64_t p = g->rp[v]; p < g->rp[v + 1]; ++p) {
            int32_t u = g->adj[p];
            for (int64_t r = g->rp[u]; r < g->rp[u + 1]; ++r) c += q->mark[g->adj[r]];
        }
        for (int64_t p = g->rp[v]; p < g->rp[v + 1]; ++p) q->mark[g->adj[p]] = 0;
        if (c & 1) return OR_ERR_CHECK;
        out[i] = c / 2;
    }
    return OR_OK;
}
