/*
 * tc.h -- C ABI of libtc, triangle centrality on AMD Instinct MI355X (gfx950).
 *
 * Triangle centrality (Burkhardt, "Triangle Centrality", arXiv 2105.00110,
 * Definition 1 in Sec. "Formulation"):
 *
 *   TC(v) = ( 1/3 Σ_{u ∈ N△[v]} △(u) + Σ_{w ∈ N(v) \ N△(v)} △(w) ) / △(G)
 *
 * for a simple undirected graph, where △(v) counts triangles at v, △(G)
 * triangles in the graph, N△(v) = {u ∈ N(v) : N(u) ∩ N(v) ≠ ∅} is the
 * triangle neighbourhood and N△[v] = N△(v) ∪ {v} (Sec. "Notation").
 *
 * The library returns, all exactly:
 *   tri[v]      △(v)                                           uint64 [n]
 *   support[e]  triangles on canonical edge e, i.e. the value
 *               of the graph triangle matrix T = A² ∘ A at
 *               that edge (Sec. "Algebraic Form")              uint64 [m]
 *   triG        △(G)                                           uint64 [1] (or [G] for a batch)
 *   num[v]      3·△(G)·TC(v) =  △(v) + Σ_{u ∈ N△(v)} △(u)
 *                             + 3 Σ_{w ∈ N(v)\N△(v)} △(w)      uint64 [n]
 *   tc[v]       (double)num[v] / (double)(3·△(G)): one IEEE-754
 *               binary64 division, round to nearest even;
 *               0.0 for every v when △(G) = 0                  double [n]
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Vertices are int32 ids 0..n-1 (the paper labels them 1..n; ids here
 *   are 0-based, n is explicit and isolated vertices are kept).
 * - Input pairs (src[i], dst[i]) are undirected.  Self-loops are dropped
 *   and repeated pairs, in either direction, count once: the graph is
 *   "symmetrized, weights and loops removed" (Sec. "Comparison").
 * - Canonical edges: u < v, sorted lexicographically by (u, v).  support[e]
 *   and tc_get_edges() use this order.  Internal orderings never leak.
 * - mem_kind: TC_MEM_HOST (pageable or pinned host memory) or
 *   TC_MEM_DEVICE (device memory of the current HIP device).
 * - stream: a hipStream_t passed as void*; NULL is the legacy default
 *   stream.  Device work is enqueued on it.  Calls that must learn a size
 *   on the host (the edge count after deduplication) synchronise it.
 * - Ownership: the caller owns every input and output buffer and must keep
 *   inputs alive until the call returns (host inputs) or the stream has
 *   passed the call's work (device inputs).  The library owns a tc_graph
 *   and all its device memory until tc_graph_destroy().
 * - Errors: every function returns a tc_status; nothing throws across the
 *   ABI.  On an error no output is written and *out is left NULL.
 * - Threading: distinct handles may be used from distinct host threads;
 *   one handle must not be used concurrently.
 */
#ifndef TC_H_
#define TC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tc_graph tc_graph;

typedef enum tc_status {
    TC_OK = 0,
    TC_TRIANGLE_FREE = 1,       /* informational: △(G) = 0, tc[] = 0       */
    TC_ERR_INVALID_ARG = -1,    /* NULL pointer, negative size, bad kind   */
    TC_ERR_VERTEX_RANGE = -2,   /* an id outside [0, n)                     */
    TC_ERR_OOM = -3,            /* device allocation failed                 */
    TC_ERR_DEVICE = -4,         /* a HIP runtime call failed                */
    TC_ERR_OVERFLOW = -5,       /* a result would not fit its type          */
    TC_ERR_BUDGET = -6,         /* request larger than the caller's budget  */
    TC_ERR_NOT_COMPUTED = -7,   /* results requested before tc_compute()    */
    TC_ERR_UNSUPPORTED = -8,    /* size beyond the library's index types    */
    TC_ERR_IO = -9              /* a file cannot be opened, mapped or read  */
} tc_status;

#define TC_MEM_HOST 0
#define TC_MEM_DEVICE 1

/* Library version as 10000*major + 100*minor + patch. */
int32_t tc_version(void);

/* Static text for a status code. */
const char *tc_status_string(int32_t status);

/* ------------------------------------------------------------------------
 * Tuning knobs of the counting step.  They change the schedule only, never
 * a result: every valid setting yields bit-identical outputs.
 *   light_max_dplus  rows whose higher-ordered neighbourhood N_H(v) has at
 *                    most this many entries are intersected by one
 *                    wavefront each; larger rows by a whole workgroup.
 *                    Range 2..1024.
 *   heavy_block      workgroup size of the heavy-row kernel: 64..1024,
 *                    a multiple of 64.
 *   light_block      workgroup size of the light-row kernel: 64..1024,
 *                    a multiple of 64 (one row per wavefront).
 *   lds_max_entries  slots of the largest per-row LDS hash table of the
 *                    heavy kernel (power of two, 1024..16384; a table is
 *                    kept at most half full, so rows with more than
 *                    lds_max_entries/2 entries are probed by binary search
 *                    in device memory instead).
 *   algorithm        which vertex of each triangle owns the hash table:
 *                    TC_ALGO_LOW_PIVOT  the lowest-ordered one, v: N_H(v)
 *                      is hashed and N_H(u) streamed for every u in N_H(v)
 *                      (the appendix's alternative TriangleNeighbor,
 *                      Procedure 2, intersecting N_H(v) and N_H(u));
 *                    TC_ALGO_MID_PIVOT  the middle one, v: N_H(v) is
 *                      hashed (Procedure 1's marking of T) and, for every
 *                      lower neighbour u in N_L(v), only the part of N_H(u)
 *                      above v is streamed (Procedure 1's inner loop);
 *                    TC_ALGO_AUTO (0) picks the middle pivot, whose
 *                    streamed work is the number of oriented wedges, for
 *                    graphs of 600000 edges or more with an oriented row of
 *                    32 entries or more, and for every graph of 3000000
 *                    edges or more; the low pivot otherwise (fewer
 *                    launches and host round trips).
 *                    In the middle-pivot form "rows" are the pivots v and
 *                    the bins above are taken on |N_H(v)| of the pivot.
 *   item_pairs       middle pivot only: lower neighbours of one pivot per
 *                    work item of a wavefront (a workgroup item takes this
 *                    many per wavefront); 64..65536, a multiple of 64.
 *   bitmap_words     middle pivot only: workgroup pivots whose N_H(v)
 *                    spans at most 32*bitmap_words ranks are looked up in
 *                    an LDS bitmap of the span (8 bytes per 32 ranks: the
 *                    bits and the count of entries before them) instead of
 *                    the hash table; 0 turns the bitmap off, else a power
 *                    of two, 256..8192.
 *   light_bitmap_pairs  middle pivot only: wavefront pivots (|N_H(v)| <=
 *                    light_max_dplus) with at least this many lower
 *                    neighbours and a span that fits the bitmap are
 *                    counted by the workgroup bitmap kernel instead;
 *                    0 keeps all of them on the wavefront kernel.
 * ---------------------------------------------------------------------- */
#define TC_ALGO_AUTO 0
#define TC_ALGO_LOW_PIVOT 1
#define TC_ALGO_MID_PIVOT 2

typedef struct tc_tuning {
    int32_t light_max_dplus;
    int32_t heavy_block;
    int32_t light_block;
    int32_t lds_max_entries;
    int32_t algorithm;
    int32_t item_pairs;
    int32_t bitmap_words;
    int32_t light_bitmap_pairs;
} tc_tuning;

/* Writes the built-in defaults to *t. */
tc_status tc_tuning_default(tc_tuning *t);

/* ------------------------------------------------------------------------
 * Graph construction.
 *
 * tc_graph_from_edges: builds the deduplicated symmetric graph from
 *   num_pairs undirected pairs.  Any id outside [0, n) gives
 *   TC_ERR_VERTEX_RANGE and no handle.  n = 0 with num_pairs = 0 is a valid
 *   empty graph.  Limits: n < 2^31, num_pairs < 2^32.
 *
 * tc_graph_from_csr: same, from a CSR adjacency row_ptr[n+1] (int64,
 *   row_ptr[0] = 0, non-decreasing) and col[row_ptr[n]].
 *   assume_simple_sorted = 0: every stored entry (v, col[k]) is taken as an
 *     undirected pair, so one-sided and symmetric CSRs give the same graph;
 *     loops and duplicates are dropped as above (a sort and a
 *     deduplication).
 *   assume_simple_sorted = 1: the caller states that every row is strictly
 *     increasing, with ids in [0, n) and no self-loop (checked on the
 *     device: TC_ERR_INVALID_ARG and no handle otherwise).  The edges are
 *     then the entries above the diagonal (col[k] > v), read in order as the
 *     canonical edge list with no sort and no deduplication; a symmetric
 *     CSR and its upper triangle give the same graph, and entries below the
 *     diagonal are not read as edges.
 * ---------------------------------------------------------------------- */
tc_status tc_graph_from_edges(const int32_t *src, const int32_t *dst, int64_t num_pairs,
                              int32_t n, int32_t mem_kind, void *stream, tc_graph **out);

tc_status tc_graph_from_csr(const int64_t *row_ptr, const int32_t *col, int32_t n,
                            int32_t mem_kind, int32_t assume_simple_sorted, void *stream,
                            tc_graph **out);

/* ------------------------------------------------------------------------
 * Batched construction: num_graphs independent graphs in one handle.
 *   graph_pair_off[G+1]  graph g owns pairs graph_pair_off[g] ..
 *                        graph_pair_off[g+1]-1 of src/dst
 *   graph_vtx_off[G+1]   graph g owns n_g = graph_vtx_off[g+1] -
 *                        graph_vtx_off[g] vertices
 * Pair ids are LOCAL to their graph (0..n_g-1).  Results are laid out as
 * for one graph over the concatenated vertex range (vertex graph_vtx_off[g]
 * + i is local vertex i of graph g); canonical edges are grouped by graph
 * in graph order (tc_batch_edge_offsets); triG has one entry per graph and
 * tc[v] divides by 3·△ of v's own graph.  Offsets are host arrays.
 * ---------------------------------------------------------------------- */
tc_status tc_batch_create(const int32_t *src, const int32_t *dst, const int64_t *graph_pair_off,
                          const int64_t *graph_vtx_off, int32_t num_graphs, int32_t mem_kind,
                          void *stream, tc_graph **out);

/* ------------------------------------------------------------------------
 * Fused batch of small graphs: one persistent launch runs the whole path
 * (deduplication, degree order, orientation, counting with support, △(v),
 * △(G), Algorithm 2's numerator and the quotient of Definition 1) for every
 * graph of a batch, one workgroup per graph at a time, pulling graphs from
 * a device-side queue.  The counting step is the appendix's Procedure 2
 * (sorted N_H lists merged, counts in place of marks), one thread per
 * oriented edge.  Results equal tc_batch_create + tc_compute exactly.
 *
 * For callers that cannot allocate or read back: it allocates nothing (the
 * caller passes a workspace), never synchronises the stream and reads
 * nothing back, so the call can be captured into a HIP graph and replayed
 * (each replay recomputes from the inputs in place).
 *
 * All pointers are device memory of the current device, except tuning.
 *   src, dst             pairs, ids LOCAL to their graph (0..n_g-1)
 *   graph_pair_off[G+1]  graph g owns pairs [graph_pair_off[g], graph_pair_off[g+1])
 *   graph_vtx_off[G+1]   graph g owns vertices [graph_vtx_off[g], graph_vtx_off[g+1])
 *                        of the outputs below; both arrays start at 0 and end at
 *                        num_pairs and num_vertices
 *   order[G]             optional (NULL = 0..G-1): the order in which graphs are
 *                        taken from the queue, e.g. largest first
 *   num_pairs, num_vertices  the totals (host values, used to size and bound)
 * Outputs (eu, ev, support, tri, triG, num, tc may each be NULL):
 *   eu[P], ev[P], support[P]  graph g's canonical edges (u < v, local ids, in
 *                        lexicographic order) and their support at positions
 *                        graph_pair_off[g] .. graph_pair_off[g] + num_edges[g] - 1;
 *                        the rest of the range is not written
 *   num_edges[G]         m_g after deduplication (required)
 *   tri[N], num[N], tc[N]  per vertex, at graph_vtx_off[g] + local id
 *   triG[G]              △ of each graph
 *   status[G]            (required) TC_OK; TC_TRIANGLE_FREE when △(G) = 0 (tc = 0);
 *                        TC_ERR_VERTEX_RANGE if a pair of the graph has an id outside
 *                        [0, n_g); TC_ERR_UNSUPPORTED if n_g > 65535;
 *                        TC_ERR_INVALID_ARG for offsets outside the arrays or
 *                        decreasing.  A graph with an error gets no edges and zero
 *                        tri / num / tc (nothing at all for invalid offsets).
 *   workspace            device memory of at least
 *                        tc_batch_fused_workspace_bytes(num_pairs, num_vertices, G)
 *                        bytes, 256-byte aligned, used by this call only until
 *                        the stream passes it (no need to clear it)
 * Returns TC_ERR_INVALID_ARG for a NULL required pointer, a negative size, a
 * short or misaligned workspace or a bad tuning, TC_ERR_UNSUPPORTED beyond
 * 2^40 pairs or vertices, TC_ERR_DEVICE if a launch fails; otherwise TC_OK
 * once the work is queued on `stream` (per-graph outcomes are in status[]).
 * Two calls sharing a workspace must not overlap in time.
 *
 * tc_fused_tuning: block (256, 512 or 1024 threads per workgroup) and
 * wg_per_cu (1..16 persistent workgroups per compute unit).
 * ---------------------------------------------------------------------- */
typedef struct tc_fused_tuning {
    int32_t block;
    int32_t wg_per_cu;
} tc_fused_tuning;

tc_status tc_fused_tuning_default(tc_fused_tuning *t);

/* Workspace bytes of tc_batch_fused (-1 for negative sizes). */
int64_t tc_batch_fused_workspace_bytes(int64_t num_pairs, int64_t num_vertices, int32_t num_graphs);

tc_status tc_batch_fused(const int32_t *src, const int32_t *dst, const int64_t *graph_pair_off,
                         const int64_t *graph_vtx_off, const int32_t *order, int32_t num_graphs,
                         int64_t num_pairs, int64_t num_vertices, int32_t *eu, int32_t *ev,
                         uint64_t *support, int64_t *num_edges, uint64_t *tri, uint64_t *triG,
                         uint64_t *num, double *tc, int32_t *status, void *workspace,
                         int64_t workspace_bytes, const tc_fused_tuning *tuning, void *stream);

/* ------------------------------------------------------------------------
 * tc_batch_fused_noalloc: tc_batch_fused for callers that cannot allocate
 * device memory or pass a workspace (code under graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same arguments,
 * outputs and per-graph statuses as tc_batch_fused, without workspace and
 * workspace_bytes: the workspace is a fixed device array inside the library
 * of tc_batch_fused_noalloc_max_bytes() bytes (64 MiB) per GPU, held from
 * the library's first use on that GPU until the process ends.
 *   - Returns TC_ERR_BUDGET, with nothing queued, when
 *     tc_batch_fused_workspace_bytes(num_pairs, num_vertices, num_graphs)
 *     exceeds that maximum (about 20 bytes per pair plus 40 per vertex).
 *   - Calls no allocating routine: the array's device address is looked up
 *     on the first call on each device (hipGetSymbolAddress); every call
 *     then queues the same two kernels as tc_batch_fused on `stream`.
 *   - Every call on one GPU uses the same array, which keeps the last
 *     call's contents (nothing in it needs clearing: each call resets its
 *     queue counter with a kernel and writes every word before reading it).
 *     Calls whose work overlaps on one GPU (other streams or host threads
 *     before the earlier call's work has finished) race on the array and
 *     give undefined results: serialise them, e.g. on one stream.
 * ---------------------------------------------------------------------- */
int64_t tc_batch_fused_noalloc_max_bytes(void);

tc_status tc_batch_fused_noalloc(const int32_t *src, const int32_t *dst,
                                 const int64_t *graph_pair_off, const int64_t *graph_vtx_off,
                                 const int32_t *order, int32_t num_graphs, int64_t num_pairs,
                                 int64_t num_vertices, int32_t *eu, int32_t *ev, uint64_t *support,
                                 int64_t *num_edges, uint64_t *tri, uint64_t *triG, uint64_t *num,
                                 double *tc, int32_t *status, const tc_fused_tuning *tuning,
                                 void *stream);

/* Number of graphs in the handle (1 for a single graph). */
int32_t tc_num_graphs(const tc_graph *g);

/* Host array edge_off[G+1]: graph g's canonical edges are edge_off[g] ..
 * edge_off[g+1]-1 of the handle's edge order. */
tc_status tc_batch_edge_offsets(const tc_graph *g, int64_t *edge_off);

/* ------------------------------------------------------------------------
 * Computation: triangle counting on the degree-ordered orientation
 * (Sec. "Algorithm": each triangle found once, from its lowest-ordered
 * vertex, with the ordering π of Sec. "Notation"), per-edge support, △(v),
 * △(G), then Algorithm 2's aggregation and the quotient.  Asynchronous on
 * `stream`.  Returns TC_TRIANGLE_FREE (after computing) when △(G) = 0 for
 * a single graph; for a batch, the status is TC_OK and per-graph △(G) = 0
 * shows in triG.  tc_compute_tuned uses explicit knobs (NULL = defaults).
 * ---------------------------------------------------------------------- */
tc_status tc_compute(tc_graph *g, void *stream);
tc_status tc_compute_tuned(tc_graph *g, const tc_tuning *tuning, void *stream);

int64_t tc_num_vertices(const tc_graph *g);   /* n (sum over a batch); -1 if g is NULL */
int64_t tc_num_edges(const tc_graph *g);      /* m after deduplication; -1 if g is NULL */

/* Canonical edges: u[e] < v[e], e = 0..m-1.  Either pointer may be NULL. */
tc_status tc_get_edges(const tc_graph *g, int32_t *u, int32_t *v, int32_t mem_kind,
                       void *stream);

/* Results of the last tc_compute.  Any output pointer may be NULL.  Sizes:
 * tri[n], support[m], triG[num_graphs], num[n], tc[n].  With TC_MEM_HOST
 * the call returns after the copies completed (it synchronises stream). */
tc_status tc_get_results(const tc_graph *g, uint64_t *tri, uint64_t *support, uint64_t *triG,
                         uint64_t *num, double *tc, int32_t mem_kind, void *stream);

/* Numerator by the algebraic form (Sec. "Algebraic Algorithm", Algorithm 3;
 * Proposition 2): num = 1/2 (3A - 2T' + I)(T 1), where T = A^2 o A carries the
 * support of the last tc_compute and T' is its 0/1 pattern, evaluated as two
 * sparse matrix-vector passes over the symmetric adjacency.  It shares no
 * kernel with tc_compute's aggregation (Algorithm 2), so num[] here equals
 * tc_get_results' num[] exactly; tests use it as a cross-check.
 * num[n] (uint64, vertex order; per batch, concatenated like tri[]).  The
 * first call on a handle fills its symmetric adjacency (16*m bytes, held by
 * the handle until destroyed; after a middle-pivot tc_compute this first
 * sorts the edges by their larger end, with 16*m bytes of scratch).  Every
 * call allocates 4*2m + 16*n bytes of scratch and, with TC_MEM_HOST,
 * returns after the copy.  TC_ERR_NOT_COMPUTED before
 * tc_compute; TC_ERR_DEVICE if a product comes out odd (it cannot if the
 * support is a valid T). */
tc_status tc_numerator_algebraic(const tc_graph *g, uint64_t *num, int32_t mem_kind, void *stream);

/* Results of a batch handle (tc_batch_create + tc_compute): the same
 * copies as tc_get_results, named for batches.  tri[N], num[N], tc[N] over
 * the concatenated vertex range, support[m] in the handle's edge order
 * (graph g's edges at tc_batch_edge_offsets), triG[num_graphs] with one
 * △(G) per graph; tc[v] divides by 3·△ of v's own graph. */
tc_status tc_batch_get_results(const tc_graph *b, uint64_t *tri, uint64_t *support, uint64_t *triG,
                               uint64_t *num, double *tc, int32_t mem_kind, void *stream);

/* Device bytes currently held by the handle. */
tc_status tc_graph_device_bytes(const tc_graph *g, int64_t *bytes);

/* Upper bound of the device bytes tc_compute / tc_compute_tuned will
 * allocate on top of what the built handle g holds (tc_graph_device_bytes),
 * for the pivot form the tuning picks (NULL: defaults; TC_ALGO_AUTO decides
 * as tc_compute does).  For the middle pivot it includes the exact size of
 * the bit matrices of §3.3's Procedure 1, 4·Σ_v Σ_{t<d+(v)} ceil(t/32)
 * bytes over the oriented rows (about Σ_v C(d+(v), 2) / 8), which it reads
 * back from the device: the call waits for the stream.  A caller with a
 * memory budget checks it after the build, before the count, so that a
 * dense graph whose bit matrices outgrow tc_estimate_device_bytes cannot
 * overrun the budget.  *bytes is a host pointer.  TC_ERR_INVALID_ARG for a
 * NULL handle or pointer or an invalid tuning. */
tc_status tc_compute_bytes(tc_graph *g, const tc_tuning *tuning, void *stream, int64_t *bytes);

/* Limit on the device bytes the library's allocator holds on each device
 * (blocks in use plus blocks it caches for reuse; 0 = no limit, the
 * default).  An allocation that would pass it first gives the cached blocks
 * back, then fails with TC_ERR_BUDGET: the call that needed it returns
 * TC_ERR_BUDGET and the handle stays as it was before that call (a failed
 * tc_compute leaves it not computed).  The fused launch's workspace and
 * other caller-owned buffers are not counted.  TC_ERR_INVALID_ARG if
 * bytes < 0. */
tc_status tc_set_memory_limit(int64_t bytes);

/* Device bytes of the library's allocator on the current device: held
 * (in use plus cached), in use, and the peaks of both since the library
 * loaded or the last reset; reset_peaks != 0 sets the peaks to the current
 * values after reading them.  Each pointer is a host pointer or NULL. */
tc_status tc_memory_stats(int64_t *held, int64_t *in_use, int64_t *peak_held,
                          int64_t *peak_in_use, int32_t reset_peaks);

/* Estimate of the peak device bytes tc_graph_from_edges + tc_compute need
 * for num_pairs pairs over n vertices, for admission control by callers
 * with a memory budget.  It bounds the peak while the middle pivot's bit
 * matrices (Σ_v C(d+(v), 2) / 8 bytes over the oriented rows) stay within
 * about 20 bytes per pair, as on sparse graphs (R-MAT scale 24: 20 bytes
 * per pair); denser graphs, e.g. large cliques, need that much more. */
int64_t tc_estimate_device_bytes(int64_t num_pairs, int32_t n);

/* Releases the handle and its device memory (NULL is a no-op).  Waits for
 * work still queued on the handle's last stream. */
void tc_graph_destroy(tc_graph *g);

/* ------------------------------------------------------------------------
 * Ingest of text edge lists with arbitrary ids (the paper's inputs are SNAP
 * graphs relabelled to 1..n without gaps: Sec. "Comparison", Table 6).
 *
 * tc_edge_text_read (host only, no GPU): parses `path`, one pair per line,
 *   two non-negative decimal ids (< 2^63) separated by spaces or tabs;
 *   further columns are ignored; blank lines and lines starting with '#'
 *   or '%' are skipped; '\r' before the newline is accepted.  With
 *   src = dst = NULL it only counts: *num_pairs receives the number of pair
 *   lines.  Otherwise it fills src[i], dst[i] (int64, caller-owned, capacity
 *   entries each) in file order and fails with TC_ERR_INVALID_ARG if
 *   capacity < *num_pairs.  A malformed line gives TC_ERR_INVALID_ARG and
 *   its 1-based number in *bad_line (may be NULL).  TC_ERR_IO if the file
 *   cannot be opened or mapped.  nthreads <= 0 uses every hardware thread.
 *
 * tc_relabel_ids: maps the 2*num_pairs ids to 0..n-1 by their rank among
 *   the distinct ids (order-preserving), writes src32/dst32[num_pairs]
 *   (int32) and, if ids is not NULL, the sorted distinct original ids
 *   ids[n] (int64; give it 2*num_pairs entries when n is not known).  *n_out
 *   receives n.  All arrays are host or device memory as mem_kind says;
 *   the call returns after its work on `stream` has completed.  Negative
 *   ids give TC_ERR_VERTEX_RANGE; n >= 2^31 or 2*num_pairs >= 2^32 give
 *   TC_ERR_UNSUPPORTED.
 * ---------------------------------------------------------------------- */
tc_status tc_edge_text_read(const char *path, int64_t *src, int64_t *dst, int64_t capacity,
                            int64_t *num_pairs, int64_t *bad_line, int32_t nthreads);
tc_status tc_relabel_ids(const int64_t *src, const int64_t *dst, int64_t num_pairs, int32_t *src32,
                         int32_t *dst32, int64_t *ids, int64_t *n_out, int32_t mem_kind,
                         void *stream);

/* ------------------------------------------------------------------------
 * Ranking (the "who is most important" question of Sec. "Comparison"):
 * the k vertices of largest tc, ties broken by smaller vertex id, written
 * in rank order to vertices[k] (int32) and, if not NULL, values[k].  For a
 * batch, ranks over all vertices of all graphs.  Requires tc_compute.
 * k is clamped to n; *k_out receives the count written.
 * ---------------------------------------------------------------------- */
tc_status tc_top_k(const tc_graph *g, int32_t k, int32_t *vertices, double *values,
                   int32_t *k_out, int32_t mem_kind, void *stream);

/* ------------------------------------------------------------------------
 * Instrumentation (measurement only; results are unaffected).
 *
 * tc_set_profiling(on): from now on, handles record HIP events on the
 *   caller's stream around each stage of tc_graph_from_edges / _from_csr /
 *   tc_batch_create and tc_compute.  Process-wide switch.
 * tc_get_stage_ms: device milliseconds of each stage of the handle's last
 *   build and last compute, ms[TC_NUM_STAGES] in the order below (stages
 *   that did not run read 0).  Synchronises on the recorded events.
 *   Returns TC_ERR_NOT_COMPUTED if profiling was off for that work.
 * tc_get_work_stats: exact work measures of the degree-ordered orientation
 *   (Sec. "Algorithm", Lemma 1 bounds the same sums), computed on the
 *   device from the handle's oriented graph on `stream`, stats[
 *   TC_NUM_WORK_STATS] in the order below.  The candidate sums are
 *   the candidates streamed by the last tc_compute's kernels in each bin
 *   (light / heavy / huge): with the low pivot Σ_{v→u} |N_H(u)| over the
 *   oriented edges whose low end v is in the bin, with the middle pivot
 *   Σ |{w ∈ N_H(u) : w > v}| over the pairs u ∈ N_L(v) of the bin's pivots
 *   v; the edge counts are the oriented edges (low pivot) or pairs (middle
 *   pivot) of each bin.  Merge work is Σ_{v→u} (|N_H(v)| + |N_H(u)|),
 *   wedges Σ_v C(|N_H(v)|, 2), W_hash Σ_{v→u} |N_H(u)|.  The middle
 *   pivot reads the candidates of pivots among the top 2^16 ranks as 16-bit
 *   entries (rank less n - 2^16) in its wavefront and workgroup kernels;
 *   TC_STAT_CAND_HEAVY_16 is the part of the heavy bin's candidates read so
 *   (0 after the low pivot), and TC_STAT_EDGES_HEAVY_16 / _ROWS_HEAVY_16
 *   the pairs and pivots they belong to: the work of the launch timed as
 *   TC_STAGE_COUNT_HEAVY_BITMAP16 when the tuning's bitmap has at least
 *   2048 words.
 * ---------------------------------------------------------------------- */
#define TC_NUM_STAGES 14
enum {
    TC_STAGE_CSR_BUILD = 0,   /* dedup, degrees, symmetric row offsets  */
    TC_STAGE_DEGREE_RANK = 1, /* degree ordering                        */
    TC_STAGE_ORIENT = 2,      /* oriented CSR over ranks                */
    TC_STAGE_BIN = 3,         /* row binning by |N_H(v)| (+ transposed
                                 orientation on first use, middle pivot) */
    TC_STAGE_COUNT_LIGHT = 4, /* intersection, wavefront per row        */
    TC_STAGE_COUNT_HEAVY = 5, /* intersection, workgroup per row (LDS)  */
    TC_STAGE_COUNT_HUGE = 6,  /* intersection, device-memory probe      */
    TC_STAGE_FOLD = 7,        /* bit-matrix fold (middle pivot only)    */
    TC_STAGE_TRI = 8,         /* support per edge, tri(v), triG (after
                                 the low pivot: + symmetric adjacency)   */
    TC_STAGE_AGGREGATE = 9,   /* Algorithm 2 sums + quotient            */
    /* launches inside the two intersection stages above (middle pivot;
       0 after the low pivot) */
    TC_STAGE_COUNT_LIGHT_GROUPS = 10,   /* rows <= 128 entries, 16 lanes each */
    TC_STAGE_COUNT_LIGHT_WAVE = 11,     /* other wavefront rows, LDS hash    */
    TC_STAGE_COUNT_LIGHT_BITMAP = 12,   /* wavefront rows moved to a bitmap  */
    TC_STAGE_COUNT_HEAVY_BITMAP16 = 13  /* workgroup rows among the top 2^16
                                           ranks, 2048-word bitmap           */
};
#define TC_NUM_WORK_STATS 20
enum {
    TC_STAT_N = 0, TC_STAT_M = 1, TC_STAT_MAX_DPLUS = 2,
    TC_STAT_ROWS_LIGHT = 3, TC_STAT_ROWS_HEAVY = 4, TC_STAT_ROWS_HUGE = 5,
    TC_STAT_CAND_LIGHT = 6, TC_STAT_CAND_HEAVY = 7, TC_STAT_CAND_HUGE = 8,
    TC_STAT_MERGE_WORK = 9, TC_STAT_WEDGES = 10, TC_STAT_TRIANGLES = 11,
    TC_STAT_EDGES_LIGHT = 12, TC_STAT_EDGES_HEAVY = 13, TC_STAT_EDGES_HUGE = 14,
    TC_STAT_W_HASH = 15, TC_STAT_ALGORITHM = 16, TC_STAT_CAND_HEAVY_16 = 17,
    TC_STAT_EDGES_HEAVY_16 = 18, TC_STAT_ROWS_HEAVY_16 = 19
};

tc_status tc_set_profiling(int32_t on);

/* Device memory.  The library keeps the device memory of destroyed handles
 * and of its temporaries cached for reuse (per device; a block freed on one
 * stream is reused on another only after that stream's work on it is
 * done), so a sequence of builds allocates only when it needs more than
 * before.  tc_trim_memory returns every cached block that no live handle
 * uses to the device (it waits for their last work); live handles are
 * untouched.  Thread-safe. */
tc_status tc_trim_memory(void);
tc_status tc_get_stage_ms(const tc_graph *g, double *ms);
tc_status tc_get_work_stats(tc_graph *g, int64_t *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
