/*
 * tl.h -- triangle listing under a given vertex ordering, on one AMD
 * Instinct MI355X (gfx950) GPU.
 *
 * Method: Lecuyer, Jachiet, Magnien, Tabourier, "Tailored vertex ordering
 * for faster triangle listing in large graphs" (arXiv 2203.04774).
 *
 * Problem statement (Section 1.3 and Section 2.1): given a simple undirected
 * graph G = (V, E) and an ordering pi of V, orient every edge from the lower
 * to the higher index (the DAG G_pi) and report every triangle {u, v, w}
 * exactly once, as the triple with pi_u < pi_v < pi_w.  Algorithm 1 (A++)
 * seeds on the long edge (u, w) and scans N+_u against the marked N-_w;
 * Algorithm 2 (A+-) seeds on the first short edge (u, v) and scans N+_v
 * against the marked N+_u; the footnote's third form (A--) seeds on the
 * second short edge.  Definition 1 gives the costs C++ = sum d+ d+ and
 * C+- = sum d+ d-.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Vertex ids and ranks are uint32 in [0, n); rank is 0-based (the paper's
 *   pi_u is 1-based).  Offsets, counts, costs and digests are uint64.
 * - Pointers documented as "device" must point to memory on the current HIP
 *   device; "host" pointers to ordinary host memory.  `stream` is a
 *   hipStream_t passed as void* (NULL = the null stream).  All GPU work is
 *   ordered on that stream; a call returns after its host outputs are filled.
 * - Every function returns TL_OK or an error code and never throws or aborts.
 *   tl_strerror() names a code; tl_last_error() gives the calling thread's
 *   most recent detailed message.
 * - A tl_csr is used from one stream at a time.
 */
#ifndef TL_H
#define TL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque oriented graph, library-owned device memory. */
typedef struct tl_csr tl_csr;

/* Listing algorithm: A++ = Algorithm 1 (seed edge L, cost C++),
 * A+- = Algorithm 2 (seed edge S1, cost C+-), A-- = the S2-seeded variant
 * of the footnote in Section 2.1 (cost sum d- d-). */
typedef enum { TL_APP = 0, TL_APM = 1, TL_AMM = 2 } tl_algo;

enum {
    TL_OK = 0,
    TL_EINVAL = 1,    /* bad argument: NULL pointer, id >= n, rank not a permutation, size limit */
    TL_ENOMEM = 2,    /* device allocation failed */
    TL_ECAPACITY = 3, /* output buffer too small; summary->count holds the size needed */
    TL_EHIP = 4,      /* a HIP runtime call failed */
    TL_EABORT = 5     /* the chunk callback asked to stop */
};

/* Result of a listing call.
 *   count    triangles listed
 *   hash     wrapping 64-bit sum over listed triangles (a<b<c original ids)
 *            of f(f((a<<32)|b) + c), f = the splitmix64 output function;
 *            order independent, so it identifies the set (with count)
 *   work     the paper's work: elements of the scanned lists over the
 *            listed pivots' seed edges (Property 1); for a full listing it
 *            equals tl_cost for the same algorithm
 *   scanned  elements the kernels actually tested after range pruning */
typedef struct {
    uint64_t count;
    uint64_t hash;
    uint64_t work;
    uint64_t scanned;
} tl_summary;

/* Chunk sink: receives `k` triangles, 0 < k <= the chunk size (3*k uint32
 * in device memory, valid until the callback returns; the stream is
 * synchronised before the call).  Each call holds triangles of one probe
 * slice of the work items (a slice that found more than the chunk size is
 * handed out in several calls), so calls number at least (triangles / chunk
 * size) and chunks need not be full.  A non-zero return stops the listing
 * with TL_EABORT. */
typedef int (*tl_chunk_fn)(const uint32_t *tri_dev, uint64_t k, void *user);

/*
 * tl_orient -- build the oriented graph G_pi (Section 1.3).
 *   n          vertex count, 0 <= n < 2^32 - 1
 *   src, dst   device, m_in uint32 each: undirected edges {src[i], dst[i]};
 *              each edge may appear once or in both directions; self-loops
 *              and repeated pairs are dropped (the paper's datasets are
 *              simplified the same way, Section 4.1.1)
 *   m_in       input edge count, < 2^32
 *   rank       device, n uint32: rank[u] = pi_u - 1; must be a permutation
 *   out        host: receives the new handle (release with tl_csr_free)
 * The handle holds, in rank space, the forward CSR (row r = ranks of the
 * successors of the vertex of rank r, ascending), the backward CSR (the
 * predecessors), their row ids, and the inverse permutation.  Inputs are
 * not retained.  Errors: TL_EINVAL for NULL pointers with non-zero sizes,
 * an id >= n or a rank that is not a permutation (nothing allocated).
 */
int tl_orient(uint32_t n, const uint32_t *src, const uint32_t *dst, uint64_t m_in,
              const uint32_t *rank, void *stream, tl_csr **out);

/*
 * tl_cost -- Definition 1 for the handle's ordering: C++ = sum_u d+_u d+_u
 * (TL_APP), C+- = sum_u d+_u d-_u (TL_APM), sum_u d-_u d-_u (TL_AMM).
 *   cost  host, receives the value.
 */
int tl_cost(const tl_csr *g, tl_algo a, void *stream, uint64_t *cost);

/*
 * tl_list -- list every triangle once with the chosen algorithm
 * (Algorithms 1 and 2), all pivots.  Output modes:
 *   tri_dev != NULL: triangles are written to tri_dev (device, 3*cap
 *     uint32, row i = (a, b, c), a < b < c, original ids), in unspecified
 *     order.  If more than cap exist, TL_ECAPACITY is returned with
 *     out->count = the number needed; the buffer's contents are then
 *     unspecified.  The library also allocates a spill area of its own
 *     (bounded by the launch shape, not by the graph) while listing.
 *   tri_dev == NULL, cb != NULL: triangles are streamed through cb in
 *     library-owned device chunks (see tl_set_chunk_triangles).
 *   both NULL: count, digest and work only.
 *   out  host, receives the summary (filled in every mode, also on
 *        TL_ECAPACITY).
 */
int tl_list(const tl_csr *g, tl_algo a, uint32_t *tri_dev, uint64_t cap_triangles,
            tl_chunk_fn cb, void *user, void *stream, tl_summary *out);

/*
 * tl_list_range -- as tl_list, restricted to pivots whose rank lies in
 * [pivot_lo, pivot_hi).  The pivot is the vertex whose list the paper marks
 * in B: w for A++ (Algorithm 1), u for A+- (Algorithm 2), v for A--.  The
 * outer iterations are independent (Section 4.1.2), so disjoint ranges
 * partition the triangles, and counts, digests and work add up.
 */
int tl_list_range(const tl_csr *g, tl_algo a, uint32_t pivot_lo, uint32_t pivot_hi,
                  uint32_t *tri_dev, uint64_t cap_triangles, tl_chunk_fn cb, void *user,
                  void *stream, tl_summary *out);

/*
 * tl_list_count_noalloc -- tl_list in its count-only mode (both tri_dev and
 * cb NULL: count, digest and work of every triangle, all pivots) that
 * allocates nothing, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it).
 * Every device block the listing needs comes from one device array of
 * TL_NOALLOC_SCRATCH_BYTES built into the library, which each GPU the
 * library runs on holds until the process ends.
 *   g, a, stream  as for tl_list; out  host, receives the summary.
 * Returns TL_ECAPACITY, with nothing launched, when the graph's plan needs
 * more than that array (roughly 60 bytes per edge plus 28 per vertex), or
 * when its heavy-pivot tasks do not fit what is left of it (then after
 * waiting for the stream).  Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (other threads, other streams) race and
 * must be serialised by the caller.  Results equal tl_list's.
 */
#define TL_NOALLOC_SCRATCH_BYTES (64ull << 20)
int tl_list_count_noalloc(const tl_csr *g, tl_algo a, void *stream, tl_summary *out);

/* Size of the oriented graph: n and m (undirected edges after dropping
 * loops and duplicates).  Host outputs. */
int tl_csr_size(const tl_csr *g, uint32_t *n, uint64_t *m);

/*
 * tl_csr_copy_to_host -- copy the oriented graph into host buffers (for
 * inspection and tests).  Any pointer may be NULL to skip that array.
 *   off_fwd, off_bwd  n+1 uint64     adj_fwd, adj_bwd  m uint32
 *   inv               n uint32, inv[r] = vertex of rank r
 */
int tl_csr_copy_to_host(const tl_csr *g, uint64_t *off_fwd, uint32_t *adj_fwd,
                        uint64_t *off_bwd, uint32_t *adj_bwd, uint32_t *inv);

/* Release a handle and its device memory (NULL is a no-op). */
void tl_csr_free(tl_csr *g);

/*
 * Orderings computed on the device, for the full listing (ordering time
 * included) on the GPU.
 *
 * From an oriented graph g (any orientation: a vertex's degree in the
 * simple graph is its successors plus its predecessors), writes a new
 * ordering as rank_dev[u] (device uint32 array of g's n entries, the same
 * layout as tl_orient's rank argument):
 *   TL_ORDER_DEGREE  non-decreasing degree, ties by increasing vertex id
 *                    (the degree ordering of Section 2.2)
 *   TL_ORDER_SPLIT   Split (Section 3.3.3): the non-increasing degree
 *                    ordering (the degree ordering read backwards) dealt
 *                    alternately to the front and the back: the vertex at
 *                    position 2i+1 gets index i+1, the one at 2i index n+1-i
 *                    (1-based; rank = index - 1)
 *   TL_ORDER_CORE    non-decreasing coreness, ties by increasing vertex id
 *                    (a core ordering of Section 1.3; coreness computed by
 *                    level-synchronous peeling on the device)
 *   TL_ORDER_CHECK   Check (Section 3.3.2): vertices taken by non-increasing
 *                    degree (TL_ORDER_DEGREE read backwards); each goes right
 *                    after the beginning block if |N_b| (|N_e| + |N_?|) <=
 *                    (|N_b| + |N_?|) |N_e|, else right before the end block
 * Orient again with the result (tl_orient) to list under it.  Returns after
 * the stream has finished; TL_EINVAL for an unknown kind or a NULL pointer.
 */
typedef enum { TL_ORDER_DEGREE = 0, TL_ORDER_SPLIT = 1, TL_ORDER_CORE = 2, TL_ORDER_CHECK = 3 } tl_order_kind;
int tl_order(const tl_csr *g, tl_order_kind kind, uint32_t *rank_dev, void *stream);

/*
 * Neigh (Algorithm 3, Section 3.3.1): a local search that starts from the
 * ordering g is oriented by and, pass after pass, visits every vertex (by
 * increasing id) and moves it to the cheapest place among its neighbours
 * for C+-: with N_u sorted by the current order as v_1 .. v_d, place 0 is
 * right before v_1 and place p right after v_p.  A vertex whose current
 * place is among the cheapest stays; otherwise it takes the smallest
 * cheapest p.  Passes repeat while a pass brings C+- below (1 - eps) times
 * its value at the pass's start, at most max_passes times; max_visits > 0
 * stops after that many vertex visits.  The search is sequential, so it
 * runs on the host (a copy of g's CSR is read back first).
 * rank_dev: device uint32 array of g's n entries, the result as rank[u].
 * out (host, optional): C+- at the start and at the end, passes completed,
 * vertex visits, moves, wall-clock seconds.  Returns after the stream has
 * finished; TL_EINVAL for a NULL handle or eps outside [0, 1).
 */
typedef struct {
    uint64_t cpm_start, cpm;
    uint32_t passes, visits;
    uint64_t moves;
    double seconds;
} tl_neigh_result;
int tl_order_neigh(const tl_csr *g, double eps, uint32_t max_passes, uint32_t max_visits, uint32_t *rank_dev,
                   tl_neigh_result *out, void *stream);

/*
 * Batched listing: many independent graphs listed by one pass.
 *
 * The problem solved for each graph is the one of tl_orient + tl_list
 * (Section 1.3 for the orientation, Algorithms 1 and 2 for the listing);
 * the batch is the disjoint union of the graphs, oriented once, and its
 * listing attributes every triangle to its graph.  A listing pass allocates
 * nothing and never waits for the host before its end: with use_graph = 1
 * it is captured once per algorithm as a HIP graph and replayed.
 *
 * tl_batch_orient
 *   k        number of graphs (>= 1)
 *   n, m     host arrays of k entries: graph i has n[i] vertices and m[i]
 *            input edges (any order, loops and duplicates allowed, as for
 *            tl_orient)
 *   src,dst  device uint32 arrays of sum(m) entries: graph i's edges occupy
 *            [m[0] + .. + m[i-1], + m[i]) and use its local ids [0, n[i])
 *   rank     device uint32 array of sum(n) entries: graph i's permutation of
 *            [0, n[i]) at [n[0] + .. + n[i-1], + n[i])
 *   out      receives the handle (owns all device memory of the batch:
 *            the union's CSR plus listing scratch of about 48 bytes per
 *            edge, sized once here)
 *   The inputs are read only during the call.  TL_EINVAL if sum(n) >=
 *   2^32 - 1, sum(m) >= 2^32, a rank is out of its graph's range or an edge
 *   endpoint is >= its graph's n (a rank array that is not a permutation
 *   gives TL_EINVAL as in tl_orient).  TL_ENOMEM if the device is full.
 *
 * tl_batch_list
 *   algo       TL_APP, TL_APM or TL_AMM
 *   use_graph  1: replay the pass as a captured HIP graph (captured on the
 *              first call for this algo); 0: launch its kernels directly
 *   per_graph  host array of 3 * k uint64 (or NULL): for graph i, entries
 *              3i, 3i+1, 3i+2 receive its triangle count, its digest (as
 *              tl_list's hash, over the graph's local ids) and its work
 *   per_graph_dev  device array of 3 * k uint64 (or NULL): the same table,
 *              written on the stream
 *   Returns after the pass has finished on the stream.  Calls on one
 *   handle must not overlap.
 */
typedef struct tl_batch tl_batch;
int tl_batch_orient(uint32_t k, const uint32_t *n, const uint64_t *m, const uint32_t *src, const uint32_t *dst,
                    const uint32_t *rank, void *stream, tl_batch **out);
/*
 * tl_batch_from_graphs -- a batch of k graphs already oriented by
 * tl_orient (each by its own ordering): the union is built by copying their
 * arrays with shifted ranks and indices, with no sort, and equals the one
 * tl_batch_orient builds from the same inputs, so tl_batch_list gives the
 * same table.  gs is a host array of k handles, read during the call only
 * (the handles stay the caller's).  TL_EINVAL for k = 0, a NULL handle or a
 * union of 2^32 - 1 vertices or 2^32 edges or more.
 */
int tl_batch_from_graphs(uint32_t k, const tl_csr *const *gs, void *stream, tl_batch **out);
int tl_batch_list(tl_batch *b, tl_algo algo, int use_graph, uint64_t *per_graph, uint64_t *per_graph_dev,
                  void *stream);
/* k, the union's vertex count and its simple-edge count (host outputs, any may be NULL). */
int tl_batch_size(const tl_batch *b, uint32_t *k, uint32_t *n, uint64_t *m);
/* Releases the batch (NULL is ignored); waits for the device. */
void tl_batch_free(tl_batch *b);

/*
 * Listing server: continuous batching of listing jobs under a device
 * memory budget.
 *
 * Each job is the problem of tl_orient + tl_list for one graph (Section 1.3,
 * Algorithms 1 and 2).  Jobs wait in arrival order; a job is admitted when
 * its modelled device footprint (about 72 bytes per input edge plus 64 per
 * vertex) fits the budget beside the jobs already admitted.  Admitted jobs
 * are uploaded, oriented as one disjoint union and listed by the batched
 * pass, while the next batches are uploaded and oriented on other streams
 * (list_threads batches may be listed at once, each on a stream of its own);
 * a job with at least solo_edges edges is oriented and listed alone by the
 * plain listing.  A job whose footprint alone exceeds the budget finishes
 * with TL_ENOMEM; a malformed job (an endpoint >= n, a rank array that is
 * not a permutation) finishes with TL_EINVAL without failing the jobs
 * batched with it.  Results never depend on how jobs were batched.
 *
 * Resident graphs: a job with a non-zero key names its graph and ordering.
 * The first such job is uploaded and oriented alone, and its oriented graph
 * then stays resident on the device under that key; later jobs with the
 * same key are listed from it with no upload and no orientation (their
 * arrays are not read), batched with the other resident jobs into one union
 * built by copying (tl_batch_from_graphs).  Resident graphs count against
 * the budget (about 20 bytes per edge and per vertex) and the least recently
 * used ones not in use are dropped when a job needs the room.  A key must
 * always name the same graph and ordering; jobs with key 0 are never kept.
 */
typedef struct tl_server tl_server;
typedef struct {
    uint64_t hbm_budget;      /* device bytes the admitted jobs may use (> 0) */
    uint32_t max_batch_jobs;  /* jobs per batch, at most (0: 4096) */
    uint64_t max_batch_edges; /* input edges per batch, at most (0: 2^27) */
    uint64_t solo_edges;      /* jobs with at least this many edges run alone (0: 2^21) */
    uint32_t pipeline;        /* 1: orient the next batch while one lists */
    uint32_t list_threads;    /* batches listed at once, each on its own stream (0: 8; at most 8) */
} tl_server_config;

typedef struct {
    uint32_t n;               /* vertices */
    uint64_t m;               /* input edges */
    const uint32_t *src, *dst;/* host arrays of m entries */
    const uint32_t *rank;     /* host array of n entries: the ordering */
    tl_algo algo;
    uint64_t key;             /* non-zero: the graph stays resident under this key */
} tl_job;                     /* the arrays must stay valid until the job is final */

#define TL_JOB_PENDING (-1)
typedef struct {
    int status;               /* TL_JOB_PENDING, TL_OK, TL_EINVAL, TL_ENOMEM, TL_EABORT (cancelled), TL_EHIP */
    uint64_t count, hash, work; /* as tl_summary, when status is TL_OK */
    uint64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns; /* steady clock */
    uint64_t batch_id;        /* the batch that listed the job */
    uint32_t batch_jobs;      /* jobs in that batch */
} tl_job_result;

typedef struct {
    uint64_t submitted, jobs_done, batches, rejected, cancelled, split_batches;
    uint64_t reserved, peak_reserved, pending, max_batch_jobs_seen;
    uint64_t upload_ns, orient_ns, list_ns; /* thread time in each stage, summed over batches */
    uint64_t resident_hits;   /* keyed jobs listed from a resident graph */
    uint64_t resident_graphs, resident_bytes; /* graphs resident now, and their bytes */
    uint64_t resident_dropped; /* resident graphs dropped to make room */
} tl_server_stats;

/* Starts the server on the current device: an upload thread (with its copier
 * threads and page-locked staging buffers), an orient thread and
 * list_threads list threads.  TL_EINVAL for list_threads above 8, TL_ENOMEM
 * if the staging buffers cannot be allocated. */
int tl_server_create(const tl_server_config *cfg, tl_server **out);
/* Queues a job (never blocks on the device); *id identifies it. */
int tl_server_submit(tl_server *s, const tl_job *job, uint64_t *id);
/* Reads a job's result, waiting up to wait_us microseconds (< 0: until it is
 * final).  A final result is handed out once; the id is then unknown. */
int tl_server_poll(tl_server *s, uint64_t id, int64_t wait_us, tl_job_result *out);
/* Cancels a job that is not admitted yet (TL_EINVAL once it is). */
int tl_server_cancel(tl_server *s, uint64_t id);
/* paused = 1: admit no further jobs until called again with 0 (admitted
 * jobs run on).  For callers that queue a burst before letting it in. */
int tl_server_pause(tl_server *s, int paused);
int tl_server_get_stats(tl_server *s, tl_server_stats *out);
/* The modelled device footprint the admission charges for a job. */
uint64_t tl_server_job_bytes(uint32_t n, uint64_t m);
/* Cancels waiting jobs, lets admitted ones finish, stops the threads. */
void tl_server_destroy(tl_server *s);

/*
 * Launch tuning (results never depend on it).  Keys:
 *   heavy_min            items of a pivot before it gets a workgroup (>= 1)
 *   slice_min            items per heavy-pivot task, at least (>= 64)
 *   slice_mult           tasks are also >= this many times the pivot's
 *                        staging cost (>= 1)
 *   task_div             ... but at most the listing's work (Definition 1)
 *                        / (this x heavy workgroups) items, at least 65536,
 *                        so that a few hub pivots do not end the launch
 *                        alone (0..1024; 0: no such cap)
 *   heavy_blocks_per_cu  heavy-pivot workgroups launched per CU (1..64)
 *   light_blocks_per_cu  light-pivot workgroups launched per CU, at most (1..64)
 *   light_wave_items     ... and no more than one wavefront per this many
 *                        light items (64..2^30)
 *   queue                1: heavy tasks handed out by an atomic queue
 *   splits               1: wavefront start seeds precomputed per task
 *   keep_staged          1: a heavy workgroup whose next task has the same
 *                        pivot keeps that pivot's list staged in LDS
 *   lean                 1: when every heavy task has the bitmap or split
 *                        form (always, under the default keys), a heavy
 *                        kernel compiled with those two forms only runs
 *   hash                 1: a heavy pivot whose list's rank window is too
 *                        wide for the LDS bitmap keeps the list in an LDS
 *                        hash table when it fits
 *   reverse              1: a heavy pivot whose list fits no LDS form tests
 *                        each edge (y, pivot) by searching y's own sorted
 *                        list instead of the pivot's
 *   bucket               1: a heavy pivot whose list's rank window is too
 *                        wide for the LDS bitmap keeps the list in LDS with
 *                        a table of where each of 8192 equal slices of the
 *                        window starts (a search then covers one slice)
 *   split                1: a heavy pivot whose list is too long for LDS
 *                        marks the entries in the top 2^20 ranks of its
 *                        window in an LDS bitmap and searches the rest in
 *                        global memory; 2: also in place of the array and
 *                        bucket forms
 *   orient_sort          1: tl_orient builds both CSRs by device radix sorts
 *                        of packed (row, column) keys; 0: by per-vertex
 *                        counters, scatter and row sorts
 *   force_mode           testing: 0 bitmap, 1 array, 2 global, 3 reverse,
 *                        4 hash, 5 bucket, 6 split for every heavy pivot
 *                        where it fits; 255 = automatic
 *   plan_full            a seed edge whose scanned list has at most this
 *                        many entries scans all of it instead of its window
 *                        (found by binary search; 0..255; results are the
 *                        same, only the work split changes)
 * for callback mode (chunks of K triangles, tl_set_chunk_triangles):
 *   chunk_task_div       heavy tasks hold at most chunk_room x K / (this x
 *                        heavy workgroups) items, at least 65536 (1..64;
 *                        default 64)
 *   chunk_growth         1 (default): every probe slice covers chunk_room x K
 *                        scanned items, which can never overflow the chunk
 *                        (each item yields at most one triangle); above 1: a
 *                        slice may cover up to this many times the previous
 *                        slice's items, sized from its triangles per item
 *                        (1..64)
 *   chunk_margin         percent margin over the previous slice's
 *                        triangles per item when chunk_growth > 1 (100..1000;
 *                        default 125)
 *   chunk_room           the library's device chunk holds this many times K
 *                        triangles (default 4; 1..16): a slice's triangles
 *                        are handed to the callback K at a time; a slice that
 *                        finds more than the chunk holds is probed again
 *                        shorter
 * and for the batched pass (tl_batch_list; a captured pass is captured
 * again when these change):
 *   batch_heavy_min      pruned items of a pivot before its list is marked
 *                        in an LDS bitmap by a workgroup of its own
 *   batch_heavy_block    threads of such a workgroup: 256, 512 or 1024
 *   batch_heavy_per_cu   such workgroups per CU (1..2)
 *   batch_light_per_cu   workgroups of the per-item kernel per CU (1..64)
 *   batch_plan_full      as plan_full, for the batched pass
 * Values apply to later calls in this process; TL_TUNE_<KEY> environment
 * variables (upper case) set the initial values.  Unknown keys or values
 * out of range give TL_EINVAL.
 */
int tl_set_tuning(const char *key, uint64_t value);
int tl_get_tuning(const char *key, uint64_t *value);

/* Device memory for handles and per-call scratch is cached by the library
 * (one free list per stream) and reused by later calls.  This returns every
 * cached block that is not in use to the driver; it waits for the device. */
int tl_release_cached_memory(void);

/* Triangles per callback in callback mode, K (default 2^24, i.e. 192 MiB of
 * uint32 triples); the library's device chunk holds chunk_room x K of them
 * (see tl_set_tuning).  Applies to later calls in this process. */
int tl_set_chunk_triangles(uint64_t k);

/*
 * Kernel-phase timing, for measurement.  While enabled, the library records
 * HIP events on the caller's stream around each phase's kernels and, when
 * the call synchronises, adds the elapsed time to a per-phase total.
 *   phase  one of the TL_PHASE_* values below
 *   ms, calls  host outputs: accumulated milliseconds and timed launches
 */
/*
 * Work split of the calling thread's most recent listing (for measurement):
 * items are scanned-list elements after pruning; "heavy" pivots are the ones
 * listed by workgroup tasks with their list staged in LDS; heavy_work is the
 * paper's work of those pivots' seed edges, heavy_staged the total length of
 * their staged lists.
 */
typedef struct {
    uint64_t light_items, heavy_items;
    uint64_t light_seeds, heavy_seeds;
    uint64_t heavy_work, heavy_pivots, heavy_staged, heavy_triangles;
    uint64_t tasks;
    uint64_t mode_items[7]; /* heavy items by LDS form: bitmap, array, global,
                               reverse, hash, bucket, split */
    uint64_t slices;        /* probe passes: one per chunk in callback mode */
    uint64_t slices_redone; /* callback-mode slices that found more than a
                               chunk of triangles and were probed again shorter */
    /* heavy items by walk path: groups of chunks inside one seed's window,
     * groups spread over consecutive short windows, one chunk at a time */
    uint64_t items_long, items_short, items_single;
    /* SPLIT-form elements below the bitmap's rank window (each tested by a
     * search of the pivot's lower entries), and how many of those searches
     * ran in global memory because the lower entries did not fit LDS */
    uint64_t split_below, split_below_global;
    /* list entries staged in LDS by the heavy kernel's workgroups (a
     * workgroup whose next task has the same pivot keeps its list staged) */
    uint64_t heavy_task_staged;
    /* SPLIT-form groups of chunks tested together, and how many of them ran
     * the search for elements below the bitmap's window */
    uint64_t split_groups, split_below_groups;
} tl_list_stats;
int tl_last_list_stats(tl_list_stats *out);

enum {
    TL_PHASE_ORIENT = 0,      /* all of tl_orient */
    TL_PHASE_PLAN = 1,        /* windows, classes, compaction, prefix, tasks */
    TL_PHASE_PROBE = 2,       /* both probe kernels */
    TL_PHASE_COST = 3,        /* tl_cost */
    TL_PHASE_PROBE_LIGHT = 4, /* the light-pivot probe kernel alone */
    TL_PHASE_PROBE_HEAVY = 5, /* the heavy-pivot probe kernel alone */
    TL_PHASE_BATCH = 6,       /* one tl_batch_list pass (all of its kernels) */
    TL_PHASE_ORDER = 7,       /* tl_order */
    TL_NUM_PHASES = 8
};
int tl_timing_enable(int on);
int tl_timing_reset(void);
int tl_timing_read(int phase, double *ms, uint64_t *calls);

const char *tl_strerror(int code);
const char *tl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TL_H */
