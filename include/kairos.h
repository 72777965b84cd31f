/*
 * kairos.h -- C interface of libkairos, temporal minimal-path queries on an
 * AMD Instinct MI355X (gfx950).
 *
 * Model (paper §2.1): vertices 0..n-1; a temporal edge (u, v, t, lambda)
 * departs u at time t and arrives at v at time a = t + lambda.  Times are
 * uint32; 0xFFFFFFFF (KAIROS_INF) is reserved for "unreachable", so every
 * finite time is <= 0xFFFFFFFE (KAIROS_TMAX).  lambda >= 1.
 *
 * A path from src is time-respecting when each edge departs no earlier than
 * the previous one arrives (the non-strict "Succeeds" predicate of §2.2, as
 * tested by the Update function of Alg. 2).  A query (src, [t_alpha,
 * t_omega]) only uses edges with t >= t_alpha and a <= t_omega (the closed
 * query interval of Alg. 2).  Outputs, per vertex v:
 *   earliest arrival  EA[v] = min arrival at v            EA[src] = t_alpha
 *   latest departure  LD[v] = max departure from src       LD[src] = t_omega
 *   fastest           F[v]  = min (arrival - departure)    F[src]  = 0
 * (the minimal temporal paths of §2.3 and Table 4); unreachable vertices
 * get KAIROS_INF.  These values are unique, so results do not depend on
 * scheduling.
 *
 * Conventions
 *  - Pointers named "device" must point to device memory of the current HIP
 *    device (for example a torch tensor's data_ptr()); "host" pointers to
 *    host memory.  uint32 data may be stored in int32 tensors.
 *  - Every call returns a kairos_status.  On an argument error nothing is
 *    written to any output.
 *  - The library owns every handle and the device memory behind it; the
 *    caller owns the buffers it passes in.
 *  - Query calls are synchronous: on return the output is complete.
 *  - A graph is immutable after build and may be queried from several host
 *    threads at once; each concurrent query takes its own scratch state.
 */
#ifndef KAIROS_H
#define KAIROS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KAIROS_INF 0xFFFFFFFFu
#define KAIROS_TMAX 0xFFFFFFFEu

typedef enum kairos_status {
    KAIROS_OK = 0,
    KAIROS_ERR_INVALID = 1, /* null pointer, n == 0, unknown kind or option  */
    KAIROS_ERR_RANGE = 2,   /* id >= n, lambda == 0, t + lambda > TMAX,
                               t_alpha > t_omega, t_omega > TMAX, m >= 2^32 */
    KAIROS_ERR_NOMEM = 3,   /* device or host allocation failed             */
    KAIROS_ERR_DEVICE = 4,  /* a HIP call or kernel failed                  */
    KAIROS_ERR_BUSY = 5,    /* a server queue is full                       */
    KAIROS_ERR_SCRATCH = 6  /* the graph needs more state than the fixed
                               scratch of kairos_earliest_arrival_noalloc  */
} kairos_status;

typedef struct kairos_graph kairos_graph;

/* ---------------------------------------------------------------- build --
 * Temporal CSR index (§4.2), built on the device.  Out-edges are grouped by
 * tail and sorted by (tail, t, a, head); in-edges grouped by head and sorted
 * by (head, a, t, tail).  Sorting each adjacency by time is what lets a
 * traversal skip every edge that departs before the tail's arrival (the job
 * the paper gives its interval index, §3.1 and §4.3) by binary search.
 *
 *   src, dst, t, lambda  device, m entries each, read only; the library
 *                        copies what it needs, so they may be freed on return.
 *   m                    number of edges (0 allowed, < 2^32).
 *   n                    number of vertices (>= 1).
 *   hip_stream           hipStream_t for all work on this graph, or NULL for
 *                        library-owned streams.
 *   out                  host; receives the handle.
 * Errors: INVALID (null pointer with m > 0, null out, n == 0), RANGE (an id
 * >= n, lambda == 0, t + lambda > TMAX; checked on the device), NOMEM,
 * DEVICE.  On error *out is left unchanged.
 */
int kairos_graph_build(const uint32_t *src, const uint32_t *dst, const uint32_t *t,
                       const uint32_t *lambda, uint64_t m, uint32_t n, void *hip_stream,
                       kairos_graph **out);

/* Releases the graph and all device memory it holds.  NULL is ignored. */
void kairos_graph_free(kairos_graph *g);

/* n, m and the device bytes held by the index (any pointer may be NULL). */
int kairos_graph_stats(const kairos_graph *g, uint32_t *n, uint64_t *m, uint64_t *device_bytes);

/* Device pointers of the index, for inspection (read only, owned by g).
 * The index numbers vertices internally: the n_live vertices with out-edges
 * first, then the others, each part in order of decreasing in-degree (ties
 * by caller id), so that the arrival words of the most-targeted vertices
 * share cache lines and a vertex with nothing to expand is known by its id;
 * perm[v] is the internal id of caller vertex v.
 * All calls take and return caller ids.  In internal ids:
 *   off_out[n+1]  first out-edge of each tail;  out-edge e has
 *   t_out[e], and dst_a_out[2e], dst_a_out[2e+1] = head, arrival;
 *   off_in[n+1]   first in-edge of each head;   in-edge e has
 *   a_in[e], and src_t_in[2e], src_t_in[2e+1] = tail, departure. */
typedef struct kairos_index_view {
    const uint32_t *off_out, *t_out, *dst_a_out;
    const uint32_t *off_in, *a_in, *src_t_in;
    const uint32_t *perm;
    uint32_t n_live;
} kairos_index_view;
int kairos_graph_index(const kairos_graph *g, kairos_index_view *view);

/* -------------------------------------------------------------- queries --
 * Single-source queries (Alg. 2 for earliest arrival; latest departure and
 * fastest as named in §2.3 and Table 4).
 *   src             vertex id < n.
 *   t_alpha,t_omega query interval, t_alpha <= t_omega <= TMAX.
 *   out             device, n uint32, written in full.
 * Errors: INVALID (g or out null), RANGE, NOMEM, DEVICE.
 */
int kairos_earliest_arrival(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                            uint32_t *out);
int kairos_latest_departure(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                            uint32_t *out);
int kairos_fastest(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                   uint32_t *out);

/* Earliest-arrival paths (the minimal temporal paths of §2.3 with the edge
 * that realises each arrival).  out_arrival is as kairos_earliest_arrival.
 * For every vertex v other than src with a finite arrival, the last edge
 * (u, v, t, lambda) of an earliest-arrival path: among the usable edges into
 * v with t + lambda = arrival[v] and arrival[u] <= t, the latest departure
 * t, then the smallest u (edges equal in (u, v, t, lambda) are the same
 * choice).  out_pred_tail[v] = u, out_pred_departure[v] = t; both INF for
 * src and unreached vertices.  Following tails from any reached vertex ends
 * at src (arrivals strictly decrease along them).
 *   out_arrival, out_pred_tail, out_pred_departure  device, n uint32 each.
 * Errors: INVALID (a null pointer), RANGE, NOMEM, DEVICE. */
int kairos_earliest_arrival_path(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                                 uint32_t *out_arrival, uint32_t *out_pred_tail,
                                 uint32_t *out_pred_departure);

/* Temporal BFS (Table 4's T. BFS, restricted to the query interval as §6.1
 * does for BFS): out_hops[v] = the fewest edges of a time-respecting path
 * from src to v within [t_alpha, t_omega]; 0 for src, INF if unreachable.
 * The rounds are level-synchronous: round r expands the frontier from the
 * arrivals it had when r began, so the round that first reaches v is v's
 * hop count.  out_hops: device, n uint32.  Errors as above. */
int kairos_temporal_bfs(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                        uint32_t *out_hops);

/* One single-source query of a given kind under a chosen succession
 * predicate (§2.2: TemporalEdgeMap takes the predicate as a parameter).
 *   kind   KAIROS_EARLIEST_ARRIVAL, KAIROS_LATEST_DEPARTURE, KAIROS_FASTEST,
 *          KAIROS_TEMPORAL_BFS, KAIROS_LATEST_DEPARTURE_TO or
 *          KAIROS_SHORTEST_DURATION; out as for the matching call.
 *   flags  0: consecutive edges "Succeeds" (next departure >= previous
 *          arrival), as every other call here; KAIROS_STRICT: "Strictly
 *          succeeds" (next departure > previous arrival).  Under both, the
 *          first edge of a path (it has no predecessor) needs only
 *          t >= t_alpha, or t >= s when a latest-departure / fastest sweep
 *          starts the source at s.
 * Errors: INVALID (unknown kind or flag bit, null pointer), RANGE, NOMEM,
 * DEVICE. */
enum {
    KAIROS_EARLIEST_ARRIVAL = 0,
    KAIROS_LATEST_DEPARTURE = 1,
    KAIROS_FASTEST = 2,
    KAIROS_TEMPORAL_BFS = 3,
    KAIROS_LATEST_DEPARTURE_TO = 4, /* src names the target; see below */
    KAIROS_SHORTEST_DURATION = 5
};
#define KAIROS_STRICT 1u
int kairos_query(kairos_graph *g, int kind, uint32_t flags, uint32_t src, uint32_t t_alpha,
                 uint32_t t_omega, uint32_t *out);

/* Single-target latest departure (the single-target reading of §2.3's
 * latest-departure path): out[u] = the latest departure from u of a
 * time-respecting path that ends at `target` within [t_alpha, t_omega];
 * t_omega for the target, INF if u cannot reach it.  Answered on the
 * time-reversed graph (edge (u, v, t, lambda) read as (v, u, TMAX - t -
 * lambda, lambda)), which g builds from its own index on the first call and
 * keeps (another index's worth of device memory, counted by
 * kairos_graph_stats; it follows kairos_set_tuning).  KAIROS_STRICT in
 * kairos_query applies "Strictly succeeds" between consecutive edges; the
 * last edge into the target needs only an arrival by t_omega.
 *   out: device, n uint32.  Errors: INVALID, RANGE (target >= n, window),
 *   NOMEM, DEVICE. */
int kairos_latest_departure_to(kairos_graph *g, uint32_t target, uint32_t t_alpha, uint32_t t_omega,
                               uint32_t *out);

/* Earliest arrival that allocates nothing: for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, result and errors as
 * kairos_earliest_arrival, run with the same kernels; the query's state
 * lives in one fixed device array of KAIROS_NOALLOC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process exits.  The
 * call makes no hipMalloc / hipFree and no other allocation; it is not
 * profiled (kairos_profile_enable does not cover it).
 *   Limit: about 22 bytes per vertex plus a fixed chunk list must fit the
 *   array (graphs up to roughly 11 million vertices); a larger graph gets
 *   KAIROS_ERR_SCRATCH and nothing is written.
 *   Calls on one device share the array: the library serialises them with a
 *   lock (overlapping calls would race on it), and every word a query reads
 *   before writing is cleared at the start of each call.
 *   The graph must live on the current device (else INVALID).  Work runs on
 *   the graph's stream, or the null stream for a graph built without one;
 *   the call returns when out is complete. */
#define KAIROS_NOALLOC_SCRATCH_BYTES (256u << 20)
int kairos_earliest_arrival_noalloc(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                                    uint32_t *out);

/* Shortest duration (Table 4's "S. Duration" row, on which §6.1 builds
 * temporal betweenness): out[v] = the least total duration, the sum of
 * lambda over its edges, of a time-respecting path from src to v within
 * [t_alpha, t_omega]; 0 for src, INF if v is unreachable.  Waiting at a
 * vertex costs nothing, so this differs from fastest (arrival minus
 * departure).  The first call builds, once per graph, two maps from each
 * out-edge into the in-index: the position of the same edge, and that of the
 * last in-edge of its tail arriving by its departure (8 bytes per edge in
 * all, counted by kairos_graph_stats); each query also takes 4 bytes per
 * edge and 48 bytes per vertex of scratch state, pooled per graph (one set
 * per concurrent caller).  KAIROS_STRICT in kairos_query
 * applies "Strictly succeeds" between consecutive edges.
 *   out: device, n uint32.  Errors: INVALID, RANGE, NOMEM, DEVICE. */
int kairos_shortest_duration(kairos_graph *g, uint32_t src, uint32_t t_alpha, uint32_t t_omega,
                             uint32_t *out);

/* q earliest-arrival queries answered together.
 *   src, t_alpha, t_omega  host, q entries each.
 *   out                    device, q*n uint32, query-major (row i = query i).
 * Row i equals kairos_earliest_arrival for query i.  q == 0 is a no-op. */
int kairos_earliest_arrival_batch(kairos_graph *g, uint32_t q, const uint32_t *src,
                                  const uint32_t *t_alpha, const uint32_t *t_omega,
                                  uint32_t *out);

/* Temporal edges traversed by an earliest-arrival result: the number of
 * edges (u, v, t, a) with ea[u] finite, t >= max(ea[u], t_alpha) and
 * a <= t_omega.  ea: device, n entries (a result of the calls above);
 * count: host.  This is the numerator of the traversal rate. */
int kairos_traversed_edges(kairos_graph *g, uint32_t t_alpha, uint32_t t_omega,
                           const uint32_t *ea, uint64_t *count);

/* --------------------------------------------------------------- tuning --
 * Run-time parameters; they change speed, never results.  The paper derives
 * its equivalents (cost constants, selectivity threshold, index cut-off,
 * parallel grain; §5.1, §6.1) by experiment; kairos_autotune measures them
 * on a sample of the caller's own queries. */
typedef struct kairos_tuning {
    uint32_t block;          /* threads per workgroup of the push and chunk kernels
                                of single queries, sweeps and query-major
                                batches: 256 or 512 (512 launches half as many
                                blocks); the lane-dense batch, one-workgroup
                                and persistent kernels keep 256               */
    uint32_t chunk;          /* edges per chunk when a long adjacency is split     */
    uint32_t split;          /* adjacency ranges at least this long are split      */
    uint32_t pull_alpha;     /* pull when frontier out-edges > m / pull_alpha;
                                0 disables the pull kernel                          */
    uint32_t pull_beta;      /* back to push when frontier < n / pull_beta          */
    uint32_t rounds_per_sync;/* push rounds (and shortest-duration rounds)
                                queued before the host checks the frontier
                                (1 = check every round)                             */
    uint32_t batch_persistent; /* 1: a lane-dense batch (batch_layout 2) runs all
                                  its rounds in one cooperative launch with grid
                                  barriers and stops on the device; 0: one
                                  launch per phase and a host check per round   */
    uint32_t sweep_group;    /* departure times handled together by the
                                latest-departure / fastest sweep (1..64): each
                                group runs as that many queries warm-started
                                from the previous group's last one; 1 = one
                                departure time after the other; default 1
                                when m > 64 n, else 8 up to 2^21 vertices,
                                else 4                                        */
    uint32_t batch_layout;   /* 0: one wavefront per frontier vertex, one lane per
                                query, arrivals stored vertex-major (edges read
                                once per 64 queries); 1: one thread per query
                                and vertex, arrivals query-major; 2: vertex-major
                                arrivals, (vertex, query) pairs dealt densely to
                                threads; 3: sweep form -- every edge of a group's
                                windows once, in departure order, a lane per
                                query, slab by slab with fix-up passes (suits
                                groups whose windows overlap; falls back to 2
                                when a slab will not settle)                    */
    uint32_t tail_limit;     /* frontiers of at most this many entries run in one
                                workgroup that loops over rounds without host
                                round trips; 0 disables                          */
    uint32_t dense_frontier; /* single queries: a frontier of at least
                                n / dense_frontier vertices is expanded by
                                walking all vertices in id order; 0 disables     */
    uint32_t arrival_filter; /* bits (2, 4 or 8) of a per-vertex code that bounds
                                each arrival from above (the query's reachable
                                time range cut into 2^bits equal parts); an
                                edge arriving at or after its head's bound is
                                dropped before the arrival word is read.
                                0: off (the default).  Each query keeps the
                                width it started with                           */
    uint32_t single_persistent; /* 1: single queries run their rounds with more
                                than tail_limit frontier entries in one
                                cooperative launch (grid barriers, no host
                                round trip per round); needs pull_alpha 0      */
    uint32_t run_dedupe;     /* 1: lanes of a wavefront holding consecutive
                                edges into the same vertex (bursts of one
                                pair's contacts) issue one atomic per run; on
                                by default when more than 1/32 of the
                                out-edges repeat the previous edge's head     */
    uint32_t binned;         /* single earliest-arrival queries: a round whose
                                frontier holds at least this many entries is
                                destination-binned (claims, then candidates
                                counted and scattered to bins of 2^14 heads,
                                then applied bin by bin through LDS) instead
                                of relaxing each edge at its head's word;
                                0 = never.  Graphs of at most 2^26 vertices. */
} kairos_tuning;

int kairos_get_tuning(const kairos_graph *g, kairos_tuning *out);
/* KAIROS_ERR_INVALID for a value outside the documented sets.  Call it while
 * no query, batch or server of g is in flight; results never depend on it. */
int kairos_set_tuning(kairos_graph *g, const kairos_tuning *in);

/* Coordinate descent over the tuning space on q sample queries (host
 * arrays, as in the batch call): one query tunes the one-query path, more
 * tune the batch they form; the sweep group width is then tuned on
 * latest-departure queries from the first two sample sources.  Keeps the
 * fastest setting in g and copies it to *best (may be NULL).  Results never
 * change; only time does.  The sample should be held out from the queries
 * that will be timed.  When the environment variable KAIROS_TUNING_CACHE
 * names a file, settings are stored there per device and index shape
 * (architecture, compute units, n, m, vertices with out-edges, largest
 * out-degree, repeated heads, largest departure, one query or a batch) and a
 * stored setting is taken without measuring. */
int kairos_autotune(kairos_graph *g, uint32_t q, const uint32_t *src, const uint32_t *t_alpha,
                    const uint32_t *t_omega, kairos_tuning *best);

/* The same search with the objective named: KAIROS_TUNE_SINGLE times the
 * q sample queries answered one per call (kairos_earliest_arrival),
 * KAIROS_TUNE_BATCH as one batch.  kairos_autotune is this call with
 * KAIROS_TUNE_SINGLE for q == 1 and KAIROS_TUNE_BATCH otherwise.  INVALID
 * for another form. */
enum { KAIROS_TUNE_SINGLE = 0, KAIROS_TUNE_BATCH = 1 };
int kairos_autotune_form(kairos_graph *g, int form, uint32_t q, const uint32_t *src, const uint32_t *t_alpha,
                         const uint32_t *t_omega, kairos_tuning *best);

/* ------------------------------------------------------------ profiling --
 * When enabled, every kernel launch on g is bracketed by HIP events on the
 * stream it runs on and its algorithmic work is counted on the device.
 * Reading resolves the events (it synchronises g's streams) and resets. */
typedef enum kairos_kernel_class {
    KAIROS_K_PUSH = 0,  /* push temporal edge map: frontier expansion       */
    KAIROS_K_PULL = 1,  /* pull temporal edge map                           */
    KAIROS_K_INIT = 2,  /* per-query state initialisation and outputs       */
    KAIROS_K_SORT = 3,  /* index build                                      */
    KAIROS_K_CHUNK = 4, /* push temporal edge map: split long adjacencies   */
    KAIROS_K_TAIL = 5,  /* push temporal edge map: small frontiers, one
                           workgroup looping over rounds                  */
    KAIROS_K_BINNED = 6, /* push temporal edge map, destination-binned:
                           count, scatter and apply of a large round      */
    KAIROS_K_COUNT = 7
} kairos_kernel_class;

typedef struct kairos_profile {
    uint64_t launches[KAIROS_K_COUNT];
    double ms[KAIROS_K_COUNT];   /* summed event time                          */
    uint64_t edges_scanned;      /* out-edges read by the push kernel (8 B each);
                                    shortest duration: out-edges relaxed        */
    uint64_t chunk_edges;        /* out-edges read by the chunk kernel (8 B each) */
    uint64_t items;              /* frontier entries expanded by push (shortest
                                    duration: vertices expanded)                */
    uint64_t relaxations;        /* successful atomic minimum updates          */
    uint64_t relax_attempts;     /* atomic minimum updates issued              */
    uint64_t tail_edges;         /* out-edges read by the small-frontier kernel */
    uint64_t tail_items;         /* frontier entries expanded by it             */
    uint64_t pull_edges;         /* in-edges read by pull (12 B each)          */
    uint64_t pull_vertices;      /* vertices examined by pull                  */
    uint64_t rounds;             /* frontier rounds                            */
    uint64_t binned_edges;       /* out-edges claimed by destination-binned rounds */
    uint64_t binned_items;       /* frontier entries expanded by them          */
    uint64_t sweep_slabs;        /* slabs of the batch sweep form (batch_layout 3) */
    uint64_t sweep_passes;       /* its passes (pass 0 and fix-ups, all slabs)  */
    uint64_t sweep_fix_edges;    /* out-edges relaxed by its fix-up passes      */
    uint64_t sweep_fallbacks;    /* batches it handed to the lane-dense rounds  */
} kairos_profile;

int kairos_profile_enable(kairos_graph *g, int on);
int kairos_profile_read(kairos_graph *g, kairos_profile *out);

/* -------------------------------------------------------------- serving --
 * Continuous batching: queries are admitted into slots as they arrive while
 * others are on the device; each scheduler iteration runs a few frontier
 * rounds, each for every active slot in one launch, then retires finished
 * slots.  A latest-departure / fastest query moves to its next departure
 * time on the device between rounds, or, while slots are plentiful, runs
 * groups of departure times (tuning sweep_group) on consecutive slots.  A slot
 * is admitted only when one is free and the device reports at least the
 * slot's state size plus mem_reserve_bytes free.  The graph stays resident.
 */
typedef struct kairos_server kairos_server;

typedef struct kairos_server_opts {
    uint32_t max_slots;         /* concurrent queries on the device (>= 1)     */
    uint32_t queue_capacity;    /* waiting queries before submit returns BUSY  */
    uint64_t mem_reserve_bytes; /* device memory left free by admission        */
    void *hip_stream;           /* stream for server work, NULL = own stream   */
    uint32_t rounds_per_check;  /* push rounds between two host checks for
                                   finished queries (1..64; 0 = 4); more
                                   rounds spend less time in host round trips,
                                   fewer let finished queries leave sooner   */
} kairos_server_opts;

typedef struct kairos_completion {
    uint64_t ticket;
    int32_t status;             /* kairos_status of the query                  */
    int32_t kind;               /* 0 EA, 1 LD, 2 F                             */
    uint64_t t_submit_ns;       /* CLOCK_MONOTONIC at submit                   */
    uint64_t t_done_ns;         /* CLOCK_MONOTONIC when the result was ready   */
} kairos_completion;

/* g must outlive the server. */
int kairos_server_create(kairos_graph *g, const kairos_server_opts *opts, kairos_server **out);

/* Never blocks.  kind: 0 earliest arrival, 1 latest departure, 2 fastest.
 * out: device, n uint32; must stay valid until the completion is polled.
 * Returns BUSY when the waiting queue is full, RANGE/INVALID for bad
 * arguments (then no ticket is issued). */
int kairos_server_submit(kairos_server *s, int kind, uint32_t src, uint32_t t_alpha,
                         uint32_t t_omega, uint32_t *out, uint64_t *ticket);

/* Copies up to cap finished queries into done (host) and their number into
 * *n_done; never blocks. */
int kairos_server_poll(kairos_server *s, kairos_completion *done, uint32_t cap, uint32_t *n_done);

/* Waits for all submitted queries, stops the scheduler, frees the server. */
void kairos_server_free(kairos_server *s);

/* Counters of a server.  admitted_waits_mem counts the times the pool could
 * not grow for lack of device memory; pool_slots is the current pool size
 * and slot_bytes the device memory one slot takes (growing the pool from k
 * to k' slots needs k' * slot_bytes free, since the new pool is allocated
 * before the old one is released). */
typedef struct kairos_server_stats {
    uint64_t submitted, completed, iterations, admitted_waits_mem;
    uint32_t active_slots, waiting, max_slots_seen, pool_slots;
    uint64_t slot_bytes;
} kairos_server_stats;
int kairos_server_stats_read(kairos_server *s, kairos_server_stats *out);

/* Test hook: the server admits as if the device reported this many free
 * bytes (UINT64_MAX restores the real query). */
int kairos_server_set_free_bytes_override(kairos_server *s, uint64_t bytes);

/* Static description of a status code. */
const char *kairos_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* KAIROS_H */
