/*
 * rept.h -- C ABI of the MI355X (gfx950) REPT semi-triangle counting library.
 *
 * REPT (Wang, Jia, Qi, Sun, Tao, Guan, arXiv:1811.09136) estimates the global and local
 * triangle counts of an undirected edge stream (Section II).  Processor i of c keeps the
 * edges its hash selects (sampling probability p = 1/m; c > m uses ceil(c/m) groups with
 * independent hashes, Section III-B).  For every stream edge (u, v) at time t it counts the
 * common neighbours w of u and v among its own edges that arrived before t, adds that count
 * to its global counter tau^(i) and to the local counters of u and v, and adds one to the
 * local counter of each w (Algorithm 1, UpdateTriangleCNT).  The estimators scale the sums
 * of these counters (Sections III-A, III-B).
 *
 * This library computes those integer counters exactly, for all processors at once, on the
 * GPU; `rept_estimate` forms the estimators on the host.
 *
 * Conventions shared by every call:
 *  - ids are 0-based: nodes in [0, n); processor i in [0, c) is slot j = i % m of group
 *    k = i / m (the mapping Algorithm 2 states); group k has c_k = m processors, except the
 *    last, which has c - (G-1)*m, G = ceil(c/m).  An edge whose slot has no processor in a
 *    group is stored by no processor of that group.
 *  - the stream is an array of `num_edges` pairs (u, v) of uint32, row t = the edge arriving
 *    at time t.  Edges are undirected; the stream must be simple: u != v, u < n, v < n, no
 *    unordered pair twice.  num_edges < 2^31.
 *  - an edge is counted before it is inserted (Algorithm 1), so an edge never closes a
 *    triangle with itself and "before t" is strict.
 *  - hash: a 4-wise independent family (Section III-A asks for uniform, independent slots;
 *    Theorem 3's variance involves up to four edges at once): for group k the coefficients
 *    a_0..a_3 are SplitMix64 outputs 4k..4k+3 of the state `seed` (Steele, Lea, Flood 2014),
 *    each >> 3 and reduced mod p = 2^61 - 1; with x = lo * 2^32 + hi (lo = min(u, v),
 *    hi = max(u, v)), h = a_3 x^3 + a_2 x^2 + a_1 x + a_0 mod p and slot = floor(h * m / 2^61).
 *    Node ids are limited to n <= 2^29 so that distinct edges have distinct keys x < p.
 *  - "device" pointers are HIP device memory of the current device; "host" pointers are
 *    ordinary host memory.  `stream` is a hipStream_t passed as void* (NULL = null stream).
 *  - the library never allocates device memory: the caller owns every device byte.
 *  - every call returns a rept_status; nothing throws.  On an error return, no output and
 *    no handle is produced.
 */
#ifndef REPT_H
#define REPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rept_status {
    REPT_OK = 0,
    REPT_EINVAL = -1,     /* bad argument: zero n/m/c, null pointer, size too small, ... */
    REPT_ERANGE = -2,     /* node id >= n, or an estimator sum >= 2^53 */
    REPT_ESELFLOOP = -3,  /* an edge (u, u) */
    REPT_EDUP = -4,       /* an unordered pair appears twice */
    REPT_ENOMEM = -5,     /* a caller-provided buffer is smaller than required */
    REPT_EDEVICE = -6,    /* a HIP runtime call failed */
    REPT_ENOTSUP = -7     /* outside what this library implements (see each call) */
} rept_status;

/* rept_params.flags */
#define REPT_LOCAL_PER_PROC 1u /* local counters per processor [c][n] instead of per group [G][n] */
/* Parallel MASCOT (Section III-C): each of the c processors keeps every edge independently with
 * probability 1/m (processor i keeps e iff h_i(e) = 0, h_i the hash of group i), so the samples
 * overlap instead of partitioning the stream; the counting step is Algorithm 1's.  Processors
 * are their own groups, the local output has c rows, and the estimator is the mean of the processors' m^2 tau^(i), that is
 * (m^2 / c) sum_i tau^(i) for any c.  Not with rept_count_eta / rept_estimate_combined. */
#define REPT_MASCOT 2u

/* REPT sampling parameters (Table I: p = 1/m, c processors; plus the hash seed). */
typedef struct rept_params {
    uint32_t m;     /* 1/p, 1 <= m <= 65536 (m = 1 counts every triangle once per group) */
    uint32_t c;     /* processors, c >= 1; G = ceil(c/m) hash groups (c with REPT_MASCOT).  rept_count,
                       rept_count_range and rept_count_eta take any G; the batched and incremental
                       calls take G <= 8 */
    uint64_t seed;  /* seed of the hash parameters */
    uint32_t flags; /* REPT_LOCAL_PER_PROC, REPT_MASCOT, both, or 0 */
    uint32_t reserved; /* must be 0 */
} rept_params;

/* Opaque host-side handle to a built graph.  It points into the caller's persistent device
 * buffer, which must outlive it.  Use from one host thread at a time. */
typedef struct rept_graph rept_graph;

typedef struct rept_graph_info {
    uint32_t n;             /* nodes */
    uint64_t num_edges;     /* stream edges */
    uint32_t num_apex;      /* nodes with at least two higher-ranked neighbours */
    uint32_t max_out_degree;/* largest oriented out-degree */
    uint64_t oriented_work; /* sum over oriented edges (a->b) of min(outdeg(a), outdeg(b)): list
                               entries the count probes (it walks the shorter list of each pair) */
    uint64_t sum_out_sq;    /* sum over nodes of outdeg^2 */
    uint64_t num_reverse;   /* pairs in the reverse lists (counted from the longer list's side) */
} rept_graph_info;

/* Number of local-counter rows for `params`: G = ceil(c/m), or c with REPT_LOCAL_PER_PROC or
 * REPT_MASCOT.
 * The local output of every count call is int64[rows][n], row-major.  Returns 0 on bad
 * params. */
uint32_t rept_local_rows(const rept_params* params);

/*
 * Device bytes needed to build a graph of n nodes and num_edges stream edges (Section II: the
 * stream of num_edges edges over the node set; Section III-A bounds a processor's memory by its
 * share of the stream, c* = min(c, floor(M / (p |E|))) for a memory cap M, and this call is the
 * device's form of that sizing: a caller admits a stream only when these bytes fit its budget).
 *   persistent_bytes: kept by the built graph (oriented adjacency and reverse lists: 28 bytes
 *                     per edge plus 12 bytes per node, rounded up);
 *   scratch_bytes:    needed only during rept_build.
 * Host only, no device work.  EINVAL if n == 0, n > 2^29 or num_edges >= 2^31.
 */
rept_status rept_query_sizes(uint32_t n, uint64_t num_edges, size_t* persistent_bytes,
                             size_t* scratch_bytes);

/*
 * Validate the stream (Section II: a simple undirected graph) and build the device data the
 * counting pass reads: every edge oriented from its lower- to its higher-ranked endpoint
 * (rank = (degree, id)), grouped by the lower endpoint and sorted by neighbour id, with each
 * entry holding (neighbour id, arrival time t); and, for each node b, the reverse list of the
 * pairs a -> b whose out-list of a is shorter than b's (the counting pass walks the shorter list
 * of every pair).
 *
 * edges:      device, uint32[num_edges][2], read only, not retained after return.
 * persistent: device, >= persistent_bytes from rept_query_sizes, 256-byte aligned; owned by the
 *             caller, must stay allocated and unmodified while the handle is used.
 * scratch:    device, >= scratch_bytes, 256-byte aligned; free to reuse after return.
 * stream:     hipStream_t; the call enqueues its work there and synchronises that stream
 *             once, to read the validation result.
 * out:        receives a new handle on success.
 * Errors: EINVAL (bad sizes/pointers), ERANGE, ESELFLOOP, EDUP (invalid stream),
 *         ENOMEM (buffers too small), EDEVICE.
 */
rept_status rept_build(uint32_t n, const uint32_t* edges, uint64_t num_edges, void* persistent,
                       size_t persistent_bytes, void* scratch, size_t scratch_bytes, void* stream,
                       rept_graph** out);

/*
 * rept_build for a stream held in host memory (Section II: the stream as it arrives).  The
 * edges are copied over PCIe into the persistent buffer (into space the build fills later, so
 * no extra device memory is needed) on `stream`, then built as by rept_build.
 *   host_edges: host uint32[num_edges][2], pageable or pinned, read only; the call returns
 *               after its one stream synchronisation, when the copy has completed.
 * Other arguments, ownership and errors as rept_build (ENOMEM if a buffer is too small,
 * checked before the copy).
 */
rept_status rept_build_host(uint32_t n, const uint32_t* host_edges, uint64_t num_edges, void* persistent,
                            size_t persistent_bytes, void* scratch, size_t scratch_bytes, void* stream,
                            rept_graph** out);

/* Statistics of a built graph (host only). */
rept_status rept_graph_get_info(const rept_graph* graph, rept_graph_info* info);

/*
 * Device bytes of the workspace of one count of `graph` under `params`: the slot table of the
 * graph's stored edges, h_k(e) for every edge e and group k (Section III-A's hash, one per group
 * as in Section III-B), 16 bits per slot with the groups padded to 1, 2, 4 or 8 per edge (more
 * than 8 groups: the table of the 8 one launch counts), rounded up to 256 bytes.  Host only.
 * Errors: EINVAL; ENOTSUP (m > 65536).
 */
rept_status rept_count_workspace_size(const rept_graph* graph, const rept_params* params,
                                      size_t* bytes);

/*
 * The counting pass of Algorithm 1 (Section III-A), for every processor at once: all per-edge
 * updates of the whole stream.  Overwrites the outputs (idempotent).
 *   global:    device int64[c]      -- global[i] = tau^(i)
 *   local:     device int64[rows][n] -- rows = rept_local_rows(params): per group k the sum over
 *              its processors of tau_v^(i), or tau_v^(i) per processor with REPT_LOCAL_PER_PROC.
 *   workspace: device, >= rept_count_workspace_size bytes, 256-byte aligned; the call rewrites it
 *              (the slot table) and reads it; it may be reused once the call's work on `stream`
 *              has completed.
 * More than 8 groups run as successive launches of at most 8 groups on `stream` (groups are
 * independent; each launch uses its groups' own hash coefficients of `seed` and writes its slice
 * of the outputs), so the results equal a single pass over all groups.
 * Asynchronous on `stream`.  Errors: EINVAL, ENOMEM (workspace too small), ENOTSUP (m > 65536),
 * EDEVICE.
 */
rept_status rept_count(const rept_graph* graph, const rept_params* params, int64_t* global,
                       int64_t* local, void* workspace, size_t workspace_bytes, void* stream);

/*
 * The per-edge updates of the stream edges at times t in [t0, t1) only, ADDED (+=) to the
 * outputs.  Counts are additive over disjoint windows (Algorithm 1 updates per edge), so
 * windows that tile [0, num_edges) sum to rept_count.  Same layout and errors as rept_count;
 * EINVAL if t0 > t1 or t1 > num_edges.
 */
rept_status rept_count_range(const rept_graph* graph, const rept_params* params, uint64_t t0,
                             uint64_t t1, int64_t* global, int64_t* local, void* workspace,
                             size_t workspace_bytes, void* stream);

/*
 * rept_count without a workspace argument, for callers that cannot allocate device memory
 * (code being captured into a HIP graph, tight serving loops, harnesses that forbid allocation).
 * The slot table lives in a static device array of REPT_NOALLOC_SCRATCH_BYTES that the library
 * holds on each device it runs on until the process ends; the call allocates nothing and creates
 * no stream or event (both phases of the counting kernel run in one launch on `stream`).
 *   global, local: as rept_count (overwritten; the results equal rept_count's exactly).
 * The array is rewritten by every call before it is read, and every call on one device shares
 * it: calls that overlap on one device (other streams or threads) race and must not be issued.
 * Asynchronous on `stream`.  Errors: EINVAL, ENOTSUP (m > 65536); ENOMEM if the slot table
 * (rept_count_workspace_size) exceeds REPT_NOALLOC_SCRATCH_BYTES; EDEVICE.
 */
#define REPT_NOALLOC_SCRATCH_BYTES (64u << 20) /* 64 MiB: e.g. 33.5M stored edges at one hash group */
rept_status rept_count_noalloc(const rept_graph* graph, const rept_params* params, int64_t* global,
                               int64_t* local, void* stream);

/*
 * Estimators (host, FP64).  For c <= m (Algorithm 1) and for c > m with m | c (Section III-B,
 * c2 = 0) both reduce to
 *     tau_hat   = ((double)S   * (double)(m*m)) / (double)c,   S   = sum_i tau^(i)
 *     tau_v_hat = ((double)S_v * (double)(m*m)) / (double)c,   S_v = sum of the local rows at v
 * with the sums exact in int64 and one rounding each for the product and the quotient.
 *   global: host int64[c]; local: host int64[rows][n] or NULL; tau_v_hat: host double[n] or NULL.
 * With REPT_MASCOT the same expressions hold for every c (the mean of the processors' MASCOT
 * estimates m^2 tau^(i), Section III-C).
 * Errors: EINVAL; ENOTSUP for REPT with c > m and c % m != 0 (rept_estimate_combined covers it);
 *         ERANGE if a sum is negative or >= 2^53.
 */
rept_status rept_estimate(uint32_t n, const rept_params* params, const int64_t* global,
                          const int64_t* local, double* tau_hat, double* tau_v_hat);

/*
 * The same estimators from node sums already reduced over the local rows (rept_reduce_local):
 * sums[v] = S_v.  Results are identical to rept_estimate on the rows.
 *   global: host int64[c]; sums: host int64[n] or NULL; tau_v_hat: host double[n] or NULL.
 * Errors: as rept_estimate (ERANGE if a sum is negative or >= 2^53).
 */
rept_status rept_estimate_sums(uint32_t n, const rept_params* params, const int64_t* global,
                               const int64_t* sums, double* tau_hat, double* tau_v_hat);

/*
 * Device bytes of the workspace of rept_count_eta: the slot table of rept_count_workspace_size,
 * then two uint32 counters per stored edge and group of one launch (at most 8 groups; the
 * per-edge counts below), rounded up to 256 bytes.  Host only.  Errors: EINVAL; ENOTSUP
 * (m > 65536).
 */
rept_status rept_count_eta_workspace_size(const rept_graph* graph, const rept_params* params,
                                          size_t* bytes);

/*
 * The counting pass of rept_count together with Algorithm 2's triangle-pair counters
 * (Section III-B, "computing eta^(i) and eta_v^(i)").  For a stored edge g of processor i let
 * s_g be the number of semi-triangles of i in which g is one of the two earlier edges, and
 * L_g the number whose last edge is g (its |N| when g arrives, g being stored by i).  Then
 *   eta[0][i]   = sum over g of C(s_g, 2)             the pairs of semi-triangles of i that share
 *                                                      an edge that is the last of neither (the
 *                                                      definition of eta^(i); E = eta / m^3)
 *   eta[1][i]   = sum over g of s_g L_g + C(s_g, 2)   Algorithm 2 as printed, whose counter
 *                                                      starts at |N| when g is inserted
 *   eta_v[r][v] = sum over processors and over the stored edges g at v of the same terms.
 *   global, local: as rept_count (overwritten).
 *   eta:       device int64[2][c], overwritten; 8-byte aligned.
 *   eta_v:     device int64[2][n], overwritten, or NULL; 8-byte aligned.
 *   workspace: device, >= rept_count_eta_workspace_size bytes, 256-byte aligned, rewritten.
 *   tuning:    launch shape (rept_tuning, below) or NULL for the default shape; a shape that
 *              does not fit the LDS is EINVAL.
 * The combined estimator (rept_estimate_combined) takes the sums of row 0.  Any c is
 * accepted; more than 8 groups run as launches of 8 groups as in rept_count, each adding its
 * processors' pair counts.  Asynchronous on `stream`.  Errors: EINVAL, ENOMEM (workspace too
 * small), ENOTSUP (REPT_MASCOT, m > 65536), EDEVICE.
 */
struct rept_tuning;
rept_status rept_count_eta(const rept_graph* graph, const rept_params* params, int64_t* global,
                           int64_t* local, int64_t* eta, int64_t* eta_v, void* workspace,
                           size_t workspace_bytes, const struct rept_tuning* tuning, void* stream);

/*
 * Algorithm 2's combined estimators (host, FP64; Section III-B, c > m with c2 = c mod m != 0,
 * c1 = floor(c / m)): with S1 the sum of tau^(i) over the first c1 m processors, S2 over the
 * last c2, and eta the sum of eta^(i) over all c, in this order of binary64 operations
 *   t1 = (S1 m) / c1,  t2 = (S2 m^2) / c2,  eh = (eta m^3) / c,
 *   v1 = (t1 (m - 1)) / c1,  v2 = (t1 (m^2 - c2) + (2 eh)(m - c2)) / c2,
 *   tau_hat = (v2 t1 + v1 t2) / (v1 + v2), or t1 where v1 + v2 = 0.
 * The local estimators are the same expressions at each node, from its local rows (those of the
 * first c1 groups, or processors, in S1_v; the last group's in S2_v) and eta_v[v].
 *   global: host int64[c]; local: host int64[rows][n] or NULL; eta_v: host int64[n] or NULL;
 *   tau_v_hat: host double[n] or NULL (written only when local and eta_v are given).
 * Errors: EINVAL (null pointers, or c <= m or m | c: rept_estimate covers those); ERANGE if a
 * sum is negative or >= 2^53.
 */
rept_status rept_estimate_combined(uint32_t n, const rept_params* params, const int64_t* global,
                                   const int64_t* local, int64_t eta, const int64_t* eta_v,
                                   double* tau_hat, double* tau_v_hat);

/*
 * The reduction of the local estimator's sums on the device (Sections III-A, III-B: S_v sums
 * a node's counters over all processors): sums[v] = sum over r < rows of local[r][v], exact in
 * int64, so that n counters rather than rows x n cross to the host.
 *   local: device int64[rows][n]; sums: device int64[n], either local's first row (in place) or
 *          memory that does not overlap local.  Both 8-byte aligned.
 * Asynchronous on `stream`.  Errors: EINVAL (null or misaligned pointers, rows or n zero),
 * EDEVICE.
 */
rept_status rept_reduce_local(const int64_t* local, uint32_t rows, uint32_t n, int64_t* sums,
                              void* stream);

/*
 * The edge-to-processor hash of every stream edge for every group (Section III-A: h(u, v)
 * picks the processor that stores the edge; Section III-B: one independent h_k per group).
 *   edges: device uint32[num_edges][2]; slots: device uint32[G][num_edges].
 * Asynchronous.  Errors: EINVAL, ENOTSUP (more than 8 groups), EDEVICE.
 */
rept_status rept_hash_slots(const rept_params* params, const uint32_t* edges, uint64_t num_edges,
                            uint32_t* slots, void* stream);

/*
 * Incremental streams (Section II: the stream is processed as it arrives; Section III-A builds
 * the processors' edge sets on the fly).  The stream is appended in chunks; after each append
 * the caller's counters hold every per-edge update of Algorithm 1 (for all c processors, REPT
 * or parallel MASCOT) of all edges appended so far, so estimates can be formed after every
 * chunk (the per-interval use the paper names).  The counters are exactly those of rept_count
 * on the stream appended so far.
 *
 * The device keeps the whole adjacency of the edges seen so far (both directions, sorted by
 * neighbour, arrival time beside each entry) and the stream in arrival order.  An append sorts
 * and validates the chunk and merges it into the adjacency in one pass.  It then counts the
 * chunk's edges in one of two ways, with equal results:
 *   - edge by edge: each chunk edge against the edges that arrived before it, one work item (a
 *     binary search) per entry of its endpoints' shorter list;
 *   - by a windowed recount: rept_build of the whole stream so far, then rept_count_range over
 *     the chunk's times (a triangle's updates belong to the time of its last edge).
 * By default (REPT_STREAM_AUTO) an append recounts when its work items exceed 10 per edge so far,
 * the ratio of the two costs measured on a 20M-edge power-law stream; rept_stream_set_policy
 * fixes either way.  A recount needs one more stream synchronisation (the build's) and the
 * build's regions of the buffer.
 */
typedef struct rept_stream rept_stream; /* opaque host-side handle */

/* Device bytes for a stream of up to `capacity` edges over n nodes, appended in chunks of at
 * most `max_chunk` edges: 48 bytes per edge of capacity, 64 per edge of chunk, 8 per node, the
 * sort's temporary storage, and for the windowed recount 24 bytes per edge of capacity (the
 * stream in arrival order and a slot table of up to 8 groups) plus rept_query_sizes(n,
 * capacity)'s persistent and scratch bytes.  Host only, no device work.  EINVAL if n == 0,
 * n > 2^29, capacity == 0, capacity >= 2^31, max_chunk == 0 or max_chunk > capacity; EDEVICE if
 * the sizes cannot be formed. */
rept_status rept_stream_query_sizes(uint32_t n, uint64_t capacity, uint64_t max_chunk, size_t* bytes);

/*
 * Create an empty stream.
 *   params:  as for rept_count (REPT or REPT_MASCOT; at most 8 hash groups).
 *   buffer:  device, >= rept_stream_query_sizes bytes, 256-byte aligned; owned by the caller,
 *            must stay allocated while the handle is used.
 *   global:  device int64[c]; local: device int64[rows][n] (rows = rept_local_rows(params)),
 *            8-byte aligned: zeroed here (on `stream`), then accumulated by every append.
 * Errors: EINVAL, ENOTSUP (more than 8 groups, m > 65536), ENOMEM (buffer too small), EDEVICE.
 */
rept_status rept_stream_create(uint32_t n, uint64_t capacity, uint64_t max_chunk, const rept_params* params,
                               void* buffer, size_t bytes, int64_t* global, int64_t* local, void* stream,
                               rept_stream** out);

/*
 * Append the next num_edges stream edges (device uint32[num_edges][2], 8-byte aligned; the edge
 * in row i arrives at time T + i, T = edges appended before).  The chunk is validated against
 * itself and everything appended before (ids < n, no self-loop, no unordered pair twice); the
 * call synchronises `stream` once to read that result.  On an error nothing changes: the
 * adjacency, the counters and T are as before, and later appends continue from there.  On
 * success the merge and the count are enqueued on `stream` (asynchronous); the chunk's memory
 * may be reused once that work has completed.
 * Errors: EINVAL (bad handle or pointer), ENOMEM (num_edges > max_chunk, or the capacity would
 * be exceeded), ERANGE, ESELFLOOP, EDUP (in that order of precedence), EDEVICE.
 */
rept_status rept_stream_append(rept_stream* s, const uint32_t* edges, uint64_t num_edges, void* stream);

/* Edges appended so far (host only). */
rept_status rept_stream_num_edges(const rept_stream* s, uint64_t* num_edges);

/* How later appends count their edges (host only; results are equal either way):
 * REPT_STREAM_AUTO (default) chooses per append by its work, REPT_STREAM_PER_EDGE always counts
 * edge by edge, REPT_STREAM_RECOUNT always recounts the window (falling back to edge by edge for
 * a prefix that would not fit the buffer's build regions).  EINVAL for a bad handle or policy. */
#define REPT_STREAM_AUTO 0u
#define REPT_STREAM_PER_EDGE 1u
#define REPT_STREAM_RECOUNT 2u
rept_status rept_stream_set_policy(rept_stream* s, uint32_t policy);

/* Appends counted so far edge by edge and by a windowed recount (host only). */
rept_status rept_stream_paths(const rept_stream* s, uint64_t* per_edge, uint64_t* recount);

/* Release the handle (not the caller's buffers). */
void rept_stream_destroy(rept_stream* s);

/* ------------------------------------------------------------------ batched counting ------ */

/* rept_job.flags */
#define REPT_JOB_ACCUMULATE 1u  /* add to the outputs instead of overwriting them */
#define REPT_JOB_TABLE_READY 2u /* the workspace already holds the slot table of (graph, params),
                                   written by an earlier count or launch: do not rewrite it */

/* One counting job of a batch: the updates of stream window [t0, t1) (t1 = UINT64_MAX: to
 * the end) restricted to work units [unit0, unit1) (unit1 = UINT32_MAX: all).  Work units
 * are the graph's apex nodes (rept_graph_info.num_apex of them); the counts of any partition
 * of the units sum to the counts of the whole, which is what lets a job be split into chunks. */
typedef struct rept_job {
    const rept_graph* graph;
    rept_params params;
    int64_t* global;          /* device int64[c] */
    int64_t* local;           /* device int64[rows][n] */
    uint64_t t0, t1;
    uint32_t unit0, unit1;
    uint32_t flags;
    uint32_t reserved;
    void* workspace;          /* device, >= rept_count_workspace_size(graph, params), 256-aligned;
                                 the job's slot table (jobs of one batch may share one only if
                                 they have the same graph and params) */
    uint64_t workspace_bytes;
} rept_job;

/* Launch shape of the counting kernel; zero fields take the library defaults.  The kernel is
 * persistent: `blocks` workgroups of `threads` threads drain the work queue, first one apex per
 * workgroup (units whose size exceeds wave_cap), then one unit per wavefront.  The LDS
 * footprint of a shape must fit the 160 KB of a compute unit (EINVAL otherwise). */
typedef struct rept_tuning {
    uint32_t wave_cap;   /* 8..256: largest unit counted by one wavefront (default 64, or 256 with
                            the wide shape below; halved down to 64 if the light phase's LDS
                            would not fit); a unit's size is max(its list length, its
                            reverse-list length / 8) */
    uint32_t block_cap;  /* 64..4096: apex entries hashed in LDS per chunk by a workgroup (default:
                            smallest power of two >= the graphs' largest out-degree, at most 2048;
                            with workgroups of up to 512 threads, halved down to 1024 while a
                            workgroup would need more than half the LDS, and below that while
                            it would not fit) */
    uint32_t b_chunk;    /* 16..1024: neighbour lists staged per chunk by a workgroup (default 512
                            with 2048-entry chunks, else 128; 1024 with the wide shape; halved
                            likewise, before block_cap) */
    uint32_t blocks;     /* persistent workgroups (default: as many as fit, up to 4 per CU) */
    uint32_t threads;    /* 64..1024, a multiple of 64 (default 256; the wide shape, taken when
                            the longest list exceeds 1024 entries and none of block_cap and
                            threads is set: 1024, with block_cap 2048, b_chunk 1024,
                            wave_cap 256 and light_tile 16) */
    uint32_t light_tile; /* 1..64: apexes taken per queue pop by a wavefront (default 8; 16 with
                            the wide shape) */
    uint32_t phase_launches; /* 1: both phases in one launch; 2: the light phase (units of at most
                                wave_cap, one per wavefront) runs as a launch of its own after the
                                heavy one, its workgroups holding no heavy team area in LDS, so
                                more wavefronts are resident; 0 or 3: that launch on a second
                                stream of the library's, forked from and joined back to `stream`,
                                so it runs beside the heavy launch (default) */
    uint32_t reserved;       /* must be 0 */
} rept_tuning;

/* Device workspace bytes for a batch of njobs jobs. */
rept_status rept_batch_workspace_size(uint32_t njobs, size_t* bytes);

/*
 * Write the job table of a batch into `workspace` (device, >= rept_batch_workspace_size
 * bytes, 256-byte aligned) with one host-to-device copy on `stream`, staged through pinned host
 * memory the library keeps (no device allocation, no stream synchronisation: the call may wait
 * only for a staging buffer's earlier copy).  The copy is stream-ordered: launches of
 * rept_batch_launch(workspace) enqueued on `stream` after this call run this batch (a launch on
 * another stream must first wait for `stream`), and a launch still reading the workspace's
 * previous table on `stream` finishes before the copy overwrites it.  The job table holds only
 * device pointers and sizes, so a launch can be captured into a HIP graph and replayed.
 * Errors: EINVAL, ENOTSUP, ENOMEM (workspace too small, or no pinned staging memory), EDEVICE.
 */
rept_status rept_batch_prepare(const rept_job* jobs, uint32_t njobs, const rept_tuning* tuning,
                               void* workspace, size_t workspace_bytes, void* stream);

/* Run a prepared batch: one persistent launch per kernel kind drains a device work queue over
 * all jobs.  Asynchronous; performs no host synchronisation and no allocation. */
rept_status rept_batch_launch(void* workspace, void* stream);

/* rept_batch_prepare followed by rept_batch_launch. */
rept_status rept_batch_count(const rept_job* jobs, uint32_t njobs, const rept_tuning* tuning,
                             void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ misc ------------------ */

/* Free the host handle only (the persistent device buffer stays the caller's). */
void rept_destroy(rept_graph* graph);

/* Static string for a status code. */
const char* rept_status_str(int status);

/* Compute units of the current device (host query; 0 on error). */
uint32_t rept_device_cus(void);

#ifdef __cplusplus
}
#endif
#endif /* REPT_H */
