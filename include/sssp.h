/*
 * sssp.h - C ABI of the MI355X (gfx950) stepping-SSSP library, libsssp.so.
 *
 * The library solves single-source shortest paths on directed graphs with
 * non-negative integer weights by the stepping-algorithm framework of Dong,
 * Gu, Sun and Zhang, "Efficient Stepping Algorithms and Implementations for
 * Parallel Shortest Paths" (SPAA 2021):
 *
 *   Sec. 3.2, Alg. 1: delta[.] = inf; delta[s] = 0; Update(s);
 *                     while |Q| > 0: theta = ExtDist; for u in Extract(theta):
 *                     for v in N(u): if WriteMin(delta[v], delta[u] + w(u,v)):
 *                     Update(v).
 *   Sec. 3.1, Table 1: the lazy-batched priority queue (LaB-PQ) interface:
 *                     Update(id) marks id as (re)inserted with key delta[id];
 *                     Extract(theta) returns and removes every id whose key
 *                     is <= theta, and never runs concurrently with Update.
 *   Sec. 4.3:         the flat-array LaB-PQ (one flag per vertex, Extract
 *                     scans and packs), realised here as a device bitmap
 *                     plus an explicit frontier list while the queue is small
 *                     (the sparse/dense optimisation of Sec. 6).
 *   Table 2:          the threshold rules (rho-stepping, Delta*-stepping,
 *                     Bellman-Ford; theta = min for tests).
 *
 * The whole loop runs in one persistent kernel per source, without host
 * round trips between steps. All distance arithmetic is exact: weights are
 * uint32, distances uint64, and an unreachable vertex reads UINT64_MAX.
 *
 * Conventions for every entry point:
 *   - Functions return an sssp_status; nothing aborts, throws or exits.
 *   - On error, sssp_last_error() returns a thread-local detail string.
 *   - "Device pointer" means memory allocated on the current HIP device
 *     (hipMalloc or a torch tensor on that device); "host pointer" means
 *     ordinary process memory.
 *   - Streams are hipStream_t values passed as void*; NULL is the default
 *     stream.
 */
#ifndef SSSP_H
#define SSSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSSP_ABI_VERSION 4

typedef enum {
  SSSP_OK = 0,
  SSSP_ERR_INVALID_ARGUMENT = 1, /* a NULL pointer, a bad size, rule or parameter */
  SSSP_ERR_INVALID_GRAPH = 2,    /* CSR arrays violate the rules of sssp_graph_create */
  SSSP_ERR_OUT_OF_MEMORY = 3,    /* a device allocation failed */
  SSSP_ERR_NO_DEVICE = 4,        /* no HIP device, or it cannot run a cooperative launch */
  SSSP_ERR_DEVICE = 5,           /* a HIP runtime call or the kernel failed */
  SSSP_ERR_STEP_LIMIT = 6,       /* params.max_steps steps ran and the queue is not empty */
  SSSP_ERR_UNSUPPORTED = 7,      /* a valid request this build does not implement */
  SSSP_ERR_CANCELLED = 8         /* an asynchronous solve stopped by sssp_solve_cancel */
} sssp_status;

/* Threshold rules (ExtDist of Alg. 1; Table 2). Every rule yields the same
 * distance array; they differ in steps and work only. */
typedef enum {
  /* rho-stepping (Sec. 3.2 and Sec. 6): theta = the rho-th smallest key in Q,
   * estimated from s = ceil(10 * (q / rho + log q)) uniform samples of the
   * queue, log q = 1 + log2(q + 1), taking the ceil(rho * s / q)-th smallest
   * (App. B, c = 10). If q <= rho the whole queue is extracted. The first two
   * steps whose queue holds more than floor(rho / 10) vertices use
   * floor(rho / 10) instead of rho (Sec. 6). s is capped at
   * tuning.sample_cap and, in steps that scan the bitmap, by the probes
   * tuning.probe_cap allows (see sssp_tuning); the rank ceil(rho s / q) uses
   * the number of samples actually drawn. */
  SSSP_RULE_RHO = 0,
  /* Delta*-stepping (Table 2, Thm. 5.5): theta = i * Delta, i = 1, 2, ...
   * advancing every step, skipping ahead to ceil(min key / Delta) when the
   * buckets in between are empty. */
  SSSP_RULE_DELTA_STAR = 1,
  /* Bellman-Ford (Table 2): theta = +inf, every queued vertex each step. */
  SSSP_RULE_BF = 2,
  /* theta = the minimum key in Q (Table 2, Dijkstra row). Sequential by
   * nature; provided so tests can pin exact step counts. */
  SSSP_RULE_MIN = 3,
  /* rho-stepping with the exact rho-th smallest key in Q (Table 2, rho row)
   * instead of a sampled estimate: a radix selection over every queued key,
   * 8 bits per pass below the highest bit where the queue's minimum and
   * maximum keys differ. Each step then extracts at least min(rho, q)
   * vertices, exactly rho when keys are distinct. Costs one pass over the
   * queue per 8 bits (plus one for the bounds) where sampling costs one
   * small sample. rho >= 1. */
  SSSP_RULE_RHO_EXACT = 4
} sssp_rule;

typedef enum { SSSP_OFFSETS_I32 = 0, SSSP_OFFSETS_I64 = 1 } sssp_offset_width;

/* sssp_graph_create flags */
#define SSSP_INPUT_HOST 0x1u   /* offsets/targets/weights are host pointers */
#define SSSP_INPUT_DEVICE 0x2u /* offsets/targets/weights are device pointers */
#define SSSP_TRUST_INPUT 0x4u  /* skip CSR validation (caller guarantees it) */
#define SSSP_UNDIRECTED 0x10u  /* the caller asserts that every arc (u, v, w) has its reverse
                                  (v, u, w), as in an undirected graph; checked on the device with
                                  64-bit multiset checksums unless SSSP_TRUST_INPUT. Enables
                                  bidirectional relaxation (sssp_tuning.pull). */
#define SSSP_KEEP_ORDER 0x8u   /* keep the caller's vertex numbering internally (by default the
                                  library renumbers vertices by decreasing out-degree for cache
                                  locality; results are always in the caller's ids) */
#define SSSP_BORROW_DEVICE 0x20u /* with SSSP_INPUT_DEVICE: use the caller's targets and weights
                                  arrays in place instead of copying them into the library's packed
                                  arcs (saves 8 bytes per arc; each arc is then read as two 4-byte
                                  loads). Implies SSSP_KEEP_ORDER. Offsets are still copied (8 (n+1)
                                  bytes). The caller keeps both arrays allocated, at the same
                                  addresses, until sssp_graph_destroy; weights it changes in place
                                  between solves are the weights of the next solve (targets must
                                  stay valid: they are checked only at creation) */

/* Tuning knobs. Zero in any field selects the library default. None of them
 * changes the distances; they change speed, steps and work only. */
typedef struct {
  uint32_t blocks_per_cu; /* workgroups per compute unit in the persistent grid
                             (clamped to what can be co-resident) */
  uint32_t hub_degree;    /* out-degree above which a frontier vertex's edges are
                             split into chunks shared by many workgroups */
  uint32_t chunk_edges;   /* edges per hub chunk */
  uint32_t list_divisor;  /* keep an explicit frontier list while |Q| <= n / list_divisor;
                             0xFFFFFFFF disables the list (bitmap scans only) */
  uint32_t sample_cap;    /* maximum rho-stepping sample size (default 2^16: App. B's s is
                             drawn whole unless it exceeds this) */
  uint32_t probe_cap;     /* maximum bitmap probes per sampled step (default 2^16; a bitmap
                             step probes about 1.25 s n / q vertex ids, keeping those in Q,
                             so at most about probe_cap q / n samples are drawn there) */
  uint32_t no_filter;     /* 1 = skip the read-before-atomic filter in Relax */
  uint32_t teams;         /* independent solves in flight: the persistent grid is split into
                             this many teams of workgroups, each solving one source at a time
                             (must divide the grid size). 0 = 1 for a single source, else a
                             power of two >= 8, about one team per source */
  uint32_t local_budget;  /* local expansion (large neighbour sets, Sec. 6): in super-sparse
                             steps a workgroup relaxes the vertices its WriteMins bring to
                             at most theta itself, hop after hop, up to this many per step,
                             instead of returning them to Q (default 4096; 0xFFFFFFFF = off;
                             always off with SSSP_SOLVE_SNAPSHOT_KEYS). Only vertices of
                             out-degree at most 8 * super_sparse_degree (and at most
                             hub_degree) are relaxed this way; others go to Q */
  uint32_t super_sparse_degree; /* steps on the explicit list whose previous step relaxed fewer
                             arcs than this per vertex count as super-sparse (default 10;
                             the first step compares the graph's average out-degree); local
                             expansion runs only on graphs whose average out-degree is below
                             it */
  uint32_t pull;          /* bidirectional relaxation (Sec. 6): before pushing from u, lower
                             u's key with its neighbours' keys. Needs a graph created with
                             SSSP_UNDIRECTED. 0 = library default (off), 1 = on
                             (INVALID_ARGUMENT on other graphs), 0xFFFFFFFF = off; always off
                             with SSSP_SOLVE_SNAPSHOT_KEYS */
  uint32_t group_max;     /* serving only: the most teams that solve one request together.
                             A request is dispatched to k idle teams, k the largest power of
                             two with k * (waiting requests) <= idle teams, at most group_max,
                             so few requests in flight get most of the grid each (0 = all of
                             the server's teams; 1 = one team per request) */
  uint32_t queue;         /* LaB-PQ structure (Sec. 4): 0 = the flat array (a bitmap, plus an
                             explicit list while the queue is small; Sec. 4.3, 6); 1 = a
                             tournament tree (Sec. 4.2, Alg. 2) of fan-out 64 over the bitmap:
                             each node keeps the smallest key queued below it, lowered with an
                             atomic min on every successful WriteMin (Mark, stopping where a
                             node already holds a smaller key) and recomputed by the workgroup
                             that extracts below it; Extract descends only into nodes whose key
                             is at most theta. Same extracted sets, so the same distances.
                             In this mode hub_degree is capped at 64 (a workgroup extracts
                             4096 consecutive vertices, so larger rows are shared instead) */
  uint32_t repeat_skip;   /* skip pushing a vertex's arcs (or a hub chunk's) again when its key has
                             not changed since they were last pushed: every such WriteMin would
                             fail. Costs 8 bytes per vertex and per hub chunk for each team.
                             0 = library default (on for launches of one team on graphs whose
                             average out-degree is at least super_sparse_degree), 1 = on,
                             0xFFFFFFFF = off */
  uint32_t hub_defer_degree; /* SSSP_RULE_RHO, sampled steps: a queued vertex of out-degree at
                             least this (rounded down to a power of two) is extracted only when
                             its key is at most theta_h, the (rho / hub_defer_div)-th smallest
                             key of the same sample, not theta. A high-degree vertex's key keeps
                             falling while the frontier passes its many neighbours, so relaxing
                             it at once means relaxing it again after each fall. Every other
                             vertex at or below theta is still extracted and the smallest key is
                             always at or below theta_h, so the distances do not change; steps
                             and arcs relaxed do. Needs the degree numbering (ignored under
                             SSSP_KEEP_ORDER and SSSP_BORROW_DEVICE). 0 = library default
                             (off), 0xFFFFFFFF = off */
  uint32_t hub_defer_div;   /* theta_h's rank divisor for hub_defer_degree (0 = default 10) */
  uint32_t group_min;       /* serving only: the fewest teams a request is dispatched to (rounded
                             down to a power of two, at most group_max); a request waits while
                             fewer teams are idle rather than run on one or two of them (0 = 1) */
} sssp_tuning;

/* One record per step, written when params.trace is set. */
typedef struct {
  uint64_t theta;     /* threshold used by Extract (UINT64_MAX = +inf) */
  uint64_t q;         /* |Q| before Extract */
  uint64_t extracted; /* vertices returned by Extract */
  uint64_t edges;     /* arcs relaxed (out-degree sum of the extracted vertices) */
  uint64_t successes; /* WriteMin calls that lowered a distance */
  uint32_t flags;     /* bit 0: Extract scanned the bitmap (else the list);
                         bit 1: an explicit list was built for the next step;
                         bit 2: theta came from sampling;
                         bit 3: theta came from the exact selection */
  uint32_t samples;   /* sample size when bit 2 is set */
  uint64_t local;     /* vertices relaxed by local expansion */
  uint64_t extract_ns; /* wall-clock time of the step's threshold and Extract phases */
  uint64_t relax_ns;   /* wall-clock time of the step's Relax phase (with local expansion) */
} sssp_step_record;

/* sssp_params.flags */
#define SSSP_SOLVE_SNAPSHOT_KEYS 0x1u /* Relax each extracted vertex with the key it had when it was
                                         extracted, instead of its current key (which another
                                         relaxation of the same step may already have lowered).
                                         Extraction sets, step counts and traces then do not depend
                                         on the order in which concurrent WriteMins land, so runs
                                         with the Delta*, Bellman-Ford and min rules repeat exactly;
                                         usually more relaxations than the default. */

typedef struct {
  uint32_t rule;      /* sssp_rule */
  uint32_t flags;     /* SSSP_SOLVE_* bits; others must be 0 */
  uint64_t rho;       /* SSSP_RULE_RHO: rho >= 1 */
  uint64_t delta;     /* SSSP_RULE_DELTA_STAR: Delta >= 1 */
  uint64_t seed;      /* sampling seed (rho rule); affects steps and work only */
  uint64_t max_steps; /* 0 = unlimited; else stop with SSSP_ERR_STEP_LIMIT */
  const sssp_tuning* tuning; /* host pointer or NULL for defaults */
  /* Optional device pointer, n uint32 entries per source (row-major like
   * dist): entry v is incremented each time v is extracted. The caller
   * zeroes it. NULL disables counting. */
  uint32_t* extract_counts;
  /* Optional device pointer to trace_capacity records (first source only);
   * steps beyond the capacity are not recorded. NULL disables tracing. */
  sssp_step_record* trace;
  uint64_t trace_capacity;
} sssp_params;

typedef struct {
  uint64_t steps;            /* loop iterations (sum over sources) */
  uint64_t extracted;        /* sum of |Extract| over steps */
  uint64_t edges_relaxed;    /* arcs relaxed, counting repeats */
  uint64_t writemin_success; /* WriteMin calls that lowered a distance */
  uint64_t dense_steps;      /* steps whose Extract scanned the bitmap */
  uint64_t sampled_steps;    /* rho steps whose threshold came from sampling */
  double device_ms;          /* GPU time of the solve kernels, HIP events */
  /* Wall-clock split by phase, measured by the first team between its
   * consecutive barriers (over all sources it solved): [0] init (S0),
   * [1] threshold sampling (S1, rho rule), [2] Extract (S2), [3] Relax +
   * Update (S3, S4). */
  double phase_ms[4];
  /* Relax load balance in the first team, summed over its steps: [0] the
   * slowest workgroup's Relax time, [1] the mean workgroup's Relax time. */
  double relax_wg_ms[2];
  uint64_t teams;            /* teams the grid was split into */
  uint64_t queue_dense;      /* sum of |Q| over steps whose Extract scanned the bitmap */
  uint64_t queue_list;       /* sum of |Q| over steps whose Extract read the explicit list */
  uint64_t list_appends;     /* entries written to explicit lists (kept and new members) */
  uint64_t local_vertices;   /* vertices relaxed by local expansion (not counted in extracted) */
  uint64_t repeat_skipped;   /* arcs not pushed again because their tail's key had not changed since
                                they were last pushed (every such WriteMin would fail; not counted
                                in edges_relaxed) */
} sssp_stats;

typedef struct sssp_graph sssp_graph; /* opaque */

/* Fill *p with defaults: rule = RHO, rho = 2^20, delta = 2^13, seed = 1,
 * unlimited steps, default tuning, no counters, no trace. */
void sssp_default_params(sssp_params* p);

/*
 * Create a graph on the current HIP device from CSR arrays (Sec. 2 graph
 * notation: arcs (u, v) with weight w(u, v) >= 0; N(u) = row u).
 *   n        number of vertices, 1 <= n < 2^31.
 *   m        number of arcs, 0 <= m < 2^40.
 *   ow       width of `offsets` entries (SSSP_OFFSETS_I32 needs m < 2^31).
 *   offsets  n + 1 entries: offsets[0] = 0, non-decreasing, offsets[n] = m.
 *            Row u holds arcs offsets[u] .. offsets[u+1]-1.
 *   targets  m int32 entries in [0, n).
 *   weights  m uint32 entries (zero allowed). Parallel arcs and self-loops
 *            are allowed.
 *   flags    exactly one of SSSP_INPUT_HOST / SSSP_INPUT_DEVICE, optionally
 *            SSSP_TRUST_INPUT, SSSP_KEEP_ORDER, SSSP_UNDIRECTED and (with
 *            SSSP_INPUT_DEVICE) SSSP_BORROW_DEVICE.
 *   stream   stream for the upload (the call returns after it completes).
 * The library copies the arrays into its own device layout (unless
 * SSSP_BORROW_DEVICE); the caller keeps ownership of its arrays and may free
 * them on return (with SSSP_BORROW_DEVICE: only its offsets array). Errors:
 * INVALID_ARGUMENT, INVALID_GRAPH (validation failed; detail names the first
 * offending index), OUT_OF_MEMORY, NO_DEVICE, DEVICE. On error *out is NULL.
 */
sssp_status sssp_graph_create(int64_t n, int64_t m, sssp_offset_width ow, const void* offsets,
                              const int32_t* targets, const uint32_t* weights, uint32_t flags, void* stream,
                              sssp_graph** out);

/* Release the graph and its device memory. NULL is accepted. Must not race a
 * solve on the same graph; refused (INVALID_ARGUMENT) while a server runs on
 * it or an asynchronous solve is pending (sssp_solve_wait first). */
sssp_status sssp_graph_destroy(sssp_graph* g);

/* Query sizes: vertices, arcs and device bytes held (graph, with its per-arc
 * target rows once built, plus workspace). */
sssp_status sssp_graph_info(const sssp_graph* g, int64_t* n, int64_t* m, uint64_t* device_bytes);

/*
 * Solve from each of n_src sources (Alg. 1 once per source). All sources run
 * in one persistent launch: its workgroups form tuning.teams teams, and each
 * team takes the next unsolved source until none is left, so independent
 * queries proceed side by side.
 *   sources  host array of n_src vertex ids in [0, n).
 *   params   rule and parameters (see sssp_params); NULL = defaults.
 *   dist     device pointer to n_src * n uint64 entries, row-major:
 *            dist[i * n + v] = exact distance from sources[i] to v, or
 *            UINT64_MAX if v is unreachable. Overwritten completely.
 *   stream   stream the kernels run on; the call returns after they finish.
 *   stats    host pointer or NULL; receives totals over all sources.
 * The graph's workspace is reused, so calls on one graph must not overlap.
 * Errors: INVALID_ARGUMENT (bad pointer, source, rule, rho = 0 or delta = 0),
 * STEP_LIMIT (dist then holds upper bounds), DEVICE, OUT_OF_MEMORY.
 */
sssp_status sssp_solve(const sssp_graph* g, const int32_t* sources, int32_t n_src, const sssp_params* params,
                       uint64_t* dist, void* stream, sssp_stats* stats);

/*
 * sssp_solve for callers that cannot allocate device memory: code that must
 * not call hipMalloc (stream capture, tight serving loops, harnesses that
 * forbid allocation). Same arguments, results, semantics and errors as
 * sssp_solve, and likewise returns after the stream has finished; it calls no
 * hipMalloc, hipFree or other allocating routine. The solve's workspace
 * (per-team distances, queue bitmaps and lists, key bounds, extraction
 * segments, hub tasks, samples, counters and the kernel's argument block) is
 * laid out in a static device array of SSSP_NOALLOC_SCRATCH_BYTES bytes inside
 * the library, instead of the graph's own workspace (which this call neither
 * uses nor changes). Each device the library runs on holds one such array
 * until the process ends. The array keeps the last call's contents; the call
 * clears what must start at zero. Calls on one device share the array, so
 * the library serialises them with a per-device lock: a second call waits
 * for the first to return.
 * Limit: the workspace of one launch is about 8 n (relabelled graphs) +
 * 10 n + n / 4 bytes per team, plus 12 bytes per extraction slot (at least
 * 256 per workgroup, at least n in all), 16 (m / chunk_edges + m / hub_degree)
 * bytes of hub tasks per team and 8 probe_cap bytes of samples per team
 * (about 31 MB for one team at n = 2^20, m = 2^24). A launch that needs more
 * is refused with INVALID_ARGUMENT before any device work.
 * stats->device_ms is the call's host wall-clock time (no events are created).
 */
#define SSSP_NOALLOC_SCRATCH_BYTES (64ull << 20)
sssp_status sssp_solve_noalloc(const sssp_graph* g, const int32_t* sources, int32_t n_src,
                               const sssp_params* params, uint64_t* dist, void* stream, sssp_stats* stats);

/*
 * Stream-ordered form of sssp_solve: the same computation (Alg. 1 per source,
 * all sources in one launch), for callers that overlap it with other work.
 * The call enqueues the launch on `stream` and returns without waiting. `sources` and `params` are
 * read before it returns (sources are copied); `dist` is complete once the
 * stream reaches the end of the launch, so work enqueued after it on the same
 * stream may read it. One asynchronous solve may be pending per graph; until
 * sssp_solve_wait returns, sssp_solve, sssp_solve_async, sssp_server_start
 * and sssp_graph_destroy on the graph return INVALID_ARGUMENT.
 * Errors at enqueue time as for sssp_solve; errors of the run itself come
 * from sssp_solve_wait.
 */
sssp_status sssp_solve_async(const sssp_graph* g, const int32_t* sources, int32_t n_src,
                             const sssp_params* params, uint64_t* dist, void* stream);

/* Whether the pending asynchronous solve has finished on the device: *done =
 * 1 or 0 (never blocks). INVALID_ARGUMENT when none is pending. */
sssp_status sssp_solve_query(const sssp_graph* g, int* done);

/* Wait for the pending asynchronous solve and end it: stats (host pointer or
 * NULL) as for sssp_solve, and its status: OK, STEP_LIMIT, DEVICE, or
 * CANCELLED (then the rows of sources whose solve was under way hold upper
 * bounds of the distances, and rows of sources not yet started are left
 * unwritten). INVALID_ARGUMENT when none is pending. */
sssp_status sssp_solve_wait(const sssp_graph* g, sssp_stats* stats);

/* Ask the pending asynchronous solve to stop early: the kernel reads a flag in
 * host memory once per step (in the step's last barrier) and every team
 * leaves at the end of its current step. Returns at once; sssp_solve_wait
 * then reports CANCELLED unless the solve had already finished. INVALID_ARGUMENT
 * when none is pending. */
sssp_status sssp_solve_cancel(const sssp_graph* g);

/*
 * Order-independent checksum of a distance row: the sum over v of a 64-bit
 * mix of (v, dist[v]), modulo 2^64. The mix is the SplitMix64 finaliser
 * applied to dist[v] XOR (v * 0x9E3779B97F4A7C15). dist is a device pointer
 * to n entries; the result is written to the host pointer `hash`. Used to
 * compare served rows with rows solved alone without copying them.
 */
sssp_status sssp_row_hash(const uint64_t* dist, int64_t n, void* stream, uint64_t* hash);

/*
 * Serving: a persistent launch that takes single-source requests from a ring
 * in host memory while it runs (continuous batching). Its workgroups form
 * tuning.teams teams (default: teams of 16 workgroups, at most 64 teams).
 * Each posted request is dispatched to a group of idle teams, which solves
 * it (Alg. 1) into its row and marks it done, so requests join and leave the
 * running batch one by one. The group is elastic: k idle teams, k the largest
 * power of two such that every waiting request still finds a team (at most
 * tuning.group_max), so a request that arrives at a quiet server gets most of
 * the grid, and under load each team solves its own request; with
 * tuning.group_min, a request waits until at least that many teams are idle
 * instead of running on one or two of them.
 *
 * Two ways to admit requests:
 *   - sssp_server_start: the caller owns `rows` result rows and names the row
 *     of each request (sssp_server_submit); a request is admitted when the
 *     caller has a free row to give it.
 *   - sssp_server_start_budget: admission by a device-memory budget. The
 *     launch's workspace and as many result rows as fit come out of the
 *     budget; sssp_server_enqueue always accepts a request, which waits in a
 *     host queue until a row is free; a finished request holds its row until
 *     the caller reads it (sssp_server_result) and gives it back
 *     (sssp_server_release), which admits the next waiting request.
 *
 * Both start calls launch the kernel and return at once. The launch runs
 * on a stream the library creates with a hardware queue of its own (HIP
 * otherwise shares a few queues among all streams, and a queue runs its
 * kernels in order, so a persistent launch would hold back unrelated work);
 * `stream` only orders the start after work already queued on it. HIP's
 * CU-masked streams are blocking streams: while a server runs, work queued
 * on the legacy NULL stream waits for it, so keep such work on non-blocking
 * streams (hipStreamNonBlocking).
 *   params   rule and parameters as for sssp_solve (trace, extract_counts and
 *            max_steps must be unset). rho and Delta are per team: a request
 *            solved by a group of k teams uses k * rho and k * Delta (its
 *            work per step grows with its workgroups).
 *   dist_rows device pointer to rows * n uint64 entries; a request names the
 *            row its distances go to, and holds it until it is polled done
 *            (rows bound the requests in flight). The caller owns the memory.
 *   ring_capacity  most requests posted but not yet taken by a team.
 *   flags    SSSP_SERVE_HASH: also compute each finished row's checksum
 *            (as sssp_row_hash), returned by sssp_server_poll.
 *   idle_ms  a team that has waited longer than this for a request closes
 *            the launch: no further request is dispatched, the teams leave
 *            once their current requests are done, and submit / enqueue
 *            return DEVICE from then on (0 = 60000).
 * tuning.blocks_per_cu sets the grid (default 2 per compute unit, half of the
 * kernel's occupancy of 4, so that other kernels such as copies still find
 * room while the server runs). Servers on several graphs may run side by side
 * on separate streams when their blocks_per_cu sum to at most 4; otherwise
 * the launch cannot be resident and stops with SSSP_ERR_DEVICE. Kernels
 * launched meanwhile wait for free slots: with servers holding all of them, a
 * copy on another stream waits until a server ends. While a server runs,
 * sssp_solve and another server on the same graph are refused.
 * One host thread drives a server (submit, enqueue, poll, release and stop do
 * not lock).
 */
#define SSSP_SERVE_HASH 0x1u
typedef struct sssp_server sssp_server; /* opaque */

sssp_status sssp_server_start(const sssp_graph* g, const sssp_params* params, uint64_t* dist_rows, uint32_t rows,
                              uint32_t ring_capacity, uint32_t flags, uint32_t idle_ms, void* stream,
                              sssp_server** out);

/* Start a server that admits requests by a device-memory budget of
 * budget_bytes: the launch's workspace (per team: keys, queue bitmap and
 * lists, key bounds, hub tasks, samples; per workgroup: extraction segments)
 * is counted first, and the rest holds floor(rest / (8 n)) result rows (at
 * most 65536), allocated here and owned by the server; the ring holds as many
 * entries as rows. OUT_OF_MEMORY when the budget holds no row (the detail
 * gives the workspace and row sizes). The graph's own arrays are not part of
 * the budget: its CSR, and on graphs with local expansion the per-arc target
 * rows (8 bytes per arc) that the first launch builds (and skips, reading
 * the offsets instead, when the device has no room for them); the graph
 * holds them until it is destroyed. Other arguments as sssp_server_start. */
sssp_status sssp_server_start_budget(const sssp_graph* g, const sssp_params* params, uint64_t budget_bytes,
                                     uint32_t flags, uint32_t idle_ms, void* stream, sssp_server** out);

/* Post one request (host call; validated here). *ticket numbers requests in
 * posting order from 0; the request waits in ring entry ticket % capacity
 * until a team takes it. INVALID_ARGUMENT when that entry still holds an
 * untaken request (ring full), the row holds a request not yet polled done,
 * the server is stopped or started with a budget, or source / row is out of
 * range; DEVICE when the launch takes no more requests (its idle limit
 * passed, or it ended). */
sssp_status sssp_server_submit(sssp_server* s, int32_t source, uint32_t row, uint64_t* ticket);

/* Budget servers: queue one request (host call; validated here). It is
 * admitted at once when a result row is free, else when one is released;
 * *ticket numbers requests in enqueue order from 0 (the order they are
 * admitted in). INVALID_ARGUMENT for a bad source, a stopped server or one
 * started with caller rows; DEVICE when the launch takes no more requests. */
sssp_status sssp_server_enqueue(sssp_server* s, int32_t source, uint64_t* ticket);

/* Collect up to `max` requests finished since the last poll: their tickets
 * and, with SSSP_SERVE_HASH, their row checksums (hashes may be NULL).
 * *count receives the number returned. Completion order may differ from
 * posting order. DEVICE (with *count = 0) when the launch has ended while
 * requests were still unfinished or waiting (after its idle limit or an
 * error), so that no caller waits for them forever. */
sssp_status sssp_server_poll(sssp_server* s, uint64_t* tickets, uint64_t* hashes, uint32_t max, uint32_t* count);

/* Budget servers: *row = the device address of the n distances of a request
 * that sssp_server_poll has returned and that is not yet released (valid
 * until sssp_server_release). INVALID_ARGUMENT for any other ticket. */
sssp_status sssp_server_result(sssp_server* s, uint64_t ticket, const uint64_t** row);

/* Budget servers: give the row of a finished request back to the budget (the
 * caller has finished reading it, including copies it enqueued); waiting
 * requests are admitted into the free rows. INVALID_ARGUMENT for a ticket
 * that is not finished and held. */
sssp_status sssp_server_release(sssp_server* s, uint64_t ticket);

/* Budget servers: copy the row of a finished, held request into dst (n
 * uint64 entries; device or host memory) on `stream`, wait for the copy, and
 * release the row (as sssp_server_release). `stream` must not be the legacy
 * NULL stream while the server runs (it would wait for the launch to end). */
sssp_status sssp_server_take(sssp_server* s, uint64_t ticket, uint64_t* dst, void* stream);

typedef struct {
  uint64_t rows;         /* result rows (caller's or drawn from the budget) */
  uint64_t row_bytes;    /* bytes per row (8 n) */
  uint64_t budget_bytes; /* budget servers: the budget; else 0 */
  uint64_t teams;        /* teams of the launch */
  uint64_t waiting;      /* budget servers: requests queued, not yet admitted */
  uint64_t admitted;     /* requests posted to the launch and not yet polled finished */
  uint64_t held;         /* budget servers: finished requests whose rows are not yet released */
  uint64_t free_rows;    /* rows free for the next admission */
  uint64_t workspace_bytes; /* device bytes of the launch's workspace (counted in the budget) */
} sssp_server_load;

/* Current admission state of a server (host bookkeeping; no device call). */
sssp_status sssp_server_counts(const sssp_server* s, sssp_server_load* load);

/* Close the ring: the kernel finishes every posted request, then ends; waits
 * for it and fills stats (totals over all requests; device_ms = the launch's
 * lifetime). Requests finished meanwhile can still be polled; requests still
 * waiting for admission on a budget server are dropped. Idempotent. */
sssp_status sssp_server_stop(sssp_server* s, sssp_stats* stats);

/* Stop (if needed) and release the server, with its rows on a budget server.
 * NULL is accepted. Freeing its pinned ring waits for all work on the device,
 * so stop every server that shares the device before destroying any of them. */
sssp_status sssp_server_destroy(sssp_server* s);

/* Static description of a status code. */
const char* sssp_status_string(sssp_status s);

/* Detail of the last error on this thread ("" if none). */
const char* sssp_last_error(void);

/* SSSP_ABI_VERSION of the loaded library. */
int sssp_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SSSP_H */
