/*
 * gx.h -- C ABI of the MI355X (gfx950) superstep engine.
 *
 * The engine runs the per-iteration compute of an accelerator daemon in the
 * sense of GX-Plug (arXiv 2203.13005): one superstep of the algorithm
 * template MSGGen -> MSGMerge -> MSGApply (Section "Algorithm Template")
 * over one worker's edge partition, for PageRank, Bellman-Ford SSSP and
 * label propagation read as min-label connected components (the algorithms
 * of Section "Setup"), in BSP order (Section "PowerGraph" contrasts it with
 * GAS order).  Calls map onto the paper's operation interfaces (Section
 * "Operation Interfaces"):
 *
 *   connect() + transfer()          -> gx_graph_load
 *   requestGen/Merge/Apply()         -> gx_superstep
 *   iteration control                -> gx_run_until_converged
 *     (Section "Iteration Control")
 *   update(): lazy upload + skip     -> gx_sync_delta (send), gx_apply_delta (receive)
 *     (Sections "Synchronization Caching", "Synchronization Skipping")
 *   disconnect()                     -> gx_graph_free / gx_state_free
 *
 * Conventions shared by every call:
 *  - Every call returns a gx_status; nothing is thrown across the ABI.
 *    gx_last_error() returns a message for the last failing call on the
 *    calling thread (valid until the next gx_* call on that thread).
 *  - Host arrays passed in are read during the call and stay owned by the
 *    caller.
 *  - Device memory is owned by the caller: graphs and states live in
 *    caller-provided device buffers ("arenas") whose sizes the *_bytes calls
 *    report.  The library sub-allocates inside them; on the superstep path it
 *    never allocates device memory.  Arenas must be 256-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *    are asynchronous on it unless stated otherwise.
 *  - Arguments are validated on the host before any device work, so
 *    GX_EINVAL / GX_ENOMEM are reported without touching the GPU.
 *  - A device error is sticky: the handle answers GX_EDEVICE from then on.
 *  - Handles are not thread safe; distinct handles may be used concurrently
 *    on distinct streams.
 */
#ifndef GX_H
#define GX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gx_status;
#define GX_OK            0
#define GX_EINVAL        1  /* malformed argument or graph */
#define GX_ENOMEM        2  /* arena / capacity too small, or host allocation failed */
#define GX_EDEVICE       3  /* HIP runtime error (sticky per handle) */
#define GX_ENOTCONVERGED 4  /* superstep cap reached; the state is valid */
#define GX_EBUSY         5  /* serving: no room for the request right now */
#define GX_ENOTFOUND     6  /* serving: unknown graph or request id */

typedef enum {
    GX_PAGERANK = 0,  /* float32 ranks; fixed number of supersteps */
    GX_SSSP     = 1,  /* uint32 distances, INF = 0xFFFFFFFF; to convergence */
    GX_CC       = 2,  /* uint32 labels (global ids); to convergence */
    GX_PPR      = 3,  /* float32 personalised PageRank (batched / serving only) */
    GX_LP       = 4   /* uint32 labels (global ids), label propagation: the most frequent label among
                         a vertex's distinct neighbours, the smallest on a tie; runs until nothing
                         changes or max_supersteps (the evaluation caps it at 15); needs GX_NEED_SYM */
} gx_algo;

/* Which device images gx_graph_load builds (bitmask). */
#define GX_NEED_OUT 1u  /* out-CSR (dst, weight) + in-edge records (dst, src, weight): SSSP push and pull */
#define GX_NEED_IN  2u  /* in-CSR (sources ascending) + out-degree: PageRank, PPR */
#define GX_NEED_SYM 4u  /* symmetric deduplicated adjacency: CC */

/* Per-vertex flags of a partition (one part of a vertex-cut). */
#define GX_FLAG_MASTER     1u  /* this part holds the master copy */
#define GX_FLAG_REMOTE_OUT 2u  /* the vertex has an out-edge in another part */
#define GX_FLAG_REMOTE_ANY 4u  /* the vertex has any edge in another part */

/*
 * Host description of one worker's graph: out-CSR with rows sorted by
 * destination.  row_ptr[V+1] (int32, row_ptr[0] = 0, non-decreasing,
 * row_ptr[V] = E), col[E] (int32 in [0, V)), w[E] (uint32, required when
 * GX_NEED_OUT is asked; may be NULL otherwise).  l2g[V] maps local to global
 * ids (ascending; NULL = identity) and flags[V] holds GX_FLAG_* bits (NULL =
 * unpartitioned: no vertex is remote).  Self-loops are allowed in the input
 * and ignored by CC; duplicates are allowed.  E < 2^31, V < 2^31; with
 * GX_NEED_SYM also 2E < 2^31 (the symmetric image holds up to two entries
 * per edge), else GX_EINVAL.
 */
typedef struct gx_graph_desc {
    int64_t V, E;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint32_t *w;
    const int32_t *l2g;
    const uint8_t *flags;
    uint32_t needs;
    uint32_t pr_tile_edges;  /* in-edges per PageRank workgroup tile: 0 = automatic (the largest of
                                1024, 512 that still gives 2048 tiles, else 256), or one of
                                256, 512, 1024, 2048 */
    /* One part of a vertex-cut whose PageRank is exchanged between the parts
     * (gx_params.phases == GX_PHASES_MASTERS): the whole graph's vertex count
     * and, per local vertex, its out-degree in the whole graph (host array,
     * copied).  V_global = 0 and outdeg_global = NULL otherwise. */
    int64_t V_global;
    const int32_t *outdeg_global;
} gx_graph_desc;

/* Sync-set selection (gx_params.delta_mode). */
#define GX_DELTA_REMOTE  0u  /* only vertices another part needs (lazy uploading) */
#define GX_DELTA_ALL     1u  /* every changed vertex */
#define GX_DELTA_MASTERS 2u  /* masters that another part holds a replica of */

typedef struct gx_params {
    int32_t  algo;            /* gx_algo: GX_PAGERANK, GX_SSSP or GX_CC */
    float    damping;         /* PageRank damping d, in [0, 1) */
    int32_t  source;          /* SSSP source (local id); -1 = no source in this part (another part holds it) */
    uint32_t max_supersteps;  /* cap used by gx_run_until_converged (PageRank: exactly this many) */
    uint32_t delta_mode;      /* GX_DELTA_REMOTE or GX_DELTA_ALL */
    uint32_t timing;          /* nonzero: time the edge kernels of every superstep with HIP events */
    float    pull_fraction;   /* SSSP/CC: a superstep whose active out-edges exceed this fraction of
                                 all edges pulls (one sweep over every in-edge record) instead of
                                 pushing; 0 = default (0.3), >= 1 = always push */
    uint32_t phases;          /* GX_PHASES_LOCAL or GX_PHASES_MASTERS (PageRank, SSSP, CC): the state
                                 is driven by the separate template calls gx_msg_gen / gx_msg_merge /
                                 gx_msg_apply in any order an upper system uses (BSP or GAS);
                                 gx_superstep and gx_run_until_converged refuse it.  0 = fused */
} gx_params;

#define GX_PHASES_LOCAL   1u  /* the part is the whole graph */
#define GX_PHASES_MASTERS 2u  /* PageRank on one part of a vertex-cut, exchanged with the other parts:
                                 messages use the whole graph's out-degrees, MSGApply updates the
                                 masters only (x0 and teleport use V_global); see gx_partial_emit */

/* Statistics of one superstep (counts are exact). */
typedef struct gx_step_stats {
    int64_t frontier;      /* |F_k|: active vertices (PageRank: V) */
    int64_t edges;         /* messages generated: out-edges of F_k (PageRank: E) */
    int64_t changed;       /* vertices whose value changed (|F_{k+1}| for SSSP/CC) */
    int64_t pulled;        /* 1 if the superstep ran as a pull over all in-edge records */
    double  kernel_ms;     /* with gx_params.timing: HIP-event time of its edge kernels, else 0 */
} gx_step_stats;

typedef struct gx_run_stats {
    int64_t supersteps;    /* supersteps executed by this call */
    int64_t edges;         /* sum of gx_step_stats.edges over them */
    int64_t converged;     /* 1 if the last superstep changed nothing (SSSP/CC) */
    double  edge_kernel_ms;   /* with timing: summed HIP-event time of the edge kernel */
    int64_t edge_kernel_launches;
    double  wall_ms;       /* host wall time of the call */
} gx_run_stats;

typedef struct gx_graph gx_graph;
typedef struct gx_state gx_state;

const char *gx_last_error(void);
const char *gx_version(void);

/* Device arena bytes gx_graph_load needs for this description. */
gx_status gx_graph_bytes(const gx_graph_desc *desc, size_t *arena_bytes);

/*
 * connect() + transfer() (Section "Operation Interfaces"): validates the
 * host CSR, builds the requested device images inside `dev_arena` and
 * streams them host-to-device in fixed-size blocks through three rotating
 * pinned staging buffers on a copy stream (the n/c/u block rotation of
 * Section "Pipeline Shuffling").  Host packaging of block i+1 overlaps the
 * copy of block i.  `stream` waits for the copies, so work enqueued on it
 * afterwards sees the graph.  Synchronous with respect to the host arrays.
 * Errors: GX_EINVAL (bad CSR, ids out of range), GX_ENOMEM (arena too
 * small), GX_EDEVICE.
 */
gx_status gx_graph_load(const gx_graph_desc *desc, void *dev_arena, size_t arena_bytes,
                        void *stream, gx_graph **out);
gx_status gx_graph_free(gx_graph *g);
gx_status gx_graph_info(const gx_graph *g, int64_t *V, int64_t *E, uint32_t *needs);

/* Device bytes the state of `params` needs on `g`. */
gx_status gx_state_bytes(const gx_graph *g, const gx_params *params, size_t *bytes);

/*
 * Initialises a state inside `dev_state`: PageRank x0 = 1/V; SSSP dist =
 * INF, dist[source] = 0, F1 = {source}; CC label = global id, F1 = vertices
 * with an edge.  The initial values count as already synchronised.
 */
gx_status gx_state_init(gx_graph *g, const gx_params *params, void *dev_state, size_t bytes,
                        void *stream, gx_state **out);
gx_status gx_state_free(gx_state *s);

/* Device pointer to the current vertex values (float32 or uint32, V entries). */
gx_status gx_state_values(gx_state *s, void **dev_values);
/* Device pointer to the current frontier as a byte map (uint8 per vertex,
 * nonzero = vertex v is active in the next superstep); SSSP/CC only. */
gx_status gx_state_frontier(gx_state *s, void **dev_bytemap);
/* Supersteps executed since init. */
gx_status gx_state_superstep(gx_state *s, int64_t *k);

/*
 * Frees the process-wide caches the engine keeps between calls: timing
 * events and the pinned host buffers superstep counters are read through.
 * Resources held by live states are not touched (they return to the caches
 * when the states are freed).  Call it before process exit, after freeing
 * every state, so no HIP object outlives the caller's use of the runtime.
 * Safe to call at any time; later calls recreate what they need.
 */
gx_status gx_release_cached(void);

/*
 * requestGen() -> requestMerge() -> requestApply() in BSP order: one
 * superstep.  SSSP/CC: relax the active list (built with start-of-superstep
 * snapshots by the previous call or by gx_state_init) over equal tiles of
 * active out-edges (push) or as one sweep over all in-edge records (pull,
 * for large frontiers; the device picks), merge by integer min, mark
 * changed vertices in the next frontier and the dirty map, then compact the
 * next frontier.  PageRank: pull over the
 * in-CSR in equal edge tiles with a fixed summation order.
 * With stats == NULL the call is asynchronous; otherwise it synchronises
 * `stream` and fills *stats.
 */
gx_status gx_superstep(gx_state *s, void *stream, gx_step_stats *stats);

/*
 * Iteration control: SSSP/CC run supersteps until one changes nothing or
 * max_supersteps have run (GX_ENOTCONVERGED, state valid); PageRank runs
 * exactly max_supersteps.  Synchronises `stream`.  per_step (optional, room
 * for max_supersteps entries) receives every superstep's statistics.
 */
gx_status gx_run_until_converged(gx_state *s, uint32_t max_supersteps, void *stream,
                                 gx_run_stats *out, gx_step_stats *per_step);

/*
 * The algorithm template's three calls as separate requests (Section
 * "Algorithm Template": MSGGen, MSGMerge, MSGApply; Section "Operation
 * Interfaces": requestX() for each; Section "PowerGraph": BSP calls them in
 * the order Gen -> Merge -> Apply, GAS in the order Merge -> Apply -> Gen).
 * For a state initialised with gx_params.phases != 0:
 *   gx_msg_gen    MSGGen: the vertices changed since their messages were
 *                 last generated (at first: the SSSP source, every CC vertex
 *                 with an edge, every PageRank vertex) emit their messages:
 *                 SSSP/CC the active list with the values they send (each
 *                 out-edge then carries sat_add(value, w) or the value),
 *                 PageRank x[u]/outdeg(u) per vertex and the dangling mass.
 *                 GX_EINVAL if messages are already pending.
 *   gx_msg_merge  MSGMerge: the pending messages combined per destination
 *                 (integer min; PageRank the fp64 sum over in-edges in
 *                 source order) into an accumulator; no-op when nothing is
 *                 pending.
 *   gx_msg_apply  MSGApply: the merged messages applied to the vertices
 *                 (SSSP/CC new = min(old, merged), a vertex that falls is
 *                 marked for the next Gen and the sync set; PageRank
 *                 x' = (1-d)/V + d*(merged + D/V)); no-op when nothing was
 *                 merged.  Each apply that ran counts as one superstep.
 * One BSP superstep (Gen, Merge, Apply) equals gx_superstep's result.  In
 * GAS order the first Merge and Apply find nothing and do nothing, so after
 * n GAS iterations the values are those of n - 1 supersteps (the last Gen's
 * messages pending).  Asynchronous, except gx_msg_apply with stats != NULL,
 * which synchronises `stream` and reports the superstep's active vertices,
 * messages and changed vertices (all zero when the apply did nothing).
 */
gx_status gx_msg_gen(gx_state *s, void *stream);
gx_status gx_msg_merge(gx_state *s, void *stream);
gx_status gx_msg_apply(gx_state *s, void *stream, gx_step_stats *stats);

/*
 * PageRank across the parts of a vertex-cut, one state per part created with
 * GX_PHASES_MASTERS (Section "Synchronization Caching": mirrors and masters
 * exchange only what changed; the combined value is the master's).  One
 * superstep, over all parts p (the caller moves the buffers between them):
 *   gx_msg_gen(p); gx_msg_merge(p)       every part sums its own in-edges'
 *                                        messages, x[u] / outdeg_global(u);
 *   gx_dangling_get(p) summed over the parts in part order, then
 *   gx_dangling_set(p, total)            the whole graph's dangling mass;
 *   gx_partial_emit(p)                   (gid, sum) of every replica whose
 *                                        master is elsewhere and that has an
 *                                        in-edge here, ascending gid;
 *   gx_partial_add(q, pairs of p)        for every other part p, in part
 *                                        order: masters add the sums (the
 *                                        master's own sum comes first, so the
 *                                        order of the additions is fixed);
 *   gx_msg_apply(p)                      masters: x' = (1-d)/V_global +
 *                                        d*(sum + D/V_global);
 *   gx_sync_delta(p) (GX_DELTA_MASTERS)  then gx_apply_delta(q, pairs) on
 *                                        every other part: replicas take
 *                                        their masters' new ranks.
 * gx_dangling_get synchronises `stream`; gx_dangling_set and gx_partial_add
 * are asynchronous; gx_partial_emit synchronises and returns GX_ENOMEM when
 * count > cap (nothing beyond cap written).  gx_partial_emit and
 * gx_partial_add need merged, not yet applied, messages (GX_EINVAL).
 */
gx_status gx_dangling_get(gx_state *s, double *mass, void *stream);
gx_status gx_dangling_set(gx_state *s, double mass, void *stream);
gx_status gx_partial_emit(gx_state *s, int32_t *dev_gid, double *dev_val, uint32_t cap, uint32_t *count,
                          void *stream);
gx_status gx_partial_add(gx_state *s, const int32_t *dev_gid, const double *dev_val, uint32_t n, void *stream);

/*
 * update() with lazy uploading and synchronisation skipping: emits the
 * (global id, value bits) pairs of vertices that (GX_DELTA_REMOTE) another
 * part needs -- remote_out for PageRank/SSSP, remote_any for CC -- and whose
 * value differs from the last emitted one, in ascending global id; only
 * the final value is sent.  dev_gid/dev_val are device buffers of `cap`
 * entries.  *count receives the number of pairs, *skippable = (count == 0).
 * GX_ENOMEM if count > cap (nothing beyond cap is written; the sync
 * record is left unchanged).  Synchronises `stream`.
 */
gx_status gx_sync_delta(gx_state *s, int32_t *dev_gid, uint32_t *dev_val, uint32_t cap,
                        uint32_t *count, int32_t *skippable, void *stream);

/*
 * For callers that cannot allocate device memory or synchronise -- code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc: gx_sync_delta with the same pairs, order and commit rule, made
 * asynchronous.  The per-workgroup counts go to a fixed static device array
 * of 256 KiB (one per GPU, held until the process ends) instead of the
 * state's workspace, and the pair count is written to the device word
 * *dev_count instead of being returned, so the call allocates nothing,
 * copies nothing to the host and does not synchronise `stream`.  The pairs
 * are committed (dirty map cleared, synced copy updated) only when the count
 * is at most `cap`; a caller seeing *dev_count > cap has a full count and an
 * unchanged sync record, as with GX_ENOMEM of gx_sync_delta.  Limit: graphs
 * of at most 2^29 vertices (GX_EINVAL beyond).  Calls that overlap in time
 * on one GPU share the array and race: issue them on one stream, or order
 * them.  Errors: GX_EINVAL, GX_EDEVICE (also if the array's address cannot
 * be looked up).
 */
gx_status gx_sync_delta_noalloc(gx_state *s, int32_t *dev_gid, uint32_t *dev_val, uint32_t cap,
                                uint32_t *dev_count, void *stream);

/*
 * The receiving side of update(): merges the (global id, value) pairs that
 * other parts emitted with gx_sync_delta into this part's replicas, for
 * SSSP and CC (integer min; Section "Operation Interfaces", Section
 * "Synchronization Caching": mirrors and masters exchange only changed
 * values).  dev_gid / dev_val are device arrays of n pairs in any order;
 * ids this part does not hold are ignored.  A replica whose value falls
 * becomes active in the next superstep (it is not marked dirty: the parts
 * that emitted the value already sent it to every other part).  Call it
 * between gx_superstep calls: it rebuilds the active list of the next
 * superstep.  *active_next (optional) receives the next superstep's active
 * vertex count and then the call synchronises `stream`; otherwise it is
 * asynchronous.  For a PageRank state under GX_PHASES_MASTERS the values are
 * rank bits and every replica held here that is not the master takes them.
 * GX_EINVAL for other PageRank states or NULL buffers with n > 0.
 */
gx_status gx_apply_delta(gx_state *s, const int32_t *dev_gid, const uint32_t *dev_val, uint32_t n,
                         int64_t *active_next, void *stream);

/* ---------------------------------------------------------------------
 * Streamed supersteps (Section "Intra-Iteration Optimization: Pipeline
 * Shuffling", Algorithms "Pipeline Shuffle - Daemon Side" and "Agent Side",
 * Lemma "bSizeSelection").  The edge triplets stay in pinned host memory
 * (copied at creation; SSSP: the out-edges (u, v, w) in CSR order; CC: both
 * directions of every distinct undirected edge, self-loops dropped) and every
 * superstep streams them through the device in blocks of `block_edges`
 * triplets, packed (u, v, w) (CC: (u, v)) so one copy downloads a block.
 * Vertex state stays resident.  Block i runs in device buffer i mod R (R =
 * `ring`, 3 to GX_STREAM_RING_MAX): downloaded on a copy stream (n-block),
 * computed (c-block: each
 * triplet whose source is active carries sat_add(value, w) or the value, is
 * merged into the destination by integer min, and its message is written
 * into the triplet's result slot, INF when the source is inactive), and its
 * results uploaded to pinned host memory on a third stream (u-block); the
 * three stages of consecutive blocks overlap and the buffers rotate roles.
 * GX_STREAM_SERIAL runs the same stages one after the other on one stream
 * and times each (download_ms, compute_ms, upload_ms: sums over the blocks).
 * Superstep semantics are those of gx_superstep (Jacobi: messages read the
 * values of the superstep's start; the next frontier is the set of vertices
 * whose value fell).
 * --------------------------------------------------------------------- */

typedef struct gx_stream gx_stream;
#define GX_STREAM_PIPELINED 0u
#define GX_STREAM_SERIAL    1u
#define GX_STREAM_RING_MAX  8   /* device block buffers at most (3 = the n, c, u rotation itself) */

typedef struct gx_stream_stats {
    int64_t blocks;       /* s */
    int64_t triplets;     /* d: triplets streamed */
    int64_t messages;     /* triplets whose source was active */
    int64_t changed;      /* vertices in the next frontier (0: converged) */
    double  wall_ms;      /* host wall time of the superstep */
    double  download_ms, compute_ms, upload_ms;  /* GX_STREAM_SERIAL only */
} gx_stream_stats;

/* Per-entity costs of the three stages and the per-call constant of the
 * computation (Eq. "PipelineTimeSimplied2": k1, k2, k3 and a). */
typedef struct gx_pipeline_coef {
    double k1, k2, k3, a;
} gx_pipeline_coef;

/* Device arena bytes of a stream handle for this graph and largest block. */
gx_status gx_stream_bytes(const gx_graph_desc *desc, int32_t algo, uint64_t block_edges_max, int32_t ring,
                          size_t *bytes);
/* Copies the triplets into pinned host memory the handle owns, carves the
 * vertex state and `ring` block buffers of block_edges_max triplets from
 * `dev_arena`, and initialises the state (SSSP from `source`, -1 = none;
 * CC labels = global ids).  Synchronous.  GX_EINVAL, GX_ENOMEM, GX_EDEVICE. */
gx_status gx_stream_create(const gx_graph_desc *desc, int32_t algo, int32_t source, void *dev_arena,
                           size_t arena_bytes, uint64_t block_edges_max, int32_t ring, gx_stream **out);
/* Re-initialises the vertex state (superstep 0).  Synchronous. */
gx_status gx_stream_reset(gx_stream *s);
/* One streamed superstep; synchronous (returns after the last upload). */
gx_status gx_stream_superstep(gx_stream *s, uint64_t block_edges, uint32_t mode, gx_stream_stats *stats);
/* Device pointers to the values (uint32 per vertex) and to the byte map of
 * the next superstep's active vertices. */
gx_status gx_stream_values(gx_stream *s, void **dev_values, void **dev_frontier);
/* The results the last superstep uploaded: one message per triplet, in
 * triplet order, in pinned host memory the handle owns (valid until the
 * next superstep or gx_stream_free). */
gx_status gx_stream_results(gx_stream *s, const uint32_t **host_results, int64_t *n);
gx_status gx_stream_free(gx_stream *s);

/* Eq. "PipelineTimeSimplied2": the time of d entities in s equal blocks
 * (2 <= s <= d).  GX_EINVAL otherwise. */
gx_status gx_pipeline_time(const gx_pipeline_coef *k, double d, double s, double *T);
/* Lemma "bSizeSelection": the optimal block size b for d entities (a/(k1-k2)
 * or a/(k3-k2) when downloads or uploads cost most per entity and that block
 * is below Q = sqrt(a d / (k1 + k3)), else Q), then of the floor and the
 * ceiling of d / b (clamped to [2, d]) the block count with the smaller
 * modelled time.  *blocks, *block_size = d / *blocks, *T = the model's time.
 * GX_EINVAL for d < 2 or negative coefficients. */
gx_status gx_pipeline_plan(const gx_pipeline_coef *k, int64_t d, int64_t *blocks, double *block_size, double *T);

/* ---------------------------------------------------------------------
 * The CPU daemon and workload balancing (Section "Beyond-Iteration
 * Optimization: Workload Balancing", Eq. "CostModelOneIteration", Lemma
 * "minmaxcidi").  A part of a vertex-cut can run on host threads with the
 * device engine's superstep semantics (Jacobi min superstep, SSSP on the
 * out-CSR, CC on the symmetric adjacency) and exchange sync sets with parts
 * on the GPU; host arrays throughout.  `threads` = 0: all hardware threads.
 * --------------------------------------------------------------------- */

typedef struct gx_cpu gx_cpu;
/* Copies the description's CSR (E < 2^30).  GX_EINVAL, GX_ENOMEM. */
gx_status gx_cpu_create(const gx_graph_desc *desc, int32_t algo, int32_t source, int32_t threads, gx_cpu **out);
/* One superstep; fills *stats (frontier, messages, changed). */
gx_status gx_cpu_superstep(gx_cpu *c, gx_step_stats *stats);
/* Every vertex changed since the last call that another part needs (flags
 * given: remote_out for SSSP, remote_any for CC; no flags: every changed
 * vertex), (global id, value) in ascending id; GX_ENOMEM with *count set
 * when count > cap (nothing written, nothing committed). */
gx_status gx_cpu_sync_delta(gx_cpu *c, int32_t *gid, uint32_t *val, uint32_t cap, uint32_t *count);
/* Other parts' pairs merged by integer min; lowered replicas become active. */
gx_status gx_cpu_apply_delta(gx_cpu *c, const int32_t *gid, const uint32_t *val, uint32_t n, int64_t *active_next);
/* The current values (V entries, valid until the next call on the handle). */
gx_status gx_cpu_values(gx_cpu *c, const uint32_t **values);
gx_status gx_cpu_free(gx_cpu *c);
/* Lemma "minmaxcidi": the split d_j = D (1/c_j) / sum_i (1/c_i) of D entities
 * over m workers of cost c_j per entity, which minimises max_j c_j d_j.
 * GX_EINVAL for non-positive costs. */
gx_status gx_balance_split(const double *c, int32_t m, double D, double *d_out);

/* ---------------------------------------------------------------------
 * Batched lanes: B independent single-source SSSP (or personalised
 * PageRank) solves over one resident graph, run as one persistent kernel
 * over a [V x B] state tile (B contiguous per vertex).  Generalises the
 * evaluation's several SSSP sources computed simultaneously (Section
 * "Setup", first footnote).
 * --------------------------------------------------------------------- */

typedef struct gx_tune {
    uint32_t block;   /* threads per workgroup (64..1024, multiple of 64); 0 = default */
    uint32_t tile;    /* edges per work tile; 0 = default */
    uint32_t width;   /* lanes per pass (32, 64, 128 or 256, <= B); 0 = default */
    uint32_t grid;    /* workgroups of the persistent grid; 0 = occupancy bound */
} gx_tune;

/* Device workspace bytes gx_batch_run needs (excluding the output tile). */
gx_status gx_batch_bytes(const gx_graph *g, int32_t algo, uint32_t B, size_t *bytes);

/*
 * Runs B lanes to completion: SSSP lanes until no lane changes (each lane
 * equals the plain solve from its source), PPR lanes for `iters`
 * supersteps with seed sources[b].  dev_out: [V x B] uint32 (SSSP) or
 * float32 (PPR), row-major (lane b of vertex v at v*B + b).  sources: B host
 * ids.  B: 1..1024 (SSSP: multiple of 32).  tune may be NULL.  Synchronises
 * `stream`.
 */
gx_status gx_batch_run(gx_graph *g, int32_t algo, const int32_t *sources, uint32_t B,
                       float damping, uint32_t iters, void *dev_work, size_t work_bytes,
                       void *dev_out, const gx_tune *tune, void *stream, gx_run_stats *out);

/*
 * Times the candidate launch shapes of gx_batch_run on this graph (each
 * candidate runs once on `sources`) and writes the fastest to *best;
 * dev_out then holds that shape's result.  Every candidate must produce
 * the same result; the call fails with GX_EDEVICE if one does not.  When
 * the environment variable GX_TUNE_CACHE names a file, results are kept
 * there, one line per (graph signature: size, out-degrees and the device's
 * CU count; algorithm; B; iterations for PPR), and a later call with the
 * same key, in any process, returns the stored shape and time after one
 * run of it, without timing the candidates.
 */
gx_status gx_batch_autotune(gx_graph *g, int32_t algo, const int32_t *sources, uint32_t B,
                            float damping, uint32_t iters, void *dev_work, size_t work_bytes,
                            void *dev_out, void *stream, gx_tune *best, double *best_ms);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of SSSP / PPR queries over resident graphs.
 * A scheduler thread keeps per-graph lane pools; queries that arrive while
 * others run are admitted into free lanes at superstep boundaries when the
 * HBM budget allows, advance together with the running ones, and retire
 * when converged (SSSP) or after their iterations (PPR).
 * --------------------------------------------------------------------- */

typedef struct gx_server gx_server;

typedef struct gx_server_config {
    void    *dev_arena;       /* device memory for lane pools */
    size_t   arena_bytes;     /* budget: lane pools are admitted only while they fit */
    uint32_t lanes_per_pool;  /* most lanes in one pool (multiple of 32, <= 256); 0 = 64.  A new
                               * pool takes the queries of its pair waiting at that moment,
                               * rounded up to a multiple of 32 lanes, at most this many */
    uint32_t max_pools;       /* concurrently running pools (one stream each); 0 = 4 */
    uint32_t epoch_supersteps;/* PPR supersteps per pool launch before admitting/retiring; 0 = 4 */
    float    damping;         /* PPR damping; 0 = 0.85 */
    uint32_t ppr_iters;       /* PPR supersteps per query; 0 = 50 */
    uint32_t sssp_epoch_supersteps; /* SSSP supersteps per pool launch; 0 = 16.  Converged lanes
                               * cost next to nothing, and epochs that run a query to its end
                               * save the round trips behind other pools' work */
} gx_server_config;

typedef struct gx_query_result {
    int64_t  id;
    int32_t  graph;
    int32_t  algo;
    int32_t  source;
    int32_t  status;          /* GX_OK or an error */
    double   submit_s, start_s, done_s;  /* host monotonic clock, seconds */
    int64_t  supersteps;
} gx_query_result;

gx_status gx_server_bytes_per_lane(const gx_graph *g, int32_t algo, size_t *bytes);
gx_status gx_server_create(const gx_server_config *cfg, gx_server **out);
/* Registers a loaded graph (needs GX_NEED_OUT | GX_NEED_IN); returns its id. */
gx_status gx_server_add_graph(gx_server *s, gx_graph *g, int32_t *graph_id);
/*
 * Queues a query.  `result` is a host buffer of V uint32 (SSSP) or float32
 * (PPR) that receives the answer when the query completes; it must stay
 * valid until gx_server_poll reports the query.  *id receives the query id.
 */
gx_status gx_server_submit(gx_server *s, int32_t graph_id, int32_t algo, int32_t source,
                           void *result, int64_t *id);
/* Moves up to `cap` completed queries into `out`; *n receives the count.
 * With wait_ms > 0 blocks until at least one completes or the time passes. */
gx_status gx_server_poll(gx_server *s, gx_query_result *out, uint32_t cap, uint32_t *n,
                         int32_t wait_ms);
/* Queries queued, running, or finished with their result still being copied out. */
gx_status gx_server_pending(gx_server *s, int64_t *n);
gx_status gx_server_destroy(gx_server *s);

#ifdef __cplusplus
}
#endif

#endif /* GX_H */
