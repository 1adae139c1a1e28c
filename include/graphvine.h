/*
 * graphvine.h -- C ABI of the MI355X (gfx950) GraphVine dynamic-graph library.
 *
 * The library keeps a directed graph resident in GPU memory and updates it in
 * batches.  It follows the problem statement of GraphVine (Krishnan S, Tavva,
 * Nasre, arXiv 2306.08252): an initial graph, then batched vertex and edge
 * inserts and deletes (Sec. 4.3), edge queries (Sec. 4.6, Alg. 3) and the
 * memory footprint (Sec. 5.4).
 *
 * Structure.  Each vertex's adjacency lives in fixed-size edge blocks of B
 * uint32 destination slots (Sec. 4.1).  Blocks come from one pre-allocated
 * device pool (the "edge queue" of Sec. 4.2) managed as a free-list stack plus
 * a bump pointer.  A per-vertex block directory replaces the paper's complete
 * binary tree of blocks and gives block j of a vertex in O(1).  The vertex
 * dictionary capacity is a power of two (Sec. 4.1, Sec. 4.4).
 *
 * Semantics.  Adjacencies are sets: inserting an existing edge and deleting an
 * absent edge are no-ops, and duplicates inside a batch collapse.  Deletes
 * compact the adjacency and return emptied blocks to the pool, so a vertex of
 * degree d always holds exactly ceil(d / B) blocks.  Edges are never created
 * for inactive vertices: a pair whose source or destination is inactive or
 * outside the dictionary is rejected and counted, not an error.
 *
 * Memory and streams.  Every array argument named d_* is a DEVICE pointer on
 * the graph's current device, owned by the caller and read (or written) in
 * stream order on the graph's stream; the caller keeps it alive until that
 * stream has passed the call.  The library never frees caller memory.  The
 * graph owns all of its internal memory; gv_graph_destroy releases it.
 * A gv_graph must be used by one host thread at a time.
 *
 * Errors.  Every int-returning function returns a GV_* code; no C++ exception
 * crosses this boundary.  Batch calls with a NULL stats pointer are
 * asynchronous: their errors are kept and reported by the next gv_sync or
 * synchronising call.  With a non-NULL stats pointer the call waits for its
 * own completion and reports its own result.
 *
 * Device-side checks.  Every edge batch verifies its own grouping sort on the
 * device: the sorted keys must be in order and must have the same mix64 sum
 * as the packed keys, and no look-back wait between workgroups may have run
 * out.  If a check fails, that batch and every later one change nothing; the
 * next synchronising call (a batch call with stats, gv_sync) returns
 * GV_EDEVICE and the graph is unusable.
 *
 * Ids are uint32.  The largest dictionary capacity is 2^31 vertices, so the
 * largest vertex id is 2^31 - 1; 0xFFFFFFFF is never a valid id.  A batch
 * holds fewer than 2^30 - 1 pairs; a graph holds fewer than 2^30 edges when
 * it is built or dumped (GV_EINVAL otherwise).
 */
#ifndef GRAPHVINE_H
#define GRAPHVINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GV_OK = 0,
    GV_EINVAL = 1,  /* NULL pointer where data is required, or bad config     */
    GV_ERANGE = 2,  /* id outside the dictionary, or an output buffer too small */
    GV_ENOMEM = 3,  /* pool, directory or device memory exhausted; the batch is
                       not applied and the graph is unchanged                  */
    GV_EDEVICE = 4  /* a HIP runtime failure, or a batch whose device-side
                       checks failed (see below); the graph must be destroyed  */
};

#define GV_MAX_CAPACITY (1ull << 31)
#define GV_MAX_ATTR_WORDS 8

typedef struct gv_graph gv_graph;

typedef struct {
    /* Slots per edge block, a power of two in [1, 1024]; 0 selects the rule of
     * Sec. 4.3: the average degree of the non-zero-degree vertices of the
     * initial graph, rounded up to a power of two within [8, 64]. */
    uint32_t block_slots;
    uint32_t flags;            /* reserved, must be 0                            */
    /* Edge-block pool size in bytes (holds floor(pool_bytes / (4 B)) blocks);
     * 0 = twice the initial graph's blocks plus 2^20 blocks. */
    uint64_t pool_bytes;
    /* Minimum dictionary capacity; the capacity is the next power of two of
     * max(num_vertices, vertex_capacity, 1). */
    uint64_t vertex_capacity;
    /* Directory arena size in uint32 entries; 0 = default (4 entries per pool
     * block plus 2^20). */
    uint64_t directory_entries;
    /* Attribute words (uint32) per edge entry, 0..GV_MAX_ATTR_WORDS (Sec. 4.1:
     * an edge entry may carry attributes).  A new entry's attributes are
     * zero; gv_set_edge_attrs / gv_get_edge_attrs write and read them. */
    uint32_t edge_attr_words;
    uint32_t reserved;         /* must be 0 */
} gv_config;

typedef struct {
    uint64_t applied;          /* edges (vertices) actually inserted / removed   */
    uint64_t rejected;         /* pairs (ids) with an inactive or invalid end    */
    uint64_t batch_duplicates; /* valid entries minus distinct valid entries     */
} gv_batch_stats;

typedef struct {
    uint64_t block_bytes;          /* 4 * B                                     */
    uint64_t pool_capacity_blocks; /* blocks the pool can hold                  */
    uint64_t blocks_in_use;        /* = sum over vertices of ceil(deg / B)      */
    uint64_t free_list_blocks;     /* blocks on the free-list stack             */
    uint64_t bump_blocks;          /* blocks ever carved by the bump pointer    */
    uint64_t vertex_capacity;      /* dictionary capacity (power of two)        */
    uint64_t vertex_table_bytes;   /* dictionary + activity bitmap bytes        */
    uint64_t directory_entries_in_use; /* directory entries held by vertices    */
    uint64_t directory_bytes;      /* directory arena bytes reserved            */
    uint64_t live_bytes;           /* blocks_in_use * block_bytes + vertex table
                                      + 4 * directory_entries_in_use            */
    uint64_t num_edges;            /* edges stored                              */
    uint64_t reserved_bytes;       /* all device memory held by the graph       */
} gv_mem;

typedef struct {
    uint64_t vertex_capacity; /* dictionary capacity (power of two)            */
    uint32_t block_slots;     /* B                                             */
    uint32_t device;          /* HIP device ordinal                            */
} gv_info;

/* Cumulative work counters (since init) used by the benchmark's bytes model.
 * Index 0 = insert, 1 = delete, 2 = query batches. */
typedef struct {
    uint64_t batches[3];       /* edge batches handed in                        */
    uint64_t pairs[3];         /* pairs handed in                               */
    uint64_t touched[3];       /* distinct valid sources, summed over batches   */
    uint64_t scanned_slots[3]; /* block-granular slots of touched adjacencies   */
    uint64_t new_blocks;       /* blocks taken from the pool                    */
    uint64_t freed_blocks;     /* blocks returned to the pool                   */
    uint64_t written_slots;    /* slots written by appends                      */
    uint64_t moved_slots;      /* slots moved by delete compaction              */
} gv_counters;

/* Build a graph from a COO edge list (Sec. 4.3 "initialization", Sec. 5.2
 * "bulk build"): vertices 0..num_vertices-1 become active and the distinct
 * pairs (d_src[i], d_dst[i]), i < num_edges, become edges.  d_src/d_dst may be
 * NULL when num_edges is 0.  cfg may be NULL (all defaults).  hip_stream is a
 * hipStream_t (NULL = the null stream) used for this and later calls.
 * Synchronous.  Returns GV_ERANGE (and no graph) if any id >= num_vertices,
 * GV_EINVAL for a bad config or num_vertices > 2^31, GV_ENOMEM if the pool or
 * device memory is too small. */
int gv_graph_init(gv_graph** out, uint64_t num_vertices, const uint32_t* d_src,
                  const uint32_t* d_dst, uint64_t num_edges, const gv_config* cfg,
                  void* hip_stream);

/* Batched edge insertion (Sec. 4.5.1, Alg. 1) with set semantics: pairs
 * already present and repeated pairs are skipped.  All-or-nothing: if the pool
 * or directory cannot hold the result, nothing is applied (GV_ENOMEM). */
int gv_insert_edges(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                    uint64_t n, gv_batch_stats* stats_or_null);

/* Batched edge deletion (Sec. 4.5.2, Alg. 2): matching edges are removed, the
 * adjacency is compacted and emptied blocks return to the pool. */
int gv_delete_edges(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                    uint64_t n, gv_batch_stats* stats_or_null);

/* Vertex insertion (Sec. 4.4): inactive ids become active with no edges; the
 * dictionary grows to the next power of two above the largest id when needed.
 * Ids > 2^31 - 1 are rejected.  Synchronous. */
int gv_insert_vertices(gv_graph* g, const uint32_t* d_ids, uint64_t n,
                       gv_batch_stats* stats_or_null);

/* Vertex deletion (Sec. 4.4): each active id loses its out- and in-edges and
 * becomes inactive; its blocks return to the pool.  Ids >= capacity are
 * rejected; inactive ids are no-ops.  Synchronous. */
int gv_delete_vertices(gv_graph* g, const uint32_t* d_ids, uint64_t n,
                       gv_batch_stats* stats_or_null);

/* Block size over the graph's life (Sec. 6, future scope: the block size
 * may follow the graph as its average degree changes, against internal
 * fragmentation).  gv_set_block_slots re-lays the same edges (and their
 * attribute words) in blocks of block_slots slots (a power of two in
 * [1, 1024]) within the pool's byte budget; gv_adapt_block_slots first takes
 * the rule of Sec. 4.3 on the graph as it is now (average degree of the
 * vertices of non-zero degree, a power of two within [8, 64]) and reports
 * the size it chose.  Synchronous; vertex capacity and activity are kept;
 * plans recorded before become invalid (gv_plan_launch: GV_EINVAL).
 * GV_ENOMEM, graph unchanged, when the edges do not fit the pool with the
 * new size; a device allocation failure during the rebuild leaves the graph
 * unusable.  Graphs of 2^30 or more edges: GV_EINVAL. */
int gv_set_block_slots(gv_graph* g, uint32_t block_slots);
int gv_adapt_block_slots(gv_graph* g, uint32_t* block_slots);

/* Edge attributes (Sec. 4.1: an edge entry may carry attributes), for
 * graphs created with gv_config.edge_attr_words = A > 0 (else GV_EINVAL).
 * An entry's A uint32 words live at its slot and move with it; a newly
 * inserted edge starts with zeros, a deleted one loses them.
 * gv_set_edge_attrs: d_attr holds n rows of A words; every pair (d_src[i],
 * d_dst[i]) that is stored gets row i, the last row of a pair that occurs
 * several times winning; pairs not stored, or with an invalid endpoint,
 * change nothing.  Statistics: applied = distinct stored pairs written,
 * rejected = pairs with an invalid endpoint, batch_duplicates = valid pairs
 * minus distinct valid pairs.  Asynchronous without a stats pointer.
 * gv_get_edge_attrs: d_found[i] = 1 and row i of d_attr = the pair's words
 * if stored, else 0 and zeros.  Asynchronous.  Both take the path of a query
 * batch (Sec. 4.6) whose probe also records the slot it finds. */
int gv_set_edge_attrs(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                      const uint32_t* d_attr, uint64_t n, gv_batch_stats* stats_or_null);
int gv_get_edge_attrs(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                      uint8_t* d_found, uint32_t* d_attr);

/* Mixed edge updates, the tick of the served form: entry i inserts
 * (d_op[i] == 0) or deletes (d_op[i] == 1) the pair (d_src[i], d_dst[i]).
 * The graph ends as if the entries were applied one at a time in index
 * order with set semantics (the batch model of Sec. 4.3 with an order inside
 * the batch, ours): each pair's last entry decides whether it is stored;
 * entries with an inactive or out-of-range endpoint, or another op value,
 * change nothing.  All three arrays are device arrays of n entries, read
 * only.  Asynchronous, no statistics; an allocation failure is sticky
 * (reported by gv_sync) and leaves a consistent graph in which the delete
 * part may have been applied.  GV_EINVAL for null arrays with n > 0 or
 * n >= 2^30 - 1 (the limit of every edge batch). */
int gv_apply_edge_ops(gv_graph* g, const uint8_t* d_op, const uint32_t* d_src,
                      const uint32_t* d_dst, uint64_t n);

/* gv_apply_edge_ops with per-request statistics: the entries are cut into
 * n_req requests, request r being entries [d_req_end[r-1], d_req_end[r])
 * (d_req_end: device array, ascending, last == n; bad ends give meaningless
 * counts but no bad access).  d_stats (device, n_req entries) receives each
 * request's statistics as if the requests were applied alone, one after the
 * other: rejected = entries with an invalid endpoint or op; batch_duplicates
 * = entries whose previous entry of the same pair is in the same request
 * with the same op; applied = the other entries that change the graph (an
 * insert of a pair absent just before it, a delete of a pair present).  The
 * graph ends as with gv_apply_edge_ops.  Asynchronous; d_stats is valid once
 * gv_sync returns GV_OK.  GV_EINVAL for n_req == 0 with n > 0, or null
 * arrays. */
int gv_apply_edge_ops_stats(gv_graph* g, const uint8_t* d_op, const uint32_t* d_src,
                            const uint32_t* d_dst, uint64_t n, const uint64_t* d_req_end,
                            uint64_t n_req, gv_batch_stats* d_stats);

/* Edge query (Sec. 4.6, Alg. 3), batched: d_out[i] = 1 if edge
 * (d_src[i], d_dst[i]) exists, else 0, in input order.  Asynchronous. */
int gv_edge_exists(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                   uint64_t n, uint8_t* d_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): gv_edge_exists
 * with every temporary of the query batch in one fixed 64 MiB device array
 * per GPU (a static __device__ array, looked up at graph creation), so the
 * call allocates nothing.  n <= 2^18 pairs, and the batch's temporaries
 * (about 120 bytes per pair plus 32 bytes per 256 pool slots of the graph)
 * must fit the array: GV_ERANGE otherwise, before any device work.  Same
 * arguments, result and asynchrony as gv_edge_exists.  Every call on one GPU
 * shares the array: calls that overlap on a GPU (several graphs or streams)
 * race and must be serialised by the caller. */
int gv_edge_exists_noalloc(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                           uint64_t n, uint8_t* d_out);

/* Adjacency of v in ascending order into d_out (device, out_capacity
 * entries).  *degree is always set when v < capacity.  v >= capacity gives
 * GV_ERANGE with *degree = 0; out_capacity < degree gives GV_ERANGE with
 * *degree set and nothing written.  An inactive v has degree 0.  Synchronous. */
int gv_get_adjacency(gv_graph* g, uint32_t v, uint32_t* d_out,
                     uint64_t out_capacity, uint64_t* degree);

/* Memory footprint by exact block accounting (Sec. 5.4).  Synchronous. */
int gv_memory_used(gv_graph* g, gv_mem* out);

/* Canonical CSR dump for verification: d_offsets has capacity + 1 uint64
 * entries, d_dst receives each vertex's destinations in ascending order.
 * *checksum = sum over edges (u, v) of mix64((u << 32) | v) modulo 2^64 where
 * mix64 is the SplitMix64 output function.  d_offsets and d_dst may both be
 * NULL to compute only *num_edges and *checksum.  dst_capacity < edges gives
 * GV_ERANGE with *num_edges set.  Synchronous. */
int gv_dump_canonical(gv_graph* g, uint64_t* d_offsets, uint32_t* d_dst,
                      uint64_t dst_capacity, uint64_t* checksum,
                      uint64_t* num_edges);

/* Structural audit for tests: counts violations of the pool invariants
 * (every block id below the bump pointer is owned by exactly one adjacency or
 * sits on the free list exactly once; every vertex of degree d holds
 * ceil(d / B) blocks; no slot below a degree holds 0xFFFFFFFF or an inactive
 * id; inactive vertices have degree 0; the owner record of every held block
 * names its vertex and index; the vertex-delete scratch is clear).
 * *violations = 0 means consistent.
 * Synchronous. */
int gv_audit(gv_graph* g, uint64_t* violations);

int gv_graph_info(gv_graph* g, gv_info* out);
int gv_get_counters(gv_graph* g, gv_counters* out); /* synchronous */

/* Per-kernel timing with HIP events on the graph's stream.  While enabled,
 * every kernel launch is bracketed by events; gv_kernel_times returns, for
 * the kernel named `name`, the number of launches and their summed duration
 * in milliseconds since the last reset (synchronous). */
int gv_profile_enable(gv_graph* g, int enable);
/* Restrict timing to launches of one kernel name (NULL or "" = all), so that a
 * timed region carries events around that kernel only. */
int gv_profile_only(gv_graph* g, const char* name);
int gv_profile_reset(gv_graph* g);
int gv_kernel_times(gv_graph* g, const char* name, uint64_t* launches,
                    double* total_ms);
/* Names of the kernels timed since the last reset, comma-separated and
 * NUL-terminated, in order of first launch.  *needed receives the buffer size
 * the full list takes (terminator included); when cap is smaller, nothing is
 * written (buf may be NULL) and GV_ERANGE is returned.  Synchronous. */
int gv_kernel_names(gv_graph* g, char* buf, size_t cap, size_t* needed);

/* ---- Batched form ----------------------------------------------------
 * Many update batches of uneven sizes applied in order (the paper's batch
 * model, Sec. 4.3: a graph receives a sequence of vertex and edge insert /
 * delete batches).  One op is one batch; its arrays are device pointers read
 * when the op runs.  The result is the same as calling the single-batch
 * entry points in order with a NULL stats pointer. */
enum {
    GV_OP_INSERT_EDGES = 0,    /* a = src, b = dst, n pairs */
    GV_OP_DELETE_EDGES = 1,    /* a = src, b = dst, n pairs */
    GV_OP_INSERT_VERTICES = 2, /* a = ids, n ids (b unused) */
    GV_OP_DELETE_VERTICES = 3  /* a = ids, n ids (b unused) */
};
/* gv_op.flags: 0, or for a vertex insert run by gv_apply_ops,
 * GV_OP_FIT_TABLE: the caller knows every id is below the vertex capacity,
 * so the op neither grows the dictionary nor reads the device back (no host
 * wait); an id at or past the capacity then fails the op with a sticky
 * GV_ERANGE, as in a plan.  Any other flag, or the flag on another kind of
 * op, is GV_EINVAL. */
enum { GV_OP_FIT_TABLE = 1 };
typedef struct {
    uint32_t kind;
    uint32_t flags;
    const uint32_t* a;
    const uint32_t* b;
    uint64_t n;
} gv_op;

/* Tuning of one graph's batch paths.  The batched form's autotuner
 * (paper_2306_08252_amd/tuner.py) measures the settings per workload and
 * stores them in tuning.json; the binding applies them before creating a
 * plan.  Defaults: coalesce 0, max_run_pairs 0, small_sort_max 4096,
 * probe_group 32, probe_unroll 4, item_chunk 256, overlap 0.
 *   coalesce       gv_apply_ops and gv_plan_create apply every run of
 *                  consecutive edge batches (up to the next vertex batch) as
 *                  one mixed list (gv_apply_edge_ops): the same result as the
 *                  batches one after the other (each pair's last entry
 *                  decides), one grouping sort per run instead of one per
 *                  batch.  A run whose inserts do not fit the pool fails
 *                  them as a whole (sticky GV_ENOMEM) with its deletes applied.
 *   max_run_pairs  longest run coalesced, in pairs (0: 2^28; a batch
 *                  longer than the limit runs alone)
 *   small_sort_max insert / delete batches of at most this many pairs
 *                  (<= 4096) are packed and sorted by one workgroup
 *   probe_group    lanes that probe one work item against its batch
 *                  segment: 16, 32 (default) or 64
 *   probe_unroll   adjacency slots per lane per search step: 2, 4 (default)
 *                  or 8
 *   item_chunk     adjacency slots per work item, a power of two in
 *                  [64, 4096] (default 256)
 *   overlap        0 (default) or 1.  With 1, an insert or delete batch of
 *                  more than small_sort_max pairs queued by gv_insert_edges,
 *                  gv_delete_edges, gv_apply_ops or recorded by
 *                  gv_plan_create packs and sorts its pairs on a second
 *                  stream of the library's own, while the graph's stream
 *                  still runs the batches queued before it; the rest of the
 *                  batch waits for that sort on the graph's stream (a plan
 *                  records the two streams as parallel branches).  With
 *                  coalesce on, a run of more than 4096 pairs has its
 *                  gather, pack and sort on that stream too (two buffers of
 *                  the library's own, alternating), while the graph's
 *                  stream applies the run before it.
 *                  Results are those of overlap 0.  Contract: the batch's
 *                  d_src / d_dst must hold their pairs when the call is made
 *                  (written by a synchronous copy, or by work the caller has
 *                  waited for), not only once the work queued ahead of the
 *                  batch on the graph's stream has run; they must stay
 *                  unchanged until that stream has run the batch.
 *   reserved       must be 0 */
typedef struct {
    uint32_t coalesce;
    uint32_t max_run_pairs;
    uint32_t small_sort_max;
    uint32_t probe_group;
    uint32_t probe_unroll;
    uint32_t item_chunk;
    uint32_t overlap;
    uint32_t reserved;
} gv_tuning;
int gv_set_tuning(gv_graph* g, const gv_tuning* t);
int gv_get_tuning(gv_graph* g, gv_tuning* t);

/* A plan records every kernel of ops[0, n_ops) into one HIP graph, so that
 * the whole sequence is launched at once (gv_plan_launch) instead of one
 * launch per kernel per batch.  Everything a plan needs is sized when it is
 * created (synchronous): the scratch for the largest batch and, for vertex
 * deletes, buffers for a full pool (4 bytes per pool slot).  Vertex inserts
 * in a plan never grow the dictionary: an id at or past the current vertex
 * capacity makes the plan's run fail with a sticky GV_ERANGE (reserve
 * capacity with gv_config.vertex_capacity).  A plan may be launched any
 * number of times; each launch applies the ops again to the graph as it is,
 * reading the op arrays at that time (refill them between launches to stream
 * new batches of the same sizes).  gv_plan_launch is asynchronous (errors are
 * sticky, see gv_sync) and returns GV_EINVAL when a buffer the plan records
 * was reallocated since creation (a larger single call or a dictionary
 * growth in between: create the plan again).  A plan belongs to its graph
 * and must be destroyed before it. */
typedef struct gv_plan gv_plan;
int gv_plan_create(gv_graph* g, const gv_op* ops, uint64_t n_ops, gv_plan** out);
int gv_plan_launch(gv_plan* p);
void gv_plan_destroy(gv_plan* p);

/* One launch sequence per batch: ops applied in order through the
 * single-batch paths (the baseline the plan is compared with). */
int gv_apply_ops(gv_graph* g, const gv_op* ops, uint64_t n_ops);

/* ---- Paper-faithful ablation: complete binary tree of edge blocks ---------
 * The layout and algorithms of the paper itself on the same kind of device
 * pool, beside the directory path above, to measure what the redesign buys.
 * Each vertex's blocks form a complete binary tree (Sec. 4.1, Fig. 2): block
 * k (1-based, in attachment order) is level-order node k, attached by its bit
 * string (Sec. 4.5.1, Fig. 4: the binary form of k without its leading 1;
 * 0 = left, 1 = right; the 9th block gets "001").  Blocks come from an edge
 * queue popped at prefix-sum positions over all vertices (Sec. 4.5.1).
 * Insert (Alg. 1) and delete (Alg. 2) run one thread per vertex of the graph;
 * deletes leave holes and return no block (Sec. 4.5.2).  A query batch
 * (Alg. 3) collects each source's blocks by an in-order traversal, one
 * thread per query, then compares with one thread per slot.  Adjacencies are
 * sets (as above); all vertices 0 .. num_vertices - 1 exist, pairs with an
 * id past them are rejected.  There are no vertex operations.  All arrays are
 * device pointers; every call is synchronous.  Errors as above; GV_ENOMEM
 * when the edge queue cannot hold an insert batch (the batch is then not
 * applied). */
typedef struct gv_cbt gv_cbt;
int gv_cbt_init(gv_cbt** out, uint64_t num_vertices, const uint32_t* d_src,
                const uint32_t* d_dst, uint64_t num_edges, uint32_t block_slots,
                uint64_t pool_blocks, void* hip_stream);
int gv_cbt_insert_edges(gv_cbt* g, const uint32_t* d_src, const uint32_t* d_dst,
                        uint64_t n, gv_batch_stats* out_or_null);
int gv_cbt_delete_edges(gv_cbt* g, const uint32_t* d_src, const uint32_t* d_dst,
                        uint64_t n, gv_batch_stats* out_or_null);
int gv_cbt_edge_exists(gv_cbt* g, const uint32_t* d_src, const uint32_t* d_dst,
                       uint64_t n, uint8_t* d_out);
/* Canonical CSR dump (as gv_dump_canonical, without checksum): d_offsets has
 * capacity + 1 entries (capacity = the smallest power of two >= num_vertices);
 * both NULL to count only. */
int gv_cbt_dump(gv_cbt* g, uint64_t* d_offsets, uint32_t* d_dst, uint64_t dst_capacity,
                uint64_t* num_edges);
/* Blocks handed out by the edge queue (holes included: none return). */
int gv_cbt_blocks(gv_cbt* g, uint64_t* blocks_in_use);
int gv_cbt_set_stream(gv_cbt* g, void* hip_stream);
void gv_cbt_destroy(gv_cbt* g);
/* Host only: the bit string of level-order position k >= 1, NUL-terminated
 * into out (cap bytes); GV_ERANGE if it does not fit. */
int gv_cbt_bitstring(uint64_t k, char* out, uint64_t cap);

int gv_set_stream(gv_graph* g, void* hip_stream);
/* Test support: the number of extra status loads each look-back wait of a
 * batch sort makes before it gives up (default 2^24).  0 makes every wait give
 * up at once, so the failure path (GV_EDEVICE, no change to the graph) can be
 * exercised without a real stall.  Synchronous. */
int gv_debug_spin_limit(gv_graph* g, uint32_t limit);
/* Wait for all queued work; returns and clears the first error of earlier
 * asynchronous calls. */
int gv_sync(gv_graph* g);
const char* gv_strerror(int code);
/* The HIP call and HIP error text of the last GV_EDEVICE / GV_ENOMEM raised
 * by a HIP call on this host thread ("" if none); owned by the library. */
const char* gv_last_error(void);
void gv_graph_destroy(gv_graph* g);

#ifdef __cplusplus
}
#endif
#endif /* GRAPHVINE_H */
