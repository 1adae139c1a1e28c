/*
 * gv_oracle.h -- CPU oracle for the GraphVine dynamic-graph operations.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct definition that the GPU structure is checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * Model (GraphVine, Sec. 4): a vertex dictionary whose capacity is a power of
 * two (Sec. 4.1, Sec. 4.4) and, for every active vertex, its adjacency.  Here
 * the adjacency is held as an ordered set of destination ids, which gives set
 * semantics: a repeated insert is a no-op and deleting an absent edge is a
 * no-op.  Edge blocks are modelled only for memory accounting: a vertex of
 * degree d occupies ceil(d / B) blocks of B slots (Sec. 4.1 edge blocks,
 * Sec. 4.2 edge queue, with deletes reclaiming emptied blocks).
 *
 * All ids are uint32.  The largest dictionary capacity is 2^31, so the largest
 * usable vertex id is 2^31 - 1.  Error codes carry the same numeric values as
 * the GPU library's but are defined here independently.
 */
#ifndef GV_ORACLE_H
#define GV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_EINVAL = 1, /* null pointer where data is required, bad config      */
    ORC_ERANGE = 2, /* id outside the dictionary, or output buffer too small */
    ORC_ENOMEM = 3  /* the block pool would overflow; graph left unchanged   */
};

#define ORC_MAX_CAPACITY (1ull << 31)

typedef struct orc_graph orc_graph;

typedef struct {
    uint64_t applied;          /* edges (or vertices) actually added/removed  */
    uint64_t rejected;         /* pairs/ids with an inactive or bad endpoint  */
    uint64_t batch_duplicates; /* valid entries minus distinct valid entries  */
} orc_stats;

/* Smallest power of two >= max(x, 1) (dictionary sizing, Sec. 4.1 and 4.4). */
uint64_t orc_next_pow2(uint64_t x);

/* Block-size rule of Sec. 4.3: B is the average degree of the vertices of
 * non-zero degree in the first batch, rounded up to a power of two and kept
 * within [8, 64].  `edges` = distinct edges, `nonzero` = vertices with at
 * least one out-edge.  Returns 8 when there are no edges. */
uint32_t orc_paper_block_slots(uint64_t edges, uint64_t nonzero);

/* 64-bit finaliser of SplitMix64 (Steele, Lea, Flood 2014) used for the
 * order-independent edge-set checksum. */
uint64_t orc_mix64(uint64_t z);

/* Build a graph with vertices 0..num_vertices-1 active and the distinct pairs
 * of the COO list (src[i], dst[i]) as edges.  Dictionary capacity is
 * next_pow2(max(num_vertices, vertex_capacity, 1)).  Any id >= num_vertices
 * gives ORC_ERANGE and no graph.  block_slots = 0 selects the rule above;
 * otherwise it must be a power of two in [1, 1024].  pool_bytes = 0 means an
 * unbounded pool; otherwise the pool holds floor(pool_bytes / (4 B)) blocks
 * and a graph that needs more gives ORC_ENOMEM. */
int orc_graph_init(orc_graph** out, uint64_t num_vertices, const uint32_t* src,
                   const uint32_t* dst, uint64_t num_edges,
                   uint64_t vertex_capacity, uint32_t block_slots,
                   uint64_t pool_bytes);
void orc_graph_destroy(orc_graph* g);

/* Batched edge operations (Sec. 4.5).  A pair is valid when both endpoints
 * are < capacity and active.  stats may be NULL.  On ORC_ENOMEM the graph is
 * unchanged and stats are zero. */
int orc_insert_edges(orc_graph* g, const uint32_t* src, const uint32_t* dst,
                     uint64_t n, orc_stats* stats);
int orc_delete_edges(orc_graph* g, const uint32_t* src, const uint32_t* dst,
                     uint64_t n, orc_stats* stats);

/* Mixed edge updates (the tick of the served form; the order inside a batch
 * is ours, the batch model is Sec. 4.3): entry i inserts (op[i] == 0) or
 * deletes (op[i] == 1) the pair (src[i], dst[i]), the entries applied one at
 * a time in index order with set semantics.  An entry with an inactive or
 * out-of-range endpoint, or another op value, changes nothing.  The pool
 * bound is not checked. */
int orc_apply_edge_ops(orc_graph* g, const uint8_t* op, const uint32_t* src,
                       const uint32_t* dst, uint64_t n);

/* Batched vertex operations (Sec. 4.4).  Insert activates inactive ids,
 * growing the capacity to next_pow2(id + 1) when needed; ids > 2^31 - 1 are
 * rejected.  Delete removes every out- and in-edge of each active id and
 * deactivates it; ids >= capacity are rejected; inactive ids are no-ops. */
int orc_insert_vertices(orc_graph* g, const uint32_t* ids, uint64_t n,
                        orc_stats* stats);
int orc_delete_vertices(orc_graph* g, const uint32_t* ids, uint64_t n,
                        orc_stats* stats);

/* Edge query (Sec. 4.6): out[i] = 1 when src[i] is active and dst[i] is in
 * its adjacency, else 0. */
int orc_edge_exists(const orc_graph* g, const uint32_t* src,
                    const uint32_t* dst, uint64_t n, uint8_t* out);

/* Adjacency of v in ascending order.  v >= capacity: ORC_ERANGE, *degree = 0.
 * capacity < degree: ORC_ERANGE with *degree set and nothing written. */
int orc_get_adjacency(const orc_graph* g, uint32_t v, uint32_t* out,
                      uint64_t out_capacity, uint64_t* degree);

/* Canonical CSR over all capacity ids: offsets[capacity + 1] (uint64) and
 * ascending destinations per vertex.  checksum = sum over edges (u, v) of
 * mix64((u << 32) | v) modulo 2^64.  offsets/dst may be NULL to get only the
 * checksum; dst_capacity < edges gives ORC_ERANGE. */
int orc_dump_canonical(const orc_graph* g, uint64_t* offsets, uint32_t* dst,
                       uint64_t dst_capacity, uint64_t* checksum);

uint64_t orc_capacity(const orc_graph* g);
uint64_t orc_num_edges(const orc_graph* g);
uint32_t orc_block_slots(const orc_graph* g);
uint64_t orc_pool_blocks(const orc_graph* g); /* 0 = unbounded */
uint64_t orc_blocks_in_use(const orc_graph* g);
int orc_is_active(const orc_graph* g, uint32_t v);
uint64_t orc_degree(const orc_graph* g, uint32_t v);

/* Edge attributes (Sec. 4.1: an edge entry may carry attributes).
 * orc_set_attr_words gives every stored edge `words` (1..8) attribute words,
 * all zero, once per graph.  From then on a newly stored edge starts with
 * zeros and a removed edge loses its words.  orc_set_edge_attrs applies the
 * rows vals[i * A ...] one pair at a time in batch order to the pairs that
 * are stored (a later row of a pair overwrites an earlier one); stats:
 * applied = distinct stored pairs written, rejected = invalid pairs,
 * batch_duplicates = valid minus distinct valid.  orc_get_edge_attrs: found
 * flag and the words of each pair (zeros when absent). */
int orc_set_attr_words(orc_graph* g, uint32_t words);
uint32_t orc_attr_words(const orc_graph* g);
int orc_set_edge_attrs(orc_graph* g, const uint32_t* src, const uint32_t* dst,
                       const uint32_t* vals, uint64_t n, orc_stats* stats);
int orc_get_edge_attrs(const orc_graph* g, const uint32_t* src, const uint32_t* dst,
                       uint64_t n, uint8_t* found, uint32_t* vals);

/* Block size over the graph's life (Sec. 6, future scope).
 * orc_set_block_slots: the same edges, accounted in blocks of the new size
 * (power of two in [1, 1024]); a bounded pool keeps its byte budget, and a
 * graph that would not fit gives ORC_ENOMEM unchanged.
 * orc_adapted_block_slots: the rule of Sec. 4.3 applied to the current
 * graph (average degree of the non-zero-degree vertices, power of two within
 * [8, 64]). */
int orc_set_block_slots(orc_graph* g, uint32_t block_slots);
uint32_t orc_adapted_block_slots(const orc_graph* g);

#ifdef __cplusplus
}
#endif
#endif
