// gv_graph.h -- the host object behind gv_graph* and the internal entry
// points implemented by the kernel files.
#pragma once

#include "gv_device.h"
#include "gv_host.h"

struct gv_graph {
    int device = 0;
    gv::Ctx ctx;
    gv::GraphView v{};            // device pointers and sizes
    gv::DevCounters* hctr = nullptr;  // pinned host copy for read-back
    gv::Scratch scratch;          // per-call temporaries
    gv::Scratch vscr[3];          // vertex-batch buffers that outlive an inner edge batch
    gv::Scratch cscr;             // a coalesced run of edge batches (batched form)
    gv_tuning tune{0u, 0u, 4096u, 32u, 4u, 256u, 0u, 0u};
    uint64_t table_gen = 0;       // counts reallocations of the vertex table or the pool
    uint64_t item_slots = 0;      // bound on live adjacency slots (pool slots)
    // upper bound on the edges stored, kept on the host without a read-back:
    // exact after each counter read, plus the pairs of every insert since
    uint64_t edge_bound_host = 0;
    uint32_t spin_limit = gv::kSpinLimitDefault;  // bound on each look-back wait of batch sorts
    // Sort overlap (tune.overlap): a second stream packs and sorts each large
    // insert / delete batch while the graph's stream runs the batches before
    // it.  Batches alternate between two buffers: buffer 0 is `scratch`,
    // buffer 1 is ov_scr.  Every sort on the side stream is followed on the
    // graph's stream by a wait for its event, so whatever waits for the
    // graph's stream has also waited for the side stream.
    struct Overlap {
        hipStream_t stream = nullptr;
        gv::Ctx ctx;                      // launches on `stream`
        gv::Scratch scr;                  // buffer 1
        hipEvent_t sorted[2] = {nullptr, nullptr};  // side: the buffer's sort is done
        hipEvent_t done[2] = {nullptr, nullptr};    // graph's stream: done with the buffer
        hipEvent_t fence = nullptr;       // graph's stream: all work queued before a batch
        bool used[2] = {false, false};    // done[k] has been recorded
        uint64_t count = 0;               // overlapped batches (next buffer = count & 1)
        uint64_t seq = ~0ull;             // ctx.seq after the last overlapped batch
        // Coalesced runs of the batched form (mixed lists): the gather, pack
        // and sort of a run go to the side stream with buffers of their own,
        // which alternate; that work reads nothing the graph's stream
        // changes, so it waits only for the buffer's previous user.
        gv::Scratch mix[2];
        hipEvent_t msorted[2] = {nullptr, nullptr};
        hipEvent_t mdone[2] = {nullptr, nullptr};
        bool mused[2] = {false, false};
        uint64_t mcount = 0;
        // the side stream waited for the graph's stream since the capture
        // state last changed (its first wait joins a capture)
        bool joined = false;
        // id of the stream capture the state above belongs to (0: none);
        // events of another capture, or of none, are never waited for
        unsigned long long capture = 0;
    } ov;
    // device allocations owned by the graph
    void* mem_pool = nullptr;
    void* mem_free = nullptr;
    void* mem_dir = nullptr;
    void* mem_dfree = nullptr;
    void* mem_vt = nullptr;
    void* mem_active = nullptr;
    void* mem_ctr = nullptr;
    void* mem_chain = nullptr;  // ChainState of the graph's stream
    void* mem_bown = nullptr;
    void* mem_vlost = nullptr;
    void* mem_apool = nullptr;
    bool dead = false;            // set after a device failure
};

namespace gv {

enum EdgeMode { kInsert = 0, kDelete = 1, kQuery = 2 };

// queue one batched edge operation on the graph's stream (no host sync);
// `sticky` makes an allocation failure visible to later gv_sync calls
// `fixed` (optional): carve the batch's temporaries from this device buffer of
// fixed_bytes instead of the graph's growable scratch (GV_ERANGE if they do
// not fit); nothing is allocated then
void edge_batch(gv_graph* g, EdgeMode mode, const uint32_t* src, const uint32_t* dst,
                uint64_t n, uint8_t* out, bool sticky, void* fixed = nullptr,
                size_t fixed_bytes = 0);

// an insert or delete batch whose keys (src << L) | dst are already sorted,
// distinct and valid: keys[0, *count) with the count on the device (at most
// n_max); keys must not live in g->scratch, which the batch carves.
// mark_out (optional, n_max bytes): per key, 1 if the pair was stored when
// the batch started
void edge_batch_sorted(gv_graph* g, EdgeMode mode, const uint64_t* keys,
                       const unsigned long long* count, uint64_t n_max, bool sticky,
                       uint8_t* mark_out = nullptr);

// the per-device address of the fixed scratch of gv_edge_exists_noalloc,
// looked up once per device (graph creation calls it with the device current)
void noalloc_setup();

}  // namespace gv

// the query batch of gv_edge_exists_noalloc (gv_noalloc.hip)
void gv_noalloc_query(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                      uint8_t* d_out);

namespace gv {

// attributes of pairs (a query batch that also finds their slots): get
// (found flags to `found`, n * A words to `out`, zeros when absent) or set
// (`in`, n * A words; for each stored pair its last occurrence writes)
void edge_attrs(gv_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t n,
                uint8_t* found, uint32_t* out, const uint32_t* in);

// a list of (op, src, dst) entries, op 0 insert / 1 delete, applied as if one
// at a time in list order (last-writer reduction, then one delete batch and
// one insert batch; no host sync)
// With req_end (device array of n_req ascending ends, the last == n) and
// stats (device array of n_req): each request's statistics as if the
// requests were applied alone, in order.
void mixed_edges(gv_graph* g, const uint8_t* op, const uint32_t* src, const uint32_t* dst,
                 uint64_t n, const uint64_t* req_end = nullptr, uint64_t n_req = 0,
                 gv_batch_stats* stats = nullptr);

// occupancy queries made ahead of a recording
void edge_batch_warm(const gv_graph* g = nullptr);
// the side stream and events of the sort overlap (made once)
void overlap_open(gv_graph* g);
// the overlap's state for the capture the graph's stream is in: state that
// belongs to another capture (or to none) is dropped
void overlap_capture(gv_graph* g);
// the side stream waits for everything queued on the graph's stream so far
void overlap_fence(gv_graph* g);
// a mixed list (the batched form's coalesced run) whose entries are written
// by gather(ctx, op, src, dst) and packed and sorted on the overlap's side
// stream; the rest of the list runs on the graph's stream.  `fence`: the
// side stream first waits for everything queued on the graph's stream (the
// first list of a call); otherwise only for the list that used its buffer
void mixed_edges_side(gv_graph* g, uint64_t n, bool fence,
                      const std::function<void(Ctx&, uint8_t*, uint32_t*, uint32_t*)>& gather);
// bytes of each of the two buffers mixed_edges_side uses for n entries
size_t mixed_side_bytes(const gv_graph* g, uint64_t n);
bool probe_shape_ok(uint32_t group, uint32_t unroll);
void vertex_batch_warm();
// bytes of g->scratch an edge batch of n pairs carves
size_t edge_batch_bytes(const gv_graph* g, EdgeMode mode, uint64_t n);
// bytes of g->scratch ([0]) and g->vscr[0] ([1]) a mixed list of n entries needs
void mixed_bytes(const gv_graph* g, uint64_t n, size_t out[2]);
// bytes a vertex batch needs: [0] g->scratch, [1..3] g->vscr[0..2]
void vertex_batch_bytes(const gv_graph* g, bool del, uint64_t n, uint64_t edge_bound,
                        size_t out[4]);

// bulk build into a graph whose vertex table is allocated (synchronous)
void bulk_build(gv_graph* g, uint64_t num_vertices, const uint32_t* src, const uint32_t* dst,
                uint64_t m, const gv_config& cfg);

// fixed_table: never grow the dictionary (and never read back); ids past it
// raise a sticky GV_ERANGE
void vertex_insert(gv_graph* g, const uint32_t* ids, uint64_t n, gv_batch_stats* st,
                   bool fixed_table = false);
// edge_bound: upper bound on the edges stored (0: the host-side bound, no read-back)
void vertex_delete(gv_graph* g, const uint32_t* ids, uint64_t n, gv_batch_stats* st,
                   uint64_t edge_bound = 0);

void adjacency(gv_graph* g, uint32_t v, uint32_t* out, uint64_t cap, uint64_t* degree);
// the block size the rule of Sec. 4.3 gives for the graph as it is now, and
// the same graph re-laid in blocks of another size (Sec. 6), synchronous
uint32_t adapted_block_slots(gv_graph* g);
void relayout(gv_graph* g, uint32_t block_slots);
void dump(gv_graph* g, uint64_t* offsets, uint32_t* dst, uint64_t cap, uint64_t* checksum,
          uint64_t* edges);
uint64_t audit(gv_graph* g);

// copy the device counters into g->hctr (synchronous)
void read_counters(gv_graph* g);
// set one 32-bit or 64-bit device word from a kernel (stream ordered)
void set_u32(gv_graph* g, uint32_t* p, uint32_t value);
void set_u64(gv_graph* g, unsigned long long* p, unsigned long long value);

inline uint32_t log2_exact(uint64_t x) {
    uint32_t c = 0;
    while ((1ull << c) < x) ++c;
    return c;
}

}  // namespace gv
