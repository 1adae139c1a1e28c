// gv_api.hip -- the C ABI declared in include/graphvine.h.
//
// Validates arguments, keeps the graph's device current for the duration of
// a call, and turns internal failures into GV_* codes: no exception crosses
// this boundary.
#include <algorithm>
#include <cstring>
#include <new>

#include "gv_graph.h"

using namespace gv;

namespace {

struct DeviceGuard {
    int prev = -1;
    int want;
    explicit DeviceGuard(int dev) : want(dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != want) hip_check(hipSetDevice(want), "hipSetDevice");
    }
    ~DeviceGuard() {
        if (prev >= 0 && prev != want) hipSetDevice(prev);
    }
};

template <typename F>
int guarded(gv_graph* g, F&& f) {
    if (!g) return GV_EINVAL;
    if (g->dead) return GV_EDEVICE;
    try {
        DeviceGuard dg(g->device);
        f();
        return GV_OK;
    } catch (const Error& e) {
        if (e.code == GV_EDEVICE) g->dead = true;
        return e.code;
    } catch (const std::bad_alloc&) {
        return GV_ENOMEM;
    } catch (...) {
        g->dead = true;
        return GV_EDEVICE;
    }
}

void free_graph(gv_graph* g) {
    if (!g) return;
    hipStreamSynchronize(g->ctx.stream);
    g->ctx.release();
    gv_graph::Overlap& o = g->ov;
    if (o.stream) {
        hipStreamSynchronize(o.stream);
        o.ctx.release();
        hipEvent_t evs[] = {o.sorted[0],  o.sorted[1],  o.done[0],  o.done[1], o.fence,
                            o.msorted[0], o.msorted[1], o.mdone[0], o.mdone[1]};
        for (hipEvent_t e : evs)
            if (e) hipEventDestroy(e);
        hipStreamDestroy(o.stream);
        o.stream = nullptr;
    }
    o.scr.release();
    for (auto& m : o.mix) m.release();
    g->scratch.release();
    for (auto& v : g->vscr) v.release();
    g->cscr.release();
    void* mem[] = {g->mem_pool,   g->mem_free, g->mem_dir,  g->mem_dfree, g->mem_vt,
                   g->mem_active, g->mem_ctr,  g->mem_bown, g->mem_vlost, g->mem_apool,
                   g->mem_chain};
    for (void* p : mem)
        if (p) hipFree(p);
    if (g->hctr) hipHostFree(g->hctr);
    delete g;
}

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

// A batch sort that failed (a look-back wait ran out, or the sorted keys were
// out of order or not the packed keys) left its batch and every later batch
// undone, and a vertex delete that ran past one of its list bounds left its
// batch partly applied: either way the graph is unusable.  Reads the
// counters last copied to the host.
void check_sort(gv_graph* g) {
    if (g->hctr->err_wait) fail(GV_EDEVICE, "a batch sort's look-back wait ran out");
    if (g->hctr->err_order == 2) fail(GV_EDEVICE, "a batch's sorted keys were out of order");
    if (g->hctr->err_order == 4) fail(GV_EDEVICE, "a vertex delete exceeded a device-side bound");
    if (g->hctr->err_order) fail(GV_EDEVICE, "a batch's sorted keys were not its packed keys");
}

// Timed launches of both launch contexts (the graph's stream and the sort
// overlap's side stream) folded into their per-name sums.
void collect_all(gv_graph* g) {
    g->ctx.collect();
    g->ov.ctx.collect();
}

void fill_stats(gv_graph* g, gv_batch_stats* st) {
    st->applied = g->hctr->st_applied;
    st->rejected = g->hctr->st_rejected;
    st->batch_duplicates = g->hctr->st_dups;
}

}  // namespace

extern "C" {

const char* gv_last_error(void) { return last_error_text(); }

const char* gv_strerror(int code) {
    switch (code) {
        case GV_OK: return "ok";
        case GV_EINVAL: return "invalid argument";
        case GV_ERANGE: return "id or size out of range";
        case GV_ENOMEM: return "out of memory (pool, directory or device)";
        case GV_EDEVICE: return "HIP device failure";
        default: return "unknown error";
    }
}

int gv_graph_init(gv_graph** out, uint64_t num_vertices, const uint32_t* d_src,
                  const uint32_t* d_dst, uint64_t num_edges, const gv_config* cfg,
                  void* hip_stream) {
    if (!out) return GV_EINVAL;
    *out = nullptr;
    gv_config c{};
    if (cfg) c = *cfg;
    if (num_vertices > GV_MAX_CAPACITY || c.vertex_capacity > GV_MAX_CAPACITY) return GV_EINVAL;
    if (c.block_slots != 0 && (c.block_slots > 1024 || !pow2(c.block_slots))) return GV_EINVAL;
    if (c.flags != 0 || c.reserved != 0 || c.edge_attr_words > GV_MAX_ATTR_WORDS)
        return GV_EINVAL;
    if (num_edges && (!d_src || !d_dst)) return GV_EINVAL;
    gv_graph* g = new (std::nothrow) gv_graph();
    if (!g) return GV_ENOMEM;
    try {
        hip_check(hipGetDevice(&g->device), "hipGetDevice");
        g->ctx.stream = (hipStream_t)hip_stream;
        uint64_t want = std::max<uint64_t>(std::max<uint64_t>(num_vertices, c.vertex_capacity), 1);
        uint64_t cap = 1;
        while (cap < want) cap <<= 1;
        GraphView& v = g->v;
        v.n_cap = cap;
        v.L = log2_exact(cap);
        v.A = c.edge_attr_words;
        hip_check(hipMalloc(&g->mem_vt, cap * sizeof(VRec)), "hipMalloc vertex table");
        hip_check(hipMalloc(&g->mem_active, ((cap + 31) / 32) * 4), "hipMalloc active");
        hip_check(hipMalloc(&g->mem_ctr, sizeof(DevCounters)), "hipMalloc counters");
        hip_check(hipMalloc(&g->mem_chain, sizeof(ChainState)), "hipMalloc scan state");
        hip_check(hipMemsetAsync(g->mem_chain, 0, sizeof(ChainState), g->ctx.stream),
                  "hipMemsetAsync");
        hip_check(hipMalloc(&g->mem_vlost, cap * sizeof(uint32_t)), "hipMalloc vertex scratch");
        hip_check(hipMemsetAsync(g->mem_vlost, 0, cap * sizeof(uint32_t), g->ctx.stream),
                  "hipMemsetAsync");
        hip_check(hipHostMalloc((void**)&g->hctr, sizeof(DevCounters), hipHostMallocDefault),
                  "hipHostMalloc");
        hip_check(hipMemsetAsync(g->mem_ctr, 0, sizeof(DevCounters), g->ctx.stream),
                  "hipMemsetAsync");
        v.vt = (VRec*)g->mem_vt;
        v.active = (uint32_t*)g->mem_active;
        v.ctr = (DevCounters*)g->mem_ctr;
        g->ctx.chain = g->mem_chain;
        g->ctx.chain_err = &v.ctr->err_wait;
        v.vlost = (uint32_t*)g->mem_vlost;
        noalloc_setup();
        bulk_build(g, num_vertices, d_src, d_dst, num_edges, c);
    } catch (const Error& e) {
        free_graph(g);
        return e.code;
    } catch (const std::bad_alloc&) {
        free_graph(g);
        return GV_ENOMEM;
    } catch (...) {
        free_graph(g);
        return GV_EDEVICE;
    }
    *out = g;
    return GV_OK;
}

void gv_graph_destroy(gv_graph* g) {
    if (!g) return;
    const int dev = g->device;
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != dev) hipSetDevice(dev);
    free_graph(g);
    if (prev >= 0 && prev != dev) hipSetDevice(prev);
}

static int edge_update(gv_graph* g, EdgeMode mode, const uint32_t* s, const uint32_t* d,
                       uint64_t n, gv_batch_stats* st) {
    if (st) std::memset(st, 0, sizeof(*st));
    if (!g) return GV_EINVAL;
    if (n && (!s || !d)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    int rc = guarded(g, [&] {
        edge_batch(g, mode, s, d, n, nullptr, st == nullptr);
        if (st) {
            read_counters(g);
            check_sort(g);
            if (g->hctr->err_batch) fail((int)g->hctr->err_batch, "batch failed");
            fill_stats(g, st);
        }
    });
    if (rc != GV_OK && st) std::memset(st, 0, sizeof(*st));
    return rc;
}

int gv_insert_edges(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                    gv_batch_stats* st) {
    return edge_update(g, kInsert, d_src, d_dst, n, st);
}

int gv_delete_edges(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                    gv_batch_stats* st) {
    return edge_update(g, kDelete, d_src, d_dst, n, st);
}

int gv_insert_vertices(gv_graph* g, const uint32_t* d_ids, uint64_t n, gv_batch_stats* st) {
    if (st) std::memset(st, 0, sizeof(*st));
    if (!g || (n && !d_ids)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    gv_batch_stats tmp{};
    int rc = guarded(g, [&] { vertex_insert(g, d_ids, n, &tmp); });
    if (rc == GV_OK && st) *st = tmp;
    return rc;
}

int gv_delete_vertices(gv_graph* g, const uint32_t* d_ids, uint64_t n, gv_batch_stats* st) {
    if (st) std::memset(st, 0, sizeof(*st));
    if (!g || (n && !d_ids)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    gv_batch_stats tmp{};
    int rc = guarded(g, [&] {
        vertex_delete(g, d_ids, n, &tmp);
        check_sort(g);  // counters were read back for the statistics
    });
    if (rc == GV_OK && st) *st = tmp;
    return rc;
}

int gv_edge_exists(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                   uint8_t* d_out) {
    if (!g) return GV_EINVAL;
    if (n && (!d_src || !d_dst || !d_out)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    return guarded(g, [&] { edge_batch(g, kQuery, d_src, d_dst, n, d_out, true); });
}

int gv_edge_exists_noalloc(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                           uint64_t n, uint8_t* d_out) {
    if (!g) return GV_EINVAL;
    if (n && (!d_src || !d_dst || !d_out)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    return guarded(g, [&] { gv_noalloc_query(g, d_src, d_dst, n, d_out); });
}

int gv_set_block_slots(gv_graph* g, uint32_t block_slots) {
    if (!g || block_slots == 0 || block_slots > 1024 || !pow2(block_slots)) return GV_EINVAL;
    return guarded(g, [&] { relayout(g, block_slots); });
}

int gv_adapt_block_slots(gv_graph* g, uint32_t* block_slots) {
    if (!g || !block_slots) return GV_EINVAL;
    return guarded(g, [&] {
        const uint32_t b = adapted_block_slots(g);
        relayout(g, b);
        *block_slots = b;
    });
}

int gv_set_edge_attrs(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst,
                      const uint32_t* d_attr, uint64_t n, gv_batch_stats* st) {
    if (st) std::memset(st, 0, sizeof(*st));
    if (!g || !g->v.A) return GV_EINVAL;
    if (n && (!d_src || !d_dst || !d_attr)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    int rc = guarded(g, [&] {
        edge_attrs(g, d_src, d_dst, n, nullptr, nullptr, d_attr);
        if (st) {
            read_counters(g);
            check_sort(g);
            const uint64_t valid = g->hctr->tot[0];  // valid pairs of the batch
            st->applied = g->hctr->st_applied;
            st->rejected = n - valid;
            st->batch_duplicates = valid - g->hctr->n_uniq;
        }
    });
    if (rc != GV_OK && st) std::memset(st, 0, sizeof(*st));
    return rc;
}

int gv_get_edge_attrs(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                      uint8_t* d_found, uint32_t* d_attr) {
    if (!g || !g->v.A) return GV_EINVAL;
    if (n && (!d_src || !d_dst || !d_found || !d_attr)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    return guarded(g, [&] { edge_attrs(g, d_src, d_dst, n, d_found, d_attr, nullptr); });
}

int gv_apply_edge_ops(gv_graph* g, const uint8_t* d_op, const uint32_t* d_src,
                      const uint32_t* d_dst, uint64_t n) {
    if (!g) return GV_EINVAL;
    if (n && (!d_op || !d_src || !d_dst)) return GV_EINVAL;
    if (n == 0) return GV_OK;
    return guarded(g, [&] { mixed_edges(g, d_op, d_src, d_dst, n); });
}

int gv_apply_edge_ops_stats(gv_graph* g, const uint8_t* d_op, const uint32_t* d_src,
                            const uint32_t* d_dst, uint64_t n, const uint64_t* d_req_end,
                            uint64_t n_req, gv_batch_stats* d_stats) {
    if (!g) return GV_EINVAL;
    if (n && (!d_op || !d_src || !d_dst)) return GV_EINVAL;
    if (n_req == 0) return n == 0 ? GV_OK : GV_EINVAL;
    if (!d_req_end || !d_stats || n_req >= 0xffffffffull) return GV_EINVAL;
    return guarded(g, [&] { mixed_edges(g, d_op, d_src, d_dst, n, d_req_end, n_req, d_stats); });
}

int gv_get_adjacency(gv_graph* g, uint32_t v, uint32_t* d_out, uint64_t out_capacity,
                     uint64_t* degree) {
    if (!g || !degree) return GV_EINVAL;
    *degree = 0;
    uint64_t deg = 0;
    int rc = guarded(g, [&] { adjacency(g, v, d_out, out_capacity, &deg); });
    *degree = deg;
    return rc;
}

int gv_memory_used(gv_graph* g, gv_mem* out) {
    if (!g || !out) return GV_EINVAL;
    return guarded(g, [&] {
        read_counters(g);
        const GraphView& v = g->v;
        const DevCounters& c = *g->hctr;
        gv_mem m{};
        m.block_bytes = 4ull * v.B;
        m.pool_capacity_blocks = v.cap_blocks;
        m.free_list_blocks = c.free_cnt;
        m.bump_blocks = c.bump;
        m.blocks_in_use = c.bump - c.free_cnt;
        m.vertex_capacity = v.n_cap;
        m.vertex_table_bytes = v.n_cap * sizeof(VRec) + ((v.n_cap + 31) / 32) * 4;
        m.directory_entries_in_use = c.dir_live;
        uint64_t dfree_total = 0;
        for (int k = 1; k < kMaxClass; ++k) dfree_total += v.dir_cap >> k;
        m.directory_bytes = 4ull * (v.dir_cap + dfree_total);
        m.live_bytes = m.blocks_in_use * m.block_bytes + m.vertex_table_bytes + 4ull * c.dir_live;
        m.num_edges = c.live_edges;
        m.reserved_bytes = v.cap_blocks * m.block_bytes + 4ull * v.cap_blocks +
                           8ull * v.cap_blocks + 4ull * v.n_cap +
                           4ull * v.A * v.cap_blocks * v.B + m.directory_bytes +
                           m.vertex_table_bytes + sizeof(DevCounters) + sizeof(ChainState) +
                           g->scratch.cap +
                           g->ov.scr.cap + g->ov.mix[0].cap + g->ov.mix[1].cap;
        *out = m;
    });
}

int gv_dump_canonical(gv_graph* g, uint64_t* d_offsets, uint32_t* d_dst, uint64_t dst_capacity,
                      uint64_t* checksum, uint64_t* num_edges) {
    if (!g || !checksum || !num_edges) return GV_EINVAL;
    if ((d_offsets == nullptr) != (d_dst == nullptr)) return GV_EINVAL;
    uint64_t ck = 0, e = 0;
    int rc = guarded(g, [&] { dump(g, d_offsets, d_dst, dst_capacity, &ck, &e); });
    *checksum = ck;
    *num_edges = e;
    return rc;
}

int gv_audit(gv_graph* g, uint64_t* violations) {
    if (!g || !violations) return GV_EINVAL;
    uint64_t bad = 0;
    int rc = guarded(g, [&] { bad = audit(g); });
    *violations = bad;
    return rc;
}

int gv_graph_info(gv_graph* g, gv_info* out) {
    if (!g || !out) return GV_EINVAL;
    out->vertex_capacity = g->v.n_cap;
    out->block_slots = g->v.B;
    out->device = (uint32_t)g->device;
    return GV_OK;
}

int gv_get_counters(gv_graph* g, gv_counters* out) {
    if (!g || !out) return GV_EINVAL;
    return guarded(g, [&] {
        read_counters(g);
        const DevCounters& c = *g->hctr;
        for (int k = 0; k < 3; ++k) {
            out->batches[k] = c.c_batches[k];
            out->pairs[k] = c.c_pairs[k];
            out->touched[k] = c.c_touched[k];
            out->scanned_slots[k] = c.c_scanned[k];
        }
        out->new_blocks = c.c_new_blocks;
        out->freed_blocks = c.c_freed_blocks;
        out->written_slots = c.c_written;
        unsigned long long moved = 0;
        for (int k = 0; k < 64; ++k) moved += c.stripe[k][0];
        out->moved_slots = moved;
    });
}

int gv_profile_enable(gv_graph* g, int enable) {
    if (!g) return GV_EINVAL;
    return guarded(g, [&] {
        collect_all(g);
        g->ctx.prof = enable != 0;
    });
}

int gv_profile_only(gv_graph* g, const char* name) {
    if (!g) return GV_EINVAL;
    return guarded(g, [&] {
        collect_all(g);
        g->ctx.only = name ? name : "";
    });
}

int gv_profile_reset(gv_graph* g) {
    if (!g) return GV_EINVAL;
    return guarded(g, [&] {
        collect_all(g);
        g->ctx.sums.clear();
        g->ov.ctx.sums.clear();
    });
}

int gv_kernel_times(gv_graph* g, const char* name, uint64_t* launches, double* total_ms) {
    if (!g || !name || !launches || !total_ms) return GV_EINVAL;
    *launches = 0;
    *total_ms = 0;
    return guarded(g, [&] {
        collect_all(g);
        for (const Ctx* c : {&g->ctx, &g->ov.ctx})
            for (auto& s : c->sums)
                if (s.name == name) {
                    *launches += s.launches;
                    *total_ms += s.ms;
                }
    });
}

int gv_kernel_names(gv_graph* g, char* buf, size_t cap, size_t* needed) {
    if (!g || !needed) return GV_EINVAL;
    std::string all;
    const int rc = guarded(g, [&] {
        collect_all(g);
        std::vector<std::string> names;
        for (const Ctx* c : {&g->ctx, &g->ov.ctx})
            for (auto& s : c->sums)
                if (std::find(names.begin(), names.end(), s.name) == names.end())
                    names.push_back(s.name);
        for (auto& nm : names) {
            if (!all.empty()) all += ',';
            all += nm;
        }
    });
    if (rc != GV_OK) return rc;
    *needed = all.size() + 1;
    if (!buf || cap < all.size() + 1) return GV_ERANGE;
    std::memcpy(buf, all.c_str(), all.size() + 1);
    return GV_OK;
}

int gv_set_tuning(gv_graph* g, const gv_tuning* t) {
    if (!g || !t) return GV_EINVAL;
    if (t->coalesce > 1 || t->small_sort_max > 4096) return GV_EINVAL;
    if (!probe_shape_ok(t->probe_group, t->probe_unroll)) return GV_EINVAL;
    if (t->item_chunk < 64 || t->item_chunk > 4096 || !pow2(t->item_chunk)) return GV_EINVAL;
    if (t->overlap > 1 || t->reserved != 0) return GV_EINVAL;
    return guarded(g, [&] {
        hip_check(hipStreamSynchronize(g->ctx.stream), "hipStreamSynchronize");
        g->tune = *t;
    });
}

int gv_get_tuning(gv_graph* g, gv_tuning* t) {
    if (!g || !t) return GV_EINVAL;
    *t = g->tune;
    return GV_OK;
}

int gv_debug_spin_limit(gv_graph* g, uint32_t limit) {
    if (!g) return GV_EINVAL;
    return guarded(g, [&] {
        hip_check(hipStreamSynchronize(g->ctx.stream), "hipStreamSynchronize");
        g->spin_limit = limit;
    });
}

int gv_set_stream(gv_graph* g, void* hip_stream) {
    if (!g) return GV_EINVAL;
    return guarded(g, [&] {
        g->ctx.collect();
        hip_check(hipStreamSynchronize(g->ctx.stream), "hipStreamSynchronize");
        g->ctx.stream = (hipStream_t)hip_stream;
        ++g->ctx.seq;
    });
}

int gv_sync(gv_graph* g) {
    if (!g) return GV_EINVAL;
    int code = GV_OK;
    int rc = guarded(g, [&] {
        read_counters(g);
        check_sort(g);
        code = (int)g->hctr->err_sticky;
        if (code) {
            set_u32(g, &g->v.ctr->err_sticky, 0);
            hip_check(hipStreamSynchronize(g->ctx.stream), "hipStreamSynchronize");
        }
    });
    return rc != GV_OK ? rc : code;
}

}  // extern "C"
