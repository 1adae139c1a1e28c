// gv_oracle.cpp -- CPU oracle for the GraphVine dynamic-graph operations.
//
// TEST INFRASTRUCTURE ONLY (see gv_oracle.h).  Every operation is written as
// the plain definition over per-vertex ordered sets, one pair at a time, with
// no blocking, batching tricks or reordering, so that it can be checked
// against the paper by eye.  It is deliberately slow.

#include "gv_oracle.h"

#include <cstring>
#include <new>
#include <iterator>
#include <map>
#include <set>
#include <utility>
#include <vector>

struct orc_graph {
    uint64_t capacity;    // vertex dictionary size, a power of two (Sec. 4.1)
    uint32_t B;           // edge entries per edge block (Sec. 4.3)
    uint64_t pool_blocks; // blocks the edge queue can hand out; 0 = unbounded
    uint64_t pool_bytes;  // the pool's byte budget (0 = unbounded)
    std::vector<uint8_t> active;
    std::vector<std::set<uint32_t>> adj; // ordered adjacency set per vertex
    // Sec. 4.1: an edge entry may carry attributes; A words per stored edge,
    // keyed by (src << 32) | dst, present exactly for the stored edges
    uint32_t A = 0;
    std::map<uint64_t, std::vector<uint32_t>> attr;
};

static uint64_t pair_key(uint32_t u, uint32_t v) { return ((uint64_t)u << 32) | v; }

// a stored edge appears: its attributes start at zero
static void attr_new(orc_graph* g, uint32_t u, uint32_t v) {
    if (g->A) g->attr[pair_key(u, v)].assign(g->A, 0u);
}

// a stored edge disappears with its attributes
static void attr_drop(orc_graph* g, uint32_t u, uint32_t v) {
    if (g->A) g->attr.erase(pair_key(u, v));
}

extern "C" uint64_t orc_next_pow2(uint64_t x) {
    // Sec. 4.1: a dictionary for 453 vertices has 512 entries.  Read as the
    // smallest power of two that holds every vertex.
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

extern "C" uint32_t orc_paper_block_slots(uint64_t edges, uint64_t nonzero) {
    // Sec. 4.3 / Sec. 5.1: block size = average degree of the non-zero-degree
    // vertices of the first batch.  Rounded up to a power of two in [8, 64].
    if (edges == 0 || nonzero == 0) return 8;
    uint64_t avg = (edges + nonzero - 1) / nonzero;
    uint64_t b = orc_next_pow2(avg);
    if (b < 8) b = 8;
    if (b > 64) b = 64;
    return (uint32_t)b;
}

extern "C" uint64_t orc_mix64(uint64_t z) {
    // SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

static uint64_t blocks_for(const orc_graph* g, uint64_t degree) {
    return ceil_div(degree, g->B);
}

static bool valid_vertex(const orc_graph* g, uint32_t v) {
    return (uint64_t)v < g->capacity && g->active[v] != 0;
}

static void zero_stats(orc_stats* s) {
    if (s) std::memset(s, 0, sizeof(*s));
}

extern "C" uint64_t orc_blocks_in_use(const orc_graph* g) {
    // One block per B edge entries of each adjacency; emptied blocks go back to
    // the edge queue (Sec. 4.2), so only ceil(deg / B) blocks stay in use.
    uint64_t total = 0;
    for (uint64_t v = 0; v < g->capacity; ++v) total += blocks_for(g, g->adj[v].size());
    return total;
}

extern "C" int orc_graph_init(orc_graph** out, uint64_t num_vertices,
                              const uint32_t* src, const uint32_t* dst,
                              uint64_t num_edges, uint64_t vertex_capacity,
                              uint32_t block_slots, uint64_t pool_bytes) {
    if (!out) return ORC_EINVAL;
    *out = nullptr;
    if (num_edges && (!src || !dst)) return ORC_EINVAL;
    if (num_vertices > ORC_MAX_CAPACITY || vertex_capacity > ORC_MAX_CAPACITY)
        return ORC_EINVAL;
    if (block_slots != 0 &&
        (block_slots > 1024 || (block_slots & (block_slots - 1)) != 0))
        return ORC_EINVAL;
    for (uint64_t i = 0; i < num_edges; ++i)
        if ((uint64_t)src[i] >= num_vertices || (uint64_t)dst[i] >= num_vertices)
            return ORC_ERANGE;

    orc_graph* g = new (std::nothrow) orc_graph();
    if (!g) return ORC_ENOMEM;
    uint64_t want = num_vertices > vertex_capacity ? num_vertices : vertex_capacity;
    g->capacity = orc_next_pow2(want);
    g->active.assign(g->capacity, 0);
    g->adj.resize(g->capacity);
    for (uint64_t v = 0; v < num_vertices; ++v) g->active[v] = 1;

    // The initial graph is the first batch: a set of edges.
    for (uint64_t i = 0; i < num_edges; ++i) g->adj[src[i]].insert(dst[i]);

    uint64_t edges = 0, nonzero = 0;
    for (uint64_t v = 0; v < g->capacity; ++v) {
        edges += g->adj[v].size();
        nonzero += g->adj[v].empty() ? 0 : 1;
    }
    g->B = block_slots ? block_slots : orc_paper_block_slots(edges, nonzero);
    g->pool_bytes = pool_bytes;
    g->pool_blocks = pool_bytes ? pool_bytes / (4ull * g->B) : 0;
    if (g->pool_blocks && orc_blocks_in_use(g) > g->pool_blocks) {
        delete g;
        return ORC_ENOMEM;
    }
    *out = g;
    return ORC_OK;
}

extern "C" void orc_graph_destroy(orc_graph* g) { delete g; }

extern "C" int orc_apply_edge_ops(orc_graph* g, const uint8_t* op, const uint32_t* src,
                                  const uint32_t* dst, uint64_t n) {
    if (!g || (n && (!op || !src || !dst))) return ORC_EINVAL;
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t u = src[i], v = dst[i];
        if (!valid_vertex(g, u) || !valid_vertex(g, v)) continue;
        if (op[i] == 0) {
            if (g->adj[u].insert(v).second) attr_new(g, u, v);
        } else if (op[i] == 1) {
            if (g->adj[u].erase(v)) attr_drop(g, u, v);
        }
    }
    return ORC_OK;
}

extern "C" int orc_insert_edges(orc_graph* g, const uint32_t* src,
                                const uint32_t* dst, uint64_t n,
                                orc_stats* stats) {
    zero_stats(stats);
    if (!g || (n && (!src || !dst))) return ORC_EINVAL;
    orc_stats s = {0, 0, 0};
    std::set<std::pair<uint32_t, uint32_t>> seen;  // distinct valid pairs
    std::set<std::pair<uint32_t, uint32_t>> fresh; // of those, not yet edges
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t u = src[i], v = dst[i];
        if (!valid_vertex(g, u) || !valid_vertex(g, v)) {
            s.rejected++;
            continue;
        }
        if (!seen.insert({u, v}).second) {
            s.batch_duplicates++;
            continue;
        }
        if (g->adj[u].count(v) == 0) fresh.insert({u, v});
    }
    // All-or-nothing: the batch fits only if the pool can hold every
    // adjacency after it.
    if (g->pool_blocks) {
        uint64_t in_use = orc_blocks_in_use(g);
        uint64_t after = in_use;
        uint32_t cur = 0;
        uint64_t run = 0;
        bool have = false;
        for (const auto& e : fresh) { // fresh is ordered by source
            if (have && e.first != cur) {
                uint64_t d = g->adj[cur].size();
                after += blocks_for(g, d + run) - blocks_for(g, d);
                run = 0;
            }
            cur = e.first;
            have = true;
            run++;
        }
        if (have) {
            uint64_t d = g->adj[cur].size();
            after += blocks_for(g, d + run) - blocks_for(g, d);
        }
        if (after > g->pool_blocks) return ORC_ENOMEM;
    }
    for (const auto& e : fresh) {
        g->adj[e.first].insert(e.second);
        attr_new(g, e.first, e.second);
    }
    s.applied = fresh.size();
    if (stats) *stats = s;
    return ORC_OK;
}

extern "C" int orc_delete_edges(orc_graph* g, const uint32_t* src,
                                const uint32_t* dst, uint64_t n,
                                orc_stats* stats) {
    zero_stats(stats);
    if (!g || (n && (!src || !dst))) return ORC_EINVAL;
    orc_stats s = {0, 0, 0};
    std::set<std::pair<uint32_t, uint32_t>> seen;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t u = src[i], v = dst[i];
        if (!valid_vertex(g, u) || !valid_vertex(g, v)) {
            s.rejected++;
            continue;
        }
        if (!seen.insert({u, v}).second) {
            s.batch_duplicates++;
            continue;
        }
        // Sec. 4.5.2: a matching entry is removed; an absent one is a no-op.
        const uint64_t e = g->adj[u].erase(v);
        if (e) attr_drop(g, u, v);
        s.applied += e;
    }
    if (stats) *stats = s;
    return ORC_OK;
}

extern "C" int orc_insert_vertices(orc_graph* g, const uint32_t* ids,
                                   uint64_t n, orc_stats* stats) {
    zero_stats(stats);
    if (!g || (n && !ids)) return ORC_EINVAL;
    orc_stats s = {0, 0, 0};
    std::set<uint32_t> seen;
    uint64_t need = g->capacity;
    for (uint64_t i = 0; i < n; ++i) {
        if ((uint64_t)ids[i] >= ORC_MAX_CAPACITY) continue;
        if ((uint64_t)ids[i] + 1 > need) need = ids[i] + 1ull;
    }
    // Sec. 4.4: when the dictionary is full it is replaced by one of twice
    // the size, again a power of two.
    uint64_t cap = orc_next_pow2(need);
    if (cap > g->capacity) {
        g->active.resize(cap, 0);
        g->adj.resize(cap);
        g->capacity = cap;
    }
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t x = ids[i];
        if ((uint64_t)x >= ORC_MAX_CAPACITY) {
            s.rejected++;
            continue;
        }
        if (!seen.insert(x).second) {
            s.batch_duplicates++;
            continue;
        }
        if (!g->active[x]) {
            g->active[x] = 1; // an inactive vertex always has no edges
            s.applied++;
        }
    }
    if (stats) *stats = s;
    return ORC_OK;
}

extern "C" int orc_delete_vertices(orc_graph* g, const uint32_t* ids,
                                   uint64_t n, orc_stats* stats) {
    zero_stats(stats);
    if (!g || (n && !ids)) return ORC_EINVAL;
    orc_stats s = {0, 0, 0};
    std::set<uint32_t> seen, gone;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t x = ids[i];
        if ((uint64_t)x >= g->capacity) {
            s.rejected++;
            continue;
        }
        if (!seen.insert(x).second) {
            s.batch_duplicates++;
            continue;
        }
        if (g->active[x]) gone.insert(x);
    }
    // A deleted vertex loses its outgoing and its incoming edges.
    for (uint32_t x : gone) {
        for (uint32_t v : g->adj[x]) attr_drop(g, x, v);
        g->adj[x].clear();
    }
    for (uint64_t u = 0; u < g->capacity; ++u) {
        std::set<uint32_t>& a = g->adj[u];
        for (auto it = a.begin(); it != a.end();) {
            if (gone.count(*it)) {
                attr_drop(g, (uint32_t)u, *it);
                it = a.erase(it);
            } else {
                it = std::next(it);
            }
        }
    }
    for (uint32_t x : gone) g->active[x] = 0;
    s.applied = gone.size();
    if (stats) *stats = s;
    return ORC_OK;
}

extern "C" int orc_edge_exists(const orc_graph* g, const uint32_t* src,
                               const uint32_t* dst, uint64_t n, uint8_t* out) {
    if (!g || (n && (!src || !dst || !out))) return ORC_EINVAL;
    for (uint64_t i = 0; i < n; ++i)
        out[i] = (valid_vertex(g, src[i]) && g->adj[src[i]].count(dst[i])) ? 1 : 0;
    return ORC_OK;
}

extern "C" int orc_get_adjacency(const orc_graph* g, uint32_t v, uint32_t* out,
                                 uint64_t out_capacity, uint64_t* degree) {
    if (!g || !degree) return ORC_EINVAL;
    *degree = 0;
    if ((uint64_t)v >= g->capacity) return ORC_ERANGE;
    const std::set<uint32_t>& a = g->adj[v];
    *degree = a.size();
    if (out_capacity < a.size()) return ORC_ERANGE;
    if (a.size() && !out) return ORC_EINVAL;
    uint64_t i = 0;
    for (uint32_t x : a) out[i++] = x; // std::set iterates in ascending order
    return ORC_OK;
}

extern "C" int orc_dump_canonical(const orc_graph* g, uint64_t* offsets,
                                  uint32_t* dst, uint64_t dst_capacity,
                                  uint64_t* checksum) {
    if (!g) return ORC_EINVAL;
    uint64_t total = orc_num_edges(g);
    if (dst && dst_capacity < total) return ORC_ERANGE;
    uint64_t h = 0, pos = 0;
    for (uint64_t u = 0; u < g->capacity; ++u) {
        if (offsets) offsets[u] = pos;
        for (uint32_t v : g->adj[u]) {
            if (dst) dst[pos] = v;
            pos++;
            h += orc_mix64((u << 32) | (uint64_t)v);
        }
    }
    if (offsets) offsets[g->capacity] = pos;
    if (checksum) *checksum = h;
    return ORC_OK;
}

extern "C" uint64_t orc_capacity(const orc_graph* g) { return g->capacity; }

extern "C" uint64_t orc_num_edges(const orc_graph* g) {
    uint64_t total = 0;
    for (uint64_t v = 0; v < g->capacity; ++v) total += g->adj[v].size();
    return total;
}

extern "C" uint32_t orc_block_slots(const orc_graph* g) { return g->B; }
extern "C" uint64_t orc_pool_blocks(const orc_graph* g) { return g->pool_blocks; }

extern "C" int orc_is_active(const orc_graph* g, uint32_t v) {
    return (uint64_t)v < g->capacity && g->active[v] ? 1 : 0;
}

extern "C" uint64_t orc_degree(const orc_graph* g, uint32_t v) {
    return (uint64_t)v < g->capacity ? g->adj[v].size() : 0;
}

extern "C" int orc_set_attr_words(orc_graph* g, uint32_t words) {
    if (!g || g->A != 0 || words > 8) return ORC_EINVAL;
    g->A = words;
    for (uint64_t u = 0; u < g->capacity; ++u)
        for (uint32_t v : g->adj[u]) attr_new(g, (uint32_t)u, v);
    return ORC_OK;
}

extern "C" uint32_t orc_attr_words(const orc_graph* g) { return g->A; }

extern "C" int orc_set_edge_attrs(orc_graph* g, const uint32_t* src, const uint32_t* dst,
                                  const uint32_t* vals, uint64_t n, orc_stats* stats) {
    zero_stats(stats);
    if (!g || g->A == 0 || (n && (!src || !dst || !vals))) return ORC_EINVAL;
    orc_stats s = {0, 0, 0};
    std::set<std::pair<uint32_t, uint32_t>> seen;
    // one pair at a time in batch order: a later row of the same pair
    // overwrites an earlier one
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t u = src[i], v = dst[i];
        if (!valid_vertex(g, u) || !valid_vertex(g, v)) {
            s.rejected++;
            continue;
        }
        const bool first = seen.insert({u, v}).second;
        if (!first) s.batch_duplicates++;
        if (!g->adj[u].count(v)) continue;
        if (first) s.applied++;
        std::vector<uint32_t>& a = g->attr[pair_key(u, v)];
        for (uint32_t k = 0; k < g->A; ++k) a[k] = vals[i * g->A + k];
    }
    if (stats) *stats = s;
    return ORC_OK;
}

extern "C" int orc_get_edge_attrs(const orc_graph* g, const uint32_t* src, const uint32_t* dst,
                                  uint64_t n, uint8_t* found, uint32_t* vals) {
    if (!g || g->A == 0 || (n && (!src || !dst || !found || !vals))) return ORC_EINVAL;
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t u = src[i], v = dst[i];
        const bool here = valid_vertex(g, u) && g->adj[u].count(v);
        found[i] = here ? 1 : 0;
        for (uint32_t k = 0; k < g->A; ++k)
            vals[i * g->A + k] = here ? g->attr.at(pair_key(u, v))[k] : 0u;
    }
    return ORC_OK;
}

extern "C" int orc_set_block_slots(orc_graph* g, uint32_t block_slots) {
    // Sec. 6 (future scope): the edge block size may change over the life of
    // the graph; the edges stay, only the block accounting follows the new
    // size.  The pool keeps its byte budget.
    if (!g || block_slots == 0 || block_slots > 1024 || (block_slots & (block_slots - 1)) != 0)
        return ORC_EINVAL;
    const uint32_t old_b = g->B;
    const uint64_t old_blocks = g->pool_blocks;
    g->B = block_slots;
    g->pool_blocks = g->pool_bytes ? g->pool_bytes / (4ull * g->B) : 0;
    if (g->pool_blocks && orc_blocks_in_use(g) > g->pool_blocks) {
        g->B = old_b;
        g->pool_blocks = old_blocks;
        return ORC_ENOMEM;
    }
    return ORC_OK;
}

extern "C" uint32_t orc_adapted_block_slots(const orc_graph* g) {
    // the initialization rule of Sec. 4.3 applied to the graph as it is now
    // (Sec. 6: the average degree changes across batches)
    uint64_t edges = 0, nonzero = 0;
    for (uint64_t v = 0; v < g->capacity; ++v) {
        edges += g->adj[v].size();
        nonzero += g->adj[v].empty() ? 0 : 1;
    }
    return orc_paper_block_slots(edges, nonzero);
}
