// gv_build.hip -- bulk build (graph_init), canonical dump, adjacency read,
// structural audit.
//
// Bulk build (Sec. 4.3 initialisation and the "bulk" batch of Sec. 5.2): the
// COO list is sorted by (src, dst) with the radix sort, duplicates are
// dropped, each vertex's degree is read off the run boundaries, and one scan
// over the dictionary assigns every vertex a contiguous run of blocks and, if
// it needs two or more blocks, a power-of-two directory segment.  The pool is
// then exactly a CSR layout padded to whole blocks, written with coalesced
// stores.
#include <algorithm>

#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

__device__ __forceinline__ uint64_t tidx() { return (uint64_t)blockIdx.x * kThreads + threadIdx.x; }
__device__ __forceinline__ uint32_t gwave() {
    return (uint32_t)(((uint64_t)blockIdx.x * kThreads + threadIdx.x) >> 6);
}

void read_counters(gv_graph* g) {
    hip_check(hipMemcpyAsync(g->hctr, g->v.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost,
                             g->ctx.stream),
              "hipMemcpyAsync counters");
    hip_check(hipStreamSynchronize(g->ctx.stream), "hipStreamSynchronize");
    g->edge_bound_host = g->hctr->live_edges;
}

// Sort n keys of `bits` bits (n >= 2) with the one-sweep radix sort; `state`
// holds os_words(n, bits) words.  Synchronous: raises GV_EDEVICE if a
// look-back did not complete.  Returns true if the result is in k1.
static bool sort_keys(gv_graph* g, uint64_t* k0, uint64_t* k1, uint64_t n, int bits,
                      uint32_t* state) {
    Ctx& c = g->ctx;
    DevCounters* ctr = g->v.ctr;
    zero_words(c, state, os_zero_words(n, bits));
    set_u32(g, &ctr->sort_n, (uint32_t)n);
    set_u32(g, &ctr->sort_err, 0);
    const bool flip = onesweep<uint64_t, false>(c, k0, k1, nullptr, nullptr, &ctr->sort_n, n,
                                                bits, state, &ctr->sort_err);
    read_counters(g);
    if (g->hctr->sort_err) fail(GV_EDEVICE, "sort look-back did not complete");
    return flip;
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(kThreads) void k_init_vt(GraphView g, uint64_t n_active) {
    const uint64_t v = tidx();
    if (v < g.n_cap) g.vt[v] = VRec{0u, 0u, kNoDir, 0u};
    const uint64_t words = (g.n_cap + 31) / 32;
    if (v < words) {
        const uint64_t lo = v * 32;
        uint32_t w = 0;
        if (n_active >= lo + 32) w = 0xffffffffu;
        else if (n_active > lo) w = (1u << (n_active - lo)) - 1u;
        g.active[v] = w;
    }
}

// keys of the initial edges; an id out of range raises a flag (a plain store,
// taken only on error) that the host checks before any id is used as an index
__global__ __launch_bounds__(kThreads) void k_init_pack(GraphView g, const uint32_t* src,
                                                        const uint32_t* dst, uint64_t m,
                                                        uint64_t n, uint64_t* keys) {
    const uint64_t i = tidx();
    if (i >= m) return;
    const uint32_t s = src[i], d = dst[i];
    if ((uint64_t)s >= n || (uint64_t)d >= n) g.ctr->vany = 1;
    keys[i] = ((uint64_t)s << g.L) | d;
}

// first occurrence of a key in the low half, first occurrence of a source in
// the high half: one scan yields the unique positions, the number of distinct
// edges and the number of vertices of non-zero degree
struct FirstIn {
    const uint64_t* keys;
    uint64_t m;
    uint32_t L;
    __device__ unsigned long long operator()(uint64_t i) const {
        if (i >= m) return 0ull;
        if (i == 0) return 1ull | (1ull << 32);
        const uint64_t a = keys[i - 1], b = keys[i];
        return (a != b ? 1ull : 0ull) | ((a >> L) != (b >> L) ? (1ull << 32) : 0ull);
    }
};

struct LowOut {
    uint32_t* a;
    __device__ void operator()(uint64_t i, unsigned long long v) const { a[i] = (uint32_t)v; }
};

__global__ __launch_bounds__(kThreads) void k_init_unique(const uint64_t* keys, const uint32_t* pos,
                                                          uint64_t m, uint64_t* ukeys) {
    const uint64_t i = tidx();
    if (i < m && (i == 0 || keys[i] != keys[i - 1])) ukeys[pos[i]] = keys[i];
}

// run starts: first position of each source in the unique list -> aux
__global__ __launch_bounds__(kThreads) void k_init_runs(GraphView g, const uint64_t* ukeys,
                                                        uint64_t mu) {
    const uint64_t p = tidx();
    if (p >= mu) return;
    const uint32_t v = (uint32_t)(ukeys[p] >> g.L);
    if (p == 0 || (uint32_t)(ukeys[p - 1] >> g.L) != v) g.vt[v].aux = (uint32_t)p;
}

__global__ __launch_bounds__(kThreads) void k_init_deg(GraphView g, const uint64_t* ukeys,
                                                       uint64_t mu) {
    const uint64_t p = tidx();
    if (p >= mu) return;
    const uint32_t v = (uint32_t)(ukeys[p] >> g.L);
    if (p + 1 == mu || (uint32_t)(ukeys[p + 1] >> g.L) != v)
        g.vt[v].deg = (uint32_t)(p + 1) - g.vt[v].aux;
}

// per vertex: blocks in the low half, directory entries in the high half
struct LayoutIn {
    GraphView g;
    __device__ unsigned long long operator()(uint64_t v) const {
        if (v >= g.n_cap) return 0ull;
        const uint32_t nb = nblocks(g, g.vt[v].deg);
        const unsigned long long de = nb >= 2 ? (1ull << ceil_log2(nb)) : 0ull;
        return (unsigned long long)nb | (de << 32);
    }
};

__global__ __launch_bounds__(kThreads) void k_init_layout(GraphView g,
                                                          const unsigned long long* off) {
    const uint64_t v = tidx();
    if (v >= g.n_cap) return;
    VRec r = g.vt[v];
    const uint32_t nb = nblocks(g, r.deg);
    const uint32_t boff = (uint32_t)off[v];
    const uint32_t doff = (uint32_t)(off[v] >> 32);
    r.aux = 0;
    if (nb == 0) {
        r.dir = 0;
        r.dcls = kNoDir;
    } else if (nb == 1) {
        r.dir = boff;
        r.dcls = kNoDir;
    } else {
        r.dir = doff;
        r.dcls = ceil_log2(nb);
        for (uint32_t j = 0; j < nb; ++j) g.dir[(uint64_t)doff + j] = boff + j;
    }
    for (uint32_t j = 0; j < nb; ++j) g.bown[(uint64_t)boff + j] = make_uint2((uint32_t)v, j);
    g.vt[v] = r;
}

// scatter: edge p of the sorted unique list goes to slot (p - run start) of
// its vertex's contiguous blocks
__global__ __launch_bounds__(kThreads) void k_init_scatter(GraphView g, const uint64_t* ukeys,
                                                           const uint32_t* runstart,
                                                           const unsigned long long* off,
                                                           uint64_t mu) {
    const uint64_t p = tidx();
    if (p >= mu) return;
    const uint64_t k = ukeys[p];
    const uint32_t v = (uint32_t)(k >> g.L);
    const uint32_t s = (uint32_t)p - runstart[v];
    const uint64_t blk = (uint32_t)off[v] + (s >> g.log2B);
    const uint64_t a = (blk << g.log2B) + (s & (g.B - 1));
    g.pool[a] = (uint32_t)(k & ((1ull << g.L) - 1));
    attr_zero(g, a);
}

__global__ __launch_bounds__(kThreads) void k_save_runstart(GraphView g, uint32_t* runstart) {
    const uint64_t v = tidx();
    if (v < g.n_cap) runstart[v] = g.vt[v].aux;
}

__global__ void k_init_counters(GraphView g, unsigned long long blocks, unsigned long long dents,
                                unsigned long long edges) {
    DevCounters* c = g.ctr;
    c->live_edges = edges;
    c->free_cnt = 0;
    c->bump = blocks;
    c->dir_bump = dents;
    c->dir_live = dents;
    for (int k = 0; k < kMaxClass; ++k) {
        c->dfree_cnt[k] = 0;
        c->dreq[k] = 0;
    }
    c->err_batch = c->err_sticky = 0;
}

static uint32_t paper_block_rule(uint64_t edges, uint64_t nonzero) {
    // Sec. 4.3: average degree of the non-zero-degree vertices of the first
    // batch, rounded up to a power of two and kept within [8, 64].
    if (edges == 0 || nonzero == 0) return 8;
    uint64_t avg = (edges + nonzero - 1) / nonzero;
    uint64_t b = 1;
    while (b < avg) b <<= 1;
    return (uint32_t)std::min<uint64_t>(64, std::max<uint64_t>(8, b));
}

void bulk_build(gv_graph* g, uint64_t n, const uint32_t* src, const uint32_t* dst, uint64_t m,
                const gv_config& cfg) {
    Ctx& c = g->ctx;
    GraphView& v = g->v;
    const uint64_t vgrid = div_up(std::max<uint64_t>(v.n_cap, (v.n_cap + 31) / 32), kThreads);
    c.launch("init_vt", k_init_vt, vgrid, kThreads, v, n);
    set_u32(g, &v.ctr->vany, 0);

    const int bits = 2 * (int)v.L;
    uint64_t mu = 0, nonzero = 0;
    struct Arr {
        uint64_t* k0;
        uint64_t* k1;
        uint32_t* pos;
        unsigned long long* part;
        uint32_t* state;
        unsigned long long* off;
        unsigned long long* part64;
        uint32_t* runstart;
    } A{};
    const uint64_t state_words = m > 1 ? os_words(m, bits) : 0;
    auto carve = [&](Carver& cv) {
        A.k0 = cv.take<uint64_t>(std::max<uint64_t>(m, 1));
        A.k1 = cv.take<uint64_t>(std::max<uint64_t>(m, 1));
        A.pos = cv.take<uint32_t>(m + 1);
        A.part = cv.take<unsigned long long>(scan_partials_needed(m + 1));
        A.state = cv.take<uint32_t>(std::max<uint64_t>(state_words, 1));
        A.off = cv.take<unsigned long long>(v.n_cap + 1);
        A.part64 = cv.take<unsigned long long>(scan_partials_needed(v.n_cap + 1));
        A.runstart = cv.take<uint32_t>(v.n_cap);
    };
    {
        Carver mz(nullptr);
        carve(mz);
        g->scratch.ensure(mz.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve(cv);
    }
    uint64_t* ukeys = nullptr;
    if (m > 0) {
        if (m >= kOsMaxKeys) fail(GV_EINVAL, "2^30 or more edges");
        const uint64_t grid = div_up(m, kThreads);
        c.launch("init_pack", k_init_pack, grid, kThreads, v, src, dst, m, n, A.k0);
        const bool flip = m > 1 && sort_keys(g, A.k0, A.k1, m, bits, A.state);
        uint64_t* keys = flip ? A.k1 : A.k0;
        ukeys = flip ? A.k0 : A.k1;
        scan_excl<unsigned long long>(c, FirstIn{keys, m, v.L}, LowOut{A.pos}, m + 1, A.part,
                                      &v.ctr->edges);
        read_counters(g);
        if (g->hctr->vany) fail(GV_ERANGE, "edge id >= num_vertices");
        mu = g->hctr->edges & 0xffffffffull;
        nonzero = g->hctr->edges >> 32;
        c.launch("init_unique", k_init_unique, grid, kThreads, (const uint64_t*)keys,
                 (const uint32_t*)A.pos, m, ukeys);
        const uint64_t ugrid = div_up(mu, kThreads);
        c.launch("init_runs", k_init_runs, ugrid, kThreads, v, (const uint64_t*)ukeys, mu);
        c.launch("init_deg", k_init_deg, ugrid, kThreads, v, (const uint64_t*)ukeys, mu);
    }
    uint32_t B = cfg.block_slots ? cfg.block_slots : paper_block_rule(mu, nonzero);
    v.B = B;
    v.log2B = log2_exact(B);

    c.launch("save_runstart", k_save_runstart, div_up(v.n_cap, kThreads), kThreads, v,
             A.runstart);
    scan_excl<unsigned long long>(c, LayoutIn{v}, ArrOut<unsigned long long>{A.off}, v.n_cap + 1,
                                  A.part64, &v.ctr->edges);
    read_counters(g);
    const uint64_t blocks = g->hctr->edges & 0xffffffffull;
    const uint64_t dents = g->hctr->edges >> 32;

    // pool and directory sizing
    uint64_t cap_blocks = cfg.pool_bytes ? cfg.pool_bytes / (4ull * B) : 2 * blocks + (1ull << 20);
    cap_blocks = std::min<uint64_t>(cap_blocks, 0xfffffff0ull);
    if (blocks > cap_blocks) fail(GV_ENOMEM, "pool too small for the initial graph");
    uint64_t dir_cap = cfg.directory_entries ? cfg.directory_entries
                                             : 4 * cap_blocks + (1ull << 20);
    dir_cap = std::min<uint64_t>(dir_cap, 0xfffffff0ull);
    if (dents > dir_cap) fail(GV_ENOMEM, "directory too small for the initial graph");
    hip_check(hipMalloc(&g->mem_pool, std::max<uint64_t>(cap_blocks * B * 4ull, 4)),
              "hipMalloc pool");
    hip_check(hipMalloc(&g->mem_free, std::max<uint64_t>(cap_blocks * 4ull, 4)),
              "hipMalloc free list");
    hip_check(hipMalloc(&g->mem_bown, std::max<uint64_t>(cap_blocks * 8ull, 8)),
              "hipMalloc block owners");
    if (v.A)
        hip_check(hipMalloc(&g->mem_apool, cap_blocks * B * 4ull * v.A), "hipMalloc attributes");
    hip_check(hipMalloc(&g->mem_dir, std::max<uint64_t>(dir_cap * 4ull, 4)), "hipMalloc dir");
    uint64_t dfree_total = 0;
    for (int k = 0; k < kMaxClass; ++k) {
        v.dfree_base[k] = dfree_total;
        dfree_total += (k == 0) ? 0 : (dir_cap >> k);
    }
    hip_check(hipMalloc(&g->mem_dfree, std::max<uint64_t>(dfree_total * 4ull, 4)),
              "hipMalloc dir free");
    v.pool = (uint32_t*)g->mem_pool;
    v.free_stack = (uint32_t*)g->mem_free;
    v.bown = (uint2*)g->mem_bown;
    v.apool = (uint32_t*)g->mem_apool;
    v.dir = (uint32_t*)g->mem_dir;
    v.dfree = (uint32_t*)g->mem_dfree;
    v.cap_blocks = cap_blocks;
    v.dir_cap = dir_cap;
    g->item_slots = cap_blocks * B;

    c.launch("init_layout", k_init_layout, div_up(v.n_cap, kThreads), kThreads, v,
             (const unsigned long long*)A.off);
    if (mu > 0)
        c.launch("init_scatter", k_init_scatter, div_up(mu, kThreads), kThreads, v,
                 (const uint64_t*)ukeys, (const uint32_t*)A.runstart,
                 (const unsigned long long*)A.off, mu);
    c.launch("init_counters", k_init_counters, 1, 1, v, (unsigned long long)blocks,
             (unsigned long long)dents, (unsigned long long)mu);
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    g->edge_bound_host = mu;
}

// ------------------------------------------------------------------ dump
struct DegIn {
    GraphView g;
    __device__ unsigned long long operator()(uint64_t v) const {
        return v < g.n_cap ? g.vt[v].deg : 0ull;
    }
};

// one wave per vertex: checksum of its edges and (optionally) its keys at
// its CSR offset
__global__ __launch_bounds__(kThreads) void k_dump_gather(GraphView g,
                                                          const unsigned long long* offs,
                                                          uint64_t* keys) {
    const uint32_t lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    unsigned long long h = 0;
    for (uint64_t u = gwave(); u < g.n_cap; u += nw) {
        const VRec r = g.vt[u];
        for (uint32_t s = lane; s < r.deg; s += 64) {
            const uint32_t x = g.pool[slot_addr(g, r, s)];
            h += mix64((u << 32) | x);
            if (keys) keys[offs[u] + s] = (u << g.L) | x;
        }
    }
    h = wave_sum(h);
    if (lane == 0 && h) atomicAdd(&g.ctr->checksum, h);
}

__global__ __launch_bounds__(kThreads) void k_dump_extract(const uint64_t* keys, uint64_t e,
                                                           uint32_t L, uint32_t* dst) {
    const uint64_t i = tidx();
    if (i < e) dst[i] = (uint32_t)(keys[i] & ((1ull << L) - 1));
}

void dump(gv_graph* g, uint64_t* offsets, uint32_t* dst, uint64_t cap, uint64_t* checksum,
          uint64_t* edges) {
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    // offsets go to the caller's array, or to scratch when only the count and
    // checksum are wanted
    unsigned long long* offs = (unsigned long long*)offsets;
    unsigned long long* part = nullptr;
    {
        auto carve = [&](Carver& cv) {
            part = cv.take<unsigned long long>(scan_partials_needed(v.n_cap + 1));
            if (!offsets) offs = cv.take<unsigned long long>(v.n_cap + 1);
        };
        Carver mz(nullptr);
        carve(mz);
        g->scratch.ensure(mz.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve(cv);
    }
    scan_excl<unsigned long long>(c, DegIn{v}, ArrOut<unsigned long long>{offs}, v.n_cap + 1, part,
                                  &v.ctr->edges);
    set_u64(g, &v.ctr->checksum, 0);
    const uint64_t wgrid = std::min<uint64_t>(div_up(v.n_cap, kWaves), 4096);
    c.launch("dump_checksum", k_dump_gather, wgrid, kThreads, v,
             (const unsigned long long*)offs, (uint64_t*)nullptr);
    read_counters(g);
    const uint64_t e = g->hctr->edges;
    *edges = e;
    *checksum = g->hctr->checksum;
    if (!dst || !offsets) return;
    if (cap < e) fail(GV_ERANGE, "dump buffer too small");
    if (e == 0) return;
    // keys (u << L | x) at CSR positions; one sort then orders the
    // destinations of every vertex
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t* state = nullptr;
    const int bits = 2 * (int)v.L;
    auto carve2 = [&](Carver& cv) {
        k0 = cv.take<uint64_t>(e);
        k1 = cv.take<uint64_t>(e);
        state = cv.take<uint32_t>(os_words(std::max<uint64_t>(e, 2), bits));
    };
    {
        Carver mz(nullptr);
        carve2(mz);
        g->scratch.ensure(mz.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve2(cv);
    }
    c.launch("dump_gather", k_dump_gather, wgrid, kThreads, v, (const unsigned long long*)offs,
             k0);
    const bool flip = e > 1 && sort_keys(g, k0, k1, e, bits, state);
    c.launch("dump_extract", k_dump_extract, div_up(e, kThreads), kThreads,
             (const uint64_t*)(flip ? k1 : k0), e, v.L, dst);
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
}

// ------------------------------------------------------------------ adjacency
// an adjacency of at most one tile: gathered and sorted in LDS by one workgroup
__global__ __launch_bounds__(kOsThreads) void k_adj_tile(GraphView g, uint32_t u, int passes,
                                                         uint32_t* out) {
    __shared__ TileSortLds lds;
    const VRec r = g.vt[u];
    uint64_t key[kOsRounds];
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + threadIdx.x;
        key[j] = i < r.deg ? g.pool[slot_addr(g, r, (uint32_t)i)] : ~0ull;
    }
    tile_sort(key, r.deg, passes, ~0ull, lds);
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + threadIdx.x;
        if (i < r.deg) out[i] = (uint32_t)key[j];
    }
}

// a longer one: destinations as 64-bit keys for the one-sweep sort, and back
__global__ __launch_bounds__(kThreads) void k_adj_gather64(GraphView g, uint32_t u,
                                                           uint64_t* keys) {
    const VRec r = g.vt[u];
    for (uint64_t s = tidx(); s < r.deg; s += (uint64_t)gridDim.x * kThreads)
        keys[s] = g.pool[slot_addr(g, r, (uint32_t)s)];
}

__global__ __launch_bounds__(kThreads) void k_adj_low(const uint64_t* keys, uint64_t n,
                                                      uint32_t* out) {
    const uint64_t i = tidx();
    if (i < n) out[i] = (uint32_t)keys[i];
}

__global__ __launch_bounds__(kThreads) void k_copy_u32(const uint32_t* a, uint32_t* b, uint64_t n) {
    const uint64_t i = tidx();
    if (i < n) b[i] = a[i];
}

void adjacency(gv_graph* g, uint32_t u, uint32_t* out, uint64_t cap, uint64_t* degree) {
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    *degree = 0;
    if ((uint64_t)u >= v.n_cap) fail(GV_ERANGE, "vertex id >= capacity");
    VRec r;
    hip_check(hipMemcpyAsync(&r, v.vt + u, sizeof(VRec), hipMemcpyDeviceToHost, c.stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    *degree = r.deg;
    if (cap < r.deg) fail(GV_ERANGE, "adjacency buffer too small");
    if (r.deg == 0) return;
    if (!out) fail(GV_EINVAL, "null output");
    const uint64_t d = r.deg;
    const int bits = std::max<int>((int)v.L, 1);
    if (d <= kOsTile) {
        // one kernel: gather and sort in LDS
        c.launch("adj_sort", k_adj_tile, 1, kOsThreads, v, u, os_passes(bits), out);
        hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
        return;
    }
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t* state = nullptr;
    auto carve = [&](Carver& cv) {
        k0 = cv.take<uint64_t>(d);
        k1 = cv.take<uint64_t>(d);
        state = cv.take<uint32_t>(os_words(d, bits));
    };
    {
        Carver mz(nullptr);
        carve(mz);
        g->scratch.ensure(mz.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve(cv);
    }
    c.launch("adj_gather", k_adj_gather64, std::min<uint64_t>(div_up(d, kThreads), 1024),
             kThreads, v, u, k0);
    const bool flip = sort_keys(g, k0, k1, d, bits, state);  // synchronous
    c.launch("adj_copy", k_adj_low, div_up(d, kThreads), kThreads,
             (const uint64_t*)(flip ? k1 : k0), d, out);
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
}

// ------------------------------------------------------------------ audit
__global__ __launch_bounds__(kThreads) void k_zero_u32(uint32_t* a, uint64_t n) {
    const uint64_t i = tidx();
    if (i < n) a[i] = 0;
}

// one wave per vertex: owned blocks are counted, slots and records checked
__global__ __launch_bounds__(kThreads) void k_audit_vertices(GraphView g, uint32_t* seen) {
    const uint32_t lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    const unsigned long long bump = g.ctr->bump;
    unsigned long long bad = 0;
    for (uint64_t u = gwave(); u < g.n_cap; u += nw) {
        const VRec r = g.vt[u];
        const bool act = is_active(g, u);
        if (lane == 0 && g.vlost[u] != 0u) bad++;  // vertex-delete scratch left set
        if (!act) {
            if (lane == 0 && (r.deg != 0 || r.dcls != kNoDir)) bad++;
            continue;
        }
        const uint32_t nb = nblocks(g, r.deg);
        if (r.dcls != kNoDir) {
            if (r.dcls >= kMaxClass || (1ull << r.dcls) < nb ||
                (uint64_t)r.dir + (1ull << r.dcls) > g.dir_cap) {
                if (lane == 0) bad++;
                continue;
            }
        } else if (nb > 1) {
            if (lane == 0) bad++;
            continue;
        }
        for (uint32_t j = lane; j < nb; j += 64) {
            const uint32_t id = block_of(g, r, j);
            if (id >= bump) {
                bad++;
            } else {
                atomicAdd(&seen[id], 1u);
                const uint2 ow = g.bown[id];  // the owner record names this vertex and index
                if (ow.x != (uint32_t)u || ow.y != j) bad++;
            }
        }
        for (uint32_t s = lane; s < r.deg; s += 64) {
            const uint32_t id = block_of(g, r, s >> g.log2B);
            if (id >= bump) continue;
            const uint32_t x = g.pool[((uint64_t)id << g.log2B) + (s & (g.B - 1))];
            if (x == kTomb || !is_active(g, x)) bad++;
        }
    }
    bad = wave_sum(bad);
    if (lane == 0 && bad) atomicAdd(&g.ctr->violations, bad);
}

__global__ __launch_bounds__(kThreads) void k_audit_free(GraphView g, uint32_t* seen) {
    const uint64_t i = tidx();
    if (i >= g.ctr->free_cnt) return;
    const uint32_t id = g.free_stack[i];
    if (id >= g.ctr->bump) atomicAdd(&g.ctr->violations, 1ull);
    else atomicAdd(&seen[id], 1u);
}

__global__ __launch_bounds__(kThreads) void k_audit_seen(GraphView g, const uint32_t* seen,
                                                         uint64_t n) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t i = tidx();
    unsigned long long bad = (i < n && seen[i] != 1u) ? 1ull : 0ull;
    bad = block_sum(bad, lds);
    if (threadIdx.x == 0 && bad) atomicAdd(&g.ctr->violations, bad);
}

uint64_t audit(gv_graph* g) {
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    read_counters(g);
    const uint64_t bump = g->hctr->bump;
    const uint64_t nfree = g->hctr->free_cnt;
    uint64_t bad = 0;
    if (nfree > bump || bump > v.cap_blocks) bad++;
    uint32_t* seen = nullptr;
    {
        Carver mz(nullptr);
        mz.take<uint32_t>(std::max<uint64_t>(bump, 1));
        g->scratch.ensure(mz.used, c.stream);
        Carver cv(g->scratch.ptr);
        seen = cv.take<uint32_t>(std::max<uint64_t>(bump, 1));
    }
    set_u64(g, &v.ctr->violations, 0);
    c.launch("audit_zero", k_zero_u32, div_up(std::max<uint64_t>(bump, 1), kThreads), kThreads,
             seen, bump);
    c.launch("audit_vertices", k_audit_vertices,
             std::min<uint64_t>(div_up(v.n_cap, kWaves), 4096), kThreads, v, seen);
    if (nfree)
        c.launch("audit_free", k_audit_free, div_up(nfree, kThreads), kThreads, v, seen);
    if (bump)
        c.launch("audit_seen", k_audit_seen, div_up(bump, kThreads), kThreads, v,
                 (const uint32_t*)seen, bump);
    read_counters(g);
    return bad + g->hctr->violations;
}

}  // namespace gv

namespace gv {

// ------------------------------------------------------------------ block size
// blocks the adjacencies would hold with 2^lb slots per block (low half) and
// vertices of non-zero degree (high half), one atomic per workgroup
__global__ __launch_bounds__(kThreads) void k_layout_count(GraphView g, uint32_t lb,
                                                           unsigned long long* out) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t v = tidx();
    unsigned long long blocks = 0, nz = 0;
    if (v < g.n_cap && is_active(g, v)) {
        const uint32_t d = g.vt[v].deg;
        blocks = ((uint64_t)d + (1ull << lb) - 1) >> lb;
        nz = d > 0;
    }
    blocks = block_sum(blocks, lds);
    nz = block_sum(nz, lds);
    if (threadIdx.x == 0 && (blocks | nz)) atomicAdd(out, blocks | (nz << 32));
}

// source of every dumped edge: the vertex whose CSR range holds it
__global__ __launch_bounds__(kThreads) void k_layout_src(const unsigned long long* offs,
                                                         uint64_t ncap, uint64_t m,
                                                         uint32_t* src) {
    const uint64_t i = tidx();
    if (i >= m) return;
    uint64_t lo = 0, hi = ncap;  // last v with offs[v] <= i
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (offs[mid] <= i) lo = mid;
        else hi = mid;
    }
    src[i] = (uint32_t)lo;
}

namespace {

// (blocks with 2^lb slots, vertices of non-zero degree)
std::pair<uint64_t, uint64_t> layout_count(gv_graph* g, uint32_t lb) {
    const GraphView& v = g->v;
    set_u64(g, &v.ctr->checksum, 0);
    g->ctx.launch("relayout", k_layout_count, div_up(v.n_cap, kThreads), kThreads, v, lb,
                  &v.ctr->checksum);
    read_counters(g);
    const unsigned long long x = g->hctr->checksum;
    return {x & 0xffffffffull, x >> 32};
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) hipFree(p);
    }
    template <typename T>
    T* get(size_t count) {
        hip_check(hipMalloc(&p, std::max<size_t>(count * sizeof(T), 8)), "hipMalloc relayout");
        return (T*)p;
    }
};

}  // namespace

uint32_t adapted_block_slots(gv_graph* g) {
    read_counters(g);
    const uint64_t edges = g->hctr->live_edges;
    const uint64_t nonzero = layout_count(g, 0).second;
    return paper_block_rule(edges, nonzero);
}

// The same edges (and attribute words) in blocks of block_slots slots: dump,
// rebuild with the pool's byte budget, restore the activity bitmap, write the
// words back.  Checks first that the new layout fits, so that a graph that
// would not fit stays as it is (GV_ENOMEM).
void relayout(gv_graph* g, uint32_t block_slots) {
    Ctx& c = g->ctx;
    GraphView& v = g->v;
    if (block_slots == v.B) return;
    read_counters(g);
    // a rebuild clears the error words: report a pending one first
    if (g->hctr->err_sticky) fail((int)g->hctr->err_sticky, "an earlier batch failed");
    const uint64_t m = g->hctr->live_edges;
    if (m >= kOsMaxKeys) fail(GV_EINVAL, "2^30 or more edges");
    const uint64_t budget = v.cap_blocks * v.B * 4ull;
    const uint64_t cap_new = std::min<uint64_t>(budget / (4ull * block_slots), 0xfffffff0ull);
    if (layout_count(g, log2_exact(block_slots)).first > cap_new)
        fail(GV_ENOMEM, "the graph does not fit the pool with that block size");
    const uint64_t words = (v.n_cap + 31) / 32;
    DevBuf b_offs, b_dst, b_src, b_attr, b_found, b_act;
    auto* offs = b_offs.get<uint64_t>(v.n_cap + 1);
    auto* dst = b_dst.get<uint32_t>(m);
    auto* src = b_src.get<uint32_t>(m);
    auto* act = b_act.get<uint32_t>(words);
    uint32_t* attr = v.A ? b_attr.get<uint32_t>(m * v.A) : nullptr;
    uint64_t ck = 0, e = 0;
    dump(g, offs, dst, m, &ck, &e);
    if (e != m) fail(GV_EDEVICE, "edge count changed during a relayout");
    if (m)
        c.launch("relayout", k_layout_src, div_up(m, kThreads), kThreads,
                 (const unsigned long long*)offs, (uint64_t)v.n_cap, m, src);
    if (attr && m) edge_attrs(g, src, dst, m, b_found.get<uint8_t>(m), attr, nullptr);
    hip_check(hipMemcpyAsync(act, v.active, words * 4, hipMemcpyDeviceToDevice, c.stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    // from here the old layout is gone: a failure leaves the graph unusable
    g->dead = true;
    for (void** p : {&g->mem_pool, &g->mem_free, &g->mem_dir, &g->mem_dfree, &g->mem_bown,
                     &g->mem_apool}) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    gv_config cfg{};
    cfg.block_slots = block_slots;
    cfg.pool_bytes = budget;
    cfg.vertex_capacity = v.n_cap;
    cfg.edge_attr_words = v.A;
    bulk_build(g, v.n_cap, src, dst, m, cfg);
    hip_check(hipMemcpyAsync(v.active, act, words * 4, hipMemcpyDeviceToDevice, c.stream),
              "hipMemcpyAsync");
    if (attr && m) edge_attrs(g, src, dst, m, nullptr, nullptr, attr);
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    g->dead = false;
    ++g->table_gen;  // recorded plans hold the old layout
}

}  // namespace gv
