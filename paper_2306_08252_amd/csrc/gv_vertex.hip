// gv_vertex.hip -- batched vertex insertion and deletion (Sec. 4.4).
//
// Insert: ids are sorted and deduplicated; when the largest id does not fit,
// the dictionary is replaced by one of the next power-of-two capacity (copy
// kernel, then the old one is freed); inactive ids are switched on.
//
// Delete: the deleted set is marked in a bitmap.  Every adjacency is cut
// into sweep units of 256 slots; a count pass finds the slots each unit keeps
// (none for a deleted source, else those whose destination is not deleted),
// a scan over units places them, the kept slots of every vertex that loses
// any are gathered into a staging buffer and written back in order from
// slot 0, emptied blocks go on the free list (a scan over vertices places
// them), and the deleted vertices are switched off with their directory
// segments returned.  All sizes are bounds known on the host, so the path has
// no host round trip.
#include <algorithm>

#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

__device__ __forceinline__ uint64_t vt_tidx() {
    return (uint64_t)blockIdx.x * kThreads + threadIdx.x;
}

constexpr uint32_t kMaxId = 0x7fffffffu;

__device__ __forceinline__ bool bit_of(const uint32_t* bm, uint32_t x) {
    return (bm[x >> 5] >> (x & 31)) & 1u;
}

__global__ __launch_bounds__(kThreads) void k_vmax(const uint32_t* ids, uint64_t n,
                                                   DevCounters* ctr) {
    const uint64_t i = vt_tidx();
    uint32_t m = 0, any = 0;
    if (i < n && ids[i] <= kMaxId) {
        m = ids[i];
        any = 1;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
        any |= (uint32_t)__shfl_xor((int)any, o, 64);
    }
    if (lane_id() == 0 && any) {
        atomicMax(&ctr->vmax, m);
        ctr->vany = 1;
    }
}

// ids that a fixed table cannot hold raise a sticky GV_ERANGE (plain stores
// of one value)
__global__ __launch_bounds__(kThreads) void k_vfit(GraphView g, const uint32_t* ids, uint64_t n) {
    const uint64_t i = vt_tidx();
    if (i < n && ids[i] <= kMaxId && (uint64_t)ids[i] >= g.n_cap) {
        g.ctr->err_sticky = GV_ERANGE;
        g.ctr->err_batch = GV_ERANGE;
    }
}

__global__ __launch_bounds__(kThreads) void k_vcopy_ids(const uint32_t* ids, uint64_t n,
                                                        uint32_t* out) {
    const uint64_t i = vt_tidx();
    if (i < n) out[i] = ids[i];
}

__global__ __launch_bounds__(kThreads) void k_vzero(uint32_t* a, uint64_t n) {
    const uint64_t i = vt_tidx();
    if (i < n) a[i] = 0;
}

__global__ __launch_bounds__(kThreads) void k_grow_table(const VRec* vt, const uint32_t* act,
                                                         uint64_t old_cap, VRec* vt2,
                                                         uint32_t* act2, uint64_t new_cap) {
    const uint64_t v = vt_tidx();
    if (v < new_cap) vt2[v] = v < old_cap ? vt[v] : VRec{0u, 0u, kNoDir, 0u};
    const uint64_t ow = (old_cap + 31) / 32, nw = (new_cap + 31) / 32;
    if (v < nw) {
        uint32_t w = v < ow ? act[v] : 0u;
        if (v == ow - 1 && (old_cap & 31)) w &= (1u << (old_cap & 31)) - 1u;
        act2[v] = w;
    }
}

__global__ void k_vreset(DevCounters* c) {
    c->st_applied = c->st_rejected = c->st_dups = 0;
    c->n_uniq = 0;
    c->vmax = 0;
    c->vany = 0;
    c->edges = 0;
    c->checksum = 0;
}

// sorted ids: count rejected and distinct, activate the inactive ones
__global__ __launch_bounds__(kThreads) void k_vins(GraphView g, const uint32_t* keys, uint64_t n) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t i = vt_tidx();
    unsigned long long rej = 0, uniq = 0, app = 0;
    if (i < n) {
        const uint32_t id = keys[i];
        const bool valid = id <= kMaxId && (uint64_t)id < g.n_cap;
        rej = !valid;
        if (valid && (i == 0 || keys[i - 1] != id)) {
            uniq = 1;
            const uint32_t bit = 1u << (id & 31);
            const uint32_t old = atomicOr(&g.active[id >> 5], bit);
            if (!(old & bit)) {
                app = 1;
                g.vt[id] = VRec{0u, 0u, kNoDir, 0u};
            }
        }
    }
    rej = block_sum(rej, lds);
    uniq = block_sum(uniq, lds);
    app = block_sum(app, lds);
    if (threadIdx.x == 0) {
        if (rej) atomicAdd(&g.ctr->st_rejected, rej);
        if (uniq) atomicAdd(&g.ctr->n_uniq, uniq);
        if (app) atomicAdd(&g.ctr->st_applied, app);
    }
}

// sorted ids: mark the active distinct ones in the `gone` bitmap
__global__ __launch_bounds__(kThreads) void k_vdel_mark(GraphView g, const uint32_t* keys,
                                                        uint64_t n, uint32_t* gone) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t i = vt_tidx();
    unsigned long long rej = 0, uniq = 0, app = 0;
    if (i < n) {
        const uint32_t id = keys[i];
        const bool valid = (uint64_t)id < g.n_cap;
        rej = !valid;
        if (valid && (i == 0 || keys[i - 1] != id)) {
            uniq = 1;
            if (is_active(g, id)) {
                atomicOr(&gone[id >> 5], 1u << (id & 31));
                app = 1;
            }
        }
    }
    rej = block_sum(rej, lds);
    uniq = block_sum(uniq, lds);
    app = block_sum(app, lds);
    if (threadIdx.x == 0) {
        if (rej) atomicAdd(&g.ctr->st_rejected, rej);
        if (uniq) atomicAdd(&g.ctr->n_uniq, uniq);
        if (app) atomicAdd(&g.ctr->st_applied, app);
    }
}

// 16-lane groups, one vertex each: count (EMIT = false) or emit (EMIT = true)
// the edges that touch a deleted vertex; emitted pairs go to the vertex's
// scanned offset, in slot order
constexpr int kVGroup = 16;          // lanes per sweep unit
constexpr int kVUnroll = 4;          // slots per lane per step
constexpr uint32_t kVChunk = 256;    // adjacency slots per sweep unit

// Sweep units: every active vertex with edges is cut into units of kVChunk
// slots, so that a hub is swept by many groups at once.  The scan gives each
// vertex the index of its first unit.
struct UnitIn {
    GraphView g;
    struct Rec {
        VRec r;
        bool act;
    };
    __device__ uint64_t limit(uint64_t n) const { return n; }
    __device__ Rec load(uint64_t u, bool) const {
        Rec x;
        x.r = g.vt[u];
        x.act = active_bit(g, (uint32_t)u);
        return x;
    }
    __device__ void deref(Rec&) const {}
    __device__ unsigned long long value(uint64_t, const Rec& x) const {
        return x.act ? (x.r.deg + kVChunk - 1) / kVChunk : 0u;
    }
};

// plain form of UnitIn for the three-kernel scan
struct UnitCount {
    GraphView g;
    __device__ unsigned long long operator()(uint64_t u) const {
        if (u >= g.n_cap || !active_bit(g, (uint32_t)u)) return 0ull;
        return (g.vt[u].deg + kVChunk - 1) / kVChunk;
    }
};

// unit = (vertex, first slot) at the vertex's scanned offset; a lane writes
// the units of its vertex, the whole wave those of a vertex with more than 4
__global__ __launch_bounds__(kThreads) void k_vdel_units(GraphView g,
                                                         const unsigned long long* uoff,
                                                         uint2* units) {
    const uint64_t u = vt_tidx();
    uint32_t cnt = 0;
    unsigned long long base = 0;
    if (u < g.n_cap && active_bit(g, (uint32_t)u)) {
        cnt = (g.vt[u].deg + kVChunk - 1) / kVChunk;
        base = uoff[u];
    }
    if (cnt <= 4)
        for (uint32_t c = 0; c < cnt; ++c) units[base + c] = make_uint2((uint32_t)u, c * kVChunk);
    uint64_t m = ballot(cnt > 4);
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const uint32_t wu = __shfl((uint32_t)u, l, 64), wc = __shfl(cnt, l, 64);
        const unsigned long long wb = __shfl(base, l, 64);
        for (uint32_t c = lane_id(); c < wc; c += 64) units[wb + c] = make_uint2(wu, c * kVChunk);
    }
}

// Three passes over the sweep units (unit count on the device):
//   kCount   kept[k] = slots of unit k that stay
//   kGather  for a vertex that loses slots, its unit's kept values go to
//            stage[P[k] + rank] (P = exclusive scan of kept)
//   kScatter they are written back to the vertex's slots P[k] - P[first] ...
enum VPass { kCount = 0, kGather = 1, kScatter = 2 };

template <int PASS>
__global__ __launch_bounds__(kThreads) void k_vdel_pass(GraphView g, const uint32_t* gone,
                                                        const uint2* units,
                                                        const unsigned long long* uoff,
                                                        uint32_t* kept,
                                                        const unsigned long long* P,
                                                        uint32_t* stage) {
    const uint32_t lane = lane_id();
    const uint32_t gl = lane & (kVGroup - 1);
    const uint32_t g0 = lane & ~(uint32_t)(kVGroup - 1);
    const uint64_t below = (1ull << gl) - 1;
    const uint64_t ngroups = (uint64_t)gridDim.x * kThreads / kVGroup;
    const uint64_t grp = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) / kVGroup;
    const uint64_t nunits = g.ctr->v_units;
    for (uint64_t k = grp; k < nunits; k += ngroups) {
        const uint2 U = units[k];
        const VRec r = g.vt[U.x];
        const uint32_t s1 = min(r.deg, U.y + kVChunk);
        const bool src_gone = bit_of(gone, U.x);
        unsigned long long base = 0, vbase = 0;
        if (PASS != kCount) {
            // the vertex's new degree: kept slots over all its units
            const unsigned long long f = uoff[U.x];
            const unsigned long long nu = (r.deg + kVChunk - 1) / kVChunk;
            vbase = P[f];
            const unsigned long long newdeg = P[f + nu] - vbase;
            if (newdeg == r.deg) continue;  // the vertex keeps every slot
            base = P[k];
        }
        if (PASS == kScatter) {
            // stage[P[k] .. P[k] + kept[k]) -> slots P[k] - P[first] ...
            const uint32_t nk = kept[k];
            const uint32_t d0 = (uint32_t)(base - vbase);
            for (uint32_t j = gl; j < nk; j += kVGroup) {
                const uint32_t sl = d0 + j;
                g.pool[slot_addr(g, r, sl)] = stage[base + j];
            }
            continue;
        }
        uint32_t c = 0;
        for (uint32_t s0 = U.y; s0 < s1; s0 += kVGroup * kVUnroll) {
            uint32_t blk[kVUnroll], x[kVUnroll];
            bool keep[kVUnroll];
#pragma unroll
            for (int j = 0; j < kVUnroll; ++j)
                blk[j] = block_of(g, r, min(s0 + j * kVGroup + gl, s1 - 1) >> g.log2B);
#pragma unroll
            for (int j = 0; j < kVUnroll; ++j) {
                const uint32_t sl = min(s0 + j * kVGroup + gl, s1 - 1);
                x[j] = g.pool[((uint64_t)blk[j] << g.log2B) + (sl & (g.B - 1))];
            }
#pragma unroll
            for (int j = 0; j < kVUnroll; ++j)
                keep[j] = s0 + j * kVGroup + gl < s1 && !src_gone && !bit_of(gone, x[j]);
#pragma unroll
            for (int j = 0; j < kVUnroll; ++j) {
                const uint64_t m = (ballot(keep[j]) >> g0) & ((1ull << kVGroup) - 1);
                if (PASS == kGather && keep[j]) stage[base + c + popc64(m & below)] = x[j];
                c += popc64(m);
            }
        }
        if (PASS == kCount && gl == 0) kept[k] = c;
    }
}

// kept slots per unit, for the scan that places them
struct KeptIn {
    const uint32_t* kept;
    const DevCounters* ctr;
    struct Rec {
        uint32_t c;
    };
    __device__ uint64_t limit(uint64_t n) const { return min((uint64_t)ctr->v_units, n); }
    __device__ Rec load(uint64_t i, bool ok) const { return Rec{kept[ok ? i : 0]}; }
    __device__ void deref(Rec&) const {}
    __device__ unsigned long long value(uint64_t, const Rec& r) const { return r.c; }
    __device__ unsigned long long operator()(uint64_t i) const {
        return i < ctr->v_units ? kept[i] : 0ull;
    }
};

// Per vertex: blocks it gives up (low half) and slots it loses (high half).
struct LossIn {
    GraphView g;
    const unsigned long long* uoff;
    const unsigned long long* P;
    struct Rec {
        VRec r;
        unsigned long long f, a, b;
    };
    __device__ uint64_t limit(uint64_t n) const { return n; }
    __device__ Rec load(uint64_t u, bool) const {
        Rec x;
        x.r = g.vt[u];
        x.f = uoff[u];
        x.a = x.b = 0;
        return x;
    }
    __device__ void deref(Rec& x) const {
        const unsigned long long nu = (x.r.deg + kVChunk - 1) / kVChunk;
        x.a = P[x.f];
        x.b = P[x.f + nu];
    }
    __device__ unsigned long long value(uint64_t u, const Rec& x) const {
        if (!active_bit(g, (uint32_t)u)) return 0ull;
        const uint32_t nd = (uint32_t)(x.b - x.a);
        const unsigned long long lost = x.r.deg - nd;
        return (unsigned long long)(nblocks(g, x.r.deg) - nblocks(g, nd)) | (lost << 32);
    }
    __device__ unsigned long long operator()(uint64_t u) const {
        Rec x = load(u, true);
        deref(x);
        return value(u, x);
    }
};

// Per vertex that lost slots: emptied blocks to the free list (at the
// scanned position after the current free count), new degree.  A lane frees
// up to 4 blocks, the whole wave the blocks of a vertex that frees more.
__global__ __launch_bounds__(kThreads) void k_vdel_loss(GraphView g,
                                                        const unsigned long long* uoff,
                                                        const unsigned long long* P,
                                                        const unsigned long long* pre) {
    const uint64_t u = vt_tidx();
    const bool live = u < g.n_cap && active_bit(g, (uint32_t)u);
    VRec r{0u, 0u, kNoDir, 0u};
    uint32_t nd = 0, nb0 = 0, nb1 = 0;
    unsigned long long pos = 0;
    if (live) {
        r = g.vt[u];
        const unsigned long long f = uoff[u];
        nd = (uint32_t)(P[f + (r.deg + kVChunk - 1) / kVChunk] - P[f]);
        nb0 = nblocks(g, r.deg);
        nb1 = nblocks(g, nd);
        pos = g.ctr->free_cnt + (pre[u] & 0xffffffffull);
    }
    const bool changed = live && nd != r.deg;
    const uint32_t nfree = nb0 - nb1;
    if (changed && nfree <= 4)
        for (uint32_t j = 0; j < nfree; ++j) g.free_stack[pos + j] = block_of(g, r, nb1 + j);
    uint64_t m = ballot(changed && nfree > 4);
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        VRec w;
        w.deg = __shfl(r.deg, l, 64);
        w.dir = __shfl(r.dir, l, 64);
        w.dcls = __shfl(r.dcls, l, 64);
        w.aux = 0;
        const uint32_t wb1 = __shfl(nb1, l, 64), wn = __shfl(nfree, l, 64);
        const unsigned long long wp = __shfl(pos, l, 64);
        for (uint32_t j = lane_id(); j < wn; j += 64) g.free_stack[wp + j] = block_of(g, w, wb1 + j);
    }
    if (changed) {
        VRec nr = r;
        nr.deg = nd;
        if (nb1 == 0 && nr.dcls == kNoDir) nr.dir = 0;
        g.vt[u] = nr;
    }
}

__global__ void k_vdel_tail(DevCounters* c) {
    const unsigned long long fr = c->v_fr;
    c->free_cnt += fr & 0xffffffffull;
    c->c_freed_blocks += fr & 0xffffffffull;
    c->live_edges -= fr >> 32;
}

// offsets out of a scan, in both sink forms
struct U64Out {
    unsigned long long* a;
    __device__ void operator()(uint64_t i, unsigned long long v) const { a[i] = v; }
    template <typename R>
    __device__ void operator()(uint64_t i, const R&, uint64_t, unsigned long long v) const {
        a[i] = v;
    }
};

__global__ __launch_bounds__(kThreads) void k_vdel_finish(GraphView g, const uint32_t* keys,
                                                          uint64_t n, const uint32_t* gone) {
    const uint64_t i = vt_tidx();
    if (i >= n) return;
    const uint32_t id = keys[i];
    if ((uint64_t)id >= g.n_cap || (i > 0 && keys[i - 1] == id) || !bit_of(gone, id)) return;
    atomicAnd(&g.active[id >> 5], ~(1u << (id & 31)));
    const VRec r = g.vt[id];
    if (r.dcls != kNoDir) {
        const uint32_t pos = atomicAdd(&g.ctr->dfree_cnt[r.dcls], 1u);
        g.dfree[g.dfree_base[r.dcls] + pos] = r.dir;
        atomicAdd(&g.ctr->dir_live, (unsigned long long)(-(long long)(1ull << r.dcls)));
    }
    g.vt[id] = VRec{0u, 0u, kNoDir, 0u};
}

// sort a copy of the ids into `keys` (ascending); returns the sorted array
static uint32_t* sorted_ids(gv_graph* g, const uint32_t* ids, uint64_t n, uint32_t* k0,
                            uint32_t* k1) {
    Ctx& c = g->ctx;
    c.launch("vcopy", k_vcopy_ids, div_up(n, kThreads), kThreads, ids, n, k0);
    SortScratch ss{};
    {
        Carver mz(nullptr);
        carve_sort<uint32_t>(mz, ss, n);
        g->scratch.ensure(mz.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve_sort<uint32_t>(cv, ss, n);
    }
    return radix_sort<uint32_t, false>(c, k0, k1, nullptr, nullptr, n, 32, ss) ? k1 : k0;
}

// a vertex batch's own buffer, kept by the graph between calls
static void* vbuf(gv_graph* g, int slot, size_t bytes) {
    g->vscr[slot].ensure(std::max<size_t>(bytes, 4), g->ctx.stream);
    return g->vscr[slot].ptr;
}

static void grow_table(gv_graph* g, uint64_t new_cap) {
    Ctx& c = g->ctx;
    GraphView& v = g->v;
    void *vt2 = nullptr, *act2 = nullptr;
    hip_check(hipMalloc(&vt2, new_cap * sizeof(VRec)), "hipMalloc vertex table");
    const uint64_t words = (new_cap + 31) / 32;
    if (hipMalloc(&act2, words * 4) != hipSuccess) {
        hipFree(vt2);
        fail(GV_ENOMEM, "hipMalloc active bitmap");
    }
    c.launch("grow_table", k_grow_table, div_up(new_cap, kThreads), kThreads, (const VRec*)v.vt,
             (const uint32_t*)v.active, (uint64_t)v.n_cap, (VRec*)vt2, (uint32_t*)act2, new_cap);
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    hipFree(g->mem_vt);
    hipFree(g->mem_active);
    g->mem_vt = vt2;
    g->mem_active = act2;
    v.vt = (VRec*)vt2;
    v.active = (uint32_t*)act2;
    v.n_cap = new_cap;
    v.L = log2_exact(new_cap);
    ++g->table_gen;
}

void vertex_insert(gv_graph* g, const uint32_t* ids, uint64_t n, gv_batch_stats* st,
                   bool fixed_table) {
    Ctx& c = g->ctx;
    if (n >= 0xffffffffull) fail(GV_EINVAL, "batch too large");
    c.launch("vreset", k_vreset, 1, 1, g->v.ctr);
    if (fixed_table) {
        // no growth (and no read-back): an id past the table is an error
        c.launch("vfit", k_vfit, div_up(n, kThreads), kThreads, g->v, ids, n);
    } else {
        c.launch("vmax", k_vmax, div_up(n, kThreads), kThreads, ids, n, g->v.ctr);
        read_counters(g);
        if (g->hctr->vany && (uint64_t)g->hctr->vmax >= g->v.n_cap) {
            uint64_t cap = g->v.n_cap;
            while (cap <= (uint64_t)g->hctr->vmax) cap <<= 1;
            grow_table(g, cap);
        }
    }
    uint32_t* k0 = (uint32_t*)vbuf(g, 0, 2 * n * sizeof(uint32_t));
    uint32_t* sorted = sorted_ids(g, ids, n, k0, k0 + n);
    c.launch("vinsert", k_vins, div_up(n, kThreads), kThreads, g->v, (const uint32_t*)sorted, n);
    if (st) {
        read_counters(g);
        st->applied = g->hctr->st_applied;
        st->rejected = g->hctr->st_rejected;
        st->batch_duplicates = n - g->hctr->st_rejected - g->hctr->n_uniq;
    }
}

void vertex_batch_warm() {
    resident_grid(k_vdel_pass<kCount>, kThreads);
}

// Buffer sizes a vertex batch of n ids needs: g->scratch (the id sort) and
// the three graph-owned vertex buffers; edge_bound as in vertex_delete.
void vertex_batch_bytes(const gv_graph* g, bool del, uint64_t n, uint64_t edge_bound,
                        size_t out[4]) {
    SortScratch ss{};
    Carver ms(nullptr);
    carve_sort<uint32_t>(ms, ss, n);
    out[0] = ms.used;
    const uint64_t ncap = g->v.n_cap;
    const uint64_t words = (ncap + 31) / 32;
    out[1] = (2 * n + (del ? words : 0)) * sizeof(uint32_t);
    out[2] = out[3] = 0;
    if (!del) return;
    out[2] = (2 * (ncap + 1) + scan2_parts(ncap + 1) + scan_partials_needed(ncap + 1) + 2) *
             sizeof(unsigned long long);
    const uint64_t ubound = ncap + edge_bound / kVChunk + 1;
    Carver m(nullptr);
    m.take<uint2>(ubound);
    m.take<uint32_t>(ubound);
    m.take<unsigned long long>(ubound + 1);
    m.take<unsigned long long>(scan2_parts(ubound + 1) + scan_partials_needed(ubound + 1) + 2);
    m.take<uint32_t>(std::max<uint64_t>(edge_bound, 1));
    out[3] = m.used;
}

// scan over n elements with the two-kernel scan when it fits, else the
// three-kernel one; `part` holds enough partials for either
template <typename In, typename Plain, typename Out>
static void scan_any(Ctx& c, const char* name, In in, Plain plain, Out out, uint64_t n,
                     unsigned long long* part, unsigned long long* total) {
    if (scan2_parts(n) <= kScan2MaxTiles)
        scan2(c, name, in, out, n, part, total);
    else
        scan_excl<unsigned long long>(c, plain, out, n, part, total);
}

static uint64_t scan_words(uint64_t n) {
    return scan2_parts(n) + scan_partials_needed(n) + 2;
}

// edge_bound: an upper bound on the edges stored when the call runs (0: read
// it from the device, which synchronises)
void vertex_delete(gv_graph* g, const uint32_t* ids, uint64_t n, gv_batch_stats* st,
                   uint64_t edge_bound) {
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    if (n >= 0xffffffffull) fail(GV_EINVAL, "batch too large");
    const uint64_t ncap = v.n_cap;
    const uint64_t words = (ncap + 31) / 32;
    uint32_t* k0 = (uint32_t*)vbuf(g, 0, (2 * n + words) * sizeof(uint32_t));
    uint32_t* gone = k0 + 2 * n;
    c.launch("vreset", k_vreset, 1, 1, v.ctr);
    c.launch("vzero", k_vzero, div_up(words, kThreads), kThreads, gone, words);
    uint32_t* sorted = sorted_ids(g, ids, n, k0, k0 + n);
    c.launch("vdel_mark", k_vdel_mark, div_up(n, kThreads), kThreads, v, (const uint32_t*)sorted,
             n, gone);
    if (!edge_bound) {
        read_counters(g);
        if (!g->hctr->st_applied) {
            if (st) {
                st->applied = 0;
                st->rejected = g->hctr->st_rejected;
                st->batch_duplicates = n - g->hctr->st_rejected - g->hctr->n_uniq;
            }
            return;
        }
        edge_bound = g->hctr->live_edges;
    }
    // per-vertex buffers: unit offsets, loss prefixes, scan partials
    unsigned long long* uoff = (unsigned long long*)vbuf(
        g, 1, (2 * (ncap + 1) + scan_words(ncap + 1)) * sizeof(unsigned long long));
    unsigned long long* lpre = uoff + ncap + 1;
    unsigned long long* vpart = lpre + ncap + 1;
    // per-unit buffers: units, kept counts, their scan, staging
    const uint64_t ubound = ncap + edge_bound / kVChunk + 1;
    uint2* units = nullptr;
    uint32_t *kept = nullptr, *stage = nullptr;
    unsigned long long *P = nullptr, *upart = nullptr;
    auto carve = [&](Carver& cv) {
        units = cv.take<uint2>(ubound);
        kept = cv.take<uint32_t>(ubound);
        P = cv.take<unsigned long long>(ubound + 1);
        upart = cv.take<unsigned long long>(scan_words(ubound + 1));
        stage = cv.take<uint32_t>(std::max<uint64_t>(edge_bound, 1));
    };
    {
        Carver m0(nullptr);
        carve(m0);
        Carver cv(vbuf(g, 2, m0.used));
        carve(cv);
    }
    scan_any(c, "vdel_units", UnitIn{v}, UnitCount{v}, U64Out{uoff}, ncap, vpart,
             &v.ctr->v_units);
    c.launch("vdel_units", k_vdel_units, div_up(ncap, kThreads), kThreads, v,
             (const unsigned long long*)uoff, units);
    const uint64_t vgrid = std::min<uint64_t>(div_up(ubound * kVGroup, kThreads),
                                              resident_grid(k_vdel_pass<kCount>, kThreads));
    c.launch("vdel_count", k_vdel_pass<kCount>, vgrid, kThreads, v, (const uint32_t*)gone,
             (const uint2*)units, (const unsigned long long*)uoff, kept,
             (const unsigned long long*)nullptr, (uint32_t*)nullptr);
    scan_any(c, "vdel_place", KeptIn{kept, v.ctr}, KeptIn{kept, v.ctr}, U64Out{P}, ubound + 1,
             upart, &v.ctr->v_kept);
    c.launch("vdel_gather", k_vdel_pass<kGather>, vgrid, kThreads, v, (const uint32_t*)gone,
             (const uint2*)units, (const unsigned long long*)uoff, kept,
             (const unsigned long long*)P, stage);
    c.launch("vdel_scatter", k_vdel_pass<kScatter>, vgrid, kThreads, v, (const uint32_t*)gone,
             (const uint2*)units, (const unsigned long long*)uoff, kept,
             (const unsigned long long*)P, stage);
    scan_any(c, "vdel_loss", LossIn{v, uoff, P}, LossIn{v, uoff, P}, U64Out{lpre}, ncap, vpart,
             &v.ctr->v_fr);
    c.launch("vdel_loss", k_vdel_loss, div_up(ncap, kThreads), kThreads, v,
             (const unsigned long long*)uoff, (const unsigned long long*)P,
             (const unsigned long long*)lpre);
    c.launch("vdel_tail", k_vdel_tail, 1, 1, v.ctr);
    c.launch("vdel_finish", k_vdel_finish, div_up(n, kThreads), kThreads, g->v,
             (const uint32_t*)sorted, n, (const uint32_t*)gone);
    if (st) {
        read_counters(g);
        st->applied = g->hctr->st_applied;
        st->rejected = g->hctr->st_rejected;
        st->batch_duplicates = n - g->hctr->st_rejected - g->hctr->n_uniq;
    }
}

}  // namespace gv
