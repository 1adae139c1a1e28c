// gv_vertex.hip -- batched vertex insertion and deletion (Sec. 4.4).
//
// Insert: ids are sorted and deduplicated; when the largest id does not fit,
// the dictionary is replaced by one of the next power-of-two capacity (copy
// kernel, then the old one is freed); inactive ids are switched on.
//
// Delete: the deleted set is marked in a bitmap.  One sweep over the vertex
// table compacts every small adjacency in place (thread per vertex) and cuts
// the larger ones into units of 1024 slots; a wave per unit compacts a
// vertex of one unit, and a vertex of several units fills the holes below
// its new degree with its kept slots past it (three short kernels over its
// units and one over such vertices).  Emptied blocks go on the free list,
// and the deleted vertices are switched off with their directory segments
// returned.  All sizes are bounds known on the host, so the path has no host
// round trip.
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
    c->vd_units = c->vd_hubs = c->vd_pairs = 0;
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

// Vertex delete sweep.  Every active vertex with edges is visited once.
//   small (deg <= kVSmall): one thread keeps the slots whose destination
//     stays (none for a deleted source) in order from slot 0, in place, frees
//     the emptied blocks and writes the new degree, all in the sweep kernel;
//   larger vertices are cut into units of kVUnit slots, one wave per unit.  A
//     vertex of one unit is compacted by its wave (stable, in registers).  A
//     vertex of several units (a hub) takes three steps: its units count the
//     slots they lose; the hub reserves room for min(lost, new degree) moves;
//     its units list the holes below the new degree and the kept slots at or
//     past it (as many as the holes); then the hub's wave fills every hole
//     with one of those slots (any pairing: an adjacency is a set) and frees
//     the emptied blocks.
// Only the vertex table is read in full (once); slots are read once, and a
// hub's units a second time only where they hold holes or survivors.
constexpr uint32_t kVSmall = 64;         // slots compacted by one thread
constexpr uint32_t kVPer = 16;           // slots per lane in a unit
constexpr uint32_t kVUnit = 64 * kVPer;  // slots per unit
constexpr uint32_t kVSingle = 0xFFFFFFFFu;
constexpr uint32_t kVErrBound = 4;       // err_order value: a device-side bound was exceeded

struct VDel {
    const uint32_t* gone;
    uint2* units;                // {vertex, kVSingle} or {hub, unit index}
    uint32_t* ulost;             // per unit of a hub: slots lost
    uint32_t* hv;                // per hub: vertex
    uint32_t* hlost;             // per hub: slots lost
    uint32_t* hnd;               // per hub: new degree
    uint32_t* hholes;            // per hub: holes listed
    uint32_t* hsurv;             // per hub: survivors listed
    unsigned long long* hoff;    // per hub: first entry in holes / surv
    uint32_t* holes;             // slot positions
    uint32_t* surv;              // destination values
    unsigned long long ucap, hcap, pcap;
};

__device__ __forceinline__ void vd_error(const GraphView& g) {
    g.ctr->err_order = kVErrBound;
}

// new record of a vertex left with nd slots
__device__ __forceinline__ VRec vd_record(const GraphView& g, VRec r, uint32_t nd) {
    r.deg = nd;
    if (nblocks(g, nd) == 0 && r.dcls == kNoDir) r.dir = 0;
    return r;
}

// Every lane of the wave calls this: lane-wise edges lost and blocks freed
// go into the graph's counters with one atomic each per wave.
__device__ __forceinline__ void vd_count(const GraphView& g, unsigned long long lost,
                                         unsigned long long freed) {
    lost = wave_sum(lost);
    freed = wave_sum(freed);
    if (lane_id() == 0) {
        if (lost) atomicAdd(&g.ctr->live_edges, 0ull - lost);
        if (freed) atomicAdd(&g.ctr->c_freed_blocks, freed);
    }
}

// Every lane of the wave calls this: each lane pushes blocks [b0, b1) of its
// record r onto the free stack, at slots reserved with one atomic per wave.
__device__ __forceinline__ void vd_free_lanes(const GraphView& g, const VRec& r, uint32_t b0,
                                              uint32_t b1) {
    const uint32_t nf = b1 - b0;
    const uint32_t inc = wave_incl_scan(nf);
    const uint32_t tot = __shfl(inc, 63, 64);
    if (!tot) return;
    unsigned long long base = 0;
    if (lane_id() == 63) base = atomicAdd(&g.ctr->free_cnt, (unsigned long long)tot);
    base = __shfl(base, 63, 64) + (inc - nf);
    for (uint32_t j = 0; j < nf; ++j) g.free_stack[base + j] = block_of(g, r, b0 + j);
}

// One wave pushes blocks [b0, b1) of r onto the free stack.
__device__ __forceinline__ void vd_free_wave(const GraphView& g, const VRec& r, uint32_t b0,
                                             uint32_t b1) {
    if (b1 <= b0) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&g.ctr->free_cnt, (unsigned long long)(b1 - b0));
    base = __shfl(base, 0, 64);
    for (uint32_t j = lane_id(); j < b1 - b0; j += 64) g.free_stack[base + j] = block_of(g, r, b0 + j);
}

// One thread: keeps the slots of r whose destination is not in `gone`, in
// order from slot 0, and returns how many.  In place: a kept slot is written
// at or below the position being read, so nothing unread is overwritten.
__device__ uint32_t vd_compact_small(const GraphView& g, const VRec& r, const uint32_t* gone) {
    const uint32_t nb = nblocks(g, r.deg);
    uint32_t w = 0;
    for (uint32_t j = 0; j < nb; ++j) {
        const uint32_t s0 = j << g.log2B;
        const uint32_t cnt = min(g.B, r.deg - s0);
        const uint64_t base = (uint64_t)block_of(g, r, j) << g.log2B;
        if (g.B >= 4) {
            for (uint32_t o = 0; o < cnt; o += 4) {
                const uint4 q = *reinterpret_cast<const uint4*>(g.pool + base + o);
                const uint32_t xs[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (uint32_t i = 0; i < 4; ++i) {
                    if (o + i < cnt && !bit_of(gone, xs[i])) {
                        if (w != s0 + o + i) g.pool[slot_addr(g, r, w)] = xs[i];
                        ++w;
                    }
                }
            }
        } else {
            for (uint32_t o = 0; o < cnt; ++o) {
                const uint32_t x = g.pool[base + o];
                if (!bit_of(gone, x)) {
                    if (w != s0 + o) g.pool[slot_addr(g, r, w)] = x;
                    ++w;
                }
            }
        }
    }
    return w;
}

// The sweep: one thread per vertex of the table.
__global__ __launch_bounds__(kThreads) void k_vd_sweep(GraphView g, VDel d) {
    const uint64_t u = vt_tidx();
    const bool live = u < g.n_cap && active_bit(g, (uint32_t)u);
    VRec r{0u, 0u, kNoDir, 0u};
    if (live) r = g.vt[u];
    const bool small = live && r.deg > 0 && r.deg <= kVSmall;
    uint32_t nd = r.deg;
    if (small) nd = bit_of(d.gone, (uint32_t)u) ? 0u : vd_compact_small(g, r, d.gone);
    const bool changed = small && nd != r.deg;
    if (changed) g.vt[u] = vd_record(g, r, nd);
    vd_free_lanes(g, r, changed ? nblocks(g, nd) : 0u, changed ? nblocks(g, r.deg) : 0u);
    vd_count(g, changed ? r.deg - nd : 0u,
             changed ? nblocks(g, r.deg) - nblocks(g, nd) : 0u);
    // larger vertices: hubs get an index, every unit a record
    const uint32_t nu = live && r.deg > kVSmall ? (r.deg + kVUnit - 1) / kVUnit : 0u;
    const bool hub = nu > 1;
    const uint64_t hm = ballot(hub);
    unsigned long long h = 0;
    if (hm) {
        const int leader = __ffsll((unsigned long long)hm) - 1;
        if ((int)lane_id() == leader) h = atomicAdd(&g.ctr->vd_hubs, (unsigned long long)__popcll(hm));
        h = __shfl(h, leader, 64) + rank_below(hm);
    }
    const bool hub_ok = hub && h < d.hcap;
    if (hub && !hub_ok) vd_error(g);
    if (hub_ok) {
        d.hv[h] = (uint32_t)u;
        d.hlost[h] = 0u;
        d.hholes[h] = 0u;
        d.hsurv[h] = 0u;
    }
    const uint32_t mine = hub && !hub_ok ? 0u : nu;
    const uint32_t inc = wave_incl_scan(mine);
    const uint32_t tot = __shfl(inc, 63, 64);
    if (!tot) return;
    unsigned long long base = 0;
    if (lane_id() == 63) base = atomicAdd(&g.ctr->vd_units, (unsigned long long)tot);
    base = __shfl(base, 63, 64) + (inc - mine);
    for (uint32_t k = 0; k < mine; ++k) {
        if (base + k >= d.ucap) {
            vd_error(g);
            break;
        }
        d.units[base + k] = hub ? make_uint2((uint32_t)h, k) : make_uint2((uint32_t)u, kVSingle);
    }
}

// The slots of one unit in a wave's registers: lane l holds positions
// p0 + 64 j + l, j < kVPer; keep = the slot exists and stays.
struct VUnitSlots {
    uint32_t x[kVPer];
    bool valid[kVPer], keep[kVPer];
};

__device__ __forceinline__ void vd_load_unit(const GraphView& g, const VRec& r, uint32_t p0,
                                             bool src_gone, const uint32_t* gone, VUnitSlots& s) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t j = 0; j < kVPer; ++j) {
        const uint32_t p = p0 + 64 * j + lane;
        s.valid[j] = p < r.deg;
        s.x[j] = s.valid[j] ? g.pool[slot_addr(g, r, p)] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kVPer; ++j)
        s.keep[j] = s.valid[j] && !src_gone && !bit_of(gone, s.x[j]);
}

// Units, one wave each.  Pass 0: a single-unit vertex is compacted and
// finished; a hub's unit counts its lost slots.  Pass 1 (after the hubs'
// reservations): a hub's unit lists its holes below the new degree and its
// kept slots at or past it.
template <int PASS>
__global__ __launch_bounds__(kThreads) void k_vd_units(GraphView g, VDel d) {
    const uint32_t lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    const uint64_t nunits = min(g.ctr->vd_units, d.ucap);
    for (uint64_t k = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); k < nunits; k += nw) {
        const uint2 U = d.units[k];
        const bool single = U.y == kVSingle;
        if (PASS == 1 && single) continue;
        const uint32_t v = single ? U.x : d.hv[U.x];
        const VRec r = g.vt[v];
        const uint32_t p0 = single ? 0u : U.y * kVUnit;
        uint32_t nd = 0;
        if (PASS == 1) {
            nd = d.hnd[U.x];
            // nothing to list: the hub keeps every slot or none, or this unit
            // lies below the new degree and has no holes
            if (d.hlost[U.x] == 0 || nd == 0 || (p0 + kVUnit <= nd && d.ulost[k] == 0)) continue;
        }
        VUnitSlots s;
        vd_load_unit(g, r, p0, bit_of(d.gone, v), d.gone, s);
        if (PASS == 0 && !single) {
            uint32_t lost = 0;
#pragma unroll
            for (uint32_t j = 0; j < kVPer; ++j) lost += s.valid[j] && !s.keep[j];
            lost = wave_sum(lost);
            if (lane == 0) {
                d.ulost[k] = lost;
                if (lost) atomicAdd(&d.hlost[U.x], lost);
            }
            continue;
        }
        if (PASS == 1) {
            const uint32_t h = U.x;
            const uint32_t cap = min(d.hlost[h], nd);
            const unsigned long long off = d.hoff[h];
#pragma unroll
            for (uint32_t j = 0; j < kVPer; ++j) {
                const uint32_t p = p0 + 64 * j + lane;
                const bool hole = s.valid[j] && !s.keep[j] && p < nd;
                const bool sv = s.keep[j] && p >= nd;
                const uint64_t mh = ballot(hole), ms = ballot(sv);
                uint32_t bh = 0, bs = 0;
                if (lane == 0) {
                    if (mh) bh = atomicAdd(&d.hholes[h], (uint32_t)__popcll(mh));
                    if (ms) bs = atomicAdd(&d.hsurv[h], (uint32_t)__popcll(ms));
                }
                bh = __shfl(bh, 0, 64) + rank_below(mh);
                bs = __shfl(bs, 0, 64) + rank_below(ms);
                if ((hole && bh >= cap) || (sv && bs >= cap)) {
                    vd_error(g);
                } else {
                    if (hole) d.holes[off + bh] = p;
                    if (sv) d.surv[off + bs] = s.x[j];
                }
            }
            continue;
        }
        // a single-unit vertex: stable compaction of the kept slots
        uint32_t base = 0;
#pragma unroll
        for (uint32_t j = 0; j < kVPer; ++j) {
            const uint64_t m = ballot(s.keep[j]);
            const uint32_t q = base + rank_below(m);
            const uint32_t p = 64 * j + lane;
            if (s.keep[j] && q != p) g.pool[slot_addr(g, r, q)] = s.x[j];
            base += popc64(m);
        }
        if (base == r.deg) continue;
        vd_free_wave(g, r, nblocks(g, base), nblocks(g, r.deg));
        if (lane == 0) {
            g.vt[v] = vd_record(g, r, base);
            atomicAdd(&g.ctr->live_edges, 0ull - (unsigned long long)(r.deg - base));
            atomicAdd(&g.ctr->c_freed_blocks,
                      (unsigned long long)(nblocks(g, r.deg) - nblocks(g, base)));
        }
    }
}

// One thread per hub: new degree, room for min(lost, new degree) moves.
__global__ __launch_bounds__(kThreads) void k_vd_reserve(GraphView g, VDel d) {
    const uint64_t h = vt_tidx();
    if (h >= min(g.ctr->vd_hubs, d.hcap)) return;
    const uint32_t deg = g.vt[d.hv[h]].deg;
    const uint32_t lost = min(d.hlost[h], deg);
    const uint32_t nd = deg - lost;
    d.hnd[h] = nd;
    const uint32_t cap = min(lost, nd);
    const unsigned long long off = atomicAdd(&g.ctr->vd_pairs, (unsigned long long)cap);
    if (off + cap > d.pcap) {
        vd_error(g);
        d.hlost[h] = 0u;  // lists nothing and stays as it is
        d.hnd[h] = deg;
        d.hoff[h] = 0ull;
        return;
    }
    d.hoff[h] = off;
}

// One wave per hub: fill the holes, free the emptied blocks, new degree.
__global__ __launch_bounds__(kThreads) void k_vd_fill(GraphView g, VDel d) {
    const uint32_t lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    const uint64_t nh = min(g.ctr->vd_hubs, d.hcap);
    for (uint64_t h = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); h < nh; h += nw) {
        const uint32_t v = d.hv[h];
        const VRec r = g.vt[v];
        const uint32_t nd = d.hnd[h];
        if (nd == r.deg) continue;
        const uint32_t n = d.hholes[h];
        if (n != d.hsurv[h] || n > min(r.deg - nd, nd)) {
            if (lane == 0) vd_error(g);
            continue;
        }
        const unsigned long long off = d.hoff[h];
        for (uint32_t i = lane; i < n; i += 64)
            g.pool[slot_addr(g, r, d.holes[off + i])] = d.surv[off + i];
        vd_free_wave(g, r, nblocks(g, nd), nblocks(g, r.deg));
        if (lane == 0) {
            g.vt[v] = vd_record(g, r, nd);
            atomicAdd(&g.ctr->live_edges, 0ull - (unsigned long long)(r.deg - nd));
            atomicAdd(&g.ctr->c_freed_blocks,
                      (unsigned long long)(nblocks(g, r.deg) - nblocks(g, nd)));
        }
    }
}

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
    resident_grid(k_vd_units<0>, kThreads);
    resident_grid(k_vd_units<1>, kThreads);
    resident_grid(k_vd_fill, kThreads);
}

namespace {

// Capacities of a vertex delete's lists, from an upper bound on the edges
// stored (every bound holds for any graph with at most that many edges).
struct VDelCaps {
    uint64_t units, hubs, pairs;
};

VDelCaps vdel_caps(const gv_graph* g, uint64_t edge_bound) {
    VDelCaps k;
    // a vertex with units has more than kVSmall slots; a hub more than kVUnit
    const uint64_t big = std::min<uint64_t>(g->v.n_cap, edge_bound / (kVSmall + 1) + 1);
    k.units = big + edge_bound / kVUnit + 1;
    k.hubs = std::min<uint64_t>(g->v.n_cap, edge_bound / (kVUnit + 1) + 1);
    // sum over hubs of min(lost, kept) <= half their slots
    k.pairs = edge_bound / 2 + 1;
    return k;
}

void vdel_carve(Carver& cv, const VDelCaps& k, VDel& d) {
    d.units = cv.take<uint2>(k.units);
    d.ulost = cv.take<uint32_t>(k.units);
    d.hv = cv.take<uint32_t>(k.hubs);
    d.hlost = cv.take<uint32_t>(k.hubs);
    d.hnd = cv.take<uint32_t>(k.hubs);
    d.hholes = cv.take<uint32_t>(k.hubs);
    d.hsurv = cv.take<uint32_t>(k.hubs);
    d.hoff = cv.take<unsigned long long>(k.hubs);
    d.holes = cv.take<uint32_t>(k.pairs);
    d.surv = cv.take<uint32_t>(k.pairs);
    d.ucap = k.units;
    d.hcap = k.hubs;
    d.pcap = k.pairs;
}

}  // namespace

// Buffer sizes a vertex batch of n ids needs: g->scratch (the id sort) and
// the graph-owned vertex buffers; edge_bound as in vertex_delete.
void vertex_batch_bytes(const gv_graph* g, bool del, uint64_t n, uint64_t edge_bound,
                        size_t out[4]) {
    SortScratch ss{};
    Carver ms(nullptr);
    carve_sort<uint32_t>(ms, ss, n);
    out[0] = ms.used;
    const uint64_t words = (g->v.n_cap + 31) / 32;
    out[1] = (2 * n + (del ? words : 0)) * sizeof(uint32_t);
    out[2] = out[3] = 0;
    if (!del) return;
    VDel d{};
    Carver m(nullptr);
    vdel_carve(m, vdel_caps(g, edge_bound), d);
    out[2] = m.used;
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
    VDel d{};
    {
        const VDelCaps k = vdel_caps(g, edge_bound);
        Carver m0(nullptr);
        vdel_carve(m0, k, d);
        Carver cv(vbuf(g, 1, m0.used));
        vdel_carve(cv, k, d);
    }
    d.gone = gone;
    c.launch("vdel_sweep", k_vd_sweep, div_up(ncap, kThreads), kThreads, v, d);
    const uint64_t ugrid = resident_grid(k_vd_units<0>, kThreads);
    c.launch("vdel_units", k_vd_units<0>, ugrid, kThreads, v, d);
    c.launch("vdel_reserve", k_vd_reserve, div_up(d.hcap, kThreads), kThreads, v, d);
    c.launch("vdel_collect", k_vd_units<1>, ugrid, kThreads, v, d);
    c.launch("vdel_fill", k_vd_fill, resident_grid(k_vd_fill, kThreads), kThreads, v, d);
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
