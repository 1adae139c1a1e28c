// gv_vertex.hip -- batched vertex insertion and deletion (Sec. 4.4).
//
// Insert: an id's first occurrence in the batch is found with a bitmap of
// the ids seen (no sort of the ids); when the largest id does not fit,
// the dictionary is replaced by one of the next power-of-two capacity (copy
// kernel, then the old one is freed); inactive ids are switched on.
//
// Delete: the deleted set is marked in a bitmap.  One streaming pass over
// the pool's handed-out blocks finds every slot whose destination is deleted
// (checked against the block's owner record); each vertex that loses slots
// fills the holes below its new degree with the kept slots past it, emptied
// blocks go on the free list, a deleted source gives all its blocks back,
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
    c->vd_hits = c->vd_touched = c->vd_pairs = 0;
}

// Ids in input order: an id's first occurrence is the thread whose atomicOr
// sets its bit in `seen` (zeroed per call), so duplicates are found without
// sorting the ids.  Counts rejected and distinct ids and activates the
// inactive ones.
__global__ __launch_bounds__(kThreads) void k_vins(GraphView g, const uint32_t* ids, uint64_t n,
                                                   uint32_t* seen) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t i = vt_tidx();
    unsigned long long rej = 0, uniq = 0, app = 0;
    if (i < n) {
        const uint32_t id = ids[i];
        const bool valid = id <= kMaxId && (uint64_t)id < g.n_cap;
        rej = !valid;
        const uint32_t bit = 1u << (id & 31);
        if (valid && !(atomicOr(&seen[id >> 5], bit) & bit)) {
            uniq = 1;
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

// Ids in input order: the first occurrence of each valid id (its atomicOr
// sets the bit in `seen`) gets first[i] = 1, and marks the id in the `gone`
// bitmap when it is active; the later kernels of the delete take an id at
// its first occurrence only.
__global__ __launch_bounds__(kThreads) void k_vdel_mark(GraphView g, const uint32_t* ids,
                                                        uint64_t n, uint32_t* seen,
                                                        uint32_t* gone, uint8_t* first) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t i = vt_tidx();
    unsigned long long rej = 0, uniq = 0, app = 0;
    if (i < n) {
        const uint32_t id = ids[i];
        const bool valid = (uint64_t)id < g.n_cap;
        rej = !valid;
        const uint32_t bit = 1u << (id & 31);
        const bool head = valid && !(atomicOr(&seen[id >> 5], bit) & bit);
        first[i] = head ? 1 : 0;
        if (head) {
            uniq = 1;
            if (is_active(g, id)) {
                atomicOr(&gone[id >> 5], bit);
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

// Vertex delete.  The slots that lose their destination are found by one
// flat pass over the pool's handed-out blocks (streaming reads, no walk of
// any adjacency): a slot whose value is a deleted id is checked against the
// block's owner record (the owner is live, not deleted, still holds this
// block at that index, and the slot is below its degree) and becomes a hit
// (vertex, position); each owner counts its hits.  Then, per vertex with
// hits (touched), with nd = degree - hits: the hits below nd are holes and
// the kept slots in [nd, degree) are exactly as many; the k-th kept slot of
// that tail fills the k-th hole (any pairing: an adjacency is a set), the
// emptied blocks go on the free list and the degree becomes nd.  A deleted
// source gives all its blocks back.  Shared counters take one atomic per
// workgroup or per wave, not per slot.
//
// A summary of the deleted set sits in LDS for the pass over the pool: bit
// b is set when a vertex in [b << sum_shift, (b + 1) << sum_shift) is
// deleted, so most slots are cleared without touching the bitmap in memory.
constexpr uint32_t kVSumBits = 1u << 17;
constexpr uint32_t kVSumWords = kVSumBits / 32;
constexpr uint32_t kVQuads = 4;        // 4-slot groups per thread per round of the pass
constexpr uint32_t kVHitBuf = 1024;    // hits staged in LDS per workgroup
constexpr uint32_t kVLane = 32;        // tails and frees a lane takes; larger ones take the wave
constexpr uint32_t kVErrBound = 4;     // err_order value: a device-side bound was exceeded

struct VDel {
    const uint32_t* gone;
    uint32_t* summary;           // kVSumWords words
    uint32_t sum_shift, sum_words;
    uint2* hits;                 // (vertex, position) of every slot that loses its destination
    uint32_t* touched;           // vertices with hits
    uint32_t* tnd;               // per touched vertex: new degree
    uint32_t* tcap;              // per touched vertex: room for holes
    uint32_t* tholes;            // per touched vertex: holes listed
    unsigned long long* toff;    // per touched vertex: first entry in holes
    uint32_t* holes;             // positions below the new degree whose slot is lost
    unsigned long long hcap, tcapn, pcap;
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

// the summary into LDS (every thread calls it; one barrier)
__device__ __forceinline__ void vd_load_summary(const VDel& d, uint32_t* s_sum) {
    for (uint32_t i = threadIdx.x; i < d.sum_words; i += kThreads) s_sum[i] = d.summary[i];
    __syncthreads();
}

// is destination x deleted: the LDS summary first, the bitmap only when the
// summary's range holds a deleted id
__device__ __forceinline__ bool vd_gone(const VDel& d, const uint32_t* s_sum, uint32_t x) {
    const uint32_t b = x >> d.sum_shift;
    if (!((s_sum[b >> 5] >> (b & 31)) & 1u)) return false;
    return bit_of(d.gone, x);
}

// summary bits of the deleted set (one thread per bitmap word)
__global__ __launch_bounds__(kThreads) void k_vd_summary(VDel d, uint64_t words) {
    const uint64_t w = vt_tidx();
    if (w >= words) return;
    for (uint32_t m = d.gone[w]; m; m &= m - 1) {
        const uint64_t b = ((w << 5) + (uint32_t)__ffs(m) - 1) >> d.sum_shift;
        atomicOr(&d.summary[b >> 5], 1u << (b & 31));
    }
}

// exclusive prefix of x over the workgroup and one atomic add of the total
// to *counter; every thread calls it (barriers inside)
__device__ __forceinline__ unsigned long long vd_reserve(unsigned long long x,
                                                        unsigned long long* counter,
                                                        unsigned long long* lds,
                                                        unsigned long long* s_base) {
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan(x, lds, tot);
    if (threadIdx.x == 0) *s_base = tot ? atomicAdd(counter, tot) : 0ull;
    __syncthreads();
    const unsigned long long b = *s_base;
    __syncthreads();
    return b + ex;
}

// Every thread of the workgroup calls this once, at the end of a kernel:
// edges lost and blocks freed go into the graph's counters.
__device__ __forceinline__ void vd_flush(const GraphView& g, unsigned long long lost,
                                         unsigned long long freed, unsigned long long* lds) {
    lost = block_sum(lost, lds);
    freed = block_sum(freed, lds);
    if (threadIdx.x == 0) {
        if (lost) atomicAdd(&g.ctr->live_edges, 0ull - lost);
        if (freed) atomicAdd(&g.ctr->c_freed_blocks, freed);
    }
}

// a slot whose value is deleted: is it a live slot of a vertex that stays,
// and at which position
__device__ __forceinline__ bool vd_hit(const GraphView& g, const VDel& d, uint64_t s,
                                       uint32_t* v_out, uint32_t* p_out) {
    const uint64_t blk = s >> g.log2B;
    const uint2 ow = g.bown[blk];
    const uint32_t v = ow.x, j = ow.y;
    if ((uint64_t)v >= g.n_cap || bit_of(d.gone, v) || !active_bit(g, v)) return false;
    const VRec r = g.vt[v];
    if (j >= nblocks(g, r.deg) || (uint64_t)block_of(g, r, j) != blk) return false;
    const uint32_t p = (j << g.log2B) + (uint32_t)(s & (g.B - 1));
    if (p >= r.deg) return false;
    *v_out = v;
    *p_out = p;
    return true;
}

// The pass over the pool's handed-out blocks [0, bump), grid-stride in rounds
// of kThreads * kVQuads groups of 4 slots, with no barrier between rounds.
// Hits, and the vertices whose first hit this is, are staged in LDS and
// appended with one atomic per workgroup at the end (a full stage spills to
// direct appends).
__global__ __launch_bounds__(kThreads) void k_vd_scan(GraphView g, VDel d) {
    __shared__ uint32_t s_sum[kVSumWords];
    __shared__ uint2 s_hit[kVHitBuf];
    __shared__ uint32_t s_tv[kVHitBuf];
    __shared__ uint32_t s_nh, s_nt;
    __shared__ unsigned long long s_bh, s_bt;
    __shared__ unsigned long long lds[kWaves];
    vd_load_summary(d, s_sum);
    if (threadIdx.x == 0) s_nh = s_nt = 0u;
    __syncthreads();
    const uint64_t slots = (uint64_t)g.ctr->bump << g.log2B;
    const uint64_t nq = (slots + 3) / 4;
    constexpr uint64_t kRound = (uint64_t)kThreads * kVQuads;
    unsigned long long lost = 0;
    auto add_hit = [&](uint32_t v, uint32_t p) {
        ++lost;
        const uint32_t k = atomicAdd(&s_nh, 1u);
        if (k < kVHitBuf) {
            s_hit[k] = make_uint2(v, p);
        } else {
            const unsigned long long i = atomicAdd(&g.ctr->vd_hits, 1ull);
            if (i < d.hcap) d.hits[i] = make_uint2(v, p);
            else vd_error(g);
        }
        if (atomicAdd(&g.vlost[v], 1u) == 0u) {
            const uint32_t kt = atomicAdd(&s_nt, 1u);
            if (kt < kVHitBuf) {
                s_tv[kt] = v;
            } else {
                const unsigned long long i = atomicAdd(&g.ctr->vd_touched, 1ull);
                if (i < d.tcapn) d.touched[i] = v;
                else vd_error(g);
            }
        }
    };
    // the slots of one round: kVQuads groups of 4 per thread (zeros past the
    // handed-out slots)
    auto load_round = [&](uint64_t q0, uint32_t (&xs)[kVQuads][4]) {
#pragma unroll
        for (uint32_t u = 0; u < kVQuads; ++u) {
            const uint64_t q = q0 + (uint64_t)u * kThreads + threadIdx.x;
            if (q < nq && g.B >= 4) {
                const uint4 w = *reinterpret_cast<const uint4*>(g.pool + 4 * q);
                xs[u][0] = w.x;
                xs[u][1] = w.y;
                xs[u][2] = w.z;
                xs[u][3] = w.w;
            } else {
#pragma unroll
                for (uint32_t i = 0; i < 4; ++i) xs[u][i] = 4 * q + i < slots ? g.pool[4 * q + i] : 0u;
            }
        }
    };
    const uint64_t stride = (uint64_t)gridDim.x * kRound;
    uint32_t xs[kVQuads][4];
    uint64_t q0 = (uint64_t)blockIdx.x * kRound;
    if (q0 < nq) load_round(q0, xs);
    for (; q0 < nq; q0 += stride) {
        // the summary in LDS clears most slots; the bitmap words of the rest
        // are loaded together (one wait per round, not one per slot)
        uint32_t cand = 0;
#pragma unroll
        for (uint32_t u = 0; u < kVQuads; ++u) {
            const uint64_t q = q0 + (uint64_t)u * kThreads + threadIdx.x;
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) {
                const uint32_t x = xs[u][i];
                bool c = 4 * q + i < slots && (uint64_t)x < g.n_cap;
                if (c) {
                    const uint32_t b = x >> d.sum_shift;
                    c = (s_sum[b >> 5] >> (b & 31)) & 1u;
                }
                cand |= (uint32_t)c << (4 * u + i);
            }
        }
        uint32_t word[4 * kVQuads];
#pragma unroll
        for (uint32_t k = 0; k < 4 * kVQuads; ++k)
            word[k] = (cand >> k) & 1u ? d.gone[xs[k / 4][k % 4] >> 5] : 0u;
        uint32_t hm = 0;  // this thread's slots whose destination is deleted
#pragma unroll
        for (uint32_t k = 0; k < 4 * kVQuads; ++k)
            hm |= ((word[k] >> (xs[k / 4][k % 4] & 31)) & 1u) << k;
        // the next round's slots are in flight while this round's hits are
        // checked
        uint32_t xn[kVQuads][4];
        if (q0 + stride < nq) load_round(q0 + stride, xn);
        // one hit per lane per step: a step's dependent loads (owner record,
        // vertex record, directory) are waited for once for all lanes, so a
        // wave waits as many times as its busiest lane has hits, not once
        // per slot position that holds a hit in some lane
        while (hm) {
            const uint32_t k = (uint32_t)__ffs(hm) - 1u;
            hm &= hm - 1u;
            const uint64_t q = q0 + (uint64_t)(k / 4) * kThreads + threadIdx.x;
            uint32_t v, p;
            if (vd_hit(g, d, 4 * q + k % 4, &v, &p)) add_hit(v, p);
        }
#pragma unroll
        for (uint32_t u = 0; u < kVQuads; ++u)
#pragma unroll
            for (uint32_t i = 0; i < 4; ++i) xs[u][i] = xn[u][i];
    }
    // move the staged hits and touched vertices out
    __syncthreads();
    const uint32_t nh = min(s_nh, kVHitBuf), nt = min(s_nt, kVHitBuf);
    if (threadIdx.x == 0) {
        s_bh = nh ? atomicAdd(&g.ctr->vd_hits, (unsigned long long)nh) : 0ull;
        s_bt = nt ? atomicAdd(&g.ctr->vd_touched, (unsigned long long)nt) : 0ull;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nh; i += kThreads) {
        if (s_bh + i < d.hcap) d.hits[s_bh + i] = s_hit[i];
        else vd_error(g);
    }
    for (uint32_t i = threadIdx.x; i < nt; i += kThreads) {
        if (s_bt + i < d.tcapn) d.touched[s_bt + i] = s_tv[i];
        else vd_error(g);
    }
    vd_flush(g, lost, 0ull, lds);
}

// Deleted sources (one thread per id, at its first occurrence): all their blocks go on the
// free list (one reservation per workgroup), their edges off the count.
__global__ __launch_bounds__(kThreads) void k_vd_sources(GraphView g, const uint32_t* ids,
                                                         uint64_t n, const uint8_t* first,
                                                         const uint32_t* gone) {
    __shared__ unsigned long long lds[kWaves];
    __shared__ unsigned long long s_base;
    const uint64_t i = vt_tidx();
    VRec r{0u, 0u, kNoDir, 0u};
    bool mine = false;
    if (i < n && first[i]) {
        const uint32_t id = ids[i];
        mine = bit_of(gone, id);
        if (mine) r = g.vt[id];
    }
    const uint32_t nb = mine ? nblocks(g, r.deg) : 0u;
    const unsigned long long pos = vd_reserve(nb, &g.ctr->free_cnt, lds, &s_base);
    if (nb <= kVLane) {
        for (uint32_t j = 0; j < nb; ++j) g.free_stack[pos + j] = block_of(g, r, j);
    }
    uint64_t m = ballot(nb > kVLane);  // larger ones by the whole wave
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        VRec w;
        w.deg = __shfl(r.deg, l, 64);
        w.dir = __shfl(r.dir, l, 64);
        w.dcls = __shfl(r.dcls, l, 64);
        w.aux = 0;
        const uint32_t wn = __shfl(nb, l, 64);
        const unsigned long long wp = __shfl(pos, l, 64);
        for (uint32_t j = lane_id(); j < wn; j += 64) g.free_stack[wp + j] = block_of(g, w, j);
    }
    vd_flush(g, mine ? r.deg : 0u, nb, lds);
}

// One thread per touched vertex (grid-stride rounds): new degree, room for
// min(hits, new degree) holes (one reservation per workgroup round), and the
// vertex's scratch word becomes its index in the touched list.
__global__ __launch_bounds__(kThreads) void k_vd_plan(GraphView g, VDel d) {
    __shared__ unsigned long long lds[kWaves];
    __shared__ unsigned long long s_base;
    const uint64_t nt = min(g.ctr->vd_touched, d.tcapn);
    for (uint64_t t0 = (uint64_t)blockIdx.x * kThreads; t0 < nt; t0 += (uint64_t)gridDim.x * kThreads) {
        const uint64_t t = t0 + threadIdx.x;
        uint32_t v = 0, deg = 0, lost = 0, cap = 0;
        if (t < nt) {
            v = d.touched[t];
            deg = g.vt[v].deg;
            lost = min(g.vlost[v], deg);
            cap = min(lost, deg - lost);
        }
        const unsigned long long off = vd_reserve(cap, &g.ctr->vd_pairs, lds, &s_base);
        if (t < nt) {
            if (off + cap > d.pcap) {
                vd_error(g);
                d.tnd[t] = deg;  // left as it is
                d.tcap[t] = 0u;
            } else {
                d.tnd[t] = deg - lost;
                d.tcap[t] = cap;
            }
            d.toff[t] = off;
            d.tholes[t] = 0u;
            g.vlost[v] = (uint32_t)t;
        }
    }
}

// One thread per hit (grid-stride): a hit below its vertex's new degree is a
// hole.
__global__ __launch_bounds__(kThreads) void k_vd_holes(GraphView g, VDel d) {
    const uint64_t nh = min(g.ctr->vd_hits, d.hcap);
    const uint64_t nt = min(g.ctr->vd_touched, d.tcapn);
    for (uint64_t i = vt_tidx(); i < nh; i += (uint64_t)gridDim.x * kThreads) {
        const uint2 h = d.hits[i];
        const uint32_t t = g.vlost[h.x];
        if (t >= nt) {
            vd_error(g);
            continue;
        }
        if (h.y >= d.tnd[t]) continue;
        const uint32_t k = atomicAdd(&d.tholes[t], 1u);
        if (k < d.tcap[t]) d.holes[d.toff[t] + k] = h.y;
        else vd_error(g);
    }
}

// Per touched vertex (a lane each; a vertex whose tail or freed blocks
// exceed kVLane is taken by the whole wave): the kept slots of the tail
// [nd, deg) fill the holes in order, emptied blocks go on the free list, the
// record gets the new degree, the scratch word is cleared.
__global__ __launch_bounds__(kThreads) void k_vd_fill(GraphView g, VDel d) {
    __shared__ unsigned long long lds[kWaves];
    const uint32_t lane = lane_id();
    const uint64_t nt = min(g.ctr->vd_touched, d.tcapn);
    unsigned long long lost_err = 0, freed = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t t0 = (uint64_t)blockIdx.x * kThreads; t0 < nt; t0 += stride) {
        const uint64_t t = t0 + threadIdx.x;
        const bool live = t < nt;
        uint32_t v = 0, nd = 0, nh = 0;
        unsigned long long off = 0;
        VRec r{0u, 0u, kNoDir, 0u};
        if (live) {
            v = d.touched[t];
            r = g.vt[v];
            nd = d.tnd[t];
            nh = d.tholes[t];
            off = d.toff[t];
            if (nh > d.tcap[t]) {  // the holes kernel reported it; list only what was kept
                nh = d.tcap[t];
                vd_error(g);
            }
        }
        const bool change = live && nd < r.deg;
        const uint32_t b0 = change ? nblocks(g, nd) : 0u, b1 = change ? nblocks(g, r.deg) : 0u;
        const bool big = change && (r.deg - nd > kVLane || b1 - b0 > kVLane);
        if (change && !big) {
            uint32_t k = 0;
            for (uint32_t p = nd; p < r.deg; ++p) {
                const uint32_t x = g.pool[slot_addr(g, r, p)];
                if (bit_of(d.gone, x)) continue;
                if (k < nh) {
                    const uint64_t da = slot_addr(g, r, d.holes[off + k]);
                    g.pool[da] = x;
                    if (g.A) attr_move(g, da, slot_addr(g, r, p));
                }
                ++k;
            }
            if (k != nh) vd_error(g);
        }
        // frees of the lane-sized vertices: one reservation per wave
        const uint32_t nf = change && !big ? b1 - b0 : 0u;
        const uint32_t inc = wave_incl_scan(nf);
        const uint32_t tot = __shfl(inc, 63, 64);
        if (tot) {
            unsigned long long fb = 0;
            if (lane == 63) fb = atomicAdd(&g.ctr->free_cnt, (unsigned long long)tot);
            fb = __shfl(fb, 63, 64) + (inc - nf);
            for (uint32_t j = 0; j < nf; ++j) g.free_stack[fb + j] = block_of(g, r, b0 + j);
        }
        // the larger vertices, one at a time by the whole wave
        uint64_t m = ballot(big);
        while (m) {
            const int l = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            VRec w;
            w.deg = __shfl(r.deg, l, 64);
            w.dir = __shfl(r.dir, l, 64);
            w.dcls = __shfl(r.dcls, l, 64);
            w.aux = 0;
            const uint32_t wnd = __shfl(nd, l, 64), wnh = __shfl(nh, l, 64);
            const unsigned long long woff = __shfl(off, l, 64);
            uint32_t k = 0;
            for (uint32_t p0 = wnd; p0 < w.deg; p0 += 64) {
                const uint32_t p = p0 + lane;
                uint32_t x = 0;
                bool keep = false;
                if (p < w.deg) {
                    x = g.pool[slot_addr(g, w, p)];
                    keep = !bit_of(d.gone, x);
                }
                const uint64_t km = ballot(keep);
                const uint32_t kk = k + rank_below(km);
                if (keep && kk < wnh) {
                    const uint64_t da = slot_addr(g, w, d.holes[woff + kk]);
                    g.pool[da] = x;
                    if (g.A) attr_move(g, da, slot_addr(g, w, p));
                }
                k += popc64(km);
            }
            if (k != wnh && lane == 0) vd_error(g);
            const uint32_t wb0 = nblocks(g, wnd), wb1 = nblocks(g, w.deg);
            unsigned long long fb = 0;
            if (lane == 0 && wb1 > wb0) fb = atomicAdd(&g.ctr->free_cnt, (unsigned long long)(wb1 - wb0));
            fb = __shfl(fb, 0, 64);
            for (uint32_t j = lane; j < wb1 - wb0; j += 64) g.free_stack[fb + j] = block_of(g, w, wb0 + j);
        }
        if (change) {
            g.vt[v] = vd_record(g, r, nd);
            freed += b1 - b0;
        }
        if (live) g.vlost[v] = 0u;
    }
    vd_flush(g, lost_err, freed, lds);
}

__global__ __launch_bounds__(kThreads) void k_vdel_finish(GraphView g, const uint32_t* ids,
                                                          uint64_t n, const uint8_t* first,
                                                          const uint32_t* gone) {
    const uint64_t i = vt_tidx();
    if (i >= n || !first[i]) return;
    const uint32_t id = ids[i];
    if (!bit_of(gone, id)) return;
    atomicAnd(&g.active[id >> 5], ~(1u << (id & 31)));
    const VRec r = g.vt[id];
    if (r.dcls != kNoDir) {
        const uint32_t pos = atomicAdd(&g.ctr->dfree_cnt[r.dcls], 1u);
        g.dfree[g.dfree_base[r.dcls] + pos] = r.dir;
        atomicAdd(&g.ctr->dir_live, (unsigned long long)(-(long long)(1ull << r.dcls)));
    }
    g.vt[id] = VRec{0u, 0u, kNoDir, 0u};
}

// bytes of a vertex delete's id buffer: gone, summary and seen bitmaps, then
// one first-occurrence flag per id
static size_t vdel_ids_bytes(uint64_t words, uint64_t n) {
    return (2 * words + kVSumWords) * sizeof(uint32_t) + n;
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
    void* vl2 = nullptr;
    if (hipMalloc(&vl2, new_cap * sizeof(uint32_t)) != hipSuccess) {
        hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
        hipFree(vt2);
        hipFree(act2);
        fail(GV_ENOMEM, "hipMalloc vertex scratch");
    }
    c.launch("grow_table", k_vzero, div_up(new_cap, kThreads), kThreads, (uint32_t*)vl2, new_cap);
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    hipFree(g->mem_vt);
    hipFree(g->mem_active);
    hipFree(g->mem_vlost);
    g->mem_vt = vt2;
    g->mem_active = act2;
    g->mem_vlost = vl2;
    v.vlost = (uint32_t*)vl2;
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
    const uint64_t words = (g->v.n_cap + 31) / 32;
    uint32_t* seen = (uint32_t*)vbuf(g, 0, words * sizeof(uint32_t));
    c.launch("vzero", k_vzero, div_up(words, kThreads), kThreads, seen, words);
    c.launch("vinsert", k_vins, div_up(n, kThreads), kThreads, g->v, ids, n, seen);
    if (st) {
        read_counters(g);
        st->applied = g->hctr->st_applied;
        st->rejected = g->hctr->st_rejected;
        st->batch_duplicates = n - g->hctr->st_rejected - g->hctr->n_uniq;
    }
}
void vertex_batch_warm() {
    resident_grid(k_vd_scan, kThreads);
    resident_grid(k_vd_plan, kThreads);
    resident_grid(k_vd_holes, kThreads);
    resident_grid(k_vd_fill, kThreads);
}

namespace {

// Capacities of a vertex delete's lists, from an upper bound on the edges
// stored (every bound holds for any graph with at most that many edges).
struct VDelCaps {
    uint64_t hits, touched, pairs;
};

VDelCaps vdel_caps(const gv_graph* g, uint64_t edge_bound) {
    VDelCaps k;
    k.hits = edge_bound + 1;  // a hit is a stored slot
    k.touched = std::min<uint64_t>(g->v.n_cap, edge_bound + 1);
    // sum over vertices of min(lost, kept) <= half their slots
    k.pairs = edge_bound / 2 + 1;
    return k;
}

void vdel_carve(Carver& cv, const VDelCaps& k, VDel& d) {
    d.hits = cv.take<uint2>(k.hits);
    d.toff = cv.take<unsigned long long>(k.touched);
    d.touched = cv.take<uint32_t>(k.touched);
    d.tnd = cv.take<uint32_t>(k.touched);
    d.tcap = cv.take<uint32_t>(k.touched);
    d.tholes = cv.take<uint32_t>(k.touched);
    d.holes = cv.take<uint32_t>(k.pairs);
    d.hcap = k.hits;
    d.tcapn = k.touched;
    d.pcap = k.pairs;
}

}  // namespace

// Buffer sizes a vertex batch of n ids needs: g->scratch (the id sort) and
// the graph-owned vertex buffers; edge_bound as in vertex_delete.
void vertex_batch_bytes(const gv_graph* g, bool del, uint64_t n, uint64_t edge_bound,
                        size_t out[4]) {
    out[0] = 0;
    const uint64_t words = (g->v.n_cap + 31) / 32;
    out[1] = del ? vdel_ids_bytes(words, n) : words * sizeof(uint32_t);
    out[2] = out[3] = 0;
    if (!del) return;
    VDel d{};
    Carver m(nullptr);
    vdel_carve(m, vdel_caps(g, edge_bound), d);
    out[2] = m.used;
}

// edge_bound: an upper bound on the edges stored when the call runs (0: the
// graph's host-side bound, capped by the pool's slots; no read-back)
void vertex_delete(gv_graph* g, const uint32_t* ids, uint64_t n, gv_batch_stats* st,
                   uint64_t edge_bound) {
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    if (n >= 0xffffffffull) fail(GV_EINVAL, "batch too large");
    const uint64_t ncap = v.n_cap;
    const uint64_t words = (ncap + 31) / 32;
    // gone | summary | seen (zeroed together), then a first-occurrence flag per id
    uint32_t* gone = (uint32_t*)vbuf(g, 0, vdel_ids_bytes(words, n));
    uint32_t* summary = gone + words;
    uint32_t* seen = summary + kVSumWords;
    uint8_t* first = (uint8_t*)(seen + words);
    c.launch("vreset", k_vreset, 1, 1, v.ctr);
    c.launch("vzero", k_vzero, div_up(2 * words + kVSumWords, kThreads), kThreads, gone,
             2 * words + kVSumWords);
    c.launch("vdel_mark", k_vdel_mark, div_up(n, kThreads), kThreads, v, ids, n, seen, gone,
             first);
    if (!edge_bound) {
        // no read-back: the host-side bound, capped by the pool's slots (every
        // stored edge holds one)
        edge_bound = std::max<uint64_t>(
            std::min<uint64_t>(g->edge_bound_host, (uint64_t)v.cap_blocks * v.B), 1);
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
    d.summary = summary;
    d.sum_shift = v.L > 17 ? v.L - 17 : 0u;
    d.sum_words = (uint32_t)std::max<uint64_t>(((ncap >> d.sum_shift) + 31) / 32, 1);
    c.launch("vdel_summary", k_vd_summary, div_up(words, kThreads), kThreads, d, words);
    c.launch("vdel_scan", k_vd_scan, resident_grid(k_vd_scan, kThreads), kThreads, v, d);
    c.launch("vdel_sources", k_vd_sources, div_up(n, kThreads), kThreads, v, ids, n,
             (const uint8_t*)first, (const uint32_t*)gone);
    c.launch("vdel_plan", k_vd_plan, resident_grid(k_vd_plan, kThreads), kThreads, v, d);
    c.launch("vdel_holes", k_vd_holes, resident_grid(k_vd_holes, kThreads), kThreads, v, d);
    c.launch("vdel_fill", k_vd_fill, resident_grid(k_vd_fill, kThreads), kThreads, v, d);
    c.launch("vdel_finish", k_vdel_finish, div_up(n, kThreads), kThreads, g->v, ids, n,
             (const uint8_t*)first, (const uint32_t*)gone);
    if (st) {
        read_counters(g);
        st->applied = g->hctr->st_applied;
        st->rejected = g->hctr->st_rejected;
        st->batch_duplicates = n - g->hctr->st_rejected - g->hctr->n_uniq;
    }
}

}  // namespace gv
