// gv_edges.hip -- batched edge insert, delete and query.
//
// One pipeline serves the three operations (GraphVine Sec. 4.5-4.6, Alg. 1-3,
// re-designed for wave64):
//   pack      validate each pair against the activity bitmap and encode it as
//             a key (src << L) | dst; invalid pairs get a key above all valid
//             ones.  Queries also carry their input position.
//   sort      stable LSD radix sort of the keys on 2L+1 bits: the batch is
//             grouped by source and ordered by destination inside each source
//             segment (replaces the host CSR conversion of Sec. 4.3).
//   flags     segment heads (first key of a source) and first occurrences.
//   segments  the touched sources T with their segment start in the batch.
//   items     each touched adjacency is cut into work items of kChunk slots.
//   probe     one wave per work item streams the adjacency slots; each lane
//             binary-searches its slot value in the source's sorted segment.
//             Insert: marks batch entries that already exist (set semantics).
//             Delete: marks hits, remembers their slot and tombstones it.
//             Query:  marks every query equal to a stored edge.
//   insert:   keep = first occurrence and not present; scan; per-source block
//             demand and directory growth; one-thread allocation plan with a
//             capacity check before any write (all-or-nothing); blocks popped
//             from the free-list top first, then the bump pointer (the
//             prefix-sum pop of Sec. 4.5.1, without atomics); append.
//   delete:   per-source compaction pairs the holes below the new degree with
//             the survivors above it, by rank; emptied blocks are pushed on
//             the free list at scanned positions (reclamation, Sec. 4.2).
//   query:    answers are scattered back to input order.
#include <algorithm>

#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

constexpr uint8_t kHead = 1, kUniq = 2;

struct BatchArrays {
    uint64_t* keys0;
    uint64_t* keys1;
    uint32_t* vals0;
    uint32_t* vals1;
    uint8_t* flags;
    uint8_t* mark;
    uint32_t* a;        // n+1: exclusive count of segment heads
    uint32_t* b;        // n+1: exclusive count of kept (insert) / found (delete)
    uint32_t* hitpos;   // delete: slot index of each hit
    uint32_t* holes;    // delete: hole slots per segment
    uint32_t* t_vtx;    // touched source per segment
    uint32_t* t_start;  // n+1: segment start; t_start[n_T] = n_valid
    uint32_t* t_items;  // n+1: exclusive scan of work items per segment
    uint32_t* t_need;   // n+1: blocks needed (insert) / freed (delete), scanned
    uint32_t* t_dreq;   // insert: requested directory class or kNoDir
    uint32_t* t_drank;  // insert: rank among requests of that class
    uint32_t* t_dold;   // insert: replaced directory segment offset
    uint32_t* t_doldc;  // insert: replaced directory segment class or kNoDir
    uint2* items;       // (segment, chunk) work items
    uint32_t* partial;  // scan partials
    SortScratch sort;
};

static void carve_batch(Carver& cv, BatchArrays& A, uint64_t n, uint64_t icap, EdgeMode mode) {
    A = BatchArrays{};
    A.keys0 = cv.take<uint64_t>(n);
    A.keys1 = cv.take<uint64_t>(n);
    if (mode == kQuery) {
        A.vals0 = cv.take<uint32_t>(n);
        A.vals1 = cv.take<uint32_t>(n);
    }
    A.flags = cv.take<uint8_t>(n);
    A.mark = cv.take<uint8_t>(n);
    A.a = cv.take<uint32_t>(n + 1);
    A.b = cv.take<uint32_t>(n + 1);
    if (mode == kDelete) {
        A.hitpos = cv.take<uint32_t>(n);
        A.holes = cv.take<uint32_t>(n);
    }
    A.t_vtx = cv.take<uint32_t>(n);
    A.t_start = cv.take<uint32_t>(n + 1);
    A.t_items = cv.take<uint32_t>(n + 1);
    A.t_need = cv.take<uint32_t>(n + 1);
    if (mode == kInsert) {
        A.t_dreq = cv.take<uint32_t>(n);
        A.t_drank = cv.take<uint32_t>(n);
        A.t_dold = cv.take<uint32_t>(n);
        A.t_doldc = cv.take<uint32_t>(n);
    }
    A.items = cv.take<uint2>(icap);
    A.partial = cv.take<uint32_t>(scan_partials_needed(n + 1));
    carve_sort<uint64_t>(cv, A.sort, n);
}

__device__ __forceinline__ uint64_t thread_index() {
    return (uint64_t)blockIdx.x * kThreads + threadIdx.x;
}

__device__ __forceinline__ uint32_t global_wave() {
    return (uint32_t)(((uint64_t)blockIdx.x * kThreads + threadIdx.x) >> 6);
}

// ------------------------------------------------------------------ common
__global__ __launch_bounds__(kThreads) void k_pack(GraphView g, const uint32_t* src,
                                                   const uint32_t* dst, uint64_t n,
                                                   uint64_t* keys, uint32_t* vals, uint8_t* mark) {
    const uint64_t i = thread_index();
    if (i == 0) {
        g.ctr->err_batch = 0;
        g.ctr->n_uniq = 0;
    }
    if (i >= n) return;
    const uint32_t s = src[i], d = dst[i];
    const bool ok = is_active(g, s) && is_active(g, d);
    keys[i] = ok ? (((uint64_t)s << g.L) | d) : (1ull << (2 * g.L));
    if (vals) vals[i] = (uint32_t)i;
    mark[i] = 0;
}

__global__ __launch_bounds__(kThreads) void k_flags(GraphView g, const uint64_t* keys, uint64_t n,
                                                    uint8_t* flags) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t i = thread_index();
    unsigned long long uniq_count = 0;
    if (i < n) {
        const uint64_t invalid = 1ull << (2 * g.L);
        const uint64_t k = keys[i];
        const bool valid = k < invalid;
        const uint64_t prev = i ? keys[i - 1] : 0;
        const bool head = valid && (i == 0 || (k >> g.L) != (prev >> g.L));
        const bool uniq = valid && (i == 0 || k != prev);
        flags[i] = (head ? kHead : 0) | (uniq ? kUniq : 0);
        uniq_count = uniq;
        const bool next_valid = (i + 1 < n) && keys[i + 1] < invalid;
        if (valid && !next_valid) g.ctr->n_valid = (uint32_t)(i + 1);
        if (i == 0 && !valid) g.ctr->n_valid = 0;
    }
    unsigned long long c = block_sum(uniq_count, lds);
    if (threadIdx.x == 0 && c) atomicAdd(&g.ctr->n_uniq, c);
}

struct HeadIn {
    const uint8_t* flags;
    uint64_t n;
    __device__ uint32_t operator()(uint64_t i) const { return i < n ? (flags[i] & kHead) : 0u; }
};

__global__ __launch_bounds__(kThreads) void k_segments(GraphView g, const uint64_t* keys,
                                                       const uint8_t* flags, const uint32_t* a,
                                                       uint64_t n, uint32_t* t_vtx,
                                                       uint32_t* t_start) {
    const uint64_t i = thread_index();
    if (i >= n) return;
    const uint32_t nv = g.ctr->n_valid;
    if (i == 0 && nv == 0) t_start[0] = 0;
    if (i < nv && (flags[i] & kHead)) {
        const uint32_t t = a[i];
        t_vtx[t] = (uint32_t)(keys[i] >> g.L);
        t_start[t] = (uint32_t)i;
    }
    if (nv > 0 && i == nv - 1) t_start[g.ctr->n_T] = nv;
}

struct ItemIn {
    GraphView g;
    const uint32_t* t_vtx;
    __device__ uint32_t operator()(uint64_t t) const {
        if (t >= g.ctr->n_T) return 0u;
        const uint32_t d = g.vt[t_vtx[t]].deg;
        return (d + kChunk - 1) / kChunk;
    }
};

__global__ __launch_bounds__(kThreads) void k_expand(GraphView g, const uint32_t* t_vtx,
                                                     const uint32_t* t_items, uint64_t n,
                                                     uint2* items, int mode) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t t = thread_index();
    const uint32_t nT = g.ctr->n_T;
    unsigned long long slots = 0;
    if (t < nT) {
        const uint32_t d = g.vt[t_vtx[t]].deg;
        const uint32_t cnt = (d + kChunk - 1) / kChunk;
        const uint32_t base = t_items[t];
        for (uint32_t c = 0; c < cnt; ++c) items[base + c] = make_uint2((uint32_t)t, c);
        slots = (unsigned long long)nblocks(g, d) << g.log2B;
    }
    slots = block_sum(slots, lds);
    if (threadIdx.x == 0 && slots) atomicAdd(&g.ctr->c_scanned[mode], slots);
    if (t == 0) {
        g.ctr->c_touched[mode] += nT;
        g.ctr->c_batches[mode] += 1;
        g.ctr->c_pairs[mode] += n;
    }
}

// One wave per work item: lanes stream consecutive slots of one adjacency and
// binary-search them in the source's sorted batch segment.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_probe(GraphView g, const uint64_t* keys,
                                                    const uint32_t* t_vtx, const uint32_t* t_start,
                                                    const uint2* items, uint8_t* mark,
                                                    uint32_t* hitpos) {
    const uint32_t nitems = g.ctr->n_items;
    const uint32_t lane = lane_id();
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t it = global_wave(); it < nitems; it += nw) {
        const uint2 item = items[it];
        const uint32_t t = item.x;
        const uint32_t v = t_vtx[t];
        const VRec r = g.vt[v];
        const uint32_t lo = t_start[t], hi = t_start[t + 1];
        const uint32_t s0 = item.y * kChunk;
        const uint32_t s1 = min(r.deg, s0 + kChunk);
        const uint64_t vbase = (uint64_t)v << g.L;
        for (uint32_t s = s0 + lane; s < s1; s += 64) {
            const uint64_t addr = slot_addr(g, r, s);
            const uint32_t x = g.pool[addr];
            const uint64_t target = vbase | x;
            const uint32_t pos = lower_bound(keys, lo, hi, target);
            if (pos < hi && keys[pos] == target) {
                if (MODE == kInsert) {
                    mark[pos] = 1;
                } else if (MODE == kDelete) {
                    mark[pos] = 1;
                    hitpos[pos] = s;
                    g.pool[addr] = kTomb;
                } else {
                    for (uint32_t j = pos; j < hi && keys[j] == target; ++j) mark[j] = 1;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ insert
struct KeepIn {
    const uint8_t* flags;
    const uint8_t* mark;
    const DevCounters* ctr;
    __device__ uint32_t operator()(uint64_t i) const {
        if (i >= ctr->n_valid) return 0u;
        return ((flags[i] & kUniq) && !mark[i]) ? 1u : 0u;
    }
};

__global__ __launch_bounds__(kThreads) void k_plan_ins(GraphView g, const uint32_t* t_vtx,
                                                       const uint32_t* t_start, const uint32_t* b,
                                                       uint32_t* t_need, uint32_t* t_dreq,
                                                       uint32_t* t_drank) {
    __shared__ uint32_t lcnt[kMaxClass];
    __shared__ uint32_t lbase[kMaxClass];
    if (threadIdx.x < kMaxClass) lcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t = thread_index();
    const uint32_t nT = g.ctr->n_T;
    uint32_t cls = kNoDir, lrank = 0;
    if (t < nT) {
        const uint32_t kp = b[t_start[t + 1]] - b[t_start[t]];
        const VRec r = g.vt[t_vtx[t]];
        const uint32_t nb0 = nblocks(g, r.deg), nb1 = nblocks(g, r.deg + kp);
        t_need[t] = nb1 - nb0;
        const uint64_t cap0 = r.dcls == kNoDir ? 1ull : (1ull << r.dcls);
        if (nb1 > cap0) {
            cls = ceil_log2(nb1);
            lrank = atomicAdd(&lcnt[cls], 1u);
        }
        t_dreq[t] = cls;
    }
    __syncthreads();
    if (threadIdx.x < kMaxClass) {
        const uint32_t c = lcnt[threadIdx.x];
        lbase[threadIdx.x] = c ? atomicAdd(&g.ctr->dreq[threadIdx.x], c) : 0u;
    }
    __syncthreads();
    if (t < nT && cls != kNoDir) t_drank[t] = lbase[cls] + lrank;
}

struct NeedIn {
    const uint32_t* t_need;
    const DevCounters* ctr;
    __device__ uint32_t operator()(uint64_t t) const { return t < ctr->n_T ? t_need[t] : 0u; }
};

// Allocation plan for the whole batch, one thread: capacity is checked
// before any state is written, so a failing batch leaves the graph unchanged.
__global__ void k_plan(GraphView g, uint64_t n, int sticky) {
    DevCounters* c = g.ctr;
    const unsigned long long N = c->sum_b;
    const unsigned long long ff = N < c->free_cnt ? N : c->free_cnt;
    const unsigned long long fb = N - ff;
    bool ok = c->bump + fb <= g.cap_blocks;
    unsigned long long db = c->dir_bump;
    for (int k = 0; k < kMaxClass; ++k) {
        const uint32_t req = c->dreq[k];
        const uint32_t dff = req < c->dfree_cnt[k] ? req : c->dfree_cnt[k];
        c->plan_dff[k] = dff;
        c->plan_dbump[k] = db;
        db += (unsigned long long)(req - dff) << k;
    }
    ok = ok && db <= g.dir_cap;
    if (!ok) {
        c->err_batch = GV_ENOMEM;
        if (sticky && !c->err_sticky) c->err_sticky = GV_ENOMEM;
        for (int k = 0; k < kMaxClass; ++k) c->dreq[k] = 0;
        c->st_applied = c->st_rejected = c->st_dups = 0;
        return;
    }
    c->plan_free_top = c->free_cnt;
    c->plan_from_free = ff;
    c->plan_bump0 = c->bump;
    c->free_cnt -= ff;
    c->bump += fb;
    unsigned long long live = 0;
    for (int k = 0; k < kMaxClass; ++k) {
        c->plan_dtop[k] = c->dfree_cnt[k];
        c->dfree_cnt[k] -= c->plan_dff[k];
        live += (unsigned long long)c->dreq[k] << k;
        c->dreq[k] = 0;
    }
    c->dir_bump = db;
    c->dir_live += live;
    c->st_applied = c->sum_a;
    c->st_rejected = n - c->n_valid;
    c->st_dups = c->n_valid - c->n_uniq;
    c->c_new_blocks += N;
    c->c_written += c->sum_a;
    c->live_edges += c->sum_a;
}

// One wave per touched source: grow its directory segment if needed (copy the
// old entries) and record the ids of its new blocks.
__global__ __launch_bounds__(kThreads) void k_grow(GraphView g, const uint32_t* t_vtx,
                                                   const uint32_t* t_start, const uint32_t* b,
                                                   const uint32_t* t_need, const uint32_t* t_dreq,
                                                   const uint32_t* t_drank, uint32_t* t_dold,
                                                   uint32_t* t_doldc) {
    const DevCounters* c = g.ctr;
    if (c->err_batch) return;
    const uint32_t nT = c->n_T;
    const uint32_t lane = lane_id();
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t t = global_wave(); t < nT; t += nw) {
        const uint32_t v = t_vtx[t];
        const VRec r = g.vt[v];
        const uint32_t kp = b[t_start[t + 1]] - b[t_start[t]];
        const uint32_t nb0 = nblocks(g, r.deg), nb1 = nblocks(g, r.deg + kp);
        const uint32_t cls = t_dreq[t];
        VRec nr = r;
        if (cls != kNoDir) {
            const uint32_t rk = t_drank[t];
            uint32_t off;
            if (rk < c->plan_dff[cls])
                off = g.dfree[g.dfree_base[cls] + c->plan_dtop[cls] - 1 - rk];
            else
                off = (uint32_t)(c->plan_dbump[cls] +
                                 ((unsigned long long)(rk - c->plan_dff[cls]) << cls));
            for (uint32_t j = lane; j < nb0; j += 64) g.dir[(uint64_t)off + j] = block_of(g, r, j);
            if (lane == 0) {
                t_dold[t] = r.dir;
                t_doldc[t] = r.dcls;
            }
            nr.dir = off;
            nr.dcls = cls;
        } else if (lane == 0) {
            t_doldc[t] = kNoDir;
        }
        const uint64_t p0 = t_need[t];
        for (uint32_t j = nb0 + lane; j < nb1; j += 64) {
            const uint64_t p = p0 + (j - nb0);
            const uint32_t id = p < c->plan_from_free
                                    ? g.free_stack[c->plan_free_top - 1 - p]
                                    : (uint32_t)(c->plan_bump0 + (p - c->plan_from_free));
            if (nr.dcls == kNoDir) nr.dir = id;  // inline: only block 0, lane 0
            else g.dir[(uint64_t)nr.dir + j] = id;
        }
        if (lane == 0) g.vt[v] = nr;
    }
}

__global__ __launch_bounds__(kThreads) void k_append(GraphView g, const uint64_t* keys,
                                                     const uint8_t* flags, const uint8_t* mark,
                                                     const uint32_t* a, const uint32_t* b,
                                                     const uint32_t* t_vtx,
                                                     const uint32_t* t_start) {
    if (g.ctr->err_batch) return;
    const uint64_t i = thread_index();
    if (i >= g.ctr->n_valid) return;
    const uint8_t f = flags[i];
    if (!(f & kUniq) || mark[i]) return;
    const uint32_t t = a[i] + (f & kHead) - 1;
    const uint32_t v = t_vtx[t];
    const VRec r = g.vt[v];
    const uint32_t s = r.deg + (b[i] - b[t_start[t]]);
    g.pool[slot_addr(g, r, s)] = (uint32_t)(keys[i] & ((1ull << g.L) - 1));
}

__global__ __launch_bounds__(kThreads) void k_final_ins(GraphView g, const uint32_t* t_vtx,
                                                        const uint32_t* t_start, const uint32_t* b,
                                                        const uint32_t* t_dreq,
                                                        const uint32_t* t_dold,
                                                        const uint32_t* t_doldc) {
    if (g.ctr->err_batch) return;
    const uint64_t t = thread_index();
    if (t >= g.ctr->n_T) return;
    const uint32_t kp = b[t_start[t + 1]] - b[t_start[t]];
    const uint32_t v = t_vtx[t];
    if (kp) g.vt[v].deg += kp;
    if (t_dreq[t] != kNoDir) {
        const uint32_t oc = t_doldc[t];
        if (oc != kNoDir) {
            const uint32_t pos = atomicAdd(&g.ctr->dfree_cnt[oc], 1u);
            g.dfree[g.dfree_base[oc] + pos] = t_dold[t];
            atomicAdd(&g.ctr->dir_live, (unsigned long long)(-(long long)(1ull << oc)));
        }
    }
}

// ------------------------------------------------------------------ delete
struct FoundIn {
    const uint8_t* mark;
    const DevCounters* ctr;
    __device__ uint32_t operator()(uint64_t i) const {
        return i < ctr->n_valid ? (uint32_t)mark[i] : 0u;
    }
};

struct FreedIn {
    GraphView g;
    const uint32_t* t_vtx;
    const uint32_t* t_start;
    const uint32_t* b;
    __device__ uint32_t operator()(uint64_t t) const {
        if (t >= g.ctr->n_T) return 0u;
        const uint32_t r = b[t_start[t + 1]] - b[t_start[t]];
        if (!r) return 0u;
        const uint32_t d = g.vt[t_vtx[t]].deg;
        return nblocks(g, d) - nblocks(g, d - r);
    }
};

// One wave per touched source with hits: holes below the new degree (in
// batch order) receive the survivors found above it (in slot order).
__global__ __launch_bounds__(kThreads) void k_compact(GraphView g, const uint8_t* mark,
                                                      const uint32_t* hitpos, uint32_t* holes,
                                                      const uint32_t* b, const uint32_t* t_vtx,
                                                      const uint32_t* t_start,
                                                      const uint32_t* t_need) {
    const DevCounters* c = g.ctr;
    const uint32_t nT = c->n_T;
    const uint32_t lane = lane_id();
    const uint32_t nw = gridDim.x * kWaves;
    const unsigned long long fbase = c->free_cnt;
    unsigned long long moved = 0;
    for (uint32_t t = global_wave(); t < nT; t += nw) {
        const uint32_t lo = t_start[t], hi = t_start[t + 1];
        const uint32_t r = b[hi] - b[lo];
        if (!r) continue;
        const uint32_t v = t_vtx[t];
        const VRec rec = g.vt[v];
        const uint32_t d = rec.deg, dn = d - r;
        uint32_t nh = 0;
        for (uint32_t p0 = lo; p0 < hi; p0 += 64) {
            const uint32_t p = p0 + lane;
            bool hole = false;
            uint32_t hp = 0;
            if (p < hi && mark[p]) {
                hp = hitpos[p];
                hole = hp < dn;
            }
            const uint64_t m = ballot(hole);
            if (hole) holes[lo + nh + rank_below(m)] = hp;
            nh += popc64(m);
        }
        __threadfence_block();
        uint32_t ns = 0;
        for (uint32_t s0 = dn; s0 < d; s0 += 64) {
            const uint32_t s = s0 + lane;
            uint32_t x = kTomb;
            if (s < d) x = g.pool[slot_addr(g, rec, s)];
            const bool surv = x != kTomb;
            const uint64_t m = ballot(surv);
            if (surv) {
                // survivors above dn and holes below it are equal in number;
                // the guards only keep a broken invariant from writing wild
                const uint32_t q = ns + rank_below(m);
                if (q < nh) {
                    const uint32_t dest = holes[lo + q];
                    if (dest < dn) g.pool[slot_addr(g, rec, dest)] = x;
                }
            }
            ns += popc64(m);
        }
        moved += ns;
        const uint32_t nb0 = nblocks(g, d), nb1 = nblocks(g, dn);
        const unsigned long long pb = fbase + t_need[t];
        for (uint32_t j = nb1 + lane; j < nb0; j += 64)
            g.free_stack[pb + (j - nb1)] = block_of(g, rec, j);
        if (lane == 0) {
            VRec nr = rec;
            nr.deg = dn;
            if (nb1 == 0 && nr.dcls == kNoDir) nr.dir = 0;
            g.vt[v] = nr;
        }
    }
    if (lane == 0 && moved) atomicAdd(&g.ctr->c_moved, moved);
}

__global__ void k_final_del(GraphView g, uint64_t n) {
    DevCounters* c = g.ctr;
    c->free_cnt += c->sum_b;
    c->st_applied = c->sum_a;
    c->st_rejected = n - c->n_valid;
    c->st_dups = c->n_valid - c->n_uniq;
    c->c_freed_blocks += c->sum_b;
    c->live_edges -= c->sum_a;
}

// ------------------------------------------------------------------ query
__global__ __launch_bounds__(kThreads) void k_answer(GraphView g, const uint32_t* vals,
                                                     const uint8_t* mark, uint64_t n,
                                                     uint8_t* out) {
    const uint64_t i = thread_index();
    if (i >= n) return;
    out[vals[i]] = i < g.ctr->n_valid ? mark[i] : (uint8_t)0;
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }
__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

void set_u32(gv_graph* g, uint32_t* p, uint32_t value) {
    g->ctx.launch("set", k_set_u32, 1, 1, p, value);
}

void set_u64(gv_graph* g, unsigned long long* p, unsigned long long value) {
    g->ctx.launch("set", k_set_u64, 1, 1, p, value);
}

// ------------------------------------------------------------------ driver
void edge_batch(gv_graph* g, EdgeMode mode, const uint32_t* src, const uint32_t* dst, uint64_t n,
                uint8_t* out, bool sticky) {
    if (n == 0) return;
    if (n >= 0xffffffffull) fail(GV_EINVAL, "batch too large");
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    const uint64_t icap = n + div_up(g->item_slots, kChunk) + 1;
    BatchArrays A;
    {
        Carver m(nullptr);
        carve_batch(m, A, n, icap, mode);
        g->scratch.ensure(m.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve_batch(cv, A, n, icap, mode);
    }
    const uint64_t grid = div_up(n, kThreads);
    c.launch("pack", k_pack, grid, kThreads, v, src, dst, n, A.keys0,
             mode == kQuery ? A.vals0 : (uint32_t*)nullptr, A.mark);
    const int bits = 2 * (int)v.L + 1;
    bool flip;
    if (mode == kQuery)
        flip = radix_sort<uint64_t, true>(c, A.keys0, A.keys1, A.vals0, A.vals1, n, bits, A.sort);
    else
        flip = radix_sort<uint64_t, false>(c, A.keys0, A.keys1, nullptr, nullptr, n, bits, A.sort);
    const uint64_t* keys = flip ? A.keys1 : A.keys0;
    const uint32_t* vals = flip ? A.vals1 : A.vals0;

    c.launch("flags", k_flags, grid, kThreads, v, keys, n, A.flags);
    scan_excl<uint32_t>(c, HeadIn{A.flags, n}, ArrOut<uint32_t>{A.a}, n + 1, A.partial,
                        &v.ctr->n_T);
    c.launch("segments", k_segments, grid, kThreads, v, keys, (const uint8_t*)A.flags,
             (const uint32_t*)A.a, n, A.t_vtx, A.t_start);
    scan_excl<uint32_t>(c, ItemIn{v, A.t_vtx}, ArrOut<uint32_t>{A.t_items}, n + 1, A.partial,
                        &v.ctr->n_items);
    c.launch("expand", k_expand, grid, kThreads, v, (const uint32_t*)A.t_vtx,
             (const uint32_t*)A.t_items, n, A.items, (int)mode);
    const uint64_t pgrid = std::min<uint64_t>(div_up(icap, kWaves), 2048);
    const uint64_t tgrid = std::min<uint64_t>(div_up(n, kWaves), 2048);

    if (mode == kInsert) {
        c.launch("probe_insert", k_probe<kInsert>, pgrid, kThreads, v, keys,
                 (const uint32_t*)A.t_vtx, (const uint32_t*)A.t_start, (const uint2*)A.items,
                 A.mark, (uint32_t*)nullptr);
        scan_excl<uint32_t>(c, KeepIn{A.flags, A.mark, v.ctr}, ArrOut<uint32_t>{A.b}, n + 1,
                            A.partial, &v.ctr->sum_a);
        c.launch("plan_insert", k_plan_ins, grid, kThreads, v, (const uint32_t*)A.t_vtx,
                 (const uint32_t*)A.t_start, (const uint32_t*)A.b, A.t_need, A.t_dreq, A.t_drank);
        scan_excl<uint32_t>(c, NeedIn{A.t_need, v.ctr}, ArrOut<uint32_t>{A.t_need}, n + 1,
                            A.partial, &v.ctr->sum_b);
        c.launch("plan", k_plan, 1, 1, v, n, (int)sticky);
        c.launch("grow", k_grow, tgrid, kThreads, v, (const uint32_t*)A.t_vtx,
                 (const uint32_t*)A.t_start, (const uint32_t*)A.b, (const uint32_t*)A.t_need,
                 (const uint32_t*)A.t_dreq, (const uint32_t*)A.t_drank, A.t_dold, A.t_doldc);
        c.launch("append", k_append, grid, kThreads, v, keys, (const uint8_t*)A.flags,
                 (const uint8_t*)A.mark, (const uint32_t*)A.a, (const uint32_t*)A.b,
                 (const uint32_t*)A.t_vtx, (const uint32_t*)A.t_start);
        c.launch("final_insert", k_final_ins, grid, kThreads, v, (const uint32_t*)A.t_vtx,
                 (const uint32_t*)A.t_start, (const uint32_t*)A.b, (const uint32_t*)A.t_dreq,
                 (const uint32_t*)A.t_dold, (const uint32_t*)A.t_doldc);
    } else if (mode == kDelete) {
        c.launch("probe_delete", k_probe<kDelete>, pgrid, kThreads, v, keys,
                 (const uint32_t*)A.t_vtx, (const uint32_t*)A.t_start, (const uint2*)A.items,
                 A.mark, A.hitpos);
        scan_excl<uint32_t>(c, FoundIn{A.mark, v.ctr}, ArrOut<uint32_t>{A.b}, n + 1, A.partial,
                            &v.ctr->sum_a);
        scan_excl<uint32_t>(c, FreedIn{v, A.t_vtx, A.t_start, A.b}, ArrOut<uint32_t>{A.t_need},
                            n + 1, A.partial, &v.ctr->sum_b);
        c.launch("compact", k_compact, tgrid, kThreads, v, (const uint8_t*)A.mark,
                 (const uint32_t*)A.hitpos, A.holes, (const uint32_t*)A.b,
                 (const uint32_t*)A.t_vtx, (const uint32_t*)A.t_start, (const uint32_t*)A.t_need);
        c.launch("final_delete", k_final_del, 1, 1, v, n);
    } else {
        c.launch("probe_query", k_probe<kQuery>, pgrid, kThreads, v, keys,
                 (const uint32_t*)A.t_vtx, (const uint32_t*)A.t_start, (const uint2*)A.items,
                 A.mark, (uint32_t*)nullptr);
        c.launch("answer", k_answer, grid, kThreads, v, vals, (const uint8_t*)A.mark, n, out);
    }
}

}  // namespace gv
