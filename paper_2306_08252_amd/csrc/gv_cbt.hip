// gv_cbt.hip -- the paper's own layout and algorithms on the same device
// pool, as an ablation beside the directory path (GraphVine Sec. 4.1-4.6).
//
//   Layout (Sec. 4.1, Fig. 2).  Each vertex's edge blocks form a complete
//   binary tree (CBT): block k of the vertex (1-based, in the order blocks
//   were attached) sits at level-order position k, so its parent is block
//   k / 2 and it is that parent's left (k even) or right (k odd) child.  Each
//   block carries two child links beside its B slots.  A vertex's sentinel
//   holds its live edge count, the root block, the block count, the last
//   block and how many slots of the last block have been used (the last
//   insert offset).
//   Placement (Sec. 4.5.1, Fig. 4).  A new block k is attached by its bit
//   string, the binary form of k without its leading 1: every bit but the
//   last is a step from the root (0 left, 1 right) and the last bit says
//   which child of the reached block it becomes; the paper's example, the
//   9th block, gets 001.
//   Edge queue (Sec. 4.2, Sec. 4.5.1).  Pre-allocated block ids handed out
//   from a front pointer; every vertex pops its blocks at the position the
//   prefix sum of the blocks all vertices need gives it (one entry per
//   vertex of the graph), with no atomics.  Deleted edges leave holes and no
//   block goes back (Sec. 4.5.2).
//   Insert (Alg. 1), delete (Alg. 2): one thread per vertex of the graph.
//   The batch is grouped by source first (the CSR form the paper expects).
//   Insert appends after the last insert offset, then into the new blocks in
//   level order; delete traverses the tree in order and tombstones matches.
//   Query (Alg. 3): one thread per query collects its source's blocks by an
//   in-order traversal, then one thread per slot of those blocks compares.
//
// Readings shared with the directory path: set semantics (a stored pair is
// not inserted again, repeated pairs in a batch count once, absent deletes
// are no-ops), pairs with an endpoint outside the graph are rejected.  The
// membership test of a slot against the source's batch entries is a binary
// search over its sorted batch segment (the paper's Alg. 2 compares every
// pair: the same result).
#include <algorithm>
#include <cstring>
#include <new>

#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

constexpr uint32_t kCbtNone = 0xFFFFFFFFu;  // no child / no block

struct CbtVert {
    uint32_t live;   // live edges (holes excluded)
    uint32_t root;   // root block id, or kCbtNone
    uint32_t nblk;   // blocks in the tree
    uint32_t last;   // block holding the last inserted edge (level-order position nblk)
    uint32_t used;   // slots used in the last block (the last insert offset)
    uint32_t pad[3];
};

struct CbtView {
    uint32_t* pool;        // cap_blocks * B slots
    uint32_t* child;       // 2 per block: left, right
    const uint32_t* queue; // the edge queue: block ids in pop order
    CbtVert* vt;           // n_cap sentinels
    unsigned long long* ctr;  // [0] front of the queue, [1] error, [2..] batch totals
    uint64_t n, n_cap, cap_blocks;
    uint32_t B, log2B, L;
};

enum { kCbtFront = 0, kCbtErr = 1, kCbtApplied = 2, kCbtValid = 3, kCbtDistinct = 4,
       kCbtNeed = 5, kCbtSortErr = 6, kCbtWords = 8 };

}  // namespace gv

struct gv_cbt {
    int device = 0;
    gv::Ctx ctx;
    gv::CbtView v{};
    void* mem_pool = nullptr;
    void* mem_child = nullptr;
    void* mem_queue = nullptr;
    void* mem_vt = nullptr;
    void* mem_ctr = nullptr;
    unsigned long long* hctr = nullptr;
    gv::Scratch scratch;
    bool dead = false;
};

namespace gv {

// Bit string of level-order position k >= 1 (the path from the root): the
// binary form of k without its leading 1, most significant bit first.
__host__ __device__ inline int cbt_bits(uint64_t k) {
    int b = 0;
    while ((k >> (b + 1)) != 0) ++b;
    return b;  // number of path bits
}

// Block at level-order position k (1 <= k <= nblk) of a tree rooted at root.
__device__ __forceinline__ uint32_t cbt_find(const CbtView& g, uint32_t root, uint32_t k) {
    uint32_t node = root;
    for (int b = cbt_bits(k) - 1; b >= 0; --b) node = g.child[2ull * node + ((k >> b) & 1u)];
    return node;
}

// In-order traversal of the tree of a vertex (left subtree, block, right
// subtree) with an explicit stack; visit(block id, level-order position).
template <typename F>
__device__ __forceinline__ void cbt_inorder(const CbtView& g, uint32_t root, uint32_t nblk, F&& visit) {
    if (root == kCbtNone || nblk == 0) return;
    uint32_t st_id[32], st_k[32];
    int sp = 0;
    uint32_t node = root, k = 1;
    while (true) {
        while (node != kCbtNone && k <= nblk) {
            st_id[sp] = node;
            st_k[sp] = k;
            ++sp;
            node = g.child[2ull * node];
            k = 2 * k;
        }
        if (sp == 0) break;
        --sp;
        node = st_id[sp];
        k = st_k[sp];
        visit(node, k);
        node = g.child[2ull * node + 1];
        k = 2 * k + 1;
    }
}

// slots of block at position k that hold edges (or holes): all B but the last block's
__device__ __forceinline__ uint32_t cbt_slots(const CbtView& g, const CbtVert& r, uint32_t k) {
    return k == r.nblk ? r.used : g.B;
}

// first index in keys[lo, hi) whose value is >= x
__device__ __forceinline__ uint32_t seg_lower(const uint64_t* keys, uint32_t lo, uint32_t hi, uint64_t x) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ grouping
__global__ __launch_bounds__(kThreads) void k_cbt_pack(CbtView g, const uint32_t* src,
                                                       const uint32_t* dst, uint64_t n,
                                                       uint64_t sentinel, uint64_t* keys,
                                                       uint8_t* mark) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i == 0)
        for (int k = kCbtApplied; k < kCbtWords; ++k) g.ctr[k] = 0;
    if (i >= n) return;
    const uint32_t s = src[i], d = dst[i];
    const bool ok = s < g.n && d < g.n;
    keys[i] = ok ? ((uint64_t)s << g.L) | d : sentinel;
    mark[i] = 0;
}

// CSR offsets of the sorted batch: off[v] = first key with source >= v
// (invalid pairs sort after every valid key); also counts the valid and the
// distinct valid pairs
__global__ __launch_bounds__(kThreads) void k_cbt_offsets(CbtView g, const uint64_t* keys,
                                                          uint64_t n, uint64_t sentinel,
                                                          uint32_t* off) {
    const uint64_t v = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v <= g.n_cap) off[v] = seg_lower(keys, 0, (uint32_t)n, v < g.n_cap ? v << g.L : sentinel);
    if (v < n) {
        const bool valid = keys[v] != sentinel;
        const bool distinct = valid && (v == 0 || keys[v - 1] != keys[v]);
        const uint64_t bv = ballot(valid), bd = ballot(distinct);
        if (lane_id() == 0) {
            if (bv) atomicAdd(&g.ctr[kCbtValid], (unsigned long long)popc64(bv));
            if (bd) atomicAdd(&g.ctr[kCbtDistinct], (unsigned long long)popc64(bd));
        }
    }
}

// ------------------------------------------------------------------ insert
// Alg. 1, first part, one thread per vertex: mark the batch entries already
// stored (in-order traversal of the tree, each slot looked up in the sorted
// batch segment) and count the blocks the new entries need past the space
// remaining in the last block.
__global__ __launch_bounds__(kThreads) void k_cbt_need(CbtView g, const uint64_t* keys,
                                                       const uint32_t* off, uint8_t* mark,
                                                       uint32_t* need, uint32_t* fresh) {
    const uint64_t v = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= g.n_cap) return;
    const uint32_t lo = off[v], hi = off[v + 1];
    uint32_t nb = 0, nf = 0;
    if (lo < hi) {
        const CbtVert r = g.vt[v];
        const uint64_t vb = v << g.L;
        cbt_inorder(g, r.root, r.nblk, [&](uint32_t blk, uint32_t k) {
            const uint32_t ns = cbt_slots(g, r, k);
            for (uint32_t s = 0; s < ns; ++s) {
                const uint32_t x = g.pool[((uint64_t)blk << g.log2B) + s];
                if (x == kTomb) continue;
                const uint32_t p = seg_lower(keys, lo, hi, vb | x);
                if (p < hi && keys[p] == (vb | x)) mark[p] = 1;
            }
        });
        for (uint32_t i = lo; i < hi; ++i)
            if (!mark[i] && (i == lo || keys[i] != keys[i - 1])) ++nf;
        const uint32_t room = r.nblk ? g.B - r.used : 0u;  // space remaining (Sec. 4.5.1)
        nb = nf > room ? (nf - room + g.B - 1) >> g.log2B : 0u;
    }
    need[v] = nb;
    fresh[v] = nf;
}

struct U32SumIn {
    const uint32_t* a;
    uint64_t n;
    __device__ unsigned long long operator()(uint64_t i) const { return i < n ? a[i] : 0u; }
};

// capacity check before any state changes (all or nothing)
__global__ void k_cbt_check(CbtView g, const unsigned long long* total) {
    if (g.ctr[kCbtFront] + *total > g.cap_blocks) g.ctr[kCbtErr] = GV_ENOMEM;
}

// Alg. 1, second part, one thread per vertex: pop the blocks at the prefix
// position, attach each by its bit string, append the new entries after the
// last insert offset and then through the new blocks in level order.
__global__ __launch_bounds__(kThreads) void k_cbt_insert(CbtView g, const uint64_t* keys,
                                                         const uint32_t* off, const uint8_t* mark,
                                                         const uint32_t* need,
                                                         const unsigned long long* pre,
                                                         const uint32_t* fresh) {
    const uint64_t v = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= g.n_cap || g.ctr[kCbtErr]) return;
    const uint32_t nf = fresh[v];
    if (nf == 0) return;
    CbtVert r = g.vt[v];
    const uint32_t nb = need[v];
    const unsigned long long q0 = g.ctr[kCbtFront] + pre[v];
    uint32_t first_new = kCbtNone;
    for (uint32_t j = 0; j < nb; ++j) {
        const uint32_t blk = g.queue[q0 + j];
        g.child[2ull * blk] = kCbtNone;
        g.child[2ull * blk + 1] = kCbtNone;
        const uint32_t k = r.nblk + 1 + j;
        if (k == 1) {
            r.root = blk;
        } else {
            // walk the bit string but its last bit from the root, attach there
            const uint32_t parent = cbt_find(g, r.root, k >> 1);
            g.child[2ull * parent + (k & 1u)] = blk;
        }
        if (j == 0) first_new = blk;
    }
    // append: the last block's free slots, then the new blocks in order
    uint32_t cur = r.nblk && r.used < g.B ? r.last : first_new;
    uint32_t used = r.nblk && r.used < g.B ? r.used : 0u;
    uint32_t j = r.nblk && r.used < g.B ? 0u : 1u;  // next new block to move to
    const uint32_t lo = off[v], hi = off[v + 1];
    for (uint32_t i = lo; i < hi; ++i) {
        if (mark[i] || (i > lo && keys[i] == keys[i - 1])) continue;
        if (used == g.B) {
            cur = g.queue[q0 + j];
            ++j;
            used = 0;
        }
        g.pool[((uint64_t)cur << g.log2B) + used] = (uint32_t)(keys[i] & ((1ull << g.L) - 1));
        ++used;
    }
    r.live += nf;
    r.nblk += nb;
    r.last = cur;
    r.used = used;
    g.vt[v] = r;
    atomicAdd(&g.ctr[kCbtApplied], (unsigned long long)nf);
}

// the edge queue's front moves past the popped blocks (Alg. 1, last line)
__global__ void k_cbt_front(CbtView g, const unsigned long long* total) {
    if (!g.ctr[kCbtErr]) g.ctr[kCbtFront] += *total;
}

// ------------------------------------------------------------------ delete
// Alg. 2, one thread per vertex: in-order traversal, every slot looked up in
// the source's batch segment; a match becomes a hole (tombstone).
__global__ __launch_bounds__(kThreads) void k_cbt_delete(CbtView g, const uint64_t* keys,
                                                         const uint32_t* off) {
    const uint64_t v = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= g.n_cap) return;
    const uint32_t lo = off[v], hi = off[v + 1];
    if (lo >= hi) return;
    CbtVert r = g.vt[v];
    const uint64_t vb = v << g.L;
    uint32_t removed = 0;
    cbt_inorder(g, r.root, r.nblk, [&](uint32_t blk, uint32_t k) {
        const uint32_t ns = cbt_slots(g, r, k);
        for (uint32_t s = 0; s < ns; ++s) {
            uint32_t* p = g.pool + ((uint64_t)blk << g.log2B) + s;
            const uint32_t x = *p;
            if (x == kTomb) continue;
            const uint32_t q = seg_lower(keys, lo, hi, vb | x);
            if (q < hi && keys[q] == (vb | x)) {
                *p = kTomb;
                ++removed;
            }
        }
    });
    if (removed) {
        r.live -= removed;
        g.vt[v].live = r.live;
        atomicAdd(&g.ctr[kCbtApplied], (unsigned long long)removed);
    }
}

// ------------------------------------------------------------------ query
// Alg. 3: blocks per query (scanned for positions), one thread per query
// collecting its source's blocks in order, one thread per slot comparing.
__global__ __launch_bounds__(kThreads) void k_cbt_qcount(CbtView g, const uint32_t* src,
                                                         const uint32_t* dst, uint64_t n,
                                                         uint32_t* nblk, uint8_t* out) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = src[i], d = dst[i];
    nblk[i] = (s < g.n && d < g.n) ? g.vt[s].nblk : 0u;
    out[i] = 0;
}

__global__ __launch_bounds__(kThreads) void k_cbt_qcollect(CbtView g, const uint32_t* src,
                                                           const uint32_t* nblk, uint64_t n,
                                                           const unsigned long long* pos,
                                                           uint32_t* blocks, uint32_t* usedv) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n || nblk[i] == 0) return;
    const CbtVert r = g.vt[src[i]];
    unsigned long long p = pos[i];
    cbt_inorder(g, r.root, r.nblk, [&](uint32_t blk, uint32_t k) {
        blocks[p] = blk;
        usedv[p] = cbt_slots(g, r, k);
        ++p;
    });
}

// one thread per slot of the collected blocks: slot t of block entry e
__global__ __launch_bounds__(kThreads) void k_cbt_qcompare(CbtView g, const uint32_t* dst,
                                                           uint64_t n,
                                                           const unsigned long long* pos,
                                                           const unsigned long long* total,
                                                           const uint32_t* blocks,
                                                           const uint32_t* usedv, uint8_t* out) {
    const uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    const uint64_t e = t >> g.log2B;
    if (e >= *total) return;
    const uint32_t s = (uint32_t)(t & (g.B - 1));
    if (s >= usedv[e]) return;
    // the query whose blocks hold entry e: last query with pos <= e
    uint64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (pos[mid] <= e) lo = mid;
        else hi = mid;
    }
    const uint32_t x = g.pool[((uint64_t)blocks[e] << g.log2B) + s];
    if (x != kTomb && x == dst[lo]) out[lo] = 1;
}

// ------------------------------------------------------------------ dump
__global__ __launch_bounds__(kThreads) void k_cbt_count(CbtView g, uint32_t* cnt) {
    const uint64_t v = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v < g.n_cap) cnt[v] = g.vt[v].live;
}

__global__ __launch_bounds__(kThreads) void k_cbt_gather(CbtView g,
                                                         const unsigned long long* offs,
                                                         uint64_t* keys) {
    const uint64_t v = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v >= g.n_cap) return;
    const CbtVert r = g.vt[v];
    unsigned long long p = offs[v];
    const uint64_t vb = v << g.L;
    cbt_inorder(g, r.root, r.nblk, [&](uint32_t blk, uint32_t k) {
        const uint32_t ns = cbt_slots(g, r, k);
        for (uint32_t s = 0; s < ns; ++s) {
            const uint32_t x = g.pool[((uint64_t)blk << g.log2B) + s];
            if (x != kTomb) keys[p++] = vb | x;
        }
    });
}

__global__ __launch_bounds__(kThreads) void k_cbt_extract(const uint64_t* keys, uint64_t n,
                                                          uint32_t L, uint32_t* dst) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) dst[i] = (uint32_t)(keys[i] & ((1ull << L) - 1));
}

__global__ __launch_bounds__(kThreads) void k_cbt_iota(uint32_t* q, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) q[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kThreads) void k_cbt_init_vt(CbtVert* vt, uint64_t n) {
    const uint64_t v = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (v < n) vt[v] = CbtVert{0u, kCbtNone, 0u, kCbtNone, 0u, {0u, 0u, 0u}};
}

__global__ void k_cbt_zero_ctr(unsigned long long* c) {
    for (int k = 0; k < kCbtWords; ++k) c[k] = 0;
}

// ------------------------------------------------------------------ host
struct CbtArrays {
    uint64_t* keys0;
    uint64_t* keys1;
    uint8_t* mark;
    uint32_t* off;
    uint32_t* need;
    uint32_t* fresh;
    unsigned long long* pre;
    unsigned long long* part;
    uint32_t* state;
};

static void cbt_carve(Carver& cv, CbtArrays& A, uint64_t n, uint64_t n_cap, int bits) {
    A.keys0 = cv.take<uint64_t>(std::max<uint64_t>(n, 2));
    A.keys1 = cv.take<uint64_t>(std::max<uint64_t>(n, 2));
    A.mark = cv.take<uint8_t>(std::max<uint64_t>(n, 1));
    A.off = cv.take<uint32_t>(n_cap + 1);
    A.need = cv.take<uint32_t>(n_cap);
    A.fresh = cv.take<uint32_t>(n_cap);
    A.pre = cv.take<unsigned long long>(n_cap + 1);
    A.part = cv.take<unsigned long long>(scan_partials_needed(n_cap + 1));
    A.state = cv.take<uint32_t>(os_words(std::max<uint64_t>(n, 2), bits));
}

// the batch keys are sorted over 2L + 1 bits: an invalid pair gets bit 2L,
// above every valid key (src << L) | dst
static int cbt_batch_bits(const CbtView& v) { return 2 * (int)v.L + 1; }

// Groups a batch by source (sorted keys, CSR offsets per vertex).  Returns the
// sorted keys.
static const uint64_t* cbt_group(gv_cbt* g, CbtArrays& A, const uint32_t* src,
                                 const uint32_t* dst, uint64_t n) {
    Ctx& c = g->ctx;
    const CbtView& v = g->v;
    const int bits = cbt_batch_bits(v);
    const uint64_t sentinel = 1ull << (2 * v.L);
    c.launch("cbt_pack", k_cbt_pack, div_up(n, kThreads), kThreads, v, src, dst, n, sentinel,
             A.keys0, A.mark);
    zero_words(c, A.state, os_zero_words(std::max<uint64_t>(n, 2), bits));
    const bool flip = onesweep<uint64_t, false>(c, A.keys0, A.keys1, nullptr, nullptr, nullptr, n,
                                                bits, A.state, (uint32_t*)&v.ctr[kCbtSortErr]);
    const uint64_t* keys = flip ? A.keys1 : A.keys0;
    c.launch("cbt_offsets", k_cbt_offsets, div_up(std::max<uint64_t>(v.n_cap + 1, n), kThreads),
             kThreads, v, keys, n, sentinel, A.off);
    return keys;
}

static void cbt_read(gv_cbt* g) {
    hip_check(hipMemcpyAsync(g->hctr, g->v.ctr, kCbtWords * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, g->ctx.stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(g->ctx.stream), "hipStreamSynchronize");
    if (g->hctr[kCbtSortErr]) fail(GV_EDEVICE, "a batch sort's look-back wait ran out");
}

static void cbt_carve_for(gv_cbt* g, CbtArrays& A, uint64_t n) {
    const int bits = cbt_batch_bits(g->v);
    Carver m(nullptr);
    cbt_carve(m, A, n, g->v.n_cap, bits);
    g->scratch.ensure(m.used, g->ctx.stream);
    Carver cv(g->scratch.ptr);
    cbt_carve(cv, A, n, g->v.n_cap, bits);
}

static void cbt_stats(gv_cbt* g, uint64_t n, gv_batch_stats* st) {
    st->applied = g->hctr[kCbtApplied];
    st->rejected = n - g->hctr[kCbtValid];
    st->batch_duplicates = g->hctr[kCbtValid] - g->hctr[kCbtDistinct];
}

static void cbt_insert(gv_cbt* g, const uint32_t* src, const uint32_t* dst, uint64_t n,
                       gv_batch_stats* st) {
    if (n >= kOsMaxKeys) fail(GV_EINVAL, "batch too large");
    Ctx& c = g->ctx;
    const CbtView& v = g->v;
    CbtArrays A;
    cbt_carve_for(g, A, n);
    const uint64_t* keys = cbt_group(g, A, src, dst, n);
    const uint64_t vg = div_up(v.n_cap, kThreads);
    c.launch("cbt_need", k_cbt_need, vg, kThreads, v, keys, (const uint32_t*)A.off, A.mark,
             A.need, A.fresh);
    scan_excl<unsigned long long>(c, U32SumIn{A.need, v.n_cap}, ArrOut<unsigned long long>{A.pre},
                                  v.n_cap, A.part, (unsigned long long*)&v.ctr[kCbtNeed]);
    c.launch("cbt_check", k_cbt_check, 1, 1, v, (const unsigned long long*)&v.ctr[kCbtNeed]);
    c.launch("cbt_insert", k_cbt_insert, vg, kThreads, v, keys, (const uint32_t*)A.off,
             (const uint8_t*)A.mark, (const uint32_t*)A.need, (const unsigned long long*)A.pre,
             (const uint32_t*)A.fresh);
    c.launch("cbt_front", k_cbt_front, 1, 1, v, (const unsigned long long*)&v.ctr[kCbtNeed]);
    cbt_read(g);
    if (g->hctr[kCbtErr]) {
        // nothing was written: clear the flag, report the batch as refused
        hip_check(hipMemsetAsync(&v.ctr[kCbtErr], 0, sizeof(unsigned long long), c.stream),
                  "hipMemsetAsync");
        hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
        fail(GV_ENOMEM, "edge queue exhausted");
    }
    if (st) cbt_stats(g, n, st);
}

static void cbt_delete(gv_cbt* g, const uint32_t* src, const uint32_t* dst, uint64_t n,
                       gv_batch_stats* st) {
    if (n >= kOsMaxKeys) fail(GV_EINVAL, "batch too large");
    Ctx& c = g->ctx;
    const CbtView& v = g->v;
    CbtArrays A;
    cbt_carve_for(g, A, n);
    const uint64_t* keys = cbt_group(g, A, src, dst, n);
    c.launch("cbt_delete", k_cbt_delete, div_up(v.n_cap, kThreads), kThreads, v, keys,
             (const uint32_t*)A.off);
    cbt_read(g);
    if (st) cbt_stats(g, n, st);
}

static void cbt_query(gv_cbt* g, const uint32_t* src, const uint32_t* dst, uint64_t n,
                      uint8_t* out) {
    Ctx& c = g->ctx;
    const CbtView& v = g->v;
    uint32_t* nblk = nullptr;
    unsigned long long *pos = nullptr, *part = nullptr, *total = nullptr;
    uint32_t *blocks = nullptr, *usedv = nullptr;
    auto carve = [&](Carver& cv, uint64_t tot) {
        nblk = cv.take<uint32_t>(n);
        pos = cv.take<unsigned long long>(n + 1);
        part = cv.take<unsigned long long>(scan_partials_needed(n + 1));
        total = cv.take<unsigned long long>(1);
        blocks = cv.take<uint32_t>(std::max<uint64_t>(tot, 1));
        usedv = cv.take<uint32_t>(std::max<uint64_t>(tot, 1));
    };
    auto count = [&](uint64_t tot) {
        Carver m(nullptr);
        carve(m, tot);
        g->scratch.ensure(m.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve(cv, tot);
        c.launch("cbt_qcount", k_cbt_qcount, div_up(n, kThreads), kThreads, v, src, dst, n, nblk,
                 out);
        scan_excl<unsigned long long>(c, U32SumIn{nblk, n}, ArrOut<unsigned long long>{pos},
                                      n + 1, part, total);
        unsigned long long t = 0;
        hip_check(hipMemcpyAsync(&t, total, sizeof(t), hipMemcpyDeviceToHost, c.stream),
                  "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
        return (uint64_t)t;
    };
    // count the blocks of every query's source; then make room for the block
    // lists (counting again if the scratch had to grow)
    const uint64_t gen = g->scratch.gen;
    const uint64_t tot = count(0);
    if (tot == 0) return;
    {
        Carver m(nullptr);
        carve(m, tot);
        g->scratch.ensure(m.used, c.stream);
    }
    if (g->scratch.gen != gen) count(tot);
    Carver cv(g->scratch.ptr);
    carve(cv, tot);
    c.launch("cbt_qcollect", k_cbt_qcollect, div_up(n, kThreads), kThreads, v, src,
             (const uint32_t*)nblk, n, (const unsigned long long*)pos, blocks, usedv);
    c.launch("cbt_qcompare", k_cbt_qcompare, div_up(tot << v.log2B, kThreads), kThreads, v, dst, n,
             (const unsigned long long*)pos, (const unsigned long long*)total,
             (const uint32_t*)blocks, (const uint32_t*)usedv, out);
}

static void cbt_dump(gv_cbt* g, uint64_t* offsets, uint32_t* dst, uint64_t cap, uint64_t* edges) {
    Ctx& c = g->ctx;
    const CbtView& v = g->v;
    uint32_t* cnt = nullptr;
    unsigned long long* part = nullptr;
    unsigned long long* offs = (unsigned long long*)offsets;
    unsigned long long* total = nullptr;
    {
        auto carve = [&](Carver& cv) {
            cnt = cv.take<uint32_t>(v.n_cap);
            part = cv.take<unsigned long long>(scan_partials_needed(v.n_cap + 1));
            total = cv.take<unsigned long long>(1);
            if (!offsets) offs = cv.take<unsigned long long>(v.n_cap + 1);
        };
        Carver m(nullptr);
        carve(m);
        g->scratch.ensure(m.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve(cv);
    }
    c.launch("cbt_count", k_cbt_count, div_up(v.n_cap, kThreads), kThreads, v, cnt);
    scan_excl<unsigned long long>(c, U32SumIn{cnt, v.n_cap}, ArrOut<unsigned long long>{offs},
                                  v.n_cap + 1, part, total);
    unsigned long long e = 0;
    hip_check(hipMemcpyAsync(&e, total, sizeof(e), hipMemcpyDeviceToHost, c.stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    *edges = e;
    if (!dst || !offsets || e == 0) return;
    if (cap < e) fail(GV_ERANGE, "dump buffer too small");
    if (e >= kOsMaxKeys) fail(GV_EINVAL, "2^30 or more edges");
    // keys (u << L | x) at their vertex's CSR range, then one sort orders
    // every vertex's destinations (the offsets live in the caller's array)
    const int bits = 2 * (int)v.L;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t* state = nullptr;
    {
        auto carve2 = [&](Carver& cv) {
            k0 = cv.take<uint64_t>(std::max<uint64_t>(e, 2));
            k1 = cv.take<uint64_t>(std::max<uint64_t>(e, 2));
            state = cv.take<uint32_t>(os_words(std::max<uint64_t>(e, 2), bits));
        };
        Carver m(nullptr);
        carve2(m);
        g->scratch.ensure(m.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve2(cv);
    }
    c.launch("cbt_gather", k_cbt_gather, div_up(v.n_cap, kThreads), kThreads, v,
             (const unsigned long long*)offs, k0);
    zero_words(c, state, os_zero_words(std::max<uint64_t>(e, 2), bits));
    const bool flip = onesweep<uint64_t, false>(c, k0, k1, nullptr, nullptr, nullptr, e, bits, state,
                                                (uint32_t*)&v.ctr[kCbtSortErr]);
    c.launch("cbt_extract", k_cbt_extract, div_up(e, kThreads), kThreads,
             (const uint64_t*)(flip ? k1 : k0), e, v.L, dst);
    cbt_read(g);
}

template <typename F>
int cbt_guarded(gv_cbt* g, F&& f) {
    if (!g) return GV_EINVAL;
    if (g->dead) return GV_EDEVICE;
    int prev = -1;
    try {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != g->device) hip_check(hipSetDevice(g->device), "hipSetDevice");
        f();
    } catch (const Error& e) {
        if (e.code == GV_EDEVICE) g->dead = true;
        if (prev >= 0 && prev != g->device) hipSetDevice(prev);
        return e.code;
    } catch (...) {
        g->dead = true;
        if (prev >= 0 && prev != g->device) hipSetDevice(prev);
        return GV_EDEVICE;
    }
    if (prev >= 0 && prev != g->device) hipSetDevice(prev);
    return GV_OK;
}

static void cbt_free(gv_cbt* g) {
    if (!g) return;
    hipStreamSynchronize(g->ctx.stream);
    g->ctx.release();
    g->scratch.release();
    void* mem[] = {g->mem_pool, g->mem_child, g->mem_queue, g->mem_vt, g->mem_ctr};
    for (void* p : mem)
        if (p) hipFree(p);
    if (g->hctr) hipHostFree(g->hctr);
    delete g;
}

}  // namespace gv

using namespace gv;

extern "C" {

int gv_cbt_bitstring(uint64_t k, char* out, uint64_t cap) {
    if (!out || k == 0) return GV_EINVAL;
    const int b = cbt_bits(k);
    if (cap < (uint64_t)b + 1) return GV_ERANGE;
    for (int i = 0; i < b; ++i) out[i] = ((k >> (b - 1 - i)) & 1u) ? '1' : '0';
    out[b] = '\0';
    return GV_OK;
}

int gv_cbt_init(gv_cbt** out, uint64_t num_vertices, const uint32_t* d_src, const uint32_t* d_dst,
                uint64_t num_edges, uint32_t block_slots, uint64_t pool_blocks, void* hip_stream) {
    if (!out) return GV_EINVAL;
    *out = nullptr;
    if (num_vertices == 0 || num_vertices > GV_MAX_CAPACITY) return GV_EINVAL;
    if (block_slots == 0 || block_slots > 1024 || (block_slots & (block_slots - 1))) return GV_EINVAL;
    if (num_edges && (!d_src || !d_dst)) return GV_EINVAL;
    if (pool_blocks == 0 || pool_blocks >= 0xFFFFFFFFull) return GV_EINVAL;
    gv_cbt* g = new (std::nothrow) gv_cbt();
    if (!g) return GV_ENOMEM;
    try {
        hip_check(hipGetDevice(&g->device), "hipGetDevice");
        g->ctx.stream = (hipStream_t)hip_stream;
        uint64_t cap = 1;
        while (cap < num_vertices) cap <<= 1;
        CbtView& v = g->v;
        v.n = num_vertices;
        v.n_cap = cap;
        v.L = log2_exact(cap);
        v.B = block_slots;
        v.log2B = log2_exact(block_slots);
        v.cap_blocks = pool_blocks;
        hip_check(hipMalloc(&g->mem_pool, pool_blocks * block_slots * 4ull), "hipMalloc pool");
        hip_check(hipMalloc(&g->mem_child, pool_blocks * 8ull), "hipMalloc child links");
        hip_check(hipMalloc(&g->mem_queue, pool_blocks * 4ull), "hipMalloc edge queue");
        hip_check(hipMalloc(&g->mem_vt, cap * sizeof(CbtVert)), "hipMalloc sentinels");
        hip_check(hipMalloc(&g->mem_ctr, kCbtWords * sizeof(unsigned long long)), "hipMalloc ctr");
        hip_check(hipHostMalloc((void**)&g->hctr, kCbtWords * sizeof(unsigned long long),
                                hipHostMallocDefault), "hipHostMalloc");
        v.pool = (uint32_t*)g->mem_pool;
        v.child = (uint32_t*)g->mem_child;
        v.queue = (const uint32_t*)g->mem_queue;
        v.vt = (CbtVert*)g->mem_vt;
        v.ctr = (unsigned long long*)g->mem_ctr;
        Ctx& c = g->ctx;
        c.launch("cbt_init", k_cbt_zero_ctr, 1, 1, v.ctr);
        c.launch("cbt_init", k_cbt_iota, div_up(pool_blocks, kThreads), kThreads,
                 (uint32_t*)g->mem_queue, pool_blocks);
        c.launch("cbt_init", k_cbt_init_vt, div_up(cap, kThreads), kThreads, v.vt, cap);
        // the initial graph is the first batch (Alg. 1, empty adjacencies)
        if (num_edges) cbt_insert(g, d_src, d_dst, num_edges, nullptr);
        hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
    } catch (const Error& e) {
        cbt_free(g);
        return e.code;
    } catch (...) {
        cbt_free(g);
        return GV_EDEVICE;
    }
    *out = g;
    return GV_OK;
}

void gv_cbt_destroy(gv_cbt* g) { cbt_free(g); }

int gv_cbt_insert_edges(gv_cbt* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                        gv_batch_stats* st) {
    if (st) std::memset(st, 0, sizeof(*st));
    if (!g || (n && (!d_src || !d_dst))) return GV_EINVAL;
    if (n == 0) return GV_OK;
    return cbt_guarded(g, [&] { cbt_insert(g, d_src, d_dst, n, st); });
}

int gv_cbt_delete_edges(gv_cbt* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                        gv_batch_stats* st) {
    if (st) std::memset(st, 0, sizeof(*st));
    if (!g || (n && (!d_src || !d_dst))) return GV_EINVAL;
    if (n == 0) return GV_OK;
    return cbt_guarded(g, [&] { cbt_delete(g, d_src, d_dst, n, st); });
}

int gv_cbt_edge_exists(gv_cbt* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                       uint8_t* d_out) {
    if (!g || (n && (!d_src || !d_dst || !d_out))) return GV_EINVAL;
    if (n == 0) return GV_OK;
    return cbt_guarded(g, [&] { cbt_query(g, d_src, d_dst, n, d_out); });
}

int gv_cbt_dump(gv_cbt* g, uint64_t* d_offsets, uint32_t* d_dst, uint64_t dst_capacity,
                uint64_t* num_edges) {
    if (!g || !num_edges) return GV_EINVAL;
    if ((d_offsets == nullptr) != (d_dst == nullptr)) return GV_EINVAL;
    *num_edges = 0;
    uint64_t e = 0;
    const int rc = cbt_guarded(g, [&] { cbt_dump(g, d_offsets, d_dst, dst_capacity, &e); });
    *num_edges = e;
    return rc;
}

int gv_cbt_blocks(gv_cbt* g, uint64_t* blocks_in_use) {
    if (!g || !blocks_in_use) return GV_EINVAL;
    return cbt_guarded(g, [&] {
        cbt_read(g);
        *blocks_in_use = g->hctr[kCbtFront];
    });
}

int gv_cbt_set_stream(gv_cbt* g, void* hip_stream) {
    if (!g) return GV_EINVAL;
    return cbt_guarded(g, [&] {
        hip_check(hipStreamSynchronize(g->ctx.stream), "hipStreamSynchronize");
        g->ctx.stream = (hipStream_t)hip_stream;
    });
}

}  // extern "C"
