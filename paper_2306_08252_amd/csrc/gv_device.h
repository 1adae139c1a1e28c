// gv_device.h -- device-side data layout and wave64 primitives (gfx950).
//
// Layout in HBM (all arrays owned by one graph):
//   pool        cap_blocks * B uint32 slots; block b occupies [b*B, b*B + B).
//   free_stack  cap_blocks uint32 block ids; [0, free_cnt) are free blocks.
//   vt          n_cap VRec (16 B each): degree, directory handle, class.
//   active      n_cap / 32 uint32 words, one bit per vertex.
//   dir         directory arena (uint32 block ids), carved in power-of-two
//               segments; a vertex with >= 2 blocks owns one segment whose
//               first nblk entries are its block ids in order.
//   dfree       per-class free-segment stacks (class c region holds at most
//               dir_cap >> c segment offsets).
//   ctr         DevCounters: pool/directory heads, per-batch sizes, errors.
//   bown        cap_blocks (vertex, index) pairs: the owner of each block the
//               pool has handed out, written when the block is assigned (a
//               freed block keeps its last owner; readers check it).
//   vlost       n_cap uint32, zero between vertex deletions (their scratch).
//   apool       cap_blocks * B * A uint32 (graphs with A > 0 attribute words
//               per edge entry): slot a's attributes at [a * A, a * A + A).
//               Kept beside the pool, not inside it, so that every probe and
//               scan reads destinations only; entries move with their slot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gv {

constexpr uint32_t kTomb = 0xFFFFFFFFu;  // empty / deleted slot marker
constexpr uint32_t kNoDir = 0xFFu;       // vertex has no directory segment
constexpr int kMaxClass = 32;
constexpr uint32_t kSpinLimitDefault = 1u << 24;  // loads before a look-back wait gives up
constexpr int kThreads = 256;            // threads per workgroup (4 waves)
constexpr int kWaves = kThreads / 64;
#ifndef GV_PROBE_CHUNK
#define GV_PROBE_CHUNK 256
#endif
constexpr uint32_t kChunk = GV_PROBE_CHUNK;  // adjacency slots per probe work item

// One vertex dictionary entry.  The adjacency of a vertex of degree deg is the
// slots [0, deg) of its blocks 0 .. ceil(deg/B)-1 (always compacted).
struct alignas(16) VRec {
    uint32_t deg;   // number of live edge slots
    uint32_t dir;   // dcls == kNoDir: id of block 0 (if any); else arena offset
    uint32_t dcls;  // log2 of the directory segment capacity, or kNoDir
    uint32_t aux;   // scratch for bulk build and vertex deletion
};

// State of the one-kernel scans on the graph's stream (at most kChainTiles
// tiles): a ticket per workgroup, each tile's sum plus one (0: not yet
// published; the word carries its own value, so relaxed loads suffice), and
// a count of the workgroups that finished; the last workgroup of a scan
// returns all of it to zero, so every scan starts from zeros.  (A buffer of
// its own: the batch counters are copied to the host whole.)
#ifndef GV_CHAIN_TILES
#define GV_CHAIN_TILES 256
#endif
constexpr uint32_t kChainTiles = GV_CHAIN_TILES;
struct ChainState {
    uint32_t ticket, done;
    unsigned long long sum[kChainTiles];
};

struct DevCounters {
    // edge-block pool (free-list stack + bump pointer)
    unsigned long long free_cnt;
    unsigned long long bump;
    // directory arena
    unsigned long long dir_bump;
    unsigned long long dir_live;
    uint32_t dfree_cnt[kMaxClass];
    uint32_t dreq[kMaxClass];          // per-batch directory segment requests
    // allocation plan of the current insert batch
    unsigned long long plan_free_top;  // free_cnt before the batch
    unsigned long long plan_from_free; // blocks popped from the free stack
    unsigned long long plan_bump0;     // bump before the batch
    uint32_t plan_dtop[kMaxClass];     // dfree_cnt before the batch
    uint32_t plan_dff[kMaxClass];      // segments popped per class
    unsigned long long plan_dbump[kMaxClass]; // first bump offset per class
    // sizes of the current batch
    uint32_t n_valid, n_T, n_items, n_aux;
    unsigned long long n_uniq;
    uint32_t sum_a, sum_b;             // scan totals of the current batch
    // errors: err_batch is reset per batch, err_sticky accumulates; err_wait
    // is set if a bounded look-back wait ever ran out
    uint32_t err_batch, err_sticky, err_wait, n_big;
    uint32_t n_heavy;                  // sources left to whole waves this batch
    uint32_t err_order;                // a batch's sorted keys failed their check
    uint32_t sort_n, sort_err;  // count and look-back error word of whole-graph sorts
    // vertex delete: slots hit, vertices touched, hole entries reserved
    unsigned long long vd_hits, vd_touched, vd_pairs;
    // totals of the single-pass scans of the current batch
    unsigned long long tot[8];
    // statistics of the last batch
    unsigned long long st_applied, st_rejected, st_dups;
    // cumulative work counters
    unsigned long long c_batches[3], c_pairs[3], c_touched[3], c_scanned[3];
    unsigned long long c_new_blocks, c_freed_blocks, c_written, c_moved;
    // striped accumulators (one 128-byte line each) for per-wave counts
    unsigned long long stripe[64][16];
    // verification
    unsigned long long live_edges;     // edges stored
    unsigned long long checksum, edges, violations;
    uint32_t vmax, vany;
};

// A batch sort that failed (a look-back wait ran out, or the sorted keys are
// out of order or not the packed keys), or a vertex delete that ran past a
// list bound, makes every later edge-batch step a no-op; the graph reports
// GV_EDEVICE from then on.
__device__ __forceinline__ bool batch_failed(const DevCounters* c) {
    return (c->err_wait | c->err_order) != 0u;
}

// Everything a kernel needs to reach the structure, passed by value.
struct GraphView {
    uint32_t* pool;
    uint32_t* free_stack;
    uint32_t* dir;
    uint32_t* dfree;
    VRec* vt;
    uint32_t* active;
    DevCounters* ctr;
    uint2* bown;
    uint32_t* vlost;
    uint32_t* apool;     // A attribute words per pool slot (slot a: apool[a * A, a * A + A))
    unsigned long long n_cap;
    unsigned long long cap_blocks;
    unsigned long long dir_cap;
    uint32_t B, log2B, L, A;
    unsigned long long dfree_base[kMaxClass];
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return __popcll(m); }

__device__ __forceinline__ bool is_active(const GraphView& g, uint64_t v) {
    return v < g.n_cap && ((g.active[v >> 5] >> (v & 31)) & 1u);
}

// is_active without a branch around the bitmap read (ids >= n_cap read word 0)
__device__ __forceinline__ bool active_bit(const GraphView& g, uint32_t v) {
    const bool in = v < g.n_cap;
    const uint32_t c = in ? v : 0u;
    const uint32_t w = g.active[c >> 5];
    return in & (((w >> (c & 31)) & 1u) != 0u);
}

__device__ __forceinline__ uint32_t nblocks(const GraphView& g, uint32_t deg) {
    return (uint32_t)(((uint64_t)deg + g.B - 1) >> g.log2B);
}

// id of block j of a vertex whose record is r (j < ceil(deg / B))
__device__ __forceinline__ uint32_t block_of(const GraphView& g, const VRec& r, uint32_t j) {
    return r.dcls == kNoDir ? r.dir : g.dir[(uint64_t)r.dir + j];
}

__device__ __forceinline__ uint64_t slot_addr(const GraphView& g, const VRec& r, uint32_t s) {
    return ((uint64_t)block_of(g, r, s >> g.log2B) << g.log2B) + (s & (g.B - 1));
}

__device__ __forceinline__ VRec load_vrec(const GraphView& g, uint32_t v) {
    return g.vt[v];
}

// smallest c with 2^c >= x (x >= 1)
__device__ __host__ __forceinline__ uint32_t ceil_log2(uint64_t x) {
    uint32_t c = 0;
    while ((1ull << c) < x) ++c;
    return c;
}

// attributes of an entry follow it when it moves from slot `from` to `to`
__device__ __forceinline__ void attr_move(const GraphView& g, uint64_t to, uint64_t from) {
    for (uint32_t k = 0; k < g.A; ++k) g.apool[to * g.A + k] = g.apool[from * g.A + k];
}

// a new entry's attributes start at zero
__device__ __forceinline__ void attr_zero(const GraphView& g, uint64_t a) {
    for (uint32_t k = 0; k < g.A; ++k) g.apool[a * g.A + k] = 0u;
}

// SplitMix64 output function (Steele, Lea, Flood 2014): checksum mixer.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// inclusive scan across the 64 lanes of a wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Appends x to `list` (for the lanes with take set) at slots reserved with
// one atomic per wave.  Every active lane of the wave must make the call.
__device__ __forceinline__ void wave_append(bool take, uint32_t x, uint32_t* counter,
                                            uint32_t* list) {
    const uint64_t m = ballot(take);
    if (!m) return;
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader, 64);
    if (take) list[base + rank_below(m)] = x;
}

// exclusive scan across a kThreads workgroup; `total` receives the sum.
// lds must hold kWaves entries; contains barriers (call uniformly).
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* lds, T& total) {
    T inc = wave_incl_scan(x);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        T v = lds[i];
        off += (i < w) ? v : T(0);
        tot += v;
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

template <typename T>
__device__ __forceinline__ T block_sum(T x, T* lds) {
    T s = wave_sum(x);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) lds[w] = s;
    __syncthreads();
    T tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) tot += lds[i];
    __syncthreads();
    return tot;
}

// first index in keys[lo, hi) whose value is >= x
template <typename K>
__device__ __forceinline__ uint32_t lower_bound(const K* keys, uint32_t lo, uint32_t hi, K x) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace gv
