// gv_edges.hip -- batched edge insert, delete and query.
//
// One pipeline serves the three operations (GraphVine Sec. 4.5-4.6, Alg. 1-3,
// re-designed for wave64):
//   pack      insert / delete: one kernel validates each pair against the
//             activity bitmap and writes its key (src << L) | dst in place
//             (an invalid pair gets the all-ones key, which sorts last),
//             clears the batch's look-back state and counters and counts
//             the sort's digits per workgroup.  Query: a kernel clears the
//             state, then a two-kernel scan writes the valid pairs,
//             compacted, with their input positions (invalid pairs are
//             answered 0 right away).
//   sort      onesweep LSD radix sort of the valid keys on 2L bits: the batch
//             is grouped by source and ordered by destination inside each
//             source segment (the paper's host CSR conversion, Sec. 4.3).
//   segments  scan over the sorted keys: segment heads give the touched
//             sources T and their segment starts; first occurrences give the
//             distinct pairs.
//   items     scan over T: each touched adjacency is cut into work items of
//             `chunk` slots, written as self-contained 32-byte descriptors
//             (slot range, batch segment, block directory); a source with a
//             single small block and a short segment becomes one small item.
//   probe     small items one per lane (slots and segment loaded whole, all
//             pairs compared); the others by lane groups that stage the
//             segment's destinations in LDS, stream slots (directory entry,
//             then slot) and binary-search each slot value.
//             Insert: mark batch entries that already exist (set semantics).
//             Delete: mark hits, remember their slot, tombstone the slot.
//             Query:  mark every query equal to a stored edge.
//   insert:   keep = first occurrence and not present (scan); per-source
//             block demand and directory growth; a one-wave plan, run by the
//             demand scan's last workgroup, checks capacity before any state
//             is written (all-or-nothing); blocks come from the free-list top
//             first, then the bump pointer (the prefix-sum pop of Sec. 4.5.1,
//             without atomics); append; grow; old directory segments freed.
//   delete:   per-source compaction pairs the holes below the new degree with
//             the survivors above it, by rank (one launch: a workgroup per
//             hub first, then lanes and waves for the other sources); emptied
//             blocks are pushed on the free list at scanned positions
//             (reclamation, Sec. 4.2).
//   query:    answers are scattered back to input order.
#include <algorithm>
#include <type_traits>

#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

constexpr uint8_t kHead = 1, kUniq = 2;
// The probe's shape is picked at run time (gv_tuning) among compiled
// variants: G lanes per work item (16, 32, 64) and U slots per lane per step
// (2, 4, 8).
constexpr int kStageLog = 7;                   // log2(kStage)
constexpr int kStage = 1 << kStageLog;         // segment entries staged in LDS
constexpr int kWinLog = 12;                    // unrolled global search steps
#ifndef GV_BIG_R
#define GV_BIG_R 256
#endif
#ifndef GV_LANE_SEG
#define GV_LANE_SEG 16
#endif
#ifndef GV_LANE_R
#define GV_LANE_R 8
#endif
constexpr uint32_t kBigR = GV_BIG_R;           // deletes per source handled by a workgroup
constexpr uint32_t kBigGroups = 256;           // workgroups for those sources
constexpr uint32_t kLaneCopy = 8;              // directory entries a lane copies or adds
constexpr uint32_t kLaneSeg = GV_LANE_SEG;     // segment entries a lane compacts
constexpr uint32_t kLaneR = GV_LANE_R;         // hits a lane compacts
constexpr uint32_t kRelease = 0x80000000u;     // flag bit in the per-source demand
constexpr uint32_t kHeavy = 0x100u;            // flag bit in t_dreq: whole waves grow this source
constexpr uint32_t kClassMask = 0xFFu;         // t_dreq & kClassMask: requested class or kNoDir

// scan-total slots in DevCounters::tot
enum {
    kTotValid = 0, kTotSeg = 1, kTotItems = 2, kTotA = 3, kTotB = 4, kTotHash = 5,
    kTotNoHash = 6  // set for a batch whose keys arrived sorted: no multiset check
};
// probe mode of the attribute calls: a query that also records the slot of
// every occurrence it finds
constexpr int kLocate = 3;
// stripe[k][kStripeHash]: per-workgroup sums of mix64 over the sorted keys
constexpr int kStripeHash = 1;

// self-contained work item: slots [s0, s1) of vertex v, batch segment [lo, hi);
// block j is dir[dirbase + j] when the vertex has a directory segment, else
// the inline block blk0 (dirbase is then 0, so the load stays in bounds)
struct alignas(16) Item {
    uint32_t s0, s1, lo, hi;
    uint32_t v, dirbase, blk0, dcls;
};

// per-source compaction descriptor (delete)
struct alignas(16) CDesc {
    uint32_t lo, hi, r, v;
    uint32_t deg, dir, dcls, need;
};

// attribute call of a query batch: get (out) or set (in), n * A words
struct AttrOp {
    uint32_t* out;
    const uint32_t* in;
};

struct BatchArrays {
    uint64_t* keys0;
    uint64_t* keys1;
    uint32_t* vals0;
    uint32_t* vals1;
    uint8_t* flags;
    uint8_t* mark;
    uint32_t* a;        // segment index of each valid key
    uint32_t* b;        // n+1: exclusive count of kept (insert) / found (delete)
    uint32_t* hitpos;   // delete, attribute calls: slot index of each hit
    uint32_t* holes;    // delete: hole slots per segment
    uint32_t* t_vtx;    // touched source per segment
    uint32_t* t_start;  // n+1: segment start; t_start[n_T] = n_valid
    uint32_t* t_need;   // n+1: blocks needed (insert), scanned
    uint32_t* t_dreq;   // insert: requested directory class or kNoDir
    uint32_t* t_drank;  // insert: rank among requests of that class
    uint32_t* t_dold;   // insert: replaced directory segment offset
    uint32_t* t_doldc;  // insert: replaced directory segment class or kNoDir
    uint32_t* rel;      // insert: sources that give back a directory segment
    CDesc* cdesc;       // delete: compaction descriptors
    uint32_t* big;      // delete: sources with more than kBigR hits
    uint32_t* heavy;    // sources left to whole waves
    Item* items;        // work items
    Item* small;        // per touched source: its small item or an empty entry
    unsigned long long* part;  // scan partials
    uint32_t* state;    // zeroed look-back state of the sort
    uint64_t state_words;
    uint32_t* vpart;    // insert / delete: valid pairs per packing workgroup
    unsigned long long* hpart;  // insert / delete: mix64 sum of valid keys per packing workgroup
    unsigned long long* stot;   // overlapped sort: valid pairs and their mix64 sum
};

static void carve_batch(Carver& cv, BatchArrays& A, uint64_t n, uint64_t icap, EdgeMode mode,
                        int bits) {
    A = BatchArrays{};
    A.keys0 = cv.take<uint64_t>(n);
    A.keys1 = cv.take<uint64_t>(n);
    if (mode == kQuery) {
        A.vals0 = cv.take<uint32_t>(n);
        A.vals1 = cv.take<uint32_t>(n);
    }
    A.flags = cv.take<uint8_t>(n);
    A.mark = cv.take<uint8_t>(n);
    A.a = cv.take<uint32_t>(n);
    A.b = cv.take<uint32_t>(n + 1);
    if (mode == kQuery) A.hitpos = cv.take<uint32_t>(n);  // attribute calls
    if (mode == kDelete) {
        A.hitpos = cv.take<uint32_t>(n);
        A.holes = cv.take<uint32_t>(n);
        A.cdesc = cv.take<CDesc>(n);
        A.big = cv.take<uint32_t>(n);
    }
    A.heavy = cv.take<uint32_t>(n);
    A.t_vtx = cv.take<uint32_t>(n);
    A.t_start = cv.take<uint32_t>(n + 1);
    A.t_need = cv.take<uint32_t>(n + 1);
    if (mode == kInsert) {
        A.t_dreq = cv.take<uint32_t>(n);
        A.t_drank = cv.take<uint32_t>(n);
        A.t_dold = cv.take<uint32_t>(n);
        A.t_doldc = cv.take<uint32_t>(n);
        A.rel = cv.take<uint32_t>(n);
    }
    A.items = cv.take<Item>(icap);
    A.small = cv.take<Item>(n);
    A.part = cv.take<unsigned long long>(scan2_parts(n + 1));
    A.state_words = os_zero_words(n, bits);  // the part the batch zeroes
    A.state = cv.take<uint32_t>(os_words(n, bits));
    A.vpart = cv.take<uint32_t>(kHistGroups);
    A.hpart = cv.take<unsigned long long>(kHistGroups);
    A.stot = cv.take<unsigned long long>(2);
}

__device__ __forceinline__ uint64_t thread_index() {
    return (uint64_t)blockIdx.x * kThreads + threadIdx.x;
}

__device__ __forceinline__ uint32_t global_wave() {
    return (uint32_t)(((uint64_t)blockIdx.x * kThreads + threadIdx.x) >> 6);
}

// ------------------------------------------------------------------ begin
// Per-batch counters, cleared by the first kernel of a batch (threads 0..63
// of its first workgroup).
__device__ __forceinline__ void clear_batch_counters(DevCounters* c, uint32_t t) {
    if (t == 0) {
        c->err_batch = 0;
        c->n_big = 0;
        c->n_heavy = 0;
        for (int k = 0; k < 8; ++k) c->tot[k] = 0;
    }
    if (t < 64) c->stripe[t][kStripeHash] = 0;
}

__global__ __launch_bounds__(kThreads) void k_begin(GraphView g, uint32_t* state, uint64_t words) {
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = thread_index(); i < words; i += stride) state[i] = 0;
    if (blockIdx.x == 0) clear_batch_counters(g.ctr, threadIdx.x);
}

// ------------------------------------------------------------------ pack
// Scan sources follow the gather interface of scan2: load() performs every
// memory read of an element at addresses that are valid whether or not the
// element is live, value() and the sinks only compute and store.
struct PackIn {
    GraphView g;
    const uint32_t* src;
    const uint32_t* dst;
    struct Rec {
        uint32_t s, d;
        bool ok;
    };
    __device__ uint64_t limit(uint64_t n) const { return n; }
    __device__ Rec load(uint64_t i, bool) const { return Rec{src[i], dst[i], false}; }
    __device__ void deref(Rec& r) const { r.ok = active_bit(g, r.s) & active_bit(g, r.d); }
    __device__ unsigned long long value(uint64_t, const Rec& r) const { return r.ok ? 1ull : 0ull; }
};

struct PackOut {
    uint32_t L;
    uint64_t* keys;
    uint32_t* vals;     // queries: input position of each valid key
    uint8_t* answer;    // queries: invalid pairs are answered here
    uint8_t* mark;
    __device__ void operator()(uint64_t i, const PackIn::Rec& r, uint64_t,
                               unsigned long long pos) const {
        mark[i] = 0;
        if (r.ok) {
            keys[pos] = ((uint64_t)r.s << L) | r.d;
            if (vals) vals[pos] = (uint32_t)i;
        } else if (answer) {
            answer[i] = 0;
        }
    }
};

// Insert and delete batches: pack without compaction.  Every pair keeps its
// input position; a pair with an inactive or out-of-range endpoint gets the
// all-ones key of the sort's bit width, which sorts after every valid key.
// All such keys are equal, so whether or not a valid pair shares that key,
// the first n_valid sorted keys are exactly the valid ones.  The same kernel
// clears the batch's look-back state (and, with clear_ctr, the batch
// counters) and counts the sort's digits (per workgroup, summed by the next
// kernel together with the valid pairs).
__global__ __launch_bounds__(kOsThreads) void k_pack_hist(GraphView g, const uint32_t* src,
                                                          const uint32_t* dst, uint64_t n,
                                                          int passes, uint64_t sentinel,
                                                          uint64_t* keys, uint8_t* mark,
                                                          uint32_t* state, uint64_t zero_words,
                                                          uint32_t* hpart, uint32_t* vpart,
                                                          unsigned long long* kpart,
                                                          int clear_ctr) {
    __shared__ uint32_t h[kOsHistCopies][8][kRadix];
    __shared__ uint32_t s_v[kOsWaves];
    __shared__ unsigned long long s_k[kOsWaves];
    const uint32_t t = threadIdx.x;
    for (uint64_t i = (uint64_t)blockIdx.x * kOsThreads + t; i < zero_words;
         i += (uint64_t)gridDim.x * kOsThreads)
        state[i] = 0;
    if (clear_ctr && blockIdx.x == 0) clear_batch_counters(g.ctr, t);
    for (int i = t; i < kOsHistCopies * 8 * kRadix; i += kOsThreads) (&h[0][0][0])[i] = 0;
    __syncthreads();
    const uint32_t copy = kOsHistCopies == 1 ? 0u : (t >> 6) & (kOsHistCopies - 1);
    uint32_t valid = 0;
    unsigned long long khash = 0;  // multiset hash of the valid keys (checked after the sort)
    const uint64_t ntiles = (n + kOsTile - 1) / kOsTile;
    for (uint64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const uint64_t base = tl * kOsTile;
        uint32_t su[kOsRounds], du[kOsRounds];
        bool ok[kOsRounds];
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) {
            const uint64_t i = base + (uint64_t)j * kOsThreads + t;
            su[j] = i < n ? src[i] : 0u;
            du[j] = i < n ? dst[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) ok[j] = active_bit(g, su[j]) & active_bit(g, du[j]);
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) {
            const uint64_t i = base + (uint64_t)j * kOsThreads + t;
            if (i >= n) continue;
            const uint64_t key = ok[j] ? ((uint64_t)su[j] << g.L) | du[j] : sentinel;
            keys[i] = key;
            mark[i] = 0;
            valid += ok[j] ? 1u : 0u;
            khash += ok[j] ? mix64(key) : 0ull;
            for (int p = 0; p < passes; ++p)
                atomicAdd(&h[copy][p][(uint32_t)(key >> (p * kRadixBits)) & (kRadix - 1)], 1u);
        }
    }
    const uint32_t vw = (uint32_t)wave_sum((unsigned long long)valid);
    const unsigned long long kw = wave_sum(khash);
    if (lane_id() == 0) {
        s_v[t >> 6] = vw;
        s_k[t >> 6] = kw;
    }
    __syncthreads();
    uint32_t* out = hpart + (uint64_t)blockIdx.x * passes * kRadix;
    for (int i = t; i < passes * kRadix; i += kOsThreads) {
        uint32_t x = 0;
#pragma unroll
        for (int c = 0; c < kOsHistCopies; ++c) x += h[c][i / kRadix][i % kRadix];
        out[i] = x;
    }
    if (t == 0) {
        uint32_t x = 0;
        unsigned long long y = 0;
        for (int w = 0; w < kOsWaves; ++w) {
            x += s_v[w];
            y += s_k[w];
        }
        vpart[blockIdx.x] = x;
        kpart[blockIdx.x] = y;
    }
}

// Insert and delete batches of at most kOsTile pairs: one workgroup packs
// the pairs as k_pack_hist does and sorts the keys in LDS, every radix pass
// in the same kernel (the ranking of k_os_pass on a single tile, so no
// look-back), instead of the pack, histogram and pass kernels.  Writes the
// sorted keys to `keys` and the valid-pair count to tot[kTotValid].
__global__ __launch_bounds__(kOsThreads) void k_pack_sort_tile(GraphView g, const uint32_t* src,
                                                               const uint32_t* dst, uint64_t n,
                                                               int passes, uint64_t sentinel,
                                                               uint64_t* keys, uint8_t* mark) {
    __shared__ TileSortLds lds;
    __shared__ unsigned long long s_v[kOsWaves];
    const uint32_t t = threadIdx.x;
    const int w = t >> 6;
    clear_batch_counters(g.ctr, t);
    uint64_t key[kOsRounds];
    unsigned long long valid = 0, khash = 0;
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + t;
        const uint32_t su = i < n ? src[i] : 0u, du = i < n ? dst[i] : 0u;
        const bool ok = active_bit(g, su) & active_bit(g, du);
        key[j] = ok ? ((uint64_t)su << g.L) | du : sentinel;
        if (i < n) {
            mark[i] = 0;
            valid += ok ? 1u : 0u;
            khash += ok ? mix64(key[j]) : 0ull;
        }
    }
    tile_sort(key, n, passes, sentinel, lds);
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + t;
        if (i < n) keys[i] = key[j];
    }
    valid = wave_sum(valid);
    khash = wave_sum(khash);
    __shared__ unsigned long long s_k[kOsWaves];
    if (lane_id() == 0) {
        s_v[w] = valid;
        s_k[w] = khash;
    }
    __syncthreads();
    if (t == 0) {
        unsigned long long x = 0, y = 0;
        for (int k = 0; k < kOsWaves; ++k) {
            x += s_v[k];
            y += s_k[k];
        }
        g.ctr->tot[kTotValid] = x;
        g.ctr->tot[kTotHash] = y;
    }
}

// Query batches of at most kOsTile pairs: one workgroup packs each valid pair
// as its key with its input position in the low 12 bits (an invalid pair is
// answered 0 here and gets the all-ones key, after every valid one), sorts
// the tile in LDS, and writes the valid keys and their positions compacted,
// as the packing scan and the sort leave them.
constexpr int kTilePosBits = 12;  // kOsTile = 4096 positions
__global__ __launch_bounds__(kOsThreads) void k_query_sort_tile(GraphView g, const uint32_t* src,
                                                                const uint32_t* dst, uint64_t n,
                                                                int passes, uint64_t* keys,
                                                                uint32_t* vals, uint8_t* answer,
                                                                uint8_t* mark) {
    __shared__ TileSortLds lds;
    __shared__ uint32_t s_v[kOsWaves];
    const uint32_t t = threadIdx.x;
    clear_batch_counters(g.ctr, t);
    uint64_t key[kOsRounds];
    uint32_t valid = 0;
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + t;
        const uint32_t su = i < n ? src[i] : 0u, du = i < n ? dst[i] : 0u;
        const bool ok = i < n && active_bit(g, su) && active_bit(g, du);
        key[j] = ok ? ((((uint64_t)su << g.L) | du) << kTilePosBits) | i : ~0ull;
        if (i < n) {
            mark[i] = 0;
            if (!ok && answer) answer[i] = 0;
        }
        valid += ok ? 1u : 0u;
    }
    tile_sort(key, n, passes, ~0ull, lds);
    const uint32_t vw = (uint32_t)wave_sum((unsigned long long)valid);
    if (lane_id() == 0) s_v[t >> 6] = vw;
    __syncthreads();
    uint32_t nv = 0;
    for (int k = 0; k < kOsWaves; ++k) nv += s_v[k];
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + t;
        if (i < nv) {
            keys[i] = key[j] >> kTilePosBits;
            vals[i] = (uint32_t)(key[j] & ((1u << kTilePosBits) - 1));
        }
    }
    if (t == 0) g.ctr->tot[kTotValid] = nv;
}

// ------------------------------------------------------------------ segments
struct SegIn {
    const uint64_t* keys;
    const DevCounters* ctr;
    uint32_t L;
    // valid pairs: tot[kTotValid], or (sort overlap) the count the packing
    // left in the batch's buffer, with the key sum after it
    const unsigned long long* nvalid;
    // sort overlap: the batch counters, cleared by begin() and given the
    // packing's count and key sum (the previous batch used them until now)
    DevCounters* clr;
    struct Rec {
        uint64_t k, p;
    };
    __device__ void begin() const {
        if (!clr) return;
        clear_batch_counters(clr, threadIdx.x);
        if (threadIdx.x == 0) {
            clr->tot[kTotValid] = nvalid[0];
            clr->tot[kTotHash] = nvalid[1];
        }
    }
    // no segments after a look-back wait ran out (the keys are not sorted)
    __device__ uint64_t limit(uint64_t n) const {
        return ctr->err_wait ? 0ull : min((uint64_t)*nvalid, n);
    }
    __device__ Rec load(uint64_t i, bool ok) const {
        const uint64_t j = ok ? i : 0;
        return Rec{keys[j], keys[j ? j - 1 : 0]};
    }
    __device__ void deref(Rec&) const {}
    __device__ unsigned long long value(uint64_t i, const Rec& r) const {
        const unsigned long long head = i == 0 || (r.k >> L) != (r.p >> L);
        const unsigned long long uniq = i == 0 || r.k != r.p;
        return head | (uniq << 32);
    }
};

// The segment scan also checks the sort: every key is at least its
// predecessor (else err_order = 2), and the mix64 sum of the sorted keys,
// added up per workgroup in the hash stripes, must equal the packed keys'
// sum (compared by the probe, which runs next but one).
struct SegOut {
    uint32_t L;
    uint8_t* flags;
    uint32_t* a;
    uint32_t* t_vtx;
    uint32_t* t_start;
    DevCounters* ctr;
    __device__ void operator()(uint64_t i, const SegIn::Rec& r, uint64_t nv,
                               unsigned long long pre) const {
        if (i >= nv) {
            if (i == 0) t_start[0] = 0;
            return;
        }
        if (i > 0 && r.k < r.p) ctr->err_order = 2;
        const bool head = i == 0 || (r.k >> L) != (r.p >> L);
        const bool uniq = i == 0 || r.k != r.p;
        const uint32_t t = (uint32_t)pre + (head ? 1u : 0u) - 1u;  // segment of key i
        flags[i] = (head ? kHead : 0) | (uniq ? kUniq : 0);
        a[i] = t;
        if (head) {
            // masked to the table: a valid key's source is below 2^L already;
            // the mask keeps even a corrupted key's record read in bounds
            t_vtx[t] = (uint32_t)(r.k >> L) & (uint32_t)((1ull << L) - 1);
            t_start[t] = (uint32_t)i;
        }
        if (i + 1 == nv) t_start[t + 1] = (uint32_t)nv;
    }
    __device__ unsigned long long tally(uint64_t, const SegIn::Rec& r) const { return mix64(r.k); }
    __device__ void commit(unsigned long long sum) const {
        atomicAdd(&ctr->stripe[blockIdx.x & 63][kStripeHash], sum);
    }
};

// ------------------------------------------------------------------ items
// a touched source, its batch segment and its vertex record
struct TouchRec {
    uint32_t v, lo, hi;
    VRec r;
};

__device__ __forceinline__ TouchRec load_touched(const uint32_t* t_vtx, const uint32_t* t_start,
                                                 uint64_t t, bool ok) {
    const uint64_t j = ok ? t : 0;
    const uint32_t v0 = t_vtx[j], lo0 = t_start[j], hi0 = t_start[j + 1];
    TouchRec x;
    x.v = ok ? v0 : 0u;
    x.lo = ok ? lo0 : 0u;
    x.hi = ok ? hi0 : 0u;
    return x;
}

// Small items: a source with at most kSmallLanes * kSmallDeg slots and at
// most kSmallSeg pairs in its batch segment is probed by kSmallLanes lanes,
// kSmallDeg slots each, instead of a lane group.  Their descriptors go to a
// second array indexed by touched source, where the other sources get an
// empty entry (s1 = 0).
constexpr uint32_t kSmallDeg = 16;    // slots per lane (whole 16-byte groups of a block)
constexpr uint32_t kSmallLanes = 4;   // lanes per small item
#ifndef GV_SMALL_SEG
#define GV_SMALL_SEG 8
#endif
constexpr uint32_t kSmallSeg = GV_SMALL_SEG;
__device__ __forceinline__ bool small_item(uint32_t B, uint32_t deg, uint32_t len) {
    return B >= 4 && deg > 0 && deg <= kSmallLanes * kSmallDeg && len <= kSmallSeg;
}

struct ItemIn {
    static constexpr int kItems = 2;  // large records: fewer per thread
    GraphView g;
    const uint32_t* t_vtx;
    const uint32_t* t_start;
    uint32_t chunk;  // adjacency slots per work item
    using Rec = TouchRec;
    __device__ uint64_t limit(uint64_t n) const {
        return batch_failed(g.ctr) ? 0ull : min((uint64_t)(uint32_t)g.ctr->tot[kTotSeg], n);
    }
    __device__ Rec load(uint64_t t, bool ok) const { return load_touched(t_vtx, t_start, t, ok); }
    __device__ void deref(Rec& x) const { x.r = g.vt[x.v]; }
    __device__ unsigned long long value(uint64_t, const Rec& x) const {
        const unsigned long long items =
            small_item(g.B, x.r.deg, x.hi - x.lo) ? 0ull : (x.r.deg + chunk - 1) / chunk;
        return items | ((unsigned long long)nblocks(g, x.r.deg) << 32);
    }
};

// A source's work items: one per `chunk` slots.  A lane writes up to
// kLaneItems of them; sources with more are written by all the lanes of the
// wave that make the call, one item each per store.  The scan calls the sink
// for elements below its size only, so in the last wave of a scan some lanes
// may not take part: the loop counts the lanes that do.
constexpr uint32_t kLaneItems = 16;

struct ItemOut {
    Item* items;
    Item* small;        // per touched source: its small item, or s1 = 0
    uint32_t B;
    uint64_t icap;      // capacity of items (the scan of distinct sources stays below it)
    uint32_t chunk;     // adjacency slots per work item
    uint32_t* shits;    // delete: small-item hits per source, zeroed here for the others
    __device__ void operator()(uint64_t t, const TouchRec& x, uint64_t lim,
                               unsigned long long pre) const {
        const bool live = t < lim;
        const VRec r = x.r;
        const bool small = live && small_item(B, r.deg, x.hi - x.lo);
        const uint32_t cnt = live && !small ? (r.deg + chunk - 1) / chunk : 0u;
        const uint32_t base = (uint32_t)pre;
        Item it;
        it.lo = x.lo;
        it.hi = x.hi;
        it.v = x.v;
        it.dirbase = r.dcls != kNoDir ? r.dir : 0u;
        it.blk0 = r.dcls != kNoDir ? 0u : r.dir;
        it.dcls = r.dcls;
        if (small) {
            Item w = it;
            w.s0 = 0;
            w.s1 = r.deg;
            this->small[t] = w;
        } else if (live) {
            *(uint4*)&this->small[t] = make_uint4(0u, 0u, 0u, 0u);
            if (shits) shits[t] = 0u;
        }
        if (cnt <= kLaneItems) {
            for (uint32_t c = 0; c < cnt; ++c) {
                it.s0 = c * chunk;
                it.s1 = min(r.deg, it.s0 + chunk);
                if (base + c < icap) items[base + c] = it;
            }
        }
        const uint64_t act = ballot(true);
        const uint32_t nact = popc64(act), me = rank_below(act);
        uint64_t m = ballot(cnt > kLaneItems);
        while (m) {
            const int l = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            Item w;
            w.lo = __shfl(it.lo, l, 64);
            w.hi = __shfl(it.hi, l, 64);
            w.v = __shfl(it.v, l, 64);
            w.dirbase = __shfl(it.dirbase, l, 64);
            w.blk0 = __shfl(it.blk0, l, 64);
            w.dcls = __shfl(it.dcls, l, 64);
            const uint32_t wdeg = __shfl(r.deg, l, 64);
            const uint32_t wcnt = __shfl(cnt, l, 64), wbase = __shfl(base, l, 64);
            for (uint32_t c = me; c < wcnt; c += nact) {
                w.s0 = c * chunk;
                w.s1 = min(wdeg, w.s0 + chunk);
                if ((uint64_t)wbase + c < icap) items[wbase + c] = w;
            }
        }
    }
};

// ------------------------------------------------------------------ probe
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int MODE, int G, int U>
__device__ __forceinline__ void probe_load(const GraphView& g, const Item& I, const uint32_t* dp,
                                           uint32_t s, uint32_t (&x)[U],
                                           uint64_t (&addr)[U]) {
    // unconditional loads at clamped positions; lanes past the item are
    // masked out by the caller
    uint32_t e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t si = min(s + u * G, I.s1 - 1);
        e[u] = dp[si >> g.log2B];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t si = min(s + u * G, I.s1 - 1);
        addr[u] = ((uint64_t)e[u] << g.log2B) + (si & (g.B - 1));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = g.pool[addr[u]];
}

// Searches of the U slots of a lane run in lockstep, so that each step
// issues U independent reads and waits once.  Returns the lane's hits
// (delete: slots tombstoned).
template <int MODE, int G, int U>
__device__ __forceinline__ uint32_t probe_search(const GraphView& g, const Item& I, uint32_t s,
                                                 const uint32_t (&x)[U],
                                                 const uint64_t (&addr)[U], const uint32_t* st,
                                                 uint32_t steps, uint32_t shift,
                                                 const uint64_t* keys, uint8_t* mark,
                                                 uint32_t* hitpos) {
    const uint32_t len = I.hi - I.lo;
    const uint64_t vbase = (uint64_t)I.v << g.L;
    // rank among the LDS samples: st[0, 2^steps - 1) holds the sorted samples
    // padded with 0xFFFFFFFF (at least one pad entry, so the rank can reach ns)
    uint32_t lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) lo[u] = 0;
    // unrolled to the largest step count so that no loop carries outstanding
    // loads (the next step's slot loads stay in flight meanwhile)
#pragma unroll
    for (int k = kStageLog - 1; k >= 0; --k) {
        if ((uint32_t)k >= steps) continue;
        const uint32_t half = 1u << k;
        uint32_t sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = st[lo[u] + half - 1];
#pragma unroll
        for (int u = 0; u < U; ++u) lo[u] += sv[u] < x[u] ? half : 0u;
    }
    uint32_t p[U];  // first segment position whose value is >= x
    bool hit[U];
    if (shift == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            p[u] = lo[u];
            const uint32_t v = st[lo[u]];  // lo <= ns < kStage
            hit[u] = (lo[u] < len) & (v == x[u]);
        }
    } else {
        // the answer lies in ((lo - 1) * stride, lo * stride]: a window of
        // fewer than 2^shift entries before the sample at lo * stride (or
        // the end of the segment); branch-free lower bound in `shift` steps
        uint32_t end[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            p[u] = lo[u] ? ((lo[u] - 1) << shift) + 1 : 0;
            end[u] = min(lo[u] << shift, len);
        }
        auto step = [&](uint32_t half) {
            uint64_t kv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) kv[u] = keys[I.lo + min(p[u] + half - 1, len - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u)
                p[u] += (p[u] + half - 1 < end[u] && kv[u] < (vbase | x[u])) ? half : 0u;
        };
        // windows of up to 2^kWinLog entries take unrolled steps; longer ones
        // (segments beyond about half a million pairs) a loop
        for (uint32_t k = shift; k-- > kWinLog;) step(1u << k);
#pragma unroll
        for (int k = kWinLog - 1; k >= 0; --k)
            if ((uint32_t)k < shift) step(1u << k);
        uint64_t kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) kv[u] = keys[I.lo + min(p[u], len - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) hit[u] = p[u] < len && kv[u] == (vbase | x[u]);
    }
    uint32_t nhit = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t si = s + u * G;
        if (si >= I.s1 || !hit[u]) continue;
        const uint32_t pos = I.lo + p[u];
        if (MODE == kInsert) {
            mark[pos] = 1;
        } else if (MODE == kDelete) {
            mark[pos] = 1;
            hitpos[pos] = si;
            g.pool[addr[u]] = kTomb;
            ++nhit;
        } else {
            const uint64_t target = vbase | x[u];
            for (uint32_t j = pos; j < I.hi && keys[j] == target; ++j) {
                mark[j] = 1;
                if (MODE == kLocate) hitpos[j] = si;
            }
        }
    }
    return nhit;
}

// Lane q of a small item's lanes probes slots [q * kSmallDeg, (q + 1) *
// kSmallDeg) of its adjacency: those slots and the segment's destinations are
// loaded whole and compared pairwise.  Same marks as the group search: insert
// and delete mark the first occurrence of a stored pair (delete also records
// the slot and tombstones it), query marks every occurrence.  A stored pair
// sits in one slot, so one lane at most marks a segment entry.  Returns the
// lane's hits (delete).
template <int MODE>
__device__ __forceinline__ uint32_t probe_small(const GraphView& g, const Item& I, uint32_t q,
                                                const uint64_t* keys, uint8_t* mark,
                                                uint32_t* hitpos) {
    uint32_t nhit = 0;
    const uint32_t deg = I.s1;
    const uint32_t len = I.hi - I.lo;
    const uint32_t first = q * kSmallDeg;
    const uint32_t* klo = (const uint32_t*)keys;  // low words: destinations
    const uint32_t dmask = (uint32_t)((1ull << g.L) - 1);
    uint32_t d[kSmallSeg];
#pragma unroll
    for (uint32_t j = 0; j < kSmallSeg; ++j)
        d[j] = j < len ? klo[2ull * (I.lo + j)] & dmask : 0u;
    // whole 16-byte groups of a block (B >= 4, so a group stays inside it)
    uint32_t x[kSmallDeg];
    uint64_t a[kSmallDeg / 4];
#pragma unroll
    for (uint32_t u = 0; u < kSmallDeg; u += 4) {
        const uint32_t sl = first + u;
        const uint32_t j = sl >> g.log2B;
        const uint32_t blk = I.dcls != kNoDir ? g.dir[I.dirbase + (sl < deg ? j : 0u)] : I.blk0;
        a[u / 4] = ((uint64_t)blk << g.log2B) + (sl & (g.B - 1));
    }
#pragma unroll
    for (uint32_t u = 0; u < kSmallDeg; u += 4) {
        uint4 v = make_uint4(kTomb, kTomb, kTomb, kTomb);
        if (first + u < deg) v = *(const uint4*)(g.pool + a[u / 4]);
        x[u] = v.x;
        x[u + 1] = v.y;
        x[u + 2] = v.z;
        x[u + 3] = v.w;
    }
#pragma unroll
    for (uint32_t j = 0; j < kSmallSeg; ++j) {
        if (j >= len) break;
        if (MODE != kQuery && MODE != kLocate && j > 0 && d[j] == d[j - 1])
            continue;  // not a first occurrence
        uint32_t hu = kSmallDeg;
#pragma unroll
        for (uint32_t u = 0; u < kSmallDeg; ++u)
            if (first + u < deg && x[u] == d[j]) hu = u;
        if (hu == kSmallDeg) continue;
        mark[I.lo + j] = 1;
        if (MODE == kLocate) hitpos[I.lo + j] = first + hu;
        if (MODE == kDelete) {
            hitpos[I.lo + j] = first + hu;
            g.pool[a[hu / 4] + (hu & 3)] = kTomb;
            ++nhit;
        }
    }
    return nhit;
}

// shits (delete): per touched source, the hits of its small item (written
// for every small item; the items scan zeroes the other sources' entries)
template <int MODE, int G, int U>
__global__ __launch_bounds__(kThreads) void k_probe(GraphView g, const uint64_t* keys,
                                                    const Item* items, const Item* small,
                                                    uint8_t* mark, uint32_t* hitpos,
                                                    uint32_t* shits) {
    __shared__ uint32_t stage[kWaves * (64 / G)][kStage];
    __shared__ uint32_t s_hits[kWaves * (64 / G)];  // delete: hits of a group's item
    if (MODE == kDelete) {
        if (threadIdx.x < kWaves * (64 / G)) s_hits[threadIdx.x] = 0u;
        __syncthreads();
    }
    if (batch_failed(g.ctr)) return;
    if (MODE == kInsert || MODE == kDelete) {
        // the sorted keys must be the packed keys: their mix64 sums agree
        // (per-workgroup sums of the segment scan in 64 stripes; one load a lane)
        const unsigned long long sorted = wave_sum(g.ctr->stripe[lane_id()][kStripeHash]);
        if (!g.ctr->tot[kTotNoHash] && sorted != g.ctr->tot[kTotHash]) {
            if (lane_id() == 0) g.ctr->err_order = 3;
            return;
        }
    }
    {
        // small items first, kSmallLanes consecutive lanes per touched source
        const uint64_t nq = (uint64_t)(uint32_t)g.ctr->tot[kTotSeg] * kSmallLanes;
        const uint64_t stride = (uint64_t)gridDim.x * kThreads;
        for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < nq; k += stride) {
            const Item I = small[k / kSmallLanes];
            const uint32_t q = (uint32_t)(k % kSmallLanes);
            uint32_t h = 0;
            if (I.s1 > q * kSmallDeg) h = probe_small<MODE>(g, I, q, keys, mark, hitpos);
            if (MODE == kDelete) {
                // the item's kSmallLanes lanes are consecutive and all here
                static_assert(kSmallLanes == 4, "two exchange steps");
                h += __shfl_xor(h, 1, 64);
                h += __shfl_xor(h, 2, 64);
                if (q == 0 && I.s1 > 0) shits[k / kSmallLanes] = h;
            }
        }
    }
    const uint32_t nitems = (uint32_t)g.ctr->tot[kTotItems];
    const uint32_t lane = lane_id();
    const uint32_t gl = lane & (G - 1);
    const uint32_t gid_local = (threadIdx.x >> 6) * (64 / G) + (lane / G);
    uint32_t* st = stage[gid_local];
    const uint32_t ngroups = gridDim.x * kWaves * (64 / G);
    const uint64_t dmask = (1ull << g.L) - 1;
    uint32_t it = global_wave() * (64 / G) + lane / G;
    if (it >= nitems) return;
    Item I = items[it];
    while (true) {
        const uint32_t itn = it + ngroups;
        const Item In = items[min(itn, nitems - 1)];  // prefetch the next item
        // item prologue, in issue order: directory entries of the first step,
        // the segment samples, then the first step's slots; the samples go to
        // LDS once they arrive, while the slot loads are still in flight
        const uint32_t len = I.hi - I.lo;
        // LDS holds the segment (stride 1) or every stride-th entry of it,
        // padded with 0xFFFFFFFF up to a power of two (at least one pad entry
        // stays, so the rank can reach ns)
        const uint32_t q = (len + kStage - 2) / (kStage - 1);
        const uint32_t shift = q <= 1 ? 0u : 32u - __clz(q - 1);
        const uint32_t ns = (len + (1u << shift) - 1) >> shift;  // < kStage samples
        const uint32_t steps = 32u - __clz(ns);                  // 2^steps > ns
        uint32_t s = I.s0 + gl;
        // block ids come from the directory, or from the item itself for a
        // vertex whose only block is stored inline
        const uint32_t* dp = I.dcls != kNoDir ? g.dir + I.dirbase : &items[it].blk0;
        uint32_t e[U];
        if (I.dcls != kNoDir) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t si = min(s + u * G, I.s1 - 1);
                e[u] = dp[si >> g.log2B];
            }
        } else {
            // the only block: its id is in the descriptor, no load
#pragma unroll
            for (int u = 0; u < U; ++u) e[u] = I.blk0;
        }
        constexpr int kSv = kStage / G;
        const uint32_t* klo = (const uint32_t*)keys;  // low words: destinations
        uint32_t sv[kSv];
#pragma unroll
        for (int r = 0; r < kSv; ++r) {
            const uint32_t j = min(gl + r * G, ns - 1);
            sv[r] = r * G < ns ? klo[2ull * (I.lo + (j << shift))] & (uint32_t)dmask : 0u;
        }
        uint32_t x[U];
        uint64_t addr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t si = min(s + u * G, I.s1 - 1);
            addr[u] = ((uint64_t)e[u] << g.log2B) + (si & (g.B - 1));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = g.pool[addr[u]];
#pragma unroll
        for (int r = 0; r < kSv; ++r) {
            // the searches read st[0, 2^steps) only
            const uint32_t j = gl + r * G;
            if (r * G < (1u << steps)) st[j] = j < ns ? sv[r] : 0xFFFFFFFFu;
        }
        wave_lds_sync();
        // the loads of step k+1 are issued before step k is searched and
        // copied over after it, so they overlap the search
        while (true) {
            const bool more = s + G * U - gl < I.s1;  // uniform in the group
            uint32_t x2[U];
            uint64_t a2[U];
            if (more) probe_load<MODE, G, U>(g, I, dp, s + G * U, x2, a2);
            const uint32_t nhit = probe_search<MODE, G, U>(g, I, s, x, addr, st, steps, shift,
                                                           keys, mark, hitpos);
            if (MODE == kDelete && nhit) atomicAdd(&s_hits[gid_local], nhit);
            if (!more) break;
            s += G * U;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                x[u] = x2[u];
                addr[u] = a2[u];
            }
        }
        // the item's hits (summed in LDS over its steps) go to its source's
        // count: one add per group
        wave_lds_sync();
        if (MODE == kDelete && gl == 0) {
            const uint32_t h = s_hits[gid_local];
            if (h) {
                atomicAdd(&g.vlost[I.v], h);
                s_hits[gid_local] = 0u;
            }
        }
        if (itn >= nitems) break;
        it = itn;
        I = In;
    }
}

// ------------------------------------------------------------------ insert
struct KeepIn {
    const uint8_t* flags;
    const uint8_t* mark;
    const DevCounters* ctr;
    struct Rec {
        uint8_t f, m;
    };
    __device__ uint64_t limit(uint64_t n) const {
        return batch_failed(ctr) ? 0ull : min((uint64_t)ctr->tot[kTotValid], n);
    }
    __device__ Rec load(uint64_t i, bool ok) const {
        const uint64_t j = ok ? i : 0;
        return Rec{flags[j], mark[j]};
    }
    __device__ void deref(Rec&) const {}
    __device__ unsigned long long value(uint64_t, const Rec& r) const {
        return ((r.f & kUniq) && !r.m) ? 1ull : 0ull;
    }
};

struct U32Out {
    uint32_t* a;
    template <typename R>
    __device__ void operator()(uint64_t i, const R&, uint64_t, unsigned long long v) const {
        a[i] = (uint32_t)v;
    }
};

__global__ __launch_bounds__(kThreads) void k_plan_ins(GraphView g, const uint32_t* t_vtx,
                                                       const uint32_t* t_start, const uint32_t* b,
                                                       uint32_t* t_need, uint32_t* t_dreq,
                                                       uint32_t* t_drank, uint32_t* heavy) {
    __shared__ uint32_t lcnt[kMaxClass];
    __shared__ uint32_t lbase[kMaxClass];
    if (threadIdx.x < kMaxClass) lcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t = thread_index();
    if (batch_failed(g.ctr)) return;  // uniform over the launch
    const uint32_t nT = (uint32_t)g.ctr->tot[kTotSeg];
    uint32_t cls = kNoDir, lrank = 0;
    bool big = false;
    if (t < nT) {
        const uint32_t kp = b[t_start[t + 1]] - b[t_start[t]];
        const VRec r = g.vt[t_vtx[t]];
        const uint32_t nb0 = nblocks(g, r.deg), nb1 = nblocks(g, r.deg + kp);
        const uint64_t cap0 = r.dcls == kNoDir ? 1ull : (1ull << r.dcls);
        if (nb1 > cap0) {
            cls = ceil_log2(nb1);
            lrank = atomicAdd(&lcnt[cls], 1u);
        }
        // top bit: the source gives back a directory segment
        t_need[t] = (nb1 - nb0) | (cls != kNoDir && r.dcls != kNoDir ? kRelease : 0u);
        big = (cls != kNoDir && nb0 > kLaneCopy) || nb1 - nb0 > kLaneCopy;
        // the grow kernel takes this decision from here: its heavy sources'
        // records change while other waves still run the lane loop, so it
        // must not be made again from the record there
        t_dreq[t] = cls | (big ? kHeavy : 0u);
    }
    wave_append(big, (uint32_t)t, &g.ctr->n_heavy, heavy);
    __syncthreads();
    if (threadIdx.x < kMaxClass) {
        const uint32_t c = lcnt[threadIdx.x];
        lbase[threadIdx.x] = c ? atomicAdd(&g.ctr->dreq[threadIdx.x], c) : 0u;
    }
    __syncthreads();
    if (t < nT && cls != kNoDir) t_drank[t] = lbase[cls] + lrank;
}

// blocks needed in the low half, directory segments given back in the high
// half (their rank is their slot in the release list)
struct NeedIn {
    const uint32_t* t_need;
    const DevCounters* ctr;
    struct Rec {
        uint32_t need;
    };
    __device__ uint64_t limit(uint64_t n) const {
        return batch_failed(ctr) ? 0ull : min((uint64_t)(uint32_t)ctr->tot[kTotSeg], n);
    }
    __device__ Rec load(uint64_t t, bool ok) const { return Rec{t_need[ok ? t : 0]}; }
    __device__ void deref(Rec&) const {}
    __device__ unsigned long long value(uint64_t, const Rec& r) const {
        return (unsigned long long)(r.need & ~kRelease) | ((unsigned long long)(r.need >> 31) << 32);
    }
};

__device__ __forceinline__ void plan_batch(const GraphView& g, uint64_t n, int sticky);

struct NeedOut {
    uint32_t* t_need;
    uint32_t* rel;
    GraphView g;
    uint64_t n;
    int sticky;
    __device__ void operator()(uint64_t t, const NeedIn::Rec& r, uint64_t lim,
                               unsigned long long pre) const {
        t_need[t] = (uint32_t)pre;
        if (t < lim && (r.need & kRelease)) rel[(uint32_t)(pre >> 32)] = (uint32_t)t;
    }
    __device__ void finish() const { plan_batch(g, n, sticky); }
};

// Allocation plan for the whole batch, one wave (a lane per directory class):
// capacity is checked before any state is written, so a failing batch leaves
// the graph unchanged.  Run by the first wave of the demand scan's last
// workgroup, once the scan total (blocks needed) is written.
__device__ __forceinline__ void plan_batch(const GraphView& g, uint64_t n, int sticky) {
    DevCounters* c = g.ctr;
    const uint32_t k = lane_id();
    if (batch_failed(c)) {
        // nothing is committed; append, grow and release see the error
        if (k == 0) c->err_batch = GV_EDEVICE;
        return;
    }
    const bool cl = k < kMaxClass;
    const unsigned long long N = c->tot[kTotB] & 0xffffffffull;
    const unsigned long long free0 = c->free_cnt, bump0 = c->bump;
    const unsigned long long ff = N < free0 ? N : free0;
    const unsigned long long fb = N - ff;
    const uint32_t req = cl ? c->dreq[k] : 0u;
    const uint32_t have = cl ? c->dfree_cnt[k] : 0u;
    const uint32_t dff = req < have ? req : have;
    const unsigned long long grow = cl ? (unsigned long long)(req - dff) << k : 0ull;
    const unsigned long long gincl = wave_incl_scan(grow);
    const unsigned long long db0 = c->dir_bump;
    const unsigned long long db_end = db0 + __shfl(gincl, 63, 64);
    const bool ok = bump0 + fb <= g.cap_blocks && db_end <= g.dir_cap;
    if (cl) {
        c->plan_dff[k] = dff;
        c->plan_dbump[k] = db0 + gincl - grow;
        c->dreq[k] = 0;
        if (ok) {
            c->plan_dtop[k] = have;
            c->dfree_cnt[k] = have - dff;
        }
    }
    const unsigned long long live = wave_sum(cl ? (unsigned long long)req << k : 0ull);
    if (k != 0) return;
    const unsigned long long nv = c->tot[kTotValid];
    const unsigned long long nT = c->tot[kTotSeg] & 0xffffffffull;
    const unsigned long long nuniq = c->tot[kTotSeg] >> 32;
    const unsigned long long applied = c->tot[kTotA];
    c->c_batches[kInsert] += 1;
    c->c_pairs[kInsert] += n;
    c->c_touched[kInsert] += nT;
    c->c_scanned[kInsert] += (c->tot[kTotItems] >> 32) << g.log2B;
    if (!ok) {
        c->err_batch = GV_ENOMEM;
        if (sticky && !c->err_sticky) c->err_sticky = GV_ENOMEM;
        c->st_applied = c->st_rejected = c->st_dups = 0;
        return;
    }
    c->plan_free_top = free0;
    c->plan_from_free = ff;
    c->plan_bump0 = bump0;
    c->free_cnt = free0 - ff;
    c->bump = bump0 + fb;
    c->dir_bump = db_end;
    c->dir_live += live;
    c->st_applied = applied;
    c->st_rejected = n - nv;
    c->st_dups = nv - nuniq;
    c->c_new_blocks += N;
    c->c_written += applied;
    c->live_edges += applied;
}

// One wave per touched source: grow its directory segment if needed (copy the
// old entries) and record the ids of its new blocks.
// id of the p-th block the batch allocates (free-list top first, then bump)
__device__ __forceinline__ uint32_t planned_block(const GraphView& g, const DevCounters* c,
                                                  uint64_t p) {
    return p < c->plan_from_free ? g.free_stack[c->plan_free_top - 1 - p]
                                 : (uint32_t)(c->plan_bump0 + (p - c->plan_from_free));
}

// Append: every kept pair is written to slot deg + rank of its source, read
// from the vertex record as it was before the batch; new blocks come from
// the allocation plan, so this runs before the directory is updated.
__global__ __launch_bounds__(kThreads) void k_append(GraphView g, const uint64_t* keys,
                                                     const uint8_t* flags, const uint8_t* mark,
                                                     const uint32_t* a, const uint32_t* b,
                                                     const uint32_t* t_vtx,
                                                     const uint32_t* t_start,
                                                     const uint32_t* t_need) {
    const DevCounters* c = g.ctr;
    if (c->err_batch) return;
    const uint64_t i = thread_index();
    if (i >= c->tot[kTotValid]) return;
    const uint8_t f = flags[i], m = mark[i];
    const uint32_t t = a[i], bi = b[i];
    const uint64_t key = keys[i];
    if (!(f & kUniq) || m) return;
    const uint32_t v = t_vtx[t], lo = t_start[t], p0 = t_need[t];
    const VRec r = g.vt[v];
    const uint32_t sl = r.deg + (bi - b[lo]);
    const uint32_t j = sl >> g.log2B, nb0 = nblocks(g, r.deg);
    const uint32_t blk = j < nb0 ? block_of(g, r, j) : planned_block(g, c, (uint64_t)p0 + (j - nb0));
    const uint64_t sa = ((uint64_t)blk << g.log2B) + (sl & (g.B - 1));
    g.pool[sa] = (uint32_t)(key & ((1ull << g.L) - 1));
    attr_zero(g, sa);
}

__device__ __forceinline__ uint32_t planned_segment(const GraphView& g, const DevCounters* c,
                                                    uint32_t cls, uint32_t rk) {
    return rk < c->plan_dff[cls]
               ? g.dfree[g.dfree_base[cls] + c->plan_dtop[cls] - 1 - rk]
               : (uint32_t)(c->plan_dbump[cls] + ((unsigned long long)(rk - c->plan_dff[cls]) << cls));
}

// Grow: every touched source with kept pairs gets its new block ids (and,
// when its block count outgrows its directory segment, a new segment holding
// a copy of the old entries) and its new vertex record.  A lane takes a
// source that copies and adds at most kLaneCopy entries; the others, listed
// (and flagged kHeavy) by the planning kernel, are taken by whole waves.
// The lane loop skips the flagged sources by the flag: a wave that has left
// the lane loop may already have written a heavy source's new record, and a
// decision made again from that record could take the source a second time.
__global__ __launch_bounds__(kThreads) void k_grow(GraphView g, const uint32_t* t_vtx,
                                                   const uint32_t* t_start, const uint32_t* b,
                                                   const uint32_t* t_need, const uint32_t* t_dreq,
                                                   const uint32_t* t_drank, uint32_t* t_dold,
                                                   uint32_t* t_doldc, const uint32_t* heavy) {
    const DevCounters* c = g.ctr;
    if (c->err_batch) return;
    const uint32_t nT = (uint32_t)c->tot[kTotSeg];
    const uint32_t lane = lane_id();
    const uint32_t stride = gridDim.x * kThreads;
    for (uint32_t base = global_wave() * 64; base < nT; base += stride) {
        const bool live = base + lane < nT;
        const uint32_t t = live ? base + lane : nT - 1;
        const uint32_t v = t_vtx[t], lo = t_start[t], hi = t_start[t + 1];
        const uint32_t p0 = t_need[t], req = t_dreq[t], rk = t_drank[t];
        const uint32_t kp = b[hi] - b[lo];
        if (!live || !kp || (req & kHeavy)) continue;
        const uint32_t cls = req & kClassMask;
        const VRec r = g.vt[v];  // only this lane writes it
        const uint32_t nb0 = nblocks(g, r.deg), nb1 = nblocks(g, r.deg + kp);
        VRec nr = r;
        nr.deg = r.deg + kp;
        if (cls != kNoDir) {
            const uint32_t off = planned_segment(g, c, cls, rk);
            // (a record keeps its segment when its degree drops, down to zero,
            // so nb0 may be 0 here: then entry 0 of the segment is read)
            uint32_t old[kLaneCopy];
#pragma unroll
            for (uint32_t j = 0; j < kLaneCopy; ++j)
                old[j] = block_of(g, r, min(j, nb0 ? nb0 - 1 : 0u));
#pragma unroll
            for (uint32_t j = 0; j < kLaneCopy; ++j)
                if (j < nb0) g.dir[(uint64_t)off + j] = old[j];
            t_dold[t] = r.dir;
            t_doldc[t] = r.dcls;
            nr.dir = off;
            nr.dcls = cls;
        }
        const uint32_t nnew = nb1 - nb0;
        if (nnew) {
            uint32_t ids[kLaneCopy];
#pragma unroll
            for (uint32_t j = 0; j < kLaneCopy; ++j)
                ids[j] = planned_block(g, c, (uint64_t)p0 + min(j, nnew - 1));
#pragma unroll
            for (uint32_t j = 0; j < kLaneCopy; ++j) {
                if (j >= nnew) continue;
                if (nr.dcls == kNoDir) nr.dir = ids[j];  // the only block, inline
                else g.dir[(uint64_t)nr.dir + nb0 + j] = ids[j];
                g.bown[ids[j]] = make_uint2(v, nb0 + j);
            }
        }
        g.vt[v] = nr;
    }
    const uint32_t nh = c->n_heavy;
    const uint32_t nw = gridDim.x * kWaves;
    for (uint32_t k = global_wave(); k < nh; k += nw) {
        const uint32_t t = heavy[k];
        const uint32_t v = t_vtx[t];
        const VRec r = g.vt[v];
        const uint32_t kp = b[t_start[t + 1]] - b[t_start[t]];
        const uint32_t nb0 = nblocks(g, r.deg), nb1 = nblocks(g, r.deg + kp);
        const uint32_t cls = t_dreq[t] & kClassMask;
        VRec nr = r;
        nr.deg = r.deg + kp;
        if (cls != kNoDir) {
            const uint32_t off = planned_segment(g, c, cls, t_drank[t]);
            for (uint32_t j = lane; j < nb0; j += 64) g.dir[(uint64_t)off + j] = block_of(g, r, j);
            if (lane == 0) {
                t_dold[t] = r.dir;
                t_doldc[t] = r.dcls;
            }
            nr.dir = off;
            nr.dcls = cls;
        }
        const uint64_t p0 = t_need[t];
        for (uint32_t j = nb0 + lane; j < nb1; j += 64) {
            const uint32_t blk = planned_block(g, c, p0 + (j - nb0));
            g.dir[(uint64_t)nr.dir + j] = blk;
            g.bown[blk] = make_uint2(v, j);
        }
        if (lane == 0) g.vt[v] = nr;
    }
}

// Old directory segments of the sources that moved go on the per-class free
// lists (after the commit kernel has taken its segments from them).
__global__ __launch_bounds__(kThreads) void k_final_ins(GraphView g, const uint32_t* rel,
                                                        const uint32_t* t_dold,
                                                        const uint32_t* t_doldc) {
    __shared__ uint32_t lcnt[kMaxClass];
    __shared__ uint32_t lbase[kMaxClass];
    __shared__ unsigned long long lfreed;
    const uint32_t nrel = g.ctr->err_batch ? 0u : (uint32_t)(g.ctr->tot[kTotB] >> 32);
    for (uint32_t base = blockIdx.x * kThreads; base < nrel; base += gridDim.x * kThreads) {
        if (threadIdx.x < kMaxClass) lcnt[threadIdx.x] = 0;
        if (threadIdx.x == 0) lfreed = 0;
        __syncthreads();
        const uint32_t k = base + threadIdx.x;
        uint32_t oc = kNoDir, lrank = 0, old = 0;
        if (k < nrel) {
            const uint32_t t = rel[k];
            oc = t_doldc[t];
            old = t_dold[t];
            lrank = atomicAdd(&lcnt[oc], 1u);
            atomicAdd(&lfreed, 1ull << oc);
        }
        __syncthreads();
        if (threadIdx.x < kMaxClass) {
            const uint32_t c = lcnt[threadIdx.x];
            lbase[threadIdx.x] = c ? atomicAdd(&g.ctr->dfree_cnt[threadIdx.x], c) : 0u;
        }
        if (threadIdx.x == 0 && lfreed)
            atomicAdd(&g.ctr->dir_live, (unsigned long long)(-(long long)lfreed));
        __syncthreads();
        if (oc != kNoDir) g.dfree[g.dfree_base[oc] + lbase[oc] + lrank] = old;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ delete

// a source that one lane compacts by itself
__device__ __forceinline__ bool lane_compactable(uint32_t r, uint32_t lo, uint32_t hi) {
    return r <= kLaneR && hi - lo <= kLaneSeg;
}

// a touched source of a delete batch with its hit count r
struct FreedRec {
    TouchRec x;
    uint32_t r;   // hits
    uint32_t rg;  // of which counted by group items (in the vertex scratch word)
};

struct FreedIn {
    static constexpr int kItems = 4;  // large records: fewer per thread
    GraphView g;
    const uint32_t* t_vtx;
    const uint32_t* t_start;
    const uint32_t* shits;
    using Rec = FreedRec;
    __device__ uint64_t limit(uint64_t n) const {
        return batch_failed(g.ctr) ? 0ull : min((uint64_t)(uint32_t)g.ctr->tot[kTotSeg], n);
    }
    __device__ Rec load(uint64_t t, bool ok) const {
        return Rec{load_touched(t_vtx, t_start, t, ok), shits[ok ? t : 0], 0u};
    }
    // the source's hits: its small item's count plus what its group items
    // added to its vertex scratch word
    __device__ void deref(Rec& f) const {
        f.x.r = g.vt[f.x.v];
        f.rg = g.vlost[f.x.v];
        f.r += f.rg;
    }
    // freed blocks in the low half; in the high half, 1 for a source that a
    // whole wave compacts (its rank among those is its slot in the list)
    __device__ unsigned long long value(uint64_t, const Rec& f) const {
        const uint32_t d = f.x.r.deg;
        if (!f.r) return 0ull;
        const unsigned long long mid =
            f.r <= kBigR && !lane_compactable(f.r, f.x.lo, f.x.hi) ? 1ull : 0ull;
        return (unsigned long long)(nblocks(g, d) - nblocks(g, d - f.r)) | (mid << 32);
    }
};

// Also clears each source's hit count (the vertex scratch word is zero
// between calls) and adds the hits of every workgroup into tot[kTotA].
struct FreedOut {
    DevCounters* ctr;
    CDesc* cd;
    uint32_t* big;
    uint32_t* mid;  // sources for whole waves
    uint32_t* vlost;
    __device__ void operator()(uint64_t t, const FreedRec& f, uint64_t lim,
                               unsigned long long pre) const {
        if (t >= lim) return;
        if (f.rg) vlost[f.x.v] = 0u;
        if (f.r && f.r <= kBigR && !lane_compactable(f.r, f.x.lo, f.x.hi))
            mid[(uint32_t)(pre >> 32)] = (uint32_t)t;
        CDesc c;
        c.lo = f.x.lo;
        c.hi = f.x.hi;
        c.r = f.r;
        c.v = f.x.v;
        c.deg = f.x.r.deg;
        c.dir = f.x.r.dir;
        c.dcls = f.x.r.dcls;
        c.need = (uint32_t)pre;
        cd[t] = c;
        if (c.r > kBigR) big[atomicAdd(&ctr->n_big, 1u)] = (uint32_t)t;
    }
    __device__ unsigned long long tally(uint64_t, const FreedRec& f) const { return f.r; }
    __device__ void commit(unsigned long long sum) const {
        if (sum) atomicAdd(&ctr->tot[kTotA], sum);
    }
};

// Compaction of every touched source with at most kBigR hits: holes below the
// new degree (taken in batch order) receive the survivors found above it (in
// slot order), and emptied blocks go on the free list.  A lane takes a source
// with at most kLaneR hits and a short segment; the others are taken by the
// whole wave in turn.
__device__ __forceinline__ void compact_body(const GraphView& g, const uint8_t* mark,
                                             const uint32_t* hitpos, uint32_t* holes,
                                             const CDesc* cdesc, const uint32_t* mid,
                                             uint32_t vb, uint32_t vg) {
    const uint32_t gwave = (vb * kThreads + threadIdx.x) >> 6;
    const DevCounters* c = g.ctr;
    const uint32_t nT = (uint32_t)c->tot[kTotSeg];
    const uint32_t lane = lane_id();
    const uint64_t below = (1ull << lane) - 1;
    const uint32_t stride = vg * kThreads;
    const unsigned long long fbase = c->free_cnt;
    const uint32_t bm = g.B - 1;
    unsigned long long moved = 0;
    for (uint32_t base = gwave * 64; base < nT; base += stride) {
        const bool live = base + lane < nT;
        const CDesc D = cdesc[live ? base + lane : nT - 1];
        if (live && D.r && lane_compactable(D.r, D.lo, D.hi)) {
            const VRec rec{D.deg, D.dir, D.dcls, 0u};
            const uint32_t d = D.deg, dn = d - D.r;
            uint8_t mk[kLaneSeg];
            uint32_t hp[kLaneSeg], sb[kLaneR];
#pragma unroll
            for (uint32_t u = 0; u < kLaneSeg; ++u) {
                const uint32_t q = min(D.lo + u, D.hi - 1);
                mk[u] = mark[q];
                hp[u] = hitpos[q];
            }
#pragma unroll
            for (uint32_t k = 0; k < kLaneR; ++k)
                sb[k] = block_of(g, rec, min(dn + k, d - 1) >> g.log2B);
            uint32_t sv[kLaneR];
#pragma unroll
            for (uint32_t k = 0; k < kLaneR; ++k)
                sv[k] = g.pool[((uint64_t)sb[k] << g.log2B) + (min(dn + k, d - 1) & bm)];
            // holes in batch order, survivors in slot order
            uint32_t hm = 0, sm = 0;
#pragma unroll
            for (uint32_t u = 0; u < kLaneSeg; ++u)
                hm |= (D.lo + u < D.hi && mk[u] && hp[u] < dn) ? (1u << u) : 0u;
#pragma unroll
            for (uint32_t k = 0; k < kLaneR; ++k)
                sm |= (k < D.r && sv[k] != kTomb) ? (1u << k) : 0u;
            uint32_t hslot[kLaneR], hval[kLaneR], hsrc[kLaneR];
            uint32_t nmove = 0;
#pragma unroll
            for (uint32_t k = 0; k < kLaneR; ++k) {
                hslot[k] = 0;
                hval[k] = 0;
                hsrc[k] = 0;
                if (hm && sm) {
                    const uint32_t u = __builtin_ctz(hm), w = __builtin_ctz(sm);
                    hm &= hm - 1;
                    sm &= sm - 1;
                    hslot[k] = hp[u];
                    hval[k] = sv[w];
                    hsrc[k] = w;
                    nmove = k + 1;
                }
            }
            uint32_t hb[kLaneR];
#pragma unroll
            for (uint32_t k = 0; k < kLaneR; ++k) hb[k] = block_of(g, rec, hslot[k] >> g.log2B);
#pragma unroll
            for (uint32_t k = 0; k < kLaneR; ++k) {
                if (k >= nmove) continue;
                const uint64_t da = ((uint64_t)hb[k] << g.log2B) + (hslot[k] & bm);
                g.pool[da] = hval[k];
                if (g.A) {
                    // the survivor sat at slot dn + w (w < r <= kLaneR)
                    uint32_t sbw = sb[0];
#pragma unroll
                    for (uint32_t j = 1; j < kLaneR; ++j) sbw = hsrc[k] == j ? sb[j] : sbw;
                    attr_move(g, da, ((uint64_t)sbw << g.log2B) + ((dn + hsrc[k]) & bm));
                }
            }
            moved += nmove;
            const uint32_t nb0 = nblocks(g, d), nb1 = nblocks(g, dn);
            const unsigned long long pb = fbase + D.need;
#pragma unroll
            for (uint32_t k = 0; k < kLaneR; ++k)
                if (nb1 + k < nb0) g.free_stack[pb + k] = block_of(g, rec, nb1 + k);
            VRec nr = rec;
            nr.deg = dn;
            if (nb1 == 0 && nr.dcls == kNoDir) nr.dir = 0;
            g.vt[D.v] = nr;
        }
    }
    // sources with more hits or longer segments, listed by the freed scan:
    // one wave each
    const uint32_t nmid = (uint32_t)(c->tot[kTotB] >> 32);
    const uint32_t nw = vg * kWaves;
    for (uint32_t k = gwave; k < nmid; k += nw) {
        {
            const CDesc H = cdesc[mid[k]];
            const VRec rec{H.deg, H.dir, H.dcls, 0u};
            const uint32_t d = H.deg, dn = d - H.r;
            uint32_t nh = 0;
            for (uint32_t p0 = H.lo; p0 < H.hi; p0 += 64) {
                const uint32_t p = p0 + lane;
                const uint32_t q = min(p, H.hi - 1);
                const uint8_t m = mark[q];
                const uint32_t hpv = hitpos[q];
                const bool hole = p < H.hi && m && hpv < dn;
                const uint64_t bal = ballot(hole);
                if (hole) holes[H.lo + nh + popc64(bal & below)] = hpv;
                nh += popc64(bal);
            }
            __threadfence_block();
            uint32_t ns = 0;
            for (uint32_t s0 = dn; s0 < d; s0 += 64) {
                const uint32_t sl = s0 + lane;
                uint32_t x = kTomb;
                if (sl < d) x = g.pool[slot_addr(g, rec, sl)];
                const bool surv = x != kTomb;
                const uint64_t bal = ballot(surv);
                if (surv) {
                    // survivors above dn and holes below it are equal in number;
                    // the guards only keep a broken invariant from writing wild
                    const uint32_t qq = ns + popc64(bal & below);
                    if (qq < nh) {
                        const uint32_t dest = holes[H.lo + qq];
                        if (dest < dn) {
                            const uint64_t da = slot_addr(g, rec, dest);
                            g.pool[da] = x;
                            if (g.A) attr_move(g, da, slot_addr(g, rec, sl));
                        }
                    }
                }
                ns += popc64(bal);
            }
            moved += lane == 0 ? ns : 0;
            const uint32_t nb0 = nblocks(g, d), nb1 = nblocks(g, dn);
            const unsigned long long pb = fbase + H.need;
            for (uint32_t j = nb1 + lane; j < nb0; j += 64)
                g.free_stack[pb + (j - nb1)] = block_of(g, rec, j);
            if (lane == 0) {
                VRec nr = rec;
                nr.deg = dn;
                if (nb1 == 0 && nr.dcls == kNoDir) nr.dir = 0;
                g.vt[H.v] = nr;
            }
        }
    }
    moved = wave_sum(moved);
    if (lane == 0 && moved) atomicAdd(&g.ctr->stripe[gwave & 63][0], moved);
}

// One workgroup per source with more than kBigR hits (hubs), same pairing.
__device__ __forceinline__ void compact_big_body(const GraphView& g, const uint8_t* mark,
                                                 const uint32_t* hitpos, uint32_t* holes,
                                                 const CDesc* cdesc, const uint32_t* big,
                                                 uint32_t vb, uint32_t vg) {
    __shared__ uint32_t lds[kWaves];
    const DevCounters* c = g.ctr;
    const uint32_t nbig = c->n_big;
    const unsigned long long fbase = c->free_cnt;
    const uint32_t tid = threadIdx.x;
    unsigned long long moved = 0;
    for (uint32_t q = vb; q < nbig; q += vg) {
        const CDesc D = cdesc[big[q]];
        const VRec rec{D.deg, D.dir, D.dcls, 0u};
        const uint32_t d = D.deg, dn = d - D.r;
        uint32_t nh = 0;
        for (uint32_t p0 = D.lo; p0 < D.hi; p0 += kThreads) {
            const uint32_t p = p0 + tid;
            uint32_t hole = 0, hp = 0;
            if (p < D.hi && mark[p]) {
                hp = hitpos[p];
                hole = hp < dn;
            }
            uint32_t tot;
            const uint32_t ex = block_excl_scan(hole, lds, tot);
            if (hole) holes[D.lo + nh + ex] = hp;
            nh += tot;
        }
        __syncthreads();
        uint32_t ns = 0;
        for (uint32_t s0 = dn; s0 < d; s0 += kThreads) {
            const uint32_t s = s0 + tid;
            uint32_t x = kTomb;
            if (s < d) x = g.pool[slot_addr(g, rec, s)];
            const uint32_t surv = x != kTomb;
            uint32_t tot;
            const uint32_t ex = block_excl_scan(surv, lds, tot);
            if (surv) {
                const uint32_t qq = ns + ex;
                if (qq < nh) {
                    const uint32_t dest = holes[D.lo + qq];
                    if (dest < dn) {
                        const uint64_t da = slot_addr(g, rec, dest);
                        g.pool[da] = x;
                        if (g.A) attr_move(g, da, slot_addr(g, rec, s));
                    }
                }
            }
            ns += tot;
        }
        moved += tid == 0 ? ns : 0;
        const uint32_t nb0 = nblocks(g, d), nb1 = nblocks(g, dn);
        const unsigned long long pb = fbase + D.need;
        for (uint32_t j = nb1 + tid; j < nb0; j += kThreads)
            g.free_stack[pb + (j - nb1)] = block_of(g, rec, j);
        if (tid == 0) {
            VRec nr = rec;
            nr.deg = dn;
            if (nb1 == 0 && nr.dcls == kNoDir) nr.dir = 0;
            g.vt[D.v] = nr;
        }
        __syncthreads();
    }
    if (tid == 0 && moved) atomicAdd(&g.ctr->stripe[vb & 63][0], moved);
}

// Both compactions in one launch: the first nbig workgroups take the hubs
// (they run longest, so they start first), the rest the other sources.
__global__ __launch_bounds__(kThreads) void k_compact(GraphView g, const uint8_t* mark,
                                                      const uint32_t* hitpos, uint32_t* holes,
                                                      const CDesc* cdesc, const uint32_t* mid,
                                                      const uint32_t* big, uint32_t nbig) {
    if (batch_failed(g.ctr)) return;
    if (blockIdx.x < nbig)
        compact_big_body(g, mark, hitpos, holes, cdesc, big, blockIdx.x, nbig);
    else
        compact_body(g, mark, hitpos, holes, cdesc, mid, blockIdx.x - nbig, gridDim.x - nbig);
}


__global__ void k_final_del(GraphView g, uint64_t n) {
    DevCounters* c = g.ctr;
    if (batch_failed(c)) {
        c->err_batch = GV_EDEVICE;
        return;
    }
    const unsigned long long nv = c->tot[kTotValid];
    const unsigned long long nT = c->tot[kTotSeg] & 0xffffffffull;
    const unsigned long long nuniq = c->tot[kTotSeg] >> 32;
    const unsigned long long applied = c->tot[kTotA];
    const unsigned long long freed = c->tot[kTotB] & 0xffffffffull;
    c->free_cnt += freed;
    c->st_applied = applied;
    c->st_rejected = n - nv;
    c->st_dups = nv - nuniq;
    c->c_batches[kDelete] += 1;
    c->c_pairs[kDelete] += n;
    c->c_touched[kDelete] += nT;
    c->c_scanned[kDelete] += (c->tot[kTotItems] >> 32) << g.log2B;
    c->c_freed_blocks += freed;
    c->live_edges -= applied;
}

// ------------------------------------------------------------------ query
__global__ __launch_bounds__(kThreads) void k_answer(GraphView g, const uint32_t* vals,
                                                     const uint8_t* mark, uint64_t n,
                                                     uint8_t* out) {
    const uint64_t i = thread_index();
    if (batch_failed(g.ctr)) return;  // the answers are not written; the call reports the error
    const unsigned long long nv = g.ctr->tot[kTotValid];
    if (i == 0) {
        DevCounters* c = g.ctr;
        c->c_batches[kQuery] += 1;
        c->c_pairs[kQuery] += n;
        c->c_touched[kQuery] += c->tot[kTotSeg] & 0xffffffffull;
        c->c_scanned[kQuery] += (c->tot[kTotItems] >> 32) << g.log2B;
    }
    if (i < nv && vals[i] < n) out[vals[i]] = mark[i];
}

// ------------------------------------------------------------------ attributes
// get: a found pair's attributes (read at the slot the probe recorded) at
// its input position; a pair not found reads zeros
__global__ __launch_bounds__(kThreads) void k_attr_get(GraphView g, const uint64_t* keys,
                                                       const uint32_t* vals, const uint8_t* mark,
                                                       const uint32_t* hitpos, uint64_t n,
                                                       uint32_t* out) {
    const uint64_t i = thread_index();
    if (batch_failed(g.ctr)) return;
    const uint64_t nv = min((uint64_t)g.ctr->tot[kTotValid], n);
    if (i >= nv || vals[i] >= n) return;
    const uint64_t o = (uint64_t)vals[i] * g.A;
    if (!mark[i]) {
        for (uint32_t k = 0; k < g.A; ++k) out[o + k] = 0u;
        return;
    }
    const uint64_t a = slot_addr(g, g.vt[keys[i] >> g.L], hitpos[i]);
    for (uint32_t k = 0; k < g.A; ++k) out[o + k] = g.apool[a * g.A + k];
}

// set: the last occurrence of each found pair in input order (the sort is
// stable, so the last of its run) writes its attributes; counts for the
// statistics
__global__ __launch_bounds__(kThreads) void k_attr_set(GraphView g, const uint64_t* keys,
                                                       const uint32_t* vals, const uint8_t* mark,
                                                       const uint32_t* hitpos, uint64_t n,
                                                       const uint32_t* in) {
    __shared__ unsigned long long lds[kWaves];
    const uint64_t i = thread_index();
    if (batch_failed(g.ctr)) return;
    const uint64_t nv = min((uint64_t)g.ctr->tot[kTotValid], n);
    unsigned long long distinct = 0, applied = 0;
    if (i < nv) {
        const bool last = i + 1 >= nv || keys[i + 1] != keys[i];
        distinct = last;
        if (last && mark[i] && vals[i] < n) {
            applied = 1;
            const uint64_t a = slot_addr(g, g.vt[keys[i] >> g.L], hitpos[i]);
            const uint64_t o = (uint64_t)vals[i] * g.A;
            for (uint32_t k = 0; k < g.A; ++k) g.apool[a * g.A + k] = in[o + k];
        }
    }
    distinct = block_sum(distinct, lds);
    applied = block_sum(applied, lds);
    if (threadIdx.x == 0) {
        if (distinct) atomicAdd(&g.ctr->n_uniq, distinct);
        if (applied) atomicAdd(&g.ctr->st_applied, applied);
    }
}

__global__ void k_attr_begin(DevCounters* c) {
    c->n_uniq = 0;
    c->st_applied = 0;
}

__global__ __launch_bounds__(kThreads) void k_zero_attr(uint32_t* p, uint64_t n) {
    const uint64_t i = thread_index();
    if (i < n) p[i] = 0u;
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
// Runs f on the probe variant of MODE for lanes-per-item G and slots-per-lane
// U chosen at run time (the shapes the tuning accepts).
template <int MODE, typename F>
static void with_probe(uint32_t group, uint32_t unroll, F&& f) {
#define GV_PROBE_SHAPE(G, U) \
    if (group == G && unroll == U) return f(k_probe<MODE, G, U>);
    GV_PROBE_SHAPE(16, 2) GV_PROBE_SHAPE(16, 4) GV_PROBE_SHAPE(16, 8)
    GV_PROBE_SHAPE(32, 2) GV_PROBE_SHAPE(32, 4) GV_PROBE_SHAPE(32, 8)
    GV_PROBE_SHAPE(64, 2) GV_PROBE_SHAPE(64, 4) GV_PROBE_SHAPE(64, 8)
#undef GV_PROBE_SHAPE
    fail(GV_EINVAL, "probe shape");
}

bool probe_shape_ok(uint32_t group, uint32_t unroll) {
    return (group == 16 || group == 32 || group == 64) && (unroll == 2 || unroll == 4 || unroll == 8);
}

// occupancy lookups of the looping kernels, made before a recording: the
// probe shape of the graph's tuning, or every shape when g is null
void edge_batch_warm(const gv_graph* g) {
    auto warm = [](auto kernel) { resident_grid(kernel, kThreads); };
    for (uint32_t pg : {16u, 32u, 64u}) {
        for (uint32_t pu : {2u, 4u, 8u}) {
            if (g && (pg != g->tune.probe_group || pu != g->tune.probe_unroll)) continue;
            with_probe<kInsert>(pg, pu, warm);
            with_probe<kDelete>(pg, pu, warm);
            with_probe<kQuery>(pg, pu, warm);
            with_probe<kLocate>(pg, pu, warm);
        }
    }
    resident_grid(k_grow, kThreads);
    resident_grid(k_compact, kThreads);
    resident_grid(k_os_pass<uint64_t, false>, kOsThreads);
    resident_grid(k_os_pass<uint64_t, true>, kOsThreads);
}

// bytes of g->scratch edge_batch carves for n pairs (edge_batch_sorted carves
// the same)
size_t edge_batch_bytes(const gv_graph* g, EdgeMode mode, uint64_t n) {
    if (n == 0) return 0;
    BatchArrays A;
    Carver m(nullptr);
    carve_batch(m, A, n, n + div_up(g->item_slots, (uint64_t)g->tune.item_chunk) + 1, mode,
                2 * (int)g->v.L);
    return m.used;
}

// Insert and delete batches whose keys arrive sorted (keys[0, *count), the
// count on the device; they come from the library's own sort of a mixed
// list): one kernel clears the marks, and its first workgroup clears the
// batch counters, sets the valid count and turns the probe's multiset check
// off (there is no packing to compare with; the segment scan still checks
// the order).
__global__ __launch_bounds__(kThreads) void k_sorted_prep(GraphView g,
                                                          const unsigned long long* count,
                                                          uint64_t n, uint8_t* mark) {
    const uint64_t i = thread_index();
    if (i < n) mark[i] = 0;
    if (blockIdx.x == 0) {
        clear_batch_counters(g.ctr, threadIdx.x);
        if (threadIdx.x == 0) {
            g.ctr->tot[kTotValid] = *count;
            g.ctr->tot[kTotNoHash] = 1;
        }
    }
}

static void edge_run(gv_graph* g, EdgeMode mode, const uint32_t* src, const uint32_t* dst,
                     const uint64_t* sorted, const unsigned long long* sorted_n, uint64_t n,
                     uint8_t* out, bool sticky, void* fixed, size_t fixed_bytes,
                     uint8_t* mark_out, const AttrOp* aop = nullptr);

void edge_batch(gv_graph* g, EdgeMode mode, const uint32_t* src, const uint32_t* dst, uint64_t n,
                uint8_t* out, bool sticky, void* fixed, size_t fixed_bytes) {
    edge_run(g, mode, src, dst, nullptr, nullptr, n, out, sticky, fixed, fixed_bytes, nullptr);
}

void edge_batch_sorted(gv_graph* g, EdgeMode mode, const uint64_t* keys,
                       const unsigned long long* count, uint64_t n_max, bool sticky,
                       uint8_t* mark_out) {
    if (mode == kQuery) fail(GV_EINVAL, "sorted batches are inserts or deletes");
    edge_run(g, mode, nullptr, nullptr, keys, count, n_max, nullptr, sticky, nullptr, 0,
             mark_out);
}

void edge_attrs(gv_graph* g, const uint32_t* src, const uint32_t* dst, uint64_t n,
                uint8_t* found, uint32_t* out, const uint32_t* in) {
    if (n == 0) return;
    const AttrOp op{out, in};
    Ctx& c = g->ctx;
    if (out) {
        // answers of invalid pairs are written by the packing scan; their
        // attributes read zeros
        c.launch("attr_get", k_zero_attr, div_up(n * g->v.A, kThreads), kThreads, out,
                 n * g->v.A);
    } else {
        c.launch("attr_set", k_attr_begin, 1, 1, g->v.ctr);
    }
    edge_run(g, kQuery, src, dst, nullptr, nullptr, n, found, true, nullptr, 0, nullptr, &op);
}

// First kernel of an overlapped batch on the graph's stream: clears the
// batch counters and takes the valid-pair count and key sum that the batch's
// packing left in its buffer.
__global__ void k_ov_begin(GraphView g, const unsigned long long* stot) {
    clear_batch_counters(g.ctr, threadIdx.x);
    if (threadIdx.x == 0) {
        g.ctr->tot[kTotValid] = stot[0];
        g.ctr->tot[kTotHash] = stot[1];
    }
}

void overlap_open(gv_graph* g) {
    gv_graph::Overlap& o = g->ov;
    if (o.stream) return;
    hip_check(hipStreamCreateWithFlags(&o.stream, hipStreamNonBlocking), "hipStreamCreate");
    o.ctx.stream = o.stream;
    hipEvent_t* evs[] = {&o.sorted[0], &o.sorted[1], &o.done[0],    &o.done[1], &o.fence,
                         &o.msorted[0], &o.msorted[1], &o.mdone[0], &o.mdone[1]};
    for (hipEvent_t* e : evs)
        hip_check(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreate");
}

// the id of the capture the stream is in, 0 when it is not being captured
static unsigned long long capture_id(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hip_check(hipStreamGetCaptureInfo(s, &st, &id), "hipStreamGetCaptureInfo");
    return st == hipStreamCaptureStatusActive ? id : 0ull;
}

void overlap_capture(gv_graph* g) {
    gv_graph::Overlap& o = g->ov;
    const unsigned long long cap = capture_id(g->ctx.stream);
    if (cap == o.capture) return;
    o.capture = cap;
    o.used[0] = o.used[1] = false;
    o.mused[0] = o.mused[1] = false;
    o.seq = ~0ull;
    o.joined = false;
}

void overlap_fence(gv_graph* g) {
    gv_graph::Overlap& o = g->ov;
    hip_check(hipEventRecord(o.fence, g->ctx.stream), "hipEventRecord");
    hip_check(hipStreamWaitEvent(o.stream, o.fence, 0), "hipStreamWaitEvent");
    o.joined = true;
}

static void edge_run(gv_graph* g, EdgeMode mode, const uint32_t* src, const uint32_t* dst,
                     const uint64_t* sorted, const unsigned long long* sorted_n, uint64_t n,
                     uint8_t* out, bool sticky, void* fixed, size_t fixed_bytes,
                     uint8_t* mark_out, const AttrOp* aop) {
    if (n == 0) return;
    if (n >= 0x3fffffffull) fail(GV_EINVAL, "batch too large");
    if (mode == kInsert) g->edge_bound_host += n;
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    const uint64_t icap = n + div_up(g->item_slots, (uint64_t)g->tune.item_chunk) + 1;
    const int bits = 2 * (int)v.L;
    // sort overlap: this batch's pack and sort go to the side stream (also
    // while the graph's stream is captured: the side stream then joins the
    // capture through the first wait, and the recording keeps both branches)
    const bool ovb = g->tune.overlap && !sorted && !fixed && mode != kQuery && bits > 0 &&
                     n > std::min<uint64_t>(g->tune.small_sort_max, kOsTile);
    if (ovb) overlap_capture(g);
    const int ob = (int)(g->ov.count & 1);  // its buffer
    BatchArrays A;
    {
        Carver m(nullptr);
        carve_batch(m, A, n, icap, mode, bits);
        void* base = fixed;
        if (fixed) {
            if (m.used > fixed_bytes) fail(GV_ERANGE, "batch does not fit the fixed scratch");
        } else {
            // a buffer that grows first synchronises the graph's stream, and
            // with it every sort queued on the side stream
            Scratch& buf = ovb && ob ? g->ov.scr : g->scratch;
            buf.ensure(m.used, c.stream);
            base = buf.ptr;
        }
        Carver cv(base);
        carve_batch(cv, A, n, icap, mode, bits);
        // a sorted batch's probe writes its per-key result where the caller
        // wants it (n_max bytes)
        if (mark_out && sorted) A.mark = mark_out;
    }
    DevCounters* ctr = v.ctr;
    uint32_t* err = &ctr->err_wait;
    unsigned long long* tot = ctr->tot;
    const unsigned long long* n_valid = &tot[kTotValid];
    const uint64_t grid = div_up(n, kThreads);

    bool flip;
    const uint64_t* keys_in = nullptr;
    if (sorted) {
        c.launch("pack", k_sorted_prep, grid, kThreads, v, sorted_n, n, A.mark);
        keys_in = sorted;
        flip = false;
    } else if (mode == kQuery && n <= kOsTile && bits + kTilePosBits < 64) {
        c.launch("pack", k_query_sort_tile, 1, kOsThreads, v, src, dst, n,
                 os_passes(bits + kTilePosBits), A.keys0, A.vals0, out, A.mark);
        flip = false;
    } else if (mode == kQuery) {
        c.launch("begin", k_begin, std::min<uint64_t>(div_up(A.state_words, kThreads), 1024),
                 kThreads, v, A.state, A.state_words);
        scan2(c, "pack", PackIn{v, src, dst}, PackOut{v.L, A.keys0, A.vals0, out, A.mark}, n,
              A.part, &tot[kTotValid]);
        flip = onesweep<uint64_t, true>(c, A.keys0, A.keys1, A.vals0, A.vals1,
                                        (const uint32_t*)n_valid, n, bits, A.state, err,
                                        g->spin_limit);
    } else if (n <= std::min<uint64_t>(g->tune.small_sort_max, kOsTile) && bits > 0) {
        const uint64_t sentinel = bits >= 64 ? ~0ull : (1ull << bits) - 1;
        c.launch("pack", k_pack_sort_tile, 1, kOsThreads, v, src, dst, n, os_passes(bits),
                 sentinel, A.keys0, A.mark);
        flip = false;
    } else if (ovb) {
        // The side stream reads the pairs and the activity bitmap (which no
        // edge batch changes) and writes only this batch's buffer: it waits
        // for the graph's stream when anything else was queued there since
        // the last overlapped batch, and for the batch that used the buffer
        // before.  The batch counters are cleared on the graph's stream, once
        // the batch before has finished with them.
        gv_graph::Overlap& o = g->ov;
        overlap_open(g);
        Ctx& sc = o.ctx;
        sc.prof = c.prof;
        sc.only = c.only;
        if (c.seq != o.seq) {
            overlap_fence(g);
        } else if (o.used[ob]) {
            // (with a fence, the wait for the graph's stream covers this one)
            hip_check(hipStreamWaitEvent(o.stream, o.done[ob], 0), "hipStreamWaitEvent");
        }
        const uint64_t sentinel = bits >= 64 ? ~0ull : (1ull << bits) - 1;
        sc.launch("pack", k_pack_hist, os_hist_groups(n), kOsThreads, v, src, dst, n,
                  os_passes(bits), sentinel, A.keys0, A.mark, A.state, A.state_words,
                  os_hpart(A.state, n, bits), A.vpart, A.hpart, 0);
        os_hist_sum(sc, A.state, n, bits, (const uint32_t*)A.vpart, &A.stot[0],
                    (const unsigned long long*)A.hpart, &A.stot[1]);
        flip = onesweep_passes<uint64_t, false>(sc, A.keys0, A.keys1, nullptr, nullptr, nullptr, n,
                                                bits, A.state, err, g->spin_limit, true);
        sc.close_run();
        hip_check(hipEventRecord(o.sorted[ob], o.stream), "hipEventRecord");
        hip_check(hipStreamWaitEvent(c.stream, o.sorted[ob], 0), "hipStreamWaitEvent");
        // the segment scan's first kernel clears the batch counters (a batch
        // of one scan tile has no such kernel: a kernel of its own does it)
        if (scan2_tiles<SegIn>(n) <= 1)
            c.launch("pack", k_ov_begin, 1, 64, v, (const unsigned long long*)A.stot);
    } else {
        const uint64_t sentinel = bits >= 64 ? ~0ull : (1ull << bits) - 1;
        c.launch("pack", k_pack_hist, os_hist_groups(n), kOsThreads, v, src, dst, n,
                 bits > 0 ? os_passes(bits) : 0, sentinel, A.keys0, A.mark, A.state,
                 A.state_words, os_hpart(A.state, n, bits), A.vpart, A.hpart, 1);
        os_hist_sum(c, A.state, n, bits, (const uint32_t*)A.vpart, &tot[kTotValid],
                    (const unsigned long long*)A.hpart, &tot[kTotHash]);
        flip = onesweep_passes<uint64_t, false>(c, A.keys0, A.keys1, nullptr, nullptr, nullptr, n,
                                                bits, A.state, err, g->spin_limit);
    }
    const uint64_t* keys = keys_in ? keys_in : flip ? A.keys1 : A.keys0;
    const uint32_t* vals = flip ? A.vals1 : A.vals0;

    const bool seg_clears = ovb && scan2_tiles<SegIn>(n) > 1;
    scan2(c, "segments",
          SegIn{keys, ctr, v.L, ovb ? (const unsigned long long*)A.stot : n_valid,
                seg_clears ? ctr : nullptr},
          SegOut{v.L, A.flags, A.a, A.t_vtx, A.t_start, ctr}, n, A.part,
          &tot[kTotSeg]);
    const uint32_t chunk = g->tune.item_chunk;
    scan2(c, "items", ItemIn{v, A.t_vtx, A.t_start, chunk},
          ItemOut{A.items, A.small, v.B, icap, chunk, mode == kDelete ? A.b : nullptr}, n,
          A.part, &tot[kTotItems]);
    const uint32_t pg = g->tune.probe_group, pu = g->tune.probe_unroll;
    const uint64_t pwant = div_up(icap, (uint64_t)kWaves * (64 / pg));
    // launches the probe variant of the graph's tuning
    auto probe = [&](auto mode_tag, const char* name, uint32_t* hitpos) {
        constexpr int M = decltype(mode_tag)::value;
        with_probe<M>(pg, pu, [&](auto kernel) {
            c.launch(name, kernel, std::min<uint64_t>(pwant, resident_grid(kernel, kThreads)),
                     kThreads, v, keys, (const Item*)A.items, (const Item*)A.small, A.mark,
                     hitpos, A.b);
        });
    };
    const uint64_t tgrid = std::min<uint64_t>(div_up(n, kThreads), resident_grid(k_grow, kThreads));

    if (mode == kInsert) {
        probe(std::integral_constant<int, kInsert>{}, "probe_insert", nullptr);
        scan2(c, "keep", KeepIn{A.flags, A.mark, ctr}, U32Out{A.b}, n + 1, A.part,
              &tot[kTotA]);
        c.launch("plan_insert", k_plan_ins, grid, kThreads, v, (const uint32_t*)A.t_vtx,
                 (const uint32_t*)A.t_start, (const uint32_t*)A.b, A.t_need, A.t_dreq, A.t_drank,
                 A.heavy);
        scan2(c, "need", NeedIn{A.t_need, ctr}, NeedOut{A.t_need, A.rel, v, n, (int)sticky},
              n + 1, A.part, &tot[kTotB]);
        c.launch("append", k_append, grid, kThreads, v, keys, (const uint8_t*)A.flags,
                 (const uint8_t*)A.mark, (const uint32_t*)A.a, (const uint32_t*)A.b,
                 (const uint32_t*)A.t_vtx, (const uint32_t*)A.t_start,
                 (const uint32_t*)A.t_need);
        c.launch("grow", k_grow, tgrid, kThreads, v, (const uint32_t*)A.t_vtx,
                 (const uint32_t*)A.t_start, (const uint32_t*)A.b, (const uint32_t*)A.t_need,
                 (const uint32_t*)A.t_dreq, (const uint32_t*)A.t_drank, A.t_dold, A.t_doldc,
                 (const uint32_t*)A.heavy);
        c.launch("final_insert", k_final_ins, std::min<uint64_t>(grid, 64), kThreads, v,
                 (const uint32_t*)A.rel, (const uint32_t*)A.t_dold, (const uint32_t*)A.t_doldc);
    } else if (mode == kDelete) {
        probe(std::integral_constant<int, kDelete>{}, "probe_delete", A.hitpos);
        scan2(c, "freed", FreedIn{v, A.t_vtx, A.t_start, A.b},
              FreedOut{ctr, A.cdesc, A.big, A.heavy, v.vlost}, n, A.part, &tot[kTotB]);
        const uint32_t nbig = kBigGroups;
        c.launch("compact", k_compact,
                 nbig + std::min<uint64_t>(div_up(n, kThreads), resident_grid(k_compact, kThreads)),
                 kThreads, v, (const uint8_t*)A.mark, (const uint32_t*)A.hitpos, A.holes,
                 (const CDesc*)A.cdesc, (const uint32_t*)A.heavy, (const uint32_t*)A.big, nbig);
        c.launch("final_delete", k_final_del, 1, 1, v, n);
    } else if (aop) {
        probe(std::integral_constant<int, kLocate>{}, "probe_locate", A.hitpos);
        if (aop->out) {
            c.launch("answer", k_answer, grid, kThreads, v, vals, (const uint8_t*)A.mark, n, out);
            c.launch("attr_get", k_attr_get, grid, kThreads, v, keys, vals,
                     (const uint8_t*)A.mark, (const uint32_t*)A.hitpos, n, aop->out);
        } else {
            c.launch("attr_set", k_attr_set, grid, kThreads, v, keys, vals,
                     (const uint8_t*)A.mark, (const uint32_t*)A.hitpos, n, aop->in);
        }
    } else {
        probe(std::integral_constant<int, kQuery>{}, "probe_query", nullptr);
        c.launch("answer", k_answer, grid, kThreads, v, vals, (const uint8_t*)A.mark, n, out);
    }
    if (ovb) {
        gv_graph::Overlap& o = g->ov;
        hip_check(hipEventRecord(o.done[ob], c.stream), "hipEventRecord");
        o.used[ob] = true;
        ++o.count;
        o.seq = c.seq;
    }
}

}  // namespace gv
