// gv_served.hip -- mixed edge updates with last-writer reduction: the tick of
// the served form, and the unit the batched form coalesces runs of edge
// batches into.
//
// A list of (op, src, dst) entries, op 0 = insert and 1 = delete, has the
// effect of applying the entries one at a time in list order with set
// semantics (Sec. 4.3's batch model; the order inside a batch is ours): a
// pair's final membership is decided by its last entry, and entries with an
// inactive or out-of-range endpoint change nothing.  On the device: pack the
// valid entries as keys (src << L) | dst with their list position (an invalid
// entry gets bit 2L, after every valid key), sort them stably, and keep the
// last entry of every key: a scan writes the kept deletes and the kept
// inserts, compacted and still sorted, to two key lists (a list of at most
// one tile is packed and sorted by one workgroup).  The two lists are
// then applied as a delete batch and an insert batch that start from their
// sorted keys (no second sort); no key is in both, so their order does not
// matter.
#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

namespace {

__global__ __launch_bounds__(kThreads) void k_mixed_pack(GraphView g, const uint8_t* op,
                                                         const uint32_t* src,
                                                         const uint32_t* dst, uint64_t n,
                                                         uint64_t* keys, uint32_t* pos) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = src[i], d = dst[i];
    const bool ok = active_bit(g, s) & active_bit(g, d) & (op[i] <= 1);
    keys[i] = ok ? ((uint64_t)s << g.L) | d : (1ull << (2 * g.L));
    pos[i] = (uint32_t)i;
}

// Lists of at most one tile: one workgroup packs each entry as its key with
// its list position in the low 12 bits ((pair << 12) | position, an invalid
// entry with bit 2L set above the pair) and sorts the tile in LDS, which is
// the stable order by pair; the pair keys and positions go out separately,
// as the general path leaves them.
constexpr int kTilePosBits = 12;  // kOsTile = 4096 positions
__global__ __launch_bounds__(kOsThreads) void k_mixed_sort_tile(GraphView g, const uint8_t* op,
                                                                const uint32_t* src,
                                                                const uint32_t* dst, uint64_t n,
                                                                int passes, uint64_t* keys,
                                                                uint32_t* pos) {
    __shared__ TileSortLds lds;
    uint64_t key[kOsRounds];
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + threadIdx.x;
        uint64_t k = 0;
        if (i < n) {
            const uint32_t s = src[i], d = dst[i];
            const bool ok = active_bit(g, s) & active_bit(g, d) & (op[i] <= 1);
            k = ok ? ((uint64_t)s << g.L) | d : (1ull << (2 * g.L));
        }
        key[j] = (k << kTilePosBits) | (i & ((1u << kTilePosBits) - 1));
    }
    tile_sort(key, n, passes, ~0ull, lds);
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = (uint64_t)j * kOsThreads + threadIdx.x;
        if (i < n) {
            keys[i] = key[j] >> kTilePosBits;
            pos[i] = (uint32_t)(key[j] & ((1u << kTilePosBits) - 1));
        }
    }
}

// Scan source over the sorted entries: an entry counts when it is valid and
// the last of its key (the sort is stable: last in list order), as a delete
// (low half) or an insert (high half).
struct SplitIn {
    const uint64_t* keys;
    const uint32_t* pos;
    const uint8_t* op;
    uint64_t n;
    uint32_t L;
    struct Rec {
        uint64_t k;
        uint32_t p;
        uint8_t o;
        bool last;  // no later entry has the same key
    };
    __device__ uint64_t limit(uint64_t m) const { return m; }
    __device__ Rec load(uint64_t i, bool) const {
        Rec r;
        r.k = keys[i];
        r.last = i + 1 >= n || keys[i + 1] != r.k;
        r.p = pos[i];
        r.o = 0;
        return r;
    }
    __device__ void deref(Rec& r) const { r.o = op[r.p]; }
    // 0 = not kept, 1 = kept delete, 2 = kept insert
    __device__ int kind(const Rec& r) const {
        if ((r.k >> (2 * L)) != 0 || !r.last) return 0;
        return r.o == 1 ? 1 : 2;
    }
    __device__ unsigned long long value(uint64_t, const Rec& r) const {
        const int k = kind(r);
        return k == 1 ? 1ull : k == 2 ? (1ull << 32) : 0ull;
    }
};

// The scan total holds both counts; finish() splits it for the two sorted
// batches, which read one each (cnt[1] deletes, cnt[2] inserts).
struct SplitOut {
    SplitIn in;
    uint64_t* del_keys;
    uint64_t* ins_keys;
    unsigned long long* cnt;  // [0] the scan total
    __device__ void operator()(uint64_t, const SplitIn::Rec& r, uint64_t,
                               unsigned long long pre) const {
        const int k = in.kind(r);
        if (k == 1) del_keys[(uint32_t)pre] = r.k;
        else if (k == 2) ins_keys[(uint32_t)(pre >> 32)] = r.k;
    }
    __device__ void finish() const {
        if (threadIdx.x == 0) {
            cnt[1] = cnt[0] & 0xffffffffull;
            cnt[2] = cnt[0] >> 32;
        }
    }
};

// ---- per-request statistics
// Request r is entries [end[r-1], end[r]).  As if each request were applied
// alone, in order: an entry is rejected when an endpoint is invalid or the op
// is neither 0 nor 1; a duplicate when the pair's previous entry is in the
// same request with the same op; applied when it changes the graph (an
// insert of a pair absent just before it, a delete of a pair present).
// Whether a pair is present just before an entry follows from its previous
// entry in the list (an insert leaves it present, a delete absent), and for
// its first entry from the graph before the list, which the delete or insert
// batch that applies the pair's last entry reports per key.
enum : uint8_t { kFNone = 0, kFApplied = 1, kFDup = 2, kFRej = 3, kFNeedIns = 4, kFNeedDel = 5 };
constexpr uint32_t kRefIns = 0x80000000u;

__device__ __forceinline__ uint32_t request_of(const uint64_t* end, uint32_t n_req, uint64_t p) {
    uint32_t lo = 0, hi = n_req;  // first r with end[r] > p
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (end[mid] > p) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// one thread per sorted entry: its flag, and for a pair's first entry the
// index of the pair in the kept delete or insert keys
// (also zeroes the per-request statistics, one thread per request, for the
// counts added later)
__global__ __launch_bounds__(kThreads) void k_mixed_flags(
    GraphView g, const uint64_t* sk, const uint32_t* sp, const uint8_t* op, uint64_t n,
    const uint64_t* end, uint32_t n_req, const uint64_t* del_keys, const uint64_t* ins_keys,
    const unsigned long long* cnt, uint8_t* flag, uint32_t* fref, gv_batch_stats* stats) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n_req) stats[i] = gv_batch_stats{0ull, 0ull, 0ull};
    if (i >= n) return;
    const uint64_t k = sk[i];
    const uint32_t p = sp[i];
    const uint8_t o = op[p];
    uint8_t f = kFNone;
    uint32_t ref = 0;
    if ((k >> (2 * g.L)) != 0) {
        f = kFRej;
    } else if (i > 0 && sk[i - 1] == k) {
        const uint32_t pp = sp[i - 1];
        const uint8_t po = op[pp];
        if (po == o && request_of(end, n_req, pp) == request_of(end, n_req, p)) {
            f = kFDup;
        } else {
            const bool present = po == 0;
            f = (o == 0) != present ? kFApplied : kFNone;
        }
    } else {
        // the pair's last entry decides which kept list holds it
        const uint32_t hi = lower_bound(sk, (uint32_t)i + 1, (uint32_t)n, k + 1);
        const bool del = op[sp[hi - 1]] == 1;
        const uint64_t* list = del ? del_keys : ins_keys;
        const uint32_t m = (uint32_t)(del ? cnt[1] : cnt[2]);
        ref = lower_bound(list, 0u, m, k) | (del ? 0u : kRefIns);
        f = o == 0 ? kFNeedIns : kFNeedDel;
    }
    flag[p] = f;
    fref[p] = ref;
}

// Per-request counts, added into zeroed stats: each thread takes
// kStatItems consecutive entries.  A wave whose entries all belong to one
// request adds its sums from one lane; otherwise each lane adds its own sums
// per request it covers.  Entries at or past the ends of every request are
// not counted (so ends that are not ascending give wrong counts, never reads
// out of bounds).
constexpr uint32_t kStatItems = 8;
__global__ __launch_bounds__(kThreads) void k_request_stats(const uint64_t* end, uint64_t n_req,
                                                            uint64_t n,
                                                            const uint8_t* flag,
                                                            const uint32_t* fref,
                                                            const uint8_t* del_found,
                                                            const uint8_t* ins_had,
                                                            gv_batch_stats* stats) {
    const uint64_t p0 = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) * kStatItems;
    const bool live = p0 < n;
    uint32_t r = live ? request_of(end, (uint32_t)n_req, p0) : (uint32_t)n_req;
    unsigned long long a = 0, d = 0, j = 0;
    bool moved = false;  // the lane's entries span more than one request
    auto add = [&](uint32_t q) {
        if (q >= n_req) return;
        if (a) atomicAdd((unsigned long long*)&stats[q].applied, a);
        if (j) atomicAdd((unsigned long long*)&stats[q].rejected, j);
        if (d) atomicAdd((unsigned long long*)&stats[q].batch_duplicates, d);
    };
    for (uint32_t k = 0; k < kStatItems; ++k) {
        const uint64_t p = p0 + k;
        if (p >= n) break;
        if (r < n_req && end[r] <= p) {
            // the next request whose range holds p
            add(r);
            a = d = j = 0;
            moved = true;
            r = request_of(end, (uint32_t)n_req, p);
        }
        const uint8_t f = flag[p];
        if (f == kFApplied) {
            ++a;
        } else if (f == kFDup) {
            ++d;
        } else if (f == kFRej) {
            ++j;
        } else if (f >= kFNeedIns) {
            const uint32_t ref = fref[p];
            const bool present = (ref & kRefIns) ? ins_had[ref & ~kRefIns] != 0
                                                 : del_found[ref] != 0;
            a += (f == kFNeedIns) != present;
        }
    }
    // lane 0 is live whenever any lane of its wave is (p0 grows with the lane)
    const uint32_t r0 = (uint32_t)__shfl((int)r, 0, 64);
    if (ballot(live && (moved || r != r0)) == 0) {
        a = wave_sum(a);
        d = wave_sum(d);
        j = wave_sum(j);
        if (lane_id() == 0 && live) add(r);
    } else if (live) {
        add(r);
    }
}

__global__ __launch_bounds__(kThreads) void k_stats_zero(gv_batch_stats* stats, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) stats[i] = gv_batch_stats{0ull, 0ull, 0ull};
}

}  // namespace

// bytes of g->scratch and of g->vscr[0] a mixed list of n entries needs
void mixed_bytes(const gv_graph* g, uint64_t n, size_t out[2]) {
    const int bits = 2 * (int)g->v.L + 1;
    Carver m(nullptr);
    m.take<uint64_t>(n);
    m.take<uint64_t>(n);
    m.take<uint32_t>(n);
    m.take<uint32_t>(n);
    m.take<unsigned long long>(scan2_parts(n));
    m.take<uint32_t>(os_words(n, bits));
    out[0] = std::max(m.used, edge_batch_bytes(g, kInsert, n));
    out[1] = 2 * n * sizeof(uint64_t) + 4 * sizeof(unsigned long long);
}

void mixed_edges(gv_graph* g, const uint8_t* op, const uint32_t* src, const uint32_t* dst,
                 uint64_t n, const uint64_t* req_end, uint64_t n_req, gv_batch_stats* stats) {
    Ctx& c = g->ctx;
    if (n == 0) {
        if (stats && n_req)
            c.launch("mixed_stats", k_stats_zero, div_up(n_req, kThreads), kThreads, stats, n_req);
        return;
    }
    if (n >= 0x3fffffffull) fail(GV_EINVAL, "batch too large");
    const GraphView& v = g->v;
    const int bits = 2 * (int)v.L + 1;
    // the key lists, counts and statistics buffers outlive the two inner
    // batches, which carve g->scratch
    uint64_t *del_keys, *ins_keys;
    const uint64_t* end = req_end;
    unsigned long long* cnt;  // total, deletes, inserts
    uint32_t* fref = nullptr;
    uint8_t *flag = nullptr, *del_found = nullptr, *ins_had = nullptr;
    auto carve_keep = [&](Carver& cv) {
        del_keys = cv.take<uint64_t>(n);
        ins_keys = cv.take<uint64_t>(n);
        cnt = cv.take<unsigned long long>(4);
        if (stats) {
            fref = cv.take<uint32_t>(n);
            flag = cv.take<uint8_t>(n);
            del_found = cv.take<uint8_t>(n);
            ins_had = cv.take<uint8_t>(n);
        }
    };
    {
        Carver m(nullptr);
        carve_keep(m);
        g->vscr[0].ensure(m.used, c.stream);
        Carver cv(g->vscr[0].ptr);
        carve_keep(cv);
    }
    uint64_t *k0, *k1;
    uint32_t *p0, *p1, *state;
    unsigned long long* part;
    auto carve = [&](Carver& cv) {
        k0 = cv.take<uint64_t>(n);
        k1 = cv.take<uint64_t>(n);
        p0 = cv.take<uint32_t>(n);
        p1 = cv.take<uint32_t>(n);
        part = cv.take<unsigned long long>(scan2_parts(n));
        state = cv.take<uint32_t>(os_words(n, bits));
    };
    {
        Carver m(nullptr);
        carve(m);
        g->scratch.ensure(m.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve(cv);
    }
    bool flip = false;
    if (n <= kOsTile && bits + kTilePosBits <= 64) {
        c.launch("mixed_pack", k_mixed_sort_tile, 1, kOsThreads, v, op, src, dst, n,
                 os_passes(bits + kTilePosBits), k0, p0);
    } else {
        zero_words(c, state, os_zero_words(n, bits));
        c.launch("mixed_pack", k_mixed_pack, div_up(n, kThreads), kThreads, v, op, src, dst, n,
                 k0, p0);
        flip = onesweep<uint64_t, true>(c, k0, k1, p0, p1, nullptr, n, bits, state,
                                        &v.ctr->err_wait, g->spin_limit);
    }
    const uint64_t* sk = flip ? k1 : k0;
    const uint32_t* sp = flip ? p1 : p0;
    const SplitIn in{sk, sp, op, n, v.L};
    scan2(c, "mixed_split", in, SplitOut{in, del_keys, ins_keys, cnt}, n, part, &cnt[0]);
    if (stats)  // before the batches reuse the sorted entries' scratch
        c.launch("mixed_stats", k_mixed_flags, div_up(std::max<uint64_t>(n, n_req), kThreads),
                 kThreads, v, sk, sp, op, n, end, (uint32_t)n_req, (const uint64_t*)del_keys,
                 (const uint64_t*)ins_keys, (const unsigned long long*)cnt, flag, fref, stats);
    edge_batch_sorted(g, kDelete, del_keys, &cnt[1], n, true, del_found);
    edge_batch_sorted(g, kInsert, ins_keys, &cnt[2], n, true, ins_had);
    if (stats) {
        c.launch("mixed_stats", k_request_stats, div_up(n, (uint64_t)kThreads * kStatItems),
                 kThreads, end, n_req, n, (const uint8_t*)flag, (const uint32_t*)fref,
                 (const uint8_t*)del_found, (const uint8_t*)ins_had, stats);
    }
}

}  // namespace gv
