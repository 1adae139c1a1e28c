// gv_served.hip -- mixed edge updates with last-writer reduction: the tick of
// the served form, and the unit the batched form coalesces runs of edge
// batches into.
//
// A list of (op, src, dst) entries, op 0 = insert and 1 = delete, has the
// effect of applying the entries one at a time in list order with set
// semantics (Sec. 4.3's batch model; the order inside a batch is ours): a
// pair's final membership is decided by its last entry, and entries with an
// inactive or out-of-range endpoint change nothing.  On the device: pack the
// entries as keys (src << L) | dst with their list position (an entry with an
// endpoint out of range or an op above 1 gets bit 2L, after every pair key),
// sort them stably, and keep the last entry of every key whose endpoints are
// both active: a scan writes the kept deletes and the kept inserts, compacted
// and still sorted, to two key lists (a list of at most one tile is packed and
// sorted by one workgroup).  The two lists are then applied as a delete batch
// and an insert batch that start from their sorted keys (no second sort); no
// key is in both, so their order does not matter.
//
// The packing and the sort read the entries only, not the graph (activity is
// checked by the scan, on the graph's stream), so the batched form can run
// them on the sort overlap's side stream while the graph's stream applies the
// list before.
#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

namespace {

// an entry's sort key: the pair, or bit 2L when an endpoint is past the
// vertex table (2^L slots) or the op is neither insert nor delete
__device__ __forceinline__ uint64_t mixed_key(uint32_t s, uint32_t d, uint8_t o, uint32_t L) {
    const bool ok = ((uint64_t)s >> L == 0) & ((uint64_t)d >> L == 0) & (o <= 1);
    return ok ? ((uint64_t)s << L) | d : (1ull << (2 * L));
}

__global__ __launch_bounds__(kThreads) void k_mixed_pack(uint32_t L, const uint8_t* op,
                                                         const uint32_t* src,
                                                         const uint32_t* dst, uint64_t n,
                                                         uint64_t* keys, uint32_t* pos) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    keys[i] = mixed_key(src[i], dst[i], op[i], L);
    pos[i] = (uint32_t)i;
}

// Lists of at most one tile: one workgroup packs each entry as its key with
// its list position in the low 12 bits ((pair << 12) | position, an invalid
// entry with bit 2L set above the pair) and sorts the tile in LDS, which is
// the stable order by pair; the pair keys and positions go out separately,
// as the general path leaves them.
constexpr int kTilePosBits = 12;  // kOsTile = 4096 positions
__global__ __launch_bounds__(kOsThreads) void k_mixed_sort_tile(uint32_t L, const uint8_t* op,
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
        if (i < n) k = mixed_key(src[i], dst[i], op[i], L);
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

// both endpoints of a pair key active (the key is below bit 2L)
__device__ __forceinline__ bool pair_active(const uint32_t* active, uint64_t k, uint32_t L) {
    const uint32_t s = (uint32_t)(k >> L), d = (uint32_t)(k & ((1ull << L) - 1));
    return (((active[s >> 5] >> (s & 31)) & (active[d >> 5] >> (d & 31))) & 1u) != 0u;
}

// Scan source over the sorted entries: an entry counts when its key is a pair
// of active vertices and it is the last of its key (the sort is stable: last
// in list order), as a delete (low half) or an insert (high half).
struct SplitIn {
    const uint64_t* keys;
    const uint32_t* pos;
    const uint8_t* op;
    const uint32_t* active;
    uint64_t n;
    uint32_t L;
    struct Rec {
        uint64_t k;
        uint32_t p;
        uint8_t o;
        bool last;  // no later entry has the same key
        bool act;   // a pair key with both endpoints active
    };
    __device__ uint64_t limit(uint64_t m) const { return m; }
    __device__ Rec load(uint64_t i, bool) const {
        Rec r;
        r.k = keys[i];
        r.last = i + 1 >= n || keys[i + 1] != r.k;
        r.p = pos[i];
        r.o = 0;
        r.act = false;
        return r;
    }
    __device__ void deref(Rec& r) const {
        r.o = op[r.p];
        r.act = (r.k >> (2 * L)) == 0 && pair_active(active, r.k, L);
    }
    // 0 = not kept, 1 = kept delete, 2 = kept insert
    __device__ int kind(const Rec& r) const {
        if (!r.act || !r.last) return 0;
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
    if ((k >> (2 * g.L)) != 0 || !pair_active(g.active, k, g.L)) {
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

// the sort buffers of a mixed list
struct MixSort {
    uint64_t *k0, *k1;
    uint32_t *p0, *p1, *state;
    void carve(Carver& cv, uint64_t n, int bits) {
        k0 = cv.take<uint64_t>(n);
        k1 = cv.take<uint64_t>(n);
        p0 = cv.take<uint32_t>(n);
        p1 = cv.take<uint32_t>(n);
        state = cv.take<uint32_t>(os_words(n, bits));
    }
};

// the buffers that outlive the sort: the kept key lists, their counts, the
// split's scan partials and the statistics' per-entry arrays (in g->vscr[0];
// the two inner batches carve g->scratch)
struct MixKeep {
    uint64_t *del_keys, *ins_keys;
    unsigned long long* cnt;  // total, deletes, inserts
    unsigned long long* part;
    uint32_t* fref = nullptr;
    uint8_t *flag = nullptr, *del_found = nullptr, *ins_had = nullptr;
    void carve(Carver& cv, uint64_t n, bool stats) {
        del_keys = cv.take<uint64_t>(n);
        ins_keys = cv.take<uint64_t>(n);
        cnt = cv.take<unsigned long long>(4);
        part = cv.take<unsigned long long>(scan2_parts(n));
        if (stats) {
            fref = cv.take<uint32_t>(n);
            flag = cv.take<uint8_t>(n);
            del_found = cv.take<uint8_t>(n);
            ins_had = cv.take<uint8_t>(n);
        }
    }
};

// packs entries [0, n) and sorts them stably by key on c; true when the
// sorted keys and positions are in k1 / p1
bool mixed_sort(const gv_graph* g, Ctx& c, const uint8_t* op, const uint32_t* src,
                const uint32_t* dst, uint64_t n, const MixSort& b, bool concurrent) {
    const uint32_t L = g->v.L;
    const int bits = 2 * (int)L + 1;
    if (n <= kOsTile && bits + kTilePosBits <= 64) {
        c.launch("mixed_pack", k_mixed_sort_tile, 1, kOsThreads, L, op, src, dst, n,
                 os_passes(bits + kTilePosBits), b.k0, b.p0);
        return false;
    }
    zero_words(c, b.state, os_zero_words(n, bits));
    c.launch("mixed_pack", k_mixed_pack, div_up(n, kThreads), kThreads, L, op, src, dst, n, b.k0,
             b.p0);
    return onesweep<uint64_t, true>(c, b.k0, b.k1, b.p0, b.p1, nullptr, n, bits, b.state,
                                    &g->v.ctr->err_wait, g->spin_limit, concurrent);
}

// the list's entries sorted (sk, sp): the kept key lists, then (when
// `released` is given) released() once nothing reads the sorted entries or
// the ops any more, then the two batches and the statistics
void mixed_apply(gv_graph* g, const uint8_t* op, const uint64_t* sk, const uint32_t* sp,
                 uint64_t n, const uint64_t* end, uint64_t n_req, gv_batch_stats* stats,
                 const std::function<void()>* released) {
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    MixKeep k;
    {
        Carver m(nullptr);
        k.carve(m, n, stats != nullptr);
        g->vscr[0].ensure(m.used, c.stream);
        Carver cv(g->vscr[0].ptr);
        k.carve(cv, n, stats != nullptr);
    }
    const SplitIn in{sk, sp, op, v.active, n, v.L};
    scan2(c, "mixed_split", in, SplitOut{in, k.del_keys, k.ins_keys, k.cnt}, n, k.part, &k.cnt[0]);
    if (stats)
        c.launch("mixed_stats", k_mixed_flags, div_up(std::max<uint64_t>(n, n_req), kThreads),
                 kThreads, v, sk, sp, op, n, end, (uint32_t)n_req, (const uint64_t*)k.del_keys,
                 (const uint64_t*)k.ins_keys, (const unsigned long long*)k.cnt, k.flag, k.fref,
                 stats);
    if (released) (*released)();
    edge_batch_sorted(g, kDelete, k.del_keys, &k.cnt[1], n, true, k.del_found);
    edge_batch_sorted(g, kInsert, k.ins_keys, &k.cnt[2], n, true, k.ins_had);
    if (stats) {
        c.launch("mixed_stats", k_request_stats, div_up(n, (uint64_t)kThreads * kStatItems),
                 kThreads, end, n_req, n, (const uint8_t*)k.flag, (const uint32_t*)k.fref,
                 (const uint8_t*)k.del_found, (const uint8_t*)k.ins_had, stats);
    }
}

// the side stream's buffer of a list: its entries, then its sort buffers
struct MixSide {
    uint32_t *src, *dst;
    uint8_t* op;
    MixSort s;
    void carve(Carver& cv, uint64_t n, int bits) {
        src = cv.take<uint32_t>(n);
        dst = cv.take<uint32_t>(n);
        op = cv.take<uint8_t>(n);
        s.carve(cv, n, bits);
    }
};

}  // namespace

// bytes of g->scratch and of g->vscr[0] a mixed list of n entries needs
// (without statistics)
void mixed_bytes(const gv_graph* g, uint64_t n, size_t out[2]) {
    const int bits = 2 * (int)g->v.L + 1;
    Carver m(nullptr);
    MixSort s;
    s.carve(m, n, bits);
    out[0] = std::max(m.used, edge_batch_bytes(g, kInsert, n));
    Carver k(nullptr);
    MixKeep keep;
    keep.carve(k, n, false);
    out[1] = k.used;
}

size_t mixed_side_bytes(const gv_graph* g, uint64_t n) {
    Carver m(nullptr);
    MixSide b;
    b.carve(m, n, 2 * (int)g->v.L + 1);
    return m.used;
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
    MixSort b;
    {
        const int bits = 2 * (int)g->v.L + 1;
        Carver m(nullptr);
        b.carve(m, n, bits);
        g->scratch.ensure(m.used, c.stream);
        Carver cv(g->scratch.ptr);
        b.carve(cv, n, bits);
    }
    const bool flip = mixed_sort(g, c, op, src, dst, n, b, false);
    // (the statistics' flags are taken before the batches reuse g->scratch)
    mixed_apply(g, op, flip ? b.k1 : b.k0, flip ? b.p1 : b.p0, n, req_end, n_req, stats,
                nullptr);
}

void mixed_edges_side(gv_graph* g, uint64_t n, bool fence,
                      const std::function<void(Ctx&, uint8_t*, uint32_t*, uint32_t*)>& gather) {
    Ctx& c = g->ctx;
    if (n == 0) return;
    if (n >= 0x3fffffffull) fail(GV_EINVAL, "batch too large");
    gv_graph::Overlap& o = g->ov;
    overlap_open(g);
    overlap_capture(g);
    const int ob = (int)(o.mcount & 1);
    const int bits = 2 * (int)g->v.L + 1;
    const size_t need = mixed_side_bytes(g, n);
    if (o.mix[ob].cap < need) {
        // (the side stream wrote the buffer last, the graph's stream read it)
        hip_check(hipStreamSynchronize(o.stream), "hipStreamSynchronize");
        o.mix[ob].ensure(need, c.stream);
    }
    MixSide b;
    Carver cv(o.mix[ob].ptr);
    b.carve(cv, n, bits);
    Ctx& sc = o.ctx;
    sc.prof = c.prof;
    sc.only = c.only;
    // The side stream waits for the graph's stream once per call (the
    // caller's entries are ready when the call is made) and to join a
    // capture; otherwise only for the list that used the buffer before.
    if (fence || !o.joined) {
        overlap_fence(g);
    } else if (o.mused[ob]) {
        hip_check(hipStreamWaitEvent(o.stream, o.mdone[ob], 0), "hipStreamWaitEvent");
    }
    gather(sc, b.op, b.src, b.dst);
    const bool flip = mixed_sort(g, sc, b.op, b.src, b.dst, n, b.s, true);
    sc.close_run();
    hip_check(hipEventRecord(o.msorted[ob], o.stream), "hipEventRecord");
    hip_check(hipStreamWaitEvent(c.stream, o.msorted[ob], 0), "hipStreamWaitEvent");
    const std::function<void()> released = [&] {
        hip_check(hipEventRecord(o.mdone[ob], c.stream), "hipEventRecord");
        o.mused[ob] = true;
    };
    mixed_apply(g, b.op, flip ? b.s.k1 : b.s.k0, flip ? b.s.p1 : b.s.p0, n, nullptr, 0, nullptr,
                &released);
    ++o.mcount;
}

}  // namespace gv
