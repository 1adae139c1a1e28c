// gv_prim.h -- device-wide exclusive scan and stable LSD radix sort for
// wave64 (gfx950), written for this library.
//
// Scan: reduce-then-scan over tiles of kScanTile elements; inputs and outputs
// are functors so that producers and consumers fuse into the scan kernels.
//
// Sort: 8-bit digits.  Per pass, a histogram kernel counts the digits of each
// tile, the digit-major count matrix is scanned, and a scatter kernel ranks
// every key inside its tile.  Ranking is contention-free: the 64 lanes of a
// wave find the lanes holding the same digit with eight ballots (one per
// digit bit); the lowest such lane publishes the count, and waves are ordered
// through a small LDS table.  Keys keep their input order within a digit, so
// the sort is stable.
#pragma once

#include <algorithm>
#include <type_traits>
#include <utility>

#include "gv_device.h"
#include "gv_host.h"

namespace gv {

constexpr int kScanItems = 8;
constexpr uint64_t kScanTile = (uint64_t)kThreads * kScanItems;
constexpr int kSortItems = 16;
constexpr uint64_t kSortTile = (uint64_t)kThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

template <typename T>
struct ArrIn {
    const T* a;
    __device__ T operator()(uint64_t i) const { return a[i]; }
};

template <typename T>
struct ArrOut {
    T* a;
    __device__ void operator()(uint64_t i, T v) const { a[i] = v; }
};

// ------------------------------------------------------------------ scan
template <typename T, typename In>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(In in, uint64_t n, T* partial) {
    __shared__ T lds[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    T s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
        if (i < n) s += in(i);
    }
    T tot = block_sum(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the tile sums in place; total -> *total
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_partials(T* partial, uint64_t nt, T* total) {
    __shared__ T lds[kWaves];
    T carry = 0;
    for (uint64_t b = 0; b < nt; b += kThreads) {
        uint64_t i = b + threadIdx.x;
        T x = i < nt ? partial[i] : T(0);
        T tot;
        T ex = block_excl_scan(x, lds, tot);
        if (i < nt) partial[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename T, typename In, typename Out>
__global__ __launch_bounds__(kThreads) void k_scan_down(In in, Out out, uint64_t n, const T* partial) {
    __shared__ T lds[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    T carry = partial[blockIdx.x];
#pragma unroll 1
    for (int j = 0; j < kScanItems; ++j) {
        uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
        T x = i < n ? in(i) : T(0);
        T tot;
        T ex = block_excl_scan(x, lds, tot);
        if (i < n) out(i, carry + ex);
        carry += tot;
    }
}

inline uint64_t scan_partials_needed(uint64_t n) { return div_up(n, kScanTile) + 1; }

template <typename T>
__global__ void k_zero_total(T* p) {
    *p = T(0);
}

// Exclusive scan of in(0..n-1) into out(i, prefix); the sum goes to the device
// location `total` when non-null.  `partial` needs scan_partials_needed(n).
template <typename T, typename In, typename Out>
void scan_excl(Ctx& c, In in, Out out, uint64_t n, T* partial, T* total) {
    if (n == 0) {
        // a kernel, not a memset, so that the call can be recorded in a graph
        if (total) c.launch("scan_zero", k_zero_total<T>, 1, 1, total);
        return;
    }
    uint64_t nt = div_up(n, kScanTile);
    c.launch("scan_reduce", k_scan_reduce<T, In>, nt, kThreads, in, n, partial);
    c.launch("scan_partials", k_scan_partials<T>, 1, kThreads, partial, nt, total);
    c.launch("scan_down", k_scan_down<T, In, Out>, nt, kThreads, in, out, n, (const T*)partial);
}

// ------------------------------------------------------------------ sort
// lanes of this wave that are active and hold the same digit as this lane
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool act) {
    uint64_t m = ballot(act);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        bool bit = (d >> b) & 1u;
        uint64_t bal = ballot(bit);
        m &= bit ? bal : ~bal;
    }
    return m;
}

template <typename K>
__global__ __launch_bounds__(kThreads) void k_rs_hist(const K* keys, uint64_t n, int shift,
                                                       uint32_t* counts, uint64_t ntiles) {
    __shared__ uint32_t hist[kRadix];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int j = 0; j < kSortItems; ++j) {
        uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
        bool act = i < n;
        uint32_t d = act ? (uint32_t)(keys[i] >> shift) & (kRadix - 1) : 0u;
        uint64_t peers = digit_peers(d, act);
        if (act && rank_below(peers) == 0) atomicAdd(&hist[d], popc64(peers));
    }
    __syncthreads();
    counts[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

template <typename K, bool HasVal>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const K* kin, K* kout, const uint32_t* vin,
                                                          uint32_t* vout, uint64_t n, int shift,
                                                          const uint32_t* offsets, uint64_t ntiles) {
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t wcnt[kWaves][kRadix];
    const int w = threadIdx.x >> 6;
    run[threadIdx.x] = offsets[(uint64_t)threadIdx.x * ntiles + blockIdx.x];
#pragma unroll
    for (int i = 0; i < kWaves; ++i) wcnt[i][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
#pragma unroll 1
    for (int j = 0; j < kSortItems; ++j) {
        uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
        bool act = i < n;
        K key = act ? kin[i] : K(0);
        uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
        uint64_t peers = digit_peers(d, act);
        uint32_t r = rank_below(peers);
        if (act && r == 0) wcnt[w][d] = popc64(peers);
        __syncthreads();
        if (act) {
            uint32_t pos = run[d] + r;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            kout[pos] = key;
            if (HasVal) vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            add += wcnt[q][threadIdx.x];
            wcnt[q][threadIdx.x] = 0;
        }
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

struct SortScratch {
    uint32_t* counts;   // kRadix * ntiles
    uint32_t* partial;  // scan partials of counts
};

inline uint64_t sort_tiles(uint64_t n) { return div_up(n, kSortTile); }

template <typename K>
inline void carve_sort(Carver& cv, SortScratch& s, uint64_t n) {
    uint64_t nc = (uint64_t)kRadix * sort_tiles(n);
    s.counts = cv.take<uint32_t>(nc);
    s.partial = cv.take<uint32_t>(scan_partials_needed(nc));
}

// Sorts keys ascending by bits [0, bits), stably, ping-ponging between k0 and
// k1 (and v0/v1 when HasVal).  Returns true if the result ends in k1/v1.
template <typename K, bool HasVal>
bool radix_sort(Ctx& c, K* k0, K* k1, uint32_t* v0, uint32_t* v1, uint64_t n, int bits,
                const SortScratch& s) {
    if (n <= 1 || bits <= 0) return false;
    if (n > 0xffffffffull) fail(GV_EINVAL, "sort too large");
    const uint64_t nt = sort_tiles(n);
    const uint64_t nc = (uint64_t)kRadix * nt;
    bool flip = false;
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        K* kin = flip ? k1 : k0;
        K* kout = flip ? k0 : k1;
        uint32_t* vin = flip ? v1 : v0;
        uint32_t* vout = flip ? v0 : v1;
        c.launch("sort_hist", k_rs_hist<K>, nt, kThreads, (const K*)kin, n, shift, s.counts, nt);
        scan_excl<uint32_t>(c, ArrIn<uint32_t>{s.counts}, ArrOut<uint32_t>{s.counts}, nc, s.partial,
                            (uint32_t*)nullptr);
        c.launch("sort_scatter", k_rs_scatter<K, HasVal>, nt, kThreads, (const K*)kin, kout,
                 (const uint32_t*)vin, vout, n, shift, (const uint32_t*)s.counts, nt);
        flip = !flip;
    }
    return flip;
}

}  // namespace gv

// ======================================================================
// Primitives with decoupled look-back between workgroups.  Look-back status
// words live in a caller-provided region that must be zero before the launch
// (the batch pipeline clears it in its first kernel).  Every wait is bounded:
// a wait that runs out sets an error flag instead of hanging, and the callers
// treat the result as failed.
// ======================================================================
namespace gv {

constexpr uint32_t kSpinLimit = kSpinLimitDefault;

constexpr int kScan1Items = 8;

// Status words carry their own value (flag and count in one word), so no other
// data is ordered by them: relaxed loads and stores at device scope suffice.
__device__ __forceinline__ uint32_t ld_status32(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status32(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- scan2
// Two-kernel exclusive scan without inter-tile waits: the first kernel
// reduces each tile, the second recomputes its tile prefix by reducing the
// partials of all earlier tiles (up to kScan2MaxTiles, read from L2; with
// more tiles a one-workgroup kernel between the two scans the partials) and
// scans its tile.  Inputs are evaluated twice, outputs written once.  On a
// context with a scan state (the graph's stream), inputs of 2 to
// kChainTiles tiles take a one-kernel form instead (k_scan2_chain below).
//
// The source is a gather: it splits each element into its memory reads and
// the arithmetic on them, so that a thread issues the reads of all of its
// elements before it waits on any of them.
//   uint64_t limit(uint64_t n)          live elements (<= n, may be read from
//                                       device memory); the rest count 0
//   Rec load(uint64_t i, bool ok)       first-level reads of element i (always
//                                       i < n); every address must be valid
//                                       also when !ok, and no read may sit
//                                       behind a branch
//   void deref(Rec&)                    reads at addresses that load() read
//                                       (same rules)
//   ull value(uint64_t i, const Rec&)   the element's value (called when ok)
// The sink takes (i, rec, lim, exclusive prefix) for every i < n; the
// element is live when i < lim.  A sink may also define
//   ull tally(uint64_t i, const Rec&)   a 64-bit value per live element
//   void commit(ull sum)                called once per workgroup with the sum
// and
//   void finish()                       run by the first wave of the last
//                                       workgroup once the total is written
// and a source may define
//   void begin()                        run by every thread of the reduce
//                                       kernel's first workgroup (when the
//                                       scan has more than one tile), before
//                                       the apply kernel starts
// Elements per thread: In::kItems when the source defines it (sources with
// large records take fewer, to keep registers low), else kScan1Items.
template <typename In, typename = void>
struct scan2_items {
    static constexpr int value = kScan1Items;
};
template <typename In>
struct scan2_items<In, std::void_t<decltype(In::kItems)>> {
    static constexpr int value = In::kItems;
};
template <typename Out, typename = void>
struct scan2_has_tally : std::false_type {};
template <typename Out>
struct scan2_has_tally<Out, std::void_t<decltype(std::declval<const Out&>().commit(0ull))>>
    : std::true_type {};
template <typename In, typename = void>
struct scan2_has_begin : std::false_type {};
template <typename In>
struct scan2_has_begin<In, std::void_t<decltype(std::declval<const In&>().begin())>>
    : std::true_type {};
template <typename Out, typename = void>
struct scan2_has_finish : std::false_type {};
template <typename Out>
struct scan2_has_finish<Out, std::void_t<decltype(std::declval<const Out&>().finish())>>
    : std::true_type {};
constexpr int kScan2MinItems = 2;  // the fewest any source takes (scan2 checks it)

template <typename In>
__global__ __launch_bounds__(kThreads) void k_scan2_reduce(In in, uint64_t n,
                                                           unsigned long long* part) {
    constexpr int kI = scan2_items<In>::value;
    __shared__ unsigned long long s_w[kWaves];
    if constexpr (scan2_has_begin<In>::value) {
        if (blockIdx.x == 0) in.begin();
    }
    const uint64_t lim = in.limit(n);
    const uint64_t base = (uint64_t)blockIdx.x * kThreads * kI + threadIdx.x;
    typename In::Rec r[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        r[j] = in.load(i < n ? i : n - 1, i < lim);
    }
#pragma unroll
    for (int j = 0; j < kI; ++j) in.deref(r[j]);
    unsigned long long s = 0;
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        s += i < lim ? in.value(i, r[j]) : 0ull;
    }
    s = block_sum(s, s_w);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Exclusive scan of the nt tile sums in place (one workgroup), for inputs
// with more tiles than the apply kernel adds up itself.
static __global__ __launch_bounds__(kThreads) void k_scan2_partials(unsigned long long* part,
                                                                    uint64_t nt) {
    __shared__ unsigned long long lds[kWaves];
    unsigned long long carry = 0;
    for (uint64_t b = 0; b < nt; b += kThreads) {
        const uint64_t i = b + threadIdx.x;
        const unsigned long long x = i < nt ? part[i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan(x, lds, tot);
        if (i < nt) part[i] = carry + ex;
        carry += tot;
    }
}

// scanned: part already holds exclusive tile prefixes
template <typename In, typename Out>
__global__ __launch_bounds__(kThreads) void k_scan2_apply(In in, Out out, uint64_t n,
                                                          const unsigned long long* part,
                                                          int scanned,
                                                          unsigned long long* total) {
    constexpr int kI = scan2_items<In>::value;
    __shared__ unsigned long long s_w[kI][kWaves];
    __shared__ unsigned long long s_p[kWaves];
    const uint64_t lim = in.limit(n);
    const uint64_t base = (uint64_t)blockIdx.x * kThreads * kI + threadIdx.x;
    typename In::Rec r[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        r[j] = in.load(i < n ? i : n - 1, i < lim);
    }
#pragma unroll
    for (int j = 0; j < kI; ++j) in.deref(r[j]);
    unsigned long long p = 0;
    if (scanned) {
        p = threadIdx.x == 0 ? part[blockIdx.x] : 0ull;
    } else {
        for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kThreads) p += part[t];
    }
    // one wave scan per row of the tile, then a single exchange of the
    // per-wave row totals
    unsigned long long x[kI], inc[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        x[j] = i < lim ? in.value(i, r[j]) : 0ull;
        inc[j] = wave_incl_scan(x[j]);
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) {
#pragma unroll
        for (int j = 0; j < kI; ++j) s_w[j][w] = inc[j];
    }
    unsigned long long run = block_sum(p, s_p);  // its barriers publish s_w
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        unsigned long long before = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            const unsigned long long v = s_w[j][q];
            before += q < w ? v : 0ull;
            tot += v;
        }
        if (i < n) out(i, r[j], lim, run + before + inc[j] - x[j]);
        run += tot;
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) *total = run;
    if constexpr (scan2_has_tally<Out>::value) {
        // a sink may add up a 64-bit tally of the live elements: one sum per
        // workgroup goes to out.commit()
        unsigned long long t = 0;
#pragma unroll
        for (int j = 0; j < kI; ++j) {
            const uint64_t i = base + (uint64_t)j * kThreads;
            t += i < lim ? out.tally(i, r[j]) : 0ull;
        }
        t = block_sum(t, s_p);
        if (threadIdx.x == 0) out.commit(t);
    }
    if constexpr (scan2_has_finish<Out>::value) {
        // a sink may finish the scan in its last workgroup: the first wave
        // runs out.finish() once the total is written
        if (blockIdx.x == gridDim.x - 1) {
            __syncthreads();
            if (threadIdx.x < 64) out.finish();
        }
    }
}

// One-kernel form for inputs of 2 to kChainTiles tiles: a workgroup takes
// its tile by ticket (so every tile it waits for belongs to a workgroup that
// started before it), publishes the tile's sum (plus one: zero is unset), adds
// the sums of all earlier tiles (each thread a strided share of them,
// bounded waits on relaxed loads of words that carry their own value), and
// scans its tile as the apply kernel does.  A tile waits
// for the earlier tiles' own sums, not their prefixes, so the waits do not
// chain.  The first tile runs the source's begin() before it publishes, so
// every sink call comes after it.  The last workgroup to finish returns the
// state to zero.
template <typename In, typename Out>
__global__ __launch_bounds__(kThreads) void k_scan2_chain(In in, Out out, uint64_t n,
                                                          uint32_t nt, ChainState* st,
                                                          uint32_t* err,
                                                          unsigned long long* total) {
    constexpr int kI = scan2_items<In>::value;
    __shared__ unsigned long long s_w[kI][kWaves];
    __shared__ unsigned long long s_p[kWaves];
    __shared__ uint32_t s_tile, s_last;
    if (threadIdx.x == 0) s_tile = atomicAdd(&st->ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if constexpr (scan2_has_begin<In>::value) {
        if (tile == 0) {
            in.begin();
            __threadfence();  // its writes, before the tile's sum is published
        }
    }
    const uint64_t lim = in.limit(n);
    const uint64_t base = (uint64_t)tile * kThreads * kI + threadIdx.x;
    typename In::Rec r[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        r[j] = in.load(i < n ? i : n - 1, i < lim);
    }
#pragma unroll
    for (int j = 0; j < kI; ++j) in.deref(r[j]);
    unsigned long long x[kI], inc[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        x[j] = i < lim ? in.value(i, r[j]) : 0ull;
        inc[j] = wave_incl_scan(x[j]);
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) {
#pragma unroll
        for (int j = 0; j < kI; ++j) s_w[j][w] = inc[j];
    }
    __syncthreads();  // (also: the first tile's begin() is done)
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
#pragma unroll
        for (int j = 0; j < kI; ++j)
#pragma unroll
            for (int q = 0; q < kWaves; ++q) t += s_w[j][q];
        __hip_atomic_store(&st->sum[tile], t + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned long long p = 0;
    for (uint32_t k = threadIdx.x; k < tile; k += kThreads) {
        uint32_t spins = 0;
        unsigned long long x;
        while ((x = __hip_atomic_load(&st->sum[k], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT)) == 0ull) {
            if (++spins >= kSpinLimit) {
                atomicOr(err, 1u);
                x = 1ull;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        p += x - 1ull;
    }
    if constexpr (scan2_has_begin<In>::value) {
        // begin()'s writes, before this tile's sink calls (thread 0 read the
        // first tile's sum; the barrier in block_sum orders the others)
        if (threadIdx.x == 0) __threadfence();
    }
    unsigned long long run = block_sum(p, s_p);
    if constexpr (scan2_has_begin<In>::value) __threadfence();
#pragma unroll
    for (int j = 0; j < kI; ++j) {
        const uint64_t i = base + (uint64_t)j * kThreads;
        unsigned long long before = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            const unsigned long long v = s_w[j][q];
            before += q < w ? v : 0ull;
            tot += v;
        }
        if (i < n) out(i, r[j], lim, run + before + inc[j] - x[j]);
        run += tot;
    }
    const bool last = tile == nt - 1;
    if (total && last && threadIdx.x == kThreads - 1) *total = run;
    if constexpr (scan2_has_tally<Out>::value) {
        unsigned long long t = 0;
#pragma unroll
        for (int j = 0; j < kI; ++j) {
            const uint64_t i = base + (uint64_t)j * kThreads;
            t += i < lim ? out.tally(i, r[j]) : 0ull;
        }
        t = block_sum(t, s_p);
        if (threadIdx.x == 0) out.commit(t);
    }
    __syncthreads();
    if constexpr (scan2_has_finish<Out>::value) {
        if (last && threadIdx.x < 64) out.finish();
    }
    if (threadIdx.x == 0) s_last = atomicAdd(&st->done, 1u) == nt - 1 ? 1u : 0u;
    __syncthreads();
    if (s_last) {
        // every workgroup has read what it waits for
        for (uint32_t t = threadIdx.x; t < nt; t += kThreads) st->sum[t] = 0ull;
        if (threadIdx.x == 0) {
            st->ticket = 0u;
            st->done = 0u;
        }
    }
}

// tiles the apply kernel adds up itself; beyond, a middle kernel scans them
constexpr uint64_t kScan2MaxTiles = 8192;
// partial words any scan2 over n elements needs
inline uint64_t scan2_parts(uint64_t n) {
    return div_up(std::max<uint64_t>(n, 1), (uint64_t)kThreads * kScan2MinItems);
}

// tiles of a scan2 over n elements (one tile: no reduce kernel)
template <typename In>
inline uint64_t scan2_tiles(uint64_t n) {
    return div_up(n, (uint64_t)kThreads * scan2_items<In>::value);
}

// Exclusive scan of in(i), i < n, as out(i, rec, lim, prefix); total ->
// *total.  `part` holds scan2_parts(n) words.
template <typename In, typename Out>
void scan2(Ctx& c, const char* name, In in, Out out, uint64_t n, unsigned long long* part,
           unsigned long long* total) {
    static_assert(scan2_items<In>::value >= kScan2MinItems,
                  "the partials are sized for kScan2MinItems elements per thread");
    if (n == 0) return;
    const uint64_t nt = scan2_tiles<In>(n);
    if (nt > 0xffffffffull) fail(GV_EINVAL, "scan too large");
    // (a source with begin() costs a device-scope fence per workgroup: up to
    // 64 tiles)
    const uint64_t cmax = scan2_has_begin<In>::value ? std::min<uint64_t>(kChainTiles, 64)
                                                      : kChainTiles;
    if (nt > 1 && nt <= cmax && c.chain) {
        c.launch(name, k_scan2_chain<In, Out>, nt, kThreads, in, out, n, (uint32_t)nt,
                 (ChainState*)c.chain, c.chain_err, total);
        return;
    }
    // a single tile adds no earlier partials: the apply kernel is the scan
    if (nt > 1) c.launch(name, k_scan2_reduce<In>, nt, kThreads, in, n, part);
    const int scanned = nt > kScan2MaxTiles ? 1 : 0;
    if (scanned) c.launch(name, k_scan2_partials, 1, kThreads, part, nt);
    c.launch(name, k_scan2_apply<In, Out>, nt, kThreads, in, out, n,
             (const unsigned long long*)part, scanned, total);
}

// ---------------------------------------------------------------- onesweep
// Stable LSD radix sort: one histogram kernel for every pass, then one kernel
// per 8-bit digit pass.  A pass ranks its 4096-key tile locally (ballot peer
// masks per wave and round, LDS column scans), publishes its per-digit counts,
// looks back per digit for the counts of earlier tiles, and scatters.  The
// number of keys may live on the device (n_dev); grids are sized for n_max.
#ifndef GV_OS_ITEMS
#define GV_OS_ITEMS 16
#endif
constexpr int kOsItems = GV_OS_ITEMS;  // keys per tile = kThreads * kOsItems
constexpr uint64_t kOsTile = (uint64_t)kThreads * kOsItems;  // 4096
constexpr uint32_t kOsAgg = 1u << 30, kOsIncl = 2u << 30, kOsMask = (1u << 30) - 1;

inline int os_passes(int bits) { return (bits + kRadixBits - 1) / kRadixBits; }
inline uint64_t os_tiles(uint64_t n) { return div_up(std::max<uint64_t>(n, 1), kOsTile); }
// Digit histograms: every histogram workgroup writes its own counts (no
// atomics), one small kernel adds them up.
constexpr uint64_t kHistGroups = 256;
inline uint64_t os_hist_groups(uint64_t n) { return std::min<uint64_t>(os_tiles(n), kHistGroups); }
// uint32 words of state a sort needs: tile counters and look-back status
// (the first os_zero_words, which must be zeroed), then the histograms and
// the per-group histograms
// Tiles per group of the two-level prefix that workgroup-index tiles use.
constexpr uint64_t kOsGroup = 16;
inline uint64_t os_groups(uint64_t n) { return div_up(os_tiles(n), kOsGroup); }
inline uint64_t os_zero_words(uint64_t n_max, int bits) {
    const uint64_t p = (uint64_t)os_passes(bits);
    return 64 + p * os_tiles(n_max) * kRadix + p * os_groups(n_max) * kRadix;
}
inline uint64_t os_words(uint64_t n_max, int bits) {
    const uint64_t p = (uint64_t)os_passes(bits);
    return os_zero_words(n_max, bits) + p * kRadix + os_hist_groups(n_max) * p * kRadix;
}

constexpr int kOsThreads = 1024;
constexpr int kOsWaves = kOsThreads / 64;
static_assert(kOsThreads == 4 * kRadix, "the pass kernel works in four quarters of 256 threads");
constexpr int kOsRounds = (int)(kOsTile / kOsThreads);  // keys per thread
// earlier tiles whose status one look-back lane reads per round
#ifndef GV_OS_LOOK_K
#define GV_OS_LOOK_K 4
#endif
constexpr int kOsLookK = GV_OS_LOOK_K;

// exclusive scan across a kOsThreads workgroup (all threads call it)
__device__ __forceinline__ uint32_t os_block_scan(uint32_t x, uint32_t* lds, uint32_t& total) {
    uint32_t inc = wave_incl_scan(x);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kOsWaves; ++i) {
        const uint32_t v = lds[i];
        off += (i < w) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

// the same for 64-bit values
__device__ __forceinline__ unsigned long long os_block_scan64(unsigned long long x,
                                                              unsigned long long* lds,
                                                              unsigned long long& total) {
    unsigned long long inc = wave_incl_scan(x);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    unsigned long long off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kOsWaves; ++i) {
        const unsigned long long v = lds[i];
        off += (i < w) ? v : 0ull;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

// LDS of the one-tile sort below.
struct TileSortLds {
    uint16_t cnt[kOsRounds * kOsWaves][kRadix];
    uint32_t part[4][kRadix];
    uint32_t start[kRadix];
    uint32_t w[kOsWaves];
    uint64_t skey[kOsTile];
};

// Tiles of at most kTileBitonicMax keys are sorted by a bitonic network in
// LDS, in log2(m) (log2(m) + 1) / 2 compare-exchange steps for m keys padded
// to a power of two with all-ones keys, instead of five barriers per radix
// pass.  The network is not stable, but every caller's keys are whole
// records (an edge key, a destination, or a key with its input position in
// the low bits), so keys that compare equal are identical and the result is
// the array a stable sort gives.
constexpr uint64_t kTileBitonicMax = 2048;

__device__ __forceinline__ void tile_bitonic(uint64_t (&key)[kOsRounds], uint32_t n,
                                             uint64_t sentinel, TileSortLds& L) {
    static_assert(kTileBitonicMax <= kOsTile, "the network works in the tile's LDS");
    const uint32_t t = threadIdx.x;
    uint32_t m = 2;
    while (m < n) m <<= 1;
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint32_t i = (uint32_t)j * kOsThreads + t;
        if (i < m) L.skey[i] = i < n ? key[j] : ~0ull;
    }
    // Thread c compares the pair (i, i + h), i being c with a zero bit
    // inserted at h.  While h <= 64 the pairs of a wave lie in its own 128
    // elements, so a step needs the whole workgroup's barrier only when it or
    // the step before it has h >= 128; else the wave's own order suffices.
    static_assert(kTileBitonicMax / 2 <= kOsThreads, "one pair per thread");
    uint32_t hprev = m;  // the loads above cross waves
    for (uint32_t k = 2; k <= m; k <<= 1) {
        for (uint32_t h = k >> 1; h > 0; h >>= 1) {
            if (h >= 128 || hprev >= 128) {
                __syncthreads();
            } else {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            hprev = h;
            if (t < m / 2) {
                const uint32_t i = ((t & ~(h - 1)) << 1) | (t & (h - 1));
                const uint32_t p = i + h;
                const uint64_t a = L.skey[i], b = L.skey[p];
                if ((a > b) == ((i & k) == 0)) {
                    L.skey[i] = b;
                    L.skey[p] = a;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint32_t i = (uint32_t)j * kOsThreads + t;
        key[j] = i < n ? L.skey[i] : sentinel;
    }
    __syncthreads();  // the caller may reuse the LDS
}

// Stable LSD sort of one tile in LDS: thread t holds key[j] = element
// j * kOsThreads + t, the first n live; `passes` 8-bit digits (the ranking of
// the pass kernel on a single tile, so no look-back).  key[] comes back
// holding the sorted order in the same layout, `sentinel` past n.  Every
// thread of the workgroup calls it (barriers inside).  Live keys must be
// below 2^(8 * passes).
__device__ __forceinline__ void tile_sort(uint64_t (&key)[kOsRounds], uint64_t n, int passes,
                                          uint64_t sentinel, TileSortLds& L) {
    if (n <= kTileBitonicMax) {
        if (n > 1) {
            tile_bitonic(key, (uint32_t)n, sentinel, L);
        } else {
            // nothing to order: element 0 stays where it is
            if (threadIdx.x >= n) key[0] = sentinel;
#pragma unroll
            for (int j = 1; j < kOsRounds; ++j) key[j] = sentinel;
        }
        return;
    }
    const uint32_t t = threadIdx.x;
    const int w = t >> 6;
    const uint32_t d = t & (kRadix - 1), q = t >> 8;
    constexpr int kQRows = kOsRounds * kOsWaves / 4;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        {
            uint32_t* c32 = (uint32_t*)&L.cnt[0][0];
            for (int i = t; i < kOsRounds * kOsWaves * kRadix / 2; i += kOsThreads) c32[i] = 0;
        }
        __syncthreads();
        uint16_t rk[kOsRounds];
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) {
            const bool act = (uint64_t)j * kOsThreads + t < n;
            const uint32_t dg = (uint32_t)(key[j] >> shift) & (kRadix - 1);
            const uint64_t peers = digit_peers(dg, act);
            rk[j] = (uint16_t)rank_below(peers);
            if (act && rk[j] == 0) L.cnt[j * kOsWaves + w][dg] = (uint16_t)popc64(peers);
        }
        __syncthreads();
        // rows in key order: exclusive prefixes per digit, 16 rows per quarter
        uint32_t run = 0;
#pragma unroll
        for (int r = 0; r < kQRows; ++r) {
            const uint32_t c = L.cnt[q * kQRows + r][d];
            L.cnt[q * kQRows + r][d] = (uint16_t)run;
            run += c;
        }
        L.part[q][d] = run;
        __syncthreads();
        uint32_t qoff = 0;
        for (uint32_t qq = 0; qq < q; ++qq) qoff += L.part[qq][d];
        if (qoff) {
#pragma unroll
            for (int r = 0; r < kQRows; ++r) L.cnt[q * kQRows + r][d] += (uint16_t)qoff;
        }
        const uint32_t dcount = L.part[0][d] + L.part[1][d] + L.part[2][d] + L.part[3][d];
        uint32_t tot;
        const uint32_t ex = os_block_scan(q == 0 ? dcount : 0u, L.w, tot);
        if (q == 0) L.start[d] = ex;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) {
            if ((uint64_t)j * kOsThreads + t < n) {
                const uint32_t dg = (uint32_t)(key[j] >> shift) & (kRadix - 1);
                L.skey[L.start[dg] + L.cnt[j * kOsWaves + w][dg] + rk[j]] = key[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) {
            const uint64_t i = (uint64_t)j * kOsThreads + t;
            key[j] = i < n ? L.skey[i] : sentinel;
        }
        __syncthreads();  // skey and cnt are rewritten by the next pass
    }
}

// Histogram counting: 0 = the lowest lane of each group of equal digits adds
// the group's size (eight ballots per digit, no conflicting LDS atomics);
// 1 = every lane adds one to a histogram shared by a quarter of the
// workgroup (LDS atomics, conflicts only between equal digits).
#ifndef GV_OS_HIST_MODE
#define GV_OS_HIST_MODE 1
#endif
#ifndef GV_OS_HIST_COPIES
#define GV_OS_HIST_COPIES 4
#endif
constexpr int kOsHistMode = GV_OS_HIST_MODE;
constexpr int kOsHistCopies = kOsHistMode == 1 ? GV_OS_HIST_COPIES : 1;

template <typename K>
__global__ __launch_bounds__(kOsThreads) void k_os_hist(const K* keys, const uint32_t* n_dev,
                                                        uint64_t n_max, int passes,
                                                        uint32_t* hpart) {
    __shared__ uint32_t h[kOsHistCopies][8][kRadix];
    const uint64_t n = n_dev ? min<uint64_t>(*n_dev, n_max) : n_max;
    for (int i = threadIdx.x; i < kOsHistCopies * 8 * kRadix; i += kOsThreads)
        (&h[0][0][0])[i] = 0;
    __syncthreads();
    const uint32_t copy = kOsHistCopies == 1 ? 0u : (threadIdx.x >> 6) & (kOsHistCopies - 1);
    // tiles of n_max: loads need not wait for n, counting masks with it
    const uint64_t ntiles = (n_max + kOsTile - 1) / kOsTile;
    for (uint64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const uint64_t base = tl * kOsTile;
        K kk[kOsRounds];
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) {
            const uint64_t i = base + (uint64_t)j * kOsThreads + threadIdx.x;
            kk[j] = i < n_max ? keys[i] : K(0);
        }
#pragma unroll
        for (int j = 0; j < kOsRounds; ++j) {
            const uint64_t i = base + (uint64_t)j * kOsThreads + threadIdx.x;
            const bool act = i < n;
            for (int p = 0; p < passes; ++p) {
                const uint32_t d = (uint32_t)(kk[j] >> (p * kRadixBits)) & (kRadix - 1);
                if (kOsHistMode == 1) {
                    if (act) atomicAdd(&h[copy][p][d], 1u);
                } else {
                    const uint64_t peers = digit_peers(d, act);
                    if (act && rank_below(peers) == 0) atomicAdd(&h[0][p][d], popc64(peers));
                }
            }
        }
    }
    __syncthreads();
    uint32_t* out = hpart + (uint64_t)blockIdx.x * passes * kRadix;
    for (int i = threadIdx.x; i < passes * kRadix; i += kOsThreads) {
        uint32_t x = 0;
#pragma unroll
        for (int c = 0; c < kOsHistCopies; ++c) x += h[c][i / kRadix][i % kRadix];
        out[i] = x;
    }
}

// hist[i] = sum over the histogram workgroups of their count i: a
// workgroup takes 16 counters, its 16 row groups each add every 16th
// workgroup's count with independent loads, LDS adds the row groups
// (when vpart is given, workgroup 0 also adds the groups' vpart counts into
// *vtotal, and their kpart sums into *ktotal)
static __global__ __launch_bounds__(kThreads) void k_os_hist_sum(
    const uint32_t* hpart, uint32_t groups, uint32_t words, uint32_t* hist, const uint32_t* vpart,
    unsigned long long* vtotal, const unsigned long long* kpart, unsigned long long* ktotal) {
    __shared__ uint32_t red[16][17];
    __shared__ unsigned long long s_v[kWaves];
    if (vpart && blockIdx.x == 0) {
        static_assert(kHistGroups <= kThreads, "one thread per histogram group");
        const unsigned long long x = threadIdx.x < groups ? vpart[threadIdx.x] : 0u;
        const unsigned long long t = block_sum(x, s_v);
        const unsigned long long y = threadIdx.x < groups ? kpart[threadIdx.x] : 0ull;
        const unsigned long long u = block_sum(y, s_v);
        if (threadIdx.x == 0) {
            *vtotal = t;
            *ktotal = u;
        }
    }
    if (words == 0) return;
    const uint32_t col = threadIdx.x & 15, rg = threadIdx.x >> 4;
    const uint32_t i = blockIdx.x * 16 + col;
    const uint32_t ic = i < words ? i : 0u;
    uint32_t s = 0;
    constexpr uint32_t kRows = (uint32_t)(kHistGroups / 16);
#pragma unroll
    for (uint32_t r = 0; r < kRows; ++r) {
        const uint32_t gi = rg + 16 * r;
        const uint32_t x = hpart[(uint64_t)(gi < groups ? gi : 0u) * words + ic];
        s += gi < groups ? x : 0u;
    }
    red[rg][col] = s;
    __syncthreads();
    if (rg == 0 && i < words) {
        uint32_t t = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += red[k][col];
        hist[i] = t;
    }
}

// One pass over 8 bits at `shift`: rank the tile locally (ballot peer masks
// per wave and round, LDS column scans), publish per-digit tile counts, look
// back per digit for the counts of earlier tiles, scatter.
template <typename K, bool HasVal>
__global__ __launch_bounds__(kOsThreads) void k_os_pass(const K* kin, K* kout, const uint32_t* vin,
                                                        uint32_t* vout, const uint32_t* n_dev,
                                                        uint64_t n_max, int shift,
                                                        const uint32_t* hist, uint32_t* status,
                                                        uint32_t* gstatus, uint32_t* counter,
                                                        int block_tiles, uint32_t* err,
                                                        uint32_t spin_limit) {
    // cnt[round * waves + wave][digit]: counts, then exclusive prefixes
    __shared__ uint16_t cnt[kOsRounds * kOsWaves][kRadix];
    __shared__ uint32_t part[4][kRadix];
    __shared__ uint32_t s_base[kRadix];   // global start of digit run of this tile
    __shared__ uint32_t s_lstart[kRadix]; // start of digit run inside the tile
    __shared__ unsigned long long s_w64[kOsWaves];
    __shared__ uint32_t s_tile;
    __shared__ K skey[kOsTile];
    __shared__ uint32_t sval[HasVal ? kOsTile : 1];
    const uint32_t t = threadIdx.x;
    const int w = t >> 6;
    // the pass histogram and the key count do not depend on the tile
    const uint32_t hv = t < kRadix ? hist[t] : 0u;
    const uint64_t n = n_dev ? min<uint64_t>(*n_dev, n_max) : n_max;
    // Tile ids: when every tile's workgroup fits on the device at once, the
    // workgroup index (all tiles run together, so each one a tile waits for
    // is running); else a ticket in launch order, so that every tile a tile
    // waits for has started.
    uint64_t tile = blockIdx.x;
    if (!block_tiles) {
        if (t == 0) s_tile = atomicAdd(counter, 1u);
        __syncthreads();
        tile = s_tile;
    }
    const uint64_t base = tile * kOsTile;
    K key[kOsRounds];
    uint32_t val[kOsRounds];
    uint16_t rk[kOsRounds];
    // loads bounded by n_max (the buffer size), so they need not wait for n
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = base + (uint64_t)j * kOsThreads + t;
        const bool in = i < n_max;
        key[j] = in ? kin[i] : K(0);
        if (HasVal) val[j] = in ? vin[i] : 0u;
    }
    {
        uint32_t* c32 = (uint32_t*)&cnt[0][0];
        for (int i = t; i < kOsRounds * kOsWaves * kRadix / 2; i += kOsThreads) c32[i] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = base + (uint64_t)j * kOsThreads + t;
        if (i >= n) {
            key[j] = K(0);
            if (HasVal) val[j] = 0u;
        }
    }
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = base + (uint64_t)j * kOsThreads + t;
        const bool act = i < n;
        const uint32_t d = (uint32_t)(key[j] >> shift) & (kRadix - 1);
        const uint64_t peers = digit_peers(d, act);
        rk[j] = (uint16_t)rank_below(peers);
        if (act && rk[j] == 0) cnt[j * kOsWaves + w][d] = (uint16_t)popc64(peers);
    }
    __syncthreads();
    // column scans: digit d = t % 256, quarter q = t / 256 covers 16 rows
    const uint32_t d = t & (kRadix - 1), q = t >> 8;
    constexpr int kRows = kOsRounds * kOsWaves;
    constexpr int kQRows = kRows / 4;
    uint32_t run = 0;
#pragma unroll
    for (int r = 0; r < kQRows; ++r) {
        const uint32_t c = cnt[q * kQRows + r][d];
        cnt[q * kQRows + r][d] = (uint16_t)run;
        run += c;
    }
    part[q][d] = run;
    __syncthreads();
    uint32_t qoff = 0;
    for (uint32_t qq = 0; qq < q; ++qq) qoff += part[qq][d];
    const uint32_t dcount = part[0][d] + part[1][d] + part[2][d] + part[3][d];
    if (qoff) {
#pragma unroll
        for (int r = 0; r < kQRows; ++r) cnt[q * kQRows + r][d] += (uint16_t)qoff;
    }
    __shared__ uint32_t lb_prefix[kRadix];
    if (block_tiles) {
        // Every tile runs at once: a two-level prefix, two rounds of loads
        // whatever the tile's position.  Four lanes per digit add the counts
        // of the earlier tiles of the tile's group of kOsGroup; the group's
        // last tile publishes the group total; then the four lanes add the
        // totals of the earlier groups.
        if (t < kRadix) st_status32(status + tile * kRadix + t, kOsAgg | dcount);
        const uint32_t ld = t >> 2, lq = t & 3, gbase = lane_id() & ~3u;
        const uint64_t G = tile / kOsGroup;
        auto wait_sum = [&](uint32_t* base, uint64_t first, uint64_t end) {
            uint32_t wv[kOsLookK];
#pragma unroll
            for (int kk = 0; kk < kOsLookK; ++kk) {
                const uint64_t j = first + lq * kOsLookK + kk;
                wv[kk] = j < end ? ld_status32(base + j * kRadix + ld) : kOsAgg;
            }
            uint32_t sum = 0;
#pragma unroll
            for (int kk = 0; kk < kOsLookK; ++kk) {
                const uint64_t j = first + lq * kOsLookK + kk;
                if ((wv[kk] >> 30) == 0 || spin_limit == 0) {
                    uint32_t spins = 0;
                    while ((wv[kk] >> 30) == 0 && spins++ < spin_limit)
                        wv[kk] = ld_status32(base + j * kRadix + ld);
                    if ((wv[kk] >> 30) == 0 || spin_limit == 0) {
                        *err = 1;
                        wv[kk] = kOsAgg;
                    }
                }
                sum += wv[kk] & kOsMask;
            }
            uint32_t all = 0;
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) all += __shfl(sum, (int)(gbase + qq), 64);
            return all;
        };
        static_assert(kOsGroup == 4 * kOsLookK, "a group is one round of four lanes");
        const uint32_t local = wait_sum(status, G * kOsGroup, tile);
        if (tile % kOsGroup == kOsGroup - 1 && lq == 0) {
            const uint32_t own = part[0][ld] + part[1][ld] + part[2][ld] + part[3][ld];
            st_status32(gstatus + G * kRadix + ld, kOsAgg | (local + own));
        }
        uint32_t global = 0;
        for (uint64_t g0 = 0; g0 < G; g0 += kOsGroup) global += wait_sum(gstatus, g0, G);
        if (lq == 0) lb_prefix[ld] = local + global;
    } else {
    // publish this tile's counts, then look back with four consecutive lanes
    // per digit: each round a lane reads the status of kOsLookK earlier
    // tiles with independent loads, and the four lanes add them, newest
    // first, up to the first inclusive one
    if (t < kRadix) st_status32(status + tile * kRadix + t, (tile == 0 ? kOsIncl : kOsAgg) | dcount);
    {
        const uint32_t ld = t >> 2, lq = t & 3, gbase = lane_id() & ~3u;
        uint32_t lp = 0;
        bool open = tile > 0;
        int64_t j0 = (int64_t)tile - 1;
        while (open) {
            uint32_t wv[kOsLookK];
#pragma unroll
            for (int kk = 0; kk < kOsLookK; ++kk) {
                const int64_t j = j0 - (int64_t)(lq * kOsLookK + kk);
                // before tile 0: an inclusive zero
                wv[kk] = j >= 0 ? ld_status32(status + (uint64_t)j * kRadix + ld) : kOsIncl;
            }
#pragma unroll
            for (int kk = 0; kk < kOsLookK; ++kk) {
                const int64_t j = j0 - (int64_t)(lq * kOsLookK + kk);
                if ((wv[kk] >> 30) == 0 || (spin_limit == 0 && j >= 0)) {
                    uint32_t spins = 0;
                    while ((wv[kk] >> 30) == 0 && spins++ < spin_limit)
                        wv[kk] = ld_status32(status + (uint64_t)j * kRadix + ld);
                    if ((wv[kk] >> 30) == 0 || spin_limit == 0) {
                        *err = 1;
                        wv[kk] = kOsIncl;
                    }
                }
            }
            uint32_t ls = 0;
            bool lh = false;
#pragma unroll
            for (int kk = 0; kk < kOsLookK; ++kk) {
                if (!lh) {
                    ls += wv[kk] & kOsMask;
                    lh = (wv[kk] >> 30) == 2;
                }
            }
            bool hit = false;
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const uint32_t vs = __shfl(ls, (int)(gbase + qq), 64);
                const int vh = __shfl((int)lh, (int)(gbase + qq), 64);
                if (!hit) {
                    lp += vs;
                    hit = vh != 0;
                }
            }
            open = !hit;
            j0 -= 4 * kOsLookK;
        }
        if (lq == 0) lb_prefix[ld] = lp;
    }
    }
    __syncthreads();
    const uint32_t prefix = t < kRadix ? lb_prefix[t] : 0u;
    if (!block_tiles && t < kRadix && tile > 0)
        st_status32(status + tile * kRadix + t, kOsIncl | (prefix + dcount));
    // global start of each digit (pass histogram) and start inside the tile:
    // one scan of both, the histogram in the high half (neither half carries)
    unsigned long long tot;
    const unsigned long long both =
        os_block_scan64(((unsigned long long)hv << 32) | (t < kRadix ? dcount : 0u), s_w64, tot);
    const uint32_t gex = (uint32_t)(both >> 32), lex = (uint32_t)both;
    if (t < kRadix) {
        s_base[t] = gex + prefix;
        s_lstart[t] = lex;
    }
    __syncthreads();
    // place keys in tile order of their digit, then write each digit run
    // with consecutive lanes (coalesced)
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint64_t i = base + (uint64_t)j * kOsThreads + t;
        if (i < n) {
            const uint32_t dd = (uint32_t)(key[j] >> shift) & (kRadix - 1);
            const uint32_t lp = s_lstart[dd] + cnt[j * kOsWaves + w][dd] + rk[j];
            skey[lp] = key[j];
            if (HasVal) sval[lp] = val[j];
        }
    }
    __syncthreads();
    const uint64_t tn = n > base ? min<uint64_t>(n - base, kOsTile) : 0;
#pragma unroll
    for (int j = 0; j < kOsRounds; ++j) {
        const uint32_t lp = j * kOsThreads + t;
        if (lp < tn) {
            const K k = skey[lp];
            const uint32_t dd = (uint32_t)(k >> shift) & (kRadix - 1);
            const uint32_t pos = s_base[dd] + (lp - s_lstart[dd]);
            // stays below n unless a look-back wait ran out (err is set);
            // then the write is dropped rather than sent out of bounds
            if (pos < n) {
                kout[pos] = k;
                if (HasVal) vout[pos] = sval[lp];
            }
        }
    }
}

// concurrent: other kernels may hold compute units while the passes run
// (work on another stream), so tiles take tickets in launch order
template <typename K, bool HasVal>
bool onesweep_passes(Ctx& c, K* k0, K* k1, uint32_t* v0, uint32_t* v1, const uint32_t* n_dev,
                     uint64_t n_max, int bits, uint32_t* state, uint32_t* err,
                     uint32_t spin_limit = kSpinLimit, bool concurrent = false);

// Look-back counts are 30-bit fields of the status words: a sort takes fewer
// than 2^30 keys.
constexpr uint64_t kOsMaxKeys = 1ull << 30;

// Sorts n keys (n on the device when n_dev != null, n_max bounds it) by bits
// [0, bits), stably, ping-ponging k0/k1 (v0/v1).  `state` must hold
// os_words(n_max, bits) uint32 words, the first os_zero_words of them
// zeroed; `concurrent` as for onesweep_passes.  Returns true if the result is
// in k1/v1.
template <typename K, bool HasVal>
bool onesweep(Ctx& c, K* k0, K* k1, uint32_t* v0, uint32_t* v1, const uint32_t* n_dev,
              uint64_t n_max, int bits, uint32_t* state, uint32_t* err,
              uint32_t spin_limit = kSpinLimit, bool concurrent = false) {
    if (n_max <= 1 || bits <= 0) return false;
    if (n_max >= kOsMaxKeys) fail(GV_EINVAL, "sort of 2^30 or more keys");
    const int passes = os_passes(bits);
    if (passes > 8) fail(GV_EINVAL, "too many radix passes");
    const uint64_t hg = os_hist_groups(n_max);
    const uint32_t hwords = (uint32_t)passes * kRadix;
    uint32_t* hist = state + os_zero_words(n_max, bits);  // passes * 256 counters
    uint32_t* hpart = hist + hwords;      // per histogram workgroup
    c.launch("sort_hist", k_os_hist<K>, hg, kOsThreads, (const K*)k0, n_dev, n_max, passes, hpart);
    c.launch("sort_hist", k_os_hist_sum, div_up(hwords, 16), kThreads, (const uint32_t*)hpart,
             (uint32_t)hg, hwords, hist, (const uint32_t*)nullptr, (unsigned long long*)nullptr,
             (const unsigned long long*)nullptr, (unsigned long long*)nullptr);
    return onesweep_passes<K, HasVal>(c, k0, k1, v0, v1, n_dev, n_max, bits, state, err,
                                      spin_limit, concurrent);
}

// Per-group digit counts of a sort whose histogram kernel is fused into the
// kernel that writes the keys: group g writes os_passes(bits) * kRadix counts
// at os_hpart(...) + g * os_passes(bits) * kRadix, for os_hist_groups(n_max)
// groups of kOsTile-key tiles (tile t to group t % groups).
inline uint32_t* os_hpart(uint32_t* state, uint64_t n_max, int bits) {
    return state + os_zero_words(n_max, bits) + (uint64_t)os_passes(bits) * kRadix;
}

// Adds the per-group counts into the pass histograms; with vpart, also adds
// os_hist_groups(n_max) per-group counts into *vtotal and the groups' 64-bit
// kpart sums into *ktotal.  One launch, also when there is nothing to sort.
inline void os_hist_sum(Ctx& c, uint32_t* state, uint64_t n_max, int bits, const uint32_t* vpart,
                        unsigned long long* vtotal, const unsigned long long* kpart,
                        unsigned long long* ktotal) {
    const uint32_t hwords = bits > 0 ? (uint32_t)os_passes(bits) * kRadix : 0u;
    c.launch("sort_hist", k_os_hist_sum, std::max<uint64_t>(div_up(hwords, 16), 1), kThreads,
             (const uint32_t*)os_hpart(state, n_max, bits), (uint32_t)os_hist_groups(n_max), hwords,
             state + os_zero_words(n_max, bits), vpart, vtotal, kpart, ktotal);
}

// The passes of onesweep, once the pass histograms are in the state.
template <typename K, bool HasVal>
bool onesweep_passes(Ctx& c, K* k0, K* k1, uint32_t* v0, uint32_t* v1, const uint32_t* n_dev,
                     uint64_t n_max, int bits, uint32_t* state, uint32_t* err,
                     uint32_t spin_limit, bool concurrent) {
    if (n_max <= 1 || bits <= 0) return false;
    if (n_max >= kOsMaxKeys) fail(GV_EINVAL, "sort of 2^30 or more keys");
    const int passes = os_passes(bits);
    if (passes > 8) fail(GV_EINVAL, "too many radix passes");
    const uint64_t nt = os_tiles(n_max);
    uint32_t* counters = state;           // 64 words
    uint32_t* status = state + 64;        // passes * tiles * 256
    uint32_t* gstatus = status + (uint64_t)passes * nt * kRadix;  // passes * groups * 256
    const uint64_t ng = os_groups(n_max);
    uint32_t* hist = state + os_zero_words(n_max, bits);  // passes * 256 counters
    const int block_tiles =
        !concurrent && nt <= resident_grid(k_os_pass<K, HasVal>, kOsThreads) ? 1 : 0;
    bool flip = false;
    for (int p = 0; p < passes; ++p) {
        K* kin = flip ? k1 : k0;
        K* kout = flip ? k0 : k1;
        uint32_t* vin = flip ? v1 : v0;
        uint32_t* vout = flip ? v0 : v1;
        c.launch("sort_pass", k_os_pass<K, HasVal>, nt, kOsThreads, (const K*)kin, kout,
                 (const uint32_t*)vin, vout, n_dev, n_max, p * kRadixBits,
                 (const uint32_t*)(hist + (uint64_t)p * kRadix),
                 status + (uint64_t)p * nt * kRadix, gstatus + (uint64_t)p * ng * kRadix,
                 counters + p, block_tiles, err, spin_limit);
        flip = !flip;
    }
    return flip;
}

static __global__ void k_zero_words(uint32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

inline void zero_words(Ctx& c, uint32_t* p, uint64_t n) {
    if (n) c.launch("zero", k_zero_words, std::min<uint64_t>(div_up(n, kThreads), 4096), kThreads, p, n);
}

}  // namespace gv
