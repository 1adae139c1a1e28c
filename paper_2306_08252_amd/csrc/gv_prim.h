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

// Exclusive scan of in(0..n-1) into out(i, prefix); the sum goes to the device
// location `total` when non-null.  `partial` needs scan_partials_needed(n).
template <typename T, typename In, typename Out>
void scan_excl(Ctx& c, In in, Out out, uint64_t n, T* partial, T* total) {
    if (n == 0) {
        if (total) hip_check(hipMemsetAsync(total, 0, sizeof(T), c.stream), "memset");
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
