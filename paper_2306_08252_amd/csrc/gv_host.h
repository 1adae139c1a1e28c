// gv_host.h -- host-side launch context, error handling and scratch carving.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/graphvine.h"

namespace gv {

// Internal failures carry a GV_* code; they are caught at the C ABI.
struct Error {
    int code;
    const char* what;
};

[[noreturn]] inline void fail(int code, const char* what) { throw Error{code, what}; }

// Text of the last internal failure on this thread ("call: HIP error").
inline char* last_error_text() {
    static thread_local char buf[256] = "";
    return buf;
}

inline void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    std::snprintf(last_error_text(), 256, "%s: %s", what, hipGetErrorString(e));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) fail(GV_ENOMEM, what);
    fail(GV_EDEVICE, what);
}

// Workgroups of `kernel` (launched with `block` threads) that the current
// device holds at once: compute units times resident workgroups per unit.
// Kernels that loop over their work size their grid with it, so that no
// workgroup waits for a second round.  Cached per kernel and device.
template <typename... KArgs>
uint64_t resident_grid(void (*kernel)(KArgs...), uint32_t block) {
    struct Entry {
        const void* k;
        int dev;
        uint32_t block;
        uint64_t grid;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& e : cache)
        if (e.k == (const void*)kernel && e.dev == dev && e.block == block) return e.grid;
    int cus = 0, per = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
              "hipDeviceGetAttribute");
    hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, (int)block, 0),
              "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    const uint64_t grid = (uint64_t)std::max(cus, 1) * (uint64_t)std::max(per, 1);
    cache.push_back({(const void*)kernel, dev, block, grid});
    return grid;
}

// Kernel launches go through Ctx so that they can be timed with HIP events on
// the graph's stream when profiling is enabled.  With every kernel timed, each
// launch gets its own pair of events.  When only one kernel name is timed,
// one pair of events brackets each run of consecutive launches of it (the
// radix passes of a sort are one run): an event record costs GPU time of its
// own, and a run shares one, so the average per launch stays close to the
// kernels' own durations.
struct Ctx {
    hipStream_t stream = nullptr;
    uint64_t seq = 0;  // operations queued so far (launches, recorded graphs)
    // device state of the one-kernel small scans (a ChainState) and the word
    // their bounded waits flag when one runs out; null: two-kernel scans only
    void* chain = nullptr;
    uint32_t* chain_err = nullptr;
    bool prof = false;
    std::string only;  // when non-empty, only launches of this name are timed
    struct Rec {
        const char* name;
        hipEvent_t e0, e1;
        uint64_t launches;
    };
    hipEvent_t run_e0 = nullptr;   // open run of the timed kernel
    const char* run_name = nullptr;
    uint64_t run_n = 0;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    struct Sum {
        std::string name;
        uint64_t launches;
        double ms;
    };
    std::vector<Sum> sums;

    hipEvent_t event() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "hipEventCreate");
        return e;
    }

    // Closes an open run of the timed kernel (records its end event).
    void close_run() {
        if (!run_e0) return;
        hipEvent_t e1 = event();
        hip_check(hipEventRecord(e1, stream), "hipEventRecord");
        recs.push_back({run_name, run_e0, e1, run_n});
        run_e0 = nullptr;
        run_n = 0;
    }

    // Fold finished records into per-name sums (synchronises the stream).
    void collect() {
        close_run();
        if (recs.empty()) return;
        hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
        for (auto& r : recs) {
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, r.e0, r.e1), "hipEventElapsedTime");
            bool found = false;
            for (auto& s : sums)
                if (s.name == r.name) {
                    s.launches += r.launches;
                    s.ms += ms;
                    found = true;
                    break;
                }
            if (!found) sums.push_back({r.name, r.launches, (double)ms});
            spare.push_back(r.e0);
            spare.push_back(r.e1);
        }
        recs.clear();
    }

    void release() {
        if (run_e0) hipEventDestroy(run_e0);
        run_e0 = nullptr;
        for (auto& r : recs) {
            hipEventDestroy(r.e0);
            hipEventDestroy(r.e1);
        }
        recs.clear();
        for (auto e : spare) hipEventDestroy(e);
        spare.clear();
    }

    template <typename... KArgs, typename... Args>
    void launch(const char* name, void (*kernel)(KArgs...), uint64_t grid, uint32_t block,
                Args... args) {
        if (grid == 0) return;
        if (grid > 0x7fffffffull) fail(GV_EINVAL, "grid too large");
        ++seq;
        const bool timed = prof && (only.empty() || only == name);
        if (prof && !only.empty()) {
            // runs of the one timed kernel
            if (!timed) {
                close_run();
            } else if (!run_e0) {
                run_e0 = event();
                run_name = name;
                hip_check(hipEventRecord(run_e0, stream), "hipEventRecord");
            }
            hipLaunchKernelGGL(kernel, dim3((uint32_t)grid), dim3(block), 0, stream, args...);
            hip_check(hipGetLastError(), name);
            if (timed) ++run_n;
            if (recs.size() > 4096) collect();
            return;
        }
        hipEvent_t e0 = nullptr;
        if (timed) {
            e0 = event();
            hip_check(hipEventRecord(e0, stream), "hipEventRecord");
        }
        hipLaunchKernelGGL(kernel, dim3((uint32_t)grid), dim3(block), 0, stream, args...);
        hip_check(hipGetLastError(), name);
        if (timed) {
            hipEvent_t e1 = event();
            hip_check(hipEventRecord(e1, stream), "hipEventRecord");
            recs.push_back({name, e0, e1, 1});
            if (recs.size() > 4096) collect();
        }
    }
};

// Carves typed arrays out of one device buffer.  With base == nullptr it only
// measures, so a caller can size the buffer first and carve second.
struct Carver {
    char* base;
    size_t used = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(uint64_t n) {
        used = (used + 255) & ~size_t(255);
        T* p = base ? (T*)(base + used) : nullptr;
        used += (size_t)n * sizeof(T);
        return p;
    }
};

// Growable device scratch buffer owned by a graph.
struct Scratch {
    void* ptr = nullptr;
    size_t cap = 0;
    uint64_t gen = 0;  // counts reallocations
    void ensure(size_t bytes, hipStream_t s) {
        if (bytes <= cap) return;
        if (ptr) {
            hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
            hip_check(hipFree(ptr), "hipFree");
            ptr = nullptr;
            cap = 0;
        }
        size_t want = bytes + bytes / 4 + (1 << 20);
        hip_check(hipMalloc(&ptr, want), "hipMalloc scratch");
        cap = want;
        ++gen;
    }
    void release() {
        if (ptr) hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
};

inline uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace gv
