// gv_noalloc.hip -- gv_edge_exists_noalloc: the query batch of gv_edge_exists
// with its temporaries in a fixed device array instead of the graph's
// growable scratch, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable.  Its host-side name is only a
// stand-in: the device address is looked up once per device with
// hipGetSymbolAddress (at graph creation, with that device current) and only
// that address is handed to kernels.  Every call on one device uses the same
// array and leaves its contents behind; the batch's first kernel clears what
// must start at zero (look-back state and counters) with a kernel, so nothing
// depends on the previous call.  Calls that overlap on one device (two graphs
// on the same GPU, or several streams) race on the array and must be
// serialised by the caller.
#include <mutex>

#include "gv_graph.h"

namespace gv {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;     // 64 MiB per device
constexpr uint64_t kNoAllocMaxPairs = 1ull << 18;     // query pairs per call
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_mu;
void* g_ptr[kNoAllocMaxDevices];
bool g_ready[kNoAllocMaxDevices];
}  // namespace

void noalloc_setup() {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocMaxDevices) return;  // the entry point then reports GV_EINVAL
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ready[dev]) return;
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    // occupancy lookups of the query kernels, cached before any call
    edge_batch_warm();
    g_ptr[dev] = p;
    g_ready[dev] = true;
}

void* noalloc_ptr(int dev) {
    if (dev < 0 || dev >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ready[dev] ? g_ptr[dev] : nullptr;
}

}  // namespace gv

using namespace gv;

// Declared in graphvine.h; the C ABI wrapper (argument checks, device guard,
// error codes) is in gv_api.hip.
void gv_noalloc_query(gv_graph* g, const uint32_t* d_src, const uint32_t* d_dst, uint64_t n,
                      uint8_t* d_out) {
    if (n > kNoAllocMaxPairs) fail(GV_ERANGE, "more pairs than the fixed scratch holds");
    void* p = noalloc_ptr(g->device);
    if (!p) fail(GV_EINVAL, "fixed scratch not set up on this device");
    // no event records (they would create events): timing is off for this call
    const bool prof = g->ctx.prof;
    g->ctx.prof = false;
    try {
        edge_batch(g, kQuery, d_src, d_dst, n, d_out, true, p, kNoAllocBytes);
    } catch (...) {
        g->ctx.prof = prof;
        throw;
    }
    g->ctx.prof = prof;
}
