// gv_served.hip -- mixed edge updates with last-writer reduction: the tick of
// the served form.
//
// A list of (op, src, dst) entries, op 0 = insert and 1 = delete, has the
// effect of applying the entries one at a time in list order with set
// semantics (Sec. 4.3's batch model; the order inside a batch is ours): a
// pair's final membership is decided by its last entry, and entries with an
// inactive or out-of-range endpoint change nothing.  On the device: pack the
// valid entries as keys (src << L) | dst with their list position, sort them
// stably, keep the last entry of every key, and write it to the delete list
// or the insert list at its sorted position (the other positions hold an
// out-of-range pair, which the batch paths reject).  The two lists are then
// applied as one delete batch and one insert batch: no key is in both, so
// their order does not matter.
#include "gv_graph.h"
#include "gv_prim.h"

namespace gv {

namespace {

constexpr uint32_t kNoPair = 0xFFFFFFFFu;  // an id past every table

__global__ __launch_bounds__(kThreads) void k_mixed_pack(GraphView g, const uint8_t* op,
                                                         const uint32_t* src,
                                                         const uint32_t* dst, uint64_t n,
                                                         uint64_t* keys, uint32_t* pos) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = src[i], d = dst[i];
    const bool ok = active_bit(g, s) & active_bit(g, d) & (op[i] <= 1);
    // an invalid entry gets bit 2L: it sorts after every valid key
    keys[i] = ok ? ((uint64_t)s << g.L) | d : (1ull << (2 * g.L));
    pos[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kThreads) void k_mixed_split(GraphView g, const uint64_t* keys,
                                                          const uint32_t* pos, const uint8_t* op,
                                                          uint64_t n, uint32_t* ins_src,
                                                          uint32_t* ins_dst, uint32_t* del_src,
                                                          uint32_t* del_dst) {
    const uint64_t p = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n) return;
    const uint64_t k = keys[p];
    const bool valid = (k >> (2 * g.L)) == 0;
    const bool last = p + 1 == n || keys[p + 1] != k;  // stable sort: last in list order
    uint32_t is = kNoPair, id = kNoPair, ds = kNoPair, dd = kNoPair;
    if (valid && last) {
        const uint32_t s = (uint32_t)(k >> g.L);
        const uint32_t d = (uint32_t)(k & ((1ull << g.L) - 1));
        if (op[pos[p]] == 0) {
            is = s;
            id = d;
        } else {
            ds = s;
            dd = d;
        }
    }
    ins_src[p] = is;
    ins_dst[p] = id;
    del_src[p] = ds;
    del_dst[p] = dd;
}

}  // namespace

void mixed_edges(gv_graph* g, const uint8_t* op, const uint32_t* src, const uint32_t* dst,
                 uint64_t n) {
    if (n == 0) return;
    if (n >= 0x3fffffffull) fail(GV_EINVAL, "batch too large");
    Ctx& c = g->ctx;
    const GraphView& v = g->v;
    const int bits = 2 * (int)v.L + 1;
    // the lists outlive the two inner batches, which carve g->scratch
    g->vscr[0].ensure(std::max<size_t>(4 * n * sizeof(uint32_t), 4), c.stream);
    uint32_t* ins_src = (uint32_t*)g->vscr[0].ptr;
    uint32_t* ins_dst = ins_src + n;
    uint32_t* del_src = ins_dst + n;
    uint32_t* del_dst = del_src + n;
    uint64_t *k0, *k1;
    uint32_t *p0, *p1, *state;
    auto carve = [&](Carver& cv) {
        k0 = cv.take<uint64_t>(n);
        k1 = cv.take<uint64_t>(n);
        p0 = cv.take<uint32_t>(n);
        p1 = cv.take<uint32_t>(n);
        state = cv.take<uint32_t>(os_words(n, bits));
    };
    {
        Carver m(nullptr);
        carve(m);
        g->scratch.ensure(m.used, c.stream);
        Carver cv(g->scratch.ptr);
        carve(cv);
    }
    zero_words(c, state, os_zero_words(n, bits));
    c.launch("mixed_pack", k_mixed_pack, div_up(n, kThreads), kThreads, v, op, src, dst, n, k0,
             p0);
    const bool flip = onesweep<uint64_t, true>(c, k0, k1, p0, p1, nullptr, n, bits, state,
                                               &v.ctr->err_wait, g->spin_limit);
    c.launch("mixed_split", k_mixed_split, div_up(n, kThreads), kThreads, v,
             (const uint64_t*)(flip ? k1 : k0), (const uint32_t*)(flip ? p1 : p0), op, n, ins_src,
             ins_dst, del_src, del_dst);
    edge_batch(g, kDelete, del_src, del_dst, n, nullptr, true);
    edge_batch(g, kInsert, ins_src, ins_dst, n, nullptr, true);
}

}  // namespace gv
