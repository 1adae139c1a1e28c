// gv_batched.hip -- the batched form: a sequence of update batches of uneven
// sizes applied in order (Sec. 4.3), either one launch sequence per batch or
// recorded once into a HIP graph and launched as a whole.
//
// Recording needs every size known on the host: the batch scratch is sized
// for the largest batch before recording, vertex inserts keep the dictionary
// as it is, and vertex deletes size their buffers for a full pool (every
// stored edge holds a pool slot) instead of reading the edge count back.
//
// With coalescing on (gv_tuning), every run of consecutive edge batches up
// to the next vertex batch is copied into one list of (op, src, dst) entries
// (one kernel per up to 16 batches) and applied as a mixed list: the same
// result as the batches in order, since each pair's last entry decides, with
// one grouping sort per run instead of one per batch.
#include <algorithm>
#include <cstring>
#include <new>

#include "gv_graph.h"
#include "gv_prim.h"

using namespace gv;

struct gv_plan {
    gv_graph* g = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // generations of the buffers the recorded kernels point into; a launch
    // checks that none was reallocated since
    uint64_t scratch_gen = 0;
    uint64_t vscr_gen[3] = {0, 0, 0};
    uint64_t table_gen = 0;
    uint64_t cscr_gen = 0;
    uint64_t ovscr_gen = 0;     // the sort overlap's second batch buffer
    uint64_t mix_gen[2] = {0, 0};  // the sort overlap's mixed-list buffers
    uint64_t insert_pairs = 0;  // pairs the plan's inserts add to the host-side edge bound
};

namespace {

struct CopyDesc {
    const uint32_t* a;
    const uint32_t* b;
    unsigned long long n, off;
    uint32_t kind, pad;
};
constexpr int kCopyDescs = 16;
struct CopyArgs {
    CopyDesc d[kCopyDescs];
};

// batch blockIdx.y of the group goes to entries [off, off + n) of the run
__global__ __launch_bounds__(kThreads) void k_coalesce(CopyArgs args, uint8_t* op, uint32_t* src,
                                                       uint32_t* dst) {
    const CopyDesc D = args.d[blockIdx.y];
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < D.n; i += stride) {
        src[D.off + i] = D.a[i];
        dst[D.off + i] = D.b[i];
        op[D.off + i] = (uint8_t)D.kind;
    }
}

bool is_edge(const gv_op& op) {
    return op.kind == GV_OP_INSERT_EDGES || op.kind == GV_OP_DELETE_EDGES;
}

// Longest run coalesced when the tuning sets no limit (a mixed list's sort
// takes fewer than 2^30 entries).
constexpr uint64_t kRunCap = 1ull << 28;

// End of the run of edge batches that starts at i (batches of no pairs do
// not end a run), within max_pairs pairs (0: kRunCap; a run takes at least
// its first batch).
uint64_t run_end(const gv_op* ops, uint64_t n_ops, uint64_t i, uint64_t max_pairs,
                 uint64_t* pairs) {
    const uint64_t cap = max_pairs ? std::min(max_pairs, kRunCap) : kRunCap;
    uint64_t j = i, tot = 0;
    while (j < n_ops && (is_edge(ops[j]) || ops[j].n == 0)) {
        if (j > i && tot + ops[j].n > cap) break;
        tot += is_edge(ops[j]) ? ops[j].n : 0;
        ++j;
    }
    *pairs = tot;
    return j;
}

// copies the edge batches of ops[i, j) into one list on the context's stream
void gather_run(Ctx& c, const gv_op* ops, uint64_t i, uint64_t j, uint8_t* op, uint32_t* src,
                uint32_t* dst) {
    CopyArgs args{};
    uint32_t cnt = 0;
    uint64_t off = 0, big = 0;
    auto flush = [&] {
        if (!cnt) return;
        const uint64_t gx = std::min<uint64_t>(std::max<uint64_t>(div_up(big, kThreads), 1), 1024);
        hipLaunchKernelGGL(k_coalesce, dim3((uint32_t)gx, cnt), dim3(kThreads), 0, c.stream, args,
                           op, src, dst);
        hip_check(hipGetLastError(), "coalesce");
        cnt = 0;
        big = 0;
    };
    for (uint64_t k = i; k < j; ++k) {
        if (!is_edge(ops[k]) || !ops[k].n) continue;
        args.d[cnt] = CopyDesc{ops[k].a, ops[k].b, ops[k].n, off,
                               ops[k].kind == GV_OP_INSERT_EDGES ? 0u : 1u, 0u};
        off += ops[k].n;
        big = std::max<uint64_t>(big, ops[k].n);
        if (++cnt == kCopyDescs) flush();
    }
    flush();
}

// Lists longer than one sort tile have their gather and sort overlapped
// (with the overlap on); a list of one tile is sorted by one kernel.
bool side_run(const gv_graph* g, uint64_t pairs) { return g->tune.overlap && pairs > kOsTile; }

// apply a run of edge batches as one mixed list; `fenced`: a list of this
// call went to the side stream already
void run_coalesced(gv_graph* g, const gv_op* ops, uint64_t i, uint64_t j, uint64_t pairs,
                   bool& fenced) {
    Ctx& c = g->ctx;
    if (side_run(g, pairs)) {
        mixed_edges_side(g, pairs, !fenced,
                         [&](Ctx& sc, uint8_t* op, uint32_t* src, uint32_t* dst) {
                             gather_run(sc, ops, i, j, op, src, dst);
                         });
        fenced = true;
        return;
    }
    g->cscr.ensure(std::max<size_t>(pairs * 9, 4), c.stream);
    uint32_t* src = (uint32_t*)g->cscr.ptr;
    uint32_t* dst = src + pairs;
    uint8_t* op = (uint8_t*)(dst + pairs);
    gather_run(c, ops, i, j, op, src, dst);
    mixed_edges(g, op, src, dst, pairs);
}

// ops[0, n_ops) in order, coalescing runs of edge batches when the graph's
// tuning says so
void run_ops(gv_graph* g, const gv_op* ops, uint64_t n_ops, bool recorded, uint64_t bound);

int check_ops(const gv_op* ops, uint64_t n_ops) {
    if (n_ops && !ops) return GV_EINVAL;
    for (uint64_t i = 0; i < n_ops; ++i) {
        const gv_op& op = ops[i];
        if (op.kind > GV_OP_DELETE_VERTICES) return GV_EINVAL;
        if (op.flags & ~(uint32_t)GV_OP_FIT_TABLE) return GV_EINVAL;
        if (op.flags && op.kind != GV_OP_INSERT_VERTICES) return GV_EINVAL;
        if (op.n && !op.a) return GV_EINVAL;
        if (op.n && op.kind <= GV_OP_DELETE_EDGES && !op.b) return GV_EINVAL;
        if (op.n >= 0x3fffffffull) return GV_EINVAL;
    }
    return GV_OK;
}

// one op through the single-batch paths; `bound` > 0 records a vertex
// delete without reading the edge count back
void run_op(gv_graph* g, const gv_op& op, bool recorded, uint64_t bound) {
    if (op.n == 0) return;
    switch (op.kind) {
        case GV_OP_INSERT_EDGES:
            edge_batch(g, kInsert, op.a, op.b, op.n, nullptr, true);
            break;
        case GV_OP_DELETE_EDGES:
            edge_batch(g, kDelete, op.a, op.b, op.n, nullptr, true);
            break;
        case GV_OP_INSERT_VERTICES:
            vertex_insert(g, op.a, op.n, nullptr, recorded || (op.flags & GV_OP_FIT_TABLE));
            break;
        default:
            vertex_delete(g, op.a, op.n, nullptr, recorded ? bound : 0);
            break;
    }
}

template <typename F>
int guarded_call(gv_graph* g, F&& f) {
    if (!g) return GV_EINVAL;
    if (g->dead) return GV_EDEVICE;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != g->device && hipSetDevice(g->device) != hipSuccess) return GV_EDEVICE;
    int rc = GV_OK;
    try {
        f();
    } catch (const Error& e) {
        if (e.code == GV_EDEVICE) g->dead = true;
        rc = e.code;
    } catch (const std::bad_alloc&) {
        rc = GV_ENOMEM;
    } catch (...) {
        g->dead = true;
        rc = GV_EDEVICE;
    }
    if (prev >= 0 && prev != g->device) hipSetDevice(prev);
    return rc;
}

void run_ops(gv_graph* g, const gv_op* ops, uint64_t n_ops, bool recorded, uint64_t bound) {
    uint64_t i = 0;
    bool fenced = false;
    while (i < n_ops) {
        if (g->tune.coalesce && is_edge(ops[i])) {
            uint64_t pairs = 0;
            const uint64_t j = run_end(ops, n_ops, i, g->tune.max_run_pairs, &pairs);
            uint64_t batches = 0;
            for (uint64_t k = i; k < j; ++k) batches += ops[k].n ? 1 : 0;
            if (batches > 1) {
                run_coalesced(g, ops, i, j, pairs, fenced);
            } else {
                for (uint64_t k = i; k < j; ++k) run_op(g, ops[k], recorded, bound);
            }
            i = j;
            continue;
        }
        run_op(g, ops[i], recorded, bound);
        ++i;
    }
}

}  // namespace

extern "C" {

int gv_apply_ops(gv_graph* g, const gv_op* ops, uint64_t n_ops) {
    if (!g) return GV_EINVAL;
    const int rc = check_ops(ops, n_ops);
    if (rc != GV_OK) return rc;
    return guarded_call(g, [&] { run_ops(g, ops, n_ops, false, 0); });
}

int gv_plan_create(gv_graph* g, const gv_op* ops, uint64_t n_ops, gv_plan** out) {
    if (!out) return GV_EINVAL;
    *out = nullptr;
    if (!g) return GV_EINVAL;
    int rc = check_ops(ops, n_ops);
    if (rc != GV_OK) return rc;
    gv_plan* p = new (std::nothrow) gv_plan();
    if (!p) return GV_ENOMEM;
    rc = guarded_call(g, [&] {
        Ctx& c = g->ctx;
        // every stored edge holds a pool slot
        const uint64_t bound = std::max<uint64_t>(g->v.cap_blocks * (uint64_t)g->v.B, 1);
        // size every buffer for the largest op (and run)
        size_t sc = 0, vs[3] = {0, 0, 0}, csz = 0, msz = 0;
        for (uint64_t i = 0; g->tune.coalesce && i < n_ops;) {
            if (!is_edge(ops[i])) {
                ++i;
                continue;
            }
            uint64_t pairs = 0;
            const uint64_t j = run_end(ops, n_ops, i, g->tune.max_run_pairs, &pairs);
            size_t mb[2];
            mixed_bytes(g, std::max<uint64_t>(pairs, 1), mb);
            sc = std::max(sc, mb[0]);
            vs[0] = std::max(vs[0], mb[1]);
            if (side_run(g, pairs)) msz = std::max(msz, mixed_side_bytes(g, pairs));
            else csz = std::max<size_t>(csz, pairs * 9);
            i = j;
        }
        for (uint64_t i = 0; i < n_ops; ++i) {
            const gv_op& op = ops[i];
            if (!op.n) continue;
            if (op.kind == GV_OP_INSERT_EDGES || op.kind == GV_OP_DELETE_EDGES) {
                sc = std::max(sc, edge_batch_bytes(g, op.kind == GV_OP_INSERT_EDGES ? kInsert
                                                                                  : kDelete,
                                                   op.n));
            } else {
                size_t sz[4];
                vertex_batch_bytes(g, op.kind == GV_OP_DELETE_VERTICES, op.n, bound, sz);
                sc = std::max(sc, sz[0]);
                for (int k = 0; k < 3; ++k) vs[k] = std::max(vs[k], sz[k + 1]);
            }
        }
        g->scratch.ensure(std::max<size_t>(sc, 4), c.stream);
        for (int k = 0; k < 3; ++k) g->vscr[k].ensure(std::max<size_t>(vs[k], 4), c.stream);
        g->cscr.ensure(std::max<size_t>(csz, 4), c.stream);
        if (g->tune.overlap) {
            // edge batches alternate between the two batch buffers
            g->ov.scr.ensure(std::max<size_t>(sc, 4), c.stream);
            overlap_open(g);
            // and mixed lists between the two mixed-list buffers
            if (msz) {
                hip_check(hipStreamSynchronize(g->ov.stream), "hipStreamSynchronize");
                for (int k = 0; k < 2; ++k) g->ov.mix[k].ensure(msz, c.stream);
            }
        }
        hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
        edge_batch_warm(g);
        vertex_batch_warm();
        // record
        hipStream_t cs = nullptr;
        hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        const hipStream_t saved = c.stream;
        const bool saved_prof = c.prof;
        c.stream = cs;
        c.prof = false;
        hipGraph_t graph = nullptr;
        try {
            hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture");
            // nothing runs while recording: the inserts add to the host-side
            // edge bound at each launch instead
            const uint64_t bound0 = g->edge_bound_host;
            run_ops(g, ops, n_ops, true, bound);
            p->insert_pairs = g->edge_bound_host - bound0;
            g->edge_bound_host = bound0;
            hip_check(hipStreamEndCapture(cs, &graph), "hipStreamEndCapture");
        } catch (...) {
            hipGraph_t dropped = nullptr;
            hipStreamEndCapture(cs, &dropped);
            if (dropped) hipGraphDestroy(dropped);
            c.stream = saved;
            c.prof = saved_prof;
            hipStreamDestroy(cs);
            throw;
        }
        c.stream = saved;
        c.prof = saved_prof;
        hipStreamDestroy(cs);
        p->graph = graph;
        hip_check(hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        p->g = g;
        p->scratch_gen = g->scratch.gen;
        for (int k = 0; k < 3; ++k) p->vscr_gen[k] = g->vscr[k].gen;
        p->table_gen = g->table_gen;
        p->cscr_gen = g->cscr.gen;
        p->ovscr_gen = g->ov.scr.gen;
        for (int k = 0; k < 2; ++k) p->mix_gen[k] = g->ov.mix[k].gen;
    });
    if (rc != GV_OK) {
        gv_plan_destroy(p);
        return rc;
    }
    *out = p;
    return GV_OK;
}

int gv_plan_launch(gv_plan* p) {
    if (!p || !p->g || !p->exec) return GV_EINVAL;
    gv_graph* g = p->g;
    return guarded_call(g, [&] {
        bool same = g->scratch.gen == p->scratch_gen && g->table_gen == p->table_gen &&
                    g->cscr.gen == p->cscr_gen && g->ov.scr.gen == p->ovscr_gen;
        for (int k = 0; k < 3; ++k) same = same && g->vscr[k].gen == p->vscr_gen[k];
        for (int k = 0; k < 2; ++k) same = same && g->ov.mix[k].gen == p->mix_gen[k];
        if (!same) fail(GV_EINVAL, "graph buffers moved since the plan was created");
        hip_check(hipGraphLaunch(p->exec, g->ctx.stream), "hipGraphLaunch");
        ++g->ctx.seq;
        g->edge_bound_host += p->insert_pairs;
    });
}

void gv_plan_destroy(gv_plan* p) {
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    delete p;
}

}  // extern "C"
