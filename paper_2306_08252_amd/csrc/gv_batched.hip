// gv_batched.hip -- the batched form: a sequence of update batches of uneven
// sizes applied in order (Sec. 4.3), either one launch sequence per batch or
// recorded once into a HIP graph and launched as a whole.
//
// Recording needs every size known on the host: the batch scratch is sized
// for the largest batch before recording, vertex inserts keep the dictionary
// as it is, and vertex deletes size their buffers for a full pool (every
// stored edge holds a pool slot) instead of reading the edge count back.
#include <algorithm>
#include <cstring>
#include <new>

#include "gv_graph.h"

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
};

namespace {

int check_ops(const gv_op* ops, uint64_t n_ops) {
    if (n_ops && !ops) return GV_EINVAL;
    for (uint64_t i = 0; i < n_ops; ++i) {
        const gv_op& op = ops[i];
        if (op.kind > GV_OP_DELETE_VERTICES) return GV_EINVAL;
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
            vertex_insert(g, op.a, op.n, nullptr, recorded);
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

}  // namespace

extern "C" {

int gv_apply_ops(gv_graph* g, const gv_op* ops, uint64_t n_ops) {
    if (!g) return GV_EINVAL;
    const int rc = check_ops(ops, n_ops);
    if (rc != GV_OK) return rc;
    return guarded_call(g, [&] {
        for (uint64_t i = 0; i < n_ops; ++i) run_op(g, ops[i], false, 0);
    });
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
        // size every buffer for the largest op
        size_t sc = 0, vs[3] = {0, 0, 0};
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
        hip_check(hipStreamSynchronize(c.stream), "hipStreamSynchronize");
        edge_batch_warm();
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
            for (uint64_t i = 0; i < n_ops; ++i) run_op(g, ops[i], true, bound);
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
        bool same = g->scratch.gen == p->scratch_gen && g->table_gen == p->table_gen;
        for (int k = 0; k < 3; ++k) same = same && g->vscr[k].gen == p->vscr_gen[k];
        if (!same) fail(GV_EINVAL, "graph buffers moved since the plan was created");
        hip_check(hipGraphLaunch(p->exec, g->ctx.stream), "hipGraphLaunch");
    });
}

void gv_plan_destroy(gv_plan* p) {
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    delete p;
}

}  // extern "C"
