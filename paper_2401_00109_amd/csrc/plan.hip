// Batched plan: the whole compress + digitize path captured once into a HIP
// graph and replayed with one graph launch per batch.
//
// Every kernel of the path sizes its grid from host upper bounds and reads
// the live counts (domains, pieces, starting points, symbols) from device
// memory, clears its counters with fill kernels instead of memsets, and
// chooses ping-pong buffers from device-side control words; none of them
// synchronises the host.  That is what makes the capture valid and lets a
// replay run back to back with no host round trip.
#include "common.h"

struct jabba_plan {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" int jabba_plan_create(const jabba_plan_desc *d, jabba_plan **out) {
    if (!d || !out) return JABBA_EINVAL;
    *out = nullptr;
    hipStream_t st;
    JB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    int rc = JABBA_OK;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(st);  // the capture error is the one reported
        return JABBA_EHIP;
    }
    rc = jabba_compress(d->values, d->series_off, d->n_series, d->total_points, d->D, d->tol, d->max_len, &d->tuning,
                        d->len, d->inc, d->piece_off, d->n_pieces, d->compress_ws, d->compress_ws_bytes, st);
    if (rc == JABBA_OK)
        rc = jabba_digitize(d->len, d->inc, d->n_pieces, d->max_pieces, d->alpha, d->scl, d->B, &d->tuning,
                            d->symbols, &d->dict, d->digitize_ws, d->digitize_ws_bytes, st);
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (rc == JABBA_OK && ce != hipSuccess) rc = JABBA_EHIP;
    jabba_plan *p = nullptr;
    if (rc == JABBA_OK) {
        p = new jabba_plan{graph, nullptr};
        if (hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = JABBA_EHIP;
    }
    if (hipStreamDestroy(st) != hipSuccess && rc == JABBA_OK) rc = JABBA_EHIP;
    if (rc != JABBA_OK) {  // cleanup after a failure; the first error is the one reported
        if (p && p->exec) (void)hipGraphExecDestroy(p->exec);
        if (graph) (void)hipGraphDestroy(graph);
        delete p;
        p = nullptr;
    }
    *out = p;
    return rc;
}

extern "C" int jabba_plan_run(jabba_plan *plan, void *stream) {
    if (!plan || !plan->exec) return JABBA_EINVAL;
    JB_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return JABBA_OK;
}

extern "C" int jabba_plan_destroy(jabba_plan *plan) {
    if (!plan) return JABBA_OK;
    const hipError_t e1 = plan->exec ? hipGraphExecDestroy(plan->exec) : hipSuccess;
    const hipError_t e2 = plan->graph ? hipGraphDestroy(plan->graph) : hipSuccess;
    delete plan;
    return e1 == hipSuccess && e2 == hipSuccess ? JABBA_OK : JABBA_EHIP;
}
