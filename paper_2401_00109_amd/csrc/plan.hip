// Batched plan: the whole compress + digitize path captured once into a HIP
// graph and replayed with one graph launch per batch.
//
// Every kernel of the path sizes its grid from host upper bounds and reads
// the live counts (domains, pieces, starting points, symbols) from device
// memory, clears its counters with fill kernels instead of memsets, and
// chooses ping-pong buffers from device-side control words; none of them
// synchronises the host.  That is what makes the capture valid and lets a
// replay run back to back with no host round trip.
//
// Without a caller tuning the plan picks its launch shapes itself before the
// capture: it times the compression over a grid of lane widths, wavefronts
// per workgroup and workgroups per compute unit, then the digitization over
// Stage I wavefronts per workgroup, on the plan's own buffers, and keeps the
// fastest.  Each timed variant's output is compared on the device with the
// default launch's (pieces, offsets and count; symbols), when the other
// workspace can hold the reference copy, and a variant that differs is
// never chosen.
#include "common.h"

struct jabba_plan {
    hipGraph_t graph;
    hipGraphExec_t exec;
    jabba_tuning tuning;
};

namespace jabba {
namespace {

// flag[0] |= 1 where a[i] != b[i] for i < n (n from the device when n_dev)
__global__ void k_differs(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b, const int64_t *n_dev,
                          int64_t words_per_item, int64_t n_max, int32_t *__restrict__ flag) {
    int64_t n = n_dev ? *n_dev : n_max;
    n = n < 0 ? 0 : (n > n_max ? n_max : n);
    const int64_t words = n * words_per_item;
    bool diff = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        diff |= a[i] != b[i];
    if (__ballot(diff) && lane_id() == 0) atomicOr(flag, 1);
}

int differs(const void *a, const void *b, const int64_t *n_dev, int64_t words_per_item, int64_t n_max, int32_t *flag,
            hipStream_t st) {
    if (n_max <= 0) return JABBA_OK;
    int64_t blocks = (n_max * words_per_item + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    JB_LAUNCH(k_differs, dim3((unsigned)blocks), dim3(256), 0, st, (const uint32_t *)a, (const uint32_t *)b, n_dev,
              words_per_item, n_max, flag);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

int run_compress(const jabba_plan_desc *d, const jabba_tuning *t, hipStream_t st) {
    return jabba_compress(d->values, d->series_off, d->n_series, d->total_points, d->D, d->tol, d->max_len, t, d->len,
                          d->inc, d->piece_off, d->n_pieces, d->compress_ws, d->compress_ws_bytes, st);
}

int run_digitize(const jabba_plan_desc *d, const jabba_tuning *t, hipStream_t st) {
    return jabba_digitize(d->len, d->inc, d->n_pieces, d->max_pieces, d->alpha, d->scl, d->B, t, d->symbols, &d->dict,
                          d->digitize_ws, d->digitize_ws_bytes, st);
}

// best of `reps` timed runs of f (ms); a negative status when a run fails
template <class F>
int time_best(hipStream_t st, Timer &tm, int reps, F &&f, float *best) {
    *best = 3.0e38f;
    for (int r = 0; r < reps; ++r) {
        JB_HIP(hipEventRecord(tm.a, st));
        const int rc = f();
        if (rc) return rc;
        JB_HIP(hipEventRecord(tm.b, st));
        JB_HIP(hipEventSynchronize(tm.b));
        float ms = 0.0f;
        JB_HIP(hipEventElapsedTime(&ms, tm.a, tm.b));
        if (ms < *best) *best = ms;
    }
    return JABBA_OK;
}

// reads and clears the difference flag
int take_flag(int32_t *flag, hipStream_t st, bool *set) {
    int32_t h = 0;
    JB_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st));
    JB_HIP(hipStreamSynchronize(st));
    *set = h != 0;
    return fill_i32(flag, 0, 1, st);
}

constexpr int kTuneReps = 2;
constexpr int kLanes[] = {1, 2, 4};
constexpr int kWavesPerBlock[] = {1, 2, 4};
constexpr int kBlocksPerCu[] = {2, 4, 8};
constexpr int kStage1Waves[] = {1, 2, 4};

int autotune(const jabba_plan_desc *d, hipStream_t st, jabba_tuning *out) {
    *out = jabba_tuning{};
    Timer tm;
    JB_HIP(hipEventCreate(&tm.a));
    JB_HIP(hipEventCreate(&tm.b));
    const int64_t mp = d->max_pieces;
    const int64_t ns1 = d->n_series + 1;

    // compression: reference pieces (default launch) copied into the digitize
    // workspace, which is free until the digitization runs
    Carve rc_c(d->digitize_ws);
    (void)rc_c.take<int32_t>(64);  // the workspace's status words stay untouched
    int32_t *flag = rc_c.take<int32_t>(1);
    int64_t *ref_n = rc_c.take<int64_t>(1);
    int64_t *ref_off = rc_c.take<int64_t>((size_t)ns1);
    int32_t *ref_len = rc_c.take<int32_t>((size_t)mp);
    double *ref_inc = rc_c.take<double>((size_t)mp);
    const bool check_c = rc_c.bytes() <= d->digitize_ws_bytes;
    int rc = run_compress(d, nullptr, st);
    if (rc) return rc;
    if (check_c) {
        JB_HIP(hipMemcpyAsync(ref_n, d->n_pieces, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
        JB_HIP(hipMemcpyAsync(ref_off, d->piece_off, (size_t)ns1 * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
        JB_HIP(hipMemcpyAsync(ref_len, d->len, (size_t)mp * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        JB_HIP(hipMemcpyAsync(ref_inc, d->inc, (size_t)mp * sizeof(double), hipMemcpyDeviceToDevice, st));
        rc = fill_i32(flag, 0, 1, st);
        if (rc) return rc;
    }
    float best_ms = 3.0e38f;
    for (int W : kLanes)
        for (int wpb : kWavesPerBlock)
            for (int bpc : kBlocksPerCu) {
                jabba_tuning t{};
                t.lanes_per_domain = W;
                t.waves_per_block = wpb;
                t.blocks_per_cu = bpc;
                float ms = 0.0f;
                rc = time_best(st, tm, kTuneReps, [&] { return run_compress(d, &t, st); }, &ms);
                if (rc) return rc;
                bool bad = false;
                if (check_c) {
                    if ((rc = differs(ref_n, d->n_pieces, nullptr, 2, 1, flag, st)) ||
                        (rc = differs(ref_off, d->piece_off, nullptr, 2, ns1, flag, st)) ||
                        (rc = differs(ref_len, d->len, ref_n, 1, mp, flag, st)) ||
                        (rc = differs(ref_inc, d->inc, ref_n, 2, mp, flag, st)) || (rc = take_flag(flag, st, &bad)))
                        return rc;
                }
                if (!bad && ms < best_ms) {
                    best_ms = ms;
                    out->lanes_per_domain = W;
                    out->waves_per_block = wpb;
                    out->blocks_per_cu = bpc;
                }
            }
    // the plan's buffers hold the default launch's pieces again
    rc = run_compress(d, nullptr, st);
    if (rc) return rc;

    // digitization: reference symbols (default launch) in the compression
    // workspace, which the digitization does not touch
    Carve rc_d(d->compress_ws);
    (void)rc_d.take<int32_t>(64);
    int32_t *flag2 = rc_d.take<int32_t>(1);
    int32_t *ref_sym = rc_d.take<int32_t>((size_t)mp);
    const bool check_d = rc_d.bytes() <= d->compress_ws_bytes;
    rc = run_digitize(d, nullptr, st);
    if (rc) return rc;
    if (check_d) {
        JB_HIP(hipMemcpyAsync(ref_sym, d->symbols, (size_t)mp * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        rc = fill_i32(flag2, 0, 1, st);
        if (rc) return rc;
    }
    best_ms = 3.0e38f;
    for (int s1 : kStage1Waves) {
        jabba_tuning t = *out;
        t.stage1_waves = s1;
        float ms = 0.0f;
        rc = time_best(st, tm, kTuneReps, [&] { return run_digitize(d, &t, st); }, &ms);
        if (rc) return rc;
        bool bad = false;
        if (check_d) {
            if ((rc = differs(ref_sym, d->symbols, d->n_pieces, 1, mp, flag2, st)) || (rc = take_flag(flag2, st, &bad)))
                return rc;
        }
        if (!bad && ms < best_ms) {
            best_ms = ms;
            out->stage1_waves = s1;
        }
    }
    JB_HIP(hipStreamSynchronize(st));
    return JABBA_OK;
}

}  // namespace
}  // namespace jabba

extern "C" int jabba_plan_create(const jabba_plan_desc *d, jabba_plan **out) {
    if (!out) return JABBA_EINVAL;
    *out = nullptr;
    if (!d) return JABBA_EINVAL;
    JB_DEVICE_CHECK();
    hipStream_t st;
    JB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    jabba_tuning chosen{};
    int rc = JABBA_OK;
    if (d->tuning)
        chosen = *d->tuning;
    else
        rc = jabba::autotune(d, st, &chosen);
    if (rc != JABBA_OK) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
        return rc;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(st);  // the capture error is the one reported
        return JABBA_EHIP;
    }
    rc = jabba::run_compress(d, &chosen, st);
    if (rc == JABBA_OK) rc = jabba::run_digitize(d, &chosen, st);
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (rc == JABBA_OK && ce != hipSuccess) rc = JABBA_EHIP;
    jabba_plan *p = nullptr;
    if (rc == JABBA_OK) {
        p = new jabba_plan{graph, nullptr, chosen};
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

extern "C" int jabba_plan_tuning(const jabba_plan *plan, jabba_tuning *tuning) {
    if (!plan || !tuning) return JABBA_EINVAL;
    *tuning = plan->tuning;
    return JABBA_OK;
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
