// k-means digitization with a given number of symbols (Sec. 3.2: Lloyd's
// algorithm for the vector quantization objective; the symbol count is the
// parameter C of Alg. 1).
//
// One iteration: the nearest-center assignment is jabba_encode (exact
// rounded distances, ties to the lowest symbol); a convergence count of the
// changed assignments is read back; otherwise the pieces are ordered by
// symbol with the stable radix sort (members of a symbol stay in canonical
// order) and one wavefront per symbol forms its mean: the exact integer sum
// of the lengths, and the increments added one by one in canonical order,
// the chain running lane by lane over chunks of 64 members staged in
// registers.
#include "common.h"

namespace jabba {
namespace {

__global__ void k_km_init(jabba_dict dict, int64_t *iterations) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < dict.capacity;
         c += (int64_t)gridDim.x * blockDim.x) {
        dict.center_len[c] = 0.0;
        dict.center_inc[c] = 0.0;
        dict.count[c] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *iterations = 0;
}

// changed assignments (prev <- current), and the sort pairs (symbol, index)
__global__ void k_km_changed(const int32_t *__restrict__ cur, int32_t *__restrict__ prev,
                             const int64_t *__restrict__ n_dev, int64_t n_max, unsigned long long *__restrict__ changed,
                             uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    int64_t n = *n_dev;
    n = n < 0 ? 0 : (n > n_max ? n_max : n);
    unsigned long long local = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cur[i];
        local += c != prev[i] ? 1ull : 0ull;
        prev[i] = c;
        keys[i] = (uint64_t)(uint32_t)c;
        vals[i] = (uint32_t)i;
    }
    local = (unsigned long long)wave_sum_i64((int64_t)local);
    if (lane_id() == 0 && local) atomicAdd(changed, local);
}

__global__ void k_km_zero(int64_t *__restrict__ a, int64_t n, unsigned long long *__restrict__ changed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *changed = 0;
}

// run [start, end) of every symbol in the symbol-sorted order
__global__ void k_km_runs(const uint64_t *__restrict__ k0, const uint64_t *__restrict__ k1,
                          const int32_t *__restrict__ ctl, const int64_t *__restrict__ n_dev, int64_t n_max,
                          int64_t capacity, int64_t *__restrict__ run_start, int64_t *__restrict__ run_end) {
    int64_t n = *n_dev;
    n = n < 0 ? 0 : (n > n_max ? n_max : n);
    const uint64_t *keys = ctl[0] ? k1 : k0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = keys[j];
        if (c >= (uint64_t)capacity) continue;
        if (j == 0 || keys[j - 1] != c) run_start[c] = j;
        if (j == n - 1 || keys[j + 1] != c) run_end[c] = j + 1;
    }
}

// one wavefront per symbol: mean of its members
__global__ __launch_bounds__(256) void k_km_update(const int32_t *__restrict__ len, const double *__restrict__ inc,
                                                   const uint32_t *__restrict__ v0, const uint32_t *__restrict__ v1,
                                                   const int32_t *__restrict__ ctl,
                                                   const int64_t *__restrict__ run_start,
                                                   const int64_t *__restrict__ run_end, jabba_dict dict) {
    const int lane = lane_id();
    const uint32_t *perm = ctl[0] ? v1 : v0;
    const double sl = dict.params[0], si = dict.params[1], scl = dict.params[2];
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < dict.capacity; c += waves) {
        const int64_t a = run_start[c], b = run_end[c];
        if (lane == 0) dict.count[c] = b - a;
        if (b <= a) continue;
        int64_t slen = 0;
        double sinc = 0.0;
        for (int64_t j0 = a; j0 < b; j0 += kWave) {
            const int64_t j = j0 + lane;
            int32_t l = 0;
            double it = 0.0;
            if (j < b) {
                const uint32_t i = perm[j];
                l = len[i];
                it = inc[i];
            }
            slen += wave_sum_i64((int64_t)l);
            const int cnt = (int)((b - j0) < kWave ? (b - j0) : kWave);
            for (int u = 0; u < cnt; ++u) sinc = sinc + readlane_f64(it, u);
        }
        if (lane == 0) {
            const double cnt = (double)(b - a);
            const double cl = (double)slen / cnt;
            const double ci = sinc / cnt;
            dict.center_len[c] = cl;
            dict.center_inc[c] = ci;
            dict.cx[c] = scl * (cl / sl);
            dict.cy[c] = ci / si;
        }
    }
}

struct KmWs {
    void *enc;
    size_t enc_bytes;
    int32_t *prev;
    int64_t *run_start, *run_end;
    unsigned long long *changed;
    SortBuffers sb;
    size_t bytes;
};

KmWs carve_km(void *ws, int64_t max_pieces, int64_t capacity) {
    const int64_t N = max_pieces > 0 ? max_pieces : 1;
    Carve c(ws);
    KmWs w;
    size_t eb = 0;
    jabba_encode_workspace(capacity, &eb);
    w.enc_bytes = eb;
    w.enc = c.take<char>((int64_t)eb);
    w.prev = c.take<int32_t>(N);
    w.run_start = c.take<int64_t>(2 * capacity);
    w.run_end = w.run_start + capacity;
    w.changed = c.take<unsigned long long>(1);
    sort_workspace(N, c, &w.sb);
    w.bytes = c.bytes();
    return w;
}

unsigned grid_of(int64_t n) {
    int64_t b = (n + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 8;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace
}  // namespace jabba

using namespace jabba;

extern "C" int jabba_kmeans_workspace(int64_t max_pieces, int64_t capacity, size_t *bytes) {
    if (!bytes || max_pieces < 0 || capacity < 1 || capacity > (1 << 30)) return JABBA_EINVAL;
    *bytes = carve_km(nullptr, max_pieces, capacity).bytes;
    return JABBA_OK;
}

extern "C" int jabba_kmeans(const int32_t *len, const double *inc, const int64_t *n_pieces, int64_t max_pieces,
                            int32_t max_iter, const jabba_dict *dict, int32_t *symbols, int64_t *iterations,
                            void *workspace, size_t workspace_bytes, void *stream) {
    if (!dict || !n_pieces || !iterations || max_pieces < 0 || max_iter < 1) return JABBA_EINVAL;
    if (max_pieces >= ((int64_t)1 << 31) - 1) return JABBA_EOVERFLOW;
    if (max_pieces > 0 && (!len || !inc || !symbols)) return JABBA_EINVAL;
    if (dict->capacity < 1 || dict->capacity > (1 << 30) || !dict->k || !dict->params || !dict->cx || !dict->cy ||
        !dict->center_len || !dict->center_inc || !dict->count)
        return JABBA_EINVAL;
    const KmWs w0 = carve_km(nullptr, max_pieces, dict->capacity);
    if (!workspace || workspace_bytes < w0.bytes) return JABBA_ENOMEM;
    JB_DEVICE_CHECK();
    const KmWs w = carve_km(workspace, max_pieces, dict->capacity);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = max_pieces > 0 ? max_pieces : 1;
    JB_LAUNCH(k_km_init, dim3(grid_of(dict->capacity)), dim3(256), 0, st, *dict, iterations);
    JB_LAUNCH_CHECK();
    int64_t done = 0;
    for (int32_t it = 0; it < max_iter; ++it) {
        int rc = jabba_encode(len, inc, n_pieces, max_pieces, dict, symbols, w.enc, w.enc_bytes, stream);
        if (rc) return rc;
        JB_LAUNCH(k_km_zero, dim3(grid_of(2 * dict->capacity)), dim3(256), 0, st, w.run_start, 2 * dict->capacity,
                  w.changed);
        JB_LAUNCH_CHECK();
        rc = radix_sort_init(w.sb, st);
        if (rc) return rc;
        JB_LAUNCH(k_km_changed, dim3(grid_of(N)), dim3(256), 0, st, symbols, w.prev, n_pieces, max_pieces, w.changed,
                  w.sb.keys[0], w.sb.vals[0]);
        JB_LAUNCH_CHECK();
        done = it + 1;
        if (it > 0) {
            unsigned long long changed = 0;
            JB_HIP(hipMemcpyAsync(&changed, w.changed, sizeof(changed), hipMemcpyDeviceToHost, st));
            JB_HIP(hipStreamSynchronize(st));
            if (changed == 0) break;
        }
        rc = radix_global_hist(w.sb, n_pieces, N, st);
        if (rc) return rc;
        rc = radix_sort_pairs(w.sb, n_pieces, N, st, "kmeans");
        if (rc) return rc;
        JB_LAUNCH(k_km_runs, dim3(grid_of(N)), dim3(256), 0, st, w.sb.keys[0], w.sb.keys[1], w.sb.ctl, n_pieces, N,
                  dict->capacity, w.run_start, w.run_end);
        JB_LAUNCH_CHECK();
        JB_LAUNCH(k_km_update, dim3(grid_of(dict->capacity * kWave)), dim3(256), 0, st, len, inc, w.sb.vals[0],
                  w.sb.vals[1], w.sb.ctl, w.run_start, w.run_end, *dict);
        JB_LAUNCH_CHECK();
    }
    JB_HIP(hipMemcpyAsync(iterations, &done, sizeof(done), hipMemcpyHostToDevice, st));
    JB_HIP(hipStreamSynchronize(st));
    return JABBA_OK;
}
