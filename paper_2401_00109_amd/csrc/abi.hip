// Library-wide entry points of the C ABI: version, status text and the
// per-device facts the launchers size their grids with.
#include "common.h"

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace jabba {

namespace {
struct Pending {
    hipEvent_t a, b;
    int launches;
};
struct TimingSlot {
    double ms = 0.0;
    int64_t launches = 0;
    std::vector<Pending> pending;
};
std::atomic<bool> g_timing{false};
std::mutex g_tmu;
std::map<std::string, TimingSlot> g_slots;
std::vector<hipEvent_t> g_pool;

hipEvent_t ev_get() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

std::string clean_name(const char *n) {
    std::string s(n);
    std::string o;
    for (char ch : s)
        if (ch != '(' && ch != ')' && ch != ' ') o += ch;
    const size_t c = o.rfind("::");
    return c == std::string::npos ? o : o.substr(c + 2);
}

void settle(TimingSlot &t) {
    for (auto &pr : t.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(pr.b) == hipSuccess && hipEventElapsedTime(&ms, pr.a, pr.b) == hipSuccess) {
            t.ms += ms;
            t.launches += pr.launches;
        }
        g_pool.push_back(pr.a);
        g_pool.push_back(pr.b);
    }
    t.pending.clear();
}
}  // namespace

KernelTimer::KernelTimer(const char *name, hipStream_t st, int launches)
    : name_(name), st_(st), a_(nullptr), launches_(launches) {
    if (!g_timing.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> g(g_tmu);
    hipEvent_t e = ev_get();
    if (e && hipEventRecord(e, st) == hipSuccess) a_ = e;
}

KernelTimer::~KernelTimer() {
    if (!a_) return;
    std::lock_guard<std::mutex> g(g_tmu);
    hipEvent_t e = ev_get();
    if (e && hipEventRecord(e, st_) == hipSuccess)
        g_slots[clean_name(name_)].pending.push_back(Pending{(hipEvent_t)a_, e, launches_});
    else
        g_pool.push_back((hipEvent_t)a_);
}

int device_cu_count() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

int device_check() {
    static int cache[64] = {0};  // 0 unknown, 1 gfx950, 2 another device
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return JABBA_ENODEV;
    if (!cache[dev]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return JABBA_ENODEV;
        const char *a = prop.gcnArchName;
        cache[dev] = (a[0] == 'g' && a[1] == 'f' && a[2] == 'x' && a[3] == '9' && a[4] == '5' && a[5] == '0' &&
                      (a[6] == 0 || a[6] == ':')) ? 1 : 2;
    }
    return cache[dev] == 1 ? JABBA_OK : JABBA_ENODEV;
}

namespace {
__global__ void k_fp64_selftest(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ q,
                                double *__restrict__ r, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        q[i] = a[i] / b[i];
        r[i] = __dsqrt_rn(a[i]);
    }
}
}  // namespace

}  // namespace jabba

extern "C" int jabba_fp64_selftest(const double *a, const double *b, double *quot, double *root, int64_t n,
                                   void *stream) {
    if (n < 0 || (n > 0 && (!a || !b || !quot || !root))) return JABBA_EINVAL;
    if (n == 0) return JABBA_OK;
    JB_DEVICE_CHECK();
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    JB_LAUNCH(jabba::k_fp64_selftest, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a, b, quot,
                       root, n);
    JB_LAUNCH_CHECK();
    return JABBA_OK;
}

extern "C" int jabba_timing_enable(int enable) {
    std::lock_guard<std::mutex> g(jabba::g_tmu);
    for (auto &kv : jabba::g_slots) jabba::settle(kv.second);
    if (enable) jabba::g_slots.clear();
    jabba::g_timing.store(enable != 0);
    return JABBA_OK;
}

extern "C" int jabba_timing_get(const char *name, double *total_ms, int64_t *launches) {
    if (!name || !total_ms || !launches) return JABBA_EINVAL;
    std::lock_guard<std::mutex> g(jabba::g_tmu);
    auto it = jabba::g_slots.find(name);
    if (it == jabba::g_slots.end()) {
        *total_ms = 0.0;
        *launches = 0;
        return JABBA_OK;
    }
    jabba::settle(it->second);
    *total_ms = it->second.ms;
    *launches = it->second.launches;
    return JABBA_OK;
}

extern "C" int jabba_timing_names(char *buf, size_t buf_len) {
    if (!buf || buf_len == 0) return JABBA_EINVAL;
    std::lock_guard<std::mutex> g(jabba::g_tmu);
    std::string all;
    for (auto &kv : jabba::g_slots) {
        if (!all.empty()) all += ",";
        all += kv.first;
    }
    size_t n = all.size() < buf_len - 1 ? all.size() : buf_len - 1;
    for (size_t i = 0; i < n; ++i) buf[i] = all[i];
    buf[n] = 0;
    return JABBA_OK;
}

extern "C" int jabba_abi_version(void) { return JABBA_ABI_VERSION; }

extern "C" const char *jabba_status_str(int status) {
    switch (status) {
        case JABBA_OK: return "ok";
        case JABBA_EINVAL: return "invalid argument";
        case JABBA_ENOMEM: return "workspace too small";
        case JABBA_EHIP: return "HIP runtime error";
        case JABBA_ECAPACITY: return "dictionary capacity exceeded";
        case JABBA_ENONFINITE: return "non-finite input value";
        case JABBA_EOVERFLOW: return "count overflow";
        case JABBA_ENODEV: return "no gfx950 device";
        case JABBA_ELIMIT: return "size above the fixed maximum of an allocation-free call";
        default: return "unknown status";
    }
}
