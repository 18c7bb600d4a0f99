// Library-wide entry points of the C ABI: version, status text and the
// per-device facts the launchers size their grids with.
#include "common.h"

namespace jabba {

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
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(jabba::k_fp64_selftest, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a, b, quot,
                       root, n);
    JB_LAUNCH_CHECK();
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
        default: return "unknown status";
    }
}
