// lbm_util.hip -- status strings, thread-local error text and small helpers.
#include <hip/hip_runtime.h>

#include <string>

#include "lbm_internal.h"

namespace lbm {

namespace {
thread_local std::string g_last_error;
}

lbm_status set_error(lbm_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

lbm_status hip_check(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EDEVICE;
}

int device_cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

}  // namespace lbm

extern "C" const char *lbm_status_str(lbm_status s)
{
    switch (s) {
    case LBM_OK: return "LBM_OK";
    case LBM_EINVAL: return "LBM_EINVAL: invalid argument";
    case LBM_EDEVICE: return "LBM_EDEVICE: HIP call failed";
    case LBM_ENOTCONV: return "LBM_ENOTCONV: not converged within the step cap";
    case LBM_ENONFINITE: return "LBM_ENONFINITE: non-finite mean velocity";
    case LBM_EWORKSPACE: return "LBM_EWORKSPACE: workspace missing or too small";
    }
    return "unknown lbm_status";
}

extern "C" const char *lbm_last_error(void) { return lbm::g_last_error.c_str(); }
