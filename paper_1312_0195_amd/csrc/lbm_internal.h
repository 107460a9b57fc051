// lbm_internal.h -- definitions shared by the HIP sources of liblbm.
//
// D2Q9 lattice of Sec. 2 (numbering as in the paper), FP64 reductions and the
// host-side error plumbing. Device code is written for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "lbm.h"

namespace lbm {

// D2Q9 weights: 4/9 for the rest population, 1/9 for the axis directions,
// 1/36 for the diagonals.
constexpr double kW0 = 4.0 / 9.0;
constexpr double kW1 = 1.0 / 9.0;
constexpr double kW5 = 1.0 / 36.0;

__host__ __device__ constexpr double weight(int a) { return a == 0 ? kW0 : (a <= 4 ? kW1 : kW5); }
__host__ __device__ constexpr int ex(int a)
{
    return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey(int a)
{
    return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opposite(int a) { return a == 0 ? 0 : (a <= 4 ? 1 + (a + 1) % 4 : 5 + (a - 3) % 4); }

constexpr size_t kAlign = 256;
__host__ __device__ constexpr size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Host-side error state (thread local), set by the entry points.
lbm_status set_error(lbm_status s, const std::string &msg);
lbm_status hip_check(hipError_t e, const char *what);
#define LBM_HIP(call)                                            \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return ::lbm::hip_check(e_, #call); \
    } while (0)

// Number of compute units of the current device (cached per device).
int device_cu_count();

// ---------------------------------------------------------------------------
// Wave- and block-level FP64 sums with a fixed summation order, so results do
// not depend on scheduling.
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace lbm
