// Device root finding for batches (see rfr_roots.hip) and the per-root
// record it shares with the host finishing stage.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rfr_internal.h"

namespace rfr {

constexpr int ROOT_THREADS = 256;  // one thread per root (degree <= RFR_MAX_DEGREE = 256)
constexpr int ROOT_MAXIT = 400;    // Aberth iterations at most
constexpr int ROOT_POLISH = 6;     // double-double Newton steps at most

// One polynomial: primitive coefficients (ascending, degree >= 2) in device
// memory, and room for `degree` RootOut records.
struct RootJob {
    const int64_t *coeffs;
    int degree;
    RootOut *out;
};

hipError_t launch_roots(const RootJob *jobs_dev, int njobs, hipStream_t st);

}  // namespace rfr
