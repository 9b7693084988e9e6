// Device root finding for batches (see rfr_roots.hip) and the per-root
// record it shares with the host finishing stage.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rfr_internal.h"

namespace rfr {

constexpr int ROOT_LANES = 4;                                // lanes per root for a single polynomial
constexpr int ROOT_THREADS = ROOT_LANES * RFR_MAX_DEGREE;  // workgroup size at most
constexpr int ROOT_MAXIT = 400;    // Aberth iterations at most
constexpr int ROOT_POLISH = 6;     // double-double Newton steps at most

// One polynomial: primitive coefficients (ascending, degree >= 2) in device
// memory, and room for `degree` RootOut records.
struct RootJob {
    const int64_t *coeffs;
    int degree;
    RootOut *out;
};

// One workgroup per job with `lanes` (1 or ROOT_LANES) threads per root of
// the largest degree: a batch takes one lane per root (more polynomials in
// flight), a single polynomial ROOT_LANES (shorter dependent chains).
hipError_t launch_roots(const RootJob *jobs_dev, int njobs, int max_degree, int lanes, hipStream_t st);

}  // namespace rfr
