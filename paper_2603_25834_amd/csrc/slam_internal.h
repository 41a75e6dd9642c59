// slam_internal.h -- library-internal entry points of the fixed-lag SLAM backbone (slam.hip), used by
// the C-ABI calls of slam.hip and by the env step's fixed-lag backend (capi.hip).  Not part of the
// public ABI.  All launches are asynchronous on `stream`; `tab` is a device copy of the 46080-entry
// direction table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aslam {
namespace slam {

// w = q m of a match [best i, j, k, best, second, rays with a return]: q = clamp(best / (rays l_max)),
// m = clamp((best - second) / max(best, 1)).
__host__ __device__ inline double match_weight(const int32_t* m, double l_max) {
  const double best = (double)m[3], second = (double)m[4];
  const double q = m[5] <= 0 ? 0.0 : fmin(fmax(best / ((double)m[5] * l_max), 0.0), 1.0);
  const double mg = fmin(fmax((best - second) / fmax(best, 1.0), 0.0), 1.0);
  return q * mg;
}

hipError_t launch_csm_match(const int32_t* tab, const int16_t* belief, const int64_t* cell_off, const int32_t* side,
                            int32_t max_side, int32_t n, const int32_t* pose_q, const int32_t* rho_q, int32_t R,
                            const int32_t* a_off, int W, int V, int step_xy_q, int step_h, int32_t* out,
                            hipStream_t stream);

// wq (may be NULL): per-robot integration weights w_q, the scan cast from pose_q itself (match unused).
hipError_t launch_csm_integrate(const int32_t* tab, int16_t* belief, const int64_t* cell_off, const int32_t* side,
                                int32_t n, const int32_t* pose_q, const int32_t* rho_q, int32_t R,
                                const int32_t* a_off, int32_t max_side, int32_t rmax_q, const int32_t* match,
                                int step_xy, int step_h, double l_max, int32_t l_hit, int32_t l_miss,
                                int32_t l_clamp, int32_t* coded, const int32_t* wq, hipStream_t stream);

// counts (may be NULL): poses of each window (<= L, arrays strided for L); NULL = L for every window.
hipError_t launch_fixedlag(int32_t n, int32_t L, const int32_t* counts, const double* x0, const double* prior,
                           const double* odo, const double* scan, int32_t iters, double* x, double* cov,
                           hipStream_t stream);

constexpr int kMaxWindow = 64;
constexpr int kMaxHalf = 8;                 // lattice half-widths W, V <= 8
constexpr int kMaxRayHeadings = 8192;       // (2V + 1) R

}  // namespace slam
}  // namespace aslam
