// Point-list evaluation of the dense batch (tmm_rt_points and the surrogate's
// fallback); see tmm_points.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tmm_rt.h"

namespace tmm {
namespace pts {

template <typename R>
struct PtParams {
    int B, L, n_wl, n_theta;
    const R* d;
    const R* nk;
    int n_mat, dispersive;
    const int32_t* mat;  // [B][L+2] or NULL (row b*(L+2)+j)
    const R* wl;
    const R* sin_t;
    const R* cos_t;
    R* R_out;            // [B][P][n_theta][n_wl]: only the listed points are written
    R* T_out;
    const int64_t* pts64;   // flat indices (b * n_theta + k) * n_wl + i, or
    const uint32_t* pts32;  // the same in 32 bits (exactly one of the two is set)
    int64_t n_pts;          // number of points, unless
    const int* n_dev;       // a device count is given (read by the kernel)
    R* r_out = nullptr;     // complex interleaved, the layout of R_out, or null;
    R* t_out = nullptr;     // either set: the amplitude kernels
};

// Launch on the stream; max_points bounds the count (sizes the grid).
template <typename R>
hipError_t launch_points(const PtParams<R>& p, unsigned pol_mask, int64_t max_points, hipStream_t s);

}  // namespace pts
}  // namespace tmm
