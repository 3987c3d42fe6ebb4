// Opt-in device-side validation of the inputs of tmm_rt / tmm_rt_grad
// (TMM_CHECK_FINITE); see tmm_check.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tmm_rt.h"

namespace tmm {

template <typename R>
struct CheckArgs {
    int B, L, n_wl, n_theta;
    const R* d;          // [B][L]
    const R* nk;         // [nk_rows][nk_cols] complex interleaved
    int64_t nk_rows, nk_cols;
    int n_mat;
    const int32_t* mat;  // [B][L+2] or NULL
    const R* wl;         // [n_wl]
    const R* sin_t;      // [n_theta]
    const R* cos_t;      // [n_theta]
    const R* extra0;     // further real arrays checked for finiteness only (or NULL)
    int64_t n_extra0;
    const R* extra1;
    int64_t n_extra1;
};

// Scans the arrays the call will read (plus up to two extra real arrays) on
// the stream, reads the result back (synchronising the stream) and returns
// TMM_OK, TMM_ERR_NONFINITE, TMM_ERR_INVALID_ARG or TMM_ERR_HIP.
template <typename R>
tmm_status check_rt_inputs(const tmm_rt_args* a, const R* extra0, int64_t n_extra0, const R* extra1,
                           int64_t n_extra1, const char* who, hipStream_t s);

}  // namespace tmm
