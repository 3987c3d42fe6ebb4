// Host-side helpers shared by the entry points of libtmm_rt: error reporting
// and launch-shape arithmetic.  No HIP call is made before validation passes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "tmm_rt.h"

namespace tmm {

// Message of the last failure in this thread (read back by tmm_last_error).
char* last_error_buffer();

inline tmm_status fail(tmm_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(last_error_buffer(), 512, fmt, ap);
    va_end(ap);
    return s;
}

inline tmm_status ok() {
    last_error_buffer()[0] = '\0';
    return TMM_OK;
}

inline tmm_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TMM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Shared host checks of the tmm_rt_args fields (sizes, pointers, ranges);
// need_output: at least one of R, T, r, t must be given.
tmm_status check_rt_args(const tmm_rt_args* a, const char* who, bool need_output);

}  // namespace tmm
