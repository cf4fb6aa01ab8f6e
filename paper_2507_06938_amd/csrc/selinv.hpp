#pragma once
#include "common.hpp"

namespace dl {
hipError_t launch_selinv_finish(double* XC, int64_t ld, int bp, int ap,
                                const double* Y, double* out, hipStream_t s);
hipError_t launch_diag_copy(const double* A, int64_t ld, int n, double* out,
                            hipStream_t s);
hipError_t launch_zero_i64(int64_t* p, int n, hipStream_t s);
hipError_t launch_copy2d(const double* src, int64_t lds, double* dst,
                         int64_t ldd, int rows, int cols, hipStream_t s);
}  // namespace dl
