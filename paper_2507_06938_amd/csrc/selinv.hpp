#pragma once
#include "common.hpp"

namespace dl {
// One step of the selected-inversion sweep is finished per job: mirror the
// lower triangle of X_tt (bp x bp at XC, ld) to its upper triangle, copy
// X_{P,t} (rows bp.. of Y) into the arrow rows and columns of XC, and write
// diag(X_tt) to out.
struct FinishJob {
  double* XC;
  int64_t ld;
  int bp, ap;
  const double* Y;
  double* out;
};
hipError_t launch_selinv_finish(const FinishJob* jobs_dev, int count,
                                int max_bp, hipStream_t s);
}  // namespace dl
