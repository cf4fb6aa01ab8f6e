#pragma once
#include "common.hpp"

namespace dl {

constexpr int GEMV_KS = 16;  // k-splits of a column-major matrix-vector product

// out = beta*base + alpha*A*x, rows [0, split) -> out1/base1 and rows
// [split, M) -> out2/base2 (split < 0: all rows to out1).  `partial` holds
// GEMV_KS * M doubles private to this job.
struct GemvN {
  int M, K;
  const double* A;
  int64_t lda;
  const double* x;
  int tri;
  double alpha, beta;
  int split;
  const double* base1;
  double* out1;
  const double* base2;
  double* out2;
  double* partial;
  int a32;  // A stored in FP32
};

// y = beta*base + alpha*A^T*x with x = [x1 (rows < split); x2].
struct GemvT {
  int M, N;
  const double* A;
  int64_t lda;
  const double* x1;
  int split;
  const double* x2;
  int tri;
  double alpha, beta;
  const double* base;
  double* y;
  int a32;  // A stored in FP32
};

// Batched launches over job arrays in device memory; max_M / max_N bound the
// grid over all jobs.
hipError_t launch_gemv_n(const GemvN* jobs_dev, int count, int max_M,
                         hipStream_t s);
hipError_t launch_gemv_t(const GemvT* jobs_dev, int count, int max_N,
                         hipStream_t s);

}  // namespace dl
