#pragma once
#include "common.hpp"

namespace dl {

constexpr int GEMV_MAX_KS = 16;

// out = beta*base + alpha*A*x split into rows [0, split) -> out1/base1 and
// rows [split, M) -> out2/base2 (split < 0: all rows to out1).
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
};

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
};

// partial needs GEMV_MAX_KS * M doubles.
hipError_t launch_gemv_n(const GemvN& g, double* partial, hipStream_t s);
hipError_t launch_gemv_t(const GemvT& g, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t s);

}  // namespace dl
