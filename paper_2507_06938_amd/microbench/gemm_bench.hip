// Microbenchmark of the FP64 tile GEMM on the block-product shapes of the
// BTA factorisation and selected inversion (blocks of 2048, arrow of 64):
// 1 warm-up + 10 timed launches per shape and tile size, HIP events around
// the timed launches.  Operands are allocated at full size, so every access
// is in bounds; a weighted checksum of each output identifies the result.
// Used for the kernel's counter profiles (run it under rocprofv3).
#include "../csrc/gemm.hip"

#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace dl;

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_));   \
      exit(1);                                                                    \
    }                                                                             \
  } while (0)

static GemmTask mk(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                   int64_t ldc, int M, int N, int K, int flags, double alpha, double beta) {
  GemmTask t{};
  t.A = A; t.B = B; t.C = C; t.lda = lda; t.ldb = ldb; t.ldc = ldc;
  t.M = M; t.N = N; t.K = K; t.flags = flags; t.alpha = alpha; t.beta = beta;
  return t;
}

int main() {
  const int n = 2048, m = 2112;
  double *A, *B, *C, *part;
  CHECK(hipMalloc(&A, 8L * m * n));
  CHECK(hipMalloc(&B, 8L * m * n));
  CHECK(hipMalloc(&C, 8L * m * m));
  const int64_t part_elems = 160L * 1024 * 1024;  // split-k partial tiles
  CHECK(hipMalloc(&part, 8L * part_elems));
  std::vector<double> h((size_t)m * n);
  for (size_t i = 0; i < h.size(); ++i)
    h[i] = (double)((i * 2654435761ull) % 1000) / 1000.0 - 0.5;
  CHECK(hipMemcpy(A, h.data(), 8L * m * n, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(B, h.data(), 8L * m * n, hipMemcpyHostToDevice));
  struct Case {
    const char* name;
    std::vector<GemmTask> t;
    double flops;
  };
  std::vector<Case> cases = {
      {"NN 2048^3", {mk(A, n, B, n, C, n, n, n, n, F_BETA0, 1, 0)}, 2.0 * n * n * n},
      {"NT 2112x2048x2048, k < col+64 (TRSM by inverse)",
       {mk(A, m, B, n, C, m, m, n, n, F_TB | F_KHI_COL | F_BETA0, 1, 0)}, 1.0 * m * n * n},
      {"NT lower 2048^2, K 2048 (SYRK update)",
       {mk(A, n, A, n, C, n, n, n, n, F_TB | F_LOWER, -1, 1)}, 1.0 * n * n * n},
      {"NT lower 2048^2, K 2048, split k (SYRK update)",
       {mk(A, n, A, n, C, n, n, n, n, F_TB | F_LOWER | F_SPLIT, -1, 1)}, 1.0 * n * n * n},
      {"NN 2112x2048x2112 (selected inversion Y)",
       {mk(C, m, B, m, A, m, m, n, m, F_BETA0, -1, 0)}, 2.0 * m * n * m},
      {"TN lower 2048^2, k >= row (G^T G)",
       {mk(A, n, A, n, C, n, n, n, n, F_TA | F_KLO_ROW | F_KLO_COL | F_LOWER | F_BETA0, 1, 0)},
       2.0 * n * n * n / 3},
      {"NN 1024^3, k >= col (inverse, top level T)",
       {mk(A, n, B, n, C, n, 1024, 1024, 1024, F_KLO_COL | F_BETA0, 1, 0)}, 1024.0 * 1024 * 1024},
      {"NN 1024^3, k < row+64 (inverse, top level G)",
       {mk(A, n, B, n, C, n, 1024, 1024, 1024, F_KHI_ROW | F_BETA0, -1, 0)}, 1024.0 * 1024 * 1024},
  };
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  GemmTask* dt;
  CHECK(hipMalloc(&dt, sizeof(GemmTask) * 8));
  for (auto& c : cases) {
    for (int tile : {64, 128}) {
      std::vector<GemmTask> t = c.t;
      const int nt = (int)t.size();
      int nred = 0;
      int64_t nslots = 0;
      const int units = finalize_tasks(t.data(), nt, tile, &nred, &nslots);
      if (nslots * tile * tile > part_elems) {
        printf("%-50s tile %3d: partial tiles do not fit, skipped\n", c.name, tile);
        continue;
      }
      CHECK(hipMemcpy(dt, t.data(), sizeof(GemmTask) * nt, hipMemcpyHostToDevice));
      auto run = [&]() {
        CHECK(launch_gemm_tasks(dt, nt, units, 0, tile, part));
        if (nred) CHECK(launch_gemm_reduce(dt, nt, nred, part, 0, tile));
      };
      CHECK(hipMemcpy(C, h.data(), 8L * m * n, hipMemcpyHostToDevice));
      run();
      CHECK(hipDeviceSynchronize());
      std::vector<double> hc((size_t)m * m);
      CHECK(hipMemcpy(hc.data(), C, 8L * m * m, hipMemcpyDeviceToHost));
      double cs = 0;
      for (size_t i = 0; i < hc.size(); ++i) cs += hc[i] * (double)(i % 97 + 1);
      const int reps = 10;
      CHECK(hipEventRecord(e0));
      for (int r = 0; r < reps; ++r) run();
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      const double us = ms * 1e3 / reps;
      printf("%-50s tile %3d units %5d: %8.1f us %6.1f TFLOP/s  checksum %.12e\n", c.name,
             tile, units, us, c.flops / (us * 1e-6) / 1e12, cs);
      fflush(stdout);
    }
  }
  return 0;
}
