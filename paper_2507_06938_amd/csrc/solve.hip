// Memory-bound matrix-vector products of the block forward/backward solves
// (HBM-bound: each job streams one dense block once, coalesced).  One launch
// serves a batch of independent jobs (one per matrix of a batch).
#include "solve.hpp"

namespace dl {

// Workgroup (i, s, j): rows 64i..64i+63 of job j, k-split s; lane = row, the
// 4 waves interleave columns (wave w takes columns k0 + w + 4m), each wave
// keeps four independent partial sums (columns 16 apart) so four loads are in
// flight, and the sums are combined in a fixed order.  `tri`: A is lower
// triangular, columns k > row are skipped.
template <typename TA>
__device__ __forceinline__ double gemv_n_rows(const TA* __restrict__ A, int64_t lda,
                                              const double* __restrict__ x, int row, int k,
                                              int k1) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const TA* p = A + row;
  for (; k + 12 < k1; k += 16) {
    a0 += (double)p[(int64_t)k * lda] * x[k];
    a1 += (double)p[(int64_t)(k + 4) * lda] * x[k + 4];
    a2 += (double)p[(int64_t)(k + 8) * lda] * x[k + 8];
    a3 += (double)p[(int64_t)(k + 12) * lda] * x[k + 12];
  }
  for (; k < k1; k += 4) a0 += (double)p[(int64_t)k * lda] * x[k];
  return (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(256) void k_gemv_n_partial(
    const GemvN* __restrict__ jobs) {
  __shared__ double sh[4][64];
  const GemvN g = jobs[blockIdx.z];
  if ((int)blockIdx.x * 64 >= g.M) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + lane;
  const int ks_len = (g.K + GEMV_KS - 1) / GEMV_KS;
  const int k0 = blockIdx.y * ks_len;
  int k1 = min(g.K, k0 + ks_len);
  if (g.tri) k1 = min(k1, (int)blockIdx.x * 64 + 64);
  double acc = 0.0;
  if (row < g.M)
    acc = g.a32 ? gemv_n_rows((const float*)g.A, g.lda, g.x, row, k0 + wave, k1)
                : gemv_n_rows(g.A, g.lda, g.x, row, k0 + wave, k1);
  sh[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && row < g.M)
    g.partial[(int64_t)blockIdx.y * g.M + row] =
        (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

__global__ void k_gemv_n_finish(const GemvN* __restrict__ jobs) {
  const GemvN g = jobs[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.M) return;
  double s = 0.0;
  for (int k = 0; k < GEMV_KS; ++k) s += g.partial[(int64_t)k * g.M + i];
  const int split = g.split < 0 ? g.M : g.split;
  if (i < split) {
    const double b = g.base1 ? g.beta * g.base1[i] : 0.0;
    g.out1[i] = b + g.alpha * s;
  } else {
    const double b = g.base2 ? g.beta * g.base2[i - split] : 0.0;
    g.out2[i - split] = b + g.alpha * s;
  }
}

hipError_t launch_gemv_n(const GemvN* jobs, int count, int max_M, hipStream_t s) {
  if (count <= 0 || max_M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemv_n_partial, dim3((max_M + 63) / 64, GEMV_KS, count),
                     dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(k_gemv_n_finish, dim3((max_M + 255) / 256, count), dim3(256),
                     0, s, jobs);
  return hipGetLastError();
}

// One wave per column j of job blockIdx.y, lanes stride the rows with four
// independent partial sums (rows 64 apart, four loads in flight), combined in
// a fixed order and then by a fixed butterfly.  `tri`: A lower triangular
// (rows i < j skipped).  y must not alias x.
template <typename TA>
__device__ __forceinline__ double gemv_t_col(const TA* __restrict__ col, const GemvT& g,
                                             int i, int split) {
  auto xv = [&](int r) { return (r < split) ? g.x1[r] : g.x2[r - split]; };
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (; i + 192 < g.M; i += 256) {
    a0 += (double)col[i] * xv(i);
    a1 += (double)col[i + 64] * xv(i + 64);
    a2 += (double)col[i + 128] * xv(i + 128);
    a3 += (double)col[i + 192] * xv(i + 192);
  }
  for (; i < g.M; i += 64) a0 += (double)col[i] * xv(i);
  return (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(256) void k_gemv_t(const GemvT* __restrict__ jobs) {
  const GemvT g = jobs[blockIdx.y];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 4 + wave;
  if (j >= g.N) return;
  const int split = g.split < 0 ? g.M : g.split;
  const int i0 = g.tri ? (j & ~63) : 0;
  double acc = g.a32 ? gemv_t_col((const float*)g.A + (int64_t)j * g.lda, g, i0 + lane, split)
                     : gemv_t_col(g.A + (int64_t)j * g.lda, g, i0 + lane, split);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) g.y[j] = (g.base ? g.beta * g.base[j] : 0.0) + g.alpha * acc;
}

hipError_t launch_gemv_t(const GemvT* jobs, int count, int max_N, hipStream_t s) {
  if (count <= 0 || max_N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemv_t, dim3((max_N + 3) / 4, count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace dl
