// Memory-bound matrix-vector products for the block forward/backward solves
// (HBM-bound: each launch streams one dense block once, coalesced).
#include "common.hpp"
#include "solve.hpp"

namespace dl {

// y = beta*base + alpha*A*x, A column-major M x K.  Grid (ceil(M/64), KS):
// workgroup (i, s) sums columns of its k-split into partial[s*M + row];
// lane = row, the 4 waves interleave columns and are combined in a fixed
// order.  `tri`: A is lower triangular, columns k > row are skipped.
__global__ __launch_bounds__(256) void k_gemv_n_partial(
    int M, int K, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ x, int tri, int ks_len,
    double* __restrict__ partial) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + lane;
  int k0 = blockIdx.y * ks_len;
  int k1 = min(K, k0 + ks_len);
  if (tri) k1 = min(k1, blockIdx.x * 64 + 64);
  double acc = 0.0;
  if (row < M) {
    for (int k = k0 + wave; k < k1; k += 4)
      acc += A[(int64_t)row + (int64_t)k * lda] * x[k];
  }
  sh[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && row < M)
    partial[(int64_t)blockIdx.y * M + row] =
        (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

__global__ void k_gemv_n_finish(int M, int KS, const double* __restrict__ partial,
                                double alpha, double beta, int split,
                                const double* base1, double* out1,
                                const double* base2, double* out2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double s = 0.0;
  for (int k = 0; k < KS; ++k) s += partial[(int64_t)k * M + i];
  if (i < split) {
    const double b = base1 ? beta * base1[i] : 0.0;
    out1[i] = b + alpha * s;
  } else {
    const double b = base2 ? beta * base2[i - split] : 0.0;
    out2[i - split] = b + alpha * s;
  }
}

hipError_t launch_gemv_n(const GemvN& g, double* partial, hipStream_t s) {
  if (g.M <= 0) return hipSuccess;
  int KS = (g.K + 255) / 256;
  if (KS < 1) KS = 1;
  if (KS > GEMV_MAX_KS) KS = GEMV_MAX_KS;
  const int ks_len = (g.K + KS - 1) / KS;
  dim3 grid((g.M + 63) / 64, KS);
  hipLaunchKernelGGL(k_gemv_n_partial, grid, dim3(256), 0, s, g.M, g.K, g.A,
                     g.lda, g.x, g.tri, ks_len, partial);
  hipLaunchKernelGGL(k_gemv_n_finish, dim3((g.M + 255) / 256), dim3(256), 0, s,
                     g.M, KS, partial, g.alpha, g.beta,
                     g.split < 0 ? g.M : g.split, g.base1, g.out1, g.base2,
                     g.out2);
  return hipGetLastError();
}

// y[j] = beta*base[j] + alpha * sum_i A[i, j] x[i]; x[i] = x1[i] for
// i < split, x2[i - split] otherwise.  One wave per column, lanes stride the
// rows, then a fixed butterfly.  `tri`: A lower triangular (rows i < j
// skipped).  y must not alias x.
__global__ __launch_bounds__(256) void k_gemv_t(
    int M, int N, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ x1, int split, const double* __restrict__ x2,
    int tri, double alpha, double beta, const double* base,
    double* __restrict__ y) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 4 + wave;
  if (j >= N) return;
  const double* col = A + (int64_t)j * lda;
  const int i0 = tri ? (j & ~63) : 0;
  double acc = 0.0;
  for (int i = i0 + lane; i < M; i += 64) {
    const double xv = (i < split) ? x1[i] : x2[i - split];
    acc += col[i] * xv;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[j] = (base ? beta * base[j] : 0.0) + alpha * acc;
}

hipError_t launch_gemv_t(const GemvT& g, hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemv_t, dim3((g.N + 3) / 4), dim3(256), 0, s, g.M, g.N,
                     g.A, g.lda, g.x1, g.split < 0 ? g.M : g.split, g.x2, g.tri,
                     g.alpha, g.beta, g.base, g.y);
  return hipGetLastError();
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst,
                       int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace dl
