// Small dense kernels: 64x64 diagonal-tile Cholesky + inverse, tile copies,
// fills, deterministic log-sum reductions.
#include "common.hpp"

namespace dl {

namespace {
constexpr int NB = 64;
constexpr int SLD = NB + 1;  // padded LDS stride
}

// One workgroup factors one 64x64 SPD tile (right-looking, column by
// column, in LDS), then forms L^{-1} by forward elimination on the identity.
__global__ __launch_bounds__(256) void k_potrf_tile(PotrfTileArgs a) {
  __shared__ double S[NB * SLD];   // S[r*SLD + c]
  __shared__ double G[NB * SLD];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    S[r * SLD + c] = a.A[(int64_t)r + (int64_t)c * a.lda];
    G[r * SLD + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  for (int k = 0; k < NB; ++k) {
    const double dkk = S[k * SLD + k];
    const bool ok = dkk > 0.0;  // false for NaN too
    const double d = ok ? sqrt(dkk) : __builtin_nan("");
    if (t > k && t < NB) S[t * SLD + k] = S[t * SLD + k] / d;
    __syncthreads();
    if (t == 0) {
      S[k * SLD + k] = d;
      if (a.logdiag) a.logdiag[k] = log(d);
      if (!ok && bad == 0) {
        bad = 1;
        if (a.info)
          atomicCAS((unsigned long long*)a.info, 0ull,
                    (unsigned long long)(a.row0 + k + 1));
      }
    }
    const int w = NB - 1 - k;  // trailing order
    for (int idx = t; idx < w * w; idx += 256) {
      const int i = k + 1 + idx / w;
      const int j = k + 1 + idx % w;
      if (j <= i) S[i * SLD + j] -= S[i * SLD + k] * S[j * SLD + k];
    }
    __syncthreads();
  }

  // L G = I by elimination: scale row k, eliminate it from rows below.
  for (int k = 0; k < NB; ++k) {
    const double lkk = S[k * SLD + k];
    if (t <= k) G[k * SLD + t] = G[k * SLD + t] / lkk;
    __syncthreads();
    const int rows = NB - 1 - k, cols = k + 1;
    for (int idx = t; idx < rows * cols; idx += 256) {
      const int i = k + 1 + idx / cols;
      const int j = idx % cols;
      G[i * SLD + j] -= S[i * SLD + k] * G[k * SLD + j];
    }
    __syncthreads();
  }

  for (int idx = t; idx < NB * NB; idx += 256) {
    const int r = idx & 63, c = idx >> 6;
    a.A[(int64_t)r + (int64_t)c * a.lda] = (r >= c) ? S[r * SLD + c] : 0.0;
    if (a.Ginv) a.Ginv[r + c * NB] = (r >= c) ? G[r * SLD + c] : 0.0;
  }
}

hipError_t launch_potrf_tile(const PotrfTileArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void k_copy_tile64(const double* __restrict__ src, int64_t lds,
                              double* __restrict__ dst, int64_t ldd,
                              int64_t sstride, int64_t dstride) {
  const double* s = src + sstride * blockIdx.x;
  double* d = dst + dstride * blockIdx.x;
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int r = idx & 63, c = idx >> 6;
    d[(int64_t)r + (int64_t)c * ldd] = s[(int64_t)r + (int64_t)c * lds];
  }
}

hipError_t launch_copy_tile64(const double* src, int64_t lds, double* dst,
                              int64_t ldd, int ntiles, int64_t sstride,
                              int64_t dstride, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_tile64, dim3(ntiles), dim3(256), 0, s, src, lds,
                     dst, ldd, sstride, dstride);
  return hipGetLastError();
}

// Zero the tiles strictly above the diagonal tiles of an n x n (n % 64 == 0)
// column-major matrix.
__global__ void k_zero_upper_tiles(double* A, int64_t ld, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i % n), c = (int)(i / n);
    if ((r >> 6) < (c >> 6)) A[r + (int64_t)c * ld] = 0.0;
  }
}

hipError_t launch_zero_upper_tiles(double* A, int64_t ld, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_upper_tiles, dim3(1024), dim3(256), 0, s, A, ld, n);
  return hipGetLastError();
}

__global__ void k_fill(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Deterministic sum: each block reduces a fixed contiguous range with a
// fixed tree; block partials are then reduced by one block in index order.
__device__ __forceinline__ double block_sum_256(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_sum_partial(const double* x, int64_t n,
                                                     int64_t per_block,
                                                     double* partial) {
  __shared__ double sh[256];
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = min(n, b0 + per_block);
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) acc += x[i];
  const double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sum_final(const double* partial, int np,
                                                   double scale, double* out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += partial[i];
  const double s = block_sum_256(acc, sh);
  if (threadIdx.x == 0) out[0] = scale * s;
}

// out[0] = scale * sum(x[0..n)); `partial` needs 256 doubles.
hipError_t launch_sum_log(const double* x, int64_t n, double scale,
                          double* out, double* partial, hipStream_t s) {
  int64_t per = (n + 255) / 256;
  if (per < 1024) per = 1024;
  int nb = (int)((n + per - 1) / per);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(256), 0, s, x, n, per,
                     partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nb, scale,
                     out);
  return hipGetLastError();
}

}  // namespace dl
