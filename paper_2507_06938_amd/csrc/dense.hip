// Small dense kernels: 64x64 diagonal-tile Cholesky + inverse, tile copies,
// fills, deterministic log-sum reductions.
#include "common.hpp"

namespace dl {

namespace {
constexpr int NB = 64;
constexpr int SLD = NB + 1;  // padded LDS stride
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// One workgroup of 4 waves factors one 64x64 SPD tile.  Lane i of wave w
// keeps row i, columns 16w..16w+15, in registers.  At column k the wave that
// owns it reads the pivot from lane k, scales its column and publishes it to
// LDS; after one barrier every wave applies the rank-1 update to its own
// columns (the FP64 work of a step is spread over the 4 SIMDs).  L^{-1} is
// formed the same way with lane c owning column c of the inverse.  The 16
// steps of one owner wave are unrolled (register indices stay static); the
// loop over the 4 owners is not, which keeps the code within the
// instruction cache.
constexpr int CW = 16;  // columns per wave

__global__ __launch_bounds__(256) void k_potrf_tile(PotrfTileArgs a) {
  __shared__ double Lc[NB][SLD];   // Lc[k][i] = L(i, k)
  __shared__ double Gk[NB][SLD];   // Gk[k][c] = L^{-1}(k, c)
  __shared__ int sbad;
  const int i = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  if (threadIdx.x == 0) sbad = NB;
  double r[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q)
    r[q] = a.A[(int64_t)i + (int64_t)(CW * w + q) * a.lda];
#pragma unroll 1
  for (int kb = 0; kb < NB / CW; ++kb) {
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int k = kb * CW + q;
      if (w == kb) {
        const double dkk = readlane_f64(r[q], k);
        const bool ok = dkk > 0.0;  // false for NaN too
        if (!ok && i == 0) atomicMin(&sbad, k);
        const double d = ok ? sqrt(dkk) : __builtin_nan("");
        const double lik = (i > k) ? r[q] / d : (i == k ? d : 0.0);
        r[q] = lik;
        Lc[k][i] = lik;
      }
      __syncthreads();
      if (w > kb) {
        const double lik = Lc[k][i];
#pragma unroll
        for (int qq = 0; qq < CW; ++qq) r[qq] -= lik * Lc[k][CW * w + qq];
      } else if (w == kb) {
        const double lik = r[q];
#pragma unroll
        for (int qq = q + 1; qq < CW; ++qq) r[qq] -= lik * Lc[k][CW * w + qq];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CW; ++q)
    a.A[(int64_t)i + (int64_t)(CW * w + q) * a.lda] = r[q];
  if (w == 0 && a.logdiag) a.logdiag[i] = log(Lc[i][i]);
  if (threadIdx.x == 0 && sbad < NB && a.info)
    atomicCAS((unsigned long long*)a.info, 0ull,
              (unsigned long long)(a.row0 + sbad + 1));
  if (!a.Ginv) return;
  const int c = i;
  double g[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) g[q] = (CW * w + q == c) ? 1.0 : 0.0;
#pragma unroll 1
  for (int kb = 0; kb < NB / CW; ++kb) {
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int k = kb * CW + q;
      if (w == kb) {
        g[q] = g[q] / Lc[k][k];
        Gk[k][c] = g[q];
      }
      __syncthreads();
      if (w > kb) {
        const double gk = Gk[k][c];
#pragma unroll
        for (int qq = 0; qq < CW; ++qq) g[qq] -= Lc[k][CW * w + qq] * gk;
      } else if (w == kb) {
        const double gk = g[q];
#pragma unroll
        for (int qq = q + 1; qq < CW; ++qq) g[qq] -= Lc[k][CW * w + qq] * gk;
      }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int rr = idx & 63, cc = idx >> 6;
    a.Ginv[rr + cc * NB] = (rr >= cc) ? Gk[rr][cc] : 0.0;
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
