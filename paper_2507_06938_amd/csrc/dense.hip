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

__global__ __launch_bounds__(256) void k_potrf_tile(const PotrfTileArgs* __restrict__ args) {
  const PotrfTileArgs a = args[blockIdx.x];
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
  if (a.mode == 0) {
#pragma unroll
    for (int q = 0; q < CW; ++q)
      a.A[(int64_t)i + (int64_t)(CW * w + q) * a.lda] = r[q];
  }
  if (w == 0 && a.logdiag) a.logdiag[i] = log(Lc[i][i]);
  if (threadIdx.x == 0 && sbad < NB && a.info)
    atomicCAS((unsigned long long*)a.info, 0ull,
              (unsigned long long)(a.row0 + sbad + 1));
  if (a.mode == 0 && !a.Ginv) return;
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
  double* dst = a.mode == 0 ? a.Ginv : a.A;
  const int64_t ldd = a.mode == 0 ? NB : a.lda;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int rr = idx & 63, cc = idx >> 6;
    dst[rr + cc * ldd] = (rr >= cc) ? Gk[rr][cc] : 0.0;
  }
}

hipError_t launch_potrf_tiles(const PotrfTileArgs* args, int count,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_potrf_tile, dim3(count), dim3(256), 0, s, args);
  return hipGetLastError();
}

// Batched element-wise jobs: grid (blocks, jobs).
__global__ __launch_bounds__(256) void k_misc(const MiscJob* __restrict__ jobs) {
  const MiscJob J = jobs[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  switch (J.kind) {
    case MJ_FILL:
      for (int64_t i = i0; i < J.n; i += stride) J.dst[i] = J.v;
      break;
    case MJ_COPY:
      for (int64_t i = i0; i < J.n; i += stride) J.dst[i] = J.src[i];
      break;
    case MJ_ZERO_I64:
      for (int64_t i = i0; i < J.n; i += stride) ((int64_t*)J.dst)[i] = 0;
      break;
    case MJ_DIAG:
      for (int64_t i = i0; i < J.n; i += stride) J.dst[i] = J.src[i * (J.lds + 1)];
      break;
    case MJ_COPY2D: {
      const int64_t tot = (int64_t)J.rows * J.cols;
      for (int64_t i = i0; i < tot; i += stride) {
        const int64_t r = i % J.rows, c = i / J.rows;
        J.dst[r + c * J.ldd] = J.src[r + c * J.lds];
      }
      break;
    }
    case MJ_COPY2D_F32: {
      const float* src32 = (const float*)J.src;
      const int64_t tot = (int64_t)J.rows * J.cols;
      for (int64_t i = i0; i < tot; i += stride) {
        const int64_t r = i % J.rows, c = i / J.rows;
        J.dst[r + c * J.ldd] = (double)src32[r + c * J.lds];
      }
      break;
    }
    case MJ_AXPY:
      for (int64_t i = i0; i < J.n; i += stride) J.dst[i] += J.src[i];
      break;
    case MJ_ZERO_UPPER_TILES: {
      const int64_t tot = (int64_t)J.rows * J.rows;
      for (int64_t i = i0; i < tot; i += stride) {
        const int64_t r = i % J.rows, c = i / J.rows;
        if ((r >> 6) < (c >> 6)) J.dst[r + c * J.ldd] = 0.0;
      }
      break;
    }
  }
}

hipError_t launch_misc(const MiscJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_misc, dim3(256, count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

// Deterministic sums: block b of job j reduces a fixed contiguous range with
// a fixed tree; the job's block partials are then reduced in index order.
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

__global__ __launch_bounds__(256) void k_sum_partial(const SumJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const SumJob J = jobs[blockIdx.y];
  const int64_t per = (J.n + SUM_BLOCKS - 1) / SUM_BLOCKS;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min(J.n, b0 + per);
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) acc += J.src[i];
  const double v = block_sum_256(acc, sh);
  if (threadIdx.x == 0) J.partial[blockIdx.x] = v;
}

__global__ __launch_bounds__(256) void k_sum_final(const SumJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const SumJob J = jobs[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < SUM_BLOCKS; i += 256) acc += J.partial[i];
  const double v = block_sum_256(acc, sh);
  if (threadIdx.x == 0) J.dst[0] = J.scale * v;
}

hipError_t launch_sums(const SumJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_partial, dim3(SUM_BLOCKS, count), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(k_sum_final, dim3(count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace dl
