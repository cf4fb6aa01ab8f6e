// Helpers of the Takahashi selected inversion sweep.
#include "common.hpp"
#include "selinv.hpp"

namespace dl {

// After X_tt (lower triangle) is formed in XC (ld = bp+ap):
//   * mirror its lower triangle to the upper one (X_tt is symmetric and the
//     next step multiplies with the full block);
//   * place X_{P,t} (rows bp.. of Y) into XC's arrow rows and, transposed,
//     its arrow columns;
//   * write diag(X_tt) to out.
// Workgroups 0..ntri-1 mirror one lower 64x64 tile pair each through LDS;
// the next ceil(bp/64) workgroups copy the arrow rows/columns and the
// diagonal of one 64-column strip.
__global__ __launch_bounds__(256) void k_selinv_finish(double* XC, int64_t ld,
                                                       int bp, int ap,
                                                       const double* Y,
                                                       double* out, int ntri) {
  __shared__ double tile[64][65];
  const int tid = threadIdx.x;
  int blk = blockIdx.x;
  if (blk < ntri) {
    int I = (int)((sqrt(8.0 * (double)blk + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= blk) ++I;
    while (I * (I + 1) / 2 > blk) --I;
    const int J = blk - I * (I + 1) / 2;
    const int r0 = I * 64, c0 = J * 64;
    for (int idx = tid; idx < 64 * 64; idx += 256) {
      const int r = idx & 63, c = idx >> 6;
      tile[r][c] = XC[(int64_t)(r0 + r) + (int64_t)(c0 + c) * ld];
    }
    __syncthreads();
    // upper tile (J, I): element (c0 + c, r0 + r) = lower (r0 + r, c0 + c)
    for (int idx = tid; idx < 64 * 64; idx += 256) {
      const int c = idx & 63, r = idx >> 6;  // row c0+c of the upper tile
      if (I == J && c >= r) continue;        // diagonal tile: strict upper only
      XC[(int64_t)(c0 + c) + (int64_t)(r0 + r) * ld] = tile[r][c];
    }
    return;
  }
  blk -= ntri;
  const int c0 = blk * 64;
  for (int idx = tid; idx < 64 * ap; idx += 256) {
    const int i = idx % ap, c = c0 + idx / ap;
    if (c >= bp) continue;
    const double v = Y[(int64_t)(bp + i) + (int64_t)c * ld];
    XC[(int64_t)(bp + i) + (int64_t)c * ld] = v;
    XC[(int64_t)c + (int64_t)(bp + i) * ld] = v;
  }
  if (tid < 64 && c0 + tid < bp)
    out[c0 + tid] = XC[(int64_t)(c0 + tid) * (ld + 1)];
}

hipError_t launch_selinv_finish(double* XC, int64_t ld, int bp, int ap,
                                const double* Y, double* out, hipStream_t s) {
  const int T = bp / 64;
  const int ntri = T * (T + 1) / 2;
  hipLaunchKernelGGL(k_selinv_finish, dim3(ntri + T), dim3(256), 0, s, XC, ld,
                     bp, ap, Y, out, ntri);
  return hipGetLastError();
}

__global__ void k_diag_copy(const double* A, int64_t ld, int n, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = A[(int64_t)i * (ld + 1)];
}

hipError_t launch_diag_copy(const double* A, int64_t ld, int n, double* out,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_copy, dim3((n + 255) / 256), dim3(256), 0, s, A, ld,
                     n, out);
  return hipGetLastError();
}

__global__ void k_zero_i64(int64_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_zero_i64(int64_t* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// Copy the leading rows x cols of a column-major matrix.
__global__ void k_copy2d(const double* src, int64_t lds, double* dst,
                         int64_t ldd, int rows, int cols) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i % rows), c = (int)(i / rows);
    dst[r + (int64_t)c * ldd] = src[r + (int64_t)c * lds];
  }
}

hipError_t launch_copy2d(const double* src, int64_t lds, double* dst,
                         int64_t ldd, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy2d, dim3(1024), dim3(256), 0, s, src, lds, dst, ldd,
                     rows, cols);
  return hipGetLastError();
}

}  // namespace dl
