// Helpers of the Takahashi selected inversion sweep.
#include "common.hpp"
#include "selinv.hpp"

namespace dl {

// Workgroups 0..ntri-1 of job blockIdx.y mirror one lower 64x64 tile each
// through LDS; the next bp/64 workgroups copy the arrow rows/columns and the
// diagonal of one 64-column strip.
__global__ __launch_bounds__(256) void k_selinv_finish(const FinishJob* __restrict__ jobs) {
  __shared__ double tile[64][65];
  const FinishJob F = jobs[blockIdx.y];
  const int T = F.bp / 64;
  const int ntri = T * (T + 1) / 2;
  const int tid = threadIdx.x;
  int blk = blockIdx.x;
  double* XC = F.XC;
  const int64_t ld = F.ld;
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
  if (blk >= T) return;
  const int c0 = blk * 64;
  const int ap = F.ap, bp = F.bp;
  for (int idx = tid; idx < 64 * ap; idx += 256) {
    const int i = idx % ap, c = c0 + idx / ap;
    const double v = F.Y[(int64_t)(bp + i) + (int64_t)c * ld];
    XC[(int64_t)(bp + i) + (int64_t)c * ld] = v;
    XC[(int64_t)c + (int64_t)(bp + i) * ld] = v;
  }
  if (tid < 64) F.out[c0 + tid] = XC[(int64_t)(c0 + tid) * (ld + 1)];
}

hipError_t launch_selinv_finish(const FinishJob* jobs, int count, int max_bp,
                                hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int T = max_bp / 64;
  hipLaunchKernelGGL(k_selinv_finish, dim3(T * (T + 1) / 2 + T, count), dim3(256),
                     0, s, jobs);
  return hipGetLastError();
}

}  // namespace dl
