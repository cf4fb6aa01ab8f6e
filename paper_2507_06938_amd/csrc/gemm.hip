// FP64 MFMA tile GEMM over a list of tasks (gfx950).
//
// One workgroup (256 threads = 4 wave64) computes one 64x64 tile of C for one
// task of a launch.  Tiles of all tasks of a launch are numbered
// consecutively; a workgroup finds its task by binary search over the
// tasks' first tile.  The inner product runs on v_mfma_f64_16x16x4_f64 with
// operands staged through double-buffered LDS (16-deep k chunks).
//
// MFMA lane layout used (f64 16x16x4, wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; its accumulator register r holds D[l/16 + 4r][l%16]
// (checked against host GEMMs by the GPU tests).  The kernel feeds op(B) as
// the MFMA "A" and op(A) as the MFMA "B", so D = C^T and each lane holds 4 C
// values of one row, 16 consecutive rows per lane group: the epilogue writes
// 128-byte column segments of the column-major C.
#include "common.hpp"

namespace dl {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {
constexpr int BK = 16;
constexpr int LDS_LD = GEMM_BM + 2;  // padded LDS row (doubles)

__device__ __forceinline__ int find_task(const GemmTask* __restrict__ tasks,
                                         int ntask, int tile) {
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Stage 4 doubles of op(X) per thread: op(X)[r][k] for a 64-row, 16-deep
// chunk.  `trans` = X stored K x R (contiguous along k).
__device__ __forceinline__ void load_chunk(const double* __restrict__ X,
                                           int64_t ldx, bool trans, int r0,
                                           int R, int k0, int kend, int tid,
                                           double (&v)[4]) {
  if (!trans) {
    // X[r + k*ldx]; lanes run along r (64 consecutive rows per k).
    const int r = r0 + (tid & 63);
    const int kb = k0 + (tid >> 6) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = kb + i;
      v[i] = (r < R && k < kend) ? X[(int64_t)r + (int64_t)k * ldx] : 0.0;
    }
  } else {
    // X[k + r*ldx]; lanes run along k (16 consecutive k per row).
    const int k = k0 + (tid & 15);
    const int rb = r0 + (tid >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = rb + i;
      v[i] = (r < R && k < kend) ? X[(int64_t)k + (int64_t)r * ldx] : 0.0;
    }
  }
}

__device__ __forceinline__ void store_chunk(double* __restrict__ S, bool trans,
                                            int tid, const double (&v)[4]) {
  if (!trans) {
    const int r = tid & 63;
    const int kb = (tid >> 6) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) S[(kb + i) * LDS_LD + r] = v[i];
  } else {
    const int k = tid & 15;
    const int rb = (tid >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) S[k * LDS_LD + rb + i] = v[i];
  }
}

__device__ __forceinline__ void tile_coords(const GemmTask& T, int lt, int& tm,
                                            int& tn) {
  if (T.flags & F_LOWER) {
    // row-major enumeration of the lower triangle of a square tile grid
    int I = (int)((sqrt(8.0 * (double)lt + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= lt) ++I;
    while (I * (I + 1) / 2 > lt) --I;
    tm = I;
    tn = lt - I * (I + 1) / 2;
  } else {
    tm = lt % T.tiles_m;
    tn = lt / T.tiles_m;
  }
}
}  // namespace

__global__ __launch_bounds__(256) void k_gemm_tasks(
    const GemmTask* __restrict__ tasks, int ntask) {
  __shared__ double As[2][BK * LDS_LD];
  __shared__ double Bs[2][BK * LDS_LD];

  const int tid = threadIdx.x;
  const int ti = find_task(tasks, ntask, blockIdx.x);
  const GemmTask T = tasks[ti];
  int tm, tn;
  tile_coords(T, blockIdx.x - T.tile_begin, tm, tn);
  const int m0 = tm * GEMM_BM;
  const int n0 = tn * GEMM_BN;
  const bool ta = T.flags & F_TA;
  const bool tb = T.flags & F_TB;

  int kb = 0, ke = T.K;
  if (T.flags & F_KLO_COL) kb = max(kb, n0);
  if (T.flags & F_KHI_COL) ke = min(ke, n0 + GEMM_BN);
  if (T.flags & F_KLO_ROW) kb = max(kb, m0);
  if (T.flags & F_KHI_ROW) ke = min(ke, m0 + GEMM_BM);
  kb = (kb / BK) * BK;
  const int nchunks = ke > kb ? (ke - kb + BK - 1) / BK : 0;

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int lrow = lane & 15, lk = lane >> 4;

  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  double va[4], vb[4];
  if (nchunks > 0) {
    load_chunk(T.A, T.lda, ta, m0, T.M, kb, ke, tid, va);
    load_chunk(T.B, T.ldb, !tb, n0, T.N, kb, ke, tid, vb);
    store_chunk(As[0], ta, tid, va);
    store_chunk(Bs[0], !tb, tid, vb);
  }
  __syncthreads();

  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    const bool more = (c + 1) < nchunks;
    if (more) {
      const int k1 = kb + (c + 1) * BK;
      load_chunk(T.A, T.lda, ta, m0, T.M, k1, ke, tid, va);
      load_chunk(T.B, T.ldb, !tb, n0, T.N, k1, ke, tid, vb);
    }
    const double* __restrict__ as = As[buf];
    const double* __restrict__ bs = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      double fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = as[kk * LDS_LD + wm * 32 + i * 16 + lrow];
#pragma unroll
      for (int j = 0; j < 2; ++j) fb[j] = bs[kk * LDS_LD + wn * 32 + j * 16 + lrow];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[j], fa[i],
                                                           acc[i][j], 0, 0, 0);
    }
    if (more) {
      store_chunk(As[buf ^ 1], ta, tid, va);
      store_chunk(Bs[buf ^ 1], !tb, tid, vb);
    }
    __syncthreads();
  }

  // epilogue: lane holds C[m][n0' + lk + 4r], m = row of lane
  const bool lower = T.flags & F_LOWER;
  const bool beta0 = T.flags & F_BETA0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + wm * 32 + i * 16 + lrow;
    if (m >= T.M) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wn * 32 + j * 16 + lk + 4 * r;
        if (n >= T.N || (lower && n > m)) continue;
        double* p = T.C + (int64_t)m + (int64_t)n * T.ldc;
        double v = T.alpha * acc[i][j][r];
        if (!beta0) v += T.beta * (*p);
        *p = v;
      }
    }
  }
}

int finalize_tasks(GemmTask* t, int n) {
  int total = 0;
  for (int i = 0; i < n; ++i) {
    t[i].tiles_m = (t[i].M + GEMM_BM - 1) / GEMM_BM;
    t[i].tiles_n = (t[i].N + GEMM_BN - 1) / GEMM_BN;
    if (t[i].M <= 0 || t[i].N <= 0) {
      t[i].ntiles = 0;
    } else if (t[i].flags & F_LOWER) {
      int T = t[i].tiles_m;  // square tile grid
      t[i].ntiles = T * (T + 1) / 2;
    } else {
      t[i].ntiles = t[i].tiles_m * t[i].tiles_n;
    }
    t[i].tile_begin = total;
    total += t[i].ntiles;
  }
  return total;
}

hipError_t launch_gemm_tasks(const GemmTask* tasks_dev, int ntask,
                             int total_tiles, hipStream_t s) {
  if (total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_tasks, dim3(total_tiles), dim3(256), 0, s,
                     tasks_dev, ntask);
  return hipGetLastError();
}

}  // namespace dl
