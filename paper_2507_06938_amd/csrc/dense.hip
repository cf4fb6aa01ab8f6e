// Small dense kernels: 64x64 diagonal-tile Cholesky + inverse, tile copies,
// fills, deterministic log-sum reductions.
#include "common.hpp"

namespace dl {

namespace {
constexpr int NB = 64;
constexpr int LDL = NB + 2;         // LDS row stride: 528 B, 16-byte aligned rows
constexpr int TILE_LDS = NB * LDL;  // doubles of one staged 64 x 64 tile
constexpr int POTRF_CW = 8;         // columns per wave of the tile factor
constexpr int POTRF_NT = NB / POTRF_CW * 64;  // threads of a tile-factor workgroup
typedef double v4d __attribute__((ext_vector_type(4)));
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps
// y <- y + (y/2)(1 - x y^2), each of which squares the relative error.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = __builtin_fma(-(x * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
  }
  return y;
}

// Two 16x16 blocks of a 64-deep product of LDS tiles stored S[k*LDL + c]:
//   D[a][b] = sum_k P[k][p0 + a] Q[k][q0 + b]   (and q0 + 16 for acc1),
// on v_mfma_f64_16x16x4_f64 (lane l supplies P[k0 + l/16][p0 + l%16] as the
// "A" operand and Q[k0 + l/16][q0 + l%16] as "B"; register r of lane l
// receives D[l/16 + 4r][l%16]).
__device__ __forceinline__ void mfma2_k64(const double* P, int p0, const double* Q,
                                          int q0, v4d& acc0, v4d& acc1) {
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = l >> 4;
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += 4) {
    const double a = P[(k0 + lk) * LDL + p0 + lr];
    const double b0 = Q[(k0 + lk) * LDL + q0 + lr];
    const double b1 = Q[(k0 + lk) * LDL + q0 + 16 + lr];
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc1, 0, 0, 0);
  }
}

// S[k*LDL + r] = X[r + k*ldx] for the 64 x 64 tile X (column-major).
template <int NT>
__device__ __forceinline__ void stage_tile(const double* __restrict__ X, int64_t ldx,
                                           double* S) {
#pragma unroll
  for (int idx = threadIdx.x; idx < NB * NB; idx += NT) {
    const int r = idx & 63, k = idx >> 6;
    S[k * LDL + r] = X[r + (int64_t)k * ldx];
  }
}

// Cholesky A = L L^T of one 64 x 64 SPD tile and G = L^{-1}, by one
// workgroup of 8 waves.  Lane i of wave w keeps row i of columns
// CW*w .. CW*w+CW-1 of the trailing matrix (r) and rows CW*w .. CW*w+CW-1 of
// column i of the inverse being eliminated (g).  Step s (one barrier a step):
//  * the wave owning column s reads the pivot from lane s, forms
//    L(:, s) = A(:, s) / sqrt(A(s, s)) (zero above the diagonal) with one
//    reciprocal square root, and publishes it to LDS;
//  * the wave owning row s-1 of the inverse scales it by 1/L(s-1, s-1)
//    (the reciprocal it formed one step earlier) and publishes it;
//  * after the barrier every wave applies the rank-1 update of column s to
//    its columns and the elimination of row s-1 to its rows of G.
// Both updates are applied to every column / row a wave holds: the
// multipliers above the diagonal are exact zeros, and the one column (row)
// that an update spoils is already final in LDS, from where the results are
// written.  Every LDS slot is written once, so one barrier a step suffices.
// The loop over owners is rolled and the CW steps of one owner unrolled
// (static register indices, code within the instruction cache).
//
// src/lds: the tile (column-major, global or LDS); Lc, Gk: two LDS tiles of
// TILE_LDS doubles (Lc[k*LDL + i] = L(i, k), Gk[k*LDL + c] = G(k, c)).
// Outputs as described for PotrfTileArgs (A/lda: where mode 0 writes L and
// mode 1 writes G).
template <int CW>
__device__ __forceinline__ void potrf_body(const double* src, int64_t lds, double* Lc,
                                           double* Gk, int* sbad, double* A, int64_t lda,
                                           double* Ginv, double* logdiag, int64_t* info,
                                           int64_t row0, int mode, double* Mout) {
  constexpr int NW = NB / CW;
  constexpr int NT = NW * 64;
  const int i = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x == 0) *sbad = NB;
  double r[CW], g[CW], lp[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    r[q] = src[(int64_t)i + (int64_t)(CW * wv + q) * lds];
    g[q] = (CW * wv + q == i) ? 1.0 : 0.0;
    lp[q] = 0.0;
  }
  double rsp = 0.0;  // owner's 1/L(s-1, s-1) from its previous step
  __syncthreads();
#pragma unroll 1
  for (int kb = 0; kb < NW; ++kb) {
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      const int s = kb * CW + q;
      // row s-1 of the inverse: owned by the wave that owned column s-1
      if (q > 0 ? (wv == kb) : (kb > 0 && wv == kb - 1)) {
        Gk[(s - 1) * LDL + i] = g[(q + CW - 1) % CW] * rsp;
      }
      if (wv == kb) {
        const double d = readlane_f64(r[q], s);
        const bool ok = d > 0.0;  // false for NaN too
        if (!ok && i == 0) atomicMin(sbad, s);
        const double rs = ok ? rsqrt_nr(d) : __builtin_nan("");
        Lc[s * LDL + i] = (i > s) ? r[q] * rs : (i == s ? d * rs : 0.0);
        rsp = rs;
      }
      __syncthreads();
      const double lik = Lc[s * LDL + i];
      double ls[CW];
#pragma unroll
      for (int qq = 0; qq < CW; ++qq) ls[qq] = Lc[s * LDL + CW * wv + qq];
#pragma unroll
      for (int qq = 0; qq < CW; ++qq) r[qq] = __builtin_fma(-lik, ls[qq], r[qq]);
      if (s > 0) {
        const double gk = Gk[(s - 1) * LDL + i];
#pragma unroll
        for (int qq = 0; qq < CW; ++qq) g[qq] = __builtin_fma(-lp[qq], gk, g[qq]);
      }
#pragma unroll
      for (int qq = 0; qq < CW; ++qq) lp[qq] = ls[qq];
    }
  }
  if (wv == NW - 1) Gk[(NB - 1) * LDL + i] = g[CW - 1] * rsp;
  __syncthreads();
  if (wv == 0 && logdiag) logdiag[i] = log(Lc[i * LDL + i]);
  if (threadIdx.x == 0 && *sbad < NB && info)
    atomicCAS((unsigned long long*)info, 0ull, (unsigned long long)(row0 + *sbad + 1));
  if (mode == 0) {
    for (int idx = threadIdx.x; idx < NB * NB; idx += NT) {
      const int rr = idx & 63, cc = idx >> 6;
      A[rr + (int64_t)cc * lda] = Lc[cc * LDL + rr];
    }
  }
  double* dst = mode == 0 ? Ginv : A;
  const int64_t ldd = mode == 0 ? NB : lda;
  if (dst) {
    for (int idx = threadIdx.x; idx < NB * NB; idx += NT) {
      const int rr = idx & 63, cc = idx >> 6;
      dst[rr + cc * ldd] = (rr >= cc) ? Gk[rr * LDL + cc] : 0.0;
    }
  }
  if (Mout) {
    // M = G^T G: M(a, b) = sum_k G(k, a) G(k, b); only a >= b is taken from
    // the product and written to both halves (exact symmetry).
    static_assert(NW == 8, "M product assumes 8 waves");
    const int l = threadIdx.x & 63;
    const int a0 = 16 * (wv >> 1), b0 = 32 * (wv & 1);
    v4d m0 = {0.0, 0.0, 0.0, 0.0}, m1 = {0.0, 0.0, 0.0, 0.0};
    mfma2_k64(Gk, a0, Gk, b0, m0, m1);
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) {
      const int a = a0 + (l >> 4) + 4 * rg;
      const int b = b0 + (l & 15);
      if (a >= b) {
        Mout[a + b * NB] = m0[rg];
        Mout[b + a * NB] = m0[rg];
      }
      if (a >= b + 16) {
        Mout[a + (b + 16) * NB] = m1[rg];
        Mout[(b + 16) + a * NB] = m1[rg];
      }
    }
  }
}

__global__ __launch_bounds__(POTRF_NT) void k_potrf_tile(const PotrfTileArgs* __restrict__ args) {
  const PotrfTileArgs a = args[blockIdx.x];
  __shared__ __align__(16) double Lc[TILE_LDS];
  __shared__ __align__(16) double Gk[TILE_LDS];
  __shared__ int sbad;
  potrf_body<POTRF_CW>(a.A, a.lda, Lc, Gk, &sbad, a.A, a.lda, a.Ginv, a.logdiag, a.info,
                       a.row0, a.mode, a.M);
}

hipError_t launch_potrf_tiles(const PotrfTileArgs* args, int count,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_potrf_tile, dim3(count), dim3(POTRF_NT), 0, s, args);
  return hipGetLastError();
}

// ---- fused panel step ---------------------------------------------------------------
//
// Workgroup g < ntask factors: it updates diagonal tile j+1 of task g and then
// factors it; the others update one lower tile (I, J) each.  Per tile, with
// the 64 x 64 operands staged in LDS (S0 = P_j(I), S1 = M_j, S2 = P_j(J)):
//   T^T = M_j P_j(I)^T               (S1, S0)  -> T stored back over S0,
//   (T P_j(J)^T)^T = P_j(J) T^T      (S2, S0)  -> subtracted from A(I, J),
// both on FP64 MFMA with the operand roles chosen so that a lane's results
// lie along the rows of the column-major output (coalesced stores).  The
// factoring workgroup stages the updated tile in LDS (S1) instead and runs
// the tile factor on it with S0 and S2 as its scratch tiles.
__global__ __launch_bounds__(POTRF_NT) void k_panel_update(const PanelTask* __restrict__ tasks,
                                                           int ntask) {
  __shared__ __align__(16) double pool[3 * TILE_LDS];
  __shared__ int sbad;
  double* S0 = pool;
  double* S1 = pool + TILE_LDS;
  double* S2 = pool + 2 * TILE_LDS;
  const bool fac = (int)blockIdx.x < ntask;
  int ti, lt;
  if (fac) {
    ti = blockIdx.x;
    lt = 0;
  } else {
    const int g = blockIdx.x - ntask;
    int lo = 0, hi = ntask - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].tile_begin <= g) lo = mid; else hi = mid - 1;
    }
    ti = lo;
    lt = 1 + g - tasks[ti].tile_begin;
  }
  const PanelTask T = tasks[ti];
  // row-major enumeration of the lower triangle of the trailing tile grid
  int I = (int)((sqrt(8.0 * (double)lt + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= lt) ++I;
  while (I * (I + 1) / 2 > lt) --I;
  const int J = lt - I * (I + 1) / 2;
  const int64_t ti0 = (int64_t)(T.j + 1 + I) * NB, tj0 = (int64_t)(T.j + 1 + J) * NB;
  const int64_t pc = (int64_t)T.j * NB * T.ld;
  stage_tile<POTRF_NT>(T.A + ti0 + pc, T.ld, S0);
  stage_tile<POTRF_NT>(T.M, NB, S1);
  stage_tile<POTRF_NT>(T.A + tj0 + pc, T.ld, S2);
  __syncthreads();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = l >> 4;
  const int p0 = 16 * (wv >> 1), q0 = 32 * (wv & 1);
  v4d t0 = {0.0, 0.0, 0.0, 0.0}, t1 = {0.0, 0.0, 0.0, 0.0};
  mfma2_k64(S1, p0, S0, q0, t0, t1);  // t: T(m = q0 + lr (+16), c = p0 + lk + 4r)
  __syncthreads();
#pragma unroll
  for (int rg = 0; rg < 4; ++rg) {
    const int c = p0 + lk + 4 * rg;
    S0[c * LDL + q0 + lr] = t0[rg];
    S0[c * LDL + q0 + 16 + lr] = t1[rg];
  }
  __syncthreads();
  v4d u0 = {0.0, 0.0, 0.0, 0.0}, u1 = {0.0, 0.0, 0.0, 0.0};
  mfma2_k64(S2, p0, S0, q0, u0, u1);  // u: update(m = q0 + lr (+16), n = p0 + lk + 4r)
  double* C = T.A + ti0 + tj0 * T.ld;
  if (!fac) {
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) {
      const int64_t n = p0 + lk + 4 * rg;
      double* c0 = C + (q0 + lr) + n * T.ld;
      *c0 -= u0[rg];
      c0[16] -= u1[rg];
    }
    return;
  }
#pragma unroll
  for (int rg = 0; rg < 4; ++rg) {
    const int n = p0 + lk + 4 * rg;
    const double* c0 = C + (q0 + lr) + (int64_t)n * T.ld;
    S1[n * LDL + q0 + lr] = c0[0] - u0[rg];
    S1[n * LDL + q0 + 16 + lr] = c0[16] - u1[rg];
  }
  __syncthreads();
  potrf_body<POTRF_CW>(S1, LDL, S0, S2, &sbad, C, T.ld, nullptr, T.logdiag, T.info,
                       T.row0, 1, T.Mnext);
}

int finalize_panels(PanelTask* t, int n) {
  int total = 0;
  for (int i = 0; i < n; ++i) {
    const int m = t[i].nbk - t[i].j - 1;
    t[i].ntiles = m * (m + 1) / 2;
    t[i].tile_begin = total;
    total += t[i].ntiles - 1;
  }
  return n + total;
}

hipError_t launch_panel_updates(const PanelTask* tasks, int ntask, int grid,
                                hipStream_t s) {
  if (ntask <= 0 || grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_update, dim3(grid), dim3(POTRF_NT), 0, s, tasks, ntask);
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
