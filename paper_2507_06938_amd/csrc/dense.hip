// Small dense kernels: 64x64 diagonal-tile Cholesky + inverse, tile copies,
// fills, deterministic log-sum reductions.
#include "common.hpp"

#define DL_DAG_FN __host__ __device__ inline
#include "dag.hpp"

namespace dl {

namespace {
constexpr int NB = 64;
constexpr int LDL = NB + 2;         // LDS row stride: 528 B, 16-byte aligned rows
constexpr int TILE_LDS = NB * LDL;  // doubles of one staged 64 x 64 tile
constexpr int POTRF_CW = 4;         // columns per wave (one panel) of the tile factor
constexpr int POTRF_NT = NB / POTRF_CW * 64;  // threads of a tile-factor workgroup (16 waves)
typedef double v4d __attribute__((ext_vector_type(4)));
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Device-coherent accesses (agent-scope relaxed atomics: sc1 loads and
// stores that bypass the per-XCD caches): the persistent factorisation
// exchanges tiles between workgroups on different XCDs with these.
// (global address space: keeps them off the generic load path)
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ double cload(const double* p) {
  return __hip_atomic_load((const gdouble*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cstore(double* p, double v) {
  __hip_atomic_store((gdouble*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// p must point to global memory
__device__ __forceinline__ double global_load(const double* p) { return *(const gdouble*)p; }
// COH: a device-coherent load of global memory; otherwise a plain load
// through a generic pointer (the tile factor also reads LDS tiles this way)
template <bool COH>
__device__ __forceinline__ double gload(const double* p) {
  if constexpr (COH) return cload(p);
  else return *p;
}
template <bool COH>
__device__ __forceinline__ void gstore(double* p, double v) {
  if constexpr (COH) cstore(p, v);
  else *p = v;
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

// One 16x16 block of a product of LDS tiles stored S[k*LDL + c]:
//   D[a][b] = sum_{k < kmax} P[k][p0 + a] Q[k][q0 + b],
// on v_mfma_f64_16x16x4_f64 (lane l supplies P[k0 + l/16][p0 + l%16] as the
// "A" operand and Q[k0 + l/16][q0 + l%16] as "B"; register r of lane l
// receives D[l/16 + 4r][l%16]).  kmax: multiple of 4, at most 64.
__device__ __forceinline__ void mfma1_k64(const double* P, int p0, const double* Q,
                                          int q0, v4d& acc, int kmax = NB) {
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = l >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < kmax; k0 += 4) {
    const double a = P[(k0 + lk) * LDL + p0 + lr];
    const double b = Q[(k0 + lk) * LDL + q0 + lr];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
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
// workgroup of NB/CW waves.  Lane i of wave w keeps row i of the CW columns
// CW*w .. CW*w+CW-1 (panel w) of the trailing matrix (r) and the same rows of
// column i of the inverse being eliminated (g).  Panels are factored in
// order, one barrier each.  Iteration k:
//  * wave k factors panel k in its registers: per column s, the pivot from
//    lane s (v_readlane), one reciprocal square root, L(:, s) = A(:, s) /
//    sqrt(A(s, s)) (zero above the diagonal), and the update of the panel's
//    later columns with L(c, s) taken from lane c; it then forms rows
//    CW*k .. of G by the same eliminations on g, and publishes both to LDS;
//  * after the barrier every later wave applies the rank-CW update of panel
//    k to its columns and its rows of G (L and G rows read back from LDS).
// Each element receives its updates one FMA per column, in column order, so
// the results do not depend on CW.  Every LDS slot is written once, so one
// barrier a panel suffices.
//
// src/lds: the tile (column-major, global or LDS); Lc, Gk: two LDS tiles of
// TILE_LDS doubles (Lc[k*LDL + i] = L(i, k), Gk[k*LDL + c] = G(k, c)).
// Outputs as described for PotrfTileArgs (A/lda: where mode 0 writes L and
// mode 1 writes G).
// COH: G (and L) are stored device-coherent; COH_SRC: src is global memory
// read device-coherent (false: a plain load, for LDS or same-workgroup data).
template <int CW, bool COH = false, bool COH_SRC = COH>
__device__ __forceinline__ void potrf_body(const double* src, int64_t lds, double* Lc,
                                           double* Gk, int* sbad, double* A, int64_t lda,
                                           double* Ginv, double* logdiag, int64_t* info,
                                           int64_t row0, int mode) {
  constexpr int NW = NB / CW;
  constexpr int NT = NW * 64;
  const int i = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x == 0) *sbad = NB;
  double r[CW], g[CW];
#pragma unroll
  for (int q = 0; q < CW; ++q) {
    r[q] = gload<COH_SRC>(&src[(int64_t)i + (int64_t)(CW * wv + q) * lds]);
    g[q] = (CW * wv + q == i) ? 1.0 : 0.0;
  }
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < NW; ++k) {
    const int c0 = CW * k;
    if (wv == k) {
      double rsv[CW], Ls[CW][CW];
      int bad = NB;
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        const int s = c0 + q;
        const double d = readlane_f64(r[q], s);
        const bool ok = d > 0.0;  // false for NaN too
        bad = ok ? bad : min(bad, s);
        const double rs = rsqrt_nr(ok ? d : __builtin_nan(""));
        rsv[q] = rs;
        r[q] = (i > s) ? r[q] * rs : (i == s ? d * rs : 0.0);
#pragma unroll
        for (int qq = q + 1; qq < CW; ++qq) {
          Ls[qq][q] = readlane_f64(r[q], c0 + qq);  // L(c0 + qq, s)
          r[qq] = __builtin_fma(-r[q], Ls[qq][q], r[qq]);
        }
      }
#pragma unroll
      for (int q = 0; q < CW; ++q) Lc[(c0 + q) * LDL + i] = r[q];
      // rows c0 .. of G: scale by 1/L(s, s), eliminate within the panel
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        g[q] *= rsv[q];
#pragma unroll
        for (int qq = q + 1; qq < CW; ++qq) g[qq] = __builtin_fma(-Ls[qq][q], g[q], g[qq]);
      }
#pragma unroll
      for (int q = 0; q < CW; ++q) Gk[(c0 + q) * LDL + i] = g[q];
      if (bad < NB && i == 0) atomicMin(sbad, bad);
    }
    __syncthreads();
    if (wv > k) {
      double li[CW], gi[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        li[q] = Lc[(c0 + q) * LDL + i];
        gi[q] = Gk[(c0 + q) * LDL + i];
      }
#pragma unroll
      for (int q = 0; q < CW; ++q) {
#pragma unroll
        for (int qq = 0; qq < CW; ++qq) {
          const double ls = Lc[(c0 + q) * LDL + CW * wv + qq];  // L(CW*wv + qq, c0 + q)
          r[qq] = __builtin_fma(-li[q], ls, r[qq]);
          g[qq] = __builtin_fma(-ls, gi[q], g[qq]);
        }
      }
    }
  }
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
      gstore<COH>(&dst[rr + cc * ldd], (rr >= cc) ? Gk[rr * LDL + cc] : 0.0);
    }
  }
}

__global__ __launch_bounds__(POTRF_NT) void k_potrf_tile(const PotrfTileArgs* __restrict__ args) {
  const PotrfTileArgs a = args[blockIdx.x];
  __shared__ __align__(16) double Lc[TILE_LDS];
  __shared__ __align__(16) double Gk[TILE_LDS];
  __shared__ int sbad;
  potrf_body<POTRF_CW>(a.A, a.lda, Lc, Gk, &sbad, a.A, a.lda, a.Ginv, a.logdiag, a.info,
                       a.row0, a.mode);
}

hipError_t launch_potrf_tiles(const PotrfTileArgs* args, int count,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_potrf_tile, dim3(count), dim3(POTRF_NT), 0, s, args);
  return hipGetLastError();
}

// ---- fused panel step ---------------------------------------------------------------
//
// Per tile, with the 64 x 64 operands staged in LDS (S0 = L(I, j), S2 =
// L(J, j)):  A(I, J) -= L(I, j) L(J, j)^T  on FP64 MFMA, one 16 x 16 block
// per wave, with the operand roles chosen so that a lane's results lie along
// the rows of the column-major output (coalesced stores).  Every global load
// (the operand tiles and the elements a lane updates) is issued before the
// first LDS store, so their latencies overlap.  The factoring workgroup
// stages its updated tile in LDS (S1) and runs the tile factor on it with S0
// and S2 as scratch.  A column workgroup also updates the diagonal tile j+1
// (from L(J, j) in S2: the factoring workgroup's product, bit for bit),
// factors it in LDS without writing it, and stores L(I, j+1) = A(I, j+1) G^T
// in place of its tile.  The inverse's workgroups form one or two tile
// products each (see PanelTask).

// S[k*LDL + r] = X(r, k) for the 64 x 64 tile X (ld), coalesced along r.
template <bool COH = false>
__device__ __forceinline__ void stage_cols(const double* __restrict__ X, int64_t ld, double* S) {
  for (int idx = threadIdx.x; idx < NB * NB; idx += POTRF_NT) {
    const int r = idx & 63, k = idx >> 6;
    S[k * LDL + r] = gload<COH>(&X[r + (int64_t)k * ld]);
  }
}

// S[k*LDL + r] = X(k, r) (the transpose), coalesced along k.
template <bool COH = false>
__device__ __forceinline__ void stage_rows(const double* __restrict__ X, int64_t ld, double* S) {
  for (int idx = threadIdx.x; idx < NB * NB; idx += POTRF_NT) {
    const int k = idx & 63, r = idx >> 6;
    S[k * LDL + r] = gload<COH>(&X[k + (int64_t)r * ld]);
  }
}

__device__ __forceinline__ double* stage_tile(const PanelTask& T, int r, int c) {
  return T.stage + ((int64_t)(r * (r - 1) / 2 + c)) * (NB * NB);
}

// The inverse's workgroups of step j (role 2: row j, column c; role 3:
// accumulator (r, c), r > j).  With X(r', c) the product Y X^T of staged
// tiles (mfma1_k64), lane results lie at (q0 + lr, p0 + lk + 4 rg).
__device__ void panel_inverse(const PanelTask& T, int role, int loc, double* S0, double* S1) {
  const int j = T.j;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = l >> 4;
  const int p0 = 16 * (wv >> 2), q0 = 16 * (wv & 3);
  const int64_t ld = T.ld;
  double* const A = T.A;
  auto tileA = [&](int r, int c) { return A + (int64_t)r * NB + (int64_t)c * NB * ld; };
  const int r = (role == 2) ? j : j + 1 + loc / j;
  const int c = (role == 2) ? loc : loc % j;
  if (role == 2 && c == 0 && j >= 2) {
    // G(j-1, j-2) from stage into place (L(j-1, j-2) is read no more)
    const double* src = stage_tile(T, j - 1, j - 2);
    double* dst = tileA(j - 1, j - 2);
    for (int idx = threadIdx.x; idx < NB * NB; idx += POTRF_NT)
      dst[(idx & 63) + (int64_t)(idx >> 6) * ld] = src[idx];
  }
  // G(j-1, c): the diagonal tile, the staged G(j-1, j-2), or in place
  const double* Gk;
  int64_t ldg;
  if (c == j - 1) { Gk = tileA(j - 1, j - 1); ldg = ld; }
  else if (c == j - 2) { Gk = stage_tile(T, j - 1, j - 2); ldg = NB; }
  else { Gk = tileA(j - 1, c); ldg = ld; }
  double prev[4] = {0.0, 0.0, 0.0, 0.0};
  if (c <= j - 2) {
    const double* Sp = stage_tile(T, r, c);
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) prev[rg] = Sp[(q0 + lr) + (p0 + lk + 4 * rg) * NB];
  }
  stage_cols(tileA(r, j - 1), ld, S0);  // Y = L(r, j-1)
  stage_rows(Gk, ldg, S1);              // X = G(j-1, c)^T
  __syncthreads();
  v4d t = {prev[0], prev[1], prev[2], prev[3]};
  mfma1_k64(S1, p0, S0, q0, t);         // t = S(r, c) + L(r, j-1) G(j-1, c)
  if (role == 3) {
    double* Sd = stage_tile(T, r, c);
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) Sd[(q0 + lr) + (p0 + lk + 4 * rg) * NB] = t[rg];
    return;
  }
  // G(j, c) = -G_jj t: G_jj from the side ring during the panel steps, in
  // place for the closing launch
  const double* Gjj = T.last ? tileA(j, j) : T.gside + (int64_t)(j & 1) * NB * NB;
  const int64_t ldj = T.last ? ld : NB;
  __syncthreads();  // S0, S1 are read no more
  stage_cols(Gjj, ldj, S0);             // Y = G_jj
#pragma unroll
  for (int rg = 0; rg < 4; ++rg) S1[(q0 + lr) * LDL + p0 + lk + 4 * rg] = t[rg];  // X = t^T
  __syncthreads();
  v4d g = {0.0, 0.0, 0.0, 0.0};
  mfma1_k64(S1, p0, S0, q0, g, q0 + 16);  // G_jj is lower triangular
  double* dst;
  int64_t ldd;
  if (c == j - 1) { dst = stage_tile(T, j, j - 1); ldd = NB; }
  else { dst = tileA(j, c); ldd = ld; }
#pragma unroll
  for (int rg = 0; rg < 4; ++rg) dst[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * ldd] = -g[rg];
}

__global__ __launch_bounds__(POTRF_NT) void k_panel_update(const PanelTask* __restrict__ tasks,
                                                           int ntask) {
  __shared__ __align__(16) double pool[3 * TILE_LDS];
  __shared__ int sbad;
  double* S0 = pool;
  double* S1 = pool + TILE_LDS;
  double* S2 = pool + 2 * TILE_LDS;
  // role segments: 0 factor, 1 column, 2 inverse row, 3 inverse accumulate,
  // 4 rest; then the task whose share of the segment holds this workgroup
  int g = blockIdx.x, role = 0;
  while (role < 4 && g >= tasks[0].tot[role]) {
    g -= tasks[0].tot[role];
    ++role;
  }
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].beg[role] <= g) lo = mid; else hi = mid - 1;
  }
  const int loc = g - tasks[lo].beg[role];
  const PanelTask T = tasks[lo];
  if (role == 2 || role == 3) {
    panel_inverse(T, role, loc, S0, S1);
    return;
  }
  int I, J;
  if (role == 0) {
    I = J = 0;
  } else if (role == 1) {
    I = 1 + loc;
    J = 0;
  } else {
    // row-major enumeration of the lower triangle of tiles (I, J), J >= 1
    int R = (int)((sqrt(8.0 * (double)loc + 1.0) - 1.0) * 0.5);
    while ((R + 1) * (R + 2) / 2 <= loc) ++R;
    while (R * (R + 1) / 2 > loc) --R;
    I = R + 1;
    J = loc - R * (R + 1) / 2 + 1;
  }
  const int64_t ti0 = (int64_t)(T.j + 1 + I) * NB, tj0 = (int64_t)(T.j + 1 + J) * NB;
  const int64_t pc = (int64_t)T.j * NB * T.ld;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = l >> 4;
  const int p0 = 16 * (wv >> 2), q0 = 16 * (wv & 3);  // this wave's 16 x 16 block
  double* C = T.A + ti0 + tj0 * T.ld;
  const bool diag = (I == J);
  constexpr int PER = NB * NB / POTRF_NT;
  double vp[PER], vq[PER], cpre[4], dpre[4];
  {
    const double* Li = T.A + ti0 + pc;
    const double* Lj = T.A + tj0 + pc;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + e * POTRF_NT;
      const int64_t o = (idx & 63) + (int64_t)(idx >> 6) * T.ld;
      vp[e] = Li[o];
      vq[e] = diag ? 0.0 : Lj[o];
    }
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) cpre[rg] = C[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * T.ld];
    if (role == 1) {
      const double* Dj = T.A + (int64_t)(T.j + 1) * NB * (T.ld + 1);
#pragma unroll
      for (int rg = 0; rg < 4; ++rg)
        dpre[rg] = Dj[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * T.ld];
    }
    if (role == 0 && T.j >= 1) {
      // G_j from the side ring into diagonal tile j (read by nobody now)
      const double* src = T.gside + (int64_t)(T.j & 1) * NB * NB;
      double* dst = T.A + (int64_t)T.j * NB * (T.ld + 1);
      for (int idx = threadIdx.x; idx < NB * NB; idx += POTRF_NT)
        dst[(idx & 63) + (int64_t)(idx >> 6) * T.ld] = src[idx];
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = threadIdx.x + e * POTRF_NT;
      const int o = (idx >> 6) * LDL + (idx & 63);
      S0[o] = vp[e];
      if (!diag) S2[o] = vq[e];
    }
  }
  __syncthreads();
  // (L_I L_J^T)^T = L_J L_I^T: D[n][m] = sum_c L_J(n, c) L_I(m, c)
  const double* LJ = diag ? S0 : S2;
  v4d u0 = {0.0, 0.0, 0.0, 0.0};
  mfma1_k64(LJ, p0, S0, q0, u0);  // u: update(m = q0 + lr, n = p0 + lk + 4r)
  if (role == 4) {
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
      C[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * T.ld] = cpre[rg] - u0[rg];
    return;
  }
  if (role == 1) {
    // the diagonal tile j+1 updated exactly as the factoring workgroup does
    v4d v0 = {0.0, 0.0, 0.0, 0.0};
    mfma1_k64(S2, p0, S2, q0, v0);
    __syncthreads();  // S0, S2 are read no more
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) S1[(p0 + lk + 4 * rg) * LDL + q0 + lr] = dpre[rg] - v0[rg];
    __syncthreads();
    potrf_body<POTRF_CW>(S1, LDL, S0, S2, &sbad, nullptr, 0, nullptr, nullptr, nullptr, 0, 1);
    __syncthreads();
    // G staged as S1[k][r] = G(r, k) (zero above the diagonal); the updated
    // panel tile as S0[c][m] = A(m, c)
    for (int idx = threadIdx.x; idx < NB * NB; idx += POTRF_NT) {
      const int r = idx & 63, k = idx >> 6;
      S1[k * LDL + r] = (r >= k) ? S2[r * LDL + k] : 0.0;
    }
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) S0[(p0 + lk + 4 * rg) * LDL + q0 + lr] = cpre[rg] - u0[rg];
    __syncthreads();
    // L^T = G A^T: D[c][m] = sum_k G(c, k) A(m, k), k <= c < p0 + 16
    v4d a0 = {0.0, 0.0, 0.0, 0.0};
    mfma1_k64(S1, p0, S0, q0, a0, p0 + 16);  // L(m = q0 + lr, c = p0 + lk + 4r)
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
      C[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * T.ld] = a0[rg];
    return;
  }
  __syncthreads();  // S0 is read no more
#pragma unroll
  for (int rg = 0; rg < 4; ++rg) S1[(p0 + lk + 4 * rg) * LDL + q0 + lr] = cpre[rg] - u0[rg];
  __syncthreads();
  // while column j+1 below reads diagonal tile j+1, G_{j+1} goes to the ring
  const bool side = T.j + 2 < T.nbk;
  double* dst = side ? T.gside + (int64_t)((T.j + 1) & 1) * NB * NB : C;
  potrf_body<POTRF_CW>(S1, LDL, S0, S2, &sbad, dst, side ? NB : T.ld, nullptr, T.logdiag,
                       T.info, T.row0, 1);
}

int finalize_panels(PanelTask* t, int n) {
  int tot[5] = {0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    const int j = t[i].j, nbk = t[i].nbk;
    int cnt[5];
    if (t[i].last) {
      cnt[0] = cnt[1] = cnt[3] = cnt[4] = 0;
      cnt[2] = j;
    } else {
      const int m = nbk - j - 1;  // trailing tile rows (>= 1)
      cnt[0] = 1;
      cnt[1] = m - 1;
      cnt[2] = t[i].inv ? j : 0;
      cnt[3] = t[i].inv ? (nbk - 1 - j) * j : 0;
      cnt[4] = m * (m - 1) / 2;
    }
    for (int k = 0; k < 5; ++k) {
      t[i].beg[k] = tot[k];
      tot[k] += cnt[k];
    }
  }
  int grid = 0;
  for (int k = 0; k < 5; ++k) grid += tot[k];
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 5; ++k) t[i].tot[k] = tot[k];
  return grid;
}

hipError_t launch_panel_updates(const PanelTask* tasks, int ntask, int grid,
                                hipStream_t s) {
  if (ntask <= 0 || grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_update, dim3(grid), dim3(POTRF_NT), 0, s, tasks, ntask);
  return hipGetLastError();
}

// ---- persistent tile-task factorisation of diagonal blocks ----------------------------
//
// Workgroups of 16 waves take task words from the launch's list in order
// (one atomic add on head[0] each), wait until the counters the task depends
// on are set (one lane polls, 0.5 s limit), run the task on 64 x 64 tiles
// staged in two LDS tiles and set the task's counter.  The tile operations
// are those of the panel path: the same staging, the same MFMA products
// (mfma1_k64), the same tile factor (potrf_body).
//
// Hand-over between workgroups, which may sit on different XCDs (each with
// its own L2), without cache write-back or invalidation: every value a task
// writes for another task (A, G, L and accumulator tiles) is stored
// device-coherently (sc1), and every value that another task may have
// rewritten during the launch (A, G and accumulator tiles) is loaded
// device-coherently.  L tiles are written once per launch, after which
// nobody writes them, and nobody reads them before, so they are read through
// the caches (each is read by many update tasks).  A task's stores are
// complete (s_waitcnt) in every lane before the barrier after which its
// counter is set; the counters themselves are relaxed device-scope atomics.

namespace {
constexpr long long kDagWaitTicks = 50000000;  // 0.5 s of the 100 MHz constant clock
constexpr int DPER = NB * NB / POTRF_NT;        // elements of a tile per lane

typedef __attribute__((address_space(1))) int32_t gint;
__device__ __forceinline__ int dag_load(const int32_t* p) {
  return __hip_atomic_load((const gint*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dag_store(int32_t* p, int v) {
  __hip_atomic_store((gint*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// true once *p >= value; false after the time limit, or at once when the
// launch has given up (*abort set by a wait that timed out)
__device__ bool dag_wait(const int32_t* p, int value, int32_t* abort) {
  if (dag_load(p) >= value) return true;
  const long long t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    if (dag_load(p) >= value) return true;
    if (dag_load(abort) != 0) return false;
    if (wall_clock64() - t0 > kDagWaitTicks) {
      dag_store(abort, 1);
      return false;
    }
  }
}

// The lane's DPER elements of the 64 x 64 tile X (global, ld): element idx =
// threadIdx.x + e * POTRF_NT is X(idx & 63, idx >> 6).  All loads are issued
// before any is used.
template <bool COH>
__device__ __forceinline__ void tile_regs(const double* __restrict__ X, int64_t ld,
                                          double (&v)[DPER]) {
#pragma unroll
  for (int e = 0; e < DPER; ++e) {
    const int idx = threadIdx.x + e * POTRF_NT;
    const double* p = &X[(idx & 63) + (int64_t)(idx >> 6) * ld];
    v[e] = COH ? cload(p) : global_load(p);
  }
}
// as stage_cols: S[k*LDL + r] = X(r, k)
__device__ __forceinline__ void regs_to_cols(const double (&v)[DPER], double* S) {
#pragma unroll
  for (int e = 0; e < DPER; ++e) {
    const int idx = threadIdx.x + e * POTRF_NT;
    S[(idx >> 6) * LDL + (idx & 63)] = v[e];
  }
}
// as stage_rows: S[k*LDL + r] = X(k, r)
__device__ __forceinline__ void regs_to_rows(const double (&v)[DPER], double* S) {
#pragma unroll
  for (int e = 0; e < DPER; ++e) {
    const int idx = threadIdx.x + e * POTRF_NT;
    S[(idx & 63) * LDL + (idx >> 6)] = v[e];
  }
}
}  // namespace

__global__ __launch_bounds__(POTRF_NT) void k_dag_chol(const uint64_t* __restrict__ tasks,
                                                       int ntask,
                                                       const DagBlock* __restrict__ blocks,
                                                       int nblocks, int32_t* head) {
  __shared__ __align__(16) double pool[3 * TILE_LDS];
  __shared__ int s_task, s_bad, s_last;
  double* S0 = pool;
  double* S1 = pool + TILE_LDS;
  double* S2 = pool + 2 * TILE_LDS;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = l >> 4;
  const int p0 = 16 * (wv >> 2), q0 = 16 * (wv & 3);  // this wave's 16 x 16 block
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(head, 1);
    __syncthreads();
    const int ti = s_task;
    if (ti >= ntask) break;
    int bi = 0;
    const dag::Task t = dag::unpack(tasks[ti], &bi);
    const DagBlock B = blocks[bi];
    const int64_t ld = B.ld;
    auto tile = [&](double* base, int r, int c) {
      return base + (int64_t)r * NB + (int64_t)c * NB * ld;
    };
    if (threadIdx.x == 0) {
      dag::Wait w[4], set;
      const int nw = dag::waits_of(B.nbk, t, w, &set);
      bool ok = true;
      for (int e = 0; e < nw; ++e) ok = dag_wait(B.ctr + w[e].ctr, w[e].value, head + 2) && ok;
      if (!ok)
        atomicCAS((unsigned long long*)B.info, 0ull, (unsigned long long)(int64_t)DL_INFO_TIMEOUT);
    }
    __syncthreads();
    switch (t.type) {
      case dag::T_F: {
        double* Akk = tile(B.A, t.k, t.k);
        potrf_body<POTRF_CW, true>(Akk, ld, S0, S1, &s_bad, Akk, ld, nullptr,
                                   B.logdiag + (int64_t)t.k * NB, B.info,
                                   B.row0 + (int64_t)t.k * NB, 1);
        break;
      }
      case dag::T_C: {
        // S(k+1, k), then U(k+1, k+1, k) and F(k+1) on the tiles in LDS
        const int k = t.k, k1 = t.k + 1;
        double vg[DPER], va[DPER], dpre[4];
        tile_regs<true>(tile(B.A, k, k), ld, vg);    // G_kk
        tile_regs<true>(tile(B.A, k1, k), ld, va);   // A(k+1, k)
        double* Ad = tile(B.A, k1, k1);               // A(k+1, k+1), final but for U(., ., k)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) dpre[rg] = cload(&Ad[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * ld]);
        regs_to_cols(vg, S1);
        regs_to_cols(va, S0);
        __syncthreads();
        v4d a0 = {0.0, 0.0, 0.0, 0.0};
        mfma1_k64(S1, p0, S0, q0, a0, p0 + 16);  // L(m = q0 + lr, c = p0 + lk + 4r)
        double* Lo = tile(B.L, k1, k);
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
          cstore(&Lo[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * ld], a0[rg]);
          S2[(p0 + lk + 4 * rg) * LDL + q0 + lr] = a0[rg];  // S2[c][m] = L(m, c)
        }
        __syncthreads();
        v4d u0 = {0.0, 0.0, 0.0, 0.0};
        mfma1_k64(S2, p0, S2, q0, u0);  // (L L^T)(m = q0 + lr, n = p0 + lk + 4r)
        // the updated tile, column-major in S0 (read no more since the barrier)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) S0[(p0 + lk + 4 * rg) * LDL + q0 + lr] = dpre[rg] - u0[rg];
        // L(k+1, k) published once every lane's stores are complete (their
        // latency overlaps the update above)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
          dag::Wait m;
          dag::mid_set(t, &m);
          dag_store(B.ctr + m.ctr, m.value);
        }
        potrf_body<POTRF_CW, true, false>(S0, LDL, S1, S2, &s_bad, Ad, ld, nullptr,
                                          B.logdiag + (int64_t)k1 * NB, B.info,
                                          B.row0 + (int64_t)k1 * NB, 1);
        break;
      }
      case dag::T_S: {
        // L(i, k) = A(i, k) G_kk^T: S1[q][r] = G(r, q), S0[c][m] = A(m, c)
        double vg[DPER], va[DPER];
        tile_regs<true>(tile(B.A, t.k, t.k), ld, vg);
        tile_regs<true>(tile(B.A, t.i, t.k), ld, va);
        regs_to_cols(vg, S1);
        regs_to_cols(va, S0);
        __syncthreads();
        v4d a0 = {0.0, 0.0, 0.0, 0.0};
        mfma1_k64(S1, p0, S0, q0, a0, p0 + 16);  // L(m = q0 + lr, c = p0 + lk + 4r)
        double* Lo = tile(B.L, t.i, t.k);
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) cstore(&Lo[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * ld], a0[rg]);
        break;
      }
      case dag::T_U: {
        // A(i, k) -= L(i, j) L(k, j)^T
        const bool diag = t.i == t.k;
        double vp[DPER], vq[DPER], cpre[4];
        tile_regs<false>(tile(B.L, t.i, t.j), ld, vp);
        if (!diag) tile_regs<false>(tile(B.L, t.k, t.j), ld, vq);
        double* C = tile(B.A, t.i, t.k);
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) cpre[rg] = cload(&C[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * ld]);
        regs_to_cols(vp, S0);
        if (!diag) regs_to_cols(vq, S1);
        __syncthreads();
        v4d u0 = {0.0, 0.0, 0.0, 0.0};
        mfma1_k64(diag ? S0 : S1, p0, S0, q0, u0);  // update(m = q0 + lr, n = p0 + lk + 4r)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
          cstore(&C[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * ld], cpre[rg] - u0[rg]);
        break;
      }
      case dag::T_A:
      case dag::T_R: {
        // A(r, c, m): S(r, c) (+)= L(r, m) G(m, c);
        // R(j, c):    t = S(j, c) + L(j, j-1) G(j-1, c), G(j, c) = -G_jj t
        const bool row = t.type == dag::T_R;
        const int r = t.i, c = t.k, m = row ? t.i - 1 : t.j;
        double* Sd = B.stage + ((int64_t)r * (r - 1) / 2 + c) * (NB * NB);
        const bool acc = row ? (r - 1 > c) : (m > c);
        double prev[4] = {0.0, 0.0, 0.0, 0.0};
        if (acc) {
#pragma unroll
          for (int rg = 0; rg < 4; ++rg) prev[rg] = cload(&Sd[(q0 + lr) + (p0 + lk + 4 * rg) * NB]);
        }
        double vy[DPER], vx[DPER], vg[DPER];
        tile_regs<false>(tile(B.L, r, m), ld, vy);  // Y = L(r, m)
        tile_regs<true>(tile(B.A, m, c), ld, vx);   // X = G(m, c)
        if (row) tile_regs<true>(tile(B.A, r, r), ld, vg);  // G_jj, for the second product
        regs_to_cols(vy, S0);
        regs_to_rows(vx, S1);
        __syncthreads();
        v4d tv = {prev[0], prev[1], prev[2], prev[3]};
        mfma1_k64(S1, p0, S0, q0, tv);  // (Y X)(q0 + lr, p0 + lk + 4r)
        if (!row) {
#pragma unroll
          for (int rg = 0; rg < 4; ++rg) cstore(&Sd[(q0 + lr) + (p0 + lk + 4 * rg) * NB], tv[rg]);
          break;
        }
        __syncthreads();  // S0, S1 are read no more
        regs_to_cols(vg, S0);  // G_jj
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) S1[(q0 + lr) * LDL + p0 + lk + 4 * rg] = tv[rg];
        __syncthreads();
        v4d g = {0.0, 0.0, 0.0, 0.0};
        mfma1_k64(S1, p0, S0, q0, g, q0 + 16);  // G_jj is lower triangular
        double* dst = tile(B.A, r, c);
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) cstore(&dst[(q0 + lr) + (int64_t)(p0 + lk + 4 * rg) * ld], -g[rg]);
        break;
      }
    }
    // every lane's stores complete before the counter is set
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      dag::Wait w[4], set;
      (void)dag::waits_of(B.nbk, t, w, &set);
      dag_store(B.ctr + set.ctr, set.value);
    }
  }
  // the last workgroup out (every task is then complete) zeroes the
  // counters and the head for the next launch
  if (threadIdx.x == 0) s_last = atomicAdd(head + 1, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (s_last) {
    for (int b = 0; b < nblocks; ++b) {
      const int64_t nc = dag::counters_per_block(blocks[b].nbk);
      for (int64_t i = threadIdx.x; i < nc; i += POTRF_NT) dag_store(blocks[b].ctr + i, 0);
    }
    if (threadIdx.x == 0) {
      dag_store(head, 0);
      dag_store(head + 1, 0);
      dag_store(head + 2, 0);
    }
  }
}

hipError_t launch_dag_chol(const uint64_t* tasks, int ntask, const DagBlock* blocks,
                           int nblocks, int32_t* head, int workers, hipStream_t s) {
  if (ntask <= 0 || nblocks <= 0 || workers <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dag_chol, dim3(workers), dim3(POTRF_NT), 0, s, tasks, ntask, blocks,
                     nblocks, head);
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
    case MJ_AXPY_UNCONV:
      if (!(J.norms[0] <= J.tol2[0] * J.norms[1]))
        for (int64_t i = i0; i < J.n; i += stride) J.dst[i] += J.src[i];
      break;
    case MJ_COPY2D_TO_F32: {
      float* dst32 = (float*)J.dst;
      const int64_t tot = (int64_t)J.rows * J.cols;
      for (int64_t i = i0; i < tot; i += stride) {
        const int64_t r = i % J.rows, c = i / J.rows;
        dst32[r + c * J.ldd] = (float)J.src[r + c * J.lds];
      }
      break;
    }
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
