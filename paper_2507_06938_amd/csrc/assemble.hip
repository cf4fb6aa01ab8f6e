// theta -> coefficients, sparse-to-dense BTA assembly of Q_p and Q_c, the
// right-hand side A^T D y, quadratic forms and the f_obj combination.
#include <math.h>

#include "model.hpp"

namespace dl {

// ---- a1: theta -> model coefficients ------------------------------------------
//
// Parameters (internal theta): univariate [log kappa, phi, log tau_u,
// log tau_y]; coregional [log kappa_i, phi_i, log sigma_i, lambda_k,
// log tau_y_j], rho = tanh(phi/2).  Lambda is the lower-triangular matrix of
// Eq. 5; the joint precision has blocks (k, j) = sum_i (Lambda^-1)_{ik}
// (Lambda^-1)_{ij} Q^i (Eq. 11).  Separable family: Q^i = T^i (x) Q_s^i,
// Q_s = kappa^4 C + 2 kappa^2 G + G C^-1 G, T the unit-variance AR1
// precision.  Diffusion family (log gamma_s, log gamma_t in the slots of
// log kappa, phi): Q^i = M0 (x) K3 + 2 gamma_t M1 (x) K2 + gamma_t^2 M2 (x) K1
// with K1 = g C + G, K2 = g^2 C + 2g G + G C^-1 G, K3 = g^3 C + 3g^2 G +
// 3g G C^-1 G + G C^-1 G C^-1 G (g = gamma_s^2, the binomial expansion of
// K_{k+1} = K1 C^-1 K_k), M0 = 1/2 | 1 | 1/2, M1 = 1/2 | 0 | 1/2 and
// M2 = 1 | 2 | 1 on the diagonal (end | inside | end), -1 off it.  Either
// way Q^i's diagonal and sub-diagonal blocks are weighted sums of the four
// FEM pieces; wd/wb below hold those weights per process.
__global__ void k_theta_coeffs(const ThetaJob* __restrict__ jobs) {
  if (threadIdx.x != 0) return;
  const ThetaJob J = jobs[blockIdx.x];
  const ModelDev& m = *J.m;
  const double* __restrict__ theta = J.theta;
  double* __restrict__ coef = J.coef;
  const int nv = m.nv;
  double kap[3], rho[3], tau[3], Li[3][3];
  double Mw[3][3][3];
  int bad = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Li[i][j] = 0.0;
      for (int k = 0; k < 3; ++k) Mw[i][j][k] = 0.0;
    }
  // Poisson responses have no noise precision in theta (tau = 1, unused)
  const bool gauss = m.likelihood == DL_LIK_GAUSSIAN;
  if (nv == 1) {
    kap[0] = exp(theta[0]);
    rho[0] = tanh(0.5 * theta[1]);
    const double tau_u = exp(theta[2]);
    tau[0] = gauss ? exp(theta[3]) : 1.0;
    Mw[0][0][0] = tau_u;
  } else {
    const int nl = nv * (nv - 1) / 2;
    double sg[3], lam[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < nv; ++i) {
      kap[i] = exp(theta[i]);
      rho[i] = tanh(0.5 * theta[nv + i]);
      sg[i] = exp(theta[2 * nv + i]);
      tau[i] = gauss ? exp(theta[3 * nv + nl + i]) : 1.0;
    }
    for (int k = 0; k < nl; ++k) lam[k] = theta[3 * nv + k];
    // Lambda of Eq. 5 (nv = 2 keeps its leading 2x2 block)
    double L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    L[0][0] = sg[0];
    L[1][0] = lam[0] * sg[0];
    L[1][1] = sg[1];
    if (nv == 3) {
      L[2][0] = (lam[2] + lam[0] * lam[1]) * sg[0];
      L[2][1] = lam[1] * sg[1];
      L[2][2] = sg[2];
    }
    // inverse of the lower-triangular Lambda, column by column
    for (int c = 0; c < nv; ++c) {
      for (int r = 0; r < nv; ++r) {
        if (r < c) { Li[r][c] = 0.0; continue; }
        double acc = (r == c) ? 1.0 : 0.0;
        for (int k = c; k < r; ++k) acc -= L[r][k] * Li[k][c];
        Li[r][c] = acc / L[r][r];
      }
    }
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < nv; ++j)
        for (int k = 0; k < nv; ++k) Mw[i][j][k] = Li[i][j] * Li[i][k];
  }
  // wd[i][tt][c]: weight of FEM piece c in a diagonal block of Q^i (tt = 0
  // end step, 1 inside, 2 single step); wb[i][c]: sub-diagonal block
  double wd[3][3][NPIECE], wb[3][NPIECE];
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < NPIECE; ++c) {
      wb[i][c] = 0.0;
      for (int tt = 0; tt < 3; ++tt) wd[i][tt][c] = 0.0;
    }
  const bool diffusion = m.family == DL_MODEL_DIFFUSION;
  for (int i = 0; i < nv; ++i) {
    if (!isfinite(kap[i]) || !isfinite(tau[i])) bad = 1;
    if (diffusion) {
      const double g = kap[i] * kap[i];
      const double gt = exp(theta[nv + i]);
      if (!isfinite(gt)) bad = 1;
      const double K1[NPIECE] = {g, 1.0, 0.0, 0.0};
      const double K2[NPIECE] = {g * g, 2.0 * g, 1.0, 0.0};
      const double K3[NPIECE] = {g * g * g, 3.0 * g * g, 3.0 * g, 1.0};
      for (int c = 0; c < NPIECE; ++c) {
        wd[i][0][c] = 0.5 * K3[c] + gt * K2[c] + gt * gt * K1[c];
        wd[i][1][c] = K3[c] + 2.0 * gt * gt * K1[c];
        wd[i][2][c] = wd[i][0][c];  // nt = 1 is rejected at model creation
        wb[i][c] = -gt * gt * K1[c];
      }
    } else {
      const double k2 = kap[i] * kap[i];
      const double q[NPIECE] = {k2 * k2, 2.0 * k2, 1.0, 0.0};
      const double r = rho[i];
      const double den = 1.0 - r * r;
      if (!(den > 0.0)) bad = 1;
      const double Tend = 1.0 / den, Tmid = (1.0 + r * r) / den, Toff = -r / den;
      for (int c = 0; c < NPIECE; ++c) {
        wd[i][0][c] = Tend * q[c];
        wd[i][1][c] = Tmid * q[c];
        wd[i][2][c] = q[c];
        wb[i][c] = Toff * q[c];
      }
    }
  }
  for (int tt = 0; tt < 3; ++tt)
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j)
        for (int c = 0; c < NPIECE; ++c) {
          double v = 0.0;
          if (k < nv && j < nv)
            for (int i = 0; i < nv; ++i) v += Mw[i][k][j] * wd[i][tt][c];
          coef[C_D + ((tt * 3 + k) * 3 + j) * NPIECE + c] = v;
        }
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < NPIECE; ++c) {
        double v = 0.0;
        if (k < nv && j < nv)
          for (int i = 0; i < nv; ++i) v += Mw[i][k][j] * wb[i][c];
        coef[C_B + (k * 3 + j) * NPIECE + c] = v;
      }
  const double two_pi = 6.283185307179586476925286766559;
  double lp = 0.0;
  const double sd = m.theta_prior_sd;
  for (int d = 0; d < m.dim_theta; ++d) {
    const double z = (theta[d] - m.theta_prior_mean[d]) / sd;
    lp += -0.5 * log(two_pi * sd * sd) - 0.5 * z * z;
  }
  double llc = 0.0;
  for (int j = 0; j < nv; ++j) {
    const double mj = (double)(m.m_off[j + 1] - m.m_off[j]);
    if (gauss) llc += 0.5 * mj * log(tau[j]) - 0.5 * mj * log(two_pi);
    coef[C_TAU + j] = tau[j];
  }
  for (int d = 0; d < m.dim_theta; ++d)
    if (!isfinite(theta[d])) bad = 1;
  coef[C_LOGPRIOR] = lp;
  coef[C_LLCONST] = llc;
  coef[C_BAD] = bad ? 1.0 : 0.0;
}

hipError_t launch_theta_coeffs(const ThetaJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_theta_coeffs, dim3(count), dim3(64), 0, s, jobs);
  return hipGetLastError();
}

// ---- a2: sparse -> dense BTA assembly --------------------------------------------
//
// One workgroup builds column c of time step t in LDS and writes it, whole
// and coalesced, to the dense blocks: the diagonal block D_t (lower triangle;
// rows above c are written as zero), the sub-diagonal block B_t of rows t+1,
// and for Q_c the arrow block R_t.  Q_c's column is Q_p's plus the
// observation terms tau_j w w^T (Eq. 4; d_row w w^T with the per-row weights
// of a non-Gaussian likelihood), added by one thread in a fixed order
// so the result does not depend on scheduling.  Padding columns c >= b
// (up to the padded block size bp) carry a unit diagonal, which leaves the
// log-determinant unchanged.
__global__ __launch_bounds__(256) void k_assemble_cols(const AsmJob* __restrict__ jobs) {
  extern __shared__ double lds[];
  const AsmJob J = jobs[blockIdx.z];
  const ModelDev& m = *J.m;
  const AssembleOut& o = J.o;
  const int c = blockIdx.x;
  const int tl = blockIdx.y;
  const int bp = m.bp, ap = m.ap, ns = m.ns, nv = m.nv;
  if (c >= bp || tl >= J.nt) return;
  const int t = J.t0 + tl;
  const int tid = threadIdx.x;
  const int64_t ldbr = bp + ap;
  double* colD = lds;            // bp
  double* colB = lds + bp;       // bp
  double* colR = lds + 2 * bp;   // ap (<= 64)
  __shared__ double rhs_s;
  const bool hasB = t + 1 < m.nt;
  double* Dp = o.Dp ? o.Dp + tl * o.dp_stride + (int64_t)c * bp : nullptr;
  double* Bp = o.Bp ? o.Bp + tl * o.bp_stride + (int64_t)c * bp : nullptr;
  double* Dc = o.Dc ? o.Dc + tl * o.dc_stride + (int64_t)c * bp : nullptr;
  double* BRc = o.BRc ? o.BRc + tl * o.brc_stride + (int64_t)c * ldbr : nullptr;

  const bool b32 = o.b32 != 0;
  float* Bp32 = o.Bp ? (float*)o.Bp + tl * o.bp_stride + (int64_t)c * bp : nullptr;
  float* BRc32 = o.BRc ? (float*)o.BRc + tl * o.brc_stride + (int64_t)c * ldbr : nullptr;
  if (c >= m.b) {
    for (int r = tid; r < bp; r += 256) {
      const double v = (r == c) ? 1.0 : 0.0;
      if (Dp) Dp[r] = v;
      if (Bp) { if (b32) Bp32[r] = 0.f; else Bp[r] = 0.0; }
      if (Dc) Dc[r] = v;
    }
    if (BRc)
      for (int r = tid; r < bp + ap; r += 256) {
        if (b32) BRc32[r] = 0.f; else BRc[r] = 0.0;
      }
    if (Dc && tid == 0) o.rhs[(int64_t)t * bp + c] = 0.0;
    return;
  }
  const int j = c / ns;
  const int s = c - j * ns;
  for (int r = tid; r < 2 * bp + ap; r += 256) lds[r] = 0.0;
  __syncthreads();
  const int tt = (m.nt == 1) ? 2 : ((t == 0 || t == m.nt - 1) ? 0 : 1);
  const int e0 = m.sp_ptr[s], e1 = m.sp_ptr[s + 1];
  const int ne = (e1 - e0) * nv;
  for (int idx = tid; idx < ne; idx += 256) {
    const int e = e0 + idx / nv;
    const int k = idx % nv;
    const int r = k * ns + m.sp_col[e];
    const double pc = m.sp_C[e], pg = m.sp_G[e], pg2 = m.sp_G2[e], pg3 = m.sp_G3[e];
    const double* cd = J.coef + C_D + ((tt * 3 + k) * 3 + j) * NPIECE;
    colD[r] = cd[0] * pc + cd[1] * pg + cd[2] * pg2 + cd[3] * pg3;
    if (hasB) {
      const double* cb = J.coef + C_B + (k * 3 + j) * NPIECE;
      colB[r] = cb[0] * pc + cb[1] * pg + cb[2] * pg2 + cb[3] * pg3;
    }
  }
  __syncthreads();
  if (Dp)
    for (int r = tid; r < bp; r += 256) Dp[r] = (r >= c) ? colD[r] : 0.0;
  if (Bp)
    for (int r = tid; r < bp; r += 256) {
      if (b32) Bp32[r] = (float)colB[r]; else Bp[r] = colB[r];
    }
  if (!Dc) return;
  __syncthreads();
  if (tid == 0) {
    const double tau = J.coef[C_TAU + j];
    const double* __restrict__ od = o.obs_d;
    const double* __restrict__ oz = o.obs_z;
    const int64_t key = ((int64_t)j * m.nt + t) * ns + s;
    double racc = 0.0;
    const int nr = m.nr;
    for (int64_t p = m.no_ptr[key]; p < m.no_ptr[key + 1]; ++p) {
      const int64_t row = m.no_row[p];
      const int qs = m.no_q[p];
      const double wq = m.obs_w[row * 3 + qs];
      const double wr = od ? od[row] : tau;
      for (int q2 = 0; q2 < 3; ++q2) {
        const int r = j * ns + m.obs_nodes[row * 3 + q2];
        colD[r] += wr * m.obs_w[row * 3 + q2] * wq;
      }
      for (int rr = 0; rr < nr; ++rr)
        colR[j * nr + rr] += wr * m.obs_x[row * nr + rr] * wq;
      racc += od ? wq * oz[row] : tau * wq * m.obs_y[row];
    }
    rhs_s = racc;
  }
  __syncthreads();
  for (int r = tid; r < bp; r += 256) {
    Dc[r] = (r >= c) ? colD[r] : 0.0;
    if (b32) BRc32[r] = (float)colB[r]; else BRc[r] = colB[r];
  }
  for (int r = tid; r < ap; r += 256) {
    if (b32) BRc32[bp + r] = (float)colR[r]; else BRc[bp + r] = colR[r];
  }
  if (tid == 0) o.rhs[(int64_t)t * bp + c] = rhs_s;
}

// Tips (a x a, identity-padded to ap) and the fixed-effect part of the
// right-hand side.  Workgroup 0 writes every tip entry outside the
// per-response covariate blocks; workgroup 1 + e computes one covariate
// Gram entry (response j, r >= r2) or one right-hand-side entry, summing
// the response's rows with a fixed reduction tree.
__global__ __launch_bounds__(256) void k_assemble_tip(const AsmJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const AsmJob J = jobs[blockIdx.y];
  const ModelDev& m = *J.m;
  const AssembleOut& o = J.o;
  const double* __restrict__ coef = J.coef;
  const int tid = threadIdx.x;
  if (m.ap == 0) return;
  const int nr = m.nr, nv = m.nv, ap = m.ap, a = m.a;
  const int ngram = nv * nr * nr;
  if (blockIdx.x == 0) {
    for (int idx = tid; idx < ap * ap; idx += 256) {
      const int r = idx % ap, cc = idx / ap;
      double vp = 0.0;
      if (r == cc) vp = (r < a) ? m.prior_fixed : 1.0;
      if (o.Pp) o.Pp[idx] = (r >= cc) ? vp : 0.0;
      const bool own = r < a && cc < a && (r / (nr > 0 ? nr : 1)) ==
                                              (cc / (nr > 0 ? nr : 1));
      if (o.Pc && !(own && r >= cc)) o.Pc[idx] = (r >= cc) ? vp : 0.0;
    }
    if (o.Pc)
      for (int i = a + tid; i < ap; i += 256) o.rhs[(int64_t)m.nt * m.bp + i] = 0.0;
    return;
  }
  if (!o.Pc) return;
  int e = blockIdx.x - 1;
  if (e >= ngram + nv * nr) return;
  int j, r, r2;
  bool gram = e < ngram;
  if (gram) {
    j = e / (nr * nr);
    const int rem = e % (nr * nr);
    r = rem / nr;
    r2 = rem % nr;
    if (r2 > r) return;
  } else {
    e -= ngram;
    j = e / nr;
    r = e % nr;
    r2 = 0;
  }
  const int64_t b0 = m.m_off[j], b1 = m.m_off[j + 1];
  const double* __restrict__ od = o.obs_d;
  const double* __restrict__ oz = o.obs_z;
  double acc = 0.0;
  for (int64_t row = b0 + tid; row < b1; row += 256) {
    const double xr = m.obs_x[row * nr + r];
    if (od)  // per-row weights: sum d x_r x_r2 and x_r z, no tau
      acc += gram ? od[row] * xr * m.obs_x[row * nr + r2] : xr * oz[row];
    else
      acc += gram ? xr * m.obs_x[row * nr + r2] : xr * m.obs_y[row];
  }
  sh[tid] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) sh[tid] += sh[tid + st];
    __syncthreads();
  }
  if (tid == 0) {
    const double tau = od ? 1.0 : coef[C_TAU + j];
    if (gram) {
      const int rr = j * nr + r, cc = j * nr + r2;
      o.Pc[rr + (int64_t)cc * ap] = tau * sh[0] + (rr == cc ? m.prior_fixed : 0.0);
    } else {
      o.rhs[(int64_t)m.nt * m.bp + j * nr + r] = tau * sh[0];
    }
  }
}

hipError_t launch_assemble_cols(const AsmJob* jobs, int count, int max_bp,
                                int max_nt, int max_shmem_doubles, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t shmem = (size_t)max_shmem_doubles * sizeof(double);
  hipLaunchKernelGGL(k_assemble_cols, dim3(max_bp, max_nt, count), dim3(256),
                     shmem, s, jobs);
  return hipGetLastError();
}

// Allow the column kernel its dynamic LDS (2*bp + ap doubles) beyond the
// default 64 KiB; called once per workspace, outside any graph capture.
hipError_t prepare_assemble(int max_shmem_doubles) {
  const size_t shmem = (size_t)max_shmem_doubles * sizeof(double);
  if (shmem <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)k_assemble_cols,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
}

// max_blocks = 1 + max over jobs of nv*nr*nr + nv*nr
hipError_t launch_assemble_tips(const AsmJob* jobs, int count, int max_blocks,
                                hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble_tip, dim3(max_blocks, count), dim3(256), 0, s,
                     jobs);
  return hipGetLastError();
}

// ---- a8: quadratic forms --------------------------------------------------------
//
// mu^T Q_p mu with Q_p applied from its stencil (no dense blocks): row
// (t, k, s') of Q_p mu = sum over time neighbours t' in {t-1, t, t+1},
// responses j and spatial neighbours s of coef(t,t')_{kj} . (C, G, GC^-1G,
// GC^-1GC^-1G) at (s', s) times mu(t', j, s); fixed effects add
// prior_fixed * |mu_f|^2.
// (y - A mu)^T D (y - A mu) row by row (Poisson: -2 log l(y | A mu) with
// log(y!) = lgamma(y + 1)).  Both are reduced with a fixed tree per block,
// then over blocks in order.
__device__ __forceinline__ double blk_sum(double v, double* sh) {
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

__global__ __launch_bounds__(256) void k_quad_prior(const QuadJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const QuadJob Q = jobs[blockIdx.y];
  const ModelDev& m = *Q.m;
  const double* __restrict__ coef = Q.coef;
  const double* __restrict__ mu = Q.mu;
  double* __restrict__ partial = Q.partial;
  const int64_t nrows = (int64_t)m.nt * m.b;
  const int ns = m.ns, nv = m.nv, bp = m.bp;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nrows;
       i += (int64_t)gridDim.x * 256) {
    const int t = (int)(i / m.b);
    const int rl = (int)(i - (int64_t)t * m.b);
    const int k = rl / ns, sp = rl - k * ns;
    const int tt = (m.nt == 1) ? 2 : ((t == 0 || t == m.nt - 1) ? 0 : 1);
    double qmu = 0.0;
    for (int dt = -1; dt <= 1; ++dt) {
      const int t2 = t + dt;
      if (t2 < 0 || t2 >= m.nt) continue;
      for (int j = 0; j < nv; ++j) {
        const double* cf = (dt == 0) ? coef + C_D + ((tt * 3 + k) * 3 + j) * NPIECE
                                     : coef + C_B + (k * 3 + j) * NPIECE;
        const double* x = mu + (int64_t)t2 * bp + j * ns;
        for (int e = m.sp_ptr[sp]; e < m.sp_ptr[sp + 1]; ++e) {
          const double qv = cf[0] * m.sp_C[e] + cf[1] * m.sp_G[e] + cf[2] * m.sp_G2[e] +
                            cf[3] * m.sp_G3[e];
          qmu += qv * x[m.sp_col[e]];
        }
      }
    }
    acc += mu[(int64_t)t * bp + rl] * qmu;
  }
  if (blockIdx.x == 0)
    for (int f = threadIdx.x; f < m.a; f += 256) {
      const double v = mu[(int64_t)m.nt * bp + f];
      acc += m.prior_fixed * v * v;
    }
  const double s = blk_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_quad_obs(const QuadJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const QuadJob Q = jobs[blockIdx.y];
  const ModelDev& m = *Q.m;
  const double* __restrict__ coef = Q.coef;
  const double* __restrict__ mu = Q.mu;
  double* __restrict__ partial = Q.partial + QF_BLOCKS;
  const int ns = m.ns, nr = m.nr, bp = m.bp;
  double acc = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x; row < m.m_total;
       row += (int64_t)gridDim.x * 256) {
    int j = 0;
    while (j + 1 < m.nv && row >= m.m_off[j + 1]) ++j;
    const int t = m.obs_t[row];
    const double* x = mu + (int64_t)t * bp + j * ns;
    double pred = 0.0;
    for (int q = 0; q < 3; ++q) pred += m.obs_w[row * 3 + q] * x[m.obs_nodes[row * 3 + q]];
    const double* xf = mu + (int64_t)m.nt * bp + j * nr;
    for (int r = 0; r < nr; ++r) pred += m.obs_x[row * nr + r] * xf[r];
    const double y = m.obs_y[row];
    if (m.likelihood == DL_LIK_POISSON) {
      acc += -2.0 * (y * pred - exp(pred) - lgamma(y + 1.0));
    } else {
      const double res = y - pred;
      acc += coef[C_TAU + j] * res * res;
    }
  }
  const double s = blk_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_quad_final(const QuadJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const QuadJob Q = jobs[blockIdx.x];
  const double* partial = Q.partial;
  double* out2 = Q.out2;
  for (int w = 0; w < 2; ++w) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < QF_BLOCKS; i += 256) acc += partial[w * QF_BLOCKS + i];
    const double s = blk_sum(acc, sh);
    if (threadIdx.x == 0) out2[w] = s;
  }
}

hipError_t launch_quadforms(const QuadJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quad_prior, dim3(QF_BLOCKS, count), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(k_quad_obs, dim3(QF_BLOCKS, count), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(k_quad_final, dim3(count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

// f_obj of Eq. 8 at x = mu, where the Gaussian p_G term has zero quadratic
// part and the (2 pi)^{-N/2} factors of Eq. 1 and Eq. 3 cancel:
// f = log p(theta) + [sum_j m_j/2 log tau_j - m/2 log 2pi - 1/2 quad_obs]
//     + 1/2 log|Q_p| - 1/2 mu^T Q_p mu - 1/2 log|Q_c|.
__global__ void k_combine(const CombineJob* __restrict__ jobs) {
  if (threadIdx.x != 0) return;
  const CombineJob C = jobs[blockIdx.x];
  const double* coef = C.coef;
  const double* logdet2 = C.logdet2;
  const int64_t* info2 = C.info2;
  const double* quad2 = C.quad2;
  double* f = C.f;
  dl_fobj_parts* parts = C.parts;
  int64_t* info_out = C.info_out;
  const double lp = coef[C_LOGPRIOR];
  const double llc = coef[C_LLCONST];
  double v = lp + llc - 0.5 * quad2[1] + 0.5 * logdet2[0] - 0.5 * quad2[0] -
             0.5 * logdet2[1];
  const bool fail = info2[0] != 0 || info2[1] != 0 || coef[C_BAD] != 0.0 ||
                    !isfinite(v);
  if (fail) v = -__builtin_inf();
  if (f) f[0] = v;
  if (parts) {
    parts->f = v;
    parts->logdet_p = logdet2[0];
    parts->logdet_c = logdet2[1];
    parts->quad_p = quad2[0];
    parts->quad_obs = quad2[1];
    parts->log_prior = lp;
    parts->log_lik_const = llc;
    parts->rel_residual = C.rnorm ? sqrt(C.rnorm[0] / (C.rnorm[1] > 0.0 ? C.rnorm[1] : 1.0)) : 0.0;
  }
  if (info_out) {
    info_out[0] = info2[0];
    info_out[1] = info2[1];
    // a refined mean whose residual missed the tolerance (the pivots were
    // fine): reported, f is kept
    if (info2[1] == 0 && C.tol2 && C.rnorm &&
        !(C.rnorm[0] <= C.tol2[0] * C.rnorm[1]))
      info_out[1] = DL_INFO_NOTCONV;
  }
}

hipError_t launch_combine(const CombineJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3(count), dim3(64), 0, s, jobs);
  return hipGetLastError();
}

// padded (t*bp + i, arrow at nt*bp) <-> packed (t*b + i, arrow at nt*b)
__global__ void k_pack(ModelDev m, const double* __restrict__ in,
                       double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m.N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = i / m.b;
    const int64_t src = (t < m.nt) ? t * m.bp + (i - t * m.b)
                                   : (int64_t)m.nt * m.bp + (i - (int64_t)m.nt * m.b);
    out[i] = in[src];
  }
}

__global__ void k_unpack(ModelDev m, const double* __restrict__ in,
                         double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m.Np;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = i / m.bp;
    double v = 0.0;
    if (t < m.nt) {
      const int64_t r = i - t * m.bp;
      if (r < m.b) v = in[t * m.b + r];
    } else {
      const int64_t r = i - (int64_t)m.nt * m.bp;
      if (r < m.a) v = in[(int64_t)m.nt * m.b + r];
    }
    out[i] = v;
  }
}

hipError_t launch_pack(const ModelDev& m, const double* padded, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(1024), dim3(256), 0, s, m, padded, out);
  return hipGetLastError();
}

hipError_t launch_unpack(const ModelDev& m, const double* in, double* padded,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(1024), dim3(256), 0, s, m, in, padded);
  return hipGetLastError();
}

// ---- FP64 residual of the conditional system (iterative refinement) ------------
//
// out = rhs - Q_c v with Q_c = Q_p + A^T D A, Q_p applied from its stencil as
// in the quadratic form above and A^T D A as (A v) per observation row
// followed by a gather over the rows touching each node (no atomics).
__global__ __launch_bounds__(256) void k_res_av(const ResJob* __restrict__ jobs) {
  const ResJob R = jobs[blockIdx.y];
  const ModelDev& m = *R.m;
  const int ns = m.ns, nr = m.nr, bp = m.bp;
  for (int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x; row < m.m_total;
       row += (int64_t)gridDim.x * 256) {
    int j = 0;
    while (j + 1 < m.nv && row >= m.m_off[j + 1]) ++j;
    const int t = m.obs_t[row];
    const double* x = R.v + (int64_t)t * bp + j * ns;
    double a = 0.0;
    for (int q = 0; q < 3; ++q) a += m.obs_w[row * 3 + q] * x[m.obs_nodes[row * 3 + q]];
    const double* xf = R.v + (int64_t)m.nt * bp + j * nr;
    for (int r = 0; r < nr; ++r) a += m.obs_x[row * nr + r] * xf[r];
    R.av[row] = (R.obs_d ? R.obs_d[row] : R.coef[C_TAU + j]) * a;
  }
}

__global__ __launch_bounds__(256) void k_res_rows(const ResJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const ResJob R = jobs[blockIdx.y];
  const ModelDev& m = *R.m;
  const double* __restrict__ coef = R.coef;
  const int ns = m.ns, nv = m.nv, bp = m.bp;
  const int64_t nrows = (int64_t)m.nt * m.b;
  double acc_r = 0.0, acc_b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nrows;
       i += (int64_t)gridDim.x * 256) {
    const int t = (int)(i / m.b);
    const int rl = (int)(i - (int64_t)t * m.b);
    const int k = rl / ns, sp = rl - k * ns;
    const int tt = (m.nt == 1) ? 2 : ((t == 0 || t == m.nt - 1) ? 0 : 1);
    double q = 0.0;
    for (int dt = -1; dt <= 1; ++dt) {
      const int t2 = t + dt;
      if (t2 < 0 || t2 >= m.nt) continue;
      for (int j = 0; j < nv; ++j) {
        const double* cf = (dt == 0) ? coef + C_D + ((tt * 3 + k) * 3 + j) * NPIECE
                                     : coef + C_B + (k * 3 + j) * NPIECE;
        const double* x = R.v + (int64_t)t2 * bp + j * ns;
        for (int e = m.sp_ptr[sp]; e < m.sp_ptr[sp + 1]; ++e) {
          const double qv = cf[0] * m.sp_C[e] + cf[1] * m.sp_G[e] + cf[2] * m.sp_G2[e] +
                            cf[3] * m.sp_G3[e];
          q += qv * x[m.sp_col[e]];
        }
      }
    }
    const int64_t key = ((int64_t)k * m.nt + t) * ns + sp;
    for (int64_t p = m.no_ptr[key]; p < m.no_ptr[key + 1]; ++p)
      q += m.obs_w[(int64_t)m.no_row[p] * 3 + m.no_q[p]] * R.av[m.no_row[p]];
    const int64_t o = (int64_t)t * bp + rl;
    const double res = R.rhs[o] - q;
    R.out[o] = res;
    acc_r += res * res;
    acc_b += R.rhs[o] * R.rhs[o];
  }
  const double s1 = blk_sum(acc_r, sh);
  const double s2 = blk_sum(acc_b, sh);
  if (threadIdx.x == 0) {
    R.partial[blockIdx.x] = s1;
    R.partial[QF_BLOCKS + blockIdx.x] = s2;
  }
}

// fixed-effect rows (one workgroup per (response, effect)) and the final
// norms; padded entries of out are zero
__global__ __launch_bounds__(256) void k_res_tip(const ResJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const ResJob R = jobs[blockIdx.y];
  const ModelDev& m = *R.m;
  const int nr = m.nr, nv = m.nv;
  const int e = blockIdx.x;
  const int64_t base = (int64_t)m.nt * m.bp;
  if (e < nv * nr) {
    const int j = e / nr, r = e % nr;
    double acc = 0.0;
    for (int64_t row = m.m_off[j] + threadIdx.x; row < m.m_off[j + 1]; row += 256)
      acc += m.obs_x[row * nr + r] * R.av[row];
    const double s = blk_sum(acc, sh);
    if (threadIdx.x == 0) {
      const int64_t o = base + e;
      const double q = s + m.prior_fixed * R.v[o];
      R.out[o] = R.rhs[o] - q;
    }
    return;
  }
  if (e == nv * nr) {
    // padding rows and columns of the blocks carry zeros
    for (int t = 0; t < m.nt; ++t)
      for (int i = m.b + threadIdx.x; i < m.bp; i += 256) R.out[(int64_t)t * m.bp + i] = 0.0;
    for (int i = m.a + threadIdx.x; i < m.ap; i += 256) R.out[base + i] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_res_final(const ResJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const ResJob R = jobs[blockIdx.x];
  const ModelDev& m = *R.m;
  double a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < QF_BLOCKS; i += 256) {
    a1 += R.partial[i];
    a2 += R.partial[QF_BLOCKS + i];
  }
  const int64_t base = (int64_t)m.nt * m.bp;
  if (threadIdx.x == 0)
    for (int f = 0; f < m.a; ++f) {
      a1 += R.out[base + f] * R.out[base + f];
      a2 += R.rhs[base + f] * R.rhs[base + f];
    }
  const double s1 = blk_sum(a1, sh);
  const double s2 = blk_sum(a2, sh);
  if (threadIdx.x == 0) {
    R.norms[0] = s1;
    R.norms[1] = s2;
  }
}

hipError_t launch_residual(const ResJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_res_av, dim3(QF_BLOCKS, count), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(k_res_rows, dim3(QF_BLOCKS, count), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(k_res_tip, dim3(3 * 64 + 1, count), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(k_res_final, dim3(count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

// ---- inner Newton iteration of a Poisson likelihood -----------------------------
//
// Observation weights from the current iterate x: eta = (A x)_row (its three
// barycentric nodes at its time step and its covariates), D = exp(eta) and
// the right-hand-side value z = (y - exp(eta)) + D eta, which the assembly
// gathers into A^T z.
__global__ __launch_bounds__(256) void k_lap_weights(const LapJob* __restrict__ jobs) {
  const LapJob J = jobs[blockIdx.y];
  const ModelDev& m = *J.m;
  const int ns = m.ns, nr = m.nr, bp = m.bp;
  for (int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x; row < m.m_total;
       row += (int64_t)gridDim.x * 256) {
    int j = 0;
    while (j + 1 < m.nv && row >= m.m_off[j + 1]) ++j;
    const int t = m.obs_t[row];
    const double* x = J.x + (int64_t)t * bp + j * ns;
    double eta = 0.0;
    for (int q = 0; q < 3; ++q) eta += m.obs_w[row * 3 + q] * x[m.obs_nodes[row * 3 + q]];
    const double* xf = J.x + (int64_t)m.nt * bp + j * nr;
    for (int r = 0; r < nr; ++r) eta += m.obs_x[row * nr + r] * xf[r];
    const double d = exp(eta);
    J.obs_d[row] = d;
    J.obs_z[row] = (m.obs_y[row] - d) + d * eta;
  }
}

hipError_t launch_lap_weights(const LapJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lap_weights, dim3(QF_BLOCKS, count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

__device__ __forceinline__ double blk_max(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// mu = x + alpha (xN - x) over the padded vector (alpha = 0 keeps x exactly:
// an instance that has converged), with the block maxima of |xN - x| and
// |xN| (NaN propagates through fmax only when both operands are NaN, so a
// non-finite entry is flagged as +inf).
__global__ __launch_bounds__(256) void k_trial(const TrialJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const TrialJob T = jobs[blockIdx.y];
  const int64_t n = T.m->Np;
  const double a = *T.alpha;
  double dmax = 0.0, nmax = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const double xi = T.x[i], xn = T.xN[i];
    T.mu[i] = (a == 0.0) ? xi : xi + a * (xn - xi);
    const double dv = fabs(xn - xi), nv = fabs(xn);
    dmax = fmax(dmax, isfinite(dv) ? dv : __builtin_inf());
    nmax = fmax(nmax, isfinite(nv) ? nv : __builtin_inf());
  }
  const double d = blk_max(dmax, sh);
  const double v = blk_max(nmax, sh);
  if (threadIdx.x == 0) {
    T.partial[blockIdx.x] = d;
    T.partial[QF_BLOCKS + blockIdx.x] = v;
  }
}

__global__ __launch_bounds__(256) void k_trial_gather(const TrialJob* __restrict__ jobs) {
  __shared__ double sh[256];
  const TrialJob T = jobs[blockIdx.x];
  for (int w = 0; w < 2; ++w) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < QF_BLOCKS; i += 256) acc = fmax(acc, T.partial[w * QF_BLOCKS + i]);
    const double r = blk_max(acc, sh);
    if (threadIdx.x == 0) T.out4[w] = r;
  }
  if (threadIdx.x == 0) {
    T.out4[2] = T.quad2[0];
    T.out4[3] = T.quad2[1];
  }
}

hipError_t launch_trial(const TrialJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trial, dim3(QF_BLOCKS, count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_trial_gather(const TrialJob* jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trial_gather, dim3(count), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace dl
