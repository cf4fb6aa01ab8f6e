// Device-side model description and per-theta coefficient table layout.
#pragma once
#include "common.hpp"

namespace dl {

// Coefficient table written by k_theta_coeffs (FP64, device):
//   [C_LOGPRIOR]        log p(theta)
//   [C_LLCONST]         sum_j m_j/2 log tau_j - m/2 log 2pi (Poisson: 0)
//   [C_BAD]             1 if theta maps outside the model (NaN, |rho| = 1)
//   [C_TAU + j]         tau_y of response j (Poisson: 1, unused)
//   [C_D + ((tt*3 + k)*3 + j)*NPIECE + c]
//                       weight of FEM piece c (0: C, 1: G, 2: G C^-1 G,
//                       3: G C^-1 G C^-1 G) in block (k, j) of a diagonal
//                       block; tt = 0 first/last time step, 1 interior
//                       step, 2 single step (nt = 1)
//   [C_B + (k*3 + j)*NPIECE + c]  the same for a sub-diagonal block
enum : int {
  NPIECE = 4,
  C_LOGPRIOR = 0,
  C_LLCONST = 1,
  C_BAD = 2,
  C_TAU = 4,
  C_D = 8,
  C_B = 8 + 27 * NPIECE,
  C_SIZE = 8 + 36 * NPIECE + 4
};

struct ModelDev {
  int nx, nt, nv, nr, ns, b, a, bp, ap, dim_theta;
  int family;             // DL_MODEL_SEPARABLE or DL_MODEL_DIFFUSION
  int likelihood;         // DL_LIK_GAUSSIAN or DL_LIK_POISSON
  int64_t N, Np;          // unpadded and padded vector lengths
  // spatial pattern (13 points, or 25 for the diffusion model), CSR over
  // nodes, with the values of the four FEM pieces (G3 is zero for the
  // separable model)
  const int* sp_ptr;
  const int* sp_col;
  const double* sp_C;
  const double* sp_G;
  const double* sp_G2;
  const double* sp_G3;
  // observations of all responses, concatenated
  int64_t m_total;
  int64_t m_off[4];
  const int* obs_t;
  const int* obs_nodes;   // m x 3
  const double* obs_w;    // m x 3
  const double* obs_x;    // m x nr
  const double* obs_y;    // m
  // per (response j, time t, node s): observation rows touching the node
  const int64_t* no_ptr;  // nv*nt*ns + 1
  const int* no_row;
  const int* no_q;
  const double* theta_prior_mean;
  double theta_prior_sd;
  double prior_fixed;
};

// Dense targets of one assembly job.  Time step t0 + k of the job writes
// Dp + k*dp_stride (Q_p diagonal block, ld bp), Bp + k*bp_stride (Q_p
// sub-diagonal block, ld bp), Dc + k*dc_stride, BRc + k*brc_stride
// ([B_t; R_t] of Q_c, ld bp+ap) and the right-hand side rhs[t*bp + c]
// (with Q_c).  A null pointer skips that matrix.
struct AssembleOut {
  double* Dp;
  int64_t dp_stride;
  double* Bp;
  int64_t bp_stride;
  double* Dc;
  int64_t dc_stride;
  double* BRc;
  int64_t brc_stride;
  double* Pp;   // ap x ap (tip of Q_p), ld ap
  double* Pc;   // ap x ap (tip of Q_c)
  double* rhs;  // Np
  int b32;      // Bp and BRc are stored in FP32 (mixed precision)
  // per-observation D and right-hand-side values (m_total each) in place of
  // tau_y and tau_y y (non-Gaussian likelihoods; null: Gaussian)
  const double* obs_d;
  const double* obs_z;
};

struct ThetaJob {
  const ModelDev* m;
  const double* theta;
  double* coef;
};

struct AsmJob {
  const ModelDev* m;
  const double* coef;
  AssembleOut o;
  int t0, nt;
};

struct QuadJob {
  const ModelDev* m;
  const double* coef;
  const double* mu;
  double* partial;  // 2 * QF_BLOCKS
  double* out2;     // [mu^T Q_p mu, (y - A mu)^T D (y - A mu)]; Poisson:
                    // [mu^T Q_p mu, -2 log l(y | A mu)]
};

struct CombineJob {
  const double* coef;
  const double* logdet2;
  const int64_t* info2;
  const double* quad2;
  double* f;
  dl_fobj_parts* parts;
  int64_t* info_out;
  const double* rnorm;  // [|rhs - Q_c mu|^2, |rhs|^2] (may be null)
  const double* tol2;   // squared tolerance of the refined mean: a larger
                        // relative residual sets info_out[1] to
                        // DL_INFO_NOTCONV (null: no check)
};

constexpr int QF_BLOCKS = 256;

hipError_t launch_theta_coeffs(const ThetaJob* jobs, int count, hipStream_t s);
// max_bp / max_nt bound the grid over the jobs; max_shmem_doubles = max over
// the jobs' models of 2*bp + ap.
hipError_t launch_assemble_cols(const AsmJob* jobs, int count, int max_bp,
                                int max_nt, int max_shmem_doubles, hipStream_t s);
hipError_t prepare_assemble(int max_shmem_doubles);
hipError_t launch_assemble_tips(const AsmJob* jobs, int count, int max_blocks,
                                hipStream_t s);
hipError_t launch_quadforms(const QuadJob* jobs, int count, hipStream_t s);

// out = rhs - Q_c v (FP64, from the stencil of Q_p and the observation rows;
// used by the iterative refinement of the mixed-precision solve), and
// norms[0] = |out|_2^2, norms[1] = |rhs|_2^2 (fixed reduction order).
struct ResJob {
  const ModelDev* m;
  const double* coef;
  const double* v;    // Np (padded BTA order)
  const double* rhs;  // Np
  double* out;        // Np
  double* av;         // m_total scratch: (A v)_row
  double* partial;    // 2 * QF_BLOCKS
  double* norms;      // 2
  const double* obs_d;  // per-observation D (non-Gaussian), else null
};
hipError_t launch_residual(const ResJob* jobs, int count, hipStream_t s);
hipError_t launch_combine(const CombineJob* jobs, int count, hipStream_t s);

// Inner Newton iteration of a Poisson likelihood (Section II-A, conditional Gaussian distribution): from the
// iterate x (padded BTA order) every observation row gets eta = (A x)_row,
// d = exp(eta) and z = y - d + d eta (the gradient plus D eta).
struct LapJob {
  const ModelDev* m;
  const double* x;
  double* obs_d;   // m_total
  double* obs_z;   // m_total
};
hipError_t launch_lap_weights(const LapJob* jobs, int count, hipStream_t s);

// Trial point mu = x + alpha (xN - x) of a damped Newton step, and
// out4 = [max |xN - x|, max |xN|, mu^T Q_p mu, -2 log l] (the last two
// copied from the quadratic forms of mu, run in between).
struct TrialJob {
  const ModelDev* m;
  const double* x;
  const double* xN;
  double* mu;
  const double* alpha;
  double* partial;       // 2 * QF_BLOCKS
  const double* quad2;
  double* out4;
};
hipError_t launch_trial(const TrialJob* jobs, int count, hipStream_t s);
hipError_t launch_trial_gather(const TrialJob* jobs, int count, hipStream_t s);
hipError_t launch_pack(const ModelDev& m, const double* padded, double* out,
                       hipStream_t s);
hipError_t launch_unpack(const ModelDev& m, const double* in, double* padded,
                         hipStream_t s);

}  // namespace dl
