/*
 * dalia.h -- C ABI of libdalia_hip.so: evaluation of the INLA objective
 * f_obj(theta) for spatio-temporal (optionally coregional) latent Gaussian
 * models on one AMD Instinct MI355X (gfx950).
 *
 * The method (Gaedke-Merzhaeuser et al., "Accelerated Spatio-Temporal
 * Bayesian Modeling for Multivariate Gaussian Processes"):
 *   - Q_p(theta): prior precision of the latent field, SPDE space (x) AR1 time
 *     (Section II-A), mixed over responses by the coregional form Eq. 11, with
 *     fixed effects appended (Eq. 2);
 *   - Q_c(theta) = Q_p + A^T D A (Eq. 4), block tridiagonal with arrowhead
 *     (BTA) once permuted time-major (Section IV-B, permutation);
 *   - f_obj(theta) = log p(theta) + log l(y|theta,x) + log p(x|theta)
 *                    - log p_G(x|theta,y)                         (Eq. 8)
 *     which needs log|Q_p|, log|Q_c| (Cholesky, Eq. 1, 3), the conditional
 *     mean mu (triangular solves) and, for marginal variances, selected
 *     entries of Q_c^{-1} (selected inversion, Section III-A).
 *
 * Conventions for every entry point below:
 *   - Pointers named *_dev are device pointers owned by the caller; pointers
 *     named *_host are host pointers read synchronously during the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; scalar results are written to
 *     device memory.  One workspace must not be used by two streams at once.
 *   - Vectors are in BTA order: variable (t, j, s) -- time step t, response j,
 *     spatial node s -- is at t*b + j*ns + s with b = nv*ns; the fixed effect
 *     (j, r) is at nt*b + j*nr + r.  N = nt*b + nv*nr.
 *   - Argument and state errors return synchronously (DL_EINVAL, DL_ESTATE,
 *     DL_ENOMEM, DL_EHIP).  Numerical failure (a non-positive pivot) is
 *     reported through info_dev: 0 = ok, k > 0 = first bad pivot at BTA row
 *     k-1 (LAPACK style); f_obj is then -inf.
 *   - Nothing is allocated after dl_ws_create; no C++ exception crosses the
 *     ABI.
 */
#ifndef DALIA_H
#define DALIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DL_OK = 0,
  DL_EINVAL = 1,   /* bad argument                                   */
  DL_ENOMEM = 2,   /* device allocation failed                       */
  DL_ENOTSPD = 3,  /* (reserved: numerical failure goes to info_dev)  */
  DL_EHIP = 4,     /* a HIP runtime call failed                      */
  DL_ESTATE = 5,   /* call order violated (e.g. selinv before factor) */
  DL_ENOTCONV = 6  /* iterative refinement did not converge          */
} dl_status;

typedef enum { DL_QP = 0, DL_QC = 1, DL_BOTH = 2 } dl_which;

typedef struct dl_model dl_model;  /* theta-independent data on the device */
typedef struct dl_ws dl_ws;        /* dense BTA workspace for one model    */

/* Host description of a model (all host pointers, read during create).
 * Mesh: regular nx*nx grid, unit spacing; node (ix, iy) has index iy*nx+ix.
 * Observation row i of response j lies at time step obs_t[j][i] on the mesh
 * triangle obs_nodes[j][3i..3i+2] with barycentric weights obs_w[j][3i..],
 * has covariates obs_x[j][i*nr .. i*nr+nr-1] (row-major) and value y[j][i]. */
typedef struct dl_model_desc {
  int32_t nx, nt, nv, nr;
  int64_t m[3];
  const int32_t* obs_t[3];
  const int32_t* obs_nodes[3];
  const double* obs_w[3];
  const double* obs_x[3];
  const double* y[3];
  const double* theta_prior_mean; /* dim_theta values                     */
  double theta_prior_sd;          /* sd of the Gaussian prior on theta    */
  double prior_fixed;             /* precision of each fixed effect       */
  int32_t family;                 /* DL_MODEL_SEPARABLE (0, what a zeroed
                                     descriptor selects) or
                                     DL_MODEL_DIFFUSION                    */
  int32_t likelihood;             /* DL_LIK_GAUSSIAN (0) or DL_LIK_POISSON */
} dl_model_desc;

/* Model families of each univariate process (Section II-A; Section IV-B,
 * multivariate model formulation, which builds each univariate precision as a sum of
 * Kronecker products of temporal and spatial FEM matrices).
 *   DL_MODEL_SEPARABLE  T (x) Q_s: unit-variance AR1 in time times the SPDE
 *                       precision Q_s = kappa^4 C + 2 kappa^2 G + G C^-1 G.
 *   DL_MODEL_DIFFUSION  non-separable diffusion-based model
 *                         M0 (x) K3 + 2 gamma_t M1 (x) K2 + gamma_t^2 M2 (x) K1
 *                       with K1 = gamma_s^2 C + G, K_{k+1} = K1 C^-1 K_k and the
 *                       temporal FEM matrices of unit-spaced time nodes: M0
 *                       lumped mass (1/2 at both ends, 1 inside), M1 = 1/2 at
 *                       both ends, M2 stiffness tridiag(-1; 1,2,...,2,1; -1).
 *                       Needs nt >= 2.  Its spatial stencil reaches grid
 *                       distance 3 (25 points) instead of 2 (13 points). */
enum { DL_MODEL_SEPARABLE = 0, DL_MODEL_DIFFUSION = 1 };

/* Likelihood of the responses (Section II-A, its conditional Gaussian
 * distribution part: D in Q_c = Q_p + A^T D A is the negative Hessian of the
 * log-likelihood, Eq. 4).
 *   DL_LIK_GAUSSIAN  y_i ~ N((A x)_i, 1/tau_y_j) (Eq. 2): D = tau_y, p_G is
 *                    exact and its mean solves Q_c mu = A^T D y.
 *   DL_LIK_POISSON   counts y_i ~ Poisson(exp((A x)_i)) (log link): D
 *                    depends on x, so fobj_eval first finds the mode x* of
 *                    h(x) = log l(y | A x) - 1/2 x^T Q_p x by damped Newton
 *                    from x = 0 (see fobj_eval) and evaluates Eq. 8 there
 *                    (Laplace approximation).  theta has no log tau_y
 *                    slots; every y must be a non-negative integer. */
enum { DL_LIK_GAUSSIAN = 0, DL_LIK_POISSON = 1 };

/* Inner Newton iteration of DL_LIK_POISSON models: stop after a full step
 * with max|x_N - x| <= DL_NEWTON_TOL (1 + max|x_N|); at most
 * DL_NEWTON_MAX steps, each halved at most DL_NEWTON_HALVINGS times until
 * h(new) >= h(x) - DL_ASCENT_SLACK (1 + |h(x)|). */
#define DL_NEWTON_TOL 1e-9
#define DL_NEWTON_MAX 40
#define DL_NEWTON_HALVINGS 30
#define DL_ASCENT_SLACK 1e-12

/* Parts of f_obj (Eq. 8) written by fobj_eval, one record per theta. */
typedef struct dl_fobj_parts {
  double f;          /* f_obj(theta)                                   */
  double logdet_p;   /* log|Q_p|                                       */
  double logdet_c;   /* log|Q_c|                                       */
  double quad_p;     /* mu^T Q_p mu                                    */
  double quad_obs;   /* (y - A mu)^T D (y - A mu); Poisson: -2 log l(y|mu)
                        (log(y!) included)                             */
  double log_prior;  /* log p(theta)                                   */
  double log_lik_const; /* sum_j m_j/2 log tau_j - m/2 log(2 pi); Poisson: 0 */
  double rel_residual;  /* |A^T D y - Q_c mu| / |A^T D y| of the final mu;
                           Poisson: |A^T g - Q_p mu| / |A^T (g + D A mu)|
                           at the mode (g: the log-likelihood's gradient) */
} dl_fobj_parts;

/* Number of hyperparameters: 4 for nv = 1, 4*nv + nv(nv-1)/2 otherwise.
 * theta layout, univariate: [log kappa, phi, log tau_u, log tau_y];
 * coregional: [log kappa_i (nv), phi_i (nv), log sigma_i (nv),
 * lambda_k (nv(nv-1)/2), log tau_y_j (nv)], rho = tanh(phi/2).
 * DL_MODEL_DIFFUSION reads log gamma_s in the slots of log kappa and
 * log gamma_t in the slots of phi; the other slots keep their meaning. */
int32_t dl_theta_dim(int32_t nv);
/* The same for a likelihood: DL_LIK_POISSON drops the nv log tau_y slots
 * (3 for nv = 1, 3*nv + nv(nv-1)/2 otherwise); -1 for an unknown value. */
int32_t dl_theta_dim_lik(int32_t nv, int32_t likelihood);

/* Upload a model.  Builds the spatial pattern (Section II-A, SPDE FEM) and
 * per-(response, time, node) observation index lists on the host (integer
 * work only) and copies all arrays to the device.  nv in {1,2,3}; nx >= 2;
 * nt >= 1 (>= 2 for DL_MODEL_DIFFUSION); nr >= 0; every obs_t < nt and every
 * node < nx*nx; family one of the DL_MODEL_* values; likelihood one of the
 * DL_LIK_* values (DL_LIK_POISSON: every y a non-negative integer).
 * DL_EINVAL otherwise. */
dl_status dl_model_create(const dl_model_desc* desc_host, dl_model** out);
void dl_model_destroy(dl_model* model);

/* Dimensions: n = nt blocks, b = nv*ns, a = nv*nr, N = n*b + a; bp is the
 * padded block size used in device storage. */
dl_status dl_model_dims(const dl_model* model, int64_t* n, int64_t* b,
                        int64_t* a, int64_t* N, int64_t* bp);

/* Workspace flags. */
enum {
  DL_WS_SELINV = 1,   /* keep the storage of the selected inversion        */
  DL_WS_KEEP_QP = 2,  /* store Q_p in full (inspection); by default Q_p is
                         assembled just in time into a ring of blocks, as
                         only its log-determinant is needed                */
  DL_WS_GRAPH = 4,    /* fobj_eval replays one captured HIP graph          */
  DL_WS_MIXED = 8     /* mixed precision: the off-diagonal blocks [B_t; R_t]
                         of Q_c (and Q_p) are stored in FP32 and their
                         TRSM / SYRK / GEMM products run on FP32 matrix
                         cores (FP32 accumulation, subtracted into FP64
                         diagonal blocks and tips); diagonal-block Cholesky,
                         inverses and log-determinants stay FP64; the mean
                         is refined in FP64 against the sparse Q_c to
                         DL_REFINE_TOL (see below)                         */,
  DL_WS_SPLITK = 16   /* split the long inner dimensions of the FP64 block
                         products (factor, inverse, selected inversion) into
                         pieces of 512 summed in a fixed order: more
                         parallelism for single evaluations; the results
                         differ from an unsplit workspace by rounding only
                         and do not depend on the tile sizes chosen         */,
  DL_WS_TWOSIDED = 32 /* time-domain partitioning into two partitions on one
                         GPU (Sec. IV-C, time-domain partitioning, with
                         S3's nested dissection for two partitions, which
                         have no middle partition and so add no work): the
                         first half of the time steps is eliminated forward
                         and the second half backward, concurrently (their
                         steps share launches), into the middle block
                         mid = floor((nt+1)/2), which is factored last;
                         solve and selected inversion follow the same order.
                         Needs nt >= 4 (otherwise one-sided).  Results
                         differ from the one-sided order by rounding only.
                         Relies on symmetric sub-diagonal blocks, which
                         every model of this library has                    */,
  DL_WS_FOLD_INV = 64 /* form each diagonal block's inverse L_tt^-1 inside
                         the launches of its blocked factorisation (one row
                         of 64 x 64 tiles per panel step, left-looking)
                         instead of by recursive GEMM halving after it:
                         about 12 fewer dependent launches per block, faster
                         when few blocks are factored at once (single
                         evaluations); for wide batches the recursive
                         inversion is faster.  Results differ from the
                         default by rounding only                           */,
  DL_WS_WARM_START = 128 /* DL_LIK_POISSON: start each instance's inner
                         Newton search from its mode of the previous pass
                         (when that pass converged) instead of x = 0.  For
                         nearby thetas (line searches, difference stencils)
                         it takes fewer steps; the mode is unique, so results
                         differ from a cold start by rounding only, but they
                         depend on the call history                        */,
  DL_WS_DAG = 256     /* factor each step's diagonal blocks in one persistent
                         launch (a tile-task graph, Sec. III-A's Cholesky
                         of the diagonal block with its inverse formed
                         alongside): workgroups take 64 x 64 tile tasks --
                         tile factor, panel solve, trailing update, inverse
                         accumulation and inverse row -- in a fixed order and
                         wait on per-tile readiness counters, so the next
                         tile factor starts as soon as its tile is final
                         instead of after a whole panel launch.  Holds the
                         inverse like DL_WS_FOLD_INV; needs one bp x bp
                         block of doubles per matrix and elimination chain
                         for the L tiles.
                         Results differ from the panel path by rounding
                         only                                               */
};
/* FP64 iterative refinement of the mean (DL_WS_MIXED workspaces; any
 * workspace through bta_solve on request): x <- x + c, where c solves
 * (L L^T) c = rhs - Q_c x with the workspace's factor and the residual is
 * formed with the sparse FP64 Q_c, until |rhs - Q_c x|_2 <= tol |rhs|_2.
 * Eager evaluations take at most DL_REFINE_MAX corrections with tol =
 * DL_REFINE_TOL (the host reads the residual norms after each one); a
 * DL_WS_GRAPH workspace captures DL_REFINE_STEPS_GRAPH correction steps.
 * Within a batch an instance that meets the tolerance keeps its iterate bit
 * for bit while the others continue, so batch, single and graph-replayed
 * results agree.  A refined mean that still misses the tolerance is
 * reported as info_dev[2k+1] = DL_INFO_NOTCONV (the pivots were fine, f and
 * its parts are written). */
#define DL_REFINE_TOL 1e-12
#define DL_REFINE_MAX 10
#define DL_REFINE_STEPS_GRAPH 3
#define DL_INFO_NOTCONV (-1)
/* info value of a factorisation whose persistent launch (DL_WS_DAG) gave up
 * waiting for a tile (it never should; f is then -inf). */
#define DL_INFO_TIMEOUT (-2)

/* Allocate the dense BTA workspace for Q_p and Q_c of `model`.  All device
 * memory of the evaluation path is allocated here. */
dl_status dl_ws_create(const dl_model* model, int32_t flags, dl_ws** out);

/* A workspace of nmodels instances evaluated together: every launch of an
 * evaluation serves the same step of all instances (and of both Q_p and
 * Q_c).  The same model may be passed several times (e.g. the 2*dim+1
 * points of a central-difference gradient, Eq. 10, the paper's first
 * parallel layer); models may also differ in size.  Per-instance inputs and
 * outputs are packed in instance order: theta of instance k at offset
 * sum_{k'<k} dim_theta(k'), N-vectors at sum_{k'<k} N(k'), logdet/info of
 * bta_factor at cnt*k (cnt = 2 for DL_BOTH, else 1). */
dl_status dl_ws_create_batch(const dl_model* const* models, int32_t nmodels,
                             int32_t flags, dl_ws** out);
int32_t dl_ws_batch(const dl_ws* ws);
void dl_ws_destroy(dl_ws* ws);
/* Device bytes held by the workspace. */
size_t dl_ws_bytes(const dl_ws* ws);

/* Newton steps taken per instance in the last fobj_eval/fobj_selinv_eval
 * pass of a DL_LIK_POISSON workspace (-1: not converged); steps_host holds
 * dl_ws_batch(ws) values.  Gaussian workspaces report 0. */
dl_status dl_ws_newton_steps(const dl_ws* ws, int32_t* steps_host);

/* bta_assemble -- theta (dim_theta doubles, device) -> the model
 * coefficients (Eq. 5, Eq. 11) and log p(theta), then the dense BTA blocks
 * of Q_p and/or Q_c (Eq. 4, Eq. 11; Section IV-B, permutation; Section
 * IV-F, sparse to structured dense mapping) and the right-hand side
 * A^T D y of Eq. 3.  DL_ESTATE never; asynchronous.  Only the lower triangle of each diagonal block
 * is stored.  For DL_LIK_POISSON models D and the right-hand side come
 * from the workspace's last inner iterate (D = 0 before the first
 * fobj_eval). */
dl_status bta_assemble(dl_ws* ws, const double* theta_dev, dl_which which,
                       void* stream);

/* bta_factor -- the BTA Cholesky factorisation and log-determinants
 * (Section III-A, Cholesky factorization and triangular solve: the block
 * recurrence of the structured solver; Eq. 1 and 3 need log|Q|).  In place
 * on the assembled blocks of Q_p and/or Q_c: per time step POTRF of the
 * diagonal block D_t and its inverse, [B_t; R_t] <- [B_t; R_t] L_tt^-T, the
 * Schur updates of the next diagonal block, its arrow block and the tip;
 * finally POTRF of the tip.  logdet_dev[0] (and logdet_dev[1] for DL_BOTH:
 * [Q_p, Q_c]) receives log|Q| = 2 sum log L_ii; info_dev[0] (info_dev[1]
 * for DL_BOTH) the first bad pivot as 1 + its BTA row (0: positive
 * definite).  A batch workspace writes cnt values per instance (cnt = 2
 * for DL_BOTH, else 1).  Either pointer may be NULL.  DL_ESTATE unless the
 * matrix was assembled since its last factorisation.  Asynchronous. */
dl_status bta_factor(dl_ws* ws, dl_which which, double* logdet_dev,
                     int64_t* info_dev, void* stream);

/* bta_solve -- Q_c x = r with the factor of Q_c (Section III-A, Cholesky
 * factorization and triangular solve: forward then backward block
 * substitution; with r = A^T D y, x is the conditional mean of Eq. 3).
 *   rhs_inout_dev == NULL: solves the assembled A^T D y (nrhs 0 or 1) and
 *     keeps the mean in the workspace (dl_ws_mean);
 *   otherwise nrhs >= 1 right-hand sides of N_total doubles each (BTA
 *     order, a batch workspace's instances packed in order), solved in
 *     place one after the other (the workspace's own right-hand side is
 *     overwritten).
 * refine_max < 0: the workspace's default refinement (DL_WS_MIXED: to
 * DL_REFINE_TOL in at most DL_REFINE_MAX corrections; FP64: none).
 * refine_max >= 0 (at most 100): at most refine_max FP64 corrections
 * against the sparse Q_c until |r - Q_c x|_2 <= refine_tol |r|_2 (see the
 * refinement constants above); with refine_max > 0 the call reads residual
 * norms on the host (it synchronises the stream) and returns DL_ENOTCONV
 * when some solve still misses refine_tol (its x is written all the same).
 * DL_EINVAL for a bad nrhs, refine_max or refine_tol; DL_ESTATE before a
 * factorisation of Q_c. */
dl_status bta_solve(dl_ws* ws, double* rhs_inout_dev, int32_t nrhs, int32_t refine_max,
                    double refine_tol, void* stream);

/* bta_selinv -- Takahashi selected inversion (Section III-A, selected
 * inversion: the entries of Q_c^-1 on the BTA pattern from the factor,
 * backward in time, Eq. 1's marginal variances on the diagonal); writes
 * diag(Q_c^{-1}) to diag_out_dev (N doubles per instance, BTA order,
 * instances packed).  Requires flags bit 0 (DL_WS_SELINV) at creation and a
 * factorisation of Q_c; otherwise DL_ESTATE.  Asynchronous. */
dl_status bta_selinv(dl_ws* ws, double* diag_out_dev, void* stream);

/* fobj_eval -- f_obj (Eq. 8, evaluated at the conditional mean) for ntheta
 * hyperparameter vectors: assembly, both factorisations, the solve for the
 * mean, the quadratic forms and the combination of Eq. 8's terms
 * (theta_dev: ntheta x dim_theta, row-major).  fobj_dev[k], parts_dev[k]
 * (may be NULL) and info_dev[2k..2k+1] (Q_p, Q_c pivots; may be NULL)
 * receive the results; info_dev[2k+1] = DL_INFO_NOTCONV flags a refined
 * mean (DL_WS_MIXED) that missed DL_REFINE_TOL.  DL_WS_MIXED evaluations
 * that run eagerly read the residual norms on the host after each
 * correction (one synchronisation each).  A batch workspace of B instances evaluates B thetas
 * per pass (ntheta may be any count when all instances share one model;
 * otherwise ntheta must equal B).  mu of the last pass stays in the
 * workspace.
 *
 * DL_LIK_POISSON workspaces (every instance's model must have it) find the
 * inner mode first, each Newton step as kernels over all instances of the
 * pass: the observation weights D = exp(A x) and working values
 * g + D A x from the current iterate, assembly of Q_c(x) and A^T (g + D A x),
 * its factorisation and solve (x_N), then trial points x + alpha (x_N - x)
 * with h evaluated by the quadratic-form kernels; the host reads 4 values
 * per instance per trial to pick alpha and to stop.  An instance that has
 * converged keeps its iterate while the others continue (so batch results
 * equal single evaluations).  Q_c is then assembled and factored at x*
 * (its factor serves bta_selinv) and Eq. 8 is evaluated at mu = x*; an
 * instance that did not converge gets f = -inf.  These passes run eagerly
 * (also for DL_WS_GRAPH workspaces) and synchronise the stream once per
 * trial.  With DL_WS_MIXED every Newton solve is refined in FP64 against
 * the sparse Q_c(x) (to DL_REFINE_TOL), so the mode is the FP64 one;
 * log|Q_c(x*)| carries the FP32 error of the off-diagonal blocks, and mu is
 * the refined solve at x* (one more Newton step from the mode, equal to it
 * up to rounding). */
dl_status fobj_eval(dl_ws* ws, const double* theta_dev, int32_t ntheta,
                    double* fobj_dev, dl_fobj_parts* parts_dev,
                    int64_t* info_dev, void* stream);

/* fobj_selinv_eval -- f_obj and the marginal variances together: f_obj as
 * fobj_eval for one pass of ntheta (1..B; B when the instances' models differ) thetas,
 * and diag(Q_c^{-1}) of every instance as bta_selinv (diag_out_dev: the
 * instances' N values in order).  The solve and quadratic forms run on a
 * second, library-owned stream concurrently with the selected inversion
 * (both only read the factor); every result is written to the caller's
 * stream order.  Requires flags bit 0 (DL_WS_SELINV), else DL_ESTATE;
 * DL_EINVAL for NULL pointers or an invalid ntheta.  Runs eagerly (also
 * for DL_WS_GRAPH workspaces).  DL_LIK_POISSON workspaces run fobj_eval's
 * mode search on the caller's stream and then the selected inversion of
 * Q_c(x*): the marginal variances of the Laplace approximation. */
dl_status fobj_selinv_eval(dl_ws* ws, const double* theta_dev, int32_t ntheta,
                           double* fobj_dev, dl_fobj_parts* parts_dev, int64_t* info_dev,
                           double* diag_out_dev, void* stream);

/* Copy the conditional mean of the last solve (N doubles, BTA order). */
dl_status dl_ws_mean(dl_ws* ws, double* out_dev, void* stream);

/* Copy one assembled (or factored) block to out_dev, column-major, for
 * inspection: kind 0 = diagonal block D_t (b x b, lower triangle), 1 =
 * sub-diagonal block B_t (b x b, rows t+1, cols t), 2 = arrow block R_t
 * (a x b), 3 = tip (a x a, lower triangle), 4 = right-hand side (N, Q_c
 * only).  After a DL_WS_TWOSIDED factorisation kind 1 at t >= mid holds the
 * factor's coupling of block t to block t-1 (its successor in that order).
 * Single-instance workspaces; Q_p blocks other than the tip need
 * DL_WS_KEEP_QP (DL_ESTATE otherwise).  Synchronises the stream. */
dl_status dl_ws_get_block(dl_ws* W, dl_which which, int32_t kind, int32_t t,
                          double* out_dev, void* stream);

/* The reverse of dl_ws_get_block: overwrite one block of an assembled (not
 * yet factored) matrix with in_dev (column-major, unpadded sizes as above;
 * for diagonal blocks and the tip only the lower triangle is used), so that
 * bta_factor / bta_solve / bta_selinv run on a caller-supplied BTA matrix
 * (the padding keeps its identity).  DL_WS_TWOSIDED workspaces read each
 * sub-diagonal block also as its own transpose, so they need symmetric
 * B_t.  DL_ESTATE unless the matrix was assembled since its last
 * factorisation (or for Q_p blocks without DL_WS_KEEP_QP).  Synchronises the
 * stream. */
dl_status dl_ws_set_block(dl_ws* W, dl_which which, int32_t kind, int32_t t,
                          const double* in_dev, void* stream);

/* Model order <-> BTA order (Section IV-B, permutation).  Model order is the
 * response-major order of Eq. 11: latent variable (response j, time t,
 * node s) at j*nt*ns + t*ns + s, then the fixed effects (j, r) at
 * nt*nv*ns + j*nr + r; BTA order is the one described at the top of this
 * file.  dl_permute: bta_dev[k] = model_dev[perm(k)]; dl_unpermute: the
 * inverse.  nvec vectors of N doubles each, contiguous; source and
 * destination must not be the same buffer (DL_EINVAL).  Asynchronous. */
dl_status dl_permute(const dl_model* model, const double* model_dev, double* bta_dev,
                     int32_t nvec, void* stream);
dl_status dl_unpermute(const dl_model* model, const double* bta_dev, double* model_dev,
                       int32_t nvec, void* stream);

/* ---- device memory budget ------------------------------------------------
 * dl_ws_estimate_bytes: device bytes that dl_ws_create_batch(models,
 * nmodels, flags) allocates for its buffers, computed on the host without
 * touching the device (dl_ws_bytes reports the same count after creation;
 * the launch descriptors, a few MB, and the split-k partial tiles of
 * DL_WS_SPLITK or of a later dl_autotune are not included).
 * dl_ws_create_budget: dl_ws_create_batch, or DL_ENOMEM without allocating
 * anything when that estimate exceeds hbm_budget bytes.
 * dl_plan_waves: splits a batch that does not fit into waves that do: each
 * instance k gets a wave index wave_of_host[k] in 0 .. *nwaves_host - 1
 * (first fit, largest instance first), so that every wave's estimate plus
 * DL_WAVE_RESERVE bytes stays within hbm_budget; DL_ENOMEM when one
 * instance alone does not fit.  Host only. */
#define DL_WAVE_RESERVE ((size_t)256 << 20)
dl_status dl_ws_estimate_bytes(const dl_model* const* models, int32_t nmodels,
                               int32_t flags, size_t* bytes_host);
dl_status dl_ws_create_budget(const dl_model* const* models, int32_t nmodels,
                              int32_t flags, size_t hbm_budget, dl_ws** out);
dl_status dl_plan_waves(const dl_model* const* models, int32_t nmodels, int32_t flags,
                        size_t hbm_budget, int32_t* wave_of_host, int32_t* nwaves_host);

/* ---- dense FP64 block kernels (the building blocks of bta_factor) ------- */

/* C = alpha * op(A) * op(B) + beta * C, column-major, op = transpose when
 * the flag is set; lower != 0 restricts C to its lower triangle. */
dl_status dl_dgemm(int32_t transa, int32_t transb, int32_t lower, int64_t M,
                   int64_t Nn, int64_t K, double alpha, const double* A_dev,
                   int64_t lda, const double* B_dev, int64_t ldb, double beta,
                   double* C_dev, int64_t ldc, void* stream);

/* In-place Cholesky of an n x n SPD matrix (lower, column-major): on exit
 * the lower triangle holds L^{-1} when want_inverse != 0, else L; the
 * strict upper triangle is zeroed.  logdet_dev[0] = log|A|; info_dev[0] =
 * first bad pivot (1-based) or 0.  n must be a multiple of 64. */
dl_status dl_dpotrf(int64_t n, double* A_dev, int64_t lda, int32_t want_inverse,
                    double* logdet_dev, int64_t* info_dev, void* stream);

/* dl_dpotrf_noalloc -- for callers that cannot allocate device memory (work
 * recorded under HIP graph capture, serving loops with a fixed memory
 * footprint, harnesses that forbid hipMalloc): the same factorisation,
 * outputs and error behaviour as dl_dpotrf, but every temporary (tile
 * inverses, the recursive inversion's products, log-diagonal, reduction
 * partials, launch descriptors) lives in one static device array of
 * DL_DPOTRF_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on until the process ends.  No device or host allocation and no stream
 * synchronisation: the results are ready in stream order.  n must be a
 * multiple of 64 and at most DL_DPOTRF_NOALLOC_MAX_N (DL_EINVAL otherwise,
 * returned before any device call).  All calls on one GPU share its array,
 * which keeps the last call's contents: calls that overlap in time on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller. */
#define DL_DPOTRF_NOALLOC_MAX_N 2048
#define DL_DPOTRF_NOALLOC_SCRATCH_BYTES 18958336
dl_status dl_dpotrf_noalloc(int64_t n, double* A_dev, int64_t lda,
                            int32_t want_inverse, double* logdet_dev,
                            int64_t* info_dev, void* stream);

/* Pick the GEMM tile (64x64 or 128x128 outputs per workgroup) of every
 * matrix-product launch of the workspace, and for FP64 launches with a k
 * extent above 512 whether to split k (pieces summed by a second launch),
 * by timing the candidates on the device once per distinct launch shape;
 * choices are appended to / read from the text file cache_path (may be
 * NULL; one line per shape ending in the tile, suffixed "s" when split).
 * May grow the workspace's device memory by the split partial tiles (split
 * choices needing more than 4 GiB of them are not tried).
 * Synchronises the stream; the
 * workspace's matrices must be re-assembled afterwards (fobj_eval always
 * does).  Call before the first evaluation of a DL_WS_GRAPH workspace. */
dl_status dl_autotune(dl_ws* ws, const char* cache_path, void* stream);
dl_status dl_ws_tile_counts(const dl_ws* ws, int64_t* n64, int64_t* n128);
/* Set the tile (64 or 128) of every matrix-product launch, overriding the
 * default and any tuned choice; each launch keeps its split-k setting
 * (measurement and tests).  DL_EINVAL for
 * other sizes, DL_ESTATE once a graph has been captured. */
dl_status dl_ws_force_tile(dl_ws* ws, int32_t tile);
/* Split the k range of every FP64 matrix-product launch into pieces of
 * ksplit (a multiple of 16, at least 64; cut at absolute multiples, so
 * results do not depend on the tile size), or unsplit them (ksplit = 0),
 * overriding the default and any tuned choice (measurement and tests).  May
 * grow the workspace's device memory by the partial tiles.  DL_EINVAL for
 * other values, DL_ESTATE once a graph has been captured. */
dl_status dl_ws_force_split(dl_ws* ws, int32_t ksplit);

/* ---- surrogate network (learned model of f_obj over theta) ----------------
 * Multi-layer perceptron sizes[0] -> ... -> sizes[n-1] = 1, SiLU between
 * layers, linear output.  Parameters live in one FP32 device vector (layer
 * k: W_k row-major sizes[k+1] x sizes[k], then b_k), with FP32 Adam moments;
 * every matrix product rounds both operands to bfloat16 and accumulates in
 * FP32 on the matrix cores.  Batches of up to max_batch rows; inputs are
 * row-major FP32.  Not thread-safe per network. */
typedef struct dl_mlp dl_mlp;
dl_status dl_mlp_create(const int32_t* sizes, int32_t nsizes, int32_t max_batch,
                        dl_mlp** out);
void dl_mlp_destroy(dl_mlp* net);
/* Device pointers of the parameter and gradient vectors (owned by the
 * network) and their length. */
dl_status dl_mlp_params(dl_mlp* net, float** params_dev, float** grads_dev,
                        int64_t* count);
/* yhat_dev[i] = net(X_dev row i); keeps the activations for mlp_bwd. */
dl_status mlp_fwd(dl_mlp* net, const float* X_dev, int32_t n, float* yhat_dev,
                  void* stream);
/* Back-propagate dy_dev (n, d loss / d yhat) through the last forward:
 * parameter gradients are overwritten; dX_dev (n x sizes[0], may be NULL)
 * receives d loss / d X (with dy = 1: the network's input gradient). */
dl_status mlp_bwd(dl_mlp* net, const float* dy_dev, int32_t n, float* dX_dev,
                  void* stream);
/* dy = 2 (yhat - y) / n for the mean squared error of the last forward;
 * loss_dev[0] = the loss (may be NULL). */
dl_status mlp_mse_grad(dl_mlp* net, const float* y_dev, int32_t n, float* dy_dev,
                       float* loss_dev, void* stream);
/* One Adam step (Kingma & Ba) of all parameters with the current gradients. */
dl_status mlp_adam(dl_mlp* net, float lr, float beta1, float beta2, float eps,
                   void* stream);

/* ---- launch profiling ------------------------------------------------------
 * Launch categories of the evaluation path.  With profiling enabled for a
 * category mask, every launch of those categories is bracketed by HIP events
 * on the stream it runs on; dl_ws_profile_end waits for them and returns,
 * per category, the summed kernel time, the number of launches and the
 * algorithmic floating-point operations and HBM bytes of those launches
 * (unpadded block sizes; operations that exist only because of padding or
 * of the inverse-based triangular solve are not counted).  For measurement
 * only; not for use while the workspace runs in two streams. */
enum {
  DL_CAT_POTRF_TILE = 0,  /* 64x64 diagonal-tile Cholesky + inverse       */
  DL_CAT_PANEL_TRSM = 1,  /* tiles below a diagonal tile times its inverse */
  DL_CAT_PANEL_SYRK = 2,  /* trailing update inside a diagonal block,
                             fused with the next diagonal tile's factor   */
  DL_CAT_TRTRI = 3,       /* inverse of the diagonal-block factor          */
  DL_CAT_TRSM = 4,        /* [B_t; R_t] L_tt^{-T}                          */
  DL_CAT_UPDATE = 5,      /* D_{t+1}, R_{t+1}, tip Schur updates           */
  DL_CAT_SOLVE = 6,       /* block forward/backward substitution           */
  DL_CAT_SELINV = 7,      /* selected-inversion block products             */
  DL_CAT_ASSEMBLE = 8,    /* sparse-to-dense assembly                      */
  DL_CAT_OTHER = 9,
  DL_NCAT = 10
};
/* With DL_PROFILE_BY_KERNEL or-ed into category_mask, launches of the
 * selected categories are aggregated by kernel instead (index = one of the
 * DL_KERNEL_* values below) -- the grouping a kernel-level profiler uses. */
enum {
  DL_PROFILE_BY_KERNEL = 1 << 16,
  DL_KERNEL_GEMM = 0,        /* the FP64 MFMA tile GEMM                  */
  DL_KERNEL_POTRF_TILE = 1,  /* 64x64 Cholesky + inverse                 */
  DL_KERNEL_GEMV = 2,        /* solve matrix-vector products             */
  DL_KERNEL_ASSEMBLE = 3,    /* assembly                                 */
  DL_KERNEL_OTHER = 4,
  DL_KERNEL_PANEL = 5,       /* fused trailing update + next tile factor */
  DL_KERNEL_GEMM_REDUCE = 6, /* sum of the pieces of split-k products    */
  DL_KERNEL_DAG = 7          /* persistent diagonal-block factorisation  */
};
dl_status dl_ws_profile_begin(dl_ws* ws, int32_t category_mask,
                              int32_t max_launches);
dl_status dl_ws_profile_end(dl_ws* ws, double* ms_by_cat,
                            int64_t* launches_by_cat, double* flops_by_cat,
                            double* bytes_by_cat);
/* Pause (on = 0) or resume (on != 0) the recording started by
 * dl_ws_profile_begin without touching its event pool, so that a caller can
 * bracket the launches of chosen calls only (each pair of events costs a
 * few microseconds of stream time).  Recording starts resumed. */
dl_status dl_ws_profile_enable(dl_ws* ws, int32_t on);

const char* dl_status_string(dl_status s);

#ifdef __cplusplus
}
#endif
#endif /* DALIA_H */
