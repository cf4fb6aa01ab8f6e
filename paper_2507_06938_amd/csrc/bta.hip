// Model and workspace management, launch plans of the BTA factorisation,
// solve and selected inversion, and the C-ABI entry points.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "model.hpp"
#include "selinv.hpp"
#include "solve.hpp"

namespace dl {

// ---- launch plans -----------------------------------------------------------------
//
// A plan is the theta-independent sequence of launches of one operation;
// GEMM task descriptors of every plan live in one device array built at
// workspace creation, so executing a plan allocates and copies nothing.

enum OpKind : int {
  OP_GEMM,
  OP_POTRF_TILE,
  OP_COPY_TILES,
  OP_FILL,
  OP_GEMV_N,
  OP_GEMV_T,
  OP_SUMLOG,
  OP_SELINV_FINISH,
  OP_DIAG,
  OP_COPY,
};

struct Op {
  OpKind kind;
  int task_off = 0, ntask = 0, ntiles = 0;
  PotrfTileArgs pt{};
  GemvN gn{};
  GemvT gt{};
  // generic pointers / sizes for the small ops
  const double* src = nullptr;
  double* dst = nullptr;
  double* aux = nullptr;
  int64_t n = 0, lds = 0, ldd = 0, sstride = 0, dstride = 0;
  int i0 = 0, i1 = 0;
  double v = 0.0;
  int cat = DL_CAT_OTHER;  // profiling category
  double flops = 0.0;      // algorithmic floating-point operations
  double bytes = 0.0;      // algorithmic HBM bytes
};

struct Plan {
  std::vector<Op> ops;
};

struct PlanBuilder {
  std::vector<GemmTask>& tasks;
  Plan& plan;

  void gemm(std::vector<GemmTask> ts, int cat = DL_CAT_OTHER, double flops = 0.0) {
    if (ts.empty()) return;
    Op op;
    op.kind = OP_GEMM;
    op.cat = cat;
    op.flops = flops;
    op.task_off = (int)tasks.size();
    op.ntask = (int)ts.size();
    op.ntiles = finalize_tasks(ts.data(), op.ntask);
    if (op.ntiles == 0) return;
    tasks.insert(tasks.end(), ts.begin(), ts.end());
    plan.ops.push_back(op);
  }
  void push(const Op& op) { plan.ops.push_back(op); }
};

static GemmTask mk(const double* A, int64_t lda, const double* B, int64_t ldb,
                   double* C, int64_t ldc, int M, int N, int K, int flags,
                   double alpha, double beta) {
  GemmTask t{};
  t.A = A; t.B = B; t.C = C;
  t.lda = lda; t.ldb = ldb; t.ldc = ldc;
  t.M = M; t.N = N; t.K = K; t.flags = flags;
  t.alpha = alpha; t.beta = beta;
  return t;
}

// Blocked right-looking Cholesky of the n x n block A (n multiple of 64):
// per 64-column panel j: factor the diagonal tile (and its inverse, kept in
// Gd), L(I,j) = A(I,j) L_jj^{-T} for the tiles below, then the lower
// trailing update A(I,J) -= L(I,j) L(J,j)^T.
static void add_potrf(PlanBuilder& pb, double* A, int64_t ld, int n, double* Gd,
                      double* logdiag, int64_t* info, int64_t row0,
                      int breal) {
  const int nbk = n / 64;
  for (int j = 0; j < nbk; ++j) {
    // algorithmic work of panel j restricted to the unpadded rows
    const double w = (double)std::max(0, std::min(64, breal - j * 64));
    const double below = (double)std::max(0, breal - (j + 1) * 64);
    Op op;
    op.kind = OP_POTRF_TILE;
    op.cat = DL_CAT_POTRF_TILE;
    op.flops = w * w * w / 3.0;
    op.pt.A = A + (int64_t)j * 64 * (ld + 1);
    op.pt.lda = ld;
    op.pt.Ginv = Gd + (int64_t)j * 4096;
    op.pt.logdiag = logdiag + (int64_t)j * 64;
    op.pt.info = info;
    op.pt.row0 = row0 + (int64_t)j * 64;
    pb.push(op);
    if (j + 1 < nbk) {
      const int rows = n - (j + 1) * 64;
      double* panel = A + (int64_t)(j + 1) * 64 + (int64_t)j * 64 * ld;
      pb.gemm({mk(panel, ld, Gd + (int64_t)j * 4096, 64, panel, ld, rows, 64, 64,
                  F_TB | F_BETA0, 1.0, 0.0)},
              DL_CAT_PANEL_TRSM, below * w * w);
      pb.gemm({mk(panel, ld, panel, ld, A + (int64_t)(j + 1) * 64 * (ld + 1), ld,
                  rows, rows, 64, F_TB | F_LOWER, -1.0, 1.0)},
              DL_CAT_PANEL_SYRK, below * below * w);
    }
  }
}

// In-place inverse of the lower-triangular factor (diagonal tiles' inverses
// in Gd): recursive halving, G21 = -G22 (L21 G11), all nodes of one depth
// in one launch, deepest first.  temp holds n x (n/2) doubles (ld n).
static void collect_nodes(int lo, int hi, int depth,
                          std::vector<std::vector<int>>& lv) {
  if (hi - lo <= 1) return;
  const int mid = lo + (hi - lo) / 2;
  if ((int)lv.size() <= depth) lv.resize(depth + 1);
  lv[depth].push_back(lo);
  lv[depth].push_back(hi);
  collect_nodes(lo, mid, depth + 1, lv);
  collect_nodes(mid, hi, depth + 1, lv);
}

// `breal`: unpadded size for the algorithmic operation count (0: the
// inverse is not part of the algorithm being counted).
static void add_trtri(PlanBuilder& pb, double* A, int64_t ld, int n,
                      const double* Gd, double* temp, int breal = 0) {
  auto ext = [&](int lo, int hi) {
    return (double)std::max(0, std::min(hi * 64, breal) - lo * 64);
  };
  const int nbk = n / 64;
  Op cp;
  cp.kind = OP_COPY_TILES;
  cp.src = Gd; cp.lds = 64; cp.sstride = 4096;
  cp.dst = A; cp.ldd = ld; cp.dstride = 64 * (ld + 1);
  cp.n = nbk;
  cp.cat = DL_CAT_TRTRI;
  pb.push(cp);
  // (the 64x64 diagonal inverses come from the tile factorisation)
  std::vector<std::vector<int>> lv;
  collect_nodes(0, nbk, 0, lv);
  for (int d = (int)lv.size() - 1; d >= 0; --d) {
    std::vector<GemmTask> tT, tG;
    double fT = 0.0, fG = 0.0;
    for (size_t q = 0; q < lv[d].size(); q += 2) {
      const int lo = lv[d][q], hi = lv[d][q + 1];
      const int mid = lo + (hi - lo) / 2;
      const int n1 = (mid - lo) * 64, n2 = (hi - mid) * 64;
      double* L21 = A + (int64_t)mid * 64 + (int64_t)lo * 64 * ld;
      double* G11 = A + (int64_t)lo * 64 * (ld + 1);
      double* G22 = A + (int64_t)mid * 64 * (ld + 1);
      double* T = temp + (int64_t)lo * 64;
      tT.push_back(mk(L21, ld, G11, ld, T, n, n2, n1, n1, F_KLO_COL | F_BETA0,
                      1.0, 0.0));
      tG.push_back(mk(G22, ld, T, n, L21, ld, n2, n1, n2, F_KHI_ROW | F_BETA0,
                      -1.0, 0.0));
      const double r1 = ext(lo, mid), r2 = ext(mid, hi);
      fT += r2 * r1 * r1;   // full times triangular
      fG += r1 * r2 * r2;
    }
    pb.gemm(tT, DL_CAT_TRTRI, fT);
    pb.gemm(tG, DL_CAT_TRTRI, fG);
  }
}

}  // namespace dl

using namespace dl;

// ---- model -------------------------------------------------------------------------

struct dl_model {
  ModelDev d{};
  std::vector<void*> allocs;
  int64_t m_host[3] = {0, 0, 0};
};

struct MatrixStore {
  double* D = nullptr;    // nt x bp x bp
  double* BR = nullptr;   // (nt+1) slots of ldbr x bp
  double* P = nullptr;    // ap x ap
  double* GP = nullptr;   // ap x ap inverse of the tip factor
  int64_t ldbr = 0;
  int ap = 0;             // arrow rows stored in BR (0 for Q_p)
  std::vector<int> slot_init, slot_final;
  Plan factor;
  bool assembled = false, factored = false;
};

struct dl_ws {
  const dl_model* model = nullptr;
  ModelDev m{};
  std::vector<void*> allocs;
  size_t bytes = 0;
  MatrixStore q[2];
  double* Gd[2] = {nullptr, nullptr};
  double* ttemp[2] = {nullptr, nullptr};
  double* logdiag[2] = {nullptr, nullptr};
  double* coef = nullptr;
  double* logdet2 = nullptr;   // [2]
  int64_t* info2 = nullptr;    // [2]
  double* quad2 = nullptr;     // [2]
  double* sumpart = nullptr;   // 2 x 256
  double* qpart = nullptr;     // 2 x 512
  double* rhs = nullptr;       // Np
  double* x = nullptr;         // Np
  double* mu = nullptr;        // Np
  double* u = nullptr;         // ldbr
  double* gpart = nullptr;     // GEMV_MAX_KS x ldbr
  // selected inversion
  bool sel = false;
  double* WV = nullptr;
  double* Y = nullptr;
  double* XC[2] = {nullptr, nullptr};
  double* selout = nullptr;    // Np
  Plan solve, selinv;
  GemmTask* tasks_dev = nullptr;
  bool solved = false;
  // launch profiling (measurement only)
  int prof_mask = 0;
  std::vector<hipEvent_t> prof_ev;   // start/stop pairs
  std::vector<int> prof_cat;
  std::vector<double> prof_flops, prof_bytes;
  int prof_used = 0;
  int prof_by_kernel = 0;  // aggregate by kernel kind instead of category
};

static int prof_begin(dl_ws* W, int cat, hipStream_t s, int kind = DL_KERNEL_OTHER) {
  if (!W->prof_mask || !((W->prof_mask >> cat) & 1)) return -1;
  if (W->prof_used >= (int)W->prof_cat.size()) return -1;
  const int k = W->prof_used++;
  if (hipEventRecord(W->prof_ev[2 * k], s) != hipSuccess) return -1;
  W->prof_cat[k] = W->prof_by_kernel ? kind : cat;
  return k;
}

static void prof_end(dl_ws* W, int k, double flops, double bytes,
                     hipStream_t s) {
  if (k < 0) return;
  (void)hipEventRecord(W->prof_ev[2 * k + 1], s);
  W->prof_flops[k] = flops;
  W->prof_bytes[k] = bytes;
}

static dl_status dev_alloc(std::vector<void*>& list, size_t bytes, void** out,
                           size_t* counter = nullptr) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(&p, bytes) != hipSuccess) return DL_ENOMEM;
  list.push_back(p);
  if (counter) *counter += bytes;
  *out = p;
  return DL_OK;
}

template <typename T>
static dl_status upload(std::vector<void*>& list, const std::vector<T>& h,
                        const T** out) {
  void* p = nullptr;
  dl_status st = dev_alloc(list, h.size() * sizeof(T), &p);
  if (st != DL_OK) return st;
  if (!h.empty() &&
      hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) !=
          hipSuccess)
    return DL_EHIP;
  *out = (const T*)p;
  return DL_OK;
}

extern "C" int32_t dl_theta_dim(int32_t nv) {
  return nv == 1 ? 4 : 4 * nv + nv * (nv - 1) / 2;
}

extern "C" const char* dl_status_string(dl_status s) {
  switch (s) {
    case DL_OK: return "ok";
    case DL_EINVAL: return "invalid argument";
    case DL_ENOMEM: return "device allocation failed";
    case DL_ENOTSPD: return "matrix not positive definite";
    case DL_EHIP: return "HIP runtime error";
    case DL_ESTATE: return "call order violated";
    case DL_ENOTCONV: return "iterative refinement did not converge";
  }
  return "unknown status";
}

static void free_all(std::vector<void*>& list) {
  for (void* p : list) (void)hipFree(p);
  list.clear();
}

extern "C" dl_status dl_model_create(const dl_model_desc* desc,
                                     dl_model** out) {
  if (!desc || !out) return DL_EINVAL;
  const int nx = desc->nx, nt = desc->nt, nv = desc->nv, nr = desc->nr;
  if (nx < 2 || nt < 1 || nv < 1 || nv > 3 || nr < 0 || nv * nr > 64 ||
      (2 * ((nv * nx * nx + 63) / 64) * 64 + 64) * 8 > 160 * 1024)
    return DL_EINVAL;
  if (!desc->theta_prior_mean || !(desc->theta_prior_sd > 0.0)) return DL_EINVAL;
  const int ns = nx * nx;
  for (int j = 0; j < nv; ++j) {
    if (desc->m[j] < 0) return DL_EINVAL;
    if (desc->m[j] > 0 && (!desc->obs_t[j] || !desc->obs_nodes[j] ||
                           !desc->obs_w[j] || !desc->y[j] ||
                           (nr > 0 && !desc->obs_x[j])))
      return DL_EINVAL;
    for (int64_t i = 0; i < desc->m[j]; ++i) {
      if (desc->obs_t[j][i] < 0 || desc->obs_t[j][i] >= nt) return DL_EINVAL;
      for (int q = 0; q < 3; ++q) {
        const int s = desc->obs_nodes[j][3 * i + q];
        if (s < 0 || s >= ns) return DL_EINVAL;
      }
    }
  }
  dl_model* M = new (std::nothrow) dl_model();
  if (!M) return DL_ENOMEM;
  ModelDev& d = M->d;
  d.nx = nx; d.nt = nt; d.nv = nv; d.nr = nr; d.ns = ns;
  d.b = nv * ns; d.a = nv * nr;
  d.bp = ((d.b + 63) / 64) * 64;
  d.ap = d.a > 0 ? 64 : 0;
  d.dim_theta = dl_theta_dim(nv);
  d.N = (int64_t)nt * d.b + d.a;
  d.Np = (int64_t)nt * d.bp + d.ap;
  d.theta_prior_sd = desc->theta_prior_sd;
  d.prior_fixed = desc->prior_fixed;

  // FEM pieces on the grid: C = I (lumped mass, unit spacing), G = 5-point
  // Neumann graph Laplacian, G C^-1 G = G*G.  Pattern: 13-point stencil.
  std::vector<int> ptr(ns + 1, 0), col;
  std::vector<double> vC, vG, vG2;
  auto deg = [&](int ix, int iy) {
    return (ix > 0) + (ix < nx - 1) + (iy > 0) + (iy < nx - 1);
  };
  auto gval = [&](int ax, int ay, int bx, int by) -> double {
    if (ax == bx && ay == by) return (double)deg(ax, ay);
    if (abs(ax - bx) + abs(ay - by) == 1) return -1.0;
    return 0.0;
  };
  for (int iy = 0; iy < nx; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      const int s = iy * nx + ix;
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          if (abs(dx) + abs(dy) > 2) continue;
          const int jx = ix + dx, jy = iy + dy;
          if (jx < 0 || jy < 0 || jx >= nx || jy >= nx) continue;
          // (G G)(s, s') = sum over k of G(s,k) G(k,s'), k within 1 of both
          double g2 = 0.0;
          for (int ky = iy - 1; ky <= iy + 1; ++ky)
            for (int kx = ix - 1; kx <= ix + 1; ++kx) {
              if (kx < 0 || ky < 0 || kx >= nx || ky >= nx) continue;
              if (abs(kx - ix) + abs(ky - iy) > 1) continue;
              g2 += gval(ix, iy, kx, ky) * gval(kx, ky, jx, jy);
            }
          const double c = (dx == 0 && dy == 0) ? 1.0 : 0.0;
          const double g = gval(ix, iy, jx, jy);
          if (c == 0.0 && g == 0.0 && g2 == 0.0) continue;
          col.push_back(jy * nx + jx);
          vC.push_back(c);
          vG.push_back(g);
          vG2.push_back(g2);
        }
      ptr[s + 1] = (int)col.size();
    }

  // observations, concatenated; node -> rows index per (response, time, node)
  int64_t mt = 0;
  d.m_off[0] = 0;
  for (int j = 0; j < nv; ++j) {
    M->m_host[j] = desc->m[j];
    mt += desc->m[j];
    d.m_off[j + 1] = mt;
  }
  for (int j = nv; j < 3; ++j) d.m_off[j + 1] = mt;
  d.m_total = mt;
  std::vector<int> ot(mt), on(3 * mt);
  std::vector<double> ow(3 * mt), ox((size_t)mt * (nr > 0 ? nr : 1)), oy(mt);
  const int64_t nkeys = (int64_t)nv * nt * ns;
  std::vector<int64_t> nptr(nkeys + 1, 0);
  for (int j = 0; j < nv; ++j) {
    const int64_t o = d.m_off[j];
    for (int64_t i = 0; i < desc->m[j]; ++i) {
      ot[o + i] = desc->obs_t[j][i];
      oy[o + i] = desc->y[j][i];
      for (int q = 0; q < 3; ++q) {
        on[3 * (o + i) + q] = desc->obs_nodes[j][3 * i + q];
        ow[3 * (o + i) + q] = desc->obs_w[j][3 * i + q];
        const int64_t key = ((int64_t)j * nt + ot[o + i]) * ns + on[3 * (o + i) + q];
        nptr[key + 1]++;
      }
      for (int r = 0; r < nr; ++r) ox[(o + i) * nr + r] = desc->obs_x[j][i * nr + r];
    }
  }
  for (int64_t k = 0; k < nkeys; ++k) nptr[k + 1] += nptr[k];
  std::vector<int> nrow(nptr[nkeys]), nq(nptr[nkeys]);
  {
    std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
    for (int j = 0; j < nv; ++j) {
      const int64_t o = d.m_off[j];
      for (int64_t i = 0; i < desc->m[j]; ++i)
        for (int q = 0; q < 3; ++q) {
          const int64_t key = ((int64_t)j * nt + ot[o + i]) * ns + on[3 * (o + i) + q];
          nrow[fill[key]] = (int)(o + i);
          nq[fill[key]] = q;
          fill[key]++;
        }
    }
  }
  std::vector<double> pm(desc->theta_prior_mean,
                         desc->theta_prior_mean + d.dim_theta);
  dl_status st = DL_OK;
  if ((st = upload(M->allocs, ptr, &d.sp_ptr)) != DL_OK ||
      (st = upload(M->allocs, col, &d.sp_col)) != DL_OK ||
      (st = upload(M->allocs, vC, &d.sp_C)) != DL_OK ||
      (st = upload(M->allocs, vG, &d.sp_G)) != DL_OK ||
      (st = upload(M->allocs, vG2, &d.sp_G2)) != DL_OK ||
      (st = upload(M->allocs, ot, &d.obs_t)) != DL_OK ||
      (st = upload(M->allocs, on, &d.obs_nodes)) != DL_OK ||
      (st = upload(M->allocs, ow, &d.obs_w)) != DL_OK ||
      (st = upload(M->allocs, ox, &d.obs_x)) != DL_OK ||
      (st = upload(M->allocs, oy, &d.obs_y)) != DL_OK ||
      (st = upload(M->allocs, nptr, &d.no_ptr)) != DL_OK ||
      (st = upload(M->allocs, nrow, &d.no_row)) != DL_OK ||
      (st = upload(M->allocs, nq, &d.no_q)) != DL_OK ||
      (st = upload(M->allocs, pm, &d.theta_prior_mean)) != DL_OK) {
    free_all(M->allocs);
    delete M;
    return st;
  }
  *out = M;
  return DL_OK;
}

extern "C" void dl_model_destroy(dl_model* M) {
  if (!M) return;
  free_all(M->allocs);
  delete M;
}

extern "C" dl_status dl_model_dims(const dl_model* M, int64_t* n, int64_t* b,
                                   int64_t* a, int64_t* N, int64_t* bp) {
  if (!M) return DL_EINVAL;
  if (n) *n = M->d.nt;
  if (b) *b = M->d.b;
  if (a) *a = M->d.a;
  if (N) *N = M->d.N;
  if (bp) *bp = M->d.bp;
  return DL_OK;
}

// ---- workspace and plans ----------------------------------------------------------------

static void build_factor_plan(dl_ws* W, int which,
                              std::vector<GemmTask>& tasks) {
  const ModelDev& m = W->m;
  MatrixStore& Q = W->q[which];
  PlanBuilder pb{tasks, Q.factor};
  const int bp = m.bp;
  const int64_t ldbr = Q.ldbr;
  const int apr = Q.ap;  // arrow rows in BR
  std::vector<int> slot(m.nt + 1);
  for (int t = 0; t <= m.nt; ++t) slot[t] = t;
  int spare = m.nt;
  auto BRs = [&](int sl) { return Q.BR + (int64_t)sl * ldbr * bp; };
  Q.slot_init.assign(slot.begin(), slot.begin() + m.nt);
  for (int t = 0; t < m.nt; ++t) {
    double* Dt = Q.D + (int64_t)t * bp * bp;
    add_potrf(pb, Dt, bp, bp, W->Gd[which], W->logdiag[which] + (int64_t)t * bp,
              W->info2 + which, (int64_t)t * m.b, m.b);
    // L_tt^{-1} is algorithmic work of the selected inversion (Q_c with
    // selected inversion enabled); otherwise it only serves the
    // inverse-based triangular solves and is not counted.
    add_trtri(pb, Dt, bp, bp, W->Gd[which], W->ttemp[which],
              (which == 1 && W->sel) ? m.b : 0);
    const bool last = (t + 1 == m.nt);
    const int rows_lo = last ? bp : 0;
    const int M = (last ? 0 : bp) + apr;
    if (M > 0) {
      const int nw = spare;
      // [B_t; R_t] <- [B_t; R_t] L_tt^{-T} = [B_t; R_t] G_t^T
      const double b = m.b, ar = apr ? m.a : 0;
      const double mreal = (last ? 0.0 : b) + ar;
      pb.gemm({mk(BRs(slot[t]) + rows_lo, ldbr, Dt, bp, BRs(nw) + rows_lo, ldbr,
                  M, bp, bp, F_TB | F_KHI_COL | F_BETA0, 1.0, 0.0)},
              DL_CAT_TRSM, mreal * b * b);
      spare = slot[t];
      slot[t] = nw;
      std::vector<GemmTask> up;
      double* BRt = BRs(slot[t]);
      if (!last) {
        double* Dn = Q.D + (int64_t)(t + 1) * bp * bp;
        up.push_back(mk(BRt, ldbr, BRt, ldbr, Dn, bp, bp, bp, bp,
                        F_TB | F_LOWER, -1.0, 1.0));
        if (apr)
          up.push_back(mk(BRt + bp, ldbr, BRt, ldbr, BRs(slot[t + 1]) + bp, ldbr,
                          apr, bp, bp, F_TB, -1.0, 1.0));
      }
      if (apr)
        up.push_back(mk(BRt + bp, ldbr, BRt + bp, ldbr, Q.P, m.ap, apr, apr, bp,
                        F_TB | F_LOWER, -1.0, 1.0));
      const double upd = (last ? 0.0 : b * b * b + 2.0 * ar * b * b) + ar * ar * b;
      pb.gemm(up, DL_CAT_UPDATE, upd);
    }
  }
  if (m.ap > 0) {
    Op op;
    op.kind = OP_POTRF_TILE;
    op.cat = DL_CAT_POTRF_TILE;
    op.flops = (double)m.a * m.a * m.a / 3.0;
    op.pt.A = Q.P;
    op.pt.lda = m.ap;
    op.pt.Ginv = Q.GP;
    op.pt.logdiag = W->logdiag[which] + (int64_t)m.nt * bp;
    op.pt.info = W->info2 + which;
    op.pt.row0 = (int64_t)m.nt * m.b;
    pb.push(op);
  }
  Op sl;
  sl.kind = OP_SUMLOG;
  sl.src = W->logdiag[which];
  sl.n = m.Np;
  sl.v = 2.0;
  sl.dst = W->logdet2 + which;
  sl.aux = W->sumpart + which * 256;
  pb.push(sl);
  Q.slot_final.assign(slot.begin(), slot.begin() + m.nt);
}

static void build_solve_plan(dl_ws* W, std::vector<GemmTask>& tasks) {
  (void)tasks;
  const ModelDev& m = W->m;
  MatrixStore& Q = W->q[1];
  Plan& P = W->solve;
  const int bp = m.bp, ap = Q.ap;
  const int64_t ldbr = Q.ldbr;
  auto BRs = [&](int t) { return Q.BR + (int64_t)Q.slot_final[t] * ldbr * bp; };
  auto G = [&](int t) { return Q.D + (int64_t)t * bp * bp; };
  double* x = W->x;
  double* xP = x + (int64_t)m.nt * bp;
  double* mu = W->mu;
  double* muP = mu + (int64_t)m.nt * bp;
  // algorithmic bytes: the unpadded part of the matrix read once
  auto mb = [&](int rows, int cols, int tri) {
    const double r = std::min(rows, rows == ap ? m.a : (rows > bp ? m.b + m.a : m.b));
    const double c = std::min(cols, cols == ap ? m.a : m.b);
    return 8.0 * (tri ? 0.5 * r * c : r * c);
  };
  auto gn = [&](GemvN g) {
    Op o; o.kind = OP_GEMV_N; o.gn = g; o.cat = DL_CAT_SOLVE;
    o.bytes = mb(g.M, g.K, g.tri); o.flops = o.bytes / 4.0; P.ops.push_back(o);
  };
  auto gt = [&](GemvT g) {
    Op o; o.kind = OP_GEMV_T; o.gt = g; o.cat = DL_CAT_SOLVE;
    o.bytes = mb(g.M, g.N, g.tri); o.flops = o.bytes / 4.0; P.ops.push_back(o);
  };
  // forward: L z = r
  for (int t = 0; t < m.nt; ++t) {
    double* xt = x + (int64_t)t * bp;
    if (t == 0) {
      gn({bp, bp, G(0), bp, xt, 1, 1.0, 0.0, -1, nullptr, xt, nullptr, nullptr});
    } else {
      gn({bp + ap, bp, BRs(t - 1), ldbr, x + (int64_t)(t - 1) * bp, 0, -1.0, 1.0,
          bp, xt, W->u, xP, xP});
      gn({bp, bp, G(t), bp, W->u, 1, 1.0, 0.0, -1, nullptr, xt, nullptr, nullptr});
    }
  }
  if (ap > 0) {
    gn({ap, bp, BRs(m.nt - 1) + bp, ldbr, x + (int64_t)(m.nt - 1) * bp, 0, -1.0,
        1.0, -1, xP, xP, nullptr, nullptr});
    gn({ap, ap, Q.GP, ap, xP, 1, 1.0, 0.0, -1, nullptr, xP, nullptr, nullptr});
    // backward: L^T mu = z
    gt({ap, ap, Q.GP, ap, xP, -1, nullptr, 1, 1.0, 0.0, nullptr, muP});
  }
  for (int t = m.nt - 1; t >= 0; --t) {
    double* xt = x + (int64_t)t * bp;
    if (t == m.nt - 1) {
      if (ap > 0) {
        gt({ap, bp, BRs(t) + bp, ldbr, muP, -1, nullptr, 0, -1.0, 1.0, xt, W->u});
      } else {
        Op c; c.kind = OP_COPY; c.src = xt; c.dst = W->u; c.n = bp; P.ops.push_back(c);
      }
    } else {
      gt({bp + ap, bp, BRs(t), ldbr, mu + (int64_t)(t + 1) * bp, bp, muP, 0, -1.0,
          1.0, xt, W->u});
    }
    gt({bp, bp, G(t), bp, W->u, -1, nullptr, 1, 1.0, 0.0, nullptr,
        mu + (int64_t)t * bp});
  }
}

static void build_selinv_plan(dl_ws* W, std::vector<GemmTask>& tasks) {
  const ModelDev& m = W->m;
  MatrixStore& Q = W->q[1];
  PlanBuilder pb{tasks, W->selinv};
  const int bp = m.bp, ap = Q.ap;
  const int64_t ld = Q.ldbr;  // bp + ap
  auto BRs = [&](int t) { return Q.BR + (int64_t)Q.slot_final[t] * ld * bp; };
  auto G = [&](int t) { return Q.D + (int64_t)t * bp * bp; };
  for (int k = 0; k < 2; ++k) {
    Op f; f.kind = OP_FILL; f.dst = W->XC[k]; f.n = ld * ld; f.v = 0.0;
    pb.push(f);
  }
  if (ap > 0) {
    // X_P = G_P^T G_P into the corner of both ping-pong buffers
    std::vector<GemmTask> xp;
    for (int k = 0; k < 2; ++k)
      xp.push_back(mk(Q.GP, ap, Q.GP, ap, W->XC[k] + bp + (int64_t)bp * ld, ld,
                      ap, ap, ap, F_TA | F_BETA0, 1.0, 0.0));
    pb.gemm(xp, DL_CAT_SELINV, 2.0 * (double)m.a * m.a * m.a);
    Op dg; dg.kind = OP_DIAG; dg.src = W->XC[0] + bp + (int64_t)bp * ld; dg.lds = ld;
    dg.n = ap; dg.dst = W->selout + (int64_t)m.nt * bp;
    pb.push(dg);
  }
  int cur = 0;
  for (int t = m.nt - 1; t >= 0; --t) {
    const int nxt = cur ^ 1;
    const bool last = (t + 1 == m.nt);
    if (last) {
      Op f; f.kind = OP_FILL; f.dst = W->WV; f.n = ld * bp; f.v = 0.0;
      pb.push(f);
      if (ap > 0)
        pb.gemm({mk(BRs(t) + bp, ld, G(t), bp, W->WV + bp, ld, ap, bp, bp,
                    F_KLO_COL | F_BETA0, 1.0, 0.0)},
                DL_CAT_SELINV, (double)m.a * m.b * m.b);
    } else {
      // [W_t; V_t] = [B_t; R_t]_factor G_t
      pb.gemm({mk(BRs(t), ld, G(t), bp, W->WV, ld, bp + ap, bp, bp,
                  F_KLO_COL | F_BETA0, 1.0, 0.0)},
              DL_CAT_SELINV, ((double)m.b + m.a) * m.b * m.b);
    }
    const double ba = (double)m.b + m.a, bb = (double)m.b;
    // [X_{t+1,t}; X_{P,t}] = -[[X_{t+1,t+1}, X_{t+1,P}]; [X_{P,t+1}, X_P]] WV
    pb.gemm({mk(W->XC[cur], ld, W->WV, ld, W->Y, ld, bp + ap, bp, bp + ap,
                F_BETA0, -1.0, 0.0)},
            DL_CAT_SELINV, last ? 2.0 * m.a * ba * bb : 2.0 * ba * ba * bb);
    // X_tt = G_t^T G_t - Y^T WV   (lower triangle)
    pb.gemm({mk(G(t), bp, G(t), bp, W->XC[nxt], ld, bp, bp, bp,
                F_TA | F_KLO_ROW | F_KLO_COL | F_LOWER | F_BETA0, 1.0, 0.0)},
            DL_CAT_SELINV, bb * bb * bb / 3.0);
    pb.gemm({mk(W->Y, ld, W->WV, ld, W->XC[nxt], ld, bp, bp, bp + ap,
                F_TA | F_LOWER, -1.0, 1.0)},
            DL_CAT_SELINV, last ? bb * bb * m.a : bb * bb * ba);
    Op fin;
    fin.kind = OP_SELINV_FINISH;
    fin.cat = DL_CAT_SELINV;
    fin.dst = W->XC[nxt];
    fin.src = W->Y;
    fin.aux = W->selout + (int64_t)t * bp;
    pb.push(fin);
    cur = nxt;
  }
}

static hipError_t run_plan(dl_ws* W, const Plan& P, hipStream_t s) {
  const ModelDev& m = W->m;
  for (const Op& op : P.ops) {
    hipError_t e = hipSuccess;
    int kind = DL_KERNEL_OTHER;
    if (op.kind == OP_GEMM) kind = DL_KERNEL_GEMM;
    else if (op.kind == OP_POTRF_TILE) kind = DL_KERNEL_POTRF_TILE;
    else if (op.kind == OP_GEMV_N || op.kind == OP_GEMV_T) kind = DL_KERNEL_GEMV;
    const int pk = prof_begin(W, op.cat, s, kind);
    switch (op.kind) {
      case OP_GEMM:
        e = launch_gemm_tasks(W->tasks_dev + op.task_off, op.ntask, op.ntiles, s);
        break;
      case OP_POTRF_TILE: e = launch_potrf_tile(op.pt, s); break;
      case OP_COPY_TILES:
        e = launch_copy_tile64(op.src, op.lds, op.dst, op.ldd, (int)op.n,
                               op.sstride, op.dstride, s);
        break;
      case OP_FILL: e = launch_fill(op.dst, op.n, op.v, s); break;
      case OP_GEMV_N: e = launch_gemv_n(op.gn, W->gpart, s); break;
      case OP_GEMV_T: e = launch_gemv_t(op.gt, s); break;
      case OP_SUMLOG: e = launch_sum_log(op.src, op.n, op.v, op.dst, op.aux, s); break;
      case OP_SELINV_FINISH:
        e = launch_selinv_finish(op.dst, W->q[1].ldbr, m.bp, W->q[1].ap, op.src,
                                 op.aux, s);
        break;
      case OP_DIAG: e = launch_diag_copy(op.src, op.lds, (int)op.n, op.dst, s); break;
      case OP_COPY: e = launch_copy(op.src, op.dst, op.n, s); break;
    }
    prof_end(W, pk, op.flops, op.bytes, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

extern "C" dl_status dl_ws_create(const dl_model* model, int32_t flags,
                                  dl_ws** out) {
  if (!model || !out) return DL_EINVAL;
  dl_ws* W = new (std::nothrow) dl_ws();
  if (!W) return DL_ENOMEM;
  W->model = model;
  W->m = model->d;
  const ModelDev& m = W->m;
  W->sel = (flags & 1) != 0;
  const int bp = m.bp, ap = m.ap;
  const int64_t bb = (int64_t)bp * bp;
  dl_status st = DL_OK;
  auto A = [&](size_t bytes, void** p) {
    if (st == DL_OK) st = dev_alloc(W->allocs, bytes, p, &W->bytes);
  };
  for (int w = 0; w < 2; ++w) {
    MatrixStore& Q = W->q[w];
    Q.ap = (w == 1) ? ap : 0;
    Q.ldbr = bp + Q.ap;
    A(sizeof(double) * m.nt * bb, (void**)&Q.D);
    A(sizeof(double) * (m.nt + 1) * Q.ldbr * bp, (void**)&Q.BR);
    A(sizeof(double) * (ap > 0 ? ap * ap : 1), (void**)&Q.P);
    A(sizeof(double) * (ap > 0 ? ap * ap : 1), (void**)&Q.GP);
    A(sizeof(double) * bp * 64, (void**)&W->Gd[w]);
    A(sizeof(double) * bp * (int64_t)((bp / 64) / 2 + 1) * 64, (void**)&W->ttemp[w]);
    A(sizeof(double) * m.Np, (void**)&W->logdiag[w]);
  }
  const int64_t ldbr = bp + ap;
  A(sizeof(double) * C_SIZE, (void**)&W->coef);
  A(sizeof(double) * 2, (void**)&W->logdet2);
  A(sizeof(int64_t) * 2, (void**)&W->info2);
  A(sizeof(double) * 2, (void**)&W->quad2);
  A(sizeof(double) * 512, (void**)&W->sumpart);
  A(sizeof(double) * 1024, (void**)&W->qpart);
  A(sizeof(double) * m.Np, (void**)&W->rhs);
  A(sizeof(double) * m.Np, (void**)&W->x);
  A(sizeof(double) * m.Np, (void**)&W->mu);
  A(sizeof(double) * ldbr, (void**)&W->u);
  A(sizeof(double) * GEMV_MAX_KS * ldbr, (void**)&W->gpart);
  if (W->sel) {
    A(sizeof(double) * ldbr * bp, (void**)&W->WV);
    A(sizeof(double) * ldbr * bp, (void**)&W->Y);
    A(sizeof(double) * ldbr * ldbr, (void**)&W->XC[0]);
    A(sizeof(double) * ldbr * ldbr, (void**)&W->XC[1]);
    A(sizeof(double) * m.Np, (void**)&W->selout);
  }
  if (st != DL_OK) {
    free_all(W->allocs);
    delete W;
    return st;
  }
  std::vector<GemmTask> tasks;
  build_factor_plan(W, 0, tasks);
  build_factor_plan(W, 1, tasks);
  build_solve_plan(W, tasks);
  if (W->sel) build_selinv_plan(W, tasks);
  A(sizeof(GemmTask) * (tasks.size() + 1), (void**)&W->tasks_dev);
  if (st == DL_OK && !tasks.empty() &&
      hipMemcpy(W->tasks_dev, tasks.data(), sizeof(GemmTask) * tasks.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    st = DL_EHIP;
  if (st != DL_OK) {
    free_all(W->allocs);
    delete W;
    return st;
  }
  *out = W;
  return DL_OK;
}

static void prof_free(dl_ws* W) {
  for (hipEvent_t e : W->prof_ev) (void)hipEventDestroy(e);
  W->prof_ev.clear();
  W->prof_cat.clear();
  W->prof_flops.clear();
  W->prof_bytes.clear();
  W->prof_used = 0;
  W->prof_mask = 0;
}

extern "C" dl_status dl_ws_profile_begin(dl_ws* W, int32_t mask,
                                         int32_t max_launches) {
  if (!W || max_launches <= 0 || (mask & 0xffff) == 0) return DL_EINVAL;
  prof_free(W);
  W->prof_by_kernel = (mask & DL_PROFILE_BY_KERNEL) ? 1 : 0;
  mask &= 0xffff;
  W->prof_ev.resize(2 * (size_t)max_launches);
  for (auto& e : W->prof_ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      prof_free(W);
      return DL_EHIP;
    }
  W->prof_cat.assign(max_launches, 0);
  W->prof_flops.assign(max_launches, 0.0);
  W->prof_bytes.assign(max_launches, 0.0);
  W->prof_mask = mask;
  return DL_OK;
}

extern "C" dl_status dl_ws_profile_end(dl_ws* W, double* ms, int64_t* launches,
                                       double* flops, double* bytes) {
  if (!W) return DL_EINVAL;
  for (int c = 0; c < DL_NCAT; ++c) {
    if (ms) ms[c] = 0.0;
    if (launches) launches[c] = 0;
    if (flops) flops[c] = 0.0;
    if (bytes) bytes[c] = 0.0;
  }
  dl_status st = DL_OK;
  for (int k = 0; k < W->prof_used; ++k) {
    if (hipEventSynchronize(W->prof_ev[2 * k + 1]) != hipSuccess) { st = DL_EHIP; break; }
    float t = 0.f;
    if (hipEventElapsedTime(&t, W->prof_ev[2 * k], W->prof_ev[2 * k + 1]) !=
        hipSuccess) { st = DL_EHIP; break; }
    const int c = W->prof_cat[k];
    if (ms) ms[c] += t;
    if (launches) launches[c] += 1;
    if (flops) flops[c] += W->prof_flops[k];
    if (bytes) bytes[c] += W->prof_bytes[k];
  }
  prof_free(W);
  return st;
}

extern "C" void dl_ws_destroy(dl_ws* W) {
  if (!W) return;
  prof_free(W);
  free_all(W->allocs);
  delete W;
}

extern "C" size_t dl_ws_bytes(const dl_ws* W) { return W ? W->bytes : 0; }

// ---- entry points -------------------------------------------------------------------------

static AssembleOut assemble_out(dl_ws* W, dl_which which) {
  AssembleOut o{};
  const bool p = which == DL_QP || which == DL_BOTH;
  const bool c = which == DL_QC || which == DL_BOTH;
  if (p) { o.Dp = W->q[0].D; o.Bp = W->q[0].BR; o.Pp = W->q[0].P; }
  if (c) { o.Dc = W->q[1].D; o.BRc = W->q[1].BR; o.Pc = W->q[1].P; }
  o.rhs = W->rhs;
  return o;
}

extern "C" dl_status bta_assemble(dl_ws* W, const double* theta_dev,
                                  dl_which which, void* stream) {
  if (!W || !theta_dev || which < DL_QP || which > DL_BOTH) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  DL_HIP_CHECK(launch_theta_coeffs(W->m, theta_dev, W->coef, s));
  const int pk = prof_begin(W, DL_CAT_ASSEMBLE, s, DL_KERNEL_ASSEMBLE);
  DL_HIP_CHECK(launch_assemble(W->m, W->coef, assemble_out(W, which), s));
  {
    // dense workspace written (unpadded): diagonal and sub-diagonal blocks,
    // plus the arrow and tip for Q_c
    const double n = W->m.nt, b = W->m.b, a = W->m.a;
    const double qp = n * b * b + (n - 1) * b * b + a * a;
    const double qc = qp + n * a * b;
    const double by = 8.0 * ((which != DL_QC ? qp : 0.0) + (which != DL_QP ? qc : 0.0));
    prof_end(W, pk, 0.0, by, s);
  }
  if (which != DL_QC) { W->q[0].assembled = true; W->q[0].factored = false; }
  if (which != DL_QP) { W->q[1].assembled = true; W->q[1].factored = false; }
  W->solved = false;
  return DL_OK;
}

static dl_status factor_one(dl_ws* W, int w, hipStream_t s) {
  if (!W->q[w].assembled) return DL_ESTATE;
  DL_HIP_CHECK(launch_zero_i64(W->info2 + w, 1, s));
  DL_HIP_CHECK(run_plan(W, W->q[w].factor, s));
  W->q[w].assembled = false;
  W->q[w].factored = true;
  return DL_OK;
}

extern "C" dl_status bta_factor(dl_ws* W, dl_which which, double* logdet_dev,
                                int64_t* info_dev, void* stream) {
  if (!W || which < DL_QP || which > DL_BOTH) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int w0 = which == DL_QC ? 1 : 0;
  const int w1 = which == DL_QP ? 0 : 1;
  for (int w = w0; w <= w1; ++w)
    if (!W->q[w].assembled) return DL_ESTATE;
  for (int w = w0; w <= w1; ++w) {
    dl_status st = factor_one(W, w, s);
    if (st != DL_OK) return st;
  }
  const int cnt = w1 - w0 + 1;
  if (logdet_dev)
    DL_HIP_CHECK(hipMemcpyAsync(logdet_dev, W->logdet2 + w0, cnt * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
  if (info_dev)
    DL_HIP_CHECK(hipMemcpyAsync(info_dev, W->info2 + w0, cnt * sizeof(int64_t),
                                hipMemcpyDeviceToDevice, s));
  return DL_OK;
}

extern "C" dl_status bta_solve(dl_ws* W, double* rhs_inout_dev, void* stream) {
  if (!W) return DL_EINVAL;
  if (!W->q[1].factored) return DL_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  if (rhs_inout_dev) {
    DL_HIP_CHECK(launch_unpack(W->m, rhs_inout_dev, W->x, s));
  } else {
    DL_HIP_CHECK(launch_copy(W->rhs, W->x, W->m.Np, s));
  }
  DL_HIP_CHECK(run_plan(W, W->solve, s));
  if (rhs_inout_dev) DL_HIP_CHECK(launch_pack(W->m, W->mu, rhs_inout_dev, s));
  W->solved = true;
  return DL_OK;
}

extern "C" dl_status bta_selinv(dl_ws* W, double* diag_out_dev, void* stream) {
  if (!W || !diag_out_dev) return DL_EINVAL;
  if (!W->sel || !W->q[1].factored) return DL_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  DL_HIP_CHECK(run_plan(W, W->selinv, s));
  DL_HIP_CHECK(launch_pack(W->m, W->selout, diag_out_dev, s));
  return DL_OK;
}

extern "C" dl_status dl_ws_mean(dl_ws* W, double* out_dev, void* stream) {
  if (!W || !out_dev) return DL_EINVAL;
  if (!W->solved) return DL_ESTATE;
  DL_HIP_CHECK(launch_pack(W->m, W->mu, out_dev, (hipStream_t)stream));
  return DL_OK;
}

extern "C" dl_status fobj_eval(dl_ws* W, const double* theta_dev,
                               int32_t ntheta, double* fobj_dev,
                               dl_fobj_parts* parts_dev, int64_t* info_dev,
                               void* stream) {
  if (!W || !theta_dev || ntheta < 0 || (!fobj_dev && !parts_dev)) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int dim = W->m.dim_theta;
  for (int k = 0; k < ntheta; ++k) {
    dl_status st = bta_assemble(W, theta_dev + (int64_t)k * dim, DL_BOTH, stream);
    if (st != DL_OK) return st;
    for (int w = 0; w < 2; ++w)
      if ((st = factor_one(W, w, s)) != DL_OK) return st;
    if ((st = bta_solve(W, nullptr, stream)) != DL_OK) return st;
    DL_HIP_CHECK(launch_quadforms(W->m, W->coef, W->mu, W->qpart, W->quad2, s));
    DL_HIP_CHECK(launch_combine(W->m, W->coef, W->logdet2, W->info2, W->quad2,
                                fobj_dev ? fobj_dev + k : nullptr,
                                parts_dev ? parts_dev + k : nullptr,
                                info_dev ? info_dev + 2 * k : nullptr, s));
  }
  return DL_OK;
}

extern "C" dl_status dl_ws_get_block(dl_ws* W, dl_which which, int32_t kind,
                                     int32_t t, double* out_dev, void* stream) {
  if (!W || !out_dev || (which != DL_QP && which != DL_QC)) return DL_EINVAL;
  const ModelDev& m = W->m;
  MatrixStore& Q = W->q[which == DL_QP ? 0 : 1];
  hipStream_t s = (hipStream_t)stream;
  const int bp = m.bp;
  const std::vector<int>& slot = Q.factored ? Q.slot_final : Q.slot_init;
  if (kind == 4) {
    DL_HIP_CHECK(launch_pack(m, W->rhs, out_dev, s));
    return DL_OK;
  }
  if (kind == 3) {
    if (m.a == 0) return DL_EINVAL;
    DL_HIP_CHECK(launch_copy2d(Q.P, m.ap, out_dev, m.a, m.a, m.a, s));
    return DL_OK;
  }
  if (t < 0 || t >= m.nt || slot.empty()) return DL_EINVAL;
  const double* BRt = Q.BR + (int64_t)slot[t] * Q.ldbr * bp;
  if (kind == 0) {
    DL_HIP_CHECK(launch_copy2d(Q.D + (int64_t)t * bp * bp, bp, out_dev, m.b, m.b,
                               m.b, s));
  } else if (kind == 1) {
    if (t + 1 >= m.nt) return DL_EINVAL;
    DL_HIP_CHECK(launch_copy2d(BRt, Q.ldbr, out_dev, m.b, m.b, m.b, s));
  } else if (kind == 2) {
    if (Q.ap == 0 || m.a == 0) return DL_EINVAL;
    DL_HIP_CHECK(launch_copy2d(BRt + bp, Q.ldbr, out_dev, m.a, m.a, m.b, s));
  } else {
    return DL_EINVAL;
  }
  return DL_OK;
}

// ---- dense building blocks exposed for testing ----------------------------------------------

extern "C" dl_status dl_dgemm(int32_t transa, int32_t transb, int32_t lower,
                              int64_t M, int64_t Nn, int64_t K, double alpha,
                              const double* A, int64_t lda, const double* B,
                              int64_t ldb, double beta, double* C, int64_t ldc,
                              void* stream) {
  if (M < 0 || Nn < 0 || K < 0 || !C || (K > 0 && (!A || !B))) return DL_EINVAL;
  if (lower && M != Nn) return DL_EINVAL;
  if (M > INT32_MAX || Nn > INT32_MAX || K > INT32_MAX) return DL_EINVAL;
  if (ldc < M || (!transa && lda < M) || (transa && lda < K) ||
      (!transb && ldb < K) || (transb && ldb < Nn))
    return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int flags = (transa ? F_TA : 0) | (transb ? F_TB : 0) | (lower ? F_LOWER : 0);
  if (beta == 0.0) flags |= F_BETA0;
  GemmTask t = mk(A, lda, B, ldb, C, ldc, (int)M, (int)Nn, (int)K, flags, alpha,
                  beta);
  const int total = finalize_tasks(&t, 1);
  if (total == 0) return DL_OK;
  GemmTask* d = nullptr;
  DL_HIP_CHECK(hipMalloc(&d, sizeof(GemmTask)));
  hipError_t e = hipMemcpyAsync(d, &t, sizeof(GemmTask), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_gemm_tasks(d, 1, total, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  return e == hipSuccess ? DL_OK : DL_EHIP;
}

extern "C" dl_status dl_dpotrf(int64_t n, double* A, int64_t lda,
                               int32_t want_inverse, double* logdet_dev,
                               int64_t* info_dev, void* stream) {
  if (n <= 0 || n % 64 != 0 || !A || lda < n || !logdet_dev || !info_dev)
    return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::vector<void*> tmp;
  double *Gd = nullptr, *temp = nullptr, *logdiag = nullptr, *part = nullptr;
  dl_status st = DL_OK;
  if ((st = dev_alloc(tmp, sizeof(double) * n * 64, (void**)&Gd)) != DL_OK ||
      (st = dev_alloc(tmp, sizeof(double) * n * ((n / 64) / 2 + 1) * 64,
                      (void**)&temp)) != DL_OK ||
      (st = dev_alloc(tmp, sizeof(double) * n, (void**)&logdiag)) != DL_OK ||
      (st = dev_alloc(tmp, sizeof(double) * 256, (void**)&part)) != DL_OK) {
    free_all(tmp);
    return st;
  }
  std::vector<GemmTask> tasks;
  Plan plan;
  PlanBuilder pb{tasks, plan};
  add_potrf(pb, A, lda, (int)n, Gd, logdiag, info_dev, 0, (int)n);
  if (want_inverse) add_trtri(pb, A, lda, (int)n, Gd, temp);
  GemmTask* td = nullptr;
  if ((st = dev_alloc(tmp, sizeof(GemmTask) * (tasks.size() + 1), (void**)&td)) !=
      DL_OK) {
    free_all(tmp);
    return st;
  }
  hipError_t e = hipSuccess;
  if (!tasks.empty())
    e = hipMemcpyAsync(td, tasks.data(), sizeof(GemmTask) * tasks.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_zero_i64(info_dev, 1, s);
  if (e == hipSuccess) e = launch_zero_upper_tiles(A, lda, (int)n, s);
  for (const Op& op : plan.ops) {
    if (e != hipSuccess) break;
    switch (op.kind) {
      case OP_GEMM: e = launch_gemm_tasks(td + op.task_off, op.ntask, op.ntiles, s); break;
      case OP_POTRF_TILE: e = launch_potrf_tile(op.pt, s); break;
      case OP_COPY_TILES:
        e = launch_copy_tile64(op.src, op.lds, op.dst, op.ldd, (int)op.n,
                               op.sstride, op.dstride, s);
        break;
      default: break;
    }
  }
  if (e == hipSuccess) e = launch_sum_log(logdiag, n, 2.0, logdet_dev, part, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  free_all(tmp);
  return e == hipSuccess ? DL_OK : DL_EHIP;
}
