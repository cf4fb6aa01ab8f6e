// Batched evaluation engine: workspaces of one or more instances (an
// instance = one hyperparameter vector on one model), the launch plans of
// assembly, BTA factorisation, solve and selected inversion, and the C-ABI
// entry points.
//
// Every operation is first written as a sequence of per-matrix steps (one
// sequence per instance and matrix: Q_p and Q_c of every instance).  Steps
// carry a key that orders them within their sequence; steps of different
// sequences with the same key are independent and are merged into one
// launch.  This runs Q_p and Q_c of an evaluation concurrently (the paper's
// second layer of parallelism, here inside each launch) and the
// 2*dim(theta)+1 evaluations of a finite-difference gradient concurrently
// (its first layer), while each launch still walks the time steps in order.
// All descriptors are built once at workspace creation; running a plan only
// launches kernels.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <vector>

#include "engine.hpp"
#include "selinv.hpp"
#include "solve.hpp"
#include "dag.hpp"

namespace dl {

enum OpKind : int {
  OP_GEMM, OP_POTRF, OP_MISC, OP_GEMV_N, OP_GEMV_T, OP_SUM, OP_FINISH,
  OP_ASM_COLS, OP_ASM_TIPS, OP_THETA, OP_QUAD, OP_COMBINE, OP_GEMM32, OP_RES,
  OP_PANEL, OP_DAG, OP_NKIND
};

// One step of one sequence (before merging).
struct Step {
  uint64_t key = 0;
  OpKind kind = OP_MISC;
  int cat = DL_CAT_OTHER;
  double flops = 0.0, bytes = 0.0;
  std::vector<GemmTask> gemm;
  PotrfTileArgs potrf{};
  PanelTask panel{};
  DagBlock dagb{};
  MiscJob misc{};
  GemvN gn{};
  GemvT gt{};
  SumJob sum{};
  FinishJob fin{};
  AsmJob asmj{};
  ThetaJob th{};
  QuadJob quad{};
  CombineJob comb{};
  ResJob res{};
  int gx = 0, gy = 0, gz = 0;  // grid bounds contributed by this step
};

// A merged launch.
struct Launch {
  OpKind kind;
  int cat;
  double flops, bytes;
  int off, count;     // into the per-kind descriptor array
  int gx, gy, gz;     // grid bounds (max over merged steps)
  int tile;           // GEMM output tile (64 or 128)
  int nred;           // GEMM: reduction workgroups of a split launch
};

// Default GEMM tile for a launch (before any measured choice): 128x128 when
// every task is large and the launch still has >= 200 such tiles to spread
// over the 256 compute units, else 64x64.
static int default_tile(std::vector<GemmTask>& t, int off, int count) {
  bool big = true;
  for (int i = 0; i < count; ++i) {
    const GemmTask& g = t[off + i];
    if (g.M < 512 || g.N < 512 || g.K < 256) big = false;
  }
  if (!big) return 64;
  const int n128 = finalize_tasks(t.data() + off, count, 128);
  return n128 >= 200 ? 128 : 64;
}

struct Plan {
  std::vector<int> idx;  // indices into the workspace's launch table
};

// Host-side descriptor arrays (uploaded once per workspace).
struct Descs {
  std::vector<GemmTask> gemm;
  std::vector<PotrfTileArgs> potrf;
  std::vector<PanelTask> panel;
  std::vector<DagBlock> dagb;   // blocks of the persistent factorisation launches
  std::vector<uint64_t> dagt;   // their task words (one list per launch)
  int dag_launches = 0;
  std::vector<MiscJob> misc;
  std::vector<GemvN> gn;
  std::vector<GemvT> gt;
  std::vector<SumJob> sum;
  std::vector<FinishJob> fin;
  std::vector<AsmJob> asmj;
  std::vector<ThetaJob> th;
  std::vector<QuadJob> quad;
  std::vector<CombineJob> comb;
  std::vector<ResJob> res;
};

struct DevDescs {
  GemmTask* gemm = nullptr;
  PotrfTileArgs* potrf = nullptr;
  PanelTask* panel = nullptr;
  DagBlock* dagb = nullptr;
  uint64_t* dagt = nullptr;
  MiscJob* misc = nullptr;
  GemvN* gn = nullptr;
  GemvT* gt = nullptr;
  SumJob* sum = nullptr;
  FinishJob* fin = nullptr;
  AsmJob* asmj = nullptr;
  ThetaJob* th = nullptr;
  QuadJob* quad = nullptr;
  CombineJob* comb = nullptr;
  ResJob* res = nullptr;
};

// key = (((major * 16 + group) * 256 + j) * 4 + sub)
static uint64_t K(uint64_t major, uint64_t group, uint64_t j = 0, uint64_t sub = 0) {
  return ((major * 16 + group) * 256 + j) * 4 + sub;
}

// Merge sequences: steps with equal keys and kinds form one launch; keys are
// visited in increasing order, so each sequence keeps its own order.
static void merge(const std::vector<std::vector<Step>>& seqs, Descs& D,
                  std::vector<Launch>& table, Plan& P) {
  std::map<std::pair<uint64_t, int>, std::vector<const Step*>> groups;
  for (const auto& sq : seqs)
    for (const Step& st : sq) groups[{st.key, (int)st.kind}].push_back(&st);
  for (auto& kv : groups) {
    const std::vector<const Step*>& g = kv.second;
    Launch L{};
    L.tile = 64;
    L.kind = (OpKind)kv.first.second;
    L.cat = g.front()->cat;
    L.flops = L.bytes = 0.0;
    L.gx = L.gy = L.gz = 0;
    for (const Step* st : g) {
      L.flops += st->flops;
      L.bytes += st->bytes;
      L.gx = std::max(L.gx, st->gx);
      L.gy = std::max(L.gy, st->gy);
      L.gz = std::max(L.gz, st->gz);
    }
    switch (L.kind) {
      case OP_GEMM:
      case OP_GEMM32: {
        L.off = (int)D.gemm.size();
        for (const Step* st : g) D.gemm.insert(D.gemm.end(), st->gemm.begin(), st->gemm.end());
        L.count = (int)D.gemm.size() - L.off;
        if (L.kind == OP_GEMM32)  // the FP32 kernel does not split k
          for (int i = L.off; i < L.off + L.count; ++i) D.gemm[i].flags &= ~F_SPLIT;
        L.tile = default_tile(D.gemm, L.off, L.count);
        L.gx = finalize_tasks(D.gemm.data() + L.off, L.count, L.tile, &L.nred);
        if (L.gx == 0) continue;
        break;
      }
#define PUSH(vec, fld)                                  \
  L.off = (int)D.vec.size();                            \
  for (const Step* st : g) D.vec.push_back(st->fld);    \
  L.count = (int)D.vec.size() - L.off;                  \
  break;
      case OP_POTRF: PUSH(potrf, potrf)
      case OP_PANEL: {
        L.off = (int)D.panel.size();
        for (const Step* st : g) D.panel.push_back(st->panel);
        L.count = (int)D.panel.size() - L.off;
        L.gx = finalize_panels(D.panel.data() + L.off, L.count);
        break;
      }
      case OP_DAG: {
        // one persistent launch over the blocks of the merged steps: their
        // tasks in one list (dag.hpp)
        L.off = (int)D.dagb.size();
        std::vector<int> nbks;
        for (const Step* st : g) {
          D.dagb.push_back(st->dagb);
          nbks.push_back(st->dagb.nbk);
        }
        L.count = (int)D.dagb.size() - L.off;
        const std::vector<uint64_t> tl = dag::launch_list(nbks, true);
        L.gy = (int)D.dagt.size();
        D.dagt.insert(D.dagt.end(), tl.begin(), tl.end());
        L.gx = (int)tl.size();
        L.gz = D.dag_launches++;
        break;
      }
      case OP_MISC: PUSH(misc, misc)
      case OP_GEMV_N: PUSH(gn, gn)
      case OP_GEMV_T: PUSH(gt, gt)
      case OP_SUM: PUSH(sum, sum)
      case OP_FINISH: PUSH(fin, fin)
      case OP_ASM_COLS: PUSH(asmj, asmj)
      case OP_ASM_TIPS: PUSH(asmj, asmj)
      case OP_THETA: PUSH(th, th)
      case OP_QUAD: PUSH(quad, quad)
      case OP_COMBINE: PUSH(comb, comb)
      case OP_RES: PUSH(res, res)
#undef PUSH
      default: continue;
    }
    P.idx.push_back((int)table.size());
    table.push_back(L);
  }
}

static GemmTask mk(const double* A, int64_t lda, const double* B, int64_t ldb,
                   double* C, int64_t ldc, int M, int N, int K_, int flags,
                   double alpha, double beta) {
  GemmTask t{};
  t.A = A; t.B = B; t.C = C;
  t.lda = lda; t.ldb = ldb; t.ldc = ldc;
  t.M = M; t.N = N; t.K = K_; t.flags = flags;
  t.alpha = alpha; t.beta = beta;
  return t;
}

// Pointer `elems` elements past `base` for storage of elem_bytes per element
// (FP32 blocks of mixed-precision workspaces travel in double* fields).
static double* eoff(void* base, int64_t elems, int elem_bytes) {
  return (double*)((char*)base + elems * elem_bytes);
}

static Step gemm32_step(uint64_t key, int cat, double flops, std::vector<GemmTask> ts) {
  Step s;
  s.key = key;
  s.kind = OP_GEMM32;
  s.cat = cat;
  s.flops = flops;
  s.gemm = std::move(ts);
  return s;
}

static Step gemm_step(uint64_t key, int cat, double flops, std::vector<GemmTask> ts) {
  Step s;
  s.key = key;
  s.kind = OP_GEMM;
  s.cat = cat;
  s.flops = flops;
  s.gemm = std::move(ts);
  return s;
}

static Step misc_step(uint64_t key, int cat, int kind, double* dst,
                      const double* src, int64_t n, double v = 0.0) {
  Step s;
  s.key = key;
  s.kind = OP_MISC;
  s.cat = cat;
  s.misc.kind = kind;
  s.misc.dst = dst;
  s.misc.src = src;
  s.misc.n = n;
  s.misc.v = v;
  return s;
}

// Blocked right-looking Cholesky of the n x n block A (n multiple of 64),
// panels of 64 columns.  With `fold`, the inverse G = L^{-1} is formed
// alongside and on return the block holds G (lower triangle); otherwise the
// block holds L with its diagonal tiles inverted (seq_trtri completes G).  Tile 0 is factored alone (its
// inverse in place) and its panel solved in place, L(., 0) = P_0 G_00^T;
// step j then updates the trailing tiles with L(., j), factors tile j+1,
// solves panel j+1 and advances the inverse by one row of tiles (see
// PanelTask); a closing launch forms the inverse's last row and one tile
// copy puts its G(nbk-1, nbk-2) in place.  `tmp` holds the two-tile side
// ring and the inverse's accumulators (2 + nbk (nbk - 1) / 2 tiles).
// `breal`: unpadded size (operation count); `count_inv`: count the
// inverse's b^3/3 (else it is extra work of the inverse-based solves).
// Keys (major, group 1, j, sub): (0, 0) tile 0, (0, 1) the solve of panel 0,
// (j, 2) step j and the closing launch (j = nbk - 1), (nbk - 1, 3) the copy.
static void seq_potrf(std::vector<Step>& q, uint64_t major, double* A, int64_t ld,
                      int n, double* logdiag, int64_t* info, int64_t row0,
                      int breal, double* tmp, bool count_inv, bool fold,
                      double* lbuf = nullptr, int32_t* dctr = nullptr) {
  const int nbk = n / 64;
  if (lbuf) {
    // the whole factorisation and inverse in one persistent launch (shared
    // with the other blocks of the same key)
    Step s;
    s.key = K(major, 1, 0, 2);
    s.kind = OP_DAG;
    s.cat = DL_CAT_PANEL_SYRK;
    const double b3 = (double)breal * breal * breal / 3.0;
    s.flops = b3 + (count_inv ? b3 : 0.0);
    DagBlock& d = s.dagb;
    d.A = A;
    d.ld = ld;
    d.L = lbuf;
    d.stage = tmp;
    d.logdiag = logdiag;
    d.info = info;
    d.row0 = row0;
    d.ctr = dctr;
    d.nbk = nbk;
    q.push_back(s);
    return;
  }
  auto width = [&](int j) { return (double)std::max(0, std::min(64, breal - j * 64)); };
  auto below = [&](int j) { return (double)std::max(0, breal - (j + 1) * 64); };
  double* gside = tmp;
  double* stage = tmp + 2 * 4096;
  {
    const double w = width(0);
    Step s;
    s.key = K(major, 1, 0, 0);
    s.kind = OP_POTRF;
    s.cat = DL_CAT_POTRF_TILE;
    s.flops = w * w * w / 3.0;
    s.potrf.A = A;
    s.potrf.lda = ld;
    s.potrf.logdiag = logdiag;
    s.potrf.info = info;
    s.potrf.row0 = row0;
    s.potrf.mode = 1;
    q.push_back(s);
  }
  if (nbk == 1) return;
  {
    double* panel = A + 64;
    q.push_back(gemm_step(K(major, 1, 0, 1), DL_CAT_PANEL_TRSM, below(0) * width(0) * width(0),
                          {mk(panel, ld, A, ld, panel, ld, n - 64, 64, 64, F_TB | F_BETA0,
                              1.0, 0.0)}));
  }
  for (int j = 0; j < (fold ? nbk : nbk - 1); ++j) {
    const bool last = (j + 1 == nbk);
    Step s;
    s.key = K(major, 1, j, 2);
    s.kind = OP_PANEL;
    s.cat = DL_CAT_PANEL_SYRK;
    if (!last) {
      // the trailing update of a right-looking Cholesky, the tile factor and
      // the solve of the next panel
      const double w = width(j), w1 = width(j + 1), bl = below(j);
      s.flops = bl * bl * w + w1 * w1 * w1 / 3.0 + below(j + 1) * w1 * w1;
    } else if (count_inv) {
      s.flops = (double)breal * breal * breal / 3.0;  // the whole inverse
    }
    PanelTask& t = s.panel;
    t.A = A;
    t.ld = ld;
    t.logdiag = logdiag + (int64_t)(j + 1) * 64;
    t.info = info;
    t.row0 = row0 + (int64_t)(j + 1) * 64;
    t.gside = gside;
    t.stage = stage;
    t.j = j;
    t.nbk = nbk;
    t.last = last ? 1 : 0;
    t.inv = fold ? 1 : 0;
    q.push_back(s);
  }
  if (!fold) return;
  // G(nbk-1, nbk-2) from the accumulators into place
  Step cp = misc_step(K(major, 1, nbk - 1, 3), DL_CAT_PANEL_SYRK, MJ_COPY2D,
                      A + (int64_t)(nbk - 1) * 64 + (int64_t)(nbk - 2) * 64 * ld,
                      stage + (int64_t)((nbk - 1) * (nbk - 2) / 2 + (nbk - 2)) * 4096, 0);
  cp.misc.rows = 64;
  cp.misc.cols = 64;
  cp.misc.lds = 64;
  cp.misc.ldd = ld;
  q.push_back(cp);
}

// In-place inverse of the lower-triangular factor whose diagonal tiles
// already hold their inverses: recursive halving, G21 = -G22 (L21 G11), all
// nodes of one depth merged, deepest first.  temp: n x (n/2 + 64) (ld n).
// `breal`: unpadded size for the operation count (0: not counted).
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

static void seq_trtri(std::vector<Step>& q, uint64_t major, double* A, int64_t ld,
                      int n, double* temp, int breal, int xf) {
  const int nbk = n / 64;
  auto ext = [&](int lo, int hi) {
    return (double)std::max(0, std::min(hi * 64, breal) - lo * 64);
  };
  std::vector<std::vector<int>> lv;
  collect_nodes(0, nbk, 0, lv);
  const int D = (int)lv.size();
  for (int d = D - 1; d >= 0; --d) {
    std::vector<GemmTask> tT, tG;
    double fT = 0.0, fG = 0.0;
    for (size_t k = 0; k < lv[d].size(); k += 2) {
      const int lo = lv[d][k], hi = lv[d][k + 1];
      const int mid = lo + (hi - lo) / 2;
      const int n1 = (mid - lo) * 64, n2 = (hi - mid) * 64;
      double* L21 = A + (int64_t)mid * 64 + (int64_t)lo * 64 * ld;
      double* G11 = A + (int64_t)lo * 64 * (ld + 1);
      double* G22 = A + (int64_t)mid * 64 * (ld + 1);
      double* T = temp + (int64_t)lo * 64;
      tT.push_back(mk(L21, ld, G11, ld, T, n, n2, n1, n1, F_KLO_COL | F_BETA0 | xf, 1.0, 0.0));
      tG.push_back(mk(G22, ld, T, n, L21, ld, n2, n1, n2, F_KHI_ROW | F_BETA0 | xf, -1.0, 0.0));
      const double r1 = ext(lo, mid), r2 = ext(mid, hi);
      fT += r2 * r1 * r1;
      fG += r1 * r2 * r2;
    }
    const int lvl = 15 - d;  // deeper levels first
    q.push_back(gemm_step(K(major, 2, lvl, 0), DL_CAT_TRTRI, fT, tT));
    q.push_back(gemm_step(K(major, 2, lvl, 1), DL_CAT_TRTRI, fG, tG));
  }
}

}  // namespace dl

using namespace dl;

// ---- workspace -----------------------------------------------------------------------

struct Inst {
  const dl_model* model = nullptr;
  ModelDev m{};
  int dim = 0;
  // Q_p: full storage (keep_qp) or a ring of 2 diagonal and 3 sub-diagonal
  // blocks assembled just in time (only log|Q_p| is needed)
  double *Dp = nullptr, *Bp = nullptr, *Pp = nullptr;
  bool qp_ring = true;
  // Q_c: full storage, [B_t; R_t] in nt+1 slots of (bp+ap) x bp (nt+2 when
  // two-sided: one spare slot per elimination chain)
  double *Dc = nullptr, *BRc = nullptr, *Pc = nullptr, *GPc = nullptr;
  int64_t ldbr = 0;
  std::vector<int> slot_final;
  // Elimination order.  One-sided: blocks 0..nt-2 forward, then the root
  // block nt-1.  Two-sided: chain A = 0..mid-1 forward and chain B =
  // nt-1..mid+1 backward run concurrently (their steps share launches),
  // each block eliminated into its neighbour toward the root block mid,
  // which is factored last.  Chain B accumulates its tip updates (and the
  // tip part of the forward solve) in buffers of its own.
  bool two = false;
  int mid = 0;
  double *PcB = nullptr, *ttempB[2] = {nullptr, nullptr};
  // persistent diagonal-block factorisation (DL_WS_DAG): the L tiles and the
  // readiness counters of the block each chain factors, per matrix
  double *lbuf[2] = {nullptr, nullptr}, *lbufB[2] = {nullptr, nullptr};
  int32_t *dctr[2] = {nullptr, nullptr}, *dctrB[2] = {nullptr, nullptr};
  double *uB = nullptr, *gpartB = nullptr, *xPB = nullptr;
  double *YB = nullptr, *XCB[2] = {nullptr, nullptr};
  double *theta = nullptr, *coef = nullptr, *logdiag[2] = {nullptr, nullptr};
  double *logdet2 = nullptr, *quad2 = nullptr, *sumpart = nullptr, *qpart = nullptr;
  int64_t* info2 = nullptr;
  double *rhs = nullptr, *x = nullptr, *mu = nullptr, *u = nullptr, *gpart = nullptr;
  double* ttemp[2] = {nullptr, nullptr};
  double *f = nullptr, *parts = nullptr;
  int64_t* info_out = nullptr;
  // selected inversion
  double *WV = nullptr, *Y = nullptr, *XC[2] = {nullptr, nullptr}, *selout = nullptr;
  double* GPp = nullptr;
  bool mixed = false;       // [B_t; R_t] in FP32, their products on FP32 MFMA
  int eb = 8;               // bytes per element of the [B_t; R_t] storage
  double *mu_acc = nullptr, *av = nullptr, *rpart = nullptr, *rnorm = nullptr;
  // inner Newton iteration (Poisson likelihood): per-observation weights and
  // right-hand-side values, the accepted iterate, the Newton target, the
  // trial maxima's partials, and views of the workspace's alpha / out4
  bool poisson = false;
  double *obs_d = nullptr, *obs_z = nullptr, *xcur = nullptr, *xN = nullptr;
  double *tpart = nullptr, *alpha = nullptr, *out4 = nullptr;
};

struct dl_ws {
  std::vector<Inst> inst;
  std::vector<void*> allocs;
  size_t bytes = 0;
  int flags = 0;
  bool sel = false, keep_qp = false, mixed = false;
  bool splitk = false;
  bool fold_inv = false;  // inverses inside the panel launches (DL_WS_FOLD_INV)
  bool dag = false;       // one persistent launch per diagonal block (DL_WS_DAG)
  int32_t* dag_heads = nullptr;  // [4 x launches] task head, finished workgroups, abort
  int dag_workers = 0;           // grid of the persistent launches
  double* partials = nullptr;  // split-k partial tiles (shared by all launches)
  int64_t partials_cap = 0;    // doubles allocated at `partials`
  int dim_total = 0;
  double* theta_all = nullptr;   // packed theta of all instances
  double* f_all = nullptr;       // [B]
  double* parts_all = nullptr;   // [B x 8]
  int64_t* info_all = nullptr;   // [B x 2]
  // inner Newton iteration (all instances Poisson, or none)
  bool poisson = false;
  double* alpha_all = nullptr;   // [B] step lengths of the current trial
  double* out4_all = nullptr;    // [B x 4] trial results read by the host
  LapJob* d_lap = nullptr;
  TrialJob* d_trial = nullptr;
  QuadJob* d_nquad = nullptr;
  std::vector<int32_t> newton_steps;
  bool warm = false;             // DL_WS_WARM_START
  std::vector<char> has_mode;    // instance holds a converged mode in xcur
  // refinement of the mean: residual norms of every instance ([B x 2]:
  // |rhs - Q_c x|^2, |rhs|^2), the squared relative tolerance in use (one
  // device double and its host copy) and a host buffer for the norms
  double* rnorm_all = nullptr;
  double* tol2_dev = nullptr;
  double tol2_host = 0.0;
  std::vector<double> rnorm_host;
  MiscJob* d_io = nullptr;  // one descriptor for dl_ws_get_block / set_block
  Descs H;
  DevDescs Dd;
  std::vector<Launch> table;
  // refinement plans: init (x <- mu), res (residual of x and its norms), corr
  // (solve with the factor, x += correction unless converged), fin (mu <- x
  // and the final residual), resid (the final residual of mu alone)
  Plan theta_p, asm_p[3], fac_p[3], solve_p, selinv_p, post_p, eval_p;
  Plan ref_init_p, ref_res_p, ref_corr_p, ref_fin_p, resid_p;
  bool assembled[2] = {false, false}, factored[2] = {false, false};
  bool solved = false;
  int max_shmem = 0;
  // graph of the whole evaluation plan
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  // second stream and fork/join events of fobj_selinv_eval
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool use_graph = false;
  // launch profiling (measurement only)
  int prof_mask = 0, prof_by_kernel = 0, prof_used = 0, prof_paused = 0;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_cat;
  std::vector<double> prof_flops, prof_bytes;
};

// Grow the split-k partial-tile buffer to at least `elems` doubles (work on
// `s` that may still read the old buffer is waited for first).
static dl_status ensure_partials(dl_ws* W, int64_t elems, hipStream_t s) {
  if (elems <= W->partials_cap) return DL_OK;
  if (W->partials) {
    DL_HIP_CHECK(hipStreamSynchronize(s));
    DL_HIP_CHECK(hipFree(W->partials));
    W->bytes -= sizeof(double) * (size_t)W->partials_cap;
    W->partials = nullptr;
    W->partials_cap = 0;
  }
  if (hipMalloc((void**)&W->partials, sizeof(double) * (size_t)elems) != hipSuccess) {
    W->partials = nullptr;
    return DL_ENOMEM;
  }
  W->partials_cap = elems;
  W->bytes += sizeof(double) * (size_t)elems;
  return DL_OK;
}

static int prof_begin(dl_ws* W, int cat, int kind, hipStream_t s) {
  if (!W->prof_mask || W->prof_paused || !((W->prof_mask >> cat) & 1)) return -1;
  if (W->prof_used >= (int)W->prof_cat.size()) return -1;
  const int k = W->prof_used++;
  if (hipEventRecord(W->prof_ev[2 * k], s) != hipSuccess) return -1;
  W->prof_cat[k] = W->prof_by_kernel ? kind : cat;
  return k;
}

static void prof_end(dl_ws* W, int k, double flops, double bytes, hipStream_t s) {
  if (k < 0) return;
  (void)hipEventRecord(W->prof_ev[2 * k + 1], s);
  W->prof_flops[k] = flops;
  W->prof_bytes[k] = bytes;
}

static hipError_t run_launch(dl_ws* W, const Launch& L, hipStream_t s);

static hipError_t run(dl_ws* W, const Plan& P, hipStream_t s) {
  for (int i : P.idx) {
    hipError_t e = run_launch(W, W->table[i], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t run_launch(dl_ws* W, const Launch& L, hipStream_t s) {
  const DevDescs& d = W->Dd;
  {
    int kk = DL_KERNEL_OTHER;
    if (L.kind == OP_GEMM || L.kind == OP_GEMM32) kk = DL_KERNEL_GEMM;
    else if (L.kind == OP_POTRF) kk = DL_KERNEL_POTRF_TILE;
    else if (L.kind == OP_PANEL) kk = DL_KERNEL_PANEL;
    else if (L.kind == OP_DAG) kk = DL_KERNEL_DAG;
    else if (L.kind == OP_GEMV_N || L.kind == OP_GEMV_T) kk = DL_KERNEL_GEMV;
    else if (L.kind == OP_ASM_COLS) kk = DL_KERNEL_ASSEMBLE;
    const int pk = prof_begin(W, L.cat, kk, s);
    hipError_t e = hipSuccess;
    switch (L.kind) {
      case OP_GEMM:
        e = launch_gemm_tasks(d.gemm + L.off, L.count, L.gx, s, L.tile, W->partials);
        if (e == hipSuccess && L.nred > 0) {
          // the reduction of a split launch: its own record (kernel-level
          // profiles then see the product kernel alone)
          prof_end(W, pk, L.flops, L.bytes, s);
          const int pr = prof_begin(W, L.cat, DL_KERNEL_GEMM_REDUCE, s);
          e = launch_gemm_reduce(d.gemm + L.off, L.count, L.nred, W->partials, s, L.tile);
          prof_end(W, pr, 0.0, 0.0, s);
          return e;
        }
        break;
      case OP_GEMM32:
        e = launch_gemm32_tasks(d.gemm + L.off, L.count, L.gx, s, L.tile);
        break;
      case OP_RES: e = launch_residual(d.res + L.off, L.count, s); break;
      case OP_POTRF: e = launch_potrf_tiles(d.potrf + L.off, L.count, s); break;
      case OP_PANEL: e = launch_panel_updates(d.panel + L.off, L.count, L.gx, s); break;
      case OP_DAG:
        e = launch_dag_chol(d.dagt + L.gy, L.gx, d.dagb + L.off, L.count,
                            W->dag_heads + 4 * (int64_t)L.gz,
                            std::min(L.gx, W->dag_workers), s);
        break;
      case OP_MISC: e = launch_misc(d.misc + L.off, L.count, s); break;
      case OP_GEMV_N: e = launch_gemv_n(d.gn + L.off, L.count, L.gx, s); break;
      case OP_GEMV_T: e = launch_gemv_t(d.gt + L.off, L.count, L.gx, s); break;
      case OP_SUM: e = launch_sums(d.sum + L.off, L.count, s); break;
      case OP_FINISH: e = launch_selinv_finish(d.fin + L.off, L.count, L.gx, s); break;
      case OP_ASM_COLS:
        e = launch_assemble_cols(d.asmj + L.off, L.count, L.gx, L.gy, W->max_shmem, s);
        break;
      case OP_ASM_TIPS: e = launch_assemble_tips(d.asmj + L.off, L.count, L.gx, s); break;
      case OP_THETA: e = launch_theta_coeffs(d.th + L.off, L.count, s); break;
      case OP_QUAD: e = launch_quadforms(d.quad + L.off, L.count, s); break;
      case OP_COMBINE: e = launch_combine(d.comb + L.off, L.count, s); break;
      default: break;
    }
    prof_end(W, pk, L.flops, L.bytes, s);
    return e;
  }
}

// ---- plan construction -----------------------------------------------------------------

static double asm_bytes(const ModelDev& m, bool p, bool c, int nsteps) {
  const double b = m.b, a = m.a;
  const double per = 2.0 * b * b;  // a diagonal and a sub-diagonal block
  double by = 0.0;
  if (p) by += per * nsteps;
  if (c) by += per * nsteps + a * b * nsteps;
  return 8.0 * by;
}

// theta -> coefficients, tips and fixed-effect right-hand side, and the dense
// blocks of Q_c (and Q_p when it is stored in full).
static void seq_assemble(dl_ws* W, Inst& I, bool p, bool c, std::vector<Step>& q) {
  const ModelDev& m = I.m;
  Step th;
  th.key = K(0, 0, 0, 0);
  th.kind = OP_THETA;
  th.cat = DL_CAT_ASSEMBLE;
  th.th.m = I.model->dev;
  th.th.theta = I.theta;
  th.th.coef = I.coef;
  q.push_back(th);
  Step tip;
  tip.key = K(0, 1, 0, 0);
  tip.kind = OP_ASM_TIPS;
  tip.cat = DL_CAT_ASSEMBLE;
  tip.asmj.m = I.model->dev;
  tip.asmj.coef = I.coef;
  tip.asmj.o.Pp = p ? I.Pp : nullptr;
  tip.asmj.o.Pc = c ? I.Pc : nullptr;
  tip.asmj.o.rhs = I.rhs;
  if (c && I.poisson) {
    tip.asmj.o.obs_d = I.obs_d;
    tip.asmj.o.obs_z = I.obs_z;
  }
  tip.gx = 1 + m.nv * m.nr * m.nr + m.nv * m.nr;
  q.push_back(tip);
  const bool full_p = p && !I.qp_ring;
  if (c || full_p) {
    Step s;
    s.key = K(0, 2, 0, 0);
    s.kind = OP_ASM_COLS;
    s.cat = DL_CAT_ASSEMBLE;
    s.bytes = asm_bytes(m, full_p, c, m.nt);
    AsmJob& J = s.asmj;
    J.m = I.model->dev;
    J.coef = I.coef;
    J.t0 = 0;
    J.nt = m.nt;
    const int64_t bb = (int64_t)m.bp * m.bp;
    if (full_p) {
      J.o.Dp = I.Dp; J.o.dp_stride = bb;
      J.o.Bp = I.Bp; J.o.bp_stride = bb;
    }
    if (c) {
      J.o.Dc = I.Dc; J.o.dc_stride = bb;
      J.o.BRc = I.BRc; J.o.brc_stride = I.ldbr * m.bp;
    }
    J.o.rhs = I.rhs;
    J.o.b32 = I.mixed ? 1 : 0;
    if (c && I.poisson) {
      J.o.obs_d = I.obs_d;
      J.o.obs_z = I.obs_z;
    }
    s.gx = m.bp;
    s.gy = m.nt;
    q.push_back(s);
  }
}

// BTA Cholesky of Q_p (w = 0) or Q_c (w = 1) of instance I in its
// elimination order.  Every block t other than the root is eliminated into
// its successor (t+1 in chain A, t-1 in chain B): factor D_t, scale its
// coupling block and arrow block by L_tt^-T, and subtract the Schur
// complement from D_succ, R_succ and the tip.  The coupling of a chain-B
// block t is Q(t-1, t) = B_{t-1}^T = B_{t-1}: the sub-diagonal blocks of
// these models are symmetric (each is a weighted sum of symmetric FEM
// matrices, the weights symmetric in the response pair), so chain B reads
// the assembled B_{t-1} as it is.  Keys: major = position of the block in
// its chain + 1 (0 is the prologue), the root one major after the longer
// chain, 1 + nt_max for the tip.  The two chains' updates of the root block
// fall in different launches because the chains differ in length.
static void seq_factor(dl_ws* W, Inst& I, int w, int nt_max, std::vector<Step>& q) {
  const ModelDev& m = I.m;
  const int bp = m.bp;
  const int n = m.nt;
  const int64_t bb = (int64_t)bp * bp;
  const bool ring = (w == 0) && I.qp_ring;
  const int64_t ldbr = (w == 0) ? bp : I.ldbr;
  const int apr = (w == 0) ? 0 : m.ap;
  double* P = (w == 0) ? I.Pp : I.Pc;
  double* logdiag = I.logdiag[w];
  int64_t* info = I.info2 + w;
  const bool two = I.two;
  const int mid = I.mid;
  const int lenA = mid, lenB = n - 1 - mid;
  const uint64_t root_major = (uint64_t)std::max(lenA, lenB) + 1;
  q.push_back(misc_step(K(0, 0), DL_CAT_OTHER, MJ_ZERO_I64, (double*)info, nullptr, 1));
  if (two && apr)
    q.push_back(misc_step(K(0, 0), DL_CAT_OTHER, MJ_FILL, I.PcB, nullptr,
                          (int64_t)m.ap * m.ap, 0.0));
  const int eb = I.eb;
  double* Dbase = (w == 0) ? I.Dp : I.Dc;
  double* Bbase = (w == 0) ? I.Bp : I.BRc;
  auto BRs = [&](int sl) { return eoff(Bbase, (int64_t)sl * ldbr * bp, eb); };
  auto BRo = [&](int sl, int rows) { return eoff(Bbase, (int64_t)sl * ldbr * bp + rows, eb); };
  // full storage: slot of [B_t; R_t] per block, one spare slot per chain
  std::vector<int> slot(n + 2);
  for (int t = 0; t < n + 2; ++t) slot[t] = t;
  int spare[2] = {n, n + 1};
  // Q_p ring: diagonal slots 0,1 (chain A; the root too when one-sided),
  // 2,3 (chain B), 4 (root, two-sided); coupling slots 0,1 assembled + 2
  // scaled (chain A), 3,4 assembled + 5 scaled (chain B), 6 (the root's
  // B_mid, read by chain B's last block)
  auto Dt = [&](int t) -> double* {
    if (!ring) return Dbase + (int64_t)t * bb;
    if (!two || t < mid) return Dbase + (int64_t)(t % 2) * bb;
    if (t == mid) return Dbase + 4 * bb;
    return Dbase + (int64_t)(2 + t % 2) * bb;
  };
  auto asm_qp = [&](int t, double* D, double* B, uint64_t key) {
    Step s;
    s.key = key;
    s.kind = OP_ASM_COLS;
    s.cat = DL_CAT_ASSEMBLE;
    s.bytes = asm_bytes(m, true, false, 1);
    s.asmj.m = I.model->dev;
    s.asmj.coef = I.coef;
    s.asmj.t0 = t;
    s.asmj.nt = 1;
    s.asmj.o.Dp = D;
    s.asmj.o.Bp = B;
    s.asmj.o.rhs = I.rhs;
    s.asmj.o.b32 = I.mixed ? 1 : 0;
    s.gx = bp;
    s.gy = 1;
    q.push_back(s);
  };
  if (ring) {
    asm_qp(0, Dt(0), BRs(0), K(0, 3));
    if (two) {
      asm_qp(n - 1, Dt(n - 1), BRs(3 + (n - 1) % 2), K(0, 3));
      asm_qp(mid, Dt(mid), BRs(6), K(0, 3));
    }
  }
  const bool count_inv = (w == 1) && W->sel;
  // split k of the FP64 products (FP32 launches drop the flag)
  const int xf = W->splitk ? F_SPLIT : 0;
  const int x64 = I.mixed ? F_B64 : 0;
  const int c64 = I.mixed ? F_C64 : 0;
  auto gs = [&](uint64_t key, int cat, double fl, std::vector<GemmTask> ts) {
    return I.mixed ? gemm32_step(key, cat, fl, std::move(ts))
                   : gemm_step(key, cat, fl, std::move(ts));
  };
  // chain 0: A, 1: B, 2: root
  auto eliminate = [&](int t, uint64_t major, int chain) {
    const bool root = chain == 2;
    const int succ = chain == 0 ? t + 1 : t - 1;
    if (ring) {
      if (chain == 0 && t + 1 < (two ? mid : n))
        asm_qp(t + 1, Dt(t + 1), BRs((t + 1) % 2), K(major, 0));
      if (chain == 1 && t - 1 > mid)
        asm_qp(t - 1, Dt(t - 1), BRs(3 + (t - 1) % 2), K(major, 0));
    }
    // factor and inverse of the diagonal block
    double* tmp = chain == 1 ? I.ttempB[w] : I.ttemp[w];
    double* lb = W->dag ? (chain == 1 ? I.lbufB[w] : I.lbuf[w]) : nullptr;
    int32_t* dc = W->dag ? (chain == 1 ? I.dctrB[w] : I.dctr[w]) : nullptr;
    seq_potrf(q, major, Dt(t), bp, bp, logdiag + (int64_t)t * bp, info,
              (int64_t)t * m.b, m.b, tmp, count_inv, W->fold_inv, lb, dc);
    if (!W->fold_inv && !W->dag) seq_trtri(q, major, Dt(t), bp, bp, tmp, count_inv ? m.b : 0, xf);
    const int M = (root ? 0 : bp) + apr;
    if (M <= 0) return;
    const double b = m.b, ar = apr ? m.a : 0;
    const double mreal = (root ? 0.0 : b) + ar;
    const int ci = chain == 1 ? 1 : 0;
    const int nw = ring ? (ci ? 5 : 2) : spare[ci];
    // [C_t; R_t] <- [C_t; R_t] L_tt^{-T} = [C_t; R_t] G_t^T, C_t the coupling
    const int fl = F_TB | F_KHI_COL | F_BETA0 | x64 | xf;
    std::vector<GemmTask> tr;
    if (chain == 1) {
      const double* C = ring ? BRs(t - 1 == mid ? 6 : 3 + (t - 1) % 2) : BRs(slot[t - 1]);
      tr.push_back(mk(C, ldbr, Dt(t), bp, BRs(nw), ldbr, bp, bp, bp, fl, 1.0, 0.0));
      if (apr)
        tr.push_back(mk(BRo(slot[t], bp), ldbr, Dt(t), bp, BRo(nw, bp), ldbr, apr, bp, bp,
                        fl, 1.0, 0.0));
    } else {
      const int rows_lo = root ? bp : 0;
      const int src = ring ? (t % 2) : slot[t];
      tr.push_back(mk(BRo(src, rows_lo), ldbr, Dt(t), bp, BRo(nw, rows_lo), ldbr, M, bp,
                      bp, fl, 1.0, 0.0));
    }
    q.push_back(gs(K(major, 3), DL_CAT_TRSM, mreal * b * b, std::move(tr)));
    if (!ring) {
      // the block's old slot is free: its coupling rows were read by this
      // step (chain A, root) or by the previous step of chain B, its arrow
      // rows by this step
      const int old = slot[t];
      slot[t] = nw;
      spare[ci] = old;
    }
    double* BRt = BRs(nw);
    double* RRt = BRo(nw, bp);
    double* Ptip = (chain == 1) ? I.PcB : P;
    std::vector<GemmTask> up;
    if (!root) {
      up.push_back(mk(BRt, ldbr, BRt, ldbr, Dt(succ), bp, bp, bp, bp,
                      F_TB | F_LOWER | c64 | xf, -1.0, 1.0));
      if (apr)
        up.push_back(mk(RRt, ldbr, BRt, ldbr, BRo(slot[succ], bp), ldbr, apr, bp, bp,
                        F_TB | xf, -1.0, 1.0));
    }
    if (apr)
      up.push_back(mk(RRt, ldbr, RRt, ldbr, Ptip, m.ap, apr, apr, bp,
                      F_TB | F_LOWER | c64 | xf, -1.0, 1.0));
    const double upd = (root ? 0.0 : b * b * b + 2.0 * ar * b * b) + ar * ar * b;
    q.push_back(gs(K(major, 4), DL_CAT_UPDATE, upd, std::move(up)));
  };
  for (int k = 0; k < std::max(lenA, lenB); ++k) {
    const uint64_t major = (uint64_t)k + 1;
    if (k < lenA) eliminate(k, major, 0);
    if (k < lenB) eliminate(n - 1 - k, major, 1);
  }
  eliminate(mid, root_major, 2);
  if (two && apr)
    q.push_back(misc_step(K(root_major, 5), DL_CAT_OTHER, MJ_AXPY, P, I.PcB,
                          (int64_t)m.ap * m.ap));
  const uint64_t tail = (uint64_t)nt_max + 1;
  if (m.ap > 0) {
    Step s;
    s.key = K(tail, 0);
    s.kind = OP_POTRF;
    s.cat = DL_CAT_POTRF_TILE;
    s.flops = (double)m.a * m.a * m.a / 3.0;
    s.potrf.A = P;
    s.potrf.lda = m.ap;
    s.potrf.Ginv = (w == 1) ? I.GPc : I.GPp;
    s.potrf.logdiag = logdiag + (int64_t)m.nt * bp;
    s.potrf.info = info;
    s.potrf.row0 = (int64_t)m.nt * m.b;
    s.potrf.mode = 0;
    q.push_back(s);
  }
  Step sl;
  sl.key = K(tail, 1);
  sl.kind = OP_SUM;
  sl.cat = DL_CAT_OTHER;
  sl.sum.src = logdiag;
  sl.sum.n = m.Np;
  sl.sum.scale = 2.0;
  sl.sum.dst = I.logdet2 + w;
  sl.sum.partial = I.sumpart + w * SUM_BLOCKS;
  q.push_back(sl);
  if (w == 1) I.slot_final.assign(slot.begin(), slot.begin() + m.nt);
}

static Step gn_step(uint64_t key, GemvN g, double bytes) {
  Step s;
  s.key = key;
  s.kind = OP_GEMV_N;
  s.cat = DL_CAT_SOLVE;
  s.gn = g;
  s.bytes = bytes;
  s.flops = bytes / 4.0;
  s.gx = g.M;
  return s;
}

static Step gt_step(uint64_t key, GemvT g, double bytes) {
  Step s;
  s.key = key;
  s.kind = OP_GEMV_T;
  s.cat = DL_CAT_SOLVE;
  s.gt = g;
  s.bytes = bytes;
  s.flops = bytes / 4.0;
  s.gx = g.N;
  return s;
}

// Forward and backward block substitution with the factor of Q_c, in the
// elimination order of the factor: L z = x (z overwrites x), then
// L^T mu = z.  Forward, each block subtracts the coupling of the blocks
// eliminated into it (its predecessor in the chain; both chains' last
// blocks for the root) and applies G_t; the arrow rows accumulate into the
// tip part (chain B into a tip accumulator of its own, added before the
// tip solve).  Backward runs from the tip and the root outward:
// mu_t = G_t^T (z_t - C_t^T mu_succ(t) - R_t^T mu_P).
static void seq_solve(dl_ws* W, Inst& I, int nt_max, std::vector<Step>& q) {
  const ModelDev& m = I.m;
  const int bp = m.bp, ap = m.ap;
  const int64_t ldbr = I.ldbr;
  const double b = m.b, a = m.a;
  const int eb = I.eb;
  auto BRs = [&](int t) { return eoff(I.BRc, (int64_t)I.slot_final[t] * ldbr * bp, eb); };
  auto BRo = [&](int t, int rows) {
    return eoff(I.BRc, (int64_t)I.slot_final[t] * ldbr * bp + rows, eb);
  };
  auto G = [&](int t) { return I.Dc + (int64_t)t * bp * bp; };
  const int a32 = I.mixed ? 1 : 0;
  double* x = I.x;
  double* xP = x + (int64_t)m.nt * bp;
  double* mu = I.mu;
  double* muP = mu + (int64_t)m.nt * bp;
  auto xt = [&](int t) { return x + (int64_t)t * bp; };
  const int n = m.nt, mid = I.mid;
  const int lenA = mid, lenB = n - 1 - mid;
  const int steps = std::max(lenA, lenB);
  const uint64_t root_major = (uint64_t)steps + 1;
  // per chain (0: A and the root, 1: B): temporary, GEMV partial sums and
  // tip accumulator
  double* u[2] = {I.u, I.two ? I.uB : I.u};
  double* part[2] = {I.gpart, I.two ? I.gpartB : I.gpart};
  double* tipacc[2] = {xP, I.two ? I.xPB : xP};
  if (I.two && ap > 0)
    q.push_back(misc_step(K(0, 0), DL_CAT_SOLVE, MJ_FILL, I.xPB, nullptr, ap, 0.0));
  auto fwd = [&](int t, uint64_t major, int chain) {
    const int ci = chain == 1 ? 1 : 0;
    int preds[2][2];
    int np = 0;
    if (chain == 0 && t > 0) { preds[np][0] = t - 1; preds[np][1] = 0; ++np; }
    if (chain == 1 && t < n - 1) { preds[np][0] = t + 1; preds[np][1] = 1; ++np; }
    if (chain == 2) {
      if (lenA > 0) { preds[np][0] = mid - 1; preds[np][1] = 0; ++np; }
      if (lenB > 0) { preds[np][0] = mid + 1; preds[np][1] = 1; ++np; }
    }
    const double* base = xt(t);
    for (int k = 0; k < np; ++k) {
      const int pb = preds[k][0], pc = preds[k][1];
      q.push_back(gn_step(K(major, 0, 0, k), {bp + ap, bp, BRs(pb), ldbr, xt(pb), 0, -1.0,
                                              1.0, bp, base, u[ci], tipacc[pc], tipacc[pc],
                                              part[ci], a32},
                          8.0 * (b + a) * b));
      base = u[ci];
    }
    q.push_back(gn_step(K(major, 1), {bp, bp, G(t), bp, np > 0 ? u[ci] : xt(t), 1, 1.0,
                                      0.0, -1, nullptr, xt(t), nullptr, nullptr, part[ci]},
                        4.0 * b * b));
  };
  for (int k = 0; k < steps; ++k) {
    if (k < lenA) fwd(k, (uint64_t)k + 1, 0);
    if (k < lenB) fwd(n - 1 - k, (uint64_t)k + 1, 1);
  }
  fwd(mid, root_major, 2);
  const uint64_t tk = (uint64_t)nt_max + 1;
  if (ap > 0) {
    q.push_back(gn_step(K(tk, 0), {ap, bp, BRo(mid, bp), ldbr, xt(mid), 0, -1.0, 1.0, -1,
                                   xP, xP, nullptr, nullptr, part[0], a32},
                        8.0 * a * b));
    if (I.two)
      q.push_back(misc_step(K(tk, 0, 0, 1), DL_CAT_SOLVE, MJ_AXPY, xP, I.xPB, ap));
    q.push_back(gn_step(K(tk, 1), {ap, ap, I.GPc, ap, xP, 1, 1.0, 0.0, -1, nullptr,
                                   xP, nullptr, nullptr, part[0]},
                        4.0 * a * a));
    q.push_back(gt_step(K(tk, 2), {ap, ap, I.GPc, ap, xP, -1, nullptr, 1, 1.0, 0.0,
                                   nullptr, muP},
                        4.0 * a * a));
  }
  auto bwd = [&](int t, uint64_t major, int chain) {
    const int ci = chain == 1 ? 1 : 0;
    if (chain == 2) {
      if (ap > 0)
        q.push_back(gt_step(K(major, 0), {ap, bp, BRo(t, bp), ldbr, muP, -1, nullptr, 0,
                                          -1.0, 1.0, xt(t), u[0], a32},
                            8.0 * a * b));
      else
        q.push_back(misc_step(K(major, 0), DL_CAT_SOLVE, MJ_COPY, u[0], xt(t), bp));
    } else {
      const int succ = chain == 0 ? t + 1 : t - 1;
      q.push_back(gt_step(K(major, 0), {bp + ap, bp, BRs(t), ldbr,
                                        mu + (int64_t)succ * bp, bp, muP, 0, -1.0, 1.0,
                                        xt(t), u[ci], a32},
                          8.0 * (b + a) * b));
    }
    q.push_back(gt_step(K(major, 1), {bp, bp, G(t), bp, u[ci], -1, nullptr, 1, 1.0, 0.0,
                                      nullptr, mu + (int64_t)t * bp},
                        4.0 * b * b));
  };
  bwd(mid, tk + 1, 2);
  for (int k = 0; k < steps; ++k) {
    const uint64_t major = tk + 2 + (uint64_t)k;
    if (k < lenA) bwd(mid - 1 - k, major, 0);
    if (k < lenB) bwd(mid + 1 + k, major, 1);
  }
}

// Takahashi selected inversion of Q_c from the factor's off-diagonal blocks
// and the diagonal-block inverses G_t, in the reverse of the elimination
// order: the root block first, then each chain outward.  Block t needs the
// inverse entries of its successor s (the block it was eliminated into):
//   [X_{s,t}; X_{P,t}] = -[[X_{s,s}, X_{s,P}]; [X_{P,s}, X_P]] [W_t; V_t],
//   X_tt = G_t^T G_t - [X_{s,t}; X_{P,t}]^T [W_t; V_t],
// [W_t; V_t] = [C_t; R_t]_factor G_t (the root has no coupling rows).  Each
// chain keeps the current [X_{s,s}, X_{s,P}; X_{P,s}, X_P] in a pair of
// ping-pong buffers; chain B starts from the root's buffer of chain A.
static void seq_selinv(dl_ws* W, Inst& I, int nt_max, std::vector<Step>& q) {
  const ModelDev& m = I.m;
  const int bp = m.bp, ap = m.ap;
  const int64_t ld = I.ldbr;  // bp + ap
  const double b = m.b, a = m.a;
  const int eb = I.eb;
  auto BRs = [&](int t) { return eoff(I.BRc, (int64_t)I.slot_final[t] * ld * bp, eb); };
  auto BRo = [&](int t, int rows) {
    return eoff(I.BRc, (int64_t)I.slot_final[t] * ld * bp + rows, eb);
  };
  auto G = [&](int t) { return I.Dc + (int64_t)t * bp * bp; };
  // mixed precision: W = [B;R]G and the products with it run on FP32 MFMA
  const bool mx = I.mixed;
  auto gs = [&](uint64_t key, int cat, double fl, std::vector<GemmTask> ts) {
    return mx ? gemm32_step(key, cat, fl, std::move(ts)) : gemm_step(key, cat, fl, std::move(ts));
  };
  const int fB64 = mx ? F_B64 : 0, fA64 = mx ? F_A64 : 0, fC64 = mx ? F_C64 : 0;
  const int xf = W->splitk ? F_SPLIT : 0;  // dropped by FP32 launches
  const int n = m.nt, mid = I.mid;
  const int lenA = mid, lenB = n - 1 - mid;
  const int nch = I.two ? 2 : 1;
  double* XCc[2][2] = {{I.XC[0], I.XC[1]}, {I.XCB[0], I.XCB[1]}};
  double* Yc[2] = {I.Y, I.YB};
  // [W_t; V_t] of every step, eb bytes per element, ld x bp each
  auto WVt = [&](int t) { return eoff(I.WV, (int64_t)t * ld * bp, eb); };
  for (int c = 0; c < nch; ++c)
    for (int k = 0; k < 2; ++k)
      q.push_back(misc_step(K(0, 0, 0, 2 * c + k), DL_CAT_SELINV, MJ_FILL, XCc[c][k],
                            nullptr, ld * ld, 0.0));
  if (ap > 0) {
    // X_P = G_P^T G_P into the corner of every ping-pong buffer
    std::vector<GemmTask> xp;
    for (int c = 0; c < nch; ++c)
      for (int k = 0; k < 2; ++k)
        xp.push_back(mk(I.GPc, ap, I.GPc, ap, XCc[c][k] + bp + (int64_t)bp * ld, ld, ap,
                        ap, ap, F_TA | F_BETA0, 1.0, 0.0));
    q.push_back(gemm_step(K(0, 1), DL_CAT_SELINV, 2.0 * a * a * a, xp));
    Step dg = misc_step(K(0, 2), DL_CAT_SELINV, MJ_DIAG,
                        I.selout + (int64_t)m.nt * bp, I.XC[0] + bp + (int64_t)bp * ld,
                        ap);
    dg.misc.lds = ld;
    q.push_back(dg);
  }
  // [W_t; V_t] = [C_t; R_t]_factor G_t for all t: independent of the
  // recursion, so one launch (the root has only the arrow rows; its W block
  // is zero)
  {
    q.push_back(misc_step(K(0, 3), DL_CAT_SELINV, MJ_FILL, WVt(mid), nullptr,
                          ld * bp * eb / 8));
    std::vector<GemmTask> wv;
    double fl = 0.0;
    for (int t = 0; t < m.nt; ++t) {
      if (t == mid) {
        if (ap > 0) {
          wv.push_back(mk(BRo(t, bp), ld, G(t), bp, eoff(WVt(t), bp, eb), ld, ap, bp, bp,
                          F_KLO_COL | F_BETA0 | fB64 | xf, 1.0, 0.0));
          fl += a * b * b;
        }
      } else {
        wv.push_back(mk(BRs(t), ld, G(t), bp, WVt(t), ld, bp + ap, bp, bp,
                        F_KLO_COL | F_BETA0 | fB64 | xf, 1.0, 0.0));
        fl += (b + a) * b * b;
      }
    }
    if (!wv.empty()) q.push_back(gs(K(0, 4), DL_CAT_SELINV, fl, wv));
  }
  auto step = [&](int t, uint64_t mj, double* Xin, double* Xout, double* Y, bool root) {
    const double ba = b + a;
    // [X_{s,t}; X_{P,t}] = -X(s) WV and, independent of it (same launch
    // when both run in FP64), X_tt = G_t^T G_t (lower triangle)
    q.push_back(gs(K(mj, 2), DL_CAT_SELINV, root ? 2.0 * a * ba * b : 2.0 * ba * ba * b,
                   {mk(Xin, ld, WVt(t), ld, Y, ld, bp + ap, bp, bp + ap,
                       F_BETA0 | fA64 | fC64 | xf, -1.0, 0.0)}));
    q.push_back(gemm_step(K(mj, 2), DL_CAT_SELINV, b * b * b / 3.0,
                          {mk(G(t), bp, G(t), bp, Xout, ld, bp, bp, bp,
                              F_TA | F_KLO_ROW | F_KLO_COL | F_LOWER | F_BETA0 | xf, 1.0,
                              0.0)}));
    // X_tt -= Y^T WV   (lower triangle)
    q.push_back(gs(K(mj, 4), DL_CAT_SELINV, root ? b * b * a : b * b * ba,
                   {mk(Y, ld, WVt(t), ld, Xout, ld, bp, bp, bp + ap,
                       F_TA | F_LOWER | fA64 | fC64 | xf, -1.0, 1.0)}));
    Step fin;
    fin.key = K(mj, 5);
    fin.kind = OP_FINISH;
    fin.cat = DL_CAT_SELINV;
    fin.fin.XC = Xout;
    fin.fin.ld = ld;
    fin.fin.bp = bp;
    fin.fin.ap = ap;
    fin.fin.Y = Y;
    fin.fin.out = I.selout + (int64_t)t * bp;
    fin.gx = bp;
    q.push_back(fin);
  };
  step(mid, 1, XCc[0][0], XCc[0][1], Yc[0], true);
  int cur[2] = {1, -1};  // chain B reads the root's buffer first
  for (int k = 0; k < std::max(lenA, lenB); ++k) {
    const uint64_t mj = 2 + (uint64_t)k;
    if (k < lenA) {
      step(mid - 1 - k, mj, XCc[0][cur[0]], XCc[0][cur[0] ^ 1], Yc[0], false);
      cur[0] ^= 1;
    }
    if (k < lenB) {
      double* in = (k == 0) ? XCc[0][1] : XCc[1][cur[1]];
      const int out = (k == 0) ? 0 : (cur[1] ^ 1);
      step(mid + 1 + k, mj, in, XCc[1][out], Yc[1], false);
      cur[1] = out;
    }
  }
}

// FP64 iterative refinement of the mean (mixed precision) and the final
// residual |rhs - Q_c mu| / |rhs| of every workspace.  Each refinement step:
// x = rhs - Q_c mu_acc (FP64, sparse), solve with the factor (x -> mu),
// mu_acc += mu.
static Step res_step(uint64_t key, Inst& I, const double* v, double* out) {
  Step s;
  s.key = key;
  s.kind = OP_RES;
  s.cat = DL_CAT_SOLVE;
  s.res.m = I.model->dev;
  s.res.coef = I.coef;
  s.res.v = v;
  s.res.rhs = I.rhs;
  s.res.out = out;
  s.res.av = I.av;
  s.res.partial = I.rpart;
  s.res.norms = I.rnorm;
  s.res.obs_d = I.poisson ? I.obs_d : nullptr;
  return s;
}

// The pieces of one refinement: init copies mu to the iterate mu_acc; res
// forms x = rhs - Q_c mu_acc and its norms; corr solves with the factor
// (x -> mu) and adds mu to mu_acc unless the residual was already within
// the tolerance (the iterate then stays as it is, bit for bit); fin copies
// mu_acc back to mu and forms its residual; resid forms the residual of mu.
static void seq_refine_corr(dl_ws* W, Inst& I, int nt_max, std::vector<Step>& q) {
  seq_solve(W, I, nt_max, q);
  Step ax = misc_step(K(2 * (uint64_t)nt_max + 8, 0), DL_CAT_SOLVE, MJ_AXPY_UNCONV, I.mu_acc,
                      I.mu, I.m.Np);
  ax.misc.norms = I.rnorm;
  ax.misc.tol2 = W->tol2_dev;
  q.push_back(ax);
}

// mu^T Q_p mu, (y - A mu)^T D (y - A mu) and f_obj, per instance.
static void seq_post(dl_ws* W, Inst& I, int k, std::vector<Step>& q) {
  Step s;
  s.key = K(0, 0);
  s.kind = OP_QUAD;
  s.cat = DL_CAT_OTHER;
  s.quad.m = I.model->dev;
  s.quad.coef = I.coef;
  s.quad.mu = I.mu;
  s.quad.partial = I.qpart;
  s.quad.out2 = I.quad2;
  q.push_back(s);
  Step c;
  c.key = K(0, 1);
  c.kind = OP_COMBINE;
  c.cat = DL_CAT_OTHER;
  c.comb.coef = I.coef;
  c.comb.logdet2 = I.logdet2;
  c.comb.info2 = I.info2;
  c.comb.quad2 = I.quad2;
  c.comb.f = W->f_all + k;
  c.comb.parts = (dl_fobj_parts*)(W->parts_all + 8 * (int64_t)k);
  c.comb.info_out = W->info_all + 2 * (int64_t)k;
  c.comb.rnorm = I.rnorm;
  c.comb.tol2 = (I.mixed && !I.poisson) ? W->tol2_dev : nullptr;
  q.push_back(c);
}

static void append(Plan& dst, const Plan& src) {
  dst.idx.insert(dst.idx.end(), src.idx.begin(), src.idx.end());
}

static dl_status build_plans(dl_ws* W) {
  int nt_max = 0;
  for (auto& I : W->inst) nt_max = std::max(nt_max, I.m.nt);
  Descs& H = W->H;
  // assembly: which = 0 (Q_p), 1 (Q_c), 2 (both)
  for (int wh = 0; wh < 3; ++wh) {
    std::vector<std::vector<Step>> seqs;
    for (auto& I : W->inst) {
      seqs.emplace_back();
      seq_assemble(W, I, wh != 1, wh != 0, seqs.back());
    }
    merge(seqs, H, W->table, W->asm_p[wh]);
  }
  for (int wh = 0; wh < 3; ++wh) {
    std::vector<std::vector<Step>> seqs;
    for (auto& I : W->inst)
      for (int w = 0; w < 2; ++w) {
        if ((wh == 0 && w == 1) || (wh == 1 && w == 0)) continue;
        seqs.emplace_back();
        seq_factor(W, I, w, nt_max, seqs.back());
      }
    merge(seqs, H, W->table, W->fac_p[wh]);
  }
  {
    std::vector<std::vector<Step>> seqs;
    for (auto& I : W->inst) {
      seqs.emplace_back();
      seqs.back().push_back(misc_step(K(0, 0), DL_CAT_SOLVE, MJ_COPY, I.x, I.rhs, I.m.Np));
      std::vector<Step> s2;
      seq_solve(W, I, nt_max, s2);
      for (auto& st : s2) st.key += K(1, 0);  // after the copy
      seqs.back().insert(seqs.back().end(), s2.begin(), s2.end());
    }
    merge(seqs, H, W->table, W->solve_p);
  }
  {
    std::vector<std::vector<Step>> init, res, corr, fin, resid;
    for (auto& I : W->inst) {
      init.push_back({misc_step(K(0, 0), DL_CAT_SOLVE, MJ_COPY, I.mu_acc, I.mu, I.m.Np)});
      res.push_back({res_step(K(0, 0), I, I.mu_acc, I.x)});
      corr.emplace_back();
      seq_refine_corr(W, I, nt_max, corr.back());
      fin.push_back({misc_step(K(0, 0), DL_CAT_SOLVE, MJ_COPY, I.mu, I.mu_acc, I.m.Np),
                     res_step(K(0, 1), I, I.mu, I.x)});
      resid.push_back({res_step(K(0, 0), I, I.mu, I.x)});
    }
    merge(init, H, W->table, W->ref_init_p);
    merge(res, H, W->table, W->ref_res_p);
    merge(corr, H, W->table, W->ref_corr_p);
    merge(fin, H, W->table, W->ref_fin_p);
    merge(resid, H, W->table, W->resid_p);
  }
  {
    std::vector<std::vector<Step>> seqs;
    for (size_t k = 0; k < W->inst.size(); ++k) {
      seqs.emplace_back();
      seq_post(W, W->inst[k], (int)k, seqs.back());
    }
    merge(seqs, H, W->table, W->post_p);
  }
  if (W->sel) {
    std::vector<std::vector<Step>> seqs;
    for (auto& I : W->inst) {
      seqs.emplace_back();
      seq_selinv(W, I, nt_max, seqs.back());
    }
    merge(seqs, H, W->table, W->selinv_p);
  }
  W->eval_p.idx.clear();
  append(W->eval_p, W->asm_p[2]);
  append(W->eval_p, W->fac_p[2]);
  append(W->eval_p, W->solve_p);
  if (W->mixed) {
    // a captured graph runs a fixed number of correction steps (instances
    // that meet the tolerance earlier stay as they are)
    append(W->eval_p, W->ref_init_p);
    for (int r = 0; r < DL_REFINE_STEPS_GRAPH; ++r) {
      append(W->eval_p, W->ref_res_p);
      append(W->eval_p, W->ref_corr_p);
    }
    append(W->eval_p, W->ref_fin_p);
  } else {
    append(W->eval_p, W->resid_p);
  }
  append(W->eval_p, W->post_p);
  // split-k partial tiles: the largest need of any launch, for either tile
  int64_t pmax = 0;
  for (const Launch& L : W->table) {
    if (L.kind != OP_GEMM) continue;
    for (int tile : {64, 128}) {
      std::vector<GemmTask> tmp(H.gemm.begin() + L.off, H.gemm.begin() + L.off + L.count);
      int64_t slots = 0;
      (void)finalize_tasks(tmp.data(), L.count, tile, nullptr, &slots);
      pmax = std::max(pmax, slots * tile * tile);
    }
  }
  // upload descriptor arrays
  dl_status st = DL_OK;
  if (pmax > 0) st = ensure_partials(W, pmax, nullptr);
  auto up = [&](auto& vec, auto*& dptr) {
    using T = typename std::remove_reference<decltype(vec)>::type::value_type;
    if (st != DL_OK) return;
    void* p = nullptr;
    st = dev_alloc(W->allocs, sizeof(T) * (vec.size() + 1), &p, &W->bytes);
    if (st != DL_OK) return;
    if (!vec.empty() &&
        hipMemcpy(p, vec.data(), sizeof(T) * vec.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
      st = DL_EHIP;
    dptr = (T*)p;
  };
  up(H.gemm, W->Dd.gemm);
  up(H.potrf, W->Dd.potrf);
  up(H.panel, W->Dd.panel);
  up(H.dagb, W->Dd.dagb);
  up(H.dagt, W->Dd.dagt);
  if (st == DL_OK && H.dag_launches > 0) {
    const size_t hb = sizeof(int32_t) * 4 * (size_t)H.dag_launches;
    st = dev_alloc(W->allocs, hb, (void**)&W->dag_heads, &W->bytes);
    if (st == DL_OK && hipMemset(W->dag_heads, 0, hb) != hipSuccess) st = DL_EHIP;
    int dev = 0, cus = 0;
    if (st == DL_OK && (hipGetDevice(&dev) != hipSuccess ||
                        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                              dev) != hipSuccess))
      st = DL_EHIP;
    W->dag_workers = 2 * std::max(cus, 1);
  }
  up(H.misc, W->Dd.misc);
  up(H.gn, W->Dd.gn);
  up(H.gt, W->Dd.gt);
  up(H.sum, W->Dd.sum);
  up(H.fin, W->Dd.fin);
  up(H.asmj, W->Dd.asmj);
  up(H.th, W->Dd.th);
  up(H.quad, W->Dd.quad);
  up(H.comb, W->Dd.comb);
  up(H.res, W->Dd.res);
  if (W->poisson) {
    std::vector<LapJob> lap;
    std::vector<TrialJob> trial;
    std::vector<QuadJob> nquad;
    for (auto& I : W->inst) {
      lap.push_back(LapJob{I.model->dev, I.xcur, I.obs_d, I.obs_z});
      trial.push_back(TrialJob{I.model->dev, I.xcur, I.xN, I.mu, I.alpha, I.tpart,
                               I.quad2, I.out4});
      nquad.push_back(QuadJob{I.model->dev, I.coef, I.mu, I.qpart, I.quad2});
    }
    up(lap, W->d_lap);
    up(trial, W->d_trial);
    up(nquad, W->d_nquad);
  }
  return st;
}

static void ws_free(dl_ws* W) {
  if (!W) return;
  for (hipEvent_t e : W->prof_ev) (void)hipEventDestroy(e);
  if (W->graph_exec) (void)hipGraphExecDestroy(W->graph_exec);
  if (W->graph) (void)hipGraphDestroy(W->graph);
  if (W->cap_stream) (void)hipStreamDestroy(W->cap_stream);
  if (W->aux_stream) (void)hipStreamDestroy(W->aux_stream);
  if (W->ev_fork) (void)hipEventDestroy(W->ev_fork);
  if (W->ev_join) (void)hipEventDestroy(W->ev_join);
  if (W->partials) (void)hipFree(W->partials);
  free_all(W->allocs);
  delete W;
}

// Storage layout of instance I (host fields only) for the workspace flags.
static void inst_layout(const dl_ws* W, Inst& I, const dl_model* model, bool two_sided) {
  I.model = model;
  I.m = model->d;
  I.dim = I.m.dim_theta;
  const ModelDev& m = I.m;
  I.qp_ring = !W->keep_qp;
  I.ldbr = m.bp + m.ap;
  I.mixed = W->mixed;
  I.eb = I.mixed ? 4 : 8;
  // two chains need at least one block each besides the root
  I.two = two_sided && m.nt >= 4;
  I.mid = I.two ? (m.nt + 1) / 2 : m.nt - 1;
  I.poisson = W->poisson;
}

// The device buffers of instance I (laid out by inst_layout): A(bytes, &ptr)
// allocates them, or only counts them when the workspace is being sized.
template <typename Alloc>
static void inst_buffers(const dl_ws* W, Inst& I, Alloc&& A) {
  const ModelDev& m = I.m;
  const int bp = m.bp, ap = m.ap;
  const int64_t bb = (int64_t)bp * bp;
  const int xs = I.two ? 1 : 0;  // extra spare slot of chain B
  const size_t eb = I.eb;
  if (I.qp_ring) {
    A(sizeof(double) * (I.two ? 5 : 2) * bb, (void**)&I.Dp);
    A(eb * (I.two ? 7 : 3) * bb, (void**)&I.Bp);
  } else {
    A(sizeof(double) * m.nt * bb, (void**)&I.Dp);
    A(eb * (m.nt + 1 + xs) * bb, (void**)&I.Bp);
  }
  A(sizeof(double) * m.nt * bb, (void**)&I.Dc);
  A(eb * (m.nt + 1 + xs) * I.ldbr * bp, (void**)&I.BRc);
  A(sizeof(double) * m.Np, (void**)&I.mu_acc);
  A(sizeof(double) * (m.m_total + 1), (void**)&I.av);
  A(sizeof(double) * 2 * QF_BLOCKS, (void**)&I.rpart);
  const size_t tip = sizeof(double) * (ap > 0 ? ap * ap : 1);
  A(tip, (void**)&I.Pp);
  A(tip, (void**)&I.Pc);
  A(tip, (void**)&I.GPc);
  A(tip, (void**)&I.GPp);
  // per diagonal-block factorisation: the side ring and the folded
  // inverse's accumulators (2 + nbk (nbk - 1) / 2 tiles of 64 x 64), or
  // the recursive inverse's bp x (bp / 2 + 64) temporary (the larger)
  const int64_t nbk = bp / 64;
  const size_t ftemp = sizeof(double) * std::max<int64_t>(
      4096 * (2 + nbk * (nbk - 1) / 2), (int64_t)bp * (nbk / 2 + 1) * 64);
  for (int w = 0; w < 2; ++w) {
    A(ftemp, (void**)&I.ttemp[w]);
    A(sizeof(double) * m.Np, (void**)&I.logdiag[w]);
  }
  A(sizeof(double) * (I.dim + 1), (void**)&I.theta);
  A(sizeof(double) * C_SIZE, (void**)&I.coef);
  A(sizeof(double) * 2, (void**)&I.logdet2);
  A(sizeof(int64_t) * 2, (void**)&I.info2);
  A(sizeof(double) * 2, (void**)&I.quad2);
  A(sizeof(double) * 2 * SUM_BLOCKS, (void**)&I.sumpart);
  A(sizeof(double) * 2 * QF_BLOCKS, (void**)&I.qpart);
  A(sizeof(double) * m.Np, (void**)&I.rhs);
  A(sizeof(double) * m.Np, (void**)&I.x);
  A(sizeof(double) * m.Np, (void**)&I.mu);
  A(sizeof(double) * I.ldbr, (void**)&I.u);
  A(sizeof(double) * GEMV_KS * I.ldbr, (void**)&I.gpart);
  if (I.poisson) {
    A(sizeof(double) * (m.m_total + 1), (void**)&I.obs_d);
    A(sizeof(double) * (m.m_total + 1), (void**)&I.obs_z);
    A(sizeof(double) * m.Np, (void**)&I.xcur);
    A(sizeof(double) * m.Np, (void**)&I.xN);
    A(sizeof(double) * 2 * QF_BLOCKS, (void**)&I.tpart);
  }
  if (W->dag) {
    const size_t nc = sizeof(int32_t) * (size_t)dag::counters_per_block((int)nbk);
    for (int w = 0; w < 2; ++w) {
      A(sizeof(double) * bb, (void**)&I.lbuf[w]);
      A(nc, (void**)&I.dctr[w]);
      if (I.two) {
        A(sizeof(double) * bb, (void**)&I.lbufB[w]);
        A(nc, (void**)&I.dctrB[w]);
      }
    }
  }
  if (I.two) {
    A(tip, (void**)&I.PcB);
    for (int w = 0; w < 2; ++w) A(ftemp, (void**)&I.ttempB[w]);
    A(sizeof(double) * I.ldbr, (void**)&I.uB);
    A(sizeof(double) * GEMV_KS * I.ldbr, (void**)&I.gpartB);
    A(sizeof(double) * (ap > 0 ? ap : 1), (void**)&I.xPB);
  }
  if (W->sel) {
    // [W_t; V_t] = [B_t; R_t] G_t of every time step (formed up front)
    A((size_t)I.eb * m.nt * I.ldbr * bp, (void**)&I.WV);
    A(sizeof(double) * I.ldbr * bp, (void**)&I.Y);
    A(sizeof(double) * I.ldbr * I.ldbr, (void**)&I.XC[0]);
    A(sizeof(double) * I.ldbr * I.ldbr, (void**)&I.XC[1]);
    A(sizeof(double) * m.Np, (void**)&I.selout);
    if (I.two) {
      A(sizeof(double) * I.ldbr * bp, (void**)&I.YB);
      A(sizeof(double) * I.ldbr * I.ldbr, (void**)&I.XCB[0]);
      A(sizeof(double) * I.ldbr * I.ldbr, (void**)&I.XCB[1]);
    }
  }
}

// The workspace-wide buffers of a batch of nmodels instances.
template <typename Alloc>
static void ws_buffers(dl_ws* W, int nmodels, int dim_total, Alloc&& A) {
  A(sizeof(double) * (dim_total + 1), (void**)&W->theta_all);
  A(sizeof(double) * nmodels, (void**)&W->f_all);
  A(sizeof(double) * 8 * nmodels, (void**)&W->parts_all);
  A(sizeof(int64_t) * 2 * nmodels, (void**)&W->info_all);
  A(sizeof(double) * 2 * nmodels, (void**)&W->rnorm_all);
  A(sizeof(double), (void**)&W->tol2_dev);
  A(sizeof(MiscJob), (void**)&W->d_io);
  if (W->poisson) {
    A(sizeof(double) * nmodels, (void**)&W->alpha_all);
    A(sizeof(double) * 4 * nmodels, (void**)&W->out4_all);
  }
}

// Flags of a workspace (host fields only).
static void ws_flags(dl_ws* W, int32_t flags) {
  W->flags = flags;
  W->sel = (flags & DL_WS_SELINV) != 0;
  W->keep_qp = (flags & DL_WS_KEEP_QP) != 0;
  W->mixed = (flags & DL_WS_MIXED) != 0;
  W->use_graph = (flags & DL_WS_GRAPH) != 0;
  W->splitk = (flags & DL_WS_SPLITK) != 0;
  W->fold_inv = (flags & DL_WS_FOLD_INV) != 0;
  W->warm = (flags & DL_WS_WARM_START) != 0;
  W->dag = (flags & DL_WS_DAG) != 0;
}

// Bytes of the buffers of each instance and of the workspace-wide ones,
// without allocating (the launch descriptors built at creation and the
// split-k partial tiles of DL_WS_SPLITK or of a later dl_autotune are not
// included).
static dl_status ws_sizes(const dl_model* const* models, int32_t nmodels, int32_t flags,
                          std::vector<size_t>* per_inst, size_t* shared) {
  if (!models || nmodels <= 0) return DL_EINVAL;
  dl_ws W;
  ws_flags(&W, flags);
  W.poisson = models[0] && models[0]->d.likelihood == DL_LIK_POISSON;
  per_inst->assign(nmodels, 0);
  int dim_total = 0;
  for (int k = 0; k < nmodels; ++k) {
    if (!models[k]) return DL_EINVAL;
    if ((models[k]->d.likelihood == DL_LIK_POISSON) != W.poisson) return DL_EINVAL;
    Inst I;
    inst_layout(&W, I, models[k], (flags & DL_WS_TWOSIDED) != 0);
    dim_total += I.dim;
    size_t bytes = 0;
    inst_buffers(&W, I, [&](size_t b, void** p) { bytes += b; *p = nullptr; });
    (*per_inst)[k] = bytes;
  }
  size_t sh = 0;
  ws_buffers(&W, nmodels, dim_total, [&](size_t b, void** p) { sh += b; *p = nullptr; });
  *shared = sh;
  return DL_OK;
}

extern "C" dl_status dl_ws_create_batch(const dl_model* const* models,
                                        int32_t nmodels, int32_t flags,
                                        dl_ws** out) {
  if (!models || nmodels <= 0 || !out) return DL_EINVAL;
  for (int k = 0; k < nmodels; ++k)
    if (!models[k]) return DL_EINVAL;
  dl_ws* W = new (std::nothrow) dl_ws();
  if (!W) return DL_ENOMEM;
  ws_flags(W, flags);
  const bool two_sided = (flags & DL_WS_TWOSIDED) != 0;
  // one likelihood per workspace
  W->poisson = models[0]->d.likelihood == DL_LIK_POISSON;
  for (int k = 0; k < nmodels; ++k)
    if ((models[k]->d.likelihood == DL_LIK_POISSON) != W->poisson) {
      delete W;
      return DL_EINVAL;
    }
  W->newton_steps.assign(nmodels, 0);
  W->has_mode.assign(nmodels, 0);
  W->inst.resize(nmodels);
  dl_status st = DL_OK;
  auto A = [&](size_t bytes, void** p) {
    if (st == DL_OK) st = dev_alloc(W->allocs, bytes, p, &W->bytes);
  };
  int dim_total = 0;
  for (int k = 0; k < nmodels; ++k) {
    Inst& I = W->inst[k];
    inst_layout(W, I, models[k], two_sided);
    dim_total += I.dim;
    W->max_shmem = std::max(W->max_shmem, 2 * I.m.bp + I.m.ap);
    inst_buffers(W, I, A);
    if (I.poisson && st == DL_OK &&
        (hipMemset(I.obs_d, 0, sizeof(double) * (I.m.m_total + 1)) != hipSuccess ||
         hipMemset(I.obs_z, 0, sizeof(double) * (I.m.m_total + 1)) != hipSuccess))
      st = DL_EHIP;
    if (W->dag && st == DL_OK) {
      const size_t nc = sizeof(int32_t) * (size_t)dag::counters_per_block(I.m.bp / 64);
      for (int w = 0; w < 2 && st == DL_OK; ++w)
        for (int32_t* c : {I.dctr[w], I.dctrB[w]})
          if (c && hipMemset(c, 0, nc) != hipSuccess) st = DL_EHIP;
    }

  }
  W->dim_total = dim_total;
  ws_buffers(W, nmodels, dim_total, A);
  if (st != DL_OK) {
    ws_free(W);
    return st;
  }
  // instance theta buffers are views of the packed array, residual norms
  // views of theirs
  {
    int off = 0;
    for (size_t k = 0; k < W->inst.size(); ++k) {
      Inst& I = W->inst[k];
      I.theta = W->theta_all + off;
      off += I.dim;
      I.rnorm = W->rnorm_all + 2 * k;
    }
  }
  W->rnorm_host.assign(2 * (size_t)nmodels, 0.0);
  W->tol2_host = DL_REFINE_TOL * DL_REFINE_TOL;
  if (hipMemcpy(W->tol2_dev, &W->tol2_host, sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(W->rnorm_all, 0, sizeof(double) * 2 * nmodels) != hipSuccess) {
    ws_free(W);
    return DL_EHIP;
  }
  if (W->poisson)
    for (int k = 0; k < nmodels; ++k) {
      W->inst[k].alpha = W->alpha_all + k;
      W->inst[k].out4 = W->out4_all + 4 * k;
    }
  if (W->max_shmem * 8 > 160 * 1024 ||
      prepare_assemble(W->max_shmem) != hipSuccess) {
    ws_free(W);
    return DL_EINVAL;
  }
  if ((st = build_plans(W)) != DL_OK) {
    ws_free(W);
    return st;
  }
  *out = W;
  return DL_OK;
}

extern "C" dl_status dl_ws_estimate_bytes(const dl_model* const* models, int32_t nmodels,
                                          int32_t flags, size_t* bytes_host) {
  if (!bytes_host) return DL_EINVAL;
  std::vector<size_t> per;
  size_t shared = 0;
  const dl_status st = ws_sizes(models, nmodels, flags, &per, &shared);
  if (st != DL_OK) return st;
  size_t tot = shared;
  for (size_t b : per) tot += b;
  *bytes_host = tot;
  return DL_OK;
}

extern "C" dl_status dl_ws_create_budget(const dl_model* const* models, int32_t nmodels,
                                         int32_t flags, size_t hbm_budget, dl_ws** out) {
  if (!out) return DL_EINVAL;
  size_t need = 0;
  const dl_status st = dl_ws_estimate_bytes(models, nmodels, flags, &need);
  if (st != DL_OK) return st;
  if (need > hbm_budget) return DL_ENOMEM;
  return dl_ws_create_batch(models, nmodels, flags, out);
}

extern "C" dl_status dl_plan_waves(const dl_model* const* models, int32_t nmodels,
                                   int32_t flags, size_t hbm_budget, int32_t* wave_of_host,
                                   int32_t* nwaves_host) {
  if (!wave_of_host || !nwaves_host) return DL_EINVAL;
  std::vector<size_t> per;
  size_t shared = 0;
  dl_status st = ws_sizes(models, nmodels, flags, &per, &shared);
  if (st != DL_OK) return st;
  // first fit, largest instance first; each wave also holds the
  // workspace-wide buffers of the whole batch (an upper bound) and
  // DL_WAVE_RESERVE bytes for its launch descriptors
  const size_t fixed = shared + (size_t)DL_WAVE_RESERVE;
  std::vector<int> order(nmodels);
  for (int k = 0; k < nmodels; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return per[a] > per[b]; });
  std::vector<size_t> used;
  for (int k : order) {
    if (per[k] + fixed > hbm_budget) return DL_ENOMEM;
    int w = 0;
    while (w < (int)used.size() && used[w] + per[k] > hbm_budget) ++w;
    if (w == (int)used.size()) used.push_back(fixed);
    used[w] += per[k];
    wave_of_host[k] = w;
  }
  *nwaves_host = (int32_t)used.size();
  return DL_OK;
}

extern "C" dl_status dl_ws_create(const dl_model* model, int32_t flags,
                                  dl_ws** out) {
  const dl_model* ms[1] = {model};
  return dl_ws_create_batch(ms, 1, flags, out);
}

extern "C" void dl_ws_destroy(dl_ws* W) { ws_free(W); }
extern "C" size_t dl_ws_bytes(const dl_ws* W) { return W ? W->bytes : 0; }
extern "C" int32_t dl_ws_batch(const dl_ws* W) { return W ? (int32_t)W->inst.size() : 0; }

// ---- entry points --------------------------------------------------------------------------

static dl_status copy_theta_in(dl_ws* W, const double* theta_dev, int n_inst,
                               hipStream_t s) {
  int dims = 0;
  for (int k = 0; k < n_inst; ++k) dims += W->inst[k].dim;
  DL_HIP_CHECK(hipMemcpyAsync(W->theta_all, theta_dev, sizeof(double) * dims,
                              hipMemcpyDeviceToDevice, s));
  return DL_OK;
}

// ---- iterative refinement of the mean -----------------------------------------------------

__global__ void k_set_double(double* p, double v) {
  if (threadIdx.x == 0) p[0] = v;
}

// Make tol the relative tolerance the refinement kernels read (stream
// order; the value travels as a kernel argument).
static dl_status set_refine_tol(dl_ws* W, double tol, hipStream_t s) {
  const double t2 = tol * tol;
  if (t2 == W->tol2_host) return DL_OK;
  W->tol2_host = t2;
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(64), 0, s, W->tol2_dev, t2);
  DL_HIP_CHECK(hipGetLastError());
  return DL_OK;
}

// Read every instance's residual norms (synchronises s); true when all are
// within the tolerance.
static dl_status refine_all_converged(dl_ws* W, hipStream_t s, bool* conv) {
  const size_t B = W->inst.size();
  DL_HIP_CHECK(hipMemcpyAsync(W->rnorm_host.data(), W->rnorm_all, sizeof(double) * 2 * B,
                              hipMemcpyDeviceToHost, s));
  DL_HIP_CHECK(hipStreamSynchronize(s));
  bool all = true;
  for (size_t k = 0; k < B; ++k)
    all = all && W->rnorm_host[2 * k] <= W->tol2_host * W->rnorm_host[2 * k + 1];
  *conv = all;
  return DL_OK;
}

// Refine mu (the solve of the workspace's right-hand sides) with at most
// max_steps corrections, stopping once every instance meets tol (the host
// reads the norms after each residual); then the final residual of mu.
// *conv (may be null) receives whether every final residual meets tol
// (read only when max_steps > 0).
static dl_status refine_eager(dl_ws* W, hipStream_t s, int max_steps, double tol, bool* conv) {
  dl_status st = set_refine_tol(W, tol, s);
  if (st != DL_OK) return st;
  if (max_steps <= 0) {
    DL_HIP_CHECK(run(W, W->resid_p, s));
    if (conv) *conv = true;
    return DL_OK;
  }
  DL_HIP_CHECK(run(W, W->ref_init_p, s));
  for (int r = 0; r < max_steps; ++r) {
    DL_HIP_CHECK(run(W, W->ref_res_p, s));
    bool all = false;
    if ((st = refine_all_converged(W, s, &all)) != DL_OK) return st;
    if (all) break;
    DL_HIP_CHECK(run(W, W->ref_corr_p, s));
  }
  DL_HIP_CHECK(run(W, W->ref_fin_p, s));
  if (conv) {
    bool all = false;
    if ((st = refine_all_converged(W, s, &all)) != DL_OK) return st;
    *conv = all;
  }
  return DL_OK;
}

extern "C" dl_status bta_assemble(dl_ws* W, const double* theta_dev,
                                  dl_which which, void* stream) {
  if (!W || !theta_dev || which < DL_QP || which > DL_BOTH) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  dl_status st = copy_theta_in(W, theta_dev, (int)W->inst.size(), s);
  if (st != DL_OK) return st;
  DL_HIP_CHECK(run(W, W->asm_p[which], s));
  if (which != DL_QC) { W->assembled[0] = true; W->factored[0] = false; }
  if (which != DL_QP) { W->assembled[1] = true; W->factored[1] = false; }
  W->solved = false;
  return DL_OK;
}

extern "C" dl_status bta_factor(dl_ws* W, dl_which which, double* logdet_dev,
                                int64_t* info_dev, void* stream) {
  if (!W || which < DL_QP || which > DL_BOTH) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int w0 = which == DL_QC ? 1 : 0;
  const int w1 = which == DL_QP ? 0 : 1;
  for (int w = w0; w <= w1; ++w)
    if (!W->assembled[w]) return DL_ESTATE;
  DL_HIP_CHECK(run(W, W->fac_p[which], s));
  for (int w = w0; w <= w1; ++w) {
    W->assembled[w] = false;
    W->factored[w] = true;
  }
  const int cnt = w1 - w0 + 1;
  for (size_t k = 0; k < W->inst.size(); ++k) {
    Inst& I = W->inst[k];
    if (logdet_dev)
      DL_HIP_CHECK(hipMemcpyAsync(logdet_dev + cnt * k, I.logdet2 + w0,
                                  cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (info_dev)
      DL_HIP_CHECK(hipMemcpyAsync(info_dev + cnt * k, I.info2 + w0,
                                  cnt * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  }
  return DL_OK;
}

extern "C" dl_status bta_solve(dl_ws* W, double* rhs_inout_dev, int32_t nrhs,
                               int32_t refine_max, double refine_tol, void* stream) {
  if (!W) return DL_EINVAL;
  if (rhs_inout_dev ? nrhs < 1 : (nrhs != 0 && nrhs != 1)) return DL_EINVAL;
  if (refine_max > 100 || (refine_max >= 0 && !(refine_tol >= 0.0))) return DL_EINVAL;
  if (!W->factored[1]) return DL_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  // refine_max < 0: the workspace's default (mixed precision: to
  // DL_REFINE_TOL in at most DL_REFINE_MAX corrections; FP64: none)
  const int steps = refine_max < 0 ? (W->mixed ? DL_REFINE_MAX : 0) : refine_max;
  const double tol = refine_max < 0 ? DL_REFINE_TOL : refine_tol;
  bool all = true;
  dl_status st = DL_OK;
  if (!rhs_inout_dev) {
    DL_HIP_CHECK(run(W, W->solve_p, s));
    bool conv = true;
    if ((st = refine_eager(W, s, steps, tol, &conv)) != DL_OK) return st;
    all = conv;
  } else {
    int64_t ntot = 0;
    for (auto& I : W->inst) ntot += I.m.N;
    for (int c = 0; c < nrhs; ++c) {
      double* col = rhs_inout_dev + (int64_t)c * ntot;
      // the plan copies rhs -> x first, so stage the caller's vectors in rhs
      int64_t off = 0;
      for (auto& I : W->inst) {
        DL_HIP_CHECK(launch_unpack(I.m, col + off, I.rhs, s));
        off += I.m.N;
      }
      DL_HIP_CHECK(run(W, W->solve_p, s));
      bool conv = true;
      if (steps > 0 && (st = refine_eager(W, s, steps, tol, &conv)) != DL_OK) return st;
      all = all && conv;
      off = 0;
      for (auto& I : W->inst) {
        DL_HIP_CHECK(launch_pack(I.m, I.mu, col + off, s));
        off += I.m.N;
      }
    }
  }
  // evaluations after this call use the default tolerance again
  if ((st = set_refine_tol(W, DL_REFINE_TOL, s)) != DL_OK) return st;
  W->solved = true;
  return all ? DL_OK : DL_ENOTCONV;
}

extern "C" dl_status bta_selinv(dl_ws* W, double* diag_out_dev, void* stream) {
  if (!W || !diag_out_dev) return DL_EINVAL;
  if (!W->sel || !W->factored[1]) return DL_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  DL_HIP_CHECK(run(W, W->selinv_p, s));
  int64_t off = 0;
  for (auto& I : W->inst) {
    DL_HIP_CHECK(launch_pack(I.m, I.selout, diag_out_dev + off, s));
    off += I.m.N;
  }
  return DL_OK;
}

extern "C" dl_status dl_ws_mean(dl_ws* W, double* out_dev, void* stream) {
  if (!W || !out_dev) return DL_EINVAL;
  if (!W->solved) return DL_ESTATE;
  int64_t off = 0;
  for (auto& I : W->inst) {
    DL_HIP_CHECK(launch_pack(I.m, I.mu, out_dev + off, (hipStream_t)stream));
    off += I.m.N;
  }
  return DL_OK;
}

// ---- inner mode of a Poisson likelihood (Laplace approximation) ------------------
//
// Damped Newton for the mode x* of h(x) = log l(y | A x) - 1/2 x^T Q_p x
// from x = 0 (or, with DL_WS_WARM_START, from the instance's previous mode),
// for the first nk instances (the rest stay idle): each step
// assembles Q_c(x) = Q_p + A^T D(x) A and A^T (g + D A x) from the weights
// of the current iterate, factors and solves (x_N), and tries
// x + alpha (x_N - x) for alpha = 1, 1/2, ... until h does not fall (up to
// rounding); h comes from the quadratic-form kernels at the trial point.
// A converged or failed instance keeps its iterate (alpha = 0) while the
// others continue.  Then Q_c(x*) is assembled and factored and Eq. 8 is
// evaluated at mu = x*.
static dl_status eval_trials(dl_ws* W, const std::vector<double>& alpha,
                             std::vector<double>& out, hipStream_t s) {
  const int B = (int)W->inst.size();
  DL_HIP_CHECK(hipMemcpyAsync(W->alpha_all, alpha.data(), sizeof(double) * B,
                              hipMemcpyHostToDevice, s));
  DL_HIP_CHECK(launch_trial(W->d_trial, B, s));
  DL_HIP_CHECK(launch_quadforms(W->d_nquad, B, s));
  DL_HIP_CHECK(launch_trial_gather(W->d_trial, B, s));
  DL_HIP_CHECK(hipMemcpyAsync(out.data(), W->out4_all, sizeof(double) * 4 * B,
                              hipMemcpyDeviceToHost, s));
  DL_HIP_CHECK(hipStreamSynchronize(s));
  return DL_OK;
}

static dl_status laplace_pass(dl_ws* W, int nk, hipStream_t s) {
  const int B = (int)W->inst.size();
  for (int k = 0; k < B; ++k) {
    Inst& I = W->inst[k];
    if (!(W->warm && W->has_mode[k] && k < nk))
      DL_HIP_CHECK(hipMemsetAsync(I.xcur, 0, sizeof(double) * I.m.Np, s));
    DL_HIP_CHECK(hipMemsetAsync(I.xN, 0, sizeof(double) * I.m.Np, s));
  }
  // Q_p and the first step's Q_c(x0) share their launches
  DL_HIP_CHECK(launch_lap_weights(W->d_lap, B, s));
  DL_HIP_CHECK(run(W, W->asm_p[2], s));
  DL_HIP_CHECK(run(W, W->fac_p[2], s));
  // state: 0 iterating, 1 converged, -1 failed, 2 idle (k >= nk)
  std::vector<int> state(B, 0), steps(B, 0), nh(B, 0);
  std::vector<double> alpha(B, 0.0), out(4 * B, 0.0), hcur(B, 0.0);
  for (int k = nk; k < B; ++k) state[k] = 2;
  dl_status st = eval_trials(W, alpha, out, s);  // h at the start
  if (st != DL_OK) return st;
  for (int k = 0; k < B; ++k) hcur[k] = -0.5 * (out[4 * k + 2] + out[4 * k + 3]);
  auto h_of = [&](int k) { return -0.5 * (out[4 * k + 2] + out[4 * k + 3]); };
  for (int it = 0; it < DL_NEWTON_MAX; ++it) {
    bool any = false;
    for (int k = 0; k < B; ++k) any = any || state[k] == 0;
    if (!any) break;
    if (it > 0) {
      DL_HIP_CHECK(launch_lap_weights(W->d_lap, B, s));
      DL_HIP_CHECK(run(W, W->asm_p[1], s));
      DL_HIP_CHECK(run(W, W->fac_p[1], s));
    }
    DL_HIP_CHECK(run(W, W->solve_p, s));
    // mixed precision: refine x_N in FP64 against the sparse Q_c(x)
    if (W->mixed) {
      if ((st = refine_eager(W, s, DL_REFINE_MAX, DL_REFINE_TOL, nullptr)) != DL_OK) return st;
    }
    for (auto& I : W->inst)
      DL_HIP_CHECK(hipMemcpyAsync(I.xN, I.mu, sizeof(double) * I.m.Np,
                                  hipMemcpyDeviceToDevice, s));
    std::vector<int> live(B, 0);
    for (int k = 0; k < B; ++k) {
      live[k] = state[k] == 0;
      alpha[k] = live[k] ? 1.0 : 0.0;
      nh[k] = 0;
    }
    for (;;) {
      if ((st = eval_trials(W, alpha, out, s)) != DL_OK) return st;
      bool pending = false;
      for (int k = 0; k < B; ++k) {
        if (!live[k] || state[k] != 0) continue;
        const double ht = h_of(k);
        if (std::isfinite(ht) && ht >= hcur[k] - DL_ASCENT_SLACK * (1.0 + std::fabs(hcur[k])))
          continue;  // accepted at this alpha
        if (nh[k] == DL_NEWTON_HALVINGS) {
          state[k] = -1;
          alpha[k] = 0.0;
        } else {
          alpha[k] *= 0.5;
          ++nh[k];
          pending = true;
        }
      }
      if (!pending) break;
    }
    // the last trial holds every live instance's accepted point (failed ones
    // are discarded below); converged and idle ones kept x (alpha = 0)
    for (int k = 0; k < B; ++k) {
      if (!live[k] || state[k] != 0) continue;
      ++steps[k];
      hcur[k] = h_of(k);
      Inst& I = W->inst[k];
      DL_HIP_CHECK(hipMemcpyAsync(I.xcur, I.mu, sizeof(double) * I.m.Np,
                                  hipMemcpyDeviceToDevice, s));
      if (nh[k] == 0 && out[4 * k] <= DL_NEWTON_TOL * (1.0 + out[4 * k + 1])) state[k] = 1;
    }
  }
  for (int k = 0; k < B; ++k)
    if (state[k] == 0) state[k] = -1;
  // Q_c and its factor at the mode, then Eq. 8 at mu = x*
  DL_HIP_CHECK(launch_lap_weights(W->d_lap, B, s));
  DL_HIP_CHECK(run(W, W->asm_p[1], s));
  DL_HIP_CHECK(run(W, W->fac_p[1], s));
  for (auto& I : W->inst)
    DL_HIP_CHECK(hipMemcpyAsync(I.mu, I.xcur, sizeof(double) * I.m.Np,
                                hipMemcpyDeviceToDevice, s));
  if ((st = refine_eager(W, s, W->mixed ? DL_REFINE_MAX : 0, DL_REFINE_TOL, nullptr)) != DL_OK)
    return st;
  static const double kBad = 1.0;
  for (int k = 0; k < B; ++k) {
    if (state[k] == -1)
      DL_HIP_CHECK(hipMemcpyAsync(W->inst[k].coef + C_BAD, &kBad, sizeof(double),
                                  hipMemcpyHostToDevice, s));
    W->newton_steps[k] = state[k] == 1 ? steps[k] : (state[k] == 2 ? 0 : -1);
    if (state[k] != 2) W->has_mode[k] = state[k] == 1;
  }
  DL_HIP_CHECK(run(W, W->post_p, s));
  return DL_OK;
}

extern "C" dl_status dl_ws_newton_steps(const dl_ws* W, int32_t* steps_host) {
  if (!W || !steps_host) return DL_EINVAL;
  for (size_t k = 0; k < W->inst.size(); ++k) steps_host[k] = W->newton_steps[k];
  return DL_OK;
}

static dl_status run_eval(dl_ws* W, hipStream_t s) {
  dl_status st = set_refine_tol(W, DL_REFINE_TOL, s);
  if (st != DL_OK) return st;
  if (!W->use_graph) {
    DL_HIP_CHECK(run(W, W->asm_p[2], s));
    DL_HIP_CHECK(run(W, W->fac_p[2], s));
    DL_HIP_CHECK(run(W, W->solve_p, s));
    if ((st = refine_eager(W, s, W->mixed ? DL_REFINE_MAX : 0, DL_REFINE_TOL, nullptr)) !=
        DL_OK)
      return st;
    DL_HIP_CHECK(run(W, W->post_p, s));
    return DL_OK;
  }
  if (!W->graph_exec) {
    // capture the whole evaluation on a private stream once; the captured
    // launches read theta from and write results to the workspace buffers
    if (!W->cap_stream)
      DL_HIP_CHECK(hipStreamCreateWithFlags(&W->cap_stream, hipStreamNonBlocking));
    DL_HIP_CHECK(hipStreamBeginCapture(W->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = run(W, W->eval_p, W->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(W->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return DL_EHIP;
    }
    W->graph = g;
    DL_HIP_CHECK(hipGraphInstantiate(&W->graph_exec, g, nullptr, nullptr, 0));
  }
  DL_HIP_CHECK(hipGraphLaunch(W->graph_exec, s));
  return DL_OK;
}

extern "C" dl_status fobj_eval(dl_ws* W, const double* theta_dev, int32_t ntheta,
                               double* fobj_dev, dl_fobj_parts* parts_dev,
                               int64_t* info_dev, void* stream) {
  if (!W || !theta_dev || ntheta < 0 || (!fobj_dev && !parts_dev)) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)W->inst.size();
  // instances of different models take exactly one theta each
  bool uniform = true;
  for (auto& I : W->inst)
    if (I.model != W->inst[0].model) uniform = false;
  if (!uniform && ntheta != B) return DL_EINVAL;
  const int dim = W->inst[0].dim;
  for (int k0 = 0; k0 < ntheta; k0 += B) {
    const int nk = std::min(B, ntheta - k0);
    dl_status st = copy_theta_in(W, theta_dev + (int64_t)k0 * dim, nk, s);
    if (st != DL_OK) return st;
    st = W->poisson ? laplace_pass(W, nk, s) : run_eval(W, s);
    if (st != DL_OK) return st;
    if (fobj_dev)
      DL_HIP_CHECK(hipMemcpyAsync(fobj_dev + k0, W->f_all, sizeof(double) * nk,
                                  hipMemcpyDeviceToDevice, s));
    if (parts_dev)
      DL_HIP_CHECK(hipMemcpyAsync(parts_dev + k0, W->parts_all,
                                  sizeof(dl_fobj_parts) * nk,
                                  hipMemcpyDeviceToDevice, s));
    if (info_dev)
      DL_HIP_CHECK(hipMemcpyAsync(info_dev + 2 * (int64_t)k0, W->info_all,
                                  sizeof(int64_t) * 2 * nk, hipMemcpyDeviceToDevice, s));
  }
  W->assembled[0] = W->assembled[1] = false;
  W->factored[0] = W->factored[1] = true;
  W->solved = true;
  return DL_OK;
}

// f_obj and the selected inversion of one batch of thetas: after the two
// factorisations the solve, refinement and quadratic forms run on a second
// stream while the selected inversion runs on the caller's stream (they read
// the factor and write disjoint buffers); the caller's stream then waits for
// both.  Results are those of fobj_eval followed by bta_selinv.
extern "C" dl_status fobj_selinv_eval(dl_ws* W, const double* theta_dev, int32_t ntheta,
                                      double* fobj_dev, dl_fobj_parts* parts_dev,
                                      int64_t* info_dev, double* diag_out_dev,
                                      void* stream) {
  if (!W || !theta_dev || !diag_out_dev || (!fobj_dev && !parts_dev)) return DL_EINVAL;
  if (!W->sel) return DL_ESTATE;
  const int B = (int)W->inst.size();
  bool uniform = true;
  for (auto& I : W->inst)
    if (I.model != W->inst[0].model) uniform = false;
  if (ntheta < 1 || ntheta > B || (!uniform && ntheta != B)) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!W->aux_stream)
    DL_HIP_CHECK(hipStreamCreateWithFlags(&W->aux_stream, hipStreamNonBlocking));
  if (!W->ev_fork) DL_HIP_CHECK(hipEventCreateWithFlags(&W->ev_fork, hipEventDisableTiming));
  if (!W->ev_join) DL_HIP_CHECK(hipEventCreateWithFlags(&W->ev_join, hipEventDisableTiming));
  dl_status st = copy_theta_in(W, theta_dev, ntheta, s);
  if (st != DL_OK) return st;
  if (W->poisson) {
    // the mode search ends with the factor of Q_c(x*) and Eq. 8 evaluated
    if ((st = laplace_pass(W, ntheta, s)) != DL_OK) return st;
    DL_HIP_CHECK(hipEventRecord(W->ev_join, s));
  } else {
    if ((st = set_refine_tol(W, DL_REFINE_TOL, s)) != DL_OK) return st;
    DL_HIP_CHECK(run(W, W->asm_p[2], s));
    DL_HIP_CHECK(run(W, W->fac_p[2], s));
    DL_HIP_CHECK(hipEventRecord(W->ev_fork, s));
    DL_HIP_CHECK(hipStreamWaitEvent(W->aux_stream, W->ev_fork, 0));
  }
  // the selected inversion is enqueued before the solve side, whose
  // refinement may wait on the host for its residual norms
  DL_HIP_CHECK(run(W, W->selinv_p, s));
  int64_t off = 0;
  for (auto& I : W->inst) {
    DL_HIP_CHECK(launch_pack(I.m, I.selout, diag_out_dev + off, s));
    off += I.m.N;
  }
  if (!W->poisson) {
    DL_HIP_CHECK(run(W, W->solve_p, W->aux_stream));
    st = refine_eager(W, W->aux_stream, W->mixed ? DL_REFINE_MAX : 0, DL_REFINE_TOL, nullptr);
    if (st != DL_OK) return st;
    DL_HIP_CHECK(run(W, W->post_p, W->aux_stream));
    DL_HIP_CHECK(hipEventRecord(W->ev_join, W->aux_stream));
  }
  DL_HIP_CHECK(hipStreamWaitEvent(s, W->ev_join, 0));
  if (fobj_dev)
    DL_HIP_CHECK(hipMemcpyAsync(fobj_dev, W->f_all, sizeof(double) * ntheta,
                                hipMemcpyDeviceToDevice, s));
  if (parts_dev)
    DL_HIP_CHECK(hipMemcpyAsync(parts_dev, W->parts_all, sizeof(dl_fobj_parts) * ntheta,
                                hipMemcpyDeviceToDevice, s));
  if (info_dev)
    DL_HIP_CHECK(hipMemcpyAsync(info_dev, W->info_all, sizeof(int64_t) * 2 * ntheta,
                                hipMemcpyDeviceToDevice, s));
  W->assembled[0] = W->assembled[1] = false;
  W->factored[0] = W->factored[1] = true;
  W->solved = true;
  return DL_OK;
}

// Descriptor of one block copy between the workspace and a caller buffer
// (column-major, unpadded): to_ws = false reads the block into `user`,
// true writes `user` into the block.  kind 0 = D_t, 1 = B_t (rows t+1,
// cols t), 2 = R_t, 3 = tip.
static dl_status block_job(dl_ws* W, dl_which which, int32_t kind, int32_t t, bool to_ws,
                           double* user, MiscJob* J) {
  Inst& I = W->inst[0];
  const ModelDev& m = I.m;
  const int bp = m.bp;
  const bool p = which == DL_QP;
  if (p && I.qp_ring) return DL_ESTATE;
  double* ws = nullptr;
  int64_t ldw = 0;
  int rows = 0, cols = 0;
  bool f32 = false;
  if (kind == 3) {
    if (m.a == 0) return DL_EINVAL;
    ws = p ? I.Pp : I.Pc; ldw = m.ap; rows = m.a; cols = m.a;
  } else {
    if (t < 0 || t >= m.nt) return DL_EINVAL;
    const bool fact = W->factored[p ? 0 : 1];
    const int sl = (!p && fact) ? I.slot_final[t] : t;
    const int64_t ldbr = p ? bp : I.ldbr;
    double* BRt = eoff(p ? I.Bp : I.BRc, (int64_t)sl * ldbr * bp, I.eb);
    if (kind == 0) {
      ws = (p ? I.Dp : I.Dc) + (int64_t)t * bp * bp; ldw = bp; rows = m.b; cols = m.b;
    } else if (kind == 1) {
      if (t + 1 >= m.nt) return DL_EINVAL;
      ws = BRt; ldw = ldbr; rows = m.b; cols = m.b; f32 = I.mixed;
    } else if (kind == 2) {
      if (p || m.a == 0) return DL_EINVAL;
      ws = eoff((void*)BRt, bp, I.eb); ldw = ldbr; rows = m.a; cols = m.b; f32 = I.mixed;
    } else {
      return DL_EINVAL;
    }
  }
  *J = MiscJob{};
  J->rows = rows;
  J->cols = cols;
  if (to_ws) {
    J->kind = f32 ? MJ_COPY2D_TO_F32 : MJ_COPY2D;
    J->dst = ws; J->ldd = ldw; J->src = user; J->lds = rows;
  } else {
    J->kind = f32 ? MJ_COPY2D_F32 : MJ_COPY2D;
    J->dst = user; J->ldd = rows; J->src = ws; J->lds = ldw;
  }
  return DL_OK;
}

// One block copy through the workspace's descriptor slot (synchronous).
static dl_status block_copy(dl_ws* W, const MiscJob& J, hipStream_t s) {
  DL_HIP_CHECK(hipMemcpyAsync(W->d_io, &J, sizeof(MiscJob), hipMemcpyHostToDevice, s));
  DL_HIP_CHECK(launch_misc(W->d_io, 1, s));
  DL_HIP_CHECK(hipStreamSynchronize(s));
  return DL_OK;
}

extern "C" dl_status dl_ws_get_block(dl_ws* W, dl_which which, int32_t kind,
                                     int32_t t, double* out_dev, void* stream) {
  if (!W || !out_dev || (which != DL_QP && which != DL_QC)) return DL_EINVAL;
  if (W->inst.size() != 1) return DL_EINVAL;
  Inst& I = W->inst[0];
  hipStream_t s = (hipStream_t)stream;
  if (kind == 4) {
    if (which == DL_QP) return DL_EINVAL;
    DL_HIP_CHECK(launch_pack(I.m, I.rhs, out_dev, s));
    return DL_OK;
  }
  MiscJob J;
  const dl_status st = block_job(W, which, kind, t, false, out_dev, &J);
  if (st != DL_OK) return st;
  return block_copy(W, J, s);
}

extern "C" dl_status dl_ws_set_block(dl_ws* W, dl_which which, int32_t kind, int32_t t,
                                     const double* in_dev, void* stream) {
  if (!W || !in_dev || (which != DL_QP && which != DL_QC)) return DL_EINVAL;
  if (W->inst.size() != 1) return DL_EINVAL;
  const int w = which == DL_QP ? 0 : 1;
  if (!W->assembled[w]) return DL_ESTATE;
  Inst& I = W->inst[0];
  hipStream_t s = (hipStream_t)stream;
  if (kind == 4) {
    if (which == DL_QP) return DL_EINVAL;
    DL_HIP_CHECK(launch_unpack(I.m, in_dev, I.rhs, s));
    DL_HIP_CHECK(hipStreamSynchronize(s));
    return DL_OK;
  }
  MiscJob J;
  const dl_status st = block_job(W, which, kind, t, true, const_cast<double*>(in_dev), &J);
  if (st != DL_OK) return st;
  return block_copy(W, J, s);
}

// ---- profiling ----------------------------------------------------------------------------

static void prof_free(dl_ws* W) {
  for (hipEvent_t e : W->prof_ev) (void)hipEventDestroy(e);
  W->prof_ev.clear();
  W->prof_cat.clear();
  W->prof_flops.clear();
  W->prof_bytes.clear();
  W->prof_used = 0;
  W->prof_mask = 0;
}

extern "C" dl_status dl_ws_profile_begin(dl_ws* W, int32_t mask, int32_t max_launches) {
  if (!W || max_launches <= 0 || (mask & 0xffff) == 0) return DL_EINVAL;
  if (W->use_graph) return DL_ESTATE;
  prof_free(W);
  W->prof_by_kernel = (mask & DL_PROFILE_BY_KERNEL) ? 1 : 0;
  W->prof_ev.resize(2 * (size_t)max_launches, nullptr);
  for (auto& e : W->prof_ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      prof_free(W);
      return DL_EHIP;
    }
  W->prof_cat.assign(max_launches, 0);
  W->prof_flops.assign(max_launches, 0.0);
  W->prof_bytes.assign(max_launches, 0.0);
  W->prof_mask = mask & 0xffff;
  W->prof_paused = 0;
  return DL_OK;
}

extern "C" dl_status dl_ws_profile_enable(dl_ws* W, int32_t on) {
  if (!W) return DL_EINVAL;
  W->prof_paused = on ? 0 : 1;
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
    if (hipEventElapsedTime(&t, W->prof_ev[2 * k], W->prof_ev[2 * k + 1]) != hipSuccess) {
      st = DL_EHIP;
      break;
    }
    const int c = W->prof_cat[k];
    if (ms) ms[c] += t;
    if (launches) launches[c] += 1;
    if (flops) flops[c] += W->prof_flops[k];
    if (bytes) bytes[c] += W->prof_bytes[k];
  }
  prof_free(W);
  return st;
}

// ---- tile autotuner --------------------------------------------------------------------
//
// Every GEMM launch of the workspace's plans has a signature (category,
// number of tasks, shape and flags of its tasks).  For each signature both
// tile variants (64x64, 128x128) are timed in isolation with HIP events (the
// launch reads and writes the workspace's own buffers; their contents are
// rebuilt by the next assembly) and the faster one is kept for every launch
// of that signature.  Choices are cached in a text file, one line per
// signature, so later workspaces of the same shapes skip the measurement.
#include <fstream>
#include <sstream>
#include <string>
#include <unordered_map>

static std::string gemm_signature(const dl_ws* W, const Launch& L) {
  std::ostringstream o;
  o << "gfx950 " << (L.kind == OP_GEMM32 ? "gemm32" : "gemm") << " cat" << L.cat
    << " n" << L.count;
  for (int i = 0; i < L.count && i < 8; ++i) {
    const GemmTask& t = W->H.gemm[L.off + i];
    o << " " << t.M << "x" << t.N << "x" << t.K << "f" << (t.flags & ~(F_BETA0 | F_SPLIT));
  }
  return o.str();
}

// Tile size and split k of one matrix-product launch (split applies to the
// FP64 kernel only).
static dl_status retile(dl_ws* W, Launch& L, int tile, bool split, hipStream_t s,
                        int ksplit = GEMM_KSPLIT) {
  GemmTask* t = W->H.gemm.data() + L.off;
  if (L.kind == OP_GEMM)
    for (int i = 0; i < L.count; ++i) {
      t[i].flags = split ? (t[i].flags | F_SPLIT) : (t[i].flags & ~F_SPLIT);
      t[i].ksplit = ksplit;
    }
  int64_t slots = 0;
  L.tile = tile;
  L.gx = finalize_tasks(t, L.count, tile, &L.nred, &slots);
  if (slots > 0) {
    const dl_status st = ensure_partials(W, slots * tile * tile, s);
    if (st != DL_OK) return st;
  }
  DL_HIP_CHECK(hipMemcpy(W->Dd.gemm + L.off, t, sizeof(GemmTask) * L.count,
                         hipMemcpyHostToDevice));
  return DL_OK;
}

static bool launch_split(const dl_ws* W, const Launch& L) {
  return L.kind == OP_GEMM && L.count > 0 && (W->H.gemm[L.off].flags & F_SPLIT);
}

static int launch_ksplit(const dl_ws* W, const Launch& L) {
  return (L.kind == OP_GEMM && L.count > 0 && W->H.gemm[L.off].ksplit > 0)
             ? W->H.gemm[L.off].ksplit
             : GEMM_KSPLIT;
}

// Device memory the autotuner may add for split-k partial tiles (doubles):
// choices needing more are not tried.
constexpr int64_t kSplitBudgetDoubles = (int64_t)4 << 27;  // 4 GiB

// One tuned choice of a matrix-product launch.
struct TileChoice {
  int tile = 64;
  bool split = false;
  int ksplit = GEMM_KSPLIT;
};

extern "C" dl_status dl_autotune(dl_ws* W, const char* cache_path, void* stream) {
  if (!W) return DL_EINVAL;
  if (W->graph_exec) return DL_ESTATE;  // tune before the first graph capture
  hipStream_t s = (hipStream_t)stream;
  // cache lines: "<signature> <tile>", "<signature> <tile>s" (split k in
  // pieces of 512) or "<signature> <tile>s<piece>"
  std::unordered_map<std::string, TileChoice> best;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t sp = line.rfind(' ');
      if (sp == std::string::npos || sp + 1 >= line.size()) continue;
      const std::string v = line.substr(sp + 1);
      TileChoice c;
      c.tile = atoi(v.c_str());
      const size_t sx = v.find('s');
      if (sx != std::string::npos) {
        c.split = true;
        if (sx + 1 < v.size()) c.ksplit = atoi(v.c_str() + sx + 1);
      }
      if ((c.tile != 64 && c.tile != 128) || c.ksplit < 16 || c.ksplit % 16) continue;
      best[line.substr(0, sp)] = c;
    }
  }
  std::vector<std::string> fresh;
  hipEvent_t e0, e1;
  DL_HIP_CHECK(hipEventCreate(&e0));
  DL_HIP_CHECK(hipEventCreate(&e1));
  dl_status st = DL_OK;
  for (Launch& L : W->table) {
    if ((L.kind != OP_GEMM && L.kind != OP_GEMM32) || st != DL_OK) continue;
    const std::string sig = gemm_signature(W, L);
    auto it = best.find(sig);
    if (it == best.end()) {
      // candidates: both tiles, unsplit and (FP64 products with a k extent
      // above a piece length) split into pieces of 512 or 256
      int kmax = 0;
      if (L.kind == OP_GEMM)
        for (int i = 0; i < L.count; ++i) kmax = std::max(kmax, W->H.gemm[L.off + i].K);
      std::vector<TileChoice> cand;
      for (int tile : {64, 128}) {
        cand.push_back({tile, false, GEMM_KSPLIT});
        for (int ks : {512, 256}) {
          if (kmax <= ks) continue;
          // partial tiles of this choice: skipped above the budget
          std::vector<GemmTask> tmp(W->H.gemm.begin() + L.off,
                                    W->H.gemm.begin() + L.off + L.count);
          for (auto& t : tmp) {
            t.flags |= F_SPLIT;
            t.ksplit = ks;
          }
          int64_t slots = 0;
          (void)finalize_tasks(tmp.data(), L.count, tile, nullptr, &slots);
          if (slots * tile * tile <= kSplitBudgetDoubles || slots * tile * tile <= W->partials_cap)
            cand.push_back({tile, true, ks});
        }
      }
      float tbest = 1e30f;
      TileChoice choice;
      for (const TileChoice& c : cand) {
        if ((st = retile(W, L, c.tile, c.split, s, c.ksplit)) != DL_OK) break;
        float tmin = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          (void)hipEventRecord(e0, s);
          (void)run_launch(W, L, s);
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          tmin = std::min(tmin, ms);
        }
        if (tmin < tbest) {
          tbest = tmin;
          choice = c;
        }
      }
      it = best.emplace(sig, choice).first;
      fresh.push_back(sig);
    }
    const TileChoice& c = it->second;
    if (st == DL_OK && (L.tile != c.tile || launch_split(W, L) != c.split ||
                        (c.split && launch_ksplit(W, L) != c.ksplit)))
      st = retile(W, L, c.tile, c.split, s, c.ksplit);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == DL_OK && cache_path && !fresh.empty()) {
    std::ofstream out(cache_path, std::ios::app);
    for (const auto& sig : fresh) {
      const TileChoice& c = best[sig];
      out << sig << " " << c.tile;
      if (c.split) out << "s" << (c.ksplit == GEMM_KSPLIT ? std::string() : std::to_string(c.ksplit));
      out << "\n";
    }
  }
  return st;
}

extern "C" dl_status dl_ws_force_tile(dl_ws* W, int32_t tile) {
  if (!W || (tile != 64 && tile != 128)) return DL_EINVAL;
  if (W->graph_exec) return DL_ESTATE;
  for (Launch& L : W->table) {
    if (L.kind != OP_GEMM && L.kind != OP_GEMM32) continue;
    const dl_status st = retile(W, L, tile, launch_split(W, L), nullptr, launch_ksplit(W, L));
    if (st != DL_OK) return st;
  }
  return DL_OK;
}

extern "C" dl_status dl_ws_force_split(dl_ws* W, int32_t ksplit) {
  if (!W || ksplit < 0 || (ksplit > 0 && (ksplit < 64 || ksplit % 16))) return DL_EINVAL;
  if (W->graph_exec) return DL_ESTATE;
  for (Launch& L : W->table) {
    if (L.kind != OP_GEMM) continue;
    const dl_status st =
        retile(W, L, L.tile, ksplit > 0, nullptr, ksplit > 0 ? ksplit : GEMM_KSPLIT);
    if (st != DL_OK) return st;
  }
  return DL_OK;
}

// Number of GEMM launches of the workspace using each tile size.
extern "C" dl_status dl_ws_tile_counts(const dl_ws* W, int64_t* n64, int64_t* n128) {
  if (!W) return DL_EINVAL;
  int64_t a = 0, b = 0;
  for (const Launch& L : W->table)
    if (L.kind == OP_GEMM || L.kind == OP_GEMM32) (L.tile == 128 ? b : a)++;
  if (n64) *n64 = a;
  if (n128) *n128 = b;
  return DL_OK;
}
