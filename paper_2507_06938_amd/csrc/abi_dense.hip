// Dense FP64 building blocks exposed through the C ABI for testing: they run
// the same kernels as the BTA path on caller-provided matrices.  Each call
// copies its few descriptors to the device and synchronises the stream.
#include <functional>
#include <vector>

#include "engine.hpp"

using namespace dl;

static GemmTask mk_task(const double* A, int64_t lda, const double* B, int64_t ldb,
                        double* C, int64_t ldc, int M, int N, int K, int flags,
                        double alpha, double beta) {
  GemmTask t{};
  t.A = A; t.B = B; t.C = C;
  t.lda = lda; t.ldb = ldb; t.ldc = ldc;
  t.M = M; t.N = N; t.K = K; t.flags = flags;
  t.alpha = alpha; t.beta = beta;
  return t;
}

template <typename T>
static hipError_t to_dev(std::vector<void*>& tmp, const std::vector<T>& h, T** d,
                         hipStream_t s) {
  void* p = nullptr;
  if (dev_alloc(tmp, sizeof(T) * (h.size() + 1), &p) != DL_OK) return hipErrorOutOfMemory;
  *d = (T*)p;
  if (h.empty()) return hipSuccess;
  return hipMemcpyAsync(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s);
}

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
  std::vector<GemmTask> t{mk_task(A, lda, B, ldb, C, ldc, (int)M, (int)Nn, (int)K,
                                  flags, alpha, beta)};
  const int total = finalize_tasks(t.data(), 1);
  if (total == 0) return DL_OK;
  std::vector<void*> tmp;
  GemmTask* d = nullptr;
  hipError_t e = to_dev(tmp, t, &d, s);
  if (e == hipSuccess) e = launch_gemm_tasks(d, 1, total, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  free_all(tmp);
  return e == hipSuccess ? DL_OK : DL_EHIP;
}

// Right-looking blocked Cholesky (64-column panels) with the same kernels as
// the BTA diagonal blocks; with want_inverse the diagonal tiles keep their
// inverses and a recursive inversion completes L^{-1}.
extern "C" dl_status dl_dpotrf(int64_t n, double* A, int64_t lda,
                               int32_t want_inverse, double* logdet_dev,
                               int64_t* info_dev, void* stream) {
  if (n <= 0 || n % 64 != 0 || n > (1 << 20) || !A || lda < n || !logdet_dev ||
      !info_dev)
    return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nbk = (int)(n / 64);
  std::vector<void*> tmp;
  double *Gd = nullptr, *temp = nullptr, *logdiag = nullptr, *part = nullptr;
  if (dev_alloc(tmp, sizeof(double) * n * 64, (void**)&Gd) != DL_OK ||
      dev_alloc(tmp, sizeof(double) * n * (nbk / 2 + 1) * 64, (void**)&temp) != DL_OK ||
      dev_alloc(tmp, sizeof(double) * n, (void**)&logdiag) != DL_OK ||
      dev_alloc(tmp, sizeof(double) * SUM_BLOCKS, (void**)&part) != DL_OK) {
    free_all(tmp);
    return DL_ENOMEM;
  }
  std::vector<MiscJob> pre(2);
  pre[0].kind = MJ_ZERO_I64; pre[0].dst = (double*)info_dev; pre[0].n = 1;
  pre[1].kind = MJ_ZERO_UPPER_TILES; pre[1].dst = A; pre[1].rows = (int)n; pre[1].ldd = lda;
  std::vector<PotrfTileArgs> pt(nbk);
  std::vector<GemmTask> tasks;
  std::vector<int> t_off, t_cnt, t_tiles;
  auto push_tasks = [&](std::vector<GemmTask> ts) {
    const int o = (int)tasks.size();
    const int tiles = finalize_tasks(ts.data(), (int)ts.size());
    tasks.insert(tasks.end(), ts.begin(), ts.end());
    t_off.push_back(o);
    t_cnt.push_back((int)ts.size());
    t_tiles.push_back(tiles);
  };
  // mode 0 (A <- L, inverse of the tile to Gd) without the inverse; mode 1
  // (inverse in place) when the full inverse is wanted
  const int mode = want_inverse ? 1 : 0;
  for (int j = 0; j < nbk; ++j) {
    PotrfTileArgs& a = pt[j];
    a.A = A + (int64_t)j * 64 * (lda + 1);
    a.lda = lda;
    a.Ginv = mode == 0 ? Gd + (int64_t)j * 4096 : nullptr;
    a.logdiag = logdiag + (int64_t)j * 64;
    a.info = info_dev;
    a.row0 = (int64_t)j * 64;
    a.mode = mode;
    if (j + 1 < nbk) {
      const int rows = (int)n - (j + 1) * 64;
      double* panel = A + (int64_t)(j + 1) * 64 + (int64_t)j * 64 * lda;
      const double* G = mode == 0 ? Gd + (int64_t)j * 4096 : a.A;
      const int64_t ldg = mode == 0 ? 64 : lda;
      push_tasks({mk_task(panel, lda, G, ldg, panel, lda, rows, 64, 64,
                          F_TB | F_BETA0, 1.0, 0.0)});
      push_tasks({mk_task(panel, lda, panel, lda, A + (int64_t)(j + 1) * 64 * (lda + 1),
                          lda, rows, rows, 64, F_TB | F_LOWER, -1.0, 1.0)});
    }
  }
  // recursive inversion levels (deepest first)
  std::vector<std::vector<int>> lv;
  std::function<void(int, int, int)> rec = [&](int lo, int hi, int d) {
    if (hi - lo <= 1) return;
    const int mid = lo + (hi - lo) / 2;
    if ((int)lv.size() <= d) lv.resize(d + 1);
    lv[d].push_back(lo);
    lv[d].push_back(hi);
    rec(lo, mid, d + 1);
    rec(mid, hi, d + 1);
  };
  const size_t n_fac = t_off.size();
  if (want_inverse) {
    rec(0, nbk, 0);
    for (int d = (int)lv.size() - 1; d >= 0; --d) {
      std::vector<GemmTask> tT, tG;
      for (size_t k = 0; k < lv[d].size(); k += 2) {
        const int lo = lv[d][k], hi = lv[d][k + 1], mid = lo + (hi - lo) / 2;
        const int n1 = (mid - lo) * 64, n2 = (hi - mid) * 64;
        double* L21 = A + (int64_t)mid * 64 + (int64_t)lo * 64 * lda;
        double* G11 = A + (int64_t)lo * 64 * (lda + 1);
        double* G22 = A + (int64_t)mid * 64 * (lda + 1);
        double* T = temp + (int64_t)lo * 64;
        tT.push_back(mk_task(L21, lda, G11, lda, T, n, n2, n1, n1, F_KLO_COL | F_BETA0, 1.0, 0.0));
        tG.push_back(mk_task(G22, lda, T, n, L21, lda, n2, n1, n2, F_KHI_ROW | F_BETA0, -1.0, 0.0));
      }
      push_tasks(tT);
      push_tasks(tG);
    }
  }
  std::vector<SumJob> sj(1);
  sj[0].src = logdiag; sj[0].n = n; sj[0].scale = 2.0; sj[0].dst = logdet_dev; sj[0].partial = part;
  MiscJob* dpre = nullptr;
  PotrfTileArgs* dpt = nullptr;
  GemmTask* dt = nullptr;
  SumJob* dsj = nullptr;
  hipError_t e = to_dev(tmp, pre, &dpre, s);
  if (e == hipSuccess) e = to_dev(tmp, pt, &dpt, s);
  if (e == hipSuccess) e = to_dev(tmp, tasks, &dt, s);
  if (e == hipSuccess) e = to_dev(tmp, sj, &dsj, s);
  if (e == hipSuccess) e = launch_misc(dpre, 2, s);
  for (int j = 0; j < nbk && e == hipSuccess; ++j) {
    e = launch_potrf_tiles(dpt + j, 1, s);
    if (e == hipSuccess && j + 1 < nbk) {
      for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        const size_t i = 2 * j + k;
        e = launch_gemm_tasks(dt + t_off[i], t_cnt[i], t_tiles[i], s);
      }
    }
  }
  for (size_t i = n_fac; i < t_off.size() && e == hipSuccess; ++i)
    e = launch_gemm_tasks(dt + t_off[i], t_cnt[i], t_tiles[i], s);
  if (e == hipSuccess) e = launch_sums(dsj, 1, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  free_all(tmp);
  return e == hipSuccess ? DL_OK : DL_EHIP;
}
