// dl_dpotrf_noalloc: the dense Cholesky of dl_dpotrf for callers that cannot
// allocate device memory.  Its temporaries (the tile inverses of the panel
// solves, the recursive inversion's products, the log-diagonal, the
// reduction partials and the launch descriptors) live in one file-scope
// device array instead of per-call allocations; the kernels are the same as
// dl_dpotrf's and receive the array's device address like any other buffer.
#include <mutex>

#include "engine.hpp"

using namespace dl;

namespace {

constexpr int64_t kMaxN = DL_DPOTRF_NOALLOC_MAX_N;
constexpr int kMaxTiles = (int)(kMaxN / 64);
// descriptor counts for kMaxTiles tiles: 2 GEMM launches per panel, and two
// per node of the recursive halving (kMaxTiles - 1 nodes)
constexpr int kMaxGemm = 4 * kMaxTiles;
constexpr int kMaxLaunches = 2 * kMaxTiles + 2 * 16;
// scratch layout, in doubles (every region 256-byte aligned)
constexpr int64_t kDescDoubles = 8192;  // 64 KiB of launch descriptors
constexpr int64_t kGdDoubles = kMaxN * 64;
constexpr int64_t kTempDoubles = kMaxN * (kMaxTiles / 2 + 1) * 64;
constexpr int64_t kLogDoubles = kMaxN;
constexpr int64_t kPartDoubles = 256;
constexpr int64_t kScratchDoubles =
    kDescDoubles + kGdDoubles + kTempDoubles + kLogDoubles + kPartDoubles;
static_assert(kScratchDoubles * 8 == DL_DPOTRF_NOALLOC_SCRATCH_BYTES,
              "scratch size stated in the header");

}  // namespace

// The scratch array.  In host code this name is only a stand-in for the
// symbol: its device address comes from hipGetSymbolAddress (one per device).
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double* g_scratch[64] = {nullptr};

// Device address of `scratch` on the current device (looked up once).
dl_status scratch_ptr(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DL_EHIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DL_EHIP;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return DL_OK;
}

// Host -> device copy of a few KB through kernel arguments (captured by value
// at launch), so the host array may go away when the launch call returns.
constexpr int kChunkWords = 768;
struct Chunk {
  uint32_t w[kChunkWords];
};

__global__ __launch_bounds__(256) void k_put_words(uint32_t* __restrict__ dst, Chunk c,
                                                   int nwords) {
  for (int i = threadIdx.x; i < nwords; i += 256) dst[i] = c.w[i];
}

hipError_t put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint32_t* w = (const uint32_t*)src;
  size_t words = (bytes + 3) / 4;
  uint32_t* d = (uint32_t*)dst;
  while (words > 0) {
    const int nw = (int)(words < (size_t)kChunkWords ? words : (size_t)kChunkWords);
    Chunk c;
    for (int i = 0; i < nw; ++i) c.w[i] = w[i];
    hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, d, c, nw);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    w += nw;
    d += nw;
    words -= nw;
  }
  return hipSuccess;
}

template <typename T>
T* carve(char*& cursor, int count) {
  T* p = (T*)cursor;
  cursor += ((sizeof(T) * (size_t)count + 255) / 256) * 256;
  return p;
}

GemmTask task(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
              int64_t ldc, int M, int N, int K, int flags, double alpha, double beta) {
  GemmTask t{};
  t.A = A; t.B = B; t.C = C;
  t.lda = lda; t.ldb = ldb; t.ldc = ldc;
  t.M = M; t.N = N; t.K = K; t.flags = flags;
  t.alpha = alpha; t.beta = beta;
  return t;
}

}  // namespace

extern "C" dl_status dl_dpotrf_noalloc(int64_t n, double* A, int64_t lda,
                                       int32_t want_inverse, double* logdet_dev,
                                       int64_t* info_dev, void* stream) {
  if (n <= 0 || n % 64 != 0 || n > kMaxN || !A || lda < n || !logdet_dev || !info_dev)
    return DL_EINVAL;
  double* ptr = nullptr;
  const dl_status st = scratch_ptr(&ptr);
  if (st != DL_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int nbk = (int)(n / 64);

  // regions of the scratch array (device addresses)
  double* Gd = ptr + kDescDoubles;
  double* temp = Gd + kGdDoubles;
  double* logdiag = temp + kTempDoubles;
  double* part = logdiag + kLogDoubles;

  // host descriptors, in fixed-size arrays
  MiscJob pre[2] = {};
  pre[0].kind = MJ_ZERO_I64; pre[0].dst = (double*)info_dev; pre[0].n = 1;
  pre[1].kind = MJ_ZERO_UPPER_TILES; pre[1].dst = A; pre[1].rows = (int)n; pre[1].ldd = lda;
  PotrfTileArgs pt[kMaxTiles] = {};
  GemmTask tasks[kMaxGemm];
  int t_off[kMaxLaunches], t_cnt[kMaxLaunches], t_tiles[kMaxLaunches];
  int ntasks = 0, nl = 0;
  auto push1 = [&](const GemmTask& g) {
    tasks[ntasks] = g;
    t_off[nl] = ntasks;
    t_cnt[nl] = 1;
    t_tiles[nl] = finalize_tasks(tasks + ntasks, 1);
    ++ntasks;
    ++nl;
  };
  // as dl_dpotrf: mode 0 (A <- L, tile inverse to Gd) without the inverse,
  // mode 1 (inverse in place) with it
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
      push1(task(panel, lda, G, ldg, panel, lda, rows, 64, 64, F_TB | F_BETA0, 1.0, 0.0));
      push1(task(panel, lda, panel, lda, A + (int64_t)(j + 1) * 64 * (lda + 1), lda, rows,
                 rows, 64, F_TB | F_LOWER, -1.0, 1.0));
    }
  }
  const int n_fac = nl;
  if (want_inverse) {
    // recursive halving, the nodes of one depth in one launch, deepest first
    // (iterative: node (lo, hi) at depth d; at most log2(kMaxTiles) + 1 levels)
    int lo_d[16][kMaxTiles], hi_d[16][kMaxTiles], cnt_d[16] = {0};
    int depth = 0;
    int cur_lo[kMaxTiles], cur_hi[kMaxTiles], ncur = 0;
    if (nbk > 1) { cur_lo[0] = 0; cur_hi[0] = nbk; ncur = 1; }
    while (ncur > 0) {
      int nxt_lo[kMaxTiles], nxt_hi[kMaxTiles], nnxt = 0;
      for (int k = 0; k < ncur; ++k) {
        const int lo = cur_lo[k], hi = cur_hi[k], mid = lo + (hi - lo) / 2;
        lo_d[depth][cnt_d[depth]] = lo;
        hi_d[depth][cnt_d[depth]] = hi;
        ++cnt_d[depth];
        if (mid - lo > 1) { nxt_lo[nnxt] = lo; nxt_hi[nnxt] = mid; ++nnxt; }
        if (hi - mid > 1) { nxt_lo[nnxt] = mid; nxt_hi[nnxt] = hi; ++nnxt; }
      }
      for (int k = 0; k < nnxt; ++k) { cur_lo[k] = nxt_lo[k]; cur_hi[k] = nxt_hi[k]; }
      ncur = nnxt;
      ++depth;
    }
    for (int d = depth - 1; d >= 0; --d) {
      for (int pass = 0; pass < 2; ++pass) {
        const int o = ntasks;
        for (int k = 0; k < cnt_d[d]; ++k) {
          const int lo = lo_d[d][k], hi = hi_d[d][k], mid = lo + (hi - lo) / 2;
          const int n1 = (mid - lo) * 64, n2 = (hi - mid) * 64;
          double* L21 = A + (int64_t)mid * 64 + (int64_t)lo * 64 * lda;
          double* G11 = A + (int64_t)lo * 64 * (lda + 1);
          double* G22 = A + (int64_t)mid * 64 * (lda + 1);
          double* T = temp + (int64_t)lo * 64;
          tasks[ntasks++] =
              pass == 0 ? task(L21, lda, G11, lda, T, n, n2, n1, n1, F_KLO_COL | F_BETA0, 1.0, 0.0)
                        : task(G22, lda, T, n, L21, lda, n2, n1, n2, F_KHI_ROW | F_BETA0, -1.0, 0.0);
        }
        t_off[nl] = o;
        t_cnt[nl] = ntasks - o;
        t_tiles[nl] = finalize_tasks(tasks + o, ntasks - o);
        ++nl;
      }
    }
  }
  SumJob sj{};
  sj.src = logdiag; sj.n = n; sj.scale = 2.0; sj.dst = logdet_dev; sj.partial = part;

  // descriptors into the scratch array, then the launches of dl_dpotrf
  char* cursor = (char*)ptr;
  MiscJob* dpre = carve<MiscJob>(cursor, 2);
  PotrfTileArgs* dpt = carve<PotrfTileArgs>(cursor, nbk);
  GemmTask* dt = carve<GemmTask>(cursor, ntasks > 0 ? ntasks : 1);
  SumJob* dsj = carve<SumJob>(cursor, 1);
  if (cursor > (char*)(ptr + kDescDoubles)) return DL_EINVAL;  // cannot happen for n <= kMaxN
  hipError_t e = put_bytes(dpre, pre, sizeof(pre), s);
  if (e == hipSuccess) e = put_bytes(dpt, pt, sizeof(PotrfTileArgs) * nbk, s);
  if (e == hipSuccess && ntasks > 0) e = put_bytes(dt, tasks, sizeof(GemmTask) * ntasks, s);
  if (e == hipSuccess) e = put_bytes(dsj, &sj, sizeof(sj), s);
  if (e == hipSuccess) e = launch_misc(dpre, 2, s);
  for (int j = 0; j < nbk && e == hipSuccess; ++j) {
    e = launch_potrf_tiles(dpt + j, 1, s);
    if (e == hipSuccess && j + 1 < nbk) {
      for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        const int i = 2 * j + k;
        e = launch_gemm_tasks(dt + t_off[i], t_cnt[i], t_tiles[i], s);
      }
    }
  }
  for (int i = n_fac; i < nl && e == hipSuccess; ++i)
    e = launch_gemm_tasks(dt + t_off[i], t_cnt[i], t_tiles[i], s);
  if (e == hipSuccess) e = launch_sums(dsj, 1, s);
  return e == hipSuccess ? DL_OK : DL_EHIP;
}
