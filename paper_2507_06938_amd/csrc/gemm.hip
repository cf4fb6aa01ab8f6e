// FP64 MFMA tile GEMM over a list of tasks (gfx950).
//
// One workgroup computes one 64x64 tile (4 wave64, 32x32 per wave) or one
// 128x128 tile (8 wave64, 64x32 per wave; two workgroups fit one compute
// unit) of C for one task of a launch (the tile size is fixed per launch).
// Tiles of all tasks of a launch are numbered consecutively; a workgroup
// finds its task by binary search over the tasks' first tile.  Workgroups
// are renumbered so that those one XCD receives take consecutive tiles (the
// operand tiles they share then stay in that XCD's L2).  The inner product
// runs on v_mfma_f64_16x16x4_f64 with operands staged through
// double-buffered LDS in 16-deep k chunks.  Aligned operands with even
// extents are staged with 16-byte global loads (two doubles per slot, a
// fixed number of loads per chunk, zeros for slots outside the operand),
// the next one or two chunks in flight in registers while the current one
// is multiplied; other operands take a per-element bounds-checked path.
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
// LDS row padding of the staged chunks (doubles)
constexpr int LPAD = 2;

__device__ __forceinline__ int find_task(const GemmTask* __restrict__ tasks,
                                         int ntask, int tile) {
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Workgroups go to the 8 XCDs in turn (workgroup b to XCD b % 8): map them
// so that XCD x takes the consecutive tiles [x q + min(x, r), ...) of the
// nb = 8 q + r tiles.  A bijection of 0..nb-1.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, i = bid >> 3;
  return x * q + min(x, r) + i;
}

// Stage PER = BR*BK/NT doubles of op(X) per thread: op(X)[r][k] for a
// BR-row, BK-deep chunk.  `trans` = X stored K x R (contiguous along k).
template <int BR, int NT>
__device__ __forceinline__ void load_chunk(const double* __restrict__ X,
                                           int64_t ldx, bool trans, int r0,
                                           int R, int k0, int kend, int tid,
                                           double (&v)[BR * BK / NT]) {
  constexpr int PER = BR * BK / NT;
  if (!trans) {
    // X[r + k*ldx]; lanes run along r (BR consecutive rows per k).
    const int r = r0 + (tid % BR);
    const int kb = k0 + (tid / BR) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = kb + i;
      v[i] = (r < R && k < kend) ? X[(int64_t)r + (int64_t)k * ldx] : 0.0;
    }
  } else {
    // X[k + r*ldx]; lanes run along k (BK consecutive k per row).
    const int k = k0 + (tid % BK);
    const int rb = r0 + (tid / BK) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int r = rb + i;
      v[i] = (r < R && k < kend) ? X[(int64_t)k + (int64_t)r * ldx] : 0.0;
    }
  }
}

template <int BR, int NT>
__device__ __forceinline__ void store_chunk(double* __restrict__ S, bool trans,
                                            int tid, const double (&v)[BR * BK / NT]) {
  constexpr int PER = BR * BK / NT;
  constexpr int LD = BR + LPAD;
  if (!trans) {
    const int r = tid % BR;
    const int kb = (tid / BR) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) S[(kb + i) * LD + r] = v[i];
  } else {
    const int k = tid % BK;
    const int rb = (tid / BK) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) S[k * LD + rb + i] = v[i];
  }
}

// Vector staging (the usual case: operand 16-byte aligned, even leading
// dimension, even row count / k extent).  Each thread owns PV slots of two
// consecutive doubles of memory per BK-deep chunk of op(X) (BR rows).
// Untransposed X (X[r + k ldx]): slot j holds rows rl, rl+1 (rl even) of
// chunk column kq + j KS.  Transposed X (X[k + r ldx]): slot j holds chunk
// columns kq, kq+1 (kq even) of row rl + j RS.  Invalid slots (outside the
// operand or the k range) read the operand's first pair and stage zeros, so
// every chunk issues exactly PV global loads per operand and thread.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) v2d* gv2d_ptr;

template <int BR, int NT>
struct VStage {
  static constexpr int PV = BR * BK / (2 * NT);
  static constexpr int NP = BR / 2, KS = NT / NP;   // untransposed
  static constexpr int NQ = BK / 2, RS = NT / NQ;   // transposed
  static_assert(NT % NP == 0 && BK % KS == 0 && NT % NQ == 0 && BR % RS == 0, "map");
  const double* base;  // operand origin (the safe address of invalid slots)
  const double* p;     // slot 0 of the current chunk
  int64_t step, adv;
  int rl, kq;          // tile-relative row, chunk-relative k of slot 0
  int kc, kend;        // current chunk's first k, k limit
  bool trans;
  unsigned rowok;      // bit j: slot j's row(s) inside the operand

  __device__ __forceinline__ void init(const double* X, int64_t ldx, bool tr, int r0, int R,
                                       int k0, int ke, int tid) {
    base = X;
    trans = tr;
    kc = k0;
    kend = ke;
    rowok = 0;
    if (!tr) {
      rl = 2 * (tid % NP);
      kq = tid / NP;
      p = X + (r0 + rl) + (int64_t)(k0 + kq) * ldx;
      step = (int64_t)KS * ldx;
      adv = (int64_t)BK * ldx;
      if (r0 + rl < R) rowok = (1u << PV) - 1;
    } else {
      kq = 2 * (tid % NQ);
      rl = tid / NQ;
      p = X + (k0 + kq) + (int64_t)(r0 + rl) * ldx;
      step = (int64_t)RS * ldx;
      adv = BK;
#pragma unroll
      for (int j = 0; j < PV; ++j)
        if (r0 + rl + j * RS < R) rowok |= 1u << j;
    }
  }

  __device__ __forceinline__ void load(v2d (&v)[PV]) const {
#pragma unroll
    for (int j = 0; j < PV; ++j) {
      const int k = kc + kq + (trans ? 0 : j * KS);
      const bool ok = ((rowok >> j) & 1u) && k < kend;
      const double* a = ok ? p + j * step : base;
      const v2d x = *(gv2d_ptr)a;
      v[j] = ok ? x : (v2d){0.0, 0.0};
    }
  }

  __device__ __forceinline__ void next() {
    p += adv;
    kc += BK;
  }

  __device__ __forceinline__ void store(double* __restrict__ S, const v2d (&v)[PV]) const {
    constexpr int LD = BR + LPAD;
    if (!trans) {
#pragma unroll
      for (int j = 0; j < PV; ++j) *(v2d*)(S + (kq + j * KS) * LD + rl) = v[j];
    } else {
#pragma unroll
      for (int j = 0; j < PV; ++j) {
        S[kq * LD + rl + j * RS] = v[j].x;
        S[(kq + 1) * LD + rl + j * RS] = v[j].y;
      }
    }
  }
};

// Tile order within a task: bands of GROUP tile rows, each band swept
// column by column (lower-triangular tasks: the columns left of the band,
// then its triangular diagonal block).  Consecutive tiles -- and so the
// tiles one XCD holds at a time -- then form a compact patch whose operand
// rows and columns are reused from that XCD's L2.
constexpr int GROUP = 8;

__device__ __forceinline__ void tile_coords(const GemmTask& T, int lt, int& tm,
                                            int& tn) {
  constexpr int KCOL = F_KLO_COL | F_KHI_COL, KROW = F_KLO_ROW | F_KHI_ROW;
  if (!(T.flags & F_LOWER) && (T.flags & (KCOL | KROW))) {
    // k range set by the tile column (or row): whole columns (rows) in
    // order of decreasing length
    if (T.flags & KCOL) {
      const int c = lt / T.tiles_m;
      tm = lt - c * T.tiles_m;
      tn = (T.flags & F_KHI_COL) ? T.tiles_n - 1 - c : c;
    } else {
      const int r = lt / T.tiles_n;
      tn = lt - r * T.tiles_n;
      tm = (T.flags & F_KHI_ROW) ? T.tiles_m - 1 - r : r;
    }
    return;
  }
  if (T.flags & F_LOWER) {
    const int nt = T.tiles_m;  // square tile grid
    int g = (int)((sqrt(8.0 * (double)lt + 1.0) - 1.0) * 0.5) / GROUP;
    while (g > 0 && (g * GROUP) * (g * GROUP + 1) / 2 > lt) --g;
    while (((g + 1) * GROUP) * ((g + 1) * GROUP + 1) / 2 <= lt) ++g;
    const int r0 = g * GROUP;
    const int gm = min(nt - r0, GROUP);
    int loc = lt - r0 * (r0 + 1) / 2;
    if (loc < r0 * gm) {
      tm = r0 + loc % gm;
      tn = loc / gm;
      return;
    }
    loc -= r0 * gm;
    int c = 0;
    while (loc >= gm - c) {
      loc -= gm - c;
      ++c;
    }
    tm = r0 + c + loc;
    tn = r0 + c;
  } else {
    const int gs = GROUP * T.tiles_n;
    const int first = (lt / gs) * GROUP;
    const int gm = min(T.tiles_m - first, GROUP);
    const int loc = lt % gs;
    tm = first + loc % gm;
    tn = loc / gm;
  }
}
}  // namespace

// Whether an operand can be staged with VStage: 16-byte aligned, even
// leading dimension, and pairs that never straddle the row count (staged
// untransposed) or the k range (staged transposed).
__device__ __forceinline__ bool vec_operand(const double* X, int64_t ldx, bool strans, int R,
                                            int kb, int ke) {
  if ((reinterpret_cast<uintptr_t>(X) & 15) != 0 || (ldx & 1) != 0) return false;
  return strans ? ((kb & 1) == 0 && (ke & 1) == 0) : ((R & 1) == 0);
}

// acc += the product of one staged BK-deep chunk: wave (wm, wn) multiplies
// its FM x FN blocks of 16 x 16.  With few blocks per wave (64-wide tiles)
// all fragments of the chunk are read from LDS first, so the MFMAs of one
// k step overlap the reads of the next.
template <int BT, int WM, int WN>
__device__ __forceinline__ void mma_chunk(const double* __restrict__ as,
                                          const double* __restrict__ bs,
                                          v4d (&acc)[BT / WM / 16][BT / WN / 16], int wm,
                                          int wn, int lrow, int lk) {
  constexpr int LD = BT + LPAD;
  constexpr int SM = BT / WM, SN = BT / WN;
  constexpr int FM = SM / 16, FN = SN / 16;
  if constexpr (FM + FN <= 4) {
    double fa[BK / 4][FM], fb[BK / 4][FN];
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + lk;
#pragma unroll
      for (int i = 0; i < FM; ++i) fa[ks][i] = as[kk * LD + wm * SM + i * 16 + lrow];
#pragma unroll
      for (int j = 0; j < FN; ++j) fb[ks][j] = bs[kk * LD + wn * SN + j * 16 + lrow];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMAs
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[ks][j], fa[ks][i], acc[i][j],
                                                           0, 0, 0);
  } else {
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      double fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) fa[i] = as[kk * LD + wm * SM + i * 16 + lrow];
#pragma unroll
      for (int j = 0; j < FN; ++j) fb[j] = bs[kk * LD + wn * SN + j * 16 + lrow];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[j], fa[i], acc[i][j], 0, 0, 0);
    }
  }
}

// One workgroup of WM x WN waves computes one BT x BT tile; wave (wm, wn)
// owns rows wm*BT/WM .. and columns wn*BT/WN .. of it, FM x FN MFMA blocks
// of 16 x 16.  MINW: waves per SIMD the register budget must allow.
// Task of workgroup (or reduction workgroup) `u`: the last task whose
// first index is <= u (tasks with no work share their successor's first).
__device__ __forceinline__ int find_unit_task(const GemmTask* __restrict__ tasks,
                                              int ntask, int u, bool red) {
  int lo = 0, hi = ntask - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((red ? tasks[mid].red_begin : tasks[mid].unit_begin) <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int BT, int WM, int WN, int MINW, int PF>
__global__ __launch_bounds__(WM * WN * 64, MINW) void k_gemm_tasks(
    const GemmTask* __restrict__ tasks, int ntask, double* __restrict__ partials) {
  constexpr int NT = WM * WN * 64;
  constexpr int LD = BT + LPAD;
  constexpr int SM = BT / WM, SN = BT / WN;  // wave sub-tile
  constexpr int FM = SM / 16, FN = SN / 16;
  constexpr int PER = BT * BK / NT;  // staged doubles per thread per operand
  __shared__ __attribute__((aligned(16))) double As[2][BK * LD];
  __shared__ __attribute__((aligned(16))) double Bs[2][BK * LD];

  const int tid = threadIdx.x;
  const int wid = (tasks[0].flags & F_KVAR) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const int ti = find_unit_task(tasks, ntask, wid, false);
  const GemmTask T = tasks[ti];
  // slice-major: the workgroups of one XCD take one k piece of a compact
  // patch of tiles
  const int local = wid - T.unit_begin;
  const int lt = local % T.ntiles, sl = local / T.ntiles;
  int tm, tn;
  tile_coords(T, lt, tm, tn);
  const int m0 = tm * BT;
  const int n0 = tn * BT;
  const bool ta = T.flags & F_TA;
  const bool tb = T.flags & F_TB;

  int kb = 0, ke = T.K;
  if (T.flags & F_KLO_COL) kb = max(kb, n0);
  if (T.flags & F_KHI_COL) ke = min(ke, n0 + BT);
  if (T.flags & F_KLO_ROW) kb = max(kb, m0);
  if (T.flags & F_KHI_ROW) ke = min(ke, m0 + BT);
  kb = (kb / BK) * BK;
  int slot = -1;  // partial tile of this piece (split tiles only)
  if (T.kslices > 1 && ke > kb) {
    const int ks = T.ksplit;
    const int s0 = kb / ks;
    const int npieces = (ke - 1) / ks - s0 + 1;
    if (sl >= npieces) return;  // no piece here for this tile
    if (npieces > 1) slot = T.pslot_begin + lt * T.kslices + sl;
    kb = max(kb, (s0 + sl) * ks);
    ke = min(ke, (s0 + sl + 1) * ks);
  } else if (sl > 0) {
    return;
  }
  const int nchunks = ke > kb ? (ke - kb + BK - 1) / BK : 0;

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lrow = lane & 15, lk = lane >> 4;

  v4d acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  const bool vec_a = vec_operand(T.A, T.lda, ta, T.M, kb, ke);
  const bool vec_b = vec_operand(T.B, T.ldb, !tb, T.N, kb, ke);
  if (vec_a && vec_b) {
    VStage<BT, NT> sa, sb;
    sa.init(T.A, T.lda, ta, m0, T.M, kb, ke, tid);
    sb.init(T.B, T.ldb, !tb, n0, T.N, kb, ke, tid);
    constexpr int PV = VStage<BT, NT>::PV;
    v2d a0[PV], b0[PV];
    sa.load(a0); sb.load(b0); sa.next(); sb.next();
    if constexpr (PF == 1) {
      sa.store(As[0], a0); sb.store(Bs[0], b0);
      __syncthreads();
      for (int c = 0; c < nchunks; ++c) {
        sa.load(a0); sb.load(b0); sa.next(); sb.next();  // chunk c + 1
        mma_chunk<BT, WM, WN>(As[c & 1], Bs[c & 1], acc, wm, wn, lrow, lk);
        sa.store(As[(c + 1) & 1], a0); sb.store(Bs[(c + 1) & 1], b0);
        __syncthreads();
      }
    } else {
      // two chunks in flight: a0/b0 and a1/b1 alternate
      v2d a1[PV], b1[PV];
      sa.load(a1); sb.load(b1); sa.next(); sb.next();    // chunk 1
      sa.store(As[0], a0); sb.store(Bs[0], b0);
      __syncthreads();
      for (int c = 0; c < nchunks; c += 2) {
        sa.load(a0); sb.load(b0); sa.next(); sb.next();  // chunk c + 2
        mma_chunk<BT, WM, WN>(As[0], Bs[0], acc, wm, wn, lrow, lk);
        sa.store(As[1], a1); sb.store(Bs[1], b1);        // chunk c + 1
        __syncthreads();
        if (c + 1 >= nchunks) break;
        sa.load(a1); sb.load(b1); sa.next(); sb.next();  // chunk c + 3
        mma_chunk<BT, WM, WN>(As[1], Bs[1], acc, wm, wn, lrow, lk);
        sa.store(As[0], a0); sb.store(Bs[0], b0);        // chunk c + 2
        __syncthreads();
      }
    }
  } else {
    // scalar staging with per-element bounds (odd sizes, unaligned operands)
    double va[PER], vb[PER];
    if (nchunks > 0) {
      load_chunk<BT, NT>(T.A, T.lda, ta, m0, T.M, kb, ke, tid, va);
      load_chunk<BT, NT>(T.B, T.ldb, !tb, n0, T.N, kb, ke, tid, vb);
      store_chunk<BT, NT>(As[0], ta, tid, va);
      store_chunk<BT, NT>(Bs[0], !tb, tid, vb);
    }
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = (c + 1) < nchunks;
      if (more) {
        const int k1 = kb + (c + 1) * BK;
        load_chunk<BT, NT>(T.A, T.lda, ta, m0, T.M, k1, ke, tid, va);
        load_chunk<BT, NT>(T.B, T.ldb, !tb, n0, T.N, k1, ke, tid, vb);
      }
      mma_chunk<BT, WM, WN>(As[buf], Bs[buf], acc, wm, wn, lrow, lk);
      if (more) {
        store_chunk<BT, NT>(As[buf ^ 1], ta, tid, va);
        store_chunk<BT, NT>(Bs[buf ^ 1], !tb, tid, vb);
      }
      __syncthreads();
    }
  }

  if (slot >= 0) {
    // one piece of a split tile: the raw product, tile-local column-major
    double* P = partials + (int64_t)slot * BT * BT;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          P[(wm * SM + i * 16 + lrow) + (wn * SN + j * 16 + lk + 4 * r) * BT] = acc[i][j][r];
    return;
  }
  // epilogue: lane holds C[m][n0' + lk + 4r], m = row of lane
  const bool lower = T.flags & F_LOWER;
  const bool beta0 = T.flags & F_BETA0;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int m = m0 + wm * SM + i * 16 + lrow;
    if (m >= T.M) continue;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wn * SN + j * 16 + lk + 4 * r;
        if (n >= T.N || (lower && n > m)) continue;
        double* p = T.C + (int64_t)m + (int64_t)n * T.ldc;
        double v = T.alpha * acc[i][j][r];
        if (!beta0) v += T.beta * (*p);
        *p = v;
      }
    }
  }
}

// C = alpha * sum of the pieces + beta * C for the split tiles, one
// workgroup per tile; the pieces are added in k order.
template <int BT>
__global__ __launch_bounds__(256) void k_gemm_reduce(const GemmTask* __restrict__ tasks,
                                                     int ntask,
                                                     const double* __restrict__ partials) {
  const int ti = find_unit_task(tasks, ntask, blockIdx.x, true);
  const GemmTask T = tasks[ti];
  const int lt = blockIdx.x - T.red_begin;
  int tm, tn;
  tile_coords(T, lt, tm, tn);
  const int m0 = tm * BT, n0 = tn * BT;
  int kb = 0, ke = T.K;
  if (T.flags & F_KLO_COL) kb = max(kb, n0);
  if (T.flags & F_KHI_COL) ke = min(ke, n0 + BT);
  if (T.flags & F_KLO_ROW) kb = max(kb, m0);
  if (T.flags & F_KHI_ROW) ke = min(ke, m0 + BT);
  kb = (kb / BK) * BK;
  if (ke <= kb) return;
  const int npieces = (ke - 1) / T.ksplit - kb / T.ksplit + 1;
  if (npieces < 2) return;  // written directly by the product launch
  const bool lower = T.flags & F_LOWER;
  const bool beta0 = T.flags & F_BETA0;
  const double* P = partials + (int64_t)(T.pslot_begin + lt * T.kslices) * BT * BT;
  for (int e = threadIdx.x; e < BT * BT; e += 256) {
    const int m = m0 + e % BT, n = n0 + e / BT;
    if (m >= T.M || n >= T.N || (lower && n > m)) continue;
    double sum = P[e];
    for (int q = 1; q < npieces; ++q) sum += P[(int64_t)q * BT * BT + e];
    double* c = T.C + (int64_t)m + (int64_t)n * T.ldc;
    double v = T.alpha * sum;
    if (!beta0) v += T.beta * (*c);
    *c = v;
  }
}

int finalize_tasks(GemmTask* t, int n, int tile, int* nred, int64_t* nslots) {
  int total = 0, units = 0, red = 0;
  int64_t slots = 0;
  bool kvar = false;
  for (int i = 0; i < n; ++i)
    kvar = kvar || (t[i].flags & (F_KLO_COL | F_KHI_COL | F_KLO_ROW | F_KHI_ROW));
  for (int i = 0; i < n; ++i) {
    t[i].flags = kvar ? (t[i].flags | F_KVAR) : (t[i].flags & ~F_KVAR);
    t[i].tiles_m = (t[i].M + tile - 1) / tile;
    t[i].tiles_n = (t[i].N + tile - 1) / tile;
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
    if (t[i].ksplit <= 0) t[i].ksplit = GEMM_KSPLIT;
    const int ks = t[i].ksplit;
    const bool split = (t[i].flags & F_SPLIT) && t[i].K > ks;
    t[i].kslices = split ? (t[i].K + ks - 1) / ks : 1;
    t[i].unit_begin = units;
    units += t[i].ntiles * t[i].kslices;
    t[i].pslot_begin = (int32_t)slots;
    t[i].red_begin = red;
    if (split) {
      slots += (int64_t)t[i].ntiles * t[i].kslices;
      red += t[i].ntiles;
    }
  }
  if (nred) *nred = red;
  if (nslots) *nslots = slots;
  return units;
}

hipError_t launch_gemm_tasks(const GemmTask* tasks_dev, int ntask, int units,
                             hipStream_t s, int tile, double* partials) {
  if (units <= 0) return hipSuccess;
  if (tile == 128)
    hipLaunchKernelGGL((k_gemm_tasks<128, 2, 4, 4, 1>), dim3(units), dim3(512), 0, s,
                       tasks_dev, ntask, partials);
  else
    hipLaunchKernelGGL((k_gemm_tasks<64, 2, 2, 4, 1>), dim3(units), dim3(256), 0, s,
                       tasks_dev, ntask, partials);
  return hipGetLastError();
}

hipError_t launch_gemm_reduce(const GemmTask* tasks_dev, int ntask, int nred,
                              const double* partials, hipStream_t s, int tile) {
  if (nred <= 0) return hipSuccess;
  if (tile == 128)
    hipLaunchKernelGGL(k_gemm_reduce<128>, dim3(nred), dim3(256), 0, s, tasks_dev, ntask,
                       partials);
  else
    hipLaunchKernelGGL(k_gemm_reduce<64>, dim3(nred), dim3(256), 0, s, tasks_dev, ntask,
                       partials);
  return hipGetLastError();
}


// ---- FP32 MFMA variant (mixed precision) --------------------------------------
//
// Same task model and tiling as above with v_mfma_f32_16x16x4_f32 and FP32
// accumulation.  Operands are FP32 unless the task's F_A64 / F_B64 flag says
// the operand is stored in FP64 (it is then rounded to FP32 when staged);
// C is FP32 unless F_C64, in which case alpha*acc + beta*C is formed in FP64
// and stored in FP64 (Schur updates into FP64 diagonal blocks and tips).
// Lane layout of the FP32 accumulator: register r of lane l holds
// D[4(l/16) + r][l%16] (checked against host GEMMs by the GPU tests).
typedef float v4f_ __attribute__((ext_vector_type(4)));

namespace {
template <int BR>
__device__ __forceinline__ void load_chunk32(const void* __restrict__ Xv, bool x64,
                                             int64_t ldx, bool trans, int r0, int R,
                                             int k0, int kend, int tid,
                                             float (&v)[BR * BK / 256]) {
  constexpr int PER = BR * BK / 256;
  const double* X64 = (const double*)Xv;
  const float* X32 = (const float*)Xv;
  if (!trans) {
    const int r = r0 + (tid % BR);
    const int kb = k0 + (tid / BR) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = kb + i;
      const int64_t o = (int64_t)r + (int64_t)k * ldx;
      v[i] = (r < R && k < kend) ? (x64 ? (float)X64[o] : X32[o]) : 0.f;
    }
  } else {
    const int k = k0 + (tid % BK);
    const int rb = r0 + (tid / BK) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int r = rb + i;
      const int64_t o = (int64_t)k + (int64_t)r * ldx;
      v[i] = (r < R && k < kend) ? (x64 ? (float)X64[o] : X32[o]) : 0.f;
    }
  }
}

template <int BR>
__device__ __forceinline__ void store_chunk32(float* __restrict__ S, bool trans, int tid,
                                              const float (&v)[BR * BK / 256]) {
  constexpr int PER = BR * BK / 256;
  constexpr int LD = BR + 4;
  if (!trans) {
    const int r = tid % BR;
    const int kb = (tid / BR) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) S[(kb + i) * LD + r] = v[i];
  } else {
    const int k = tid % BK;
    const int rb = (tid / BK) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) S[k * LD + rb + i] = v[i];
  }
}
// Vector staging of the FP32 kernel: each slot is one 16-byte load of E
// consecutive elements of the stored operand (E = 4 floats, or 2 doubles
// rounded to FP32 when staged).  Untransposed X (X[r + k ldx]): slot j holds
// rows rl .. rl+E-1 of chunk column kq + j KS; transposed X (X[k + r ldx]):
// chunk columns kq .. kq+E-1 of row rl + j RS.  Invalid slots read the
// operand's origin and stage zeros.
template <int BR, typename TE>
struct VStage32 {
  static constexpr int E = 16 / (int)sizeof(TE);
  static constexpr int PV = BR * BK / (E * 256);
  static constexpr int NP = BR / E, KS = 256 / NP;
  static constexpr int NQ = BK / E, RS = 256 / NQ;
  static_assert(256 % NP == 0 && BK % KS == 0 && 256 % NQ == 0 && BR % RS == 0, "map");
  typedef TE vec_t __attribute__((ext_vector_type(E)));
  const TE* base;
  const TE* p;
  int64_t step, adv;
  int rl, kq, kc, kend;
  bool trans;
  unsigned rowok;

  __device__ __forceinline__ void init(const void* Xv, int64_t ldx, bool tr, int r0, int R,
                                       int k0, int ke, int tid) {
    const TE* X = (const TE*)Xv;
    base = X;
    trans = tr;
    kc = k0;
    kend = ke;
    rowok = 0;
    if (!tr) {
      rl = E * (tid % NP);
      kq = tid / NP;
      p = X + (r0 + rl) + (int64_t)(k0 + kq) * ldx;
      step = (int64_t)KS * ldx;
      adv = (int64_t)BK * ldx;
      if (r0 + rl < R) rowok = (1u << PV) - 1;
    } else {
      kq = E * (tid % NQ);
      rl = tid / NQ;
      p = X + (k0 + kq) + (int64_t)(r0 + rl) * ldx;
      step = (int64_t)RS * ldx;
      adv = BK;
#pragma unroll
      for (int j = 0; j < PV; ++j)
        if (r0 + rl + j * RS < R) rowok |= 1u << j;
    }
  }

  __device__ __forceinline__ void load(float (&v)[PV][E]) const {
#pragma unroll
    for (int j = 0; j < PV; ++j) {
      const int k = kc + kq + (trans ? 0 : j * KS);
      const bool ok = ((rowok >> j) & 1u) && k < kend;
      const TE* a = ok ? p + j * step : base;
      const vec_t x = *(const __attribute__((address_space(1))) vec_t*)a;
#pragma unroll
      for (int e = 0; e < E; ++e) v[j][e] = ok ? (float)x[e] : 0.f;
    }
  }

  __device__ __forceinline__ void next() {
    p += adv;
    kc += BK;
  }

  __device__ __forceinline__ void store(float* __restrict__ S, const float (&v)[PV][E]) const {
    constexpr int LD = BR + 4;
    if (!trans) {
#pragma unroll
      for (int j = 0; j < PV; ++j)
#pragma unroll
        for (int e = 0; e < E; ++e) S[(kq + j * KS) * LD + rl + e] = v[j][e];
    } else {
#pragma unroll
      for (int j = 0; j < PV; ++j)
#pragma unroll
        for (int e = 0; e < E; ++e) S[(kq + e) * LD + rl + j * RS] = v[j][e];
    }
  }
};

// Whether an operand of the FP32 kernel can be staged with VStage32.
__device__ __forceinline__ bool vec_operand32(const void* X, int esize, int64_t ldx,
                                              bool strans, int R, int kb, int ke) {
  const int E = 16 / esize;
  if ((reinterpret_cast<uintptr_t>(X) & 15) != 0 || (ldx % E) != 0) return false;
  return strans ? (kb % E == 0 && ke % E == 0) : (R % E == 0);
}

// acc += one staged chunk (wave (wm, wn) owns F x F blocks of 16 x 16); all
// fragments of the chunk are read from LDS ahead of the MFMAs.
template <int BT>
__device__ __forceinline__ void mma_chunk32(const float* __restrict__ as,
                                            const float* __restrict__ bs,
                                            v4f_ (&acc)[BT / 32][BT / 32], int wm, int wn,
                                            int lrow, int lk) {
  constexpr int LD = BT + 4;
  constexpr int F = BT / 32;
  float fa[BK / 4][F], fb[BK / 4][F];
#pragma unroll
  for (int ks = 0; ks < BK / 4; ++ks) {
    const int kk = ks * 4 + lk;
#pragma unroll
    for (int i = 0; i < F; ++i) fa[ks][i] = as[kk * LD + wm * (BT / 2) + i * 16 + lrow];
#pragma unroll
    for (int j = 0; j < F; ++j) fb[ks][j] = bs[kk * LD + wn * (BT / 2) + j * 16 + lrow];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int ks = 0; ks < BK / 4; ++ks)
#pragma unroll
    for (int i = 0; i < F; ++i)
#pragma unroll
      for (int j = 0; j < F; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[ks][j], fa[ks][i], acc[i][j], 0, 0, 0);
}

template <int BT, typename TA, typename TB>
__device__ __forceinline__ void gemm32_vec_loop(const GemmTask& T, bool ta, bool tb, int m0,
                                                int n0, int kb, int ke, int nchunks, int tid,
                                                float* As0, float* As1, float* Bs0, float* Bs1,
                                                v4f_ (&acc)[BT / 32][BT / 32], int wm, int wn,
                                                int lrow, int lk) {
  VStage32<BT, TA> sa;
  VStage32<BT, TB> sb;
  sa.init(T.A, T.lda, ta, m0, T.M, kb, ke, tid);
  sb.init(T.B, T.ldb, !tb, n0, T.N, kb, ke, tid);
  float va[VStage32<BT, TA>::PV][VStage32<BT, TA>::E];
  float vb[VStage32<BT, TB>::PV][VStage32<BT, TB>::E];
  sa.load(va); sb.load(vb); sa.next(); sb.next();
  sa.store(As0, va); sb.store(Bs0, vb);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    sa.load(va); sb.load(vb); sa.next(); sb.next();  // chunk c + 1
    mma_chunk32<BT>((c & 1) ? As1 : As0, (c & 1) ? Bs1 : Bs0, acc, wm, wn, lrow, lk);
    sa.store((c & 1) ? As0 : As1, va);
    sb.store((c & 1) ? Bs0 : Bs1, vb);
    __syncthreads();
  }
}
}  // namespace

template <int BT>
__global__ __launch_bounds__(256) void k_gemm32_tasks(
    const GemmTask* __restrict__ tasks, int ntask) {
  constexpr int LD = BT + 4;
  constexpr int F = BT / 32;
  constexpr int PER = BT * BK / 256;
  __shared__ __attribute__((aligned(16))) float As[2][BK * LD];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK * LD];

  const int tid = threadIdx.x;
  const int tile = (tasks[0].flags & F_KVAR) ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const int ti = find_task(tasks, ntask, tile);
  const GemmTask T = tasks[ti];
  int tm, tn;
  tile_coords(T, tile - T.tile_begin, tm, tn);
  const int m0 = tm * BT;
  const int n0 = tn * BT;
  const bool ta = T.flags & F_TA;
  const bool tb = T.flags & F_TB;
  const bool a64 = T.flags & F_A64;
  const bool b64 = T.flags & F_B64;

  int kb = 0, ke = T.K;
  if (T.flags & F_KLO_COL) kb = max(kb, n0);
  if (T.flags & F_KHI_COL) ke = min(ke, n0 + BT);
  if (T.flags & F_KLO_ROW) kb = max(kb, m0);
  if (T.flags & F_KHI_ROW) ke = min(ke, m0 + BT);
  kb = (kb / BK) * BK;
  const int nchunks = ke > kb ? (ke - kb + BK - 1) / BK : 0;

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int lrow = lane & 15, lk = lane >> 4;

  v4f_ acc[F][F];
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j) acc[i][j] = (v4f_){0.f, 0.f, 0.f, 0.f};

  const bool vec_a = vec_operand32(T.A, a64 ? 8 : 4, T.lda, ta, T.M, kb, ke);
  const bool vec_b = vec_operand32(T.B, b64 ? 8 : 4, T.ldb, !tb, T.N, kb, ke);
  if (vec_a && vec_b) {
    if (a64 && b64)
      gemm32_vec_loop<BT, double, double>(T, ta, tb, m0, n0, kb, ke, nchunks, tid, As[0], As[1],
                                          Bs[0], Bs[1], acc, wm, wn, lrow, lk);
    else if (a64)
      gemm32_vec_loop<BT, double, float>(T, ta, tb, m0, n0, kb, ke, nchunks, tid, As[0], As[1],
                                         Bs[0], Bs[1], acc, wm, wn, lrow, lk);
    else if (b64)
      gemm32_vec_loop<BT, float, double>(T, ta, tb, m0, n0, kb, ke, nchunks, tid, As[0], As[1],
                                         Bs[0], Bs[1], acc, wm, wn, lrow, lk);
    else
      gemm32_vec_loop<BT, float, float>(T, ta, tb, m0, n0, kb, ke, nchunks, tid, As[0], As[1],
                                        Bs[0], Bs[1], acc, wm, wn, lrow, lk);
  } else {
    float va[PER], vb[PER];
    if (nchunks > 0) {
      load_chunk32<BT>(T.A, a64, T.lda, ta, m0, T.M, kb, ke, tid, va);
      load_chunk32<BT>(T.B, b64, T.ldb, !tb, n0, T.N, kb, ke, tid, vb);
      store_chunk32<BT>(As[0], ta, tid, va);
      store_chunk32<BT>(Bs[0], !tb, tid, vb);
    }
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const int buf = c & 1;
      const bool more = (c + 1) < nchunks;
      if (more) {
        const int k1 = kb + (c + 1) * BK;
        load_chunk32<BT>(T.A, a64, T.lda, ta, m0, T.M, k1, ke, tid, va);
        load_chunk32<BT>(T.B, b64, T.ldb, !tb, n0, T.N, k1, ke, tid, vb);
      }
      const float* __restrict__ as = As[buf];
      const float* __restrict__ bs = Bs[buf];
  #pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kk = ks * 4 + lk;
        float fa[F], fb[F];
  #pragma unroll
        for (int i = 0; i < F; ++i) fa[i] = as[kk * LD + wm * (BT / 2) + i * 16 + lrow];
  #pragma unroll
        for (int j = 0; j < F; ++j) fb[j] = bs[kk * LD + wn * (BT / 2) + j * 16 + lrow];
  #pragma unroll
        for (int i = 0; i < F; ++i)
  #pragma unroll
          for (int j = 0; j < F; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[j], fa[i], acc[i][j], 0, 0, 0);
      }
      if (more) {
        store_chunk32<BT>(As[buf ^ 1], ta, tid, va);
        store_chunk32<BT>(Bs[buf ^ 1], !tb, tid, vb);
      }
      __syncthreads();
    }
  }
  const bool lower = T.flags & F_LOWER;
  const bool beta0 = T.flags & F_BETA0;
  const bool c64 = T.flags & F_C64;
#pragma unroll
  for (int i = 0; i < F; ++i) {
#pragma unroll
    for (int j = 0; j < F; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // accumulator element (row 4*lk + r of the 16x16 block of C^T)
        const int m = m0 + wm * (BT / 2) + i * 16 + lrow;
        const int n = n0 + wn * (BT / 2) + j * 16 + 4 * lk + r;
        if (m >= T.M || n >= T.N || (lower && n > m)) continue;
        const int64_t o = (int64_t)m + (int64_t)n * T.ldc;
        if (c64) {
          double* p = (double*)T.C + o;
          double v = T.alpha * (double)acc[i][j][r];
          if (!beta0) v += T.beta * (*p);
          *p = v;
        } else {
          float* p = (float*)T.C + o;
          float v = (float)T.alpha * acc[i][j][r];
          if (!beta0) v += (float)T.beta * (*p);
          *p = v;
        }
      }
    }
  }
}

hipError_t launch_gemm32_tasks(const GemmTask* tasks_dev, int ntask,
                               int total_tiles, hipStream_t s, int tile) {
  if (total_tiles <= 0) return hipSuccess;
  if (tile == 128)
    hipLaunchKernelGGL(k_gemm32_tasks<128>, dim3(total_tiles), dim3(256), 0, s,
                       tasks_dev, ntask);
  else
    hipLaunchKernelGGL(k_gemm32_tasks<64>, dim3(total_tiles), dim3(256), 0, s,
                       tasks_dev, ntask);
  return hipGetLastError();
}

}  // namespace dl
