// Shared host/device definitions of libdalia_hip (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <vector>

#include "../../include/dalia.h"

#define DL_HIP_CHECK(expr)                                   \
  do {                                                       \
    hipError_t e__ = (expr);                                 \
    if (e__ != hipSuccess) return DL_EHIP;                   \
  } while (0)

namespace dl {

// ---- dense tile GEMM task ------------------------------------------------------
//
// C(MxN) = alpha * op(A) * op(B) + beta * C, column-major.
//   op(A) = A (M x K, lda) or A^T (A stored K x M) when F_TA;
//   op(B) = B (K x N, ldb) or B^T (B stored N x K) when F_TB.
// Flags restricting work at tile granularity (operands that are triangular
// hold exact zeros outside their triangle, so the restriction only skips
// work):
//   F_LOWER   : only tiles/elements with row >= col of C are computed;
//   F_KLO_COL : k >= first column of the C tile; F_KHI_COL : k < last col+1;
//   F_KLO_ROW : k >= first row of the C tile;    F_KHI_ROW : k < last row+1.
enum : int {
  F_TA = 1,
  F_TB = 2,
  F_LOWER = 4,
  F_KLO_COL = 8,
  F_KHI_COL = 16,
  F_KLO_ROW = 32,
  F_KHI_ROW = 64,
  F_BETA0 = 128,   // ignore beta and the previous C (C may hold NaN)
  // FP32 kernel only: operand stored in FP64 / output accumulated in FP64
  F_A64 = 256,
  F_B64 = 512,
  F_C64 = 1024,
  // FP64 kernel: split the k range of long tiles (see below)
  F_SPLIT = 2048,
  // set by finalize_tasks on every task of a launch in which some task's k
  // range varies from tile to tile (any F_KLO_* / F_KHI_* flag): the tiles
  // of such a task are ordered longest first and the launch's workgroups are
  // dealt to the XCDs in turn, so each XCD gets the same mix of lengths
  F_KVAR = 4096,
};

// Split k.  For an F_SPLIT task with K > ksplit (the task's piece length,
// GEMM_KSPLIT when 0; a multiple of 16), the k range [kb, ke) of each tile is
// cut at the absolute multiples of ksplit and every piece
// is one workgroup.  A tile with several pieces writes each raw product to a
// partial tile (BT x BT doubles, column-major) and a second launch forms
// C = alpha * (sum of the pieces in k order) + beta * C; a tile with one
// piece writes C directly.  Cutting at absolute k makes the result
// independent of the tile size and of the other tasks of the launch.  The
// launch has kslices workgroups per tile of such a task (ordered piece by
// piece over the task's tiles); those whose piece is empty for their tile
// return at once.
constexpr int GEMM_KSPLIT = 512;

struct GemmTask {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int32_t M, N, K, flags;
  double alpha, beta;
  int32_t tiles_m, tiles_n;  // filled by finalize_tasks
  int32_t tile_begin;        // first linear tile of this task in its launch
  int32_t ntiles;
  int32_t kslices;           // workgroups per tile (1 unless split)
  int32_t unit_begin;        // first workgroup of this task in its launch
  int32_t pslot_begin;       // first partial tile of this task
  int32_t red_begin;         // first reduction workgroup of this task
  int32_t ksplit;            // split-k piece length (0: GEMM_KSPLIT; resolved
                             // by finalize_tasks)
  int32_t pad_;
};

constexpr int GEMM_BM = 64;
constexpr int GEMM_BN = 64;

// Fill the tiling fields for square tiles of `tile` (64 or 128) rows; return
// the number of workgroups of the launch.  nred / nslots (optional) receive
// the reduction workgroups and the partial tiles a split launch needs.
int finalize_tasks(GemmTask* t, int n, int tile = 64, int* nred = nullptr,
                   int64_t* nslots = nullptr);

// Launch a batch of tasks already resident in device memory (tasks_dev) with
// `units` workgroups of tile x tile outputs (tile 64 or 128, the value the
// tasks were finalised with).  partials: nslots * tile * tile doubles (may be
// null when nothing is split).
hipError_t launch_gemm_tasks(const GemmTask* tasks_dev, int ntask, int units,
                             hipStream_t s, int tile = 64, double* partials = nullptr);
// The reduction of a split launch (nred workgroups).
hipError_t launch_gemm_reduce(const GemmTask* tasks_dev, int ntask, int nred,
                              const double* partials, hipStream_t s, int tile);
// FP32 MFMA variant; A/B/C pointers are float* unless F_A64/F_B64/F_C64.
hipError_t launch_gemm32_tasks(const GemmTask* tasks_dev, int ntask,
                               int total_tiles, hipStream_t s, int tile = 64);

// Convenience: copy host tasks to a device buffer, then launch.  Used by
// the dense ABI entry points and by plan building (never inside timed
// evaluation loops, where task arrays are prebuilt).
struct DeviceTasks {
  GemmTask* dev = nullptr;
  int ntask = 0;
  int total = 0;
};

// ---- 64x64 diagonal-tile Cholesky ------------------------------------------
// Factor the 64 x 64 SPD tile at A (lda) in place.  mode 0: lower triangle
// of A <- L (upper zeroed), Ginv (64 x 64, ld 64, may be null) <- L^{-1};
// mode 1: lower triangle of A <- L^{-1} (the factor itself is not kept).
// logdiag[i] = log L_ii; on a non-positive pivot *info = row0 + i + 1 (first
// failure only).  A batch of tiles is one launch, one workgroup per tile.
struct PotrfTileArgs {
  double* A;
  int64_t lda;
  double* Ginv;
  double* logdiag;
  int64_t* info;
  int64_t row0;
  int32_t mode;
  int32_t pad_;
};
hipError_t launch_potrf_tiles(const PotrfTileArgs* args_dev, int count,
                              hipStream_t s);

// ---- fused panel step of a blocked diagonal-block Cholesky -------------------
// For the n x n block A (nbk x nbk tiles of 64, column-major, ld) whose
// tiles 0..j are factored and whose panel j below the diagonal holds
// L(., j), one step j applies the trailing update of panel j to the lower
// tiles (I, J), j < J <= I:
//     A(I, J) -= L(I, j) L(J, j)^T,
// factors the updated diagonal tile j+1 (logdiag, info) and solves the panel
// below it, L(I, j+1) = A(I, j+1) G_{j+1}^T, so the next step again finds
// its panel solved.  The same launch advances the inverse G = L^{-1}
// (left-looking, one row of tiles per step):
//     G(j, c) = -G_jj (S(j, c) + L(j, j-1) G(j-1, c)),   c < j,
//     S(r, c) += L(r, j-1) G(j-1, c),                     r > j, c < j,
// S(r, c) = sum over k = c .. j-2 of L(r, k) G(k, c) accumulated in
// `stage`.  Workgroup roles, in grid segments: factor (the workgroup of
// tile j+1), column (tiles (I, j+1), I > j+1: each updates the diagonal
// tile j+1 in LDS the same way, factors it and solves its own tile), inverse
// row (G(j, c)), inverse accumulate (S(r, c)), rest (I >= J > j+1).
// Hand-overs: while column j+1 reads diagonal tile j+1, G_{j+1} goes to the
// side ring (gside slot (j+1) % 2) and step j+1 moves it into place; while
// row j of the inverse reads L(j, j-1), G(j, j-1) stays in stage and step j+1
// moves it into place.  The closing launch (last = 1, j = nbk-1) computes
// the inverse's last row only; its G(nbk-1, nbk-2) is left in stage.
struct PanelTask {
  double* A;
  int64_t ld;
  double* logdiag;     // 64 entries for tile j+1
  int64_t* info;
  int64_t row0;        // global row of tile j+1
  double* gside;       // 2 x 64 x 64 doubles (ld 64)
  double* stage;       // tile (r, c), c < r: ((r (r-1)) / 2 + c) * 4096 (ld 64)
  int32_t j, nbk;
  int32_t last;
  int32_t inv;         // 0: no inverse workgroups (the recursive inverse follows)
  int32_t beg[5];      // first workgroup of this task in each role segment
  int32_t tot[5];      // workgroups of each role in the launch (every task)
};
// Fill beg/tot; return the grid size.
int finalize_panels(PanelTask* t, int n);
hipError_t launch_panel_updates(const PanelTask* tasks_dev, int ntask, int grid,
                                hipStream_t s);

// ---- persistent tile-task factorisation of diagonal blocks --------------------
// One launch factors several diagonal blocks (A = L L^T, G = L^{-1} formed
// alongside) by working through the task list of dag.hpp: each workgroup
// takes the next task word (in list order), waits until the counters it
// depends on are set, runs the task on 64 x 64 tiles and sets its counter.
// On return each block holds G in its lower triangle, logdiag[i] = log L_ii
// and *info the first bad pivot (as the panel path), or DL_INFO_TIMEOUT when
// a wait gave up (it never should: the list order cannot deadlock).
struct DagBlock {
  double* A;          // the block (bp x bp, ld)
  int64_t ld;
  double* L;          // tiles L(i, k), i > k, same layout and ld as A
  double* stage;      // inverse accumulators: tile (r, c) at ((r (r-1)) / 2 + c) * 4096, ld 64
  double* logdiag;    // 64 * nbk entries
  int64_t* info;
  int64_t row0;       // BTA row of the block's first row
  int32_t* ctr;       // nbk * nbk readiness counters: zero before the launch;
                      // the launch's last workgroup zeroes them again
  int32_t nbk, pad_;
};
// head[0]: next task, head[1]: finished workgroups, head[2]: set when a wait
// gave up (then every later wait gives up at once, so the launch ends
// quickly); all zero before the launch and reset by its last workgroup.
// workers: the grid size.
hipError_t launch_dag_chol(const uint64_t* tasks, int ntask, const DagBlock* blocks,
                           int nblocks, int32_t* head, int workers, hipStream_t s);

// ---- small batched element-wise jobs ------------------------------------------
// MJ_AXPY_UNCONV: dst += src unless norms[0] <= tol2[0] * norms[1] (a
// residual already within the squared relative tolerance: the iterate
// stays as it is, bit for bit);
// MJ_COPY2D_TO_F32: FP64 src into an FP32 dst.
enum : int { MJ_FILL = 0, MJ_COPY = 1, MJ_ZERO_I64 = 2, MJ_DIAG = 3,
             MJ_COPY2D = 4, MJ_ZERO_UPPER_TILES = 5, MJ_COPY2D_F32 = 6,
             MJ_AXPY = 7, MJ_AXPY_UNCONV = 8, MJ_COPY2D_TO_F32 = 9 };
struct MiscJob {
  int32_t kind, rows, cols, pad_;
  double* dst;
  const double* src;
  int64_t n, lds, ldd;
  double v;
  const double* norms;
  const double* tol2;
};
hipError_t launch_misc(const MiscJob* jobs_dev, int count, hipStream_t s);

// out[0] = scale * sum(src[0..n)) with a fixed reduction order; partial
// holds SUM_BLOCKS doubles per job.
constexpr int SUM_BLOCKS = 128;
struct SumJob {
  const double* src;
  int64_t n;
  double scale;
  double* dst;
  double* partial;
};
hipError_t launch_sums(const SumJob* jobs_dev, int count, hipStream_t s);

}  // namespace dl
