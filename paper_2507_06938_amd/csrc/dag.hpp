// Tile-task graph of one diagonal-block factorisation: the blocked
// right-looking Cholesky A = L L^T of an n x n block (nbk tiles of 64 x 64)
// with its inverse G = L^{-1} formed alongside, left-looking, as the tiles of
// L become final.  No HIP types: the engine builds the task lists of its
// persistent launches from it, the launch's kernel decodes tasks and their
// waits with it, and a CPU emulator in the tests runs the same lists on plain
// arrays.
//
// Tasks (tiles indexed (row, column), lower triangle):
//   F(k)        factor diagonal tile (k, k) (all its updates applied):
//               G_kk = L_kk^{-1} in place, log L_ii, first bad pivot
//   S(i, k)     solve L(i, k) = A(i, k) G_kk^T  (into the L buffer)
//   U(i, k, j)  A(i, k) -= L(i, j) L(k, j)^T   (j < k <= i)
//   A(r, c, m)  accumulate S(r, c) += L(r, m) G(m, c)   (c <= m <= r - 2)
//   R(j, c)     G(j, c) = -G_jj (S(j, c) + L(j, j-1) G(j-1, c))   (c < j)
//   C(k)        the chain from tile k to tile k+1 in one task: S(k+1, k),
//               then U(k+1, k+1, k) and F(k+1) on the tiles it holds
// G(j, c) goes into A(j, c) (read by nobody once S(j, c) has run), so on
// completion the block holds G in its lower triangle.  In the chained form
// (the one launches use) C(k) stands for S(k+1, k), U(k+1, k+1, k) and
// F(k+1): the factorisation's critical path -- each tile factor, the solve of
// the tile below it and that tile's last update -- then runs as one task per
// tile without handing tiles between workgroups, and C(k) publishes L(k+1, k)
// as soon as it is stored, before its update and factor.
//
// Readiness is tracked by one counter per tile and one per accumulator:
//   v(r, c): number of updates applied (0 .. c); c + 1 once L(r, c) (or G_cc
//            for r = c) is final; c + 2 once G(r, c) is final (r > c);
//   a(r, c): number of accumulated terms.
// Every task waits for counters to reach given values and then sets one
// counter (after its stores are complete).  A launch's task list is sorted
// by each task's latest start level (the longest chain of tasks after it,
// counted back from the end of the graph), ties by earliest start level, so
// every value a task waits for is set by a task earlier in the list (a
// dependency's latest start is strictly smaller), and the chain that bounds
// the factorisation -- each tile factor, the solve of the tile below it and
// that tile's last update -- comes before updates that are needed later.  A
// worker that takes tasks from the list in order only ever waits on tasks
// that running workers hold, so the launch cannot deadlock.
#pragma once

#include <stdint.h>

// Functions the device also calls (task decoding, waits) carry DL_DAG_FN,
// which a HIP translation unit defines as __host__ __device__ inline before
// including this header.
#ifndef DL_DAG_FN
#define DL_DAG_FN inline
#endif

#include <algorithm>
#include <vector>

namespace dl {
namespace dag {

enum : int { T_F = 0, T_S = 1, T_U = 2, T_A = 3, T_R = 4, T_C = 5 };

struct Task {
  int type;
  int i, k, j;  // F: (k, k, k); S: (i, k, k); U: (i, k, j); A: (r, c, m); R: (j, c, c);
                // C: (k + 1, k, k)
};

// Counter indices within a block: tiles first, then accumulators.
DL_DAG_FN int64_t tile_ctr(int r, int c) { return (int64_t)r * (r + 1) / 2 + c; }
DL_DAG_FN int64_t acc_ctr(int nbk, int r, int c) {
  return (int64_t)nbk * (nbk + 1) / 2 + (int64_t)r * (r - 1) / 2 + c;
}
DL_DAG_FN int64_t counters_per_block(int nbk) { return (int64_t)nbk * nbk; }

// One wait: counter index and the value it must reach.
struct Wait {
  int64_t ctr;
  int value;
};

// The waits of task t (at most 4) and the counter it sets (and the value)
// when it completes.
DL_DAG_FN int waits_of(int nbk, const Task& t, Wait* w, Wait* sets) {
  int n = 0;
  auto gfinal = [&](int m, int c) {  // G(m, c) final
    if (m == c) w[n++] = {tile_ctr(c, c), c + 1};
    else w[n++] = {tile_ctr(m, c), c + 2};
  };
  switch (t.type) {
    case T_F:
      w[n++] = {tile_ctr(t.k, t.k), t.k};
      *sets = {tile_ctr(t.k, t.k), t.k + 1};
      break;
    case T_S:
      w[n++] = {tile_ctr(t.i, t.k), t.k};
      w[n++] = {tile_ctr(t.k, t.k), t.k + 1};
      *sets = {tile_ctr(t.i, t.k), t.k + 1};
      break;
    case T_U:
      w[n++] = {tile_ctr(t.i, t.k), t.j};
      w[n++] = {tile_ctr(t.i, t.j), t.j + 1};
      if (t.k != t.i) w[n++] = {tile_ctr(t.k, t.j), t.j + 1};
      *sets = {tile_ctr(t.i, t.k), t.j + 1};
      break;
    case T_A:  // (r, c, m) = (i, k, j)
      if (t.j > t.k) w[n++] = {acc_ctr(nbk, t.i, t.k), t.j - t.k};
      w[n++] = {tile_ctr(t.i, t.j), t.j + 1};
      gfinal(t.j, t.k);
      *sets = {acc_ctr(nbk, t.i, t.k), t.j - t.k + 1};
      break;
    case T_R:  // (j, c) = (i, k)
      w[n++] = {tile_ctr(t.i, t.i), t.i + 1};
      if (t.i - 1 > t.k) w[n++] = {acc_ctr(nbk, t.i, t.k), t.i - 1 - t.k};
      w[n++] = {tile_ctr(t.i, t.i - 1), t.i};
      gfinal(t.i - 1, t.k);
      *sets = {tile_ctr(t.i, t.k), t.k + 2};
      break;
    case T_C:  // k = t.k: the waits of S(k+1, k), and the earlier updates of tile k+1
      w[n++] = {tile_ctr(t.k + 1, t.k), t.k};
      w[n++] = {tile_ctr(t.k, t.k), t.k + 1};
      w[n++] = {tile_ctr(t.k + 1, t.k + 1), t.k};
      *sets = {tile_ctr(t.k + 1, t.k + 1), t.k + 2};  // G(k+1, k+1) final
      break;
  }
  return n;
}

// The counter a task sets before it completes, if any: C(k) sets
// v(k+1, k) = k + 1 once L(k+1, k) is stored.  (Its final counter skips
// v(k+1, k+1) = k + 1, which only its own update would have set.)
DL_DAG_FN bool mid_set(const Task& t, Wait* s) {
  if (t.type != T_C) return false;
  *s = {tile_ctr(t.k + 1, t.k), t.k + 1};
  return true;
}

// All tasks of one block in phase order (step j: F(j), S(., j), R(j, .),
// U(., ., j), A(., ., j)), which is a valid order.  Chained: F(0), and in
// step j, C(j) in place of S(j+1, j) (it also stands for U(j+1, j+1, j) and
// F(j+1)).
inline std::vector<Task> phase_order(int nbk, bool inverse, bool chain = true) {
  std::vector<Task> q;
  for (int j = 0; j < nbk; ++j) {
    if (!chain || j == 0) q.push_back({T_F, j, j, j});
    for (int i = j + 1; i < nbk; ++i)
      q.push_back(chain && i == j + 1 ? Task{T_C, j + 1, j, j} : Task{T_S, i, j, j});
    if (inverse)
      for (int c = 0; c < j; ++c) q.push_back({T_R, j, c, c});
    for (int k = j + 1; k < nbk; ++k)
      for (int i = k; i < nbk; ++i)
        if (!(chain && i == j + 1 && k == j + 1)) q.push_back({T_U, i, k, j});
    if (inverse)
      for (int c = 0; c <= j; ++c)
        for (int r = j + 2; r < nbk; ++r) q.push_back({T_A, r, c, j});
  }
  return q;
}

// The block's tasks sorted by earliest start level (longest chain of
// predecessors), ties by latest start level, then by phase order.  Returns
// the tasks and, in `level` and `slack`, each one's earliest start level and
// the difference between its latest and earliest start levels.
inline std::vector<Task> schedule(int nbk, bool inverse, std::vector<int>* level = nullptr,
                                  std::vector<int>* slack = nullptr, bool chain = true) {
  std::vector<Task> q = phase_order(nbk, inverse, chain);
  const size_t n = q.size();
  const int64_t nc = counters_per_block(nbk);
  // producer of (counter, value): index into q
  std::vector<std::vector<int>> prod(nc);
  auto produce = [&](const Wait& s, int t) {
    std::vector<int>& p = prod[s.ctr];
    if ((int)p.size() < s.value + 1) p.resize(s.value + 1, -1);
    p[s.value] = t;
  };
  for (size_t t = 0; t < n; ++t) {
    Wait w[4], s, m;
    waits_of(nbk, q[t], w, &s);
    produce(s, (int)t);
    if (mid_set(q[t], &m)) produce(m, (int)t);
  }
  std::vector<int> asap(n, 0), alap(n, 0);
  std::vector<std::vector<int>> succ(n);
  for (size_t t = 0; t < n; ++t) {
    Wait w[4], s;
    const int nw = waits_of(nbk, q[t], w, &s);
    for (int e = 0; e < nw; ++e) {
      if (w[e].value == 0) continue;
      // the task that brings the counter to the value (or past it: C(k)
      // steps v(k+1, k+1) by two)
      const std::vector<int>& pv = prod[w[e].ctr];
      int v = w[e].value;
      while (pv[v] < 0) ++v;
      const int p = pv[v];
      asap[t] = std::max(asap[t], asap[p] + 1);
      succ[p].push_back((int)t);
    }
  }
  int depth = 0;
  for (size_t t = 0; t < n; ++t) depth = std::max(depth, asap[t]);
  for (size_t t = n; t-- > 0;) {
    int l = depth;
    for (int s2 : succ[t]) l = std::min(l, alap[s2] - 1);
    alap[t] = l;
  }
  std::vector<int> idx(n);
  for (size_t t = 0; t < n; ++t) idx[t] = (int)t;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (asap[a] != asap[b]) return asap[a] < asap[b];
    return alap[a] < alap[b];
  });
  std::vector<Task> out(n);
  if (level) level->resize(n);
  if (slack) slack->resize(n);
  for (size_t t = 0; t < n; ++t) {
    out[t] = q[idx[t]];
    if (level) (*level)[t] = asap[idx[t]];
    if (slack) (*slack)[t] = alap[idx[t]] - asap[idx[t]];
  }
  return out;
}

// A task word: type (4 bits), block within the launch (12), and the three
// tile indices (16 bits each).
DL_DAG_FN uint64_t pack(const Task& t, int block) {
  return (uint64_t)t.type | ((uint64_t)block << 4) | ((uint64_t)t.i << 16) |
         ((uint64_t)t.k << 32) | ((uint64_t)t.j << 48);
}
DL_DAG_FN Task unpack(uint64_t w, int* block) {
  *block = (int)((w >> 4) & 0xfff);
  return Task{(int)(w & 0xf), (int)((w >> 16) & 0xffff), (int)((w >> 32) & 0xffff),
              (int)((w >> 48) & 0xffff)};
}

// The task list of one launch over several blocks: all blocks' tasks
// sorted by latest start level, then earliest start level, then block, then
// phase order.
inline std::vector<uint64_t> launch_list(const std::vector<int>& nbks, bool inverse,
                                         bool chain = true) {
  struct Item {
    int alap, asap, block;
    size_t pos;
    Task t;
  };
  std::vector<Item> all;
  for (size_t b = 0; b < nbks.size(); ++b) {
    std::vector<int> lv, sl;
    std::vector<Task> s = schedule(nbks[b], inverse, &lv, &sl, chain);
    for (size_t p = 0; p < s.size(); ++p) all.push_back({lv[p] + sl[p], lv[p], (int)b, p, s[p]});
  }
  std::stable_sort(all.begin(), all.end(), [](const Item& a, const Item& b) {
    if (a.alap != b.alap) return a.alap < b.alap;
    if (a.asap != b.asap) return a.asap < b.asap;
    if (a.block != b.block) return a.block < b.block;
    return a.pos < b.pos;
  });
  std::vector<uint64_t> out;
  out.reserve(all.size());
  for (const Item& it : all) out.push_back(pack(it.t, it.block));
  return out;
}

}  // namespace dag
}  // namespace dl
