// CPU emulation of the diagonal-block task graph (csrc/dag.hpp): runs the
// task list of one launch (several blocks) through the persistent launch's
// protocol -- each worker takes the next task of the list, waits for the
// counters it needs, runs it and sets its counter -- with 1 to 512 workers
// and runnable tasks finishing in random order, on plain arrays with tiles
// of TS x TS, in the chained form (C tasks) and the unchained one, and
// checks that
//   * every value a task waits for is set by an earlier task of the list and
//     every counter steps by one (C(k)'s final counter by two, past the value
//     its own update would have set);
//   * the workers never all wait with nothing runnable (no deadlock);
//   * tasks runnable at the same time never conflict on a tile (one writes
//     what the other reads or writes): the waits order every conflicting pair;
//   * the tasks compute G = L^{-1} of A = L L^T and log|A|, against a plain
//     Cholesky and triangular inversion of the same matrix.
// Prints "ok ..." per case; exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2507_06938_amd/csrc/dag.hpp"

using namespace dl::dag;

static int fail(const char* what, int nbk, size_t t) {
  std::printf("FAIL %s nbk=%d task=%zu\n", what, nbk, t);
  return 1;
}

struct Block {
  int nbk, TS, n;
  std::vector<double> A, L, St;  // A: the block (then G); L: factor tiles; St: accumulators
  double logdet = 0.0;
  double& a(int r, int c) { return A[(size_t)c * n + r]; }
  double& l(int r, int c) { return L[(size_t)c * n + r]; }
  double& st(int R, int C, int r, int c) {  // accumulator tile (R, C), element (r, c)
    return St[((size_t)R * (R - 1) / 2 + C) * TS * TS + (size_t)c * TS + r];
  }
};

// plain dense Cholesky (lower) in place; false on a bad pivot
static bool chol(std::vector<double>& M, int n) {
  for (int j = 0; j < n; ++j) {
    double d = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= M[(size_t)k * n + j] * M[(size_t)k * n + j];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    M[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = M[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) s -= M[(size_t)k * n + i] * M[(size_t)k * n + j];
      M[(size_t)j * n + i] = s / d;
    }
  }
  return true;
}

// inverse of a lower-triangular matrix (column-major), lower part only
static void trinv(const std::vector<double>& Lm, std::vector<double>& G, int n) {
  G.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    G[(size_t)c * n + c] = 1.0 / Lm[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      double s = 0.0;
      for (int k = c; k < r; ++k) s += Lm[(size_t)k * n + r] * G[(size_t)c * n + k];
      G[(size_t)c * n + r] = -s / Lm[(size_t)r * n + r];
    }
  }
}

static void run_task(Block& B, const Task& t, int phase = 0) {
  const int TS = B.TS;
  auto R0 = [&](int i) { return i * TS; };
  if (t.type == T_C) {  // phase 0: S(k+1, k); phase 1: U(k+1, k+1, k), then F(k+1)
    const int k = t.k;
    if (phase == 0) {
      run_task(B, Task{T_S, k + 1, k, k});
    } else {
      run_task(B, Task{T_U, k + 1, k + 1, k});
      run_task(B, Task{T_F, k + 1, k + 1, k + 1});
    }
    return;
  }
  switch (t.type) {
    case T_F: {
      const int k = t.k;
      std::vector<double> T((size_t)TS * TS), G;
      for (int c = 0; c < TS; ++c)
        for (int r = 0; r < TS; ++r) T[(size_t)c * TS + r] = B.a(R0(k) + r, R0(k) + c);
      if (!chol(T, TS)) { std::printf("FAIL not SPD\n"); std::exit(1); }
      for (int i = 0; i < TS; ++i) B.logdet += 2.0 * std::log(T[(size_t)i * TS + i]);
      trinv(T, G, TS);
      for (int c = 0; c < TS; ++c)
        for (int r = 0; r < TS; ++r) B.a(R0(k) + r, R0(k) + c) = r >= c ? G[(size_t)c * TS + r] : 0.0;
      break;
    }
    case T_S: {  // L(i,k) = A(i,k) G_kk^T
      for (int r = 0; r < TS; ++r)
        for (int c = 0; c < TS; ++c) {
          double s = 0.0;
          for (int q = 0; q < TS; ++q) s += B.a(R0(t.i) + r, R0(t.k) + q) * B.a(R0(t.k) + c, R0(t.k) + q);
          B.l(R0(t.i) + r, R0(t.k) + c) = s;
        }
      break;
    }
    case T_U: {  // A(i,k) -= L(i,j) L(k,j)^T
      for (int r = 0; r < TS; ++r)
        for (int c = 0; c < TS; ++c) {
          double s = 0.0;
          for (int q = 0; q < TS; ++q) s += B.l(R0(t.i) + r, R0(t.j) + q) * B.l(R0(t.k) + c, R0(t.j) + q);
          B.a(R0(t.i) + r, R0(t.k) + c) -= s;
        }
      break;
    }
    case T_A: {  // S(r,c) (+)= L(r,m) G(m,c); G(m,c) in A(m,c)
      const int Rr = t.i, Cc = t.k, m = t.j;
      for (int r = 0; r < TS; ++r)
        for (int c = 0; c < TS; ++c) {
          double s = m > Cc ? B.st(Rr, Cc, r, c) : 0.0;
          for (int q = 0; q < TS; ++q) s += B.l(R0(Rr) + r, R0(m) + q) * B.a(R0(m) + q, R0(Cc) + c);
          B.st(Rr, Cc, r, c) = s;
        }
      break;
    }
    case T_R: {  // G(j,c) = -G_jj (S(j,c) + L(j,j-1) G(j-1,c))
      const int j = t.i, Cc = t.k;
      std::vector<double> T((size_t)TS * TS);
      for (int r = 0; r < TS; ++r)
        for (int c = 0; c < TS; ++c) {
          double s = (j - 1 > Cc) ? B.st(j, Cc, r, c) : 0.0;
          for (int q = 0; q < TS; ++q) s += B.l(R0(j) + r, R0(j - 1) + q) * B.a(R0(j - 1) + q, R0(Cc) + c);
          T[(size_t)c * TS + r] = s;
        }
      for (int r = 0; r < TS; ++r)
        for (int c = 0; c < TS; ++c) {
          double s = 0.0;
          for (int q = 0; q <= r; ++q) s += B.a(R0(j) + r, R0(j) + q) * T[(size_t)c * TS + q];
          B.a(R0(j) + r, R0(Cc) + c) = -s;
        }
      break;
    }
  }
}

// Tiles a task reads and writes, as (kind, row, col): kind 0 = A (or G), 1 =
// L, 2 = accumulator.
struct Acc { int kind, r, c; };
static void footprint(const Task& t, std::vector<Acc>& rd, std::vector<Acc>& wr,
                      int phase = 0) {
  rd.clear();
  wr.clear();
  switch (t.type) {
    case T_C:  // phase 0 also reads tile (k+1, k+1), which the kernel loads up front
      if (phase == 0) {
        rd.push_back({0, t.k + 1, t.k}); rd.push_back({0, t.k, t.k});
        rd.push_back({0, t.k + 1, t.k + 1});
        wr.push_back({1, t.k + 1, t.k});
      } else {
        rd.push_back({1, t.k + 1, t.k}); rd.push_back({0, t.k + 1, t.k + 1});
        wr.push_back({0, t.k + 1, t.k + 1});
      }
      break;
    case T_F: rd.push_back({0, t.k, t.k}); wr.push_back({0, t.k, t.k}); break;
    case T_S: rd.push_back({0, t.i, t.k}); rd.push_back({0, t.k, t.k}); wr.push_back({1, t.i, t.k}); break;
    case T_U:
      rd.push_back({1, t.i, t.j}); rd.push_back({1, t.k, t.j}); rd.push_back({0, t.i, t.k});
      wr.push_back({0, t.i, t.k});
      break;
    case T_A:
      rd.push_back({1, t.i, t.j}); rd.push_back({0, t.j, t.k});
      if (t.j > t.k) rd.push_back({2, t.i, t.k});
      wr.push_back({2, t.i, t.k});
      break;
    case T_R:
      if (t.i - 1 > t.k) rd.push_back({2, t.i, t.k});
      rd.push_back({1, t.i, t.i - 1}); rd.push_back({0, t.i - 1, t.k}); rd.push_back({0, t.i, t.i});
      wr.push_back({0, t.i, t.k});
      break;
  }
}

static bool overlap(const std::vector<Acc>& a, const std::vector<Acc>& b) {
  for (const Acc& x : a)
    for (const Acc& y : b)
      if (x.kind == y.kind && x.r == y.r && x.c == y.c) return true;
  return false;
}

// Runs one launch's task list through the persistent launch's protocol
// with `workers` workgroups: each takes the next task of the list, waits
// until the counters it needs are set, runs it and sets its counter; tasks
// whose waits are met finish in random order.  Checks that the list only
// waits on earlier tasks, that the workers never all wait with nothing
// runnable (deadlock), that tasks runnable at the same time never conflict
// on a tile, and the numerical result.
static int check_case(const std::vector<int>& nbks, int TS, unsigned seed, int workers,
                      bool chain) {
  const std::vector<uint64_t> list = launch_list(nbks, true, chain);
  const size_t n = list.size();
  std::vector<std::vector<int>> ctr(nbks.size());
  for (size_t b = 0; b < nbks.size(); ++b) ctr[b].assign(counters_per_block(nbks[b]), 0);
  {  // every wait is met by an earlier task of the list
    std::vector<std::vector<int>> c2 = ctr;
    for (size_t t = 0; t < n; ++t) {
      int b = 0;
      const Task task = unpack(list[t], &b);
      Wait w[4], st, md;
      const int nw = waits_of(nbks[b], task, w, &st);
      for (int e = 0; e < nw; ++e)
        if (c2[b][w[e].ctr] < w[e].value) return fail("wait on a later task", nbks[b], t);
      if (mid_set(task, &md)) {
        if (c2[b][md.ctr] + 1 != md.value) return fail("counter does not step by one", nbks[b], t);
        c2[b][md.ctr] = md.value;
      }
      const int step = task.type == T_C ? 2 : 1;
      if (c2[b][st.ctr] + step != st.value) return fail("counter does not step by one", nbks[b], t);
      c2[b][st.ctr] = st.value;
    }
  }
  std::vector<Block> blocks(nbks.size());
  std::vector<std::vector<double>> A0(nbks.size());
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd;
  for (size_t b = 0; b < nbks.size(); ++b) {
    Block& B = blocks[b];
    B.nbk = nbks[b];
    B.TS = TS;
    B.n = B.nbk * TS;
    const int nn = B.n;
    std::vector<double> X((size_t)nn * (nn + 3));
    for (double& x : X) x = nd(rng);
    B.A.assign((size_t)nn * nn, 0.0);
    for (int r = 0; r < nn; ++r)
      for (int c = 0; c <= r; ++c) {
        double v = 0.0;
        for (int q = 0; q < nn + 3; ++q) v += X[(size_t)q * nn + r] * X[(size_t)q * nn + c];
        v = v / nn + (r == c ? 0.5 : 0.0);
        B.a(r, c) = v;
        B.a(c, r) = v;
      }
    A0[b] = B.A;
    B.L.assign((size_t)nn * nn, 0.0);
    B.St.assign((size_t)B.nbk * B.nbk * TS * TS, 0.0);
  }
  size_t next = 0, done = 0;
  std::vector<size_t> held;  // list positions held by the workers
  std::vector<int> phase;    // 1: a C task past its published solve
  while ((int)held.size() < workers && next < n) {
    held.push_back(next++);
    phase.push_back(0);
  }
  size_t count[6] = {0, 0, 0, 0, 0, 0};
  std::vector<Acc> rd1, wr1, rd2, wr2;
  std::vector<size_t> ready;
  while (done < n) {
    ready.clear();
    for (size_t h = 0; h < held.size(); ++h) {
      int b = 0;
      const Task task = unpack(list[held[h]], &b);
      Wait w[4], st;
      const int nw = waits_of(nbks[b], task, w, &st);
      bool ok = true;
      for (int e = 0; e < nw && phase[h] == 0; ++e) ok = ok && ctr[b][w[e].ctr] >= w[e].value;
      if (ok) ready.push_back(h);
    }
    if (ready.empty()) return fail("deadlock: every worker waits", 0, done);
    // tasks runnable together must not conflict on a tile
    for (size_t x = 0; x < ready.size(); ++x)
      for (size_t y = x + 1; y < ready.size(); ++y) {
        int b1 = 0, b2 = 0;
        const Task t1 = unpack(list[held[ready[x]]], &b1);
        const Task t2 = unpack(list[held[ready[y]]], &b2);
        if (b1 != b2) continue;
        footprint(t1, rd1, wr1, phase[ready[x]]);
        footprint(t2, rd2, wr2, phase[ready[y]]);
        if (overlap(wr1, rd2) || overlap(wr1, wr2) || overlap(rd1, wr2))
          return fail("conflicting runnable tasks", nbks[b1], held[ready[x]]);
      }
    const size_t h = ready[(size_t)(rng() % ready.size())];
    int b = 0;
    const Task task = unpack(list[held[h]], &b);
    Wait w[4], st, md;
    waits_of(nbks[b], task, w, &st);
    if (task.type == T_C && phase[h] == 0) {  // the solve, then its counter
      run_task(blocks[b], task, 0);
      mid_set(task, &md);
      ctr[b][md.ctr] = md.value;
      phase[h] = 1;
      continue;
    }
    run_task(blocks[b], task, phase[h]);
    ctr[b][st.ctr] = st.value;
    ++count[task.type];
    ++done;
    if (next < n) {
      held[h] = next++;
      phase[h] = 0;
    } else {
      held.erase(held.begin() + h);
      phase.erase(phase.begin() + h);
    }
  }
  for (size_t b = 0; b < nbks.size(); ++b) {
    Block& B = blocks[b];
    const int nn = B.n, nbk = B.nbk;
    std::vector<double> M = A0[b], G;
    if (!chol(M, nn)) return fail("reference not SPD", nbk, 0);
    trinv(M, G, nn);
    double ld = 0.0, gmax = 0.0, err = 0.0;
    for (int i = 0; i < nn; ++i) ld += 2.0 * std::log(M[(size_t)i * nn + i]);
    for (int c = 0; c < nn; ++c)
      for (int r = c; r < nn; ++r) {
        gmax = std::max(gmax, std::fabs(G[(size_t)c * nn + r]));
        err = std::max(err, std::fabs(G[(size_t)c * nn + r] - B.a(r, c)));
      }
    if (!(err <= 1e-11 * gmax)) { std::printf("G error %g (max %g)\n", err, gmax); return fail("inverse", nbk, 0); }
    if (!(std::fabs(ld - B.logdet) <= 1e-11 * std::fabs(ld))) return fail("logdet", nbk, 0);
  }
  std::printf("ok %s blocks=%zu workers=%d tasks=%zu F=%zu S=%zu U=%zu A=%zu R=%zu C=%zu\n",
              chain ? "chained" : "unchained", nbks.size(), workers, n, count[0], count[1],
              count[2], count[3], count[4], count[5]);
  return 0;
}

int main() {
  const std::vector<std::vector<int>> cases = {{1}, {2}, {3}, {5}, {7, 7}, {4, 9, 2}, {16}, {32, 32, 32, 32}, {43}};
  const int workers[] = {1, 3, 16, 64, 512};
  for (size_t c = 0; c < cases.size(); ++c) {
    const int TS = cases[c][0] >= 16 ? 3 : 5;
    const bool big = cases[c].size() * cases[c][0] >= 32;
    for (int w : workers)
      for (bool chain : {true, false})
        if (!(big && (w == 3 || w == 512)) &&
            check_case(cases[c], TS, 17 + (unsigned)c * 7 + (unsigned)w, w, chain))
          return 1;
  }
  return 0;
}
