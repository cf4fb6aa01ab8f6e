// Model upload: FEM pattern of the SPDE precision and the observation index
// built on the host (integer work and the FEM stencil values), all arrays
// copied to the device once.
#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <new>
#include <vector>

#include "engine.hpp"

using namespace dl;

extern "C" int32_t dl_theta_dim(int32_t nv) {
  return nv == 1 ? 4 : 4 * nv + nv * (nv - 1) / 2;
}

extern "C" int32_t dl_theta_dim_lik(int32_t nv, int32_t likelihood) {
  if (likelihood == DL_LIK_GAUSSIAN) return dl_theta_dim(nv);
  if (likelihood == DL_LIK_POISSON) return dl_theta_dim(nv) - nv;
  return -1;
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


extern "C" dl_status dl_model_create(const dl_model_desc* desc,
                                     dl_model** out) {
  if (!desc || !out) return DL_EINVAL;
  const int nx = desc->nx, nt = desc->nt, nv = desc->nv, nr = desc->nr;
  if (nx < 2 || nt < 1 || nv < 1 || nv > 3 || nr < 0 || nv * nr > 64 ||
      (2 * ((nv * nx * nx + 63) / 64) * 64 + 64) * 8 > 160 * 1024)
    return DL_EINVAL;
  if (!desc->theta_prior_mean || !(desc->theta_prior_sd > 0.0)) return DL_EINVAL;
  const int family = desc->family;
  if (family != DL_MODEL_SEPARABLE && family != DL_MODEL_DIFFUSION) return DL_EINVAL;
  if (family == DL_MODEL_DIFFUSION && nt < 2) return DL_EINVAL;
  const int lik = desc->likelihood;
  if (lik != DL_LIK_GAUSSIAN && lik != DL_LIK_POISSON) return DL_EINVAL;
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
      if (lik == DL_LIK_POISSON) {
        const double y = desc->y[j][i];
        if (!(y >= 0.0) || !(y < 9.0e15) || y != floor(y)) return DL_EINVAL;
      }
    }
  }
  dl_model* M = new (std::nothrow) dl_model();
  if (!M) return DL_ENOMEM;
  ModelDev& d = M->d;
  d.nx = nx; d.nt = nt; d.nv = nv; d.nr = nr; d.ns = ns;
  d.family = family;
  d.b = nv * ns; d.a = nv * nr;
  d.bp = ((d.b + 63) / 64) * 64;
  d.ap = d.a > 0 ? 64 : 0;
  d.dim_theta = dl_theta_dim_lik(nv, lik);
  d.likelihood = lik;
  d.N = (int64_t)nt * d.b + d.a;
  d.Np = (int64_t)nt * d.bp + d.ap;
  d.theta_prior_sd = desc->theta_prior_sd;
  d.prior_fixed = desc->prior_fixed;

  // FEM pieces on the grid: C = I (lumped mass, unit spacing), G = 5-point
  // Neumann graph Laplacian, G C^-1 G = G*G and G C^-1 G C^-1 G = G*G*G.
  // Pattern: all nodes within grid distance 2 (13-point stencil), or 3 for
  // the diffusion model, whose K3 holds the third power of G.
  std::vector<int> ptr(ns + 1, 0), col;
  std::vector<double> vC, vG, vG2, vG3;
  auto inside = [&](int x, int y) { return x >= 0 && y >= 0 && x < nx && y < nx; };
  auto deg = [&](int ix, int iy) {
    return (ix > 0) + (ix < nx - 1) + (iy > 0) + (iy < nx - 1);
  };
  auto gval = [&](int ax, int ay, int bx, int by) -> double {
    if (ax == bx && ay == by) return (double)deg(ax, ay);
    if (abs(ax - bx) + abs(ay - by) == 1) return -1.0;
    return 0.0;
  };
  // row a of G has its nonzeros at a and its grid neighbours
  static const int nb5[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
  auto g2val = [&](int ax, int ay, int bx, int by) -> double {
    double acc = 0.0;
    for (int q = 0; q < 5; ++q) {
      const int kx = ax + nb5[q][0], ky = ay + nb5[q][1];
      if (inside(kx, ky)) acc += gval(ax, ay, kx, ky) * gval(kx, ky, bx, by);
    }
    return acc;
  };
  auto g3val = [&](int ax, int ay, int bx, int by) -> double {
    double acc = 0.0;
    for (int q = 0; q < 5; ++q) {
      const int kx = ax + nb5[q][0], ky = ay + nb5[q][1];
      if (inside(kx, ky)) acc += gval(ax, ay, kx, ky) * g2val(kx, ky, bx, by);
    }
    return acc;
  };
  const int reach = family == DL_MODEL_DIFFUSION ? 3 : 2;
  for (int iy = 0; iy < nx; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      const int s = iy * nx + ix;
      for (int dy = -reach; dy <= reach; ++dy)
        for (int dx = -reach; dx <= reach; ++dx) {
          if (abs(dx) + abs(dy) > reach) continue;
          const int jx = ix + dx, jy = iy + dy;
          if (!inside(jx, jy)) continue;
          const double c = (dx == 0 && dy == 0) ? 1.0 : 0.0;
          const double g = gval(ix, iy, jx, jy);
          const double g2 = g2val(ix, iy, jx, jy);
          const double g3 = reach == 3 ? g3val(ix, iy, jx, jy) : 0.0;
          if (c == 0.0 && g == 0.0 && g2 == 0.0 && g3 == 0.0) continue;
          col.push_back(jy * nx + jx);
          vC.push_back(c);
          vG.push_back(g);
          vG2.push_back(g2);
          vG3.push_back(g3);
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
      (st = upload(M->allocs, vG3, &d.sp_G3)) != DL_OK ||
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
  void* dv = nullptr;
  if ((st = dev_alloc(M->allocs, sizeof(ModelDev), &dv)) != DL_OK ||
      hipMemcpy(dv, &M->d, sizeof(ModelDev), hipMemcpyHostToDevice) != hipSuccess) {
    free_all(M->allocs);
    delete M;
    return st != DL_OK ? st : DL_EHIP;
  }
  M->dev = (ModelDev*)dv;
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


// ---- model order <-> BTA order ------------------------------------------------------------
//
// The time-major permutation (Section IV-B, permutation): the latent
// variable (response j, time t, node s) sits at j*nt*ns + t*ns + s in the
// model (response-major) order of Eq. 11 and at t*b + j*ns + s in the BTA
// order, b = nv*ns; the fixed effects (j, r) stay last at the same offset
// in both.  The map is computed from these formulas, nothing is stored.
namespace {
__device__ __forceinline__ int64_t model_index(int64_t k, int64_t nt, int64_t ns, int64_t b) {
  if (k >= nt * b) return k;
  const int64_t t = k / b, rem = k - t * b;
  const int64_t j = rem / ns, sp = rem - j * ns;
  return j * nt * ns + t * ns + sp;
}

__global__ __launch_bounds__(256) void k_permute(const double* __restrict__ src,
                                                 double* __restrict__ dst, int64_t N,
                                                 int64_t nt, int64_t ns, int64_t b,
                                                 int32_t nvec, int32_t to_bta) {
  const int64_t tot = N * (int64_t)nvec;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * 256) {
    const int64_t v = i / N, k = i - v * N;
    const int64_t mk = model_index(k, nt, ns, b);
    if (to_bta)
      dst[v * N + k] = src[v * N + mk];
    else
      dst[v * N + mk] = src[v * N + k];
  }
}

dl_status permute(const dl_model* M, const double* src, double* dst, int32_t nvec,
                  int to_bta, void* stream) {
  if (!M || !src || !dst || nvec < 0 || src == dst) return DL_EINVAL;
  if (nvec == 0) return DL_OK;
  const dl::ModelDev& m = M->d;
  const int64_t tot = m.N * (int64_t)nvec;
  const int64_t blocks = std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_permute, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     src, dst, m.N, (int64_t)m.nt, (int64_t)m.ns, (int64_t)m.b, nvec, to_bta);
  return hipGetLastError() == hipSuccess ? DL_OK : DL_EHIP;
}
}  // namespace

extern "C" dl_status dl_permute(const dl_model* M, const double* model_dev, double* bta_dev,
                                int32_t nvec, void* stream) {
  return permute(M, model_dev, bta_dev, nvec, 1, stream);
}

extern "C" dl_status dl_unpermute(const dl_model* M, const double* bta_dev, double* model_dev,
                                  int32_t nvec, void* stream) {
  return permute(M, bta_dev, model_dev, nvec, 0, stream);
}
