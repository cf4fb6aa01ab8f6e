// Surrogate network kernels: a multi-layer perceptron x -> SiLU(W1 x + b1)
// -> ... -> W_L h + b_L trained on the GPU.  Weights are kept in FP32
// (master copy, Adam moments); every matrix product rounds both operands to
// bfloat16 (round to nearest even) and runs on v_mfma_f32_16x16x16_bf16 with
// FP32 accumulation.
#include <math.h>
#include <stdint.h>

#include <new>
#include <vector>

#include "engine.hpp"

namespace dl {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// C[m][n] = act(alpha * sum_k A(m,k) B(n,k) + bias[n]) (+ beta * C_old),
// A(m,k) = A[m*sam + k*sak], B(n,k) = B[n*sbn + k*sbk] (FP32, any strides),
// Z (pre-activation) and H (output) row-major with leading dims ldz / ldh.
// One workgroup (4 waves) per 64x64 tile; the k loop stages 16-deep bf16
// chunks in LDS.  MFMA operands: op(B) as "A" and op(A) as "B", so the
// accumulator holds C^T and lane l, register r is C[m0 + l%16][n0 + 4(l/16)
// + r] within its 16x16 block.
struct LinJob {
  int M, N, K;
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbn, sbk;
  const float* bias;
  float alpha, beta;
  float* Z;
  int64_t ldz;
  float* H;
  int64_t ldh;
  int act;  // 0 none, 1 SiLU
};

__global__ __launch_bounds__(256) void k_mlp_linear(LinJob J) {
  __shared__ unsigned short As[64][16 + 4];
  __shared__ unsigned short Bs[64][16 + 4];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l16 = lane & 15, lg = lane >> 4;
  v4f acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < J.K; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int r = e >> 4, kk = e & 15;
      const int k = k0 + kk;
      const int m = m0 + r, n = n0 + r;
      const float a = (m < J.M && k < J.K) ? J.A[(int64_t)m * J.sam + (int64_t)k * J.sak] : 0.f;
      const float b = (n < J.N && k < J.K) ? J.B[(int64_t)n * J.sbn + (int64_t)k * J.sbk] : 0.f;
      As[r][kk] = f2bf(a);
      Bs[r][kk] = f2bf(b);
    }
    __syncthreads();
    v4s fa[2], fb[2];
    for (int i = 0; i < 2; ++i) {
      const unsigned short* p = &As[wm * 32 + i * 16 + l16][4 * lg];
      fa[i] = (v4s){(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
    }
    for (int j = 0; j < 2; ++j) {
      const unsigned short* p = &Bs[wn * 32 + j * 16 + l16][4 * lg];
      fb[j] = (v4s){(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fb[j], fa[i], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + wm * 32 + i * 16 + l16;
    if (m >= J.M) continue;
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int n = n0 + wn * 32 + j * 16 + 4 * lg + r;
        if (n >= J.N) continue;
        float z = J.alpha * acc[i][j][r] + (J.bias ? J.bias[n] : 0.f);
        if (J.Z) J.Z[(int64_t)m * J.ldz + n] = z;
        float h = z;
        if (J.act == 1) h = z / (1.f + expf(-z));
        if (J.H) {
          float* p = J.H + (int64_t)m * J.ldh + n;
          *p = (J.beta != 0.f) ? h + J.beta * (*p) : h;
        }
      }
  }
}

static hipError_t linear(const LinJob& J, hipStream_t s) {
  if (J.M <= 0 || J.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_linear, dim3((J.M + 63) / 64, (J.N + 63) / 64), dim3(256),
                     0, s, J);
  return hipGetLastError();
}

// dZ = dH * SiLU'(Z)
__global__ void k_silu_bwd(int64_t n, const float* dH, const float* Z, float* dZ) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float z = Z[i];
    const float sg = 1.f / (1.f + expf(-z));
    dZ[i] = dH[i] * sg * (1.f + z * (1.f - sg));
  }
}

// out[n] = sum over rows m of X[m*ld + n] (fixed order per column)
__global__ void k_colsum(int M, int N, const float* X, int64_t ld, float* out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += X[(int64_t)m * ld + n];
  out[n] = s;
}

// dy = 2 (yhat - y) / n; loss = mean (yhat - y)^2 (one block, fixed tree)
__global__ void k_mse(int n, const float* yhat, const float* y, float* dy, float* loss) {
  __shared__ float sh[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float r = yhat[i] - y[i];
    dy[i] = 2.f * r / (float)n;
    acc += r * r;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = sh[0] / (float)n;
}

// Adam (Kingma & Ba) on a flat parameter vector.
__global__ void k_adam(int64_t n, float* w, const float* g, float* m, float* v,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace dl

using namespace dl;

struct dl_mlp {
  std::vector<int> sizes;   // in, hidden..., out
  int max_batch = 0;
  int64_t nparam = 0;
  std::vector<int64_t> woff, boff;  // offsets of W_k (out x in, row-major), b_k
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  std::vector<float*> Z, Hs;  // pre-activations and layer inputs (H[0] = X copy)
  float *dA = nullptr, *dB = nullptr;  // gradient scratch (max_batch x max width)
  float *yhat = nullptr, *dy = nullptr, *loss = nullptr;
  int step = 0;
  int last_n = 0;
  std::vector<void*> allocs;
};

extern "C" dl_status dl_mlp_create(const int32_t* sizes, int32_t nsizes,
                                   int32_t max_batch, dl_mlp** out) {
  if (!sizes || nsizes < 2 || max_batch <= 0 || !out) return DL_EINVAL;
  for (int k = 0; k < nsizes; ++k)
    if (sizes[k] <= 0) return DL_EINVAL;
  if (sizes[nsizes - 1] != 1) return DL_EINVAL;
  dl_mlp* N = new (std::nothrow) dl_mlp();
  if (!N) return DL_ENOMEM;
  N->sizes.assign(sizes, sizes + nsizes);
  N->max_batch = max_batch;
  int64_t off = 0;
  int wmax = 0;
  for (int k = 0; k + 1 < nsizes; ++k) {
    N->woff.push_back(off);
    off += (int64_t)sizes[k] * sizes[k + 1];
    N->boff.push_back(off);
    off += sizes[k + 1];
  }
  for (int k = 0; k < nsizes; ++k) wmax = std::max(wmax, sizes[k]);
  N->nparam = off;
  dl_status st = DL_OK;
  auto A = [&](size_t bytes, void** p) {
    if (st == DL_OK) st = dev_alloc(N->allocs, bytes, p);
  };
  A(sizeof(float) * off, (void**)&N->w);
  A(sizeof(float) * off, (void**)&N->g);
  A(sizeof(float) * off, (void**)&N->m);
  A(sizeof(float) * off, (void**)&N->v);
  const int L = nsizes - 1;
  N->Z.resize(L);
  N->Hs.resize(L);
  for (int k = 0; k < L; ++k) {
    A(sizeof(float) * (size_t)max_batch * sizes[k + 1], (void**)&N->Z[k]);
    A(sizeof(float) * (size_t)max_batch * sizes[k], (void**)&N->Hs[k]);
  }
  A(sizeof(float) * (size_t)max_batch * wmax, (void**)&N->dA);
  A(sizeof(float) * (size_t)max_batch * wmax, (void**)&N->dB);
  A(sizeof(float) * max_batch, (void**)&N->yhat);
  A(sizeof(float) * max_batch, (void**)&N->dy);
  A(sizeof(float) * 4, (void**)&N->loss);
  if (st == DL_OK &&
      (hipMemset(N->m, 0, sizeof(float) * off) != hipSuccess ||
       hipMemset(N->v, 0, sizeof(float) * off) != hipSuccess))
    st = DL_EHIP;
  if (st != DL_OK) {
    free_all(N->allocs);
    delete N;
    return st;
  }
  *out = N;
  return DL_OK;
}

extern "C" void dl_mlp_destroy(dl_mlp* N) {
  if (!N) return;
  free_all(N->allocs);
  delete N;
}

extern "C" dl_status dl_mlp_params(dl_mlp* N, float** params_dev, float** grads_dev,
                                   int64_t* count) {
  if (!N) return DL_EINVAL;
  if (params_dev) *params_dev = N->w;
  if (grads_dev) *grads_dev = N->g;
  if (count) *count = N->nparam;
  return DL_OK;
}

extern "C" dl_status mlp_fwd(dl_mlp* N, const float* X, int32_t n, float* yhat,
                             void* stream) {
  if (!N || !X || n <= 0 || n > N->max_batch) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int L = (int)N->sizes.size() - 1;
  const float* hin = X;
  int64_t ldin = N->sizes[0];
  DL_HIP_CHECK(hipMemcpyAsync(N->Hs[0], X, sizeof(float) * (size_t)n * N->sizes[0],
                              hipMemcpyDeviceToDevice, s));
  hin = N->Hs[0];
  for (int k = 0; k < L; ++k) {
    const int in = N->sizes[k], outw = N->sizes[k + 1];
    LinJob J{};
    J.M = n; J.N = outw; J.K = in;
    J.A = hin; J.sam = ldin; J.sak = 1;
    J.B = N->w + N->woff[k]; J.sbn = in; J.sbk = 1;
    J.bias = N->w + N->boff[k];
    J.alpha = 1.f; J.beta = 0.f;
    J.Z = N->Z[k]; J.ldz = outw;
    const bool lastl = (k + 1 == L);
    J.H = lastl ? N->yhat : N->Hs[k + 1];
    J.ldh = outw;
    J.act = lastl ? 0 : 1;
    DL_HIP_CHECK(linear(J, s));
    hin = J.H;
    ldin = outw;
  }
  if (yhat)
    DL_HIP_CHECK(hipMemcpyAsync(yhat, N->yhat, sizeof(float) * n,
                                hipMemcpyDeviceToDevice, s));
  N->last_n = n;
  return DL_OK;
}

// Backward of the last mlp_fwd: dy (n) -> parameter gradients (overwritten)
// and, when dX != NULL, d(sum dy*yhat)/dX (n x in, row-major).
extern "C" dl_status mlp_bwd(dl_mlp* N, const float* dy, int32_t n, float* dX,
                             void* stream) {
  if (!N || !dy || n != N->last_n) return DL_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int L = (int)N->sizes.size() - 1;
  // g = dL/dZ_L (n x 1) = dy
  DL_HIP_CHECK(hipMemcpyAsync(N->dA, dy, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
  float* g = N->dA;     // current dL/dZ_k (n x out_k)
  float* other = N->dB;
  for (int k = L - 1; k >= 0; --k) {
    const int in = N->sizes[k], outw = N->sizes[k + 1];
    // dW_k = g^T H_k  (outw x in):  C[o][i] = sum_m g[m][o] H[m][i]
    LinJob Jw{};
    Jw.M = outw; Jw.N = in; Jw.K = n;
    Jw.A = g; Jw.sam = 1; Jw.sak = outw;
    Jw.B = N->Hs[k]; Jw.sbn = 1; Jw.sbk = in;
    Jw.alpha = 1.f; Jw.beta = 0.f;
    Jw.H = N->g + N->woff[k]; Jw.ldh = in;
    DL_HIP_CHECK(linear(Jw, s));
    hipLaunchKernelGGL(k_colsum, dim3((outw + 255) / 256), dim3(256), 0, s, n, outw,
                       g, (int64_t)outw, N->g + N->boff[k]);
    DL_HIP_CHECK(hipGetLastError());
    if (k == 0 && !dX) break;
    // dH_k = g W_k  (n x in): C[m][i] = sum_o g[m][o] W[o][i]
    LinJob Jh{};
    Jh.M = n; Jh.N = in; Jh.K = outw;
    Jh.A = g; Jh.sam = outw; Jh.sak = 1;
    Jh.B = N->w + N->woff[k]; Jh.sbn = 1; Jh.sbk = in;
    Jh.alpha = 1.f; Jh.beta = 0.f;
    Jh.H = (k == 0) ? dX : other; Jh.ldh = in;
    DL_HIP_CHECK(linear(Jh, s));
    if (k == 0) break;
    // dZ_{k-1} = dH_k * SiLU'(Z_{k-1})
    const int64_t cnt = (int64_t)n * in;
    hipLaunchKernelGGL(k_silu_bwd, dim3((unsigned)std::min<int64_t>(1024, (cnt + 255) / 256)),
                       dim3(256), 0, s, cnt, other, N->Z[k - 1], other);
    DL_HIP_CHECK(hipGetLastError());
    std::swap(g, other);
  }
  return DL_OK;
}

// dy = 2 (yhat - y)/n from the last forward's output; loss_dev[0] = MSE.
extern "C" dl_status mlp_mse_grad(dl_mlp* N, const float* y, int32_t n, float* dy,
                                  float* loss_dev, void* stream) {
  if (!N || !y || !dy || n != N->last_n) return DL_EINVAL;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, (hipStream_t)stream, n, N->yhat,
                     y, dy, loss_dev);
  DL_HIP_CHECK(hipGetLastError());
  return DL_OK;
}

extern "C" dl_status mlp_adam(dl_mlp* N, float lr, float b1, float b2, float eps,
                              void* stream) {
  if (!N) return DL_EINVAL;
  N->step += 1;
  const float c1 = 1.f - powf(b1, (float)N->step);
  const float c2 = 1.f - powf(b2, (float)N->step);
  hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, (hipStream_t)stream, N->nparam,
                     N->w, N->g, N->m, N->v, lr, b1, b2, eps, c1, c2);
  DL_HIP_CHECK(hipGetLastError());
  return DL_OK;
}
