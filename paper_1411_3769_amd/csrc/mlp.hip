// Warm-start network of the learned form: a three-layer perceptron
// (dims d0 -> d1 -> d2 -> d3, GELU on the hidden layers), its forward and
// backward passes and Adam, on MFMA.
//
// Products run either in FP32 (v_mfma_f32_16x16x4f32, both operands FP32) or
// in BF16 (v_mfma_f32_16x16x16bf16_1k: operands rounded to BF16 with
// nearest-even as they are staged into LDS, so the weights the products see
// are BF16), always with FP32 accumulation.  Master weights, Adam moments,
// activations and gradients are FP32 in HBM.
//
// Parameter layout (one FP32 array): [W1, b1, W2, b2, W3, b3], W_i row-major
// [d_i x d_{i-1}].  Activations are row-major [batch x width].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>

#include "internal.h"

struct psdp_mlp {
  int dims[4];
  int prec;            // PSDP_PREC_FP32 or PSDP_PREC_BF16
  int max_batch;
  int64_t nparam;
  int64_t woff[3], boff[3];
  float* params;       // master weights
  float* grads;
  float* m1;           // Adam first moment
  float* m2;           // Adam second moment
  float* z[3];         // pre-activations per layer [max_batch x d_i]
  float* a[2];         // hidden activations
  float* dz;           // scratch gradient buffers (two of max width)
  float* dz2;
  double* lossbuf;
  int step;
};

namespace psdp {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ inline unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

enum Epi {
  EPI_STORE = 0,       // C = acc
  EPI_BIAS_GELU = 1,   // C = acc + bias (pre-activation), Act = gelu(C)
  EPI_BIAS = 2,        // C = acc + bias
  EPI_GELU_BWD = 3,    // C = acc * gelu'(Zpre)
};

constexpr int kT = 64;    // output tile
constexpr int kKC = 16;   // depth staged per step

// C[M x N] = op(A)[M x K] op(B)[K x N]; op(A)(m,k) = TA ? A[k lda + m] : A[m lda + k],
// op(B)(k,n) = TB ? B[n ldb + k] : B[k ldb + n].  One 64 x 64 tile per
// workgroup of four waves (2 x 2 quadrants of 32 x 32 = 2 x 2 MFMA tiles).
template <int PR, bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_mlp_gemm(int M, int N, int K, const float* __restrict__ A,
                                                  int lda, const float* __restrict__ B, int ldb,
                                                  float* __restrict__ C, const float* __restrict__ bias,
                                                  float* __restrict__ Act,
                                                  const float* __restrict__ Zpre) {
  typedef typename std::conditional<PR == 2, unsigned short, float>::type st_t;
  __shared__ st_t sA[kT * (kKC + 1)];   // [m][k]
  __shared__ st_t sB[kT * (kKC + 1)];   // [n][k]
  const int m0 = blockIdx.y * kT, n0 = blockIdx.x * kT;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int r16 = lane & 15, kq = lane >> 4;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += kKC) {
    __syncthreads();
    for (int e = tid; e < kT * kKC; e += 256) {
      int r, k;
      if (TA) { k = e / kT; r = e % kT; } else { r = e / kKC; k = e % kKC; }
      const int gm = m0 + r, gk = k0 + k;
      float v = 0.f;
      if (gm < M && gk < K) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      if constexpr (PR == 2) sA[r * (kKC + 1) + k] = f2bf(v);
      else sA[r * (kKC + 1) + k] = v;
    }
    for (int e = tid; e < kT * kKC; e += 256) {
      int c, k;
      if (TB) { c = e / kKC; k = e % kKC; } else { k = e / kT; c = e % kT; }
      const int gn = n0 + c, gk = k0 + k;
      float v = 0.f;
      if (gn < N && gk < K) v = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      if constexpr (PR == 2) sB[c * (kKC + 1) + k] = f2bf(v);
      else sB[c * (kKC + 1) + k] = v;
    }
    __syncthreads();
    if constexpr (PR == 2) {
      v4s af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          af[i][j] = (short)sA[(wm + 16 * i + r16) * (kKC + 1) + 4 * kq + j];
          bfr[i][j] = (short)sB[(wn + 16 * i + r16) * (kKC + 1) + 4 * kq + j];
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int ks = 0; ks < kKC; ks += 4) {
        float af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          af[i] = sA[(wm + 16 * i + r16) * (kKC + 1) + ks + kq];
          bfr[i] = sB[(wn + 16 * i + r16) * (kKC + 1) + ks + kq];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + wm + 16 * i + 4 * kq + q;
        const int gn = n0 + wn + 16 * j + r16;
        if (gm >= M || gn >= N) continue;
        float v = acc[i][j][q];
        const int64_t o = (int64_t)gm * N + gn;
        if (EPI == EPI_BIAS_GELU) {
          v += bias[gn];
          C[o] = v;
          Act[o] = gelu_f(v);
        } else if (EPI == EPI_BIAS) {
          C[o] = v + bias[gn];
        } else if (EPI == EPI_GELU_BWD) {
          C[o] = v * gelu_grad_f(Zpre[o]);
        } else {
          C[o] = v;
        }
      }
}

// dOut = (out - t) / B; loss = sum (out - t)^2 / (2 B), one workgroup
__global__ void __launch_bounds__(1024) k_mse(int64_t total, int batch, const float* __restrict__ out,
                                              const float* __restrict__ t, float* __restrict__ d,
                                              double* loss) {
  __shared__ double sb[1024];
  double acc = 0.0;
  const float inv = 1.0f / (float)batch;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const float df = out[e] - t[e];
    d[e] = df * inv;
    acc += (double)df * (double)df;
  }
  sb[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sb[threadIdx.x] += sb[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sb[0] / (2.0 * batch);
}

// db[n] = sum_m dZ[m][n]
__global__ void k_colsum(int M, int N, const float* __restrict__ dZ, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(int64_t)m * N + n];
  db[n] = s;
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m1, float* __restrict__ m2, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float m = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = m;
    m2[i] = v;
    p[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
}

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t st, int prec, int M, int N, int K, const float* A, int lda, const float* B,
          int ldb, float* C, const float* bias = nullptr, float* Act = nullptr,
          const float* Zpre = nullptr) {
  const dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT);
  if (prec == PSDP_PREC_BF16)
    hipLaunchKernelGGL((k_mlp_gemm<2, TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb,
                       C, bias, Act, Zpre);
  else
    hipLaunchKernelGGL((k_mlp_gemm<1, TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb,
                       C, bias, Act, Zpre);
}

// forward: z_i = a_{i-1} W_i^T + b_i; hidden a_i = gelu(z_i)
void forward(psdp_mlp* m, const float* x, int batch, float* out, hipStream_t st) {
  const float* in = x;
  for (int l = 0; l < 3; ++l) {
    const int din = m->dims[l], dout = m->dims[l + 1];
    const float* Wl = m->params + m->woff[l];
    const float* bl = m->params + m->boff[l];
    float* zl = (l == 2 && out) ? out : m->z[l];
    if (l < 2)
      gemm<false, true, EPI_BIAS_GELU>(st, m->prec, batch, dout, din, in, din, Wl, din, zl, bl, m->a[l]);
    else
      gemm<false, true, EPI_BIAS>(st, m->prec, batch, dout, din, in, din, Wl, din, zl, bl);
    if (l < 2) in = m->a[l];
  }
}

}  // namespace
}  // namespace psdp

using namespace psdp;

static int mlp_fail(int code, const std::string& msg) { return psdp::fail(code, msg); }

#define MLP_HIP(x)                                                                \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) return mlp_fail(PSDP_EDEVICE, hipGetErrorString(e_));   \
  } while (0)

extern "C" {

int psdp_mlp_create(const int* dims, int precision, int max_batch, psdp_mlp** out) {
  if (!out || !dims) return mlp_fail(PSDP_EINVAL, "NULL argument");
  *out = nullptr;
  if (precision != PSDP_PREC_FP32 && precision != PSDP_PREC_BF16)
    return mlp_fail(PSDP_EINVAL, "precision must be FP32 or BF16");
  if (max_batch < 1 || max_batch > 65536) return mlp_fail(PSDP_EINVAL, "max_batch out of range");
  for (int i = 0; i < 4; ++i)
    if (dims[i] < 1 || dims[i] > (1 << 20)) return mlp_fail(PSDP_EINVAL, "layer width out of range");
  psdp_mlp* m = new psdp_mlp();
  std::memcpy(m->dims, dims, sizeof(m->dims));
  m->prec = precision;
  m->max_batch = max_batch;
  int64_t o = 0;
  int wmax = 0;
  for (int l = 0; l < 3; ++l) {
    m->woff[l] = o;
    o += (int64_t)dims[l + 1] * dims[l];
    m->boff[l] = o;
    o += dims[l + 1];
  }
  for (int i = 0; i < 4; ++i) wmax = dims[i] > wmax ? dims[i] : wmax;
  m->nparam = o;
  const int64_t act = (int64_t)max_batch * wmax;
  float* base = nullptr;
  const int64_t total = 4 * o + 7 * act;
  if (hipMalloc(&base, total * sizeof(float)) != hipSuccess) {
    delete m;
    return mlp_fail(PSDP_ENOMEM, "hipMalloc of the network buffers failed");
  }
  m->params = base;
  m->grads = base + o;
  m->m1 = base + 2 * o;
  m->m2 = base + 3 * o;
  float* ab = base + 4 * o;
  m->z[0] = ab; m->z[1] = ab + act; m->z[2] = ab + 2 * act;
  m->a[0] = ab + 3 * act; m->a[1] = ab + 4 * act;
  m->dz = ab + 5 * act; m->dz2 = ab + 6 * act;
  if (hipMalloc(&m->lossbuf, sizeof(double)) != hipSuccess) {
    hipFree(base);
    delete m;
    return mlp_fail(PSDP_ENOMEM, "hipMalloc failed");
  }
  if (hipMemset(base, 0, total * sizeof(float)) != hipSuccess) {
    hipFree(base);
    hipFree(m->lossbuf);
    delete m;
    return mlp_fail(PSDP_EDEVICE, "hipMemset failed");
  }
  m->step = 0;
  *out = m;
  return PSDP_OK;
}

int64_t psdp_mlp_param_count(const psdp_mlp* m) { return m ? m->nparam : -1; }

int psdp_mlp_set_params(psdp_mlp* m, const float* host) {
  if (!m || !host) return mlp_fail(PSDP_EINVAL, "NULL argument");
  for (int64_t i = 0; i < m->nparam; ++i)
    if (!std::isfinite(host[i])) return mlp_fail(PSDP_EINVAL, "non-finite parameter");
  MLP_HIP(hipMemcpy(m->params, host, m->nparam * sizeof(float), hipMemcpyHostToDevice));
  MLP_HIP(hipMemset(m->m1, 0, 2 * m->nparam * sizeof(float)));
  m->step = 0;
  return PSDP_OK;
}

int psdp_mlp_get_params(const psdp_mlp* m, float* host, float* grad_host) {
  if (!m) return mlp_fail(PSDP_EINVAL, "NULL argument");
  if (host) MLP_HIP(hipMemcpy(host, m->params, m->nparam * sizeof(float), hipMemcpyDeviceToHost));
  if (grad_host) MLP_HIP(hipMemcpy(grad_host, m->grads, m->nparam * sizeof(float), hipMemcpyDeviceToHost));
  return PSDP_OK;
}

int psdp_mlp_forward(psdp_mlp* m, const float* x, int batch, float* out, void* stream) {
  if (!m || !x || !out) return mlp_fail(PSDP_EINVAL, "NULL argument");
  if (batch < 1 || batch > m->max_batch) return mlp_fail(PSDP_EINVAL, "batch out of range");
  hipStream_t st = (hipStream_t)stream;
  forward(m, x, batch, out, st);
  MLP_HIP(hipGetLastError());
  MLP_HIP(hipStreamSynchronize(st));
  return PSDP_OK;
}

int psdp_mlp_loss_grad(psdp_mlp* m, const float* x, const float* t, int batch, double* loss,
                       void* stream) {
  if (!m || !x || !t) return mlp_fail(PSDP_EINVAL, "NULL argument");
  if (batch < 1 || batch > m->max_batch) return mlp_fail(PSDP_EINVAL, "batch out of range");
  hipStream_t st = (hipStream_t)stream;
  forward(m, x, batch, nullptr, st);
  const int d3 = m->dims[3];
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, st, (int64_t)batch * d3, batch, m->z[2], t, m->dz,
                     m->lossbuf);
  // dZ of layer l is in cur; walk the layers backwards
  float* cur = m->dz;
  float* nxt = m->dz2;
  for (int l = 2; l >= 0; --l) {
    const int din = m->dims[l], dout = m->dims[l + 1];
    const float* ain = l == 0 ? x : m->a[l - 1];
    // dW_l = dZ^T a_in  [dout x din]
    gemm<true, false, EPI_STORE>(st, m->prec, dout, din, batch, cur, dout, ain, din,
                                 m->grads + m->woff[l]);
    hipLaunchKernelGGL(k_colsum, dim3((dout + 255) / 256), dim3(256), 0, st, batch, dout, cur,
                       m->grads + m->boff[l]);
    if (l > 0) {
      // dZ_{l-1} = (dZ W_l) * gelu'(z_{l-1})  [batch x din]
      gemm<false, false, EPI_GELU_BWD>(st, m->prec, batch, din, dout, cur, dout,
                                       m->params + m->woff[l], din, nxt, nullptr, nullptr, m->z[l - 1]);
      float* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
  }
  MLP_HIP(hipGetLastError());
  if (loss) MLP_HIP(hipMemcpyAsync(loss, m->lossbuf, sizeof(double), hipMemcpyDeviceToHost, st));
  MLP_HIP(hipStreamSynchronize(st));
  return PSDP_OK;
}

int psdp_mlp_adam(psdp_mlp* m, float lr, float b1, float b2, float eps, void* stream) {
  if (!m) return mlp_fail(PSDP_EINVAL, "NULL argument");
  if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps >= 0))
    return mlp_fail(PSDP_EINVAL, "invalid Adam parameters");
  hipStream_t st = (hipStream_t)stream;
  m->step += 1;
  const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, st, m->nparam, m->params, m->grads, m->m1,
                     m->m2, lr, b1, b2, eps, c1, c2);
  MLP_HIP(hipGetLastError());
  MLP_HIP(hipStreamSynchronize(st));
  return PSDP_OK;
}

void psdp_mlp_free(psdp_mlp* m) {
  if (!m) return;
  hipFree(m->params);
  hipFree(m->lossbuf);
  delete m;
}

}  // extern "C"
