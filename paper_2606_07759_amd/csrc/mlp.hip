// Small multilayer perceptron for misregistration estimation: forward,
// backward (MSE loss) and Adam, hand-written for gfx950 in FP32.
//
// Net: x (n_in) -> h1 -> h2 -> n_out, y = x W^T + b per layer, ReLU after the
// two hidden layers.  Parameters are one packed buffer:
//   W1 [h1][n_in], b1 [h1], W2 [h2][h1], b2 [h2], W3 [n_out][h2], b3 [n_out].
// Inputs arrive compact: the input layer's non-zero inputs lie in two column
// segments of the full input (the rest is identically zero), so x is
// [B][len0 + len1] and compact column c feeds W1 column seg0 + c (c < len0) or
// seg1 + c - len0; the zero inputs contribute nothing and are skipped exactly.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace synim {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;   // GEMM tile: 256 threads, 4x4 outputs each

// C[M][N] = alpha * op(A) op(B) + beta * C (+ bias[n]) (then ReLU if relu).
// op(A) is M x K (A stored [M][lda] or, transposed, [K][lda]); op(B) is K x N
// (B stored [K][ldb] or, transposed, [N][ldb]).  FP32 FMA on 64x64 tiles
// staged through LDS, 4x4 outputs per thread.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, float alpha,
                                                   const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb,
                                                   float beta, float* __restrict__ C, int ldc,
                                                   const float* __restrict__ bias, int relu) {
  __shared__ float As[BK][BM + 4];
  __shared__ float Bs[BK][BN + 4];
  const int tid = threadIdx.x;
  const int tm = tid / 16, tn = tid % 16;   // 16 x 16 threads, 4 x 4 outputs each
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += BK) {
    // A tile: BM x BK elements, 4 per thread
    for (int e = tid; e < BM * BK; e += 256) {
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      const int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < K) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      As[kk][mm] = v;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      int nn, kk;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      const int gn = n0 + nn, gk = k0 + kk;
      float v = 0.f;
      if (gn < N && gk < K) v = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __fmaf_rn(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + tm * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tn * 4 + j;
      if (gn >= N) continue;
      float v = alpha * acc[i][j];
      if (beta != 0.f) v += beta * C[(size_t)gm * ldc + gn];
      if (bias) v += bias[gn];
      if (relu) v = fmaxf(v, 0.f);
      C[(size_t)gm * ldc + gn] = v;
    }
  }
}

template <bool TA, bool TB>
int gemm(int M, int N, int K, float alpha, const float* A, int lda, const float* B, int ldb,
         float beta, float* C, int ldc, const float* bias, int relu, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return SYNIM_OK;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
  if (grid.y > 65535) return SYNIM_E_SHAPE;
  hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, B,
                     ldb, beta, C, ldc, bias, relu);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

// Small batches (B <= 16): one workgroup per output unit, lanes split K, so the
// weight rows stream once at full bandwidth.  x [B][ldx], W rows of length ldw
// with the compact-to-full column map (seg0, len0, seg1) for the input layer.
template <int MB>
__global__ __launch_bounds__(256) void linear_small_kernel(int B, int N, int K,
                                                           const float* __restrict__ x, int ldx,
                                                           const float* __restrict__ W, int ldw,
                                                           int seg0, int len0, int seg1,
                                                           const float* __restrict__ bias,
                                                           int relu, float* __restrict__ y,
                                                           int ldy) {
  const int n = blockIdx.x;
  const float* w = W + (size_t)n * ldw;
  float acc[MB] = {};
  for (int k = threadIdx.x; k < K; k += 256) {
    const int col = k < len0 ? seg0 + k : seg1 + (k - len0);
    const float wk = w[col];
#pragma unroll
    for (int b = 0; b < MB; ++b)
      if (b < B) acc[b] = __fmaf_rn(wk, x[(size_t)b * ldx + k], acc[b]);
  }
  __shared__ float red[MB][256];
#pragma unroll
  for (int b = 0; b < MB; ++b) red[b][threadIdx.x] = acc[b];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int b = 0; b < MB; ++b) red[b][threadIdx.x] += red[b][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < MB && threadIdx.x < B) {
    float v = red[threadIdx.x][0] + (bias ? bias[n] : 0.f);
    if (relu) v = fmaxf(v, 0.f);
    y[(size_t)threadIdx.x * ldy + n] = v;
  }
}

__global__ void relu_mask_kernel(float* __restrict__ g, const float* __restrict__ h, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(h[i] > 0.f)) g[i] = 0.f;
}

// Column sums of g [B][N] (bias gradients), fixed order.
__global__ void colsum_kernel(const float* __restrict__ g, int B, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += g[(size_t)b * N + n];
  out[n] = s;
}

// dY = 2 (Y - T) / (B * n_out) and the MSE loss (one workgroup).
__global__ void mse_grad_kernel(const float* __restrict__ y, const float* __restrict__ t, int n,
                                float scale, float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d * scale;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] * scale;
}

// One Adam step.  The coefficients come from the host, formed in double from
// the double hyperparameters (1 - beta2 in float would lose five digits).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, long n, float lr,
                            float b1, float omb1, float b2, float omb2, float eps, float inv_c1,
                            float inv_c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * (gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
}

__global__ void scatter_cols_kernel(const float* __restrict__ src, int N, int K, int seg0,
                                    int len0, int seg1, float* __restrict__ dst, int ldd) {
  // dst[n][col(k)] = src[n][k] for the compact-to-full column map
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * K) return;
  const int n = (int)(i / K), k = (int)(i - (long)n * K);
  const int col = k < len0 ? seg0 + k : seg1 + (k - len0);
  dst[(size_t)n * ldd + col] = src[i];
}

__global__ void gather_cols_kernel(const float* __restrict__ W, int N, int K, int seg0, int len0,
                                   int seg1, int ldw, float* __restrict__ dst) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * K) return;
  const int n = (int)(i / K), k = (int)(i - (long)n * K);
  const int col = k < len0 ? seg0 + k : seg1 + (k - len0);
  dst[i] = W[(size_t)n * ldw + col];
}

struct Layout {
  size_t w1, b1, w2, b2, w3, b3, total;
};

Layout params_layout(const synim_mlp& net) {
  Layout L{};
  L.w1 = 0;
  L.b1 = L.w1 + (size_t)net.h1 * net.n_in;
  L.w2 = L.b1 + net.h1;
  L.b2 = L.w2 + (size_t)net.h2 * net.h1;
  L.w3 = L.b2 + net.h2;
  L.b3 = L.w3 + (size_t)net.n_out * net.h2;
  L.total = L.b3 + net.n_out;
  return L;
}

int check_net(const synim_mlp* net) {
  if (!net) return SYNIM_E_NULL;
  if (net->n_in < 1 || net->h1 < 1 || net->h2 < 1 || net->n_out < 1) return SYNIM_E_SHAPE;
  if (net->len0 < 0 || net->len1 < 0 || net->len0 + net->len1 < 1) return SYNIM_E_SHAPE;
  if (net->seg0 < 0 || net->seg0 + net->len0 > net->n_in || net->seg1 < 0 ||
      net->seg1 + net->len1 > net->n_in)
    return SYNIM_E_SHAPE;
  if (net->len0 > 0 && net->len1 > 0 && net->seg0 + net->len0 > net->seg1 &&
      net->seg1 + net->len1 > net->seg0)
    return SYNIM_E_SHAPE;   // overlapping segments
  return SYNIM_OK;
}

// Caller's scratch (floats): h1 [B][h1], h2 [B][h2] kept from the forward pass
// for the backward pass, then dy [B][n_out], dh2 [B][h2], dh1 [B][h1], and the
// used W1 columns (forward) or their gradient (backward) [h1][K].
struct Scratch {
  float *h1, *h2, *dy, *dh2, *dh1, *w1c;
  size_t total;
};

Scratch scratch_layout(const synim_mlp& net, int B, float* base) {
  const size_t K = (size_t)net.len0 + net.len1;
  Scratch S{};
  size_t off = 0;
  auto take = [&](size_t n) {
    float* p = base ? base + off : nullptr;
    off += n;
    return p;
  };
  S.h1 = take((size_t)B * net.h1);
  S.h2 = take((size_t)B * net.h2);
  S.dy = take((size_t)B * net.n_out);
  S.dh2 = take((size_t)B * net.h2);
  S.dh1 = take((size_t)B * net.h1);
  S.w1c = take((size_t)net.h1 * K);
  S.total = off;
  return S;
}

__global__ void fill_zero_kernel(float* __restrict__ p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

}  // namespace
}  // namespace synim

using namespace synim;

extern "C" size_t synim_mlp_param_count(const synim_mlp* net) {
  if (check_net(net) != SYNIM_OK) return 0;
  return params_layout(*net).total;
}

extern "C" size_t synim_mlp_scratch_floats(const synim_mlp* net, int B) {
  if (check_net(net) != SYNIM_OK || B < 1) return 0;
  return scratch_layout(*net, B, nullptr).total;
}

// Forward pass.  scratch: synim_mlp_scratch_floats floats; y: [B][n_out].
extern "C" int synim_mlp_forward(const synim_mlp* net, const float* params, const float* x, int B,
                                 float* scratch, float* y, void* stream) {
  int rc = check_net(net);
  if (rc != SYNIM_OK) return rc;
  if (!params || !x || !scratch || !y) return SYNIM_E_NULL;
  if (B < 1) return SYNIM_E_SHAPE;
  hipStream_t st = (hipStream_t)stream;
  const Layout L = params_layout(*net);
  const int K = net->len0 + net->len1;
  const Scratch S = scratch_layout(*net, B, scratch);
  float* h1 = S.h1;
  float* h2 = S.h2;
  const float* P = params;
  if (B <= 16) {
    hipLaunchKernelGGL(linear_small_kernel<16>, dim3(net->h1), dim3(256), 0, st, B, net->h1, K,
                       x, K, P + L.w1, net->n_in, net->seg0, net->len0, net->seg1, P + L.b1, 1,
                       h1, net->h1);
    SYNIM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(linear_small_kernel<16>, dim3(net->h2), dim3(256), 0, st, B, net->h2,
                       net->h1, h1, net->h1, P + L.w2, net->h1, 0, net->h1, 0, P + L.b2, 1, h2,
                       net->h2);
    SYNIM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(linear_small_kernel<16>, dim3(net->n_out), dim3(256), 0, st, B,
                       net->n_out, net->h2, h2, net->h2, P + L.w3, net->h2, 0, net->h2, 0,
                       P + L.b3, 0, y, net->n_out);
    SYNIM_HIP_TRY(hipGetLastError());
    return SYNIM_OK;
  }
  // input layer: gather the used W1 columns once, then a dense GEMM
  float* w1c = S.w1c;
  const long nk = (long)net->h1 * K;
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st,
                     P + L.w1, net->h1, K, net->seg0, net->len0, net->seg1, net->n_in, w1c);
  SYNIM_HIP_TRY(hipGetLastError());
  rc = gemm<false, true>(B, net->h1, K, 1.f, x, K, w1c, K, 0.f, h1, net->h1, P + L.b1, 1, st);
  if (rc != SYNIM_OK) return rc;
  rc = gemm<false, true>(B, net->h2, net->h1, 1.f, h1, net->h1, P + L.w2, net->h1, 0.f, h2,
                         net->h2, P + L.b2, 1, st);
  if (rc != SYNIM_OK) return rc;
  return gemm<false, true>(B, net->n_out, net->h2, 1.f, h2, net->h2, P + L.w3, net->h2, 0.f, y,
                           net->n_out, P + L.b3, 0, st);
}

// Backward pass of the MSE loss after synim_mlp_forward on the same x and
// scratch: grads (packed like params, fully overwritten; W1 columns outside
// the segments get 0), loss (device float, nullable) = mean((y - t)^2).
extern "C" int synim_mlp_backward(const synim_mlp* net, const float* params, const float* x,
                                  int B, float* scratch, const float* y, const float* t,
                                  float* grads, float* loss, void* stream) {
  int rc = check_net(net);
  if (rc != SYNIM_OK) return rc;
  if (!params || !x || !scratch || !y || !t || !grads) return SYNIM_E_NULL;
  if (B < 1) return SYNIM_E_SHAPE;
  hipStream_t st = (hipStream_t)stream;
  const Layout L = params_layout(*net);
  const int K = net->len0 + net->len1;
  const Scratch S = scratch_layout(*net, B, scratch);
  float* h1 = S.h1;
  float* h2 = S.h2;
  float* dy = S.dy;
  float* dh2 = S.dh2;
  float* dh1 = S.dh1;
  float* dw1c = S.w1c;   // [h1][K] before scattering into W1's columns
  const float* P = params;
  float* G = grads;
  const int ny = B * net->n_out;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(1), dim3(256), 0, st, y, t, ny, 1.f / ny, dy, loss);
  SYNIM_HIP_TRY(hipGetLastError());
  // layer 3: dW3 = dy^T h2, db3 = sum dy, dh2 = dy W3 (masked by h2 > 0)
  rc = gemm<true, false>(net->n_out, net->h2, B, 1.f, dy, net->n_out, h2, net->h2, 0.f, G + L.w3,
                         net->h2, nullptr, 0, st);
  if (rc != SYNIM_OK) return rc;
  hipLaunchKernelGGL(colsum_kernel, dim3((net->n_out + 255) / 256), dim3(256), 0, st, dy, B,
                     net->n_out, G + L.b3);
  SYNIM_HIP_TRY(hipGetLastError());
  rc = gemm<false, false>(B, net->h2, net->n_out, 1.f, dy, net->n_out, P + L.w3, net->h2, 0.f,
                          dh2, net->h2, nullptr, 0, st);
  if (rc != SYNIM_OK) return rc;
  const long n2 = (long)B * net->h2;
  hipLaunchKernelGGL(relu_mask_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, dh2,
                     h2, n2);
  SYNIM_HIP_TRY(hipGetLastError());
  // layer 2
  rc = gemm<true, false>(net->h2, net->h1, B, 1.f, dh2, net->h2, h1, net->h1, 0.f, G + L.w2,
                         net->h1, nullptr, 0, st);
  if (rc != SYNIM_OK) return rc;
  hipLaunchKernelGGL(colsum_kernel, dim3((net->h2 + 255) / 256), dim3(256), 0, st, dh2, B,
                     net->h2, G + L.b2);
  SYNIM_HIP_TRY(hipGetLastError());
  rc = gemm<false, false>(B, net->h1, net->h2, 1.f, dh2, net->h2, P + L.w2, net->h1, 0.f, dh1,
                          net->h1, nullptr, 0, st);
  if (rc != SYNIM_OK) return rc;
  const long n1 = (long)B * net->h1;
  hipLaunchKernelGGL(relu_mask_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, dh1,
                     h1, n1);
  SYNIM_HIP_TRY(hipGetLastError());
  // layer 1: only the used columns of W1 get gradient, the rest is zero
  rc = gemm<true, false>(net->h1, K, B, 1.f, dh1, net->h1, x, K, 0.f, dw1c, K, nullptr, 0, st);
  if (rc != SYNIM_OK) return rc;
  const long nw1 = (long)net->h1 * net->n_in;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((nw1 + 255) / 256)), dim3(256), 0, st,
                     G + L.w1, nw1);
  SYNIM_HIP_TRY(hipGetLastError());
  const long nk = (long)net->h1 * K;
  hipLaunchKernelGGL(scatter_cols_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st,
                     dw1c, net->h1, K, net->seg0, net->len0, net->seg1, G + L.w1, net->n_in);
  SYNIM_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(colsum_kernel, dim3((net->h1 + 255) / 256), dim3(256), 0, st, dh1, B,
                     net->h1, G + L.b1);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

extern "C" int synim_adam_step(float* params, const float* grads, float* m, float* v, size_t n,
                               int step, double lr, double beta1, double beta2, double eps,
                               void* stream) {
  if (!params || !grads || !m || !v) return SYNIM_E_NULL;
  if (step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
      !(eps >= 0))
    return SYNIM_E_PARAM;
  if (n == 0) return SYNIM_OK;
  const double c1 = 1.0 - std::pow(beta1, (double)step);
  const double c2 = 1.0 - std::pow(beta2, (double)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, params, grads, m, v, (long)n, (float)lr, (float)beta1,
                     (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), (float)eps,
                     (float)(1.0 / c1), (float)(1.0 / c2));
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}
