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

// ------------------------------------------------------------ FP32 GEMM
// C[m][n] = alpha sum_k X(k, m) Y(k, n) (+ beta C[m][n]) (+ bias[n]) (then
// ReLU), X(k, m) = X[k sxk + m sxm], Y(k, n) = Y[k syk + n syn], C row-major.
// On the matrix cores: one 256-thread workgroup per 64x64 tile of C, each wave
// a 32x32 quarter as 2x2 blocks of v_mfma_f32_16x16x4f32 (lane l feeds
// A[l%16][l/16] and B[l/16][l%16] and holds D[4(l/16) + r][l%16], r = 0..3,
// checked on the device).  K advances in chunks of 32 through two LDS buffers,
// the next chunk's global loads in flight while the current one is multiplied.
// Split K: workgroup z of a split launch sums k in [z kc, (z+1) kc) and writes
// its partial tile to part[z][M][N]; gemm_reduce_kernel adds the partials in z
// order (a fixed order: the result does not depend on scheduling) and applies
// alpha, beta, bias and ReLU.
constexpr int MT = 64, MK = 32, MPAD = 1;
constexpr int MLOADS = MT * MK / 256;   // elements of one operand chunk per thread

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct MGemm {
  int M, N, K;
  const float* X;
  long sxk, sxm;
  const float* Y;
  long syk, syn;
  float* C;
  long ldc;
  float alpha, beta;
  const float* bias;
  int relu;
  float* part;   // split launches: [splits][M][N]
  int kc;        // K per split (a multiple of MK)
  int splits;
};

// (kk, mm) of element q of this thread in an MK x MT chunk, consecutive
// threads along the operand's unit stride
__device__ __forceinline__ void mg_elem(long sk, int tid, int q, int& kk, int& mm) {
  const int e = tid + 256 * q;
  if (sk == 1) {
    kk = e % MK;
    mm = e / MK;
  } else {
    kk = e / MT;
    mm = e % MT;
  }
}

__device__ __forceinline__ void mg_fetch(const float* P, long sk, long sm, int k0, int k1, int m0,
                                         int M, int tid, float (&r)[MLOADS]) {
#pragma unroll
  for (int q = 0; q < MLOADS; ++q) {
    int kk, mm;
    mg_elem(sk, tid, q, kk, mm);
    const int k = k0 + kk, m = m0 + mm;
    r[q] = (k < k1 && m < M) ? P[(long)k * sk + (long)m * sm] : 0.f;
  }
}

__device__ __forceinline__ void mg_put(long sk, int tid, const float (&r)[MLOADS],
                                       float (*S)[MT + MPAD]) {
#pragma unroll
  for (int q = 0; q < MLOADS; ++q) {
    int kk, mm;
    mg_elem(sk, tid, q, kk, mm);
    S[kk][mm] = r[q];
  }
}

__device__ __forceinline__ float mg_epilogue(const MGemm& g, float acc, int m, int n) {
  float v = g.alpha * acc;
  if (g.beta != 0.f) v += g.beta * g.C[(long)m * g.ldc + n];
  if (g.bias) v += g.bias[n];
  if (g.relu) v = fmaxf(v, 0.f);
  return v;
}

__global__ __launch_bounds__(256) void gemm_mfma_kernel(MGemm g) {
  const int m0 = blockIdx.y * MT, n0 = blockIdx.x * MT;
  const int kb = blockIdx.z * g.kc, ke = min(g.K, kb + g.kc);
  __shared__ float Xs[2][MK][MT + MPAD], Ys[2][MK][MT + MPAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float rx[MLOADS], ry[MLOADS];
  mg_fetch(g.X, g.sxk, g.sxm, kb, ke, m0, g.M, tid, rx);
  mg_fetch(g.Y, g.syk, g.syn, kb, ke, n0, g.N, tid, ry);
  mg_put(g.sxk, tid, rx, Xs[0]);
  mg_put(g.syk, tid, ry, Ys[0]);
  __syncthreads();
  const int nk = ke > kb ? (ke - kb + MK - 1) / MK : 0;
  for (int c = 0; c < nk; ++c) {
    const int buf = c & 1;
    const bool more = c + 1 < nk;
    if (more) {
      mg_fetch(g.X, g.sxk, g.sxm, kb + (c + 1) * MK, ke, m0, g.M, tid, rx);
      mg_fetch(g.Y, g.syk, g.syn, kb + (c + 1) * MK, ke, n0, g.N, tid, ry);
    }
#pragma unroll
    for (int s = 0; s < MK / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Xs[buf][kr][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Ys[buf][kr][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      // the other buffer was last read in iteration c - 1, before its closing barrier
      mg_put(g.sxk, tid, rx, Xs[buf ^ 1]);
      mg_put(g.syk, tid, ry, Ys[buf ^ 1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        if (g.splits > 1)
          g.part[((long)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][r];
        else
          g.C[(long)m * g.ldc + n] = mg_epilogue(g, acc[i][j][r], m, n);
      }
}

__global__ __launch_bounds__(256) void gemm_reduce_kernel(MGemm g) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)g.M * g.N) return;
  const int m = (int)(i / g.N), n = (int)(i - (long)m * g.N);
  float s = 0.f;
  for (int z = 0; z < g.splits; ++z) s += g.part[(long)z * g.M * g.N + i];
  g.C[(long)m * g.ldc + n] = mg_epilogue(g, s, m, n);
}

// K splits of an M x N x K product: enough workgroups to cover the CUs when
// the tile grid alone is small, each split at least 4 chunks of K.
int gemm_splits(int M, int N, int K) {
  const long tiles = (long)((M + MT - 1) / MT) * ((N + MT - 1) / MT);
  long s = (256 + tiles - 1) / tiles;
  s = std::min<long>(s, std::max(1, K / (4 * MK)));
  return (int)std::max<long>(1, std::min<long>(s, 16));
}

long gemm_part_floats(int M, int N, int K) {
  const int s = gemm_splits(M, N, K);
  return s > 1 ? (long)s * M * N : 0;
}

// op(A) is M x K (A stored [M][lda] or, transposed, [K][lda]); op(B) is K x N
// (B stored [K][ldb] or, transposed, [N][ldb]).  part: gemm_part_floats floats.
template <bool TA, bool TB>
int gemm(int M, int N, int K, float alpha, const float* A, int lda, const float* B, int ldb,
         float beta, float* C, int ldc, const float* bias, int relu, float* part,
         hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return SYNIM_OK;
  MGemm g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.X = A;
  g.sxk = TA ? lda : 1;
  g.sxm = TA ? 1 : lda;
  g.Y = B;
  g.syk = TB ? 1 : ldb;
  g.syn = TB ? ldb : 1;
  g.C = C;
  g.ldc = ldc;
  g.alpha = alpha;
  g.beta = beta;
  g.bias = bias;
  g.relu = relu;
  g.splits = gemm_splits(M, N, K);
  g.kc = (K + g.splits - 1) / g.splits;
  g.kc = (g.kc + MK - 1) / MK * MK;
  g.splits = (K + g.kc - 1) / g.kc;
  g.part = part;
  if (g.splits > 1 && !part) return SYNIM_E_WORKSPACE;
  dim3 grid((N + MT - 1) / MT, (M + MT - 1) / MT, g.splits);
  if (grid.y > 65535) return SYNIM_E_SHAPE;
  hipLaunchKernelGGL(gemm_mfma_kernel, grid, dim3(256), 0, st, g);
  SYNIM_HIP_TRY(hipGetLastError());
  if (g.splits > 1) {
    const long n = (long)M * N;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g);
    SYNIM_HIP_TRY(hipGetLastError());
  }
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

// Column sums of g [B][N] (bias gradients) in a fixed order: 64 columns per
// 256-thread workgroup, each column's rows split over 4 thread groups with 4
// independent accumulators each (16 loads in flight per column instead of one
// long dependent chain), then combined in a fixed order.
constexpr int CS_COLS = 64, CS_PARTS = 4, CS_ACC = 4;
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ g, int B, int N,
                                                     float* __restrict__ out) {
  __shared__ float red[CS_PARTS][CS_COLS];
  const int c = threadIdx.x % CS_COLS, part = threadIdx.x / CS_COLS;
  const int n = blockIdx.x * CS_COLS + c;
  float acc[CS_ACC] = {};
  if (n < N) {
    int b = part;
    for (; b + (CS_ACC - 1) * CS_PARTS < B; b += CS_ACC * CS_PARTS)
#pragma unroll
      for (int u = 0; u < CS_ACC; ++u) acc[u] += g[(size_t)(b + u * CS_PARTS) * N + n];
    for (int u = 0; b < B; b += CS_PARTS, ++u) acc[u] += g[(size_t)b * N + n];
  }
  red[part][c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (part == 0 && n < N) out[n] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
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
// for the backward pass, then dy [B][n_out], dh2 [B][h2], dh1 [B][h1], the
// used W1 columns (forward) or their gradient (backward) [h1][K], and the
// split-K partial products of the largest product of either pass.
struct Scratch {
  float *h1, *h2, *dy, *dh2, *dh1, *w1c, *part;
  size_t total;
};

long part_floats(const synim_mlp& net, int B) {
  const int K = net.len0 + net.len1;
  const int shapes[8][3] = {{B, net.h1, K},         {B, net.h2, net.h1},    {B, net.n_out, net.h2},
                            {net.n_out, net.h2, B}, {B, net.h2, net.n_out}, {net.h2, net.h1, B},
                            {B, net.h1, net.h2},    {net.h1, K, B}};
  long m = 0;
  for (const auto& sh : shapes) m = std::max(m, gemm_part_floats(sh[0], sh[1], sh[2]));
  return m;
}

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
  S.part = take((size_t)part_floats(net, B));
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
  rc = gemm<false, true>(B, net->h1, K, 1.f, x, K, w1c, K, 0.f, h1, net->h1, P + L.b1, 1, S.part, st);
  if (rc != SYNIM_OK) return rc;
  rc = gemm<false, true>(B, net->h2, net->h1, 1.f, h1, net->h1, P + L.w2, net->h1, 0.f, h2,
                         net->h2, P + L.b2, 1, S.part, st);
  if (rc != SYNIM_OK) return rc;
  return gemm<false, true>(B, net->n_out, net->h2, 1.f, h2, net->h2, P + L.w3, net->h2, 0.f, y,
                           net->n_out, P + L.b3, 0, S.part, st);
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
                         net->h2, nullptr, 0, S.part, st);
  if (rc != SYNIM_OK) return rc;
  hipLaunchKernelGGL(colsum_kernel, dim3((net->n_out + CS_COLS - 1) / CS_COLS), dim3(256), 0, st, dy, B,
                     net->n_out, G + L.b3);
  SYNIM_HIP_TRY(hipGetLastError());
  rc = gemm<false, false>(B, net->h2, net->n_out, 1.f, dy, net->n_out, P + L.w3, net->h2, 0.f,
                          dh2, net->h2, nullptr, 0, S.part, st);
  if (rc != SYNIM_OK) return rc;
  const long n2 = (long)B * net->h2;
  hipLaunchKernelGGL(relu_mask_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, dh2,
                     h2, n2);
  SYNIM_HIP_TRY(hipGetLastError());
  // layer 2
  rc = gemm<true, false>(net->h2, net->h1, B, 1.f, dh2, net->h2, h1, net->h1, 0.f, G + L.w2,
                         net->h1, nullptr, 0, S.part, st);
  if (rc != SYNIM_OK) return rc;
  hipLaunchKernelGGL(colsum_kernel, dim3((net->h2 + CS_COLS - 1) / CS_COLS), dim3(256), 0, st, dh2, B,
                     net->h2, G + L.b2);
  SYNIM_HIP_TRY(hipGetLastError());
  rc = gemm<false, false>(B, net->h1, net->h2, 1.f, dh2, net->h2, P + L.w2, net->h1, 0.f, dh1,
                          net->h1, nullptr, 0, S.part, st);
  if (rc != SYNIM_OK) return rc;
  const long n1 = (long)B * net->h1;
  hipLaunchKernelGGL(relu_mask_kernel, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, dh1,
                     h1, n1);
  SYNIM_HIP_TRY(hipGetLastError());
  // layer 1: only the used columns of W1 get gradient, the rest is zero
  rc = gemm<true, false>(net->h1, K, B, 1.f, dh1, net->h1, x, K, 0.f, dw1c, K, nullptr, 0, S.part, st);
  if (rc != SYNIM_OK) return rc;
  const long nw1 = (long)net->h1 * net->n_in;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((nw1 + 255) / 256)), dim3(256), 0, st,
                     G + L.w1, nw1);
  SYNIM_HIP_TRY(hipGetLastError());
  const long nk = (long)net->h1 * K;
  hipLaunchKernelGGL(scatter_cols_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st,
                     dw1c, net->h1, K, net->seg0, net->len0, net->seg1, G + L.w1, net->n_in);
  SYNIM_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(colsum_kernel, dim3((net->h1 + CS_COLS - 1) / CS_COLS), dim3(256), 0, st, dh1, B,
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
