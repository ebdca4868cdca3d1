// Tomographic projection P_opt = (P_DM^T P_DM + lambda I)^-1 P_DM^T P_Layer
// (paper Sec. 2.5): the projection matrices sampled on the device, their Gram
// and cross products by an FP64 MFMA GEMM, a blocked Cholesky factorisation
// and two blocked triangular solves, all in FP64.
//
// Storage: a projection matrix P (rows = (direction, pupil block), columns =
// basis functions) is kept transposed, Pt[col][row], so that every basis
// function's samples are contiguous (the sampler writes them coalesced) and
// the products are  G = Pt_dm Pt_dm^T  and  B = Pt_dm Pt_layer^T.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "common.hpp"

namespace synim {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ sampling
// One thread per (row, basis function): the mean over the block's fine pupil
// pixels of the bilinear sample of the basis function at
// c + (r + h theta) / s (zero outside the component grid).  Grid: x over rows,
// y over the component's functions.
struct SampleArgs {
  const float* basis;          // [n][H][W]
  int n, H, W;
  double h, s;                 // altitude (m), pixel (m)
  const double2* dirs;         // [n_dir] (theta_x, theta_y) radians
  int n_dir;
  const int2* blocks;          // [n_blocks] (by, bx)
  int n_blocks, bin;
  const uint8_t* pupil;        // [Hp][Wp]
  int Hp, Wp;
  double sp;                   // pupil pixel (m)
  double* Pt;                  // column base: Pt + col0 * ld
  long ld;
};

__global__ __launch_bounds__(256) void proj_sample_kernel(SampleArgs g) {
  const long row = (long)blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y;
  if (row >= (long)g.n_dir * g.n_blocks) return;
  const int d = (int)(row / g.n_blocks), blk = (int)(row - (long)d * g.n_blocks);
  const int2 bb = g.blocks[blk];
  const double2 th = g.dirs[d];
  const double cy = (g.H - 1) * 0.5, cx = (g.W - 1) * 0.5;
  const double cpy = (g.Hp - 1) * 0.5, cpx = (g.Wp - 1) * 0.5;
  const float* F = g.basis + (size_t)a * g.H * g.W;
  double acc = 0.0;
  int cnt = 0;
  for (int fy = 0; fy < g.bin; ++fy)
    for (int fx = 0; fx < g.bin; ++fx) {
      const int y = bb.x * g.bin + fy, x = bb.y * g.bin + fx;
      if (!g.pupil[(size_t)y * g.Wp + x]) continue;
      const double gx = cx + ((x - cpx) * g.sp + g.h * th.x) / g.s;
      const double gy = cy + ((y - cpy) * g.sp + g.h * th.y) / g.s;
      const double fi = floor(gx), fj = floor(gy);
      const int i = (int)fi, j = (int)fj;
      const double u = gx - fi, v = gy - fj;
      auto tap = [&](int ii, int jj) -> double {
        return (ii >= 0 && ii < g.W && jj >= 0 && jj < g.H) ? (double)F[(size_t)jj * g.W + ii]
                                                            : 0.0;
      };
      acc += (1.0 - u) * (1.0 - v) * tap(i, j) + u * (1.0 - v) * tap(i + 1, j) +
             (1.0 - u) * v * tap(i, j + 1) + u * v * tap(i + 1, j + 1);
      ++cnt;
    }
  g.Pt[(size_t)a * g.ld + row] = cnt > 0 ? acc / cnt : 0.0;
}

// ---------------------------------------------------------------- FP64 GEMM
// C[m][n] = alpha sum_k X(k, m) Y(k, n) + beta C[m][n], X(k, m) = X[k sxk + m sxm],
// Y(k, n) = Y[k syk + n syn], C row-major with ldc.  One workgroup of 256
// threads per (32 BI) x (32 BJ) tile of C; each wave owns a (16 BI) x (16 BJ)
// quarter as BI x BJ blocks of v_mfma_f64_16x16x4f64 (lane l feeds
// A[l%16][l/16] and B[l/16][l%16] and holds D[4r + l/16][l%16], r = 0..3).  K
// advances in chunks of 16 through two LDS buffers: the next chunk's global
// loads are in flight while the current one feeds the matrix cores.  lower:
// only tiles with some m >= n (a symmetric result's lower triangle) are
// computed.  Two shapes: 128 x 128 (two workgroups per CU) for small products,
// 256 x 128 (one per CU, each wave's 8 x 4 accumulator blocks in the
// accumulation registers) for large ones, which halves the operand bytes each
// flop needs from L2 along m.
constexpr int GK = 16, GPAD = 2;

struct GemmArgs {
  int M, N, K;
  const double* X;
  long sxk, sxm;
  const double* Y;
  long syk, syn;
  double* C;
  long ldc;
  double alpha, beta;
  int lower;
};

// (kk, mm) of element q of this thread in a GK x T chunk, reading along the
// operand's unit stride
template <int T>
__device__ __forceinline__ void gemm_elem(long sk, int tid, int q, int& kk, int& mm) {
  const int e = tid + 256 * q;
  if (sk == 1) {
    kk = e % GK;
    mm = e / GK;
  } else {
    kk = e / T;
    mm = e % T;
  }
}

template <int T>
__device__ __forceinline__ void gemm_fetch(const double* P, long sk, long sm, int k0, int m0,
                                           int K, int M, int tid, double (&r)[GK * T / 256]) {
#pragma unroll
  for (int q = 0; q < GK * T / 256; ++q) {
    int kk, mm;
    gemm_elem<T>(sk, tid, q, kk, mm);
    const int k = k0 + kk, m = m0 + mm;
    r[q] = (k < K && m < M) ? P[(long)k * sk + (long)m * sm] : 0.0;
  }
}

template <int T>
__device__ __forceinline__ void gemm_put(long sk, int tid, const double (&r)[GK * T / 256],
                                         double (*S)[T + GPAD]) {
#pragma unroll
  for (int q = 0; q < GK * T / 256; ++q) {
    int kk, mm;
    gemm_elem<T>(sk, tid, q, kk, mm);
    S[kk][mm] = r[q];
  }
}

template <int BI, int BJ>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
  constexpr int TM = 32 * BI, TN = 32 * BJ;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  if (g.lower && m0 + TM - 1 < n0) return;   // tile wholly above the diagonal
  __shared__ double Xs[2][GK][TM + GPAD], Ys[2][GK][TN + GPAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 16 * BI, wn = (wave & 1) * 16 * BJ;
  d4 acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  double rx[GK * TM / 256], ry[GK * TN / 256];
  gemm_fetch<TM>(g.X, g.sxk, g.sxm, 0, m0, g.K, g.M, tid, rx);
  gemm_fetch<TN>(g.Y, g.syk, g.syn, 0, n0, g.K, g.N, tid, ry);
  gemm_put<TM>(g.sxk, tid, rx, Xs[0]);
  gemm_put<TN>(g.syk, tid, ry, Ys[0]);
  __syncthreads();
  const int nk = (g.K + GK - 1) / GK;
  for (int c = 0; c < nk; ++c) {
    const int buf = c & 1;
    const bool more = c + 1 < nk;
    if (more) {
      gemm_fetch<TM>(g.X, g.sxk, g.sxm, (c + 1) * GK, m0, g.K, g.M, tid, rx);
      gemm_fetch<TN>(g.Y, g.syk, g.syn, (c + 1) * GK, n0, g.K, g.N, tid, ry);
    }
    // the large shape keeps one k-step's operands live at a time (its
    // accumulators fill the accumulation registers)
#pragma unroll(BI * BJ > 16 ? 1 : GK / 4)
    for (int s = 0; s < GK / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      double a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = Xs[buf][kr][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = Ys[buf][kr][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      // the other buffer was last read in iteration c - 1, before its closing barrier
      gemm_put<TM>(g.sxk, tid, rx, Xs[buf ^ 1]);
      gemm_put<TN>(g.syk, tid, ry, Ys[buf ^ 1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * r + (lane >> 4);
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m < g.M && n < g.N && (!g.lower || m >= n)) {
          double* cp = g.C + (long)m * g.ldc + n;
          *cp = g.alpha * acc[i][j][r] + (g.beta == 0.0 ? 0.0 : g.beta * *cp);
        }
      }
}

int gemm(const GemmArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return SYNIM_OK;
  // 256 x 128 tiles once there are enough of them to fill the CUs
  const long big_tiles = (long)((a.M + 255) / 256) * ((a.N + 127) / 128);
  if (big_tiles >= 256) {
    const dim3 grid((unsigned)((a.N + 127) / 128), (unsigned)((a.M + 255) / 256));
    hipLaunchKernelGGL((gemm_f64_kernel<8, 4>), grid, dim3(256), 0, st, a);
  } else {
    const dim3 grid((unsigned)((a.N + 127) / 128), (unsigned)((a.M + 127) / 128));
    hipLaunchKernelGGL((gemm_f64_kernel<4, 4>), grid, dim3(256), 0, st, a);
  }
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

__global__ void zero_status_kernel(int* s) {
  if (threadIdx.x < 16) s[threadIdx.x] = 0;
}

__global__ void add_diag_kernel(double* A, int n, long ld, double lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[(long)i * ld + i] += lam;
}

// ------------------------------------------------------------------ Cholesky
// Lower Cholesky of a symmetric positive definite matrix held (lower triangle)
// row-major, blocked by CB: factor the diagonal block in LDS, solve the panel
// below it, update the trailing lower triangle with the GEMM.
constexpr int CB = 64;

// One workgroup: the nb x nb diagonal block at (k, k), unblocked, in LDS.  A
// pivot that is not positive sets *status (the matrix is not positive
// definite) and the block is left as it is.
// Linv (nullable): also writes the block's inverse L_kk^-1 there (CB x CB,
// row-major, zero above the diagonal and outside nb x nb), each column by
// forward substitution against the unit vector.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* A, long ld, int k, int nb,
                                                         int* status, double* Linv = nullptr) {
  __shared__ double L[CB][CB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    L[i][j] = j <= i ? A[(long)(k + i) * ld + k + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double d = L[j][j];
      if (!(d > 0.0)) bad = 1;
      L[j][j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double djj = L[j][j];
    for (int i = j + 1 + tid; i < nb; i += 256) L[i][j] /= djj;
    __syncthreads();
    // trailing update of the block's lower triangle
    const int rem = nb - j - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, c = j + 1 + e % rem;
      if (c <= i) L[i][c] -= L[i][j] * L[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    if (j <= i) A[(long)(k + i) * ld + k + j] = L[i][j];
  }
  if (tid == 0 && bad) atomicOr(status, 1);
  if (Linv == nullptr) return;
  __shared__ double X[CB][CB + 1];
  for (int e = tid; e < CB * (CB + 1); e += 256) (&X[0][0])[e] = 0.0;
  __syncthreads();
  if (tid < nb) {
    // column c = tid of L^-1: x_r = (delta_rc - sum_{c <= q < r} L[r][q] x_q) / L[r][r]
    const int c = tid;
    for (int r = c; r < nb; ++r) {
      double v = r == c ? 1.0 : 0.0;
      for (int q = c; q < r; ++q) v -= L[r][q] * X[q][c];
      X[r][c] = v / L[r][r];
    }
  }
  __syncthreads();
  for (int e = tid; e < CB * CB; e += 256) Linv[e] = X[e / CB][e % CB];
}

// Panel rows i in [r0, n): row i of block column k becomes x with
// x L_kk^T = a (forward substitution along the row).  One thread per row.
__global__ __launch_bounds__(256) void potrf_panel_kernel(double* A, long ld, int k, int nb,
                                                          int r0, int n) {
  __shared__ double L[CB][CB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    L[i][j] = j <= i ? A[(long)(k + i) * ld + k + j] : 0.0;
  }
  __syncthreads();
  const int i = r0 + blockIdx.x * 256 + tid;
  if (i >= n) return;
  double* row = A + (long)i * ld + k;
  double x[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) x[j] = j < nb ? row[j] : 0.0;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    if (j >= nb) break;
    double v = x[j];
    for (int c = 0; c < j; ++c) v -= x[c] * L[j][c];
    x[j] = v / L[j][j];
  }
#pragma unroll
  for (int j = 0; j < CB; ++j)
    if (j < nb) row[j] = x[j];
}

int potrf(double* A, int n, long ld, int* status, hipStream_t st) {
  for (int k = 0; k < n; k += CB) {
    const int nb = std::min(CB, n - k);
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, A, ld, k, nb, status);
    SYNIM_HIP_TRY(hipGetLastError());
    const int r0 = k + nb;
    if (r0 >= n) break;
    hipLaunchKernelGGL(potrf_panel_kernel, dim3((unsigned)((n - r0 + 255) / 256)), dim3(256), 0,
                       st, A, ld, k, nb, r0, n);
    SYNIM_HIP_TRY(hipGetLastError());
    // trailing lower triangle: A[r0:, r0:] -= P P^T, P = A[r0:, k:k+nb]
    GemmArgs g{};
    g.M = g.N = n - r0;
    g.K = nb;
    g.X = g.Y = A + (long)r0 * ld + k;
    g.sxk = g.syk = 1;
    g.sxm = g.syn = ld;
    g.C = A + (long)r0 * ld + r0;
    g.ldc = ld;
    g.alpha = -1.0;
    g.beta = 1.0;
    g.lower = 1;
    int rc = gemm(g, st);
    if (rc != SYNIM_OK) return rc;
  }
  return SYNIM_OK;
}

// ------------------------------------------------------- triangular solves
// B [n][m] (row-major, ldb) <- L_kk^-1 B[k:k+nb] (forward) or L_kk^-T B[k:k+nb]
// (backward) for the diagonal block at k; one thread per right-hand-side
// column, the block's rows sequential.
__global__ __launch_bounds__(256) void trsm_block_kernel(const double* L, long ld, int k, int nb,
                                                         double* B, long ldb, int m,
                                                         int backward) {
  __shared__ double T[CB][CB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    T[i][j] = j <= i ? L[(long)(k + i) * ld + k + j] : 0.0;
  }
  __syncthreads();
  const int col = blockIdx.x * 256 + tid;
  if (col >= m) return;
  double x[CB];
#pragma unroll
  for (int r = 0; r < CB; ++r) x[r] = r < nb ? B[(long)(k + r) * ldb + col] : 0.0;
  if (!backward) {
    for (int r = 0; r < nb; ++r) {
      double v = x[r];
      for (int c = 0; c < r; ++c) v -= T[r][c] * x[c];
      x[r] = v / T[r][r];
    }
  } else {
    for (int r = nb - 1; r >= 0; --r) {
      double v = x[r];
      for (int c = r + 1; c < nb; ++c) v -= T[c][r] * x[c];
      x[r] = v / T[r][r];
    }
  }
#pragma unroll
  for (int r = 0; r < CB; ++r)
    if (r < nb) B[(long)(k + r) * ldb + col] = x[r];
}

int potrs(const double* L, int n, long ld, double* B, int m, long ldb, hipStream_t st) {
  const dim3 tg((unsigned)((m + 255) / 256));
  // forward: L Y = B, right-looking
  for (int k = 0; k < n; k += CB) {
    const int nb = std::min(CB, n - k);
    hipLaunchKernelGGL(trsm_block_kernel, tg, dim3(256), 0, st, L, ld, k, nb, B, ldb, m, 0);
    SYNIM_HIP_TRY(hipGetLastError());
    if (k + nb >= n) break;
    // B[k+nb:] -= L[k+nb:, k:k+nb] Y_k
    GemmArgs g{};
    g.M = n - k - nb;
    g.N = m;
    g.K = nb;
    g.X = L + (long)(k + nb) * ld + k;
    g.sxk = 1;
    g.sxm = ld;
    g.Y = B + (long)k * ldb;
    g.syk = ldb;
    g.syn = 1;
    g.C = B + (long)(k + nb) * ldb;
    g.ldc = ldb;
    g.alpha = -1.0;
    g.beta = 1.0;
    int rc = gemm(g, st);
    if (rc != SYNIM_OK) return rc;
  }
  // backward: L^T X = Y, from the last block
  const int last = ((n - 1) / CB) * CB;
  for (int k = last; k >= 0; k -= CB) {
    const int nb = std::min(CB, n - k);
    hipLaunchKernelGGL(trsm_block_kernel, tg, dim3(256), 0, st, L, ld, k, nb, B, ldb, m, 1);
    SYNIM_HIP_TRY(hipGetLastError());
    if (k == 0) break;
    // B[0:k] -= L[k:k+nb, 0:k]^T X_k
    GemmArgs g{};
    g.M = k;
    g.N = m;
    g.K = nb;
    g.X = L + (long)k * ld;
    g.sxk = ld;
    g.sxm = 1;
    g.Y = B + (long)k * ldb;
    g.syk = ldb;
    g.syn = 1;
    g.C = B;
    g.ldc = ldb;
    g.alpha = -1.0;
    g.beta = 1.0;
    int rc = gemm(g, st);
    if (rc != SYNIM_OK) return rc;
  }
  return SYNIM_OK;
}

// dst[r][c] = src[r][c] for r < rows, c < cols (row-major, leading dimensions
// lds, ldd).
__global__ __launch_bounds__(256) void copy2d_kernel(const double* __restrict__ src, long lds,
                                                     double* __restrict__ dst, long ldd,
                                                     int rows, int cols) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e - (long)r * cols);
  dst[(long)r * ldd + c] = src[(long)r * lds + c];
}

int copy2d(const double* src, long lds, double* dst, long ldd, int rows, int cols,
           hipStream_t st) {
  const long n = (long)rows * cols;
  if (n == 0) return SYNIM_OK;
  hipLaunchKernelGGL(copy2d_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                     lds, dst, ldd, rows, cols);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

// Blocked Cholesky and solves with the diagonal blocks inverted: the panel
// below each diagonal block and the block rows of the solves become matrix-
// core GEMMs against L_kk^-1 instead of substitutions with one thread per row
// or column.  Linv: ceil(n / CB) blocks of CB x CB doubles, written by potrf_inv
// and read by potrs_inv; tmp: max(n, m) x CB doubles.
int potrf_inv(double* A, int n, long ld, int* status, double* Linv, double* tmp,
              hipStream_t st) {
  for (int k = 0; k < n; k += CB) {
    const int nb = std::min(CB, n - k);
    double* Li = Linv + (long)(k / CB) * CB * CB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, A, ld, k, nb, status, Li);
    SYNIM_HIP_TRY(hipGetLastError());
    const int r0 = k + nb;
    if (r0 >= n) break;
    // panel: A[r0:, k:k+nb] <- A[r0:, k:k+nb] L_kk^-T (from a copy)
    int rc = copy2d(A + (long)r0 * ld + k, ld, tmp, nb, n - r0, nb, st);
    if (rc != SYNIM_OK) return rc;
    GemmArgs p{};
    p.M = n - r0;
    p.N = nb;
    p.K = nb;
    p.X = tmp;   // X(q, i) = tmp[i][q]
    p.sxk = 1;
    p.sxm = nb;
    p.Y = Li;    // Y(q, j) = L_kk^-1[j][q]
    p.syk = 1;
    p.syn = CB;
    p.C = A + (long)r0 * ld + k;
    p.ldc = ld;
    p.alpha = 1.0;
    p.beta = 0.0;
    if ((rc = gemm(p, st)) != SYNIM_OK) return rc;
    // trailing lower triangle: A[r0:, r0:] -= P P^T, P = A[r0:, k:k+nb]
    GemmArgs g{};
    g.M = g.N = n - r0;
    g.K = nb;
    g.X = g.Y = A + (long)r0 * ld + k;
    g.sxk = g.syk = 1;
    g.sxm = g.syn = ld;
    g.C = A + (long)r0 * ld + r0;
    g.ldc = ld;
    g.alpha = -1.0;
    g.beta = 1.0;
    g.lower = 1;
    if ((rc = gemm(g, st)) != SYNIM_OK) return rc;
  }
  return SYNIM_OK;
}

int potrs_inv(const double* L, int n, long ld, double* B, int m, long ldb, const double* Linv,
              double* tmp, hipStream_t st) {
  // B_k <- L_kk^-1 B_k (forward) or L_kk^-T B_k (backward), from a copy
  auto diag = [&](int k, int nb, bool backward) {
    int rc = copy2d(B + (long)k * ldb, ldb, tmp, m, nb, m, st);
    if (rc != SYNIM_OK) return rc;
    const double* Li = Linv + (long)(k / CB) * CB * CB;
    GemmArgs d{};
    d.M = nb;
    d.N = m;
    d.K = nb;
    d.X = Li;   // X(q, i) = L^-1[i][q] (forward) or L^-1[q][i] (backward)
    d.sxk = backward ? CB : 1;
    d.sxm = backward ? 1 : CB;
    d.Y = tmp;  // Y(q, c) = tmp[q][c]
    d.syk = m;
    d.syn = 1;
    d.C = B + (long)k * ldb;
    d.ldc = ldb;
    d.alpha = 1.0;
    d.beta = 0.0;
    return gemm(d, st);
  };
  for (int k = 0; k < n; k += CB) {
    const int nb = std::min(CB, n - k);
    int rc = diag(k, nb, false);
    if (rc != SYNIM_OK) return rc;
    if (k + nb >= n) break;
    GemmArgs g{};
    g.M = n - k - nb;
    g.N = m;
    g.K = nb;
    g.X = L + (long)(k + nb) * ld + k;
    g.sxk = 1;
    g.sxm = ld;
    g.Y = B + (long)k * ldb;
    g.syk = ldb;
    g.syn = 1;
    g.C = B + (long)(k + nb) * ldb;
    g.ldc = ldb;
    g.alpha = -1.0;
    g.beta = 1.0;
    if ((rc = gemm(g, st)) != SYNIM_OK) return rc;
  }
  const int last = ((n - 1) / CB) * CB;
  for (int k = last; k >= 0; k -= CB) {
    const int nb = std::min(CB, n - k);
    int rc = diag(k, nb, true);
    if (rc != SYNIM_OK) return rc;
    if (k == 0) break;
    GemmArgs g{};
    g.M = k;
    g.N = m;
    g.K = nb;
    g.X = L + (long)k * ld;
    g.sxk = ld;
    g.sxm = 1;
    g.Y = B + (long)k * ldb;
    g.syk = ldb;
    g.syn = 1;
    g.C = B;
    g.ldc = ldb;
    g.alpha = -1.0;
    g.beta = 1.0;
    if ((rc = gemm(g, st)) != SYNIM_OK) return rc;
  }
  return SYNIM_OK;
}

// Kept b x b blocks of the pupil mask, row-major.
std::vector<int2> pupil_blocks(const uint8_t* pupil, int Hp, int Wp, int bin) {
  std::vector<int2> out;
  for (int by = 0; by < Hp / bin; ++by)
    for (int bx = 0; bx < Wp / bin; ++bx) {
      bool any = false;
      for (int y = by * bin; y < by * bin + bin && !any; ++y)
        for (int x = bx * bin; x < bx * bin + bin; ++x)
          if (pupil[(size_t)y * Wp + x]) {
            any = true;
            break;
          }
      if (any) out.push_back(make_int2(by, bx));
    }
  return out;
}

struct ProjLayout {
  size_t dirs, blocks, pupil, status, pt_dm, pt_l, gram, total;
};

ProjLayout proj_layout(int n_dir, int n_blocks, int Hp, int Wp, long rows, long n_dm, long n_l) {
  ProjLayout L{};
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t at = off;
    off = align_up(off + n, 256);
    return at;
  };
  L.dirs = take((size_t)n_dir * sizeof(double2));
  L.blocks = take((size_t)n_blocks * sizeof(int2));
  L.pupil = take((size_t)Hp * Wp);
  L.status = take(16 * sizeof(int));
  L.pt_dm = take((size_t)n_dm * rows * sizeof(double));
  L.pt_l = take((size_t)n_l * rows * sizeof(double));
  L.gram = take((size_t)n_dm * n_dm * sizeof(double));
  L.total = off;
  return L;
}

int check_comps(const synim_proj_component* c, int n) {
  if (!c || n < 1) return SYNIM_E_NULL;
  for (int i = 0; i < n; ++i) {
    if (!c[i].basis) return SYNIM_E_NULL;
    if (c[i].n < 1 || c[i].H < 2 || c[i].W < 2) return SYNIM_E_SHAPE;
    if (!(c[i].pixel_m > 0.0)) return SYNIM_E_PARAM;
  }
  return SYNIM_OK;
}

long total_cols(const synim_proj_component* c, int n) {
  long t = 0;
  for (int i = 0; i < n; ++i) t += c[i].n;
  return t;
}

// Samples every component into Pt (columns in component order) from the
// device tables at ws.
int sample_all(const synim_proj_component* comps, int n_comp, const double2* dirs_dev, int n_dir,
               const int2* blocks_dev, int n_blocks, int bin, const uint8_t* pupil_dev, int Hp,
               int Wp, double sp, double* Pt, long ld, hipStream_t st) {
  long col = 0;
  const long rows = (long)n_dir * n_blocks;
  for (int c = 0; c < n_comp; ++c) {
    SampleArgs g{};
    g.basis = comps[c].basis;
    g.n = comps[c].n;
    g.H = comps[c].H;
    g.W = comps[c].W;
    g.h = comps[c].altitude_m;
    g.s = comps[c].pixel_m;
    g.dirs = dirs_dev;
    g.n_dir = n_dir;
    g.blocks = blocks_dev;
    g.n_blocks = n_blocks;
    g.bin = bin;
    g.pupil = pupil_dev;
    g.Hp = Hp;
    g.Wp = Wp;
    g.sp = sp;
    g.Pt = Pt + col * ld;
    g.ld = ld;
    for (int a0 = 0; a0 < g.n; a0 += 65535) {
      SampleArgs gg = g;
      gg.basis = g.basis + (size_t)a0 * g.H * g.W;
      gg.Pt = g.Pt + (long)a0 * ld;
      gg.n = std::min(65535, g.n - a0);
      hipLaunchKernelGGL(proj_sample_kernel,
                         dim3((unsigned)((rows + 255) / 256), (unsigned)gg.n), dim3(256), 0, st,
                         gg);
      SYNIM_HIP_TRY(hipGetLastError());
    }
    col += g.n;
  }
  return SYNIM_OK;
}

int proj_common(const synim_proj_component* dms, int n_dm, const double* dirs, int n_dir,
                const uint8_t* pupil, int Hp, int Wp, double sp, int bin) {
  if (!dirs || !pupil) return SYNIM_E_NULL;
  int rc = check_comps(dms, n_dm);
  if (rc != SYNIM_OK) return rc;
  if (n_dir < 1 || Hp < 1 || Wp < 1 || bin < 1 || Hp % bin || Wp % bin) return SYNIM_E_SHAPE;
  if (!(sp > 0.0)) return SYNIM_E_PARAM;
  return SYNIM_OK;
}

}  // namespace
}  // namespace synim

using namespace synim;

extern "C" int synim_proj_rows(const uint8_t* pupil, int Hp, int Wp, int bin, int n_dir,
                               int* n_rows) {
  if (!pupil || !n_rows) return SYNIM_E_NULL;
  if (n_dir < 1 || Hp < 1 || Wp < 1 || bin < 1 || Hp % bin || Wp % bin) return SYNIM_E_SHAPE;
  *n_rows = (int)(pupil_blocks(pupil, Hp, Wp, bin).size() * (size_t)n_dir);
  return SYNIM_OK;
}

extern "C" int synim_proj_workspace(const synim_proj_component* dms, int n_dm,
                                    const synim_proj_component* layers, int n_layer, int n_dir,
                                    const uint8_t* pupil, int Hp, int Wp, int bin,
                                    size_t* bytes) {
  if (!bytes || !pupil) return SYNIM_E_NULL;
  int rc = check_comps(dms, n_dm);
  if (rc != SYNIM_OK) return rc;
  if (layers && n_layer > 0 && (rc = check_comps(layers, n_layer)) != SYNIM_OK) return rc;
  if (n_dir < 1 || Hp < 1 || Wp < 1 || bin < 1 || Hp % bin || Wp % bin) return SYNIM_E_SHAPE;
  const int nb = (int)pupil_blocks(pupil, Hp, Wp, bin).size();
  const long rows = (long)nb * n_dir;
  const long ndm = total_cols(dms, n_dm), nl = layers ? total_cols(layers, n_layer) : 0;
  *bytes = proj_layout(n_dir, nb, Hp, Wp, rows, ndm, nl).total;
  return SYNIM_OK;
}

extern "C" int synim_proj_matrix(const synim_proj_component* comps, int n_comp,
                                 const double* dirs, int n_dir, const uint8_t* pupil, int Hp,
                                 int Wp, double pupil_pixel_m, int bin, double* Pt, long ld,
                                 void* ws, size_t ws_bytes, void* stream) {
  int rc = proj_common(comps, n_comp, dirs, n_dir, pupil, Hp, Wp, pupil_pixel_m, bin);
  if (rc != SYNIM_OK) return rc;
  if (!Pt || !ws) return SYNIM_E_NULL;
  hipStream_t st = (hipStream_t)stream;
  const std::vector<int2> blocks = pupil_blocks(pupil, Hp, Wp, bin);
  const long rows = (long)blocks.size() * n_dir;
  if (ld < rows) return SYNIM_E_SHAPE;
  const ProjLayout L = proj_layout(n_dir, (int)blocks.size(), Hp, Wp, rows, 0, 0);
  if (ws_bytes < L.total) return SYNIM_E_WORKSPACE;
  char* w = static_cast<char*>(ws);
  SYNIM_HIP_TRY(hipMemcpyAsync(w + L.dirs, dirs, (size_t)n_dir * sizeof(double2),
                               hipMemcpyHostToDevice, st));
  SYNIM_HIP_TRY(hipMemcpyAsync(w + L.blocks, blocks.data(), blocks.size() * sizeof(int2),
                               hipMemcpyHostToDevice, st));
  SYNIM_HIP_TRY(hipMemcpyAsync(w + L.pupil, pupil, (size_t)Hp * Wp, hipMemcpyHostToDevice, st));
  rc = sample_all(comps, n_comp, reinterpret_cast<const double2*>(w + L.dirs), n_dir,
                  reinterpret_cast<const int2*>(w + L.blocks), (int)blocks.size(), bin,
                  reinterpret_cast<const uint8_t*>(w + L.pupil), Hp, Wp, pupil_pixel_m, Pt, ld,
                  st);
  if (rc != SYNIM_OK) return rc;
  // the host vectors must outlive the copies
  SYNIM_HIP_TRY(hipStreamSynchronize(st));
  return SYNIM_OK;
}

extern "C" int synim_gemm_f64(int M, int N, int K, double alpha, const double* X, long sxk,
                              long sxm, const double* Y, long syk, long syn, double beta,
                              double* C, long ldc, void* stream) {
  if (!C || (K > 0 && (!X || !Y))) return SYNIM_E_NULL;
  if (M < 0 || N < 0 || K < 0 || ldc < N) return SYNIM_E_SHAPE;
  if (K == 0) {
    if (beta == 1.0) return SYNIM_OK;
    // C = beta C: run the GEMM over an empty K (its epilogue scales C)
  }
  GemmArgs g{M, N, K, X, sxk, sxm, Y, syk, syn, C, ldc, alpha, beta, 0};
  return gemm(g, (hipStream_t)stream);
}

extern "C" int synim_potrf_f64(double* A, int n, long ld, int* status, void* stream) {
  if (!A || !status) return SYNIM_E_NULL;
  if (n < 1 || ld < n) return SYNIM_E_SHAPE;
  return potrf(A, n, ld, status, (hipStream_t)stream);
}

extern "C" int synim_potrs_f64(const double* L, int n, long ld, double* B, int m, long ldb,
                               void* stream) {
  if (!L || !B) return SYNIM_E_NULL;
  if (n < 1 || m < 1 || ld < n || ldb < m) return SYNIM_E_SHAPE;
  return potrs(L, n, ld, B, m, ldb, (hipStream_t)stream);
}

extern "C" int synim_proj_opt(const synim_proj_component* dms, int n_dm,
                              const synim_proj_component* layers, int n_layer, const double* dirs,
                              int n_dir, const uint8_t* pupil, int Hp, int Wp,
                              double pupil_pixel_m, int bin, double lambda, double* popt,
                              void* ws, size_t ws_bytes, void* stream) {
  int rc = proj_common(dms, n_dm, dirs, n_dir, pupil, Hp, Wp, pupil_pixel_m, bin);
  if (rc != SYNIM_OK) return rc;
  if ((rc = check_comps(layers, n_layer)) != SYNIM_OK) return rc;
  if (!popt || !ws) return SYNIM_E_NULL;
  if (!(lambda >= 0.0)) return SYNIM_E_PARAM;
  hipStream_t st = (hipStream_t)stream;
  const std::vector<int2> blocks = pupil_blocks(pupil, Hp, Wp, bin);
  const long rows = (long)blocks.size() * n_dir;
  const long ndm = total_cols(dms, n_dm), nl = total_cols(layers, n_layer);
  if (ndm > INT_MAX || nl > INT_MAX || rows > INT_MAX) return SYNIM_E_SHAPE;
  const ProjLayout L = proj_layout(n_dir, (int)blocks.size(), Hp, Wp, rows, ndm, nl);
  if (ws_bytes < L.total) return SYNIM_E_WORKSPACE;
  char* w = static_cast<char*>(ws);
  SYNIM_HIP_TRY(hipMemcpyAsync(w + L.dirs, dirs, (size_t)n_dir * sizeof(double2),
                               hipMemcpyHostToDevice, st));
  SYNIM_HIP_TRY(hipMemcpyAsync(w + L.blocks, blocks.data(), blocks.size() * sizeof(int2),
                               hipMemcpyHostToDevice, st));
  SYNIM_HIP_TRY(hipMemcpyAsync(w + L.pupil, pupil, (size_t)Hp * Wp, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(zero_status_kernel, dim3(1), dim3(64), 0, st,
                     reinterpret_cast<int*>(w + L.status));
  SYNIM_HIP_TRY(hipGetLastError());
  double* pt_dm = reinterpret_cast<double*>(w + L.pt_dm);
  double* pt_l = reinterpret_cast<double*>(w + L.pt_l);
  double* G = reinterpret_cast<double*>(w + L.gram);
  const auto* dirs_dev = reinterpret_cast<const double2*>(w + L.dirs);
  const auto* blocks_dev = reinterpret_cast<const int2*>(w + L.blocks);
  const auto* pupil_dev = reinterpret_cast<const uint8_t*>(w + L.pupil);
  rc = sample_all(dms, n_dm, dirs_dev, n_dir, blocks_dev, (int)blocks.size(), bin, pupil_dev, Hp,
                  Wp, pupil_pixel_m, pt_dm, rows, st);
  if (rc == SYNIM_OK)
    rc = sample_all(layers, n_layer, dirs_dev, n_dir, blocks_dev, (int)blocks.size(), bin,
                    pupil_dev, Hp, Wp, pupil_pixel_m, pt_l, rows, st);
  if (rc != SYNIM_OK) return rc;
  // G = Pt_dm Pt_dm^T (lower triangle) + lambda I;  B = Pt_dm Pt_l^T into popt
  GemmArgs g{(int)ndm, (int)ndm, (int)rows, pt_dm, 1, rows, pt_dm, 1, rows, G, ndm, 1.0, 0.0, 1};
  if ((rc = gemm(g, st)) != SYNIM_OK) return rc;
  hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)((ndm + 255) / 256)), dim3(256), 0, st, G,
                     (int)ndm, ndm, lambda);
  SYNIM_HIP_TRY(hipGetLastError());
  GemmArgs b{(int)ndm, (int)nl, (int)rows, pt_dm, 1, rows, pt_l, 1, rows, popt, nl, 1.0, 0.0, 0};
  if ((rc = gemm(b, st)) != SYNIM_OK) return rc;
  int* status = reinterpret_cast<int*>(w + L.status);
  // the sampled matrices are spent: their memory holds the inverted diagonal
  // blocks and the copies the solves work from
  // (where they are too small, the substitution forms need no memory)
  double* linv = pt_dm;
  double* tmp = pt_dm + ((ndm + CB - 1) / CB) * CB * CB;
  if ((size_t)(((ndm + CB - 1) / CB) * CB * CB + std::max(ndm, nl) * CB) <=
      (size_t)rows * (size_t)ndm) {
    if ((rc = potrf_inv(G, (int)ndm, ndm, status, linv, tmp, st)) != SYNIM_OK) return rc;
    if ((rc = potrs_inv(G, (int)ndm, ndm, popt, (int)nl, nl, linv, tmp, st)) != SYNIM_OK)
      return rc;
  } else {
    if ((rc = potrf(G, (int)ndm, ndm, status, st)) != SYNIM_OK) return rc;
    if ((rc = potrs(G, (int)ndm, ndm, popt, (int)nl, nl, st)) != SYNIM_OK) return rc;
  }
  // the host vectors must outlive the copies
  SYNIM_HIP_TRY(hipStreamSynchronize(st));
  int host_status = 0;
  SYNIM_HIP_TRY(hipMemcpy(&host_status, status, sizeof(int), hipMemcpyDeviceToHost));
  return host_status ? SYNIM_E_PARAM : SYNIM_OK;
}
