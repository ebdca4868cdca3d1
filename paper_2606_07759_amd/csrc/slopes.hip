// Standalone slope step (paper Sec. 2.2): central differences at every pupil
// pixel of a haloed phase map, averaged over each valid subaperture.
#include "common.hpp"

namespace synim {
namespace {

constexpr int SBLOCK = 256;   // pixel columns of one workgroup
constexpr int SROWS = 8;      // subaperture rows one workgroup walks in turn

// Pixel (x, y)'s pupil-masked central differences and pupil count, added to
// its column's sums.  The loads are unconditional (the halo keeps them in
// bounds) so that many rows' loads can be in flight together.
__device__ __forceinline__ void column_terms(const float* ph, const uint8_t* pupil, int W,
                                             int Wh, int x, int y, float& gx, float& gy,
                                             float& cnt) {
  const bool in = pupil[(size_t)y * W + x] != 0;
  const size_t c = (size_t)(y + 1) * Wh + (x + 1);
  const float ex = 0.5f * (ph[c + 1] - ph[c - 1]);
  const float ey = 0.5f * (ph[c + Wh] - ph[c - Wh]);
  gx += in ? ex : 0.f;
  gy += in ? ey : 0.f;
  cnt += in ? 1.f : 0.f;
}

// One workgroup per (phase map, group of SROWS subaperture rows, run of whole
// subapertures across SBLOCK pixel columns).  Thread t owns pixel column
// x = x0 + t: for each subaperture row of the group it reads, row by row, the
// four neighbours its central differences need (consecutive threads read
// consecutive columns, so every load is coalesced) and sums the pupil-masked
// differences and the pupil count down the subaperture row.  The
// per-subaperture sums then add those column sums in column order (a fixed
// order, so results are bit-reproducible).  Walking the group's rows in turn
// reads the pixel rows two subaperture rows share while they are still in
// cache.
__global__ __launch_bounds__(SBLOCK) void slopes_kernel(const float* __restrict__ phase,
                                                        const int32_t* __restrict__ valid,
                                                        const uint8_t* __restrict__ pupil,
                                                        int n_sub_x, int n_sub_y, int p, int nv,
                                                        int subs_per_block,
                                                        float* __restrict__ slopes) {
  __shared__ float s_gx[2][SBLOCK], s_gy[2][SBLOCK], s_n[2][SBLOCK];
  __shared__ int s_kk[SROWS * SBLOCK];
  const int t = threadIdx.x;
  const int n_runs = (n_sub_x + subs_per_block - 1) / subs_per_block;
  const int grp = blockIdx.x / n_runs;
  const int u0 = (blockIdx.x - grp * n_runs) * subs_per_block;
  const int i = blockIdx.y;
  const int W = n_sub_x * p, H = n_sub_y * p;
  const int Wh = W + 2;
  const int nu = min(subs_per_block, n_sub_x - u0);
  const int x = u0 * p + t;
  const float* ph = phase + (size_t)i * (size_t)(H + 2) * (size_t)Wh;
  float* out = slopes + (size_t)i * 2 * nv;
  const int v0 = grp * SROWS, v_end = min(n_sub_y, v0 + SROWS);
  // valid-list index of every subaperture of the group (-1: not valid), all
  // looked up at once so that the binary searches' load chains overlap
  for (int e = t; e < (v_end - v0) * nu; e += SBLOCK) {
    const int k = (v0 + e / nu) * n_sub_x + u0 + e % nu;
    int lo = 0, hi = nv - 1, kk = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int vm = valid[mid];
      if (vm == k) {
        kk = mid;
        break;
      }
      if (vm < k) lo = mid + 1; else hi = mid - 1;
    }
    s_kk[e] = kk;
  }
  // two subaperture rows per step: twice the loads in flight between barriers
  for (int v = v0; v < v_end; v += 2) {
    const int nr = min(2, v_end - v);
    float gx[2] = {0.f, 0.f}, gy[2] = {0.f, 0.f}, cnt[2] = {0.f, 0.f};
    if (t < nu * p) {
      if (nr == 2) {
#pragma unroll 2
        for (int dy = 0; dy < p; ++dy)
#pragma unroll
          for (int r = 0; r < 2; ++r) column_terms(ph, pupil, W, Wh, x, (v + r) * p + dy,
                                                   gx[r], gy[r], cnt[r]);
      } else {
#pragma unroll 4
        for (int dy = 0; dy < p; ++dy)
          column_terms(ph, pupil, W, Wh, x, v * p + dy, gx[0], gy[0], cnt[0]);
      }
    }
    __syncthreads();   // the previous step's sums have been read (and s_kk written)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      s_gx[r][t] = gx[r];
      s_gy[r][t] = gy[r];
      s_n[r][t] = cnt[r];
    }
    __syncthreads();
    for (int e = t; e < nr * nu; e += SBLOCK) {
      const int r = e / nu, u = e - r * nu;
      const int kk = s_kk[(v - v0 + r) * nu + u];
      if (kk < 0) continue;
      float sx = 0.f, sy = 0.f, n = 0.f;
      for (int c = u * p; c < u * p + p; ++c) {
        sx += s_gx[r][c];
        sy += s_gy[r][c];
        n += s_n[r][c];
      }
      out[kk] = n > 0.f ? sx / n : 0.f;
      out[nv + kk] = n > 0.f ? sy / n : 0.f;
    }
  }
}
}  // namespace
}  // namespace synim

extern "C" int synim_sa_slopes(const float* phase, int n, const synim_wfs* wfs, float* slopes,
                               void* stream) {
  using namespace synim;
  if (!phase || !slopes) return SYNIM_E_NULL;
  int st = validate_wfs(wfs);
  if (st != SYNIM_OK) return st;
  if (n < 1 || n > 65535) return SYNIM_E_SHAPE;
  if (wfs->p > SBLOCK) return SYNIM_E_SHAPE;
  const int spb = SBLOCK / wfs->p;
  const long bx = (long)((wfs->n_sub_y + SROWS - 1) / SROWS) * ((wfs->n_sub_x + spb - 1) / spb);
  if (bx > 0x7fffffffL) return SYNIM_E_SHAPE;
  hipLaunchKernelGGL(slopes_kernel, dim3((unsigned)bx, n), dim3(SBLOCK), 0, (hipStream_t)stream,
                     phase, wfs->valid_idx, wfs->pupil, wfs->n_sub_x, wfs->n_sub_y, wfs->p,
                     wfs->n_valid, spb, slopes);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}
