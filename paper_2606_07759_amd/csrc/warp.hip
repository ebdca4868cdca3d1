// Standalone single-step bilinear resampling of an IF stack onto the WFS grid
// (paper Sec. 2.1: the composite map is applied once, with one interpolation).
#include <cmath>

#include "common.hpp"

namespace synim {
namespace {

constexpr int WX = 256, WY = 4;   // four waves cover 256 consecutive output columns
// Workgroups per launch the IF loop is split for: enough to fill 256 CUs many
// times over, while each workgroup still reuses its FP64 source coordinates
// over tens of IFs (16k, 32k and 128k measured within 8% of each other).
constexpr long kTargetBlocks = 131072;

__global__ __launch_bounds__(WX* WY) void warp_kernel(const float* __restrict__ ifs, int n,
                                                      int H_in, int W_in, MapD m, int H_out,
                                                      int W_out, int halo, int if_per_block,
                                                      float* __restrict__ out,
                                                      int32_t* __restrict__ oob) {
  const int Wh = W_out + 2 * halo, Hh = H_out + 2 * halo;
  const int ox = blockIdx.x * WX + (threadIdx.x % WX);
  const int oy = blockIdx.y * WY + (threadIdx.x / WX);
  const bool active = ox < Wh && oy < Hh;

  double xs, ys;
  src_xy(m, ox - halo, oy - halo, xs, ys);
  const double fi = floor(xs), fj = floor(ys);
  const double ad = xs - fi, cd = ys - fj;
  // tap validity in FP64 first, so huge coordinates never reach an int conversion
  const bool vi0 = fi >= 0.0 && fi <= W_in - 1.0;
  const bool vi1 = fi + 1.0 >= 0.0 && fi + 1.0 <= W_in - 1.0;
  const bool vj0 = fj >= 0.0 && fj <= H_in - 1.0;
  const bool vj1 = fj + 1.0 >= 0.0 && fj + 1.0 <= H_in - 1.0;
  const int i0 = (vi0 || vi1) ? (int)fi : 0;
  const int j0 = (vj0 || vj1) ? (int)fj : 0;
  const float w00 = (float)((1.0 - ad) * (1.0 - cd));
  const float w01 = (float)(ad * (1.0 - cd));
  const float w10 = (float)((1.0 - ad) * cd);
  const float w11 = (float)(ad * cd);
  const bool t00 = active && vj0 && vi0, t01 = active && vj0 && vi1;
  const bool t10 = active && vj1 && vi0, t11 = active && vj1 && vi1;
  const size_t r0 = (size_t)j0 * W_in + i0;
  const size_t r1 = r0 + W_in;

  if (oob != nullptr && blockIdx.z == 0) {
    const bool o = active && (xs < 0.0 || xs > W_in - 1.0 || ys < 0.0 || ys > H_in - 1.0);
    const int cnt = __syncthreads_count(o);
    if (threadIdx.x == 0 && cnt > 0) atomicAdd(oob, cnt);
  }
  if (!active) return;

  const size_t plane_in = (size_t)H_in * W_in;
  const size_t plane_out = (size_t)Hh * Wh;
  const int i_begin = blockIdx.z * if_per_block;
  const int i_end = min(n, i_begin + if_per_block);
  const size_t o0 = (size_t)oy * Wh + ox;
  // UNR IFs per pass: all 4*UNR taps are loaded before the first one is used,
  // so a thread keeps that many gathers in flight instead of one IF's four.
  constexpr int UNR = 8;
  int i = i_begin;
  for (; i + UNR <= i_end; i += UNR) {
    float v[UNR][4];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const float* F = ifs + (size_t)(i + u) * plane_in;
      v[u][0] = t00 ? F[r0] : 0.0f;
      v[u][1] = t01 ? F[r0 + 1] : 0.0f;
      v[u][2] = t10 ? F[r1] : 0.0f;
      v[u][3] = t11 ? F[r1 + 1] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      float acc = 0.0f;
      if (t00) acc = __fmaf_rn(w00, v[u][0], acc);
      if (t01) acc = __fmaf_rn(w01, v[u][1], acc);
      if (t10) acc = __fmaf_rn(w10, v[u][2], acc);
      if (t11) acc = __fmaf_rn(w11, v[u][3], acc);
      out[(size_t)(i + u) * plane_out + o0] = acc;
    }
  }
  for (; i < i_end; ++i) {
    const float* F = ifs + (size_t)i * plane_in;
    float acc = 0.0f;
    if (t00) acc = __fmaf_rn(w00, F[r0], acc);
    if (t01) acc = __fmaf_rn(w01, F[r0 + 1], acc);
    if (t10) acc = __fmaf_rn(w10, F[r1], acc);
    if (t11) acc = __fmaf_rn(w11, F[r1 + 1], acc);
    out[(size_t)i * plane_out + o0] = acc;
  }
}

}  // namespace
}  // namespace synim

extern "C" int synim_affine_warp(const float* ifs, int n, int H_in, int W_in,
                                 const synim_affine* A, int H_out, int W_out, int halo, float* out,
                                 int32_t* oob_count, void* stream) {
  using namespace synim;
  if (!ifs || !A || !out) return SYNIM_E_NULL;
  if (n < 1 || H_in < 1 || W_in < 1 || H_out < 1 || W_out < 1 || halo < 0 || halo > 8)
    return SYNIM_E_SHAPE;
  if ((long)H_out + 2 * halo > 65536 || (long)W_out + 2 * halo > 65536) return SYNIM_E_SHAPE;
  const int Wh = W_out + 2 * halo, Hh = H_out + 2 * halo;
  const int bx = (Wh + WX - 1) / WX, by = (Hh + WY - 1) / WY;
  const long xy = (long)bx * by;
  int ipb = (int)std::max(1L, (long)n * xy / kTargetBlocks);
  ipb = std::min(ipb, n);
  const int bz = (n + ipb - 1) / ipb;
  if (bz > 65535) return SYNIM_E_SHAPE;
  hipLaunchKernelGGL(warp_kernel, dim3(bx, by, bz), dim3(WX * WY), 0, (hipStream_t)stream, ifs,
                     n, H_in, W_in, to_map(*A), H_out, W_out, halo, ipb, out, oob_count);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}
