// Standalone slope step (paper Sec. 2.2): central differences at every pupil
// pixel of a haloed phase map, averaged over each valid subaperture.
#include "common.hpp"

namespace synim {
namespace {

constexpr int WAVES = 4;

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wave per (valid subaperture, phase map).  Lanes walk the p*p pixels in a
// fixed order and the butterfly reduction is fixed, so results are
// bit-reproducible from run to run.
__global__ __launch_bounds__(64 * WAVES) void slopes_kernel(const float* __restrict__ phase,
                                                            const int32_t* __restrict__ valid,
                                                            const uint8_t* __restrict__ pupil,
                                                            int n_sub_x, int n_sub_y, int p,
                                                            int nv, float* __restrict__ slopes) {
  const int lane = threadIdx.x & 63;
  const int kk = blockIdx.x * WAVES + (threadIdx.x >> 6);
  const int i = blockIdx.y;
  if (kk >= nv) return;
  const int W = n_sub_x * p, H = n_sub_y * p;
  const int Wh = W + 2;
  const int k = valid[kk];
  const int u = k % n_sub_x, v = k / n_sub_x;
  const float* ph = phase + (size_t)i * (size_t)(H + 2) * (size_t)Wh;
  float sx = 0.f, sy = 0.f, cnt = 0.f;
  for (int e = lane; e < p * p; e += 64) {
    const int dy = e / p, dx = e - dy * p;
    const int x = u * p + dx, y = v * p + dy;
    if (pupil[(size_t)y * W + x]) {
      const size_t c = (size_t)(y + 1) * Wh + (x + 1);
      sx += 0.5f * (ph[c + 1] - ph[c - 1]);
      sy += 0.5f * (ph[c + Wh] - ph[c - Wh]);
      cnt += 1.f;
    }
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  cnt = wave_sum(cnt);
  if (lane == 0) {
    float* out = slopes + (size_t)i * 2 * nv;
    out[kk] = sx / cnt;
    out[nv + kk] = sy / cnt;
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
  const int bx = (wfs->n_valid + WAVES - 1) / WAVES;
  hipLaunchKernelGGL(slopes_kernel, dim3(bx, n), dim3(64 * WAVES), 0, (hipStream_t)stream, phase,
                     wfs->valid_idx, wfs->pupil, wfs->n_sub_x, wfs->n_sub_y, wfs->p,
                     wfs->n_valid, slopes);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}
