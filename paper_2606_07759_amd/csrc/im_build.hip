// Fused interaction-matrix build, its Jacobian planes and the vector-Jacobian
// product (paper Sec. 2.1 single composite interpolation + Sec. 2.2 central
// differences and subaperture means).
//
// For a fixed geometry the three steps are linear in the IF F_a and identical
// for every actuator a:
//   s_x[k](a) = sum_{q in haloed k} c_x^k(q) phi_a(q) / (2 n_k),
//   c_x^k(q)  = [q-e_x in k, P=1] - [q+e_x in k, P=1]   (central differences
//              re-indexed on the sample they read),
//   phi_a(q)  = sum_taps w_tap(q) F_a[tap(q)]            (one bilinear
//              interpolation through the composite map).
// So each valid subaperture k owns one dense weight patch W_k (PH x PW IF
// pixels starting at its origin) with s_x[k](a) = <W_k^x, F_a[patch_k]>.
//
// Plan (FP64, on the device, once per geometry):
//   plan_subaps   origin and 1/(2 n_k) of each valid subaperture;
//   plan_weights  one thread per patch entry gathers every (q, tap) that lands
//                 on it; the Jacobian planes use d w_tap / d theta_j from the
//                 floor-cell bilinear gradient and the derivative maps;
//   plan_rows     groups subapertures into tiles and lists, for every tile,
//                 the IF rows its patches touch, each trimmed to the columns
//                 they cover, packed for staging.
// Stream (FP32, the hot loop): a persistent kernel hands out (actuator chunk,
// tile) items from per-XCD queues.  For an item the workgroup loads the tile's
// weights into registers, then streams every actuator's packed tile rows from
// HBM into LDS with buffer->LDS DMA (three stages, two actuators in flight)
// and contracts them against the patches; the LPS lanes that share a
// subaperture combine their partial sums with DPP.
#include <algorithm>
#include <map>
#include <climits>
#include <cmath>
#include <mutex>
#include <utility>
#include <vector>

#include "stream.hpp"

namespace synim {
namespace {

constexpr int GMAX_VJP = 16384;   // max workgroups of a VJP launch (partials buffer)

struct Map4 {
  MapD m[4];
};

// ------------------------------------------------------------------ planning


// Everything the plan kernels need for one (WFS, map) job.  Single builds
// pass it by value; batches pass a device table indexed by blockIdx.y.  The
// map (and the derivative maps) come by value, or from device memory when the
// pointers are set, so a captured graph re-plans from whatever maps the
// buffers hold at replay time.
struct PlanJob {
  MapD m;
  Map4 dm;
  const MapD* m_dev;          // overrides m when set
  const Map4* dm_dev;         // overrides dm when set
  const int32_t* valid;
  const uint8_t* pupil;
  int n_sub_x, n_sub_y, p, nv;
  int PH, PW, n_planes, cap_floats;
  int TX, TY, NSLOT, n_tiles_x;
  int n_tiles, BHmax;
  int H_in, W_in;             // IF grid, for the out-of-grid count (0: not counted)
  // Edge repair of a pre-masked IF stack (Sec. 2.3), null dm_mask: none.
  // The repaired phase of a subaperture's haloed samples reads core samples up
  // to REPAIR_PAD pixels beyond its haloed window, so with repair on the
  // sample window grows by that much on every side.
  const uint8_t* dm_mask;     // [H_in][W_in] DM-side mask the IFs were multiplied by
  double thresh;              // strict-core threshold on the interpolated mask
  uint8_t* core;              // [(H+2)][(W+2)] strict core S over the haloed WFS window
  double* ceff;               // [nv][RW*RW][2] effective (x, y) coefficient per sample
  int engine;                 // slope engine: ENGINE_CD or ENGINE_TSUM
  int2* origin;
  int2* hrows;                // [nv] patch rows [x, y) holding a non-zero weight
  double* inv2nk;
  float* weights;             // [plane][kk][x|y][PH*PW]
  int* slot_kk;               // [tile][NSLOT]
  int4* tile_info;            // [tile] (y0, rows, packed floats, 0)
  int2* rows;                 // [tile][BHmax] (first column, packed offset)
  int* status;
  int* counters;              // the stream kernel's work and sync counters
  // [nv] pupil pixels of each subaperture, bit y*p + x (x, y within it), for
  // p <= 8; null otherwise (the weights then read the pupil itself)
  unsigned long long* submask;
  MapD minv;                  // inverse of m's linear part (used when m_dev is null)
};

// The job of this workgroup.  TABLE = false: the one job passed by value, read
// from the kernel arguments (scalar loads); TABLE = true: row blockIdx.y of a
// device job table.
template <bool TABLE>
__device__ __forceinline__ const PlanJob& job_of(const PlanJob& one, const PlanJob* jobs) {
  if constexpr (TABLE) return jobs[blockIdx.y];
  else return one;
}

constexpr int REPAIR_PAD = 2;   // P1, P2 lie one and two pixels beyond an edge pixel

// Slope engines (Sec. 2.2): central differences averaged over the pupil pixels,
// or the G-tilt by telescoping sums, the phase difference across each pupil
// run of a row (column) read at the run's two boundary points.
constexpr int ENGINE_CD = 0, ENGINE_TSUM = 1;

// Sample window side of a subaperture: its haloed window, grown by REPAIR_PAD
// on every side when the plan repairs edges.
__host__ __device__ __forceinline__ int sample_window(int p, bool repair) {
  return p + 2 + (repair ? 2 * REPAIR_PAD : 0);
}

// ---------------------------------------------------------------- edge repair
// Step 1 (strict binarisation): S = {bilinear(M, A q + b) >= thresh} for every
// haloed WFS sample q = (x, y), x in [-1, W], y in [-1, H]; M is zero outside
// the IF grid.  Evaluated in FP64 with the plan's own source coordinates.
__global__ __launch_bounds__(256) void plan_core_kernel(PlanJob J) {
  const int W = J.n_sub_x * J.p, H = J.n_sub_y * J.p;
  const int W2 = W + 2;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)W2 * (H + 2)) return;
  const int x = (int)(i % W2) - 1, y = (int)(i / W2) - 1;
  const MapD m = J.m_dev ? *J.m_dev : J.m;
  double xs, ys;
  src_xy(m, x, y, xs, ys);
  const double fi = floor(xs), fj = floor(ys);
  const int ii = (int)fi, jj = (int)fj;
  const double a = xs - fi, c = ys - fj;
  auto Mv = [&](int u, int v) -> double {
    return (u >= 0 && u < J.W_in && v >= 0 && v < J.H_in && J.dm_mask[(size_t)v * J.W_in + u])
               ? 1.0 : 0.0;
  };
  const double mv = (1.0 - a) * (1.0 - c) * Mv(ii, jj) + a * (1.0 - c) * Mv(ii + 1, jj) +
                    (1.0 - a) * c * Mv(ii, jj + 1) + a * c * Mv(ii + 1, jj + 1);
  J.core[i] = mv >= J.thresh ? 1 : 0;
}

__device__ __forceinline__ int in_sub(const uint8_t* __restrict__ pupil, int W, int x0, int y0,
                                      int p, int x, int y);

// Steps 2 and 3 folded into the slope coefficients.  The repaired phase is
// phi_r(q) = phi(q) on S, the mean of the extrapolations 2 phi(P1) - phi(P2)
// or phi(P1) over the valid directions on the edge ring E = dilate(S) \ S
// (cross dilation), and 0 elsewhere; it is linear in phi.  A subaperture's
// slope sum_q c(q) phi_r(q) is therefore sum_q' c_eff(q') phi(q') with
//   c_eff(q') = [q' in S] c(q') + sum_{e in E} c(e) R(e, q'),
// R(e, e + d) = (2 if e + 2d in S else 1) / n_e and R(e, e + 2d) = -1 / n_e for
// the directions d with e + d in S (n_e of them).  One thread per (valid
// subaperture, sample of its grown window).
__global__ __launch_bounds__(256) void plan_ceff_kernel(PlanJob J) {
  const int p = J.p;
  const int RW = sample_window(p, true);
  const long gid = (long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (long)J.nv * RW * RW) return;
  const int kk = (int)(gid / (RW * RW));
  const int e0 = (int)(gid - (long)kk * RW * RW);
  const int k = J.valid[kk];
  const int u = k % J.n_sub_x, v = k / J.n_sub_x;
  const int W = J.n_sub_x * p, H = J.n_sub_y * p;
  const int x0 = u * p, y0 = v * p;
  const int qx = x0 - 1 - REPAIR_PAD + e0 % RW, qy = y0 - 1 - REPAIR_PAD + e0 / RW;
  auto inS = [&](int x, int y) -> bool {
    return x >= -1 && x <= W && y >= -1 && y <= H && J.core[(size_t)(y + 1) * (W + 2) + (x + 1)];
  };
  auto inWin = [&](int x, int y) -> bool { return x >= -1 && x <= W && y >= -1 && y <= H; };
  auto cx = [&](int x, int y) {
    return in_sub(J.pupil, W, x0, y0, p, x - 1, y) - in_sub(J.pupil, W, x0, y0, p, x + 1, y);
  };
  auto cy = [&](int x, int y) {
    return in_sub(J.pupil, W, x0, y0, p, x, y - 1) - in_sub(J.pupil, W, x0, y0, p, x, y + 1);
  };
  const int DX[4] = {1, -1, 0, 0}, DY[4] = {0, 0, 1, -1};
  double ex = 0.0, ey = 0.0;
  if (inS(qx, qy)) {
    ex = cx(qx, qy);
    ey = cy(qx, qy);
    // edge pixels e = q' - s d (s = 1, 2) whose extrapolation reads q'
    for (int d = 0; d < 4; ++d)
      for (int st = 1; st <= 2; ++st) {
        const int ex_ = qx - st * DX[d], ey_ = qy - st * DY[d];
        if (!inWin(ex_, ey_) || inS(ex_, ey_)) continue;
        const int ccx = cx(ex_, ey_), ccy = cy(ex_, ey_);
        if (ccx == 0 && ccy == 0) continue;
        // e is on the ring iff some cross neighbour is in S; n_e counts them
        int ne = 0;
        for (int t = 0; t < 4; ++t) ne += inS(ex_ + DX[t], ey_ + DY[t]) ? 1 : 0;
        if (ne == 0) continue;
        double r = 0.0;
        if (st == 1) {
          r = inS(ex_ + 2 * DX[d], ey_ + 2 * DY[d]) ? 2.0 : 1.0;   // q' = P1 along d
        } else {
          if (!inS(ex_ + DX[d], ey_ + DY[d])) continue;            // q' = P2 needs P1
          r = -1.0;
        }
        ex += ccx * r / ne;
        ey += ccy * r / ne;
      }
  }
  J.ceff[(size_t)gid * 2] = ex;
  J.ceff[(size_t)gid * 2 + 1] = ey;
}

// Whether pixel (x, y) is a pupil pixel of the subaperture with corner (x0, y0).
__device__ __forceinline__ int in_sub(const uint8_t* __restrict__ pupil, int W, int x0, int y0,
                                      int p, int x, int y) {
  return (x >= x0 && x < x0 + p && y >= y0 && y < y0 + p && pupil[(size_t)y * W + x]) ? 1 : 0;
}

// Origin (patch corner) and 1/(2 n_k) of each valid subaperture: one wave
// per subaperture, its lanes splitting the haloed window's samples and the
// subaperture's pixels (min, max and counts do not depend on the order).
constexpr int PLAN_SUBAPS_BLOCK = 256;
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <bool TABLE>
__global__ __launch_bounds__(PLAN_SUBAPS_BLOCK) void plan_subaps_kernel(
    PlanJob one, const PlanJob* __restrict__ jobs) {
  const PlanJob& J = job_of<TABLE>(one, jobs);
  const int kk = (int)((blockIdx.x * PLAN_SUBAPS_BLOCK + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (kk >= J.nv) return;   // whole waves
  const MapD m = J.m_dev ? *J.m_dev : J.m;
  const int p = J.p;
  const int k = J.valid[kk];
  const int u = k % J.n_sub_x, v = k / J.n_sub_x;
  const int W = J.n_sub_x * p, H = J.n_sub_y * p;
  const bool repair = J.dm_mask != nullptr;
  const int pad = repair ? REPAIR_PAD : 0;
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  const int hw = sample_window(p, repair);   // (grown) haloed window side
  for (int i = lane; i < hw * hw; i += 64) {
    const int y = v * p - 1 - pad + i / hw, x = u * p - 1 - pad + i % hw;
    if (x < -1 || x > W || y < -1 || y > H) continue;   // outside the WFS window
    double xs, ys;
    src_xy(m, x, y, xs, ys);
    xmin = fmin(xmin, xs);
    xmax = fmax(xmax, xs);
    ymin = fmin(ymin, ys);
    ymax = fmax(ymax, ys);
  }
  xmin = wave_min(xmin);
  ymin = wave_min(ymin);
  xmax = wave_max(xmax);
  ymax = wave_max(ymax);
  int nk = 0;
  for (int i = lane; i < p * p; i += 64) {
    const int y = v * p + i / p, x = u * p + i % p;
    nk += J.pupil[(size_t)y * W + x] ? 1 : 0;
  }
  for (int o = 32; o >= 1; o >>= 1) nk += __shfl_xor(nk, o, 64);
  if (J.submask != nullptr) {
    // lane i holds pixel (i % p, i / p) of the subaperture (p * p <= 64)
    const bool in = lane < p * p && J.pupil[(size_t)(v * p + lane / p) * W + u * p + lane % p];
    const unsigned long long mk = __ballot(in);
    if (lane == 0) J.submask[kk] = mk;
  }
  // samples this subaperture's central differences read (a non-zero c_x or
  // c_y) whose source point lies outside the IF grid: their bilinear taps
  // are zero-filled
  // (with edge repair: a non-zero effective coefficient)
  int oob = 0;
  if (J.W_in > 0) {
    const int x0 = u * p, y0 = v * p;
    for (int i = lane; i < hw * hw; i += 64) {
      const int y = y0 - 1 - pad + i / hw, x = x0 - 1 - pad + i % hw;
      bool used;
      if (repair) {
        const double* ce = J.ceff + ((size_t)kk * hw * hw + i) * 2;
        used = ce[0] != 0.0 || ce[1] != 0.0;
      } else {
        const int cx = in_sub(J.pupil, W, x0, y0, p, x - 1, y) - in_sub(J.pupil, W, x0, y0, p, x + 1, y);
        const int cy = in_sub(J.pupil, W, x0, y0, p, x, y - 1) - in_sub(J.pupil, W, x0, y0, p, x, y + 1);
        used = cx != 0 || cy != 0;
      }
      if (!used) continue;
      double xs, ys;
      src_xy(m, x, y, xs, ys);
      if (!(xs >= 0.0 && xs <= J.W_in - 1.0 && ys >= 0.0 && ys <= J.H_in - 1.0)) ++oob;
    }
    for (int o = 32; o >= 1; o >>= 1) oob += __shfl_xor(oob, o, 64);
  }
  if (lane != 0) return;
  if (oob > 0) atomicAdd(J.status + 2, oob);
  int ox = 0, oy = 0;
  if (fabs(xmin) < 1e9 && fabs(xmax) < 1e9 && fabs(ymin) < 1e9 && fabs(ymax) < 1e9) {
    ox = (int)floor(xmin);
    oy = (int)floor(ymin);
    // the last tap column is floor(xmax) + 1
    if ((int)floor(xmax) + 2 - ox > J.PW || (int)floor(ymax) + 2 - oy > J.PH)
      atomicOr(J.status, 1);
  } else {
    atomicOr(J.status, 1);
  }
  if (nk == 0) atomicOr(J.status, 4);
  J.origin[kk] = make_int2(ox, oy);
  J.hrows[kk] = make_int2(J.PH, 0);   // narrowed by plan_weights
  J.inv2nk[kk] = nk > 0 ? 1.0 / (2.0 * nk) : 0.0;
}


// Weight patch entry gid = (valid subaperture, patch entry): gathers, in a
// fixed order, every haloed-window sample q whose bilinear cell has this entry
// as a tap.  Weights layout: [plane][kk][component x|y][PH*PW].  A used entry
// widens its subaperture's row range in s_lo/s_hi (index kk - kk0).
// MULTI = false: the IM plane alone (J.n_planes == 1); the derivative maps and
// their accumulators then take no registers.
template <bool MULTI>
__device__ __forceinline__ void plan_weight_entry(const PlanJob& J, int E, long gid, int kk0,
                                                  int* s_lo, int* s_hi) {
  const MapD m = J.m_dev ? *J.m_dev : J.m;
  const int p = J.p;
  // inverse of the linear part, for the window of candidate samples
  MapD inv = J.minv;
  if (J.m_dev) {
    const double det = m.a00 * m.a11 - m.a01 * m.a10;
    inv = MapD{m.a11 / det, -m.a01 / det, -m.a10 / det, m.a00 / det, 0, 0};
  }
  const double rx = fabs(inv.a00) + fabs(inv.a01) + 0.01;
  const double ry = fabs(inv.a10) + fabs(inv.a11) + 0.01;
  const int kk = (int)(gid / E);
  const int e = (int)(gid - (long)kk * E);
  const int r = e / J.PW, c = e - (e / J.PW) * J.PW;
  const int k = J.valid[kk];
  const int u = k % J.n_sub_x, v = k / J.n_sub_x;
  const int W = J.n_sub_x * p;
  const int2 o = J.origin[kk];
  const int X = o.x + c, Y = o.y + r;

  // candidate window: p_o = A^-1 (p_s - b) with p_s in [X-1, X+1) x [Y-1, Y+1)
  const double dx = (double)X - m.b0, dy = (double)Y - m.b1;
  const double qx = inv.a00 * dx + inv.a01 * dy;
  const double qy = inv.a10 * dx + inv.a11 * dy;
  const bool repair = J.dm_mask != nullptr;
  const int pad = repair ? REPAIR_PAD : 0;
  const int RW = sample_window(p, repair);
  const int H = J.n_sub_y * p;
  const int xl = max(max(u * p - 1 - pad, -1), (int)ceil(qx - rx));
  const int xh = min(min(u * p + p + pad, W), (int)floor(qx + rx));
  const int yl = max(max(v * p - 1 - pad, -1), (int)ceil(qy - ry));
  const int yh = min(min(v * p + p + pad, H), (int)floor(qy + ry));
  const int sx0 = u * p, sy0 = v * p;
  // pixel (x, y) of the WFS grid is a pupil pixel of subaperture kk
  const unsigned long long mk = J.submask ? J.submask[kk] : 0ull;
  auto in_k = [&](int x, int y) -> int {
    if (J.submask == nullptr) return in_sub(J.pupil, W, sx0, sy0, p, x, y);
    return (x >= sx0 && x < sx0 + p && y >= sy0 && y < sy0 + p &&
            ((mk >> ((y - sy0) * p + (x - sx0))) & 1ull))
               ? 1
               : 0;
  };
  const int n_planes = MULTI ? J.n_planes : 1;
  Map4 dm{};
  if (MULTI && n_planes > 1) dm = J.dm_dev ? *J.dm_dev : J.dm;

  constexpr int NP = MULTI ? 5 : 1;
  double acc[NP][2];
#pragma unroll
  for (int j = 0; j < NP; ++j) acc[j][0] = acc[j][1] = 0.0;
  if (!MULTI && J.engine == ENGINE_TSUM) {
    // telescoping sums: boundary points (x + 1/2, y) with coefficient
    // [x in k] - [x + 1 in k] for s_x, (x, y + 1/2) with [y in k] - [y + 1 in k]
    // for s_y; each is one bilinear sample whose taps may include (X, Y)
    for (int comp = 0; comp < 2; ++comp)
      for (int a1 = 0; a1 < p; ++a1)          // row (s_x) or column (s_y) of k
        for (int a2 = -1; a2 < p; ++a2) {     // position of the boundary along it
          const int x = comp == 0 ? sx0 + a2 : sx0 + a1;
          const int y = comp == 0 ? sy0 + a1 : sy0 + a2;
          const int cc = comp == 0 ? in_k(x, y) - in_k(x + 1, y) : in_k(x, y) - in_k(x, y + 1);
          if (cc == 0) continue;
          const double px = comp == 0 ? x + 0.5 : (double)x;
          const double py = comp == 0 ? (double)y : y + 0.5;
          const double xs = __fma_rn(m.a01, py, __fma_rn(m.a00, px, m.b0));
          const double ys = __fma_rn(m.a11, py, __fma_rn(m.a10, px, m.b1));
          const double fi = floor(xs), fj = floor(ys);
          const double di = (double)X - fi, dj = (double)Y - fj;
          if (!((di == 0.0 || di == 1.0) && (dj == 0.0 || dj == 1.0))) continue;
          const double a = xs - fi, bb = ys - fj;
          const double w = (di == 0.0 ? 1.0 - a : a) * (dj == 0.0 ? 1.0 - bb : bb);
          acc[0][comp] += cc * w;
        }
    // the plan's scale is 1 / (2 n_k); the telescoping sum divides by n_k
    acc[0][0] *= 2.0;
    acc[0][1] *= 2.0;
  } else
  for (int y = yl; y <= yh; ++y)
    for (int x = xl; x <= xh; ++x) {
      double cx, cy;
      if (repair) {
        const double* ce =
            J.ceff + ((size_t)kk * RW * RW + (y - (sy0 - 1 - pad)) * RW + (x - (sx0 - 1 - pad))) * 2;
        cx = ce[0];
        cy = ce[1];
      } else {
        cx = in_k(x - 1, y) - in_k(x + 1, y);
        cy = in_k(x, y - 1) - in_k(x, y + 1);
      }
      if (cx == 0.0 && cy == 0.0) continue;
      double xs, ys;
      src_xy(m, x, y, xs, ys);
      const double fi = floor(xs), fj = floor(ys);
      const double di = (double)X - fi, dj = (double)Y - fj;
      if (!((di == 0.0 || di == 1.0) && (dj == 0.0 || dj == 1.0))) continue;
      const double a = xs - fi, b = ys - fj;
      const double wx = di == 0.0 ? 1.0 - a : a;
      const double wy = dj == 0.0 ? 1.0 - b : b;
      const double w = wx * wy;
      acc[0][0] += cx * w;
      acc[0][1] += cy * w;
      if constexpr (MULTI) {
        if (n_planes > 1) {
          // floor-cell gradient of the tap weight w.r.t. the source point
          const double dwa = (di == 0.0 ? -1.0 : 1.0) * wy;
          const double dwb = (dj == 0.0 ? -1.0 : 1.0) * wx;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double dxs = dm.m[j].a00 * x + dm.m[j].a01 * y + dm.m[j].b0;
            const double dys = dm.m[j].a10 * x + dm.m[j].a11 * y + dm.m[j].b1;
            const double d = dwa * dxs + dwb * dys;
            acc[1 + j][0] += cx * d;
            acc[1 + j][1] += cy * d;
          }
        }
      }
    }
  const double s = J.inv2nk[kk];
  bool used = false;
#pragma unroll
  for (int j = 0; j < NP; ++j)
    if (j < n_planes) used = used || acc[j][0] != 0.0 || acc[j][1] != 0.0;
  if (used) {
    atomicMin(&s_lo[kk - kk0], r);
    atomicMax(&s_hi[kk - kk0], r + 1);
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    if (j >= n_planes) break;
    float* w = J.weights + ((size_t)j * J.nv + kk) * 2 * E;
    w[e] = (float)(acc[j][0] * s);
    w[E + e] = (float)(acc[j][1] * s);
  }
}

// One thread per (valid subaperture, patch entry), PLAN_WEIGHTS_BLOCK per
// workgroup.  MULTI: some job has derivative planes (n_planes > 1).
constexpr int PLAN_WEIGHTS_BLOCK = 256;
template <bool MULTI, bool TABLE>
__global__ __launch_bounds__(PLAN_WEIGHTS_BLOCK) void plan_weights_kernel(
    PlanJob one, const PlanJob* __restrict__ jobs) {
  const PlanJob& J = job_of<TABLE>(one, jobs);
  const int E = J.PH * J.PW;
  const long g0 = (long)blockIdx.x * PLAN_WEIGHTS_BLOCK;
  const long gid = g0 + threadIdx.x;
  // rows holding a weight, per subaperture of this workgroup (at most
  // PLAN_WEIGHTS_BLOCK of them, relative to the first): reduced in LDS, then
  // one global atomic pair per subaperture and workgroup
  __shared__ int s_lo[PLAN_WEIGHTS_BLOCK], s_hi[PLAN_WEIGHTS_BLOCK];
  const int kk0 = (int)(g0 / E);
  s_lo[threadIdx.x] = INT_MAX;
  s_hi[threadIdx.x] = INT_MIN;
  __syncthreads();
  if (gid < (long)J.nv * E) plan_weight_entry<MULTI>(J, E, gid, kk0, s_lo, s_hi);
  __syncthreads();
  const int kk = kk0 + threadIdx.x;
  if (kk < J.nv && s_lo[threadIdx.x] != INT_MAX) {
    atomicMin(&J.hrows[kk].x, s_lo[threadIdx.x]);
    atomicMax(&J.hrows[kk].y, s_hi[threadIdx.x]);
  }
}

__device__ int find_valid(const int32_t* __restrict__ valid, int nv, int k) {
  int lo = 0, hi = nv - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int vm = valid[mid];
    if (vm == k) return mid;
    if (vm < k) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// One workgroup per tile: the IF rows its patches touch, each trimmed to the
// column interval those patches cover (aligned to 4 floats), packed one after
// the other.  tile_info[t] = (y0, rows, packed floats, 0), rows = 0 for an empty
// tile; rows[t*BHmax + r] = (first column of row r, packed offset of row r).
// Row table of tile t: slot_of(s) gives slot s's (origin, patch rows
// holding a weight), or hr.x >= hr.y for an empty slot.  Writes rows[t*BHmax
// + r], tile_info[t]; flags bit 1 of status[0] for a tile that does not fit,
// counts non-empty tiles in status[1].  256 threads.
// pitched: the rows are staged at one pitch per tile instead of packed, in
// one column frame: IF pixel (y, x) sits at (y - y0) * pitch + x - X0, X0 the
// tile's leftmost staged column and the pitch the width of the tile's column
// span rounded to 4 mod 8 floats.  Eight lanes reading one column of eight
// consecutive rows then hit eight different LDS banks, and a lane's bank is
// its subaperture's origin column mod 4 plus a multiple of 4 (packed rows of
// varying widths, or rows that each start at their own first column, start
// at offsets that collide).  Then tile_info[t] = (y0, rows, X0, pitch) and
// rows[t*BHmax + r] = (first, end) of row r's staged columns relative to X0;
// the vectors outside them are not fetched (the DMA zero-fills them).
constexpr int MAX_SLOTS = 256;   // slots of a tile: block size / lanes per subaperture
template <class SlotOf>
__device__ __forceinline__ void build_tile_rows(int t, int NS, int PW, int BHmax, int cap_floats,
                                                SlotOf slot_of, int2* rows_out, int4* tile_info,
                                                int* status, bool pitched = false) {
  __shared__ int s_ox[MAX_SLOTS], s_oy[MAX_SLOTS], s_oe[MAX_SLOTS];
  // per row: the slots' column span [s_lo, s_hi), then in place the staged
  // first column (s_lo) and width (s_hi)
  __shared__ int s_lo[MAX_TILE_ROWS], s_hi[MAX_TILE_ROWS];
  __shared__ int s_ymin, s_ymax;
  int* const s_x0 = s_lo;
  int* const s_w = s_hi;
  const int tid = threadIdx.x;
  if (NS > MAX_SLOTS) {
    if (tid == 0) {
      atomicOr(status, 2);   // tile skipped: its slopes stay unwritten
      tile_info[t] = make_int4(0, 0, 0, 0);
    }
    return;
  }
  if (tid == 0) {
    s_ymin = INT_MAX;
    s_ymax = INT_MIN;
  }
  for (int r = tid; r < MAX_TILE_ROWS; r += blockDim.x) {
    s_lo[r] = INT_MAX;
    s_hi[r] = INT_MIN;
  }
  __syncthreads();
  for (int s = tid; s < NS; s += blockDim.x) {
    int2 o, hr;
    slot_of(s, o, hr);
    // rows [oy, oe) of the IF grid that the subaperture's weights touch
    int ox = INT_MIN, oy = INT_MIN, oe = INT_MIN;
    if (hr.x < hr.y) {
      ox = o.x;
      oy = o.y + hr.x;
      oe = o.y + hr.y;
      atomicMin(&s_ymin, oy);
      atomicMax(&s_ymax, oe);
    }
    s_ox[s] = ox;
    s_oy[s] = oy;
    s_oe[s] = oe;
  }
  __syncthreads();
  const int y0 = s_ymin;
  if (y0 == INT_MAX) {
    if (tid == 0) tile_info[t] = make_int4(0, 0, 0, 0);
    return;
  }
  const int bh = s_ymax - y0;
  if (bh > BHmax || bh > MAX_TILE_ROWS) {
    if (tid == 0) {
      atomicOr(status, 2);
      tile_info[t] = make_int4(0, 0, 0, 0);
    }
    return;
  }
  // each slot widens the column span of every row its weights touch
  for (int s = tid; s < NS; s += blockDim.x) {
    const int oy = s_oy[s];
    if (oy == INT_MIN) continue;
    for (int y = oy; y < s_oe[s]; ++y) {
      atomicMin(&s_lo[y - y0], s_ox[s]);
      atomicMax(&s_hi[y - y0], s_ox[s] + PW);
    }
  }
  __syncthreads();
  for (int r = tid; r < bh; r += blockDim.x) {
    const int lo = s_lo[r], hi = s_hi[r];
    if (lo == INT_MAX) {
      s_x0[r] = 0;
      s_w[r] = 0;
    } else {
      const int x0 = floor_div(lo, 4) * 4;
      s_x0[r] = x0;
      s_w[r] = (hi - x0 + 3) / 4 * 4;
    }
  }
  __syncthreads();
  if (pitched) {
    __shared__ int s_xa, s_xb;
    if (tid == 0) {
      s_xa = INT_MAX;
      s_xb = INT_MIN;
    }
    __syncthreads();
    for (int r = tid; r < bh; r += blockDim.x)
      if (s_w[r] > 0) {
        atomicMin(&s_xa, s_x0[r]);
        atomicMax(&s_xb, s_x0[r] + s_w[r]);
      }
    __syncthreads();
    // the rows of the slots' weights cover [y0, y0 + bh), so some row is
    // non-empty; X0 and the span are multiples of 4
    const int X0 = s_xa, span = s_xb - s_xa;
    const int pitch = (span & 4) == 0 ? span + 4 : span;   // 4 mod 8 floats
    for (int r = tid; r < bh; r += blockDim.x)
      rows_out[(size_t)t * BHmax + r] =
          s_w[r] > 0 ? make_int2(s_x0[r] - X0, s_x0[r] - X0 + s_w[r]) : make_int2(0, 0);
    if (tid == 0) {
      if ((long)bh * pitch > cap_floats) {
        atomicOr(status, 2);   // tile skipped: its slopes stay unwritten
        tile_info[t] = make_int4(0, 0, 0, 0);
      } else {
        tile_info[t] = make_int4(y0, bh, X0, pitch);
        atomicAdd(status + 1, 1);
      }
    }
    return;
  }
  // packed offsets: exclusive prefix sum of the row widths (Hillis-Steele in
  // LDS over blocks of blockDim rows, carried across blocks)
  __shared__ int s_scan[256];
  __shared__ int s_carry;
  if (tid == 0) s_carry = 0;
  for (int r0 = 0; r0 < bh; r0 += blockDim.x) {
    const int r = r0 + tid;
    const int w = r < bh ? s_w[r] : 0;
    s_scan[tid] = w;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      const int add = tid >= o ? s_scan[tid - o] : 0;
      __syncthreads();
      s_scan[tid] += add;
      __syncthreads();
    }
    if (r < bh) rows_out[(size_t)t * BHmax + r] = make_int2(s_x0[r], s_carry + s_scan[tid] - w);
    __syncthreads();
    if (tid == 0) s_carry += s_scan[blockDim.x - 1];
    __syncthreads();
  }
  if (tid == 0) {
    const int off = s_carry;
    if (off > cap_floats) {
      atomicOr(status, 2);   // tile skipped: its slopes stay unwritten
      tile_info[t] = make_int4(0, 0, 0, 0);
    } else {
      tile_info[t] = make_int4(y0, bh, off, 0);
      atomicAdd(status + 1, 1);   // non-empty tiles
    }
  }
}

template <bool TABLE>
__global__ __launch_bounds__(256) void plan_rows_kernel(PlanJob one,
                                                        const PlanJob* __restrict__ jobs) {
  const PlanJob& J = job_of<TABLE>(one, jobs);
  const int t = blockIdx.x;
  if (t >= J.n_tiles) return;
  const int NS = J.NSLOT;
  build_tile_rows(
      t, NS, J.PW, J.BHmax, J.cap_floats,
      [&](int s, int2& o, int2& hr) {
        // the valid subaperture (if any) slot s of tile t holds, kept for the
        // stream kernel
        const int u = (t % J.n_tiles_x) * J.TX + s % J.TX;
        const int v = (t / J.n_tiles_x) * J.TY + s / J.TX;
        int kk = -1;
        if (u < J.n_sub_x && v < J.n_sub_y) kk = find_valid(J.valid, J.nv, v * J.n_sub_x + u);
        J.slot_kk[(size_t)t * NS + s] = kk;
        o = make_int2(0, 0);
        hr = make_int2(0, 0);
        if (kk >= 0) {
          o = J.origin[kk];
          hr = J.hrows[kk];
        }
      },
      J.rows, J.tile_info, J.status);
}

// Shared tiles of a batch: slot (pair << 20 | subaperture), the pair by its
// position in the job table, reads that pair's plan (origins and row ranges).
__global__ __launch_bounds__(256) void plan_rows_shared_kernel(
    const PlanJob* __restrict__ jobs, const int* __restrict__ jslots, int n_jt, int NS, int PW,
    int BHmax, int cap_floats, int2* rows_out, int4* tile_info, int* status) {
  const int t = blockIdx.x;
  if (t >= n_jt) return;
  build_tile_rows(
      t, NS, PW, BHmax, cap_floats,
      [&](int s, int2& o, int2& hr) {
        const int e = jslots[(size_t)t * NS + s];
        o = make_int2(0, 0);
        hr = make_int2(0, 0);
        if (e >= 0) {
          const PlanJob& J = jobs[e >> 20];
          o = J.origin[e & 0xFFFFF];
          hr = J.hrows[e & 0xFFFFF];
        }
      },
      rows_out, tile_info, status, true);
}

__global__ void zero_ints_kernel(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// A single plan's status words and the counters of the stream launch that
// follows it, in the plan's first kernel launch.
__global__ void zero_plan_kernel(int* __restrict__ status, int* __restrict__ counters,
                                 int n_counters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 16) status[i] = 0;
  if (i < n_counters) counters[i] = 0;
}

__global__ void zero_job_status_kernel(const PlanJob* __restrict__ jobs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n)
    for (int k = 0; k < 16; ++k) jobs[i].status[k] = 0;
}

// The streaming kernel (im_stream_kernel) and its variant record live in
// stream.hpp; the variant table is assembled from its parts below.
__global__ void vjp_finalize_kernel(const double* __restrict__ partials, int G,
                                    double* __restrict__ grad_theta) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < G; i += 256) s += partials[(size_t)j * G + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad_theta[j] = red[0];
}

// ------------------------------------------------------------------- variants

// (block, lanes/subaperture, rows/lane, patch columns, DMA per wave per stage,
// stages).  Three stages of small tiles let several workgroups share a CU;
// deeper pipelines of one workgroup per CU keep more bytes in flight.  The
// _PACK twins put up to 4 actuators in a stage when a tile's rows fill half
// of it or less (steep or small tiles), so such stages still carry full
// loads.
const Variant* variants_table(int* n_out) {
  static std::vector<Variant> all = [] {
    std::vector<Variant> v;
    using PartFn = const Variant* (*)(int*);
    const PartFn parts[kVariantParts] = {stream_variants_0, stream_variants_1,
                                         stream_variants_2, stream_variants_3,
                                         stream_variants_4, stream_variants_5,
                                         stream_variants_6, stream_variants_7};
    for (PartFn f : parts) {
      int n = 0;
      const Variant* p = f(&n);
      v.insert(v.end(), p, p + n);
    }
    return v;
  }();
  if (n_out) *n_out = (int)all.size();
  return all.data();
}
int num_variants() {
  int n = 0;
  variants_table(&n);
  return n;
}

// Schedules of the persistent stream kernel over (actuator chunk, tile) items.
//   SCHED_DYNAMIC  short chunks dealt round-robin to the XCD queues, items
//                  taken in chunk order (load balance across workgroups);
//   SCHED_XCD      one chunk per XCD (its eighth of the actuators) and at most
//                  one tile per workgroup of that XCD: every tile of the XCD's
//                  chunk runs at once, so neighbouring tiles read the IF rows
//                  they share at about the same time (one L2 fill), and each
//                  workgroup loads its weight patches once.
constexpr int SCHED_DYNAMIC = 0, SCHED_XCD = 1;

struct Dims {
  const Variant* var;
  int PH, PW;
  int TX, TY, NSLOT, n_tiles_x, n_tiles;
  int BWmax, BHmax;
  int sched;
  int sync_every;   // SCHED_XCD: actuators per sync block (0 = no sync)
};

struct WsLayout {
  size_t status, counters, scratch, origin, hrows, inv2nk, weights, slot_kk, tile_info, rows,
      partials, core, ceff, submask, total;
};

constexpr int MAX_PLANES = 5;
// Counter ints of a plan: 8 work-item counters per plane, then one XCD sync
// counter per plane and XCD, each on its own 128-byte line.
constexpr int COUNTER_INTS = 8 * MAX_PLANES + 8 * MAX_PLANES * 32;
// The finish count of a single-pair stream launch follows them, on a line of
// its own; a plan clears all PLAN_COUNTER_INTS, and every stream launch on the
// plan leaves them zero when it ends.
constexpr int FINISH_INT = COUNTER_INTS + 32;
constexpr int PLAN_COUNTER_INTS = FINISH_INT + 32;

// Patch size (columns, rows) a map needs for subapertures of p pixels: the
// haloed subaperture spans (p+1) output pixels, which the map stretches by
// the row sums of |A|; a bilinear tap adds one more column/row.
void patch_need(const synim_affine& A, int p, int* pw, int* ph) {
  const double ax = std::fabs(A.A[0][0]) + std::fabs(A.A[0][1]);
  const double ay = std::fabs(A.A[1][0]) + std::fabs(A.A[1][1]);
  *pw = (int)std::floor(ax * (p + 1) + 1e-7) + 3;
  *ph = (int)std::floor(ay * (p + 1) + 1e-7) + 3;
}

// Staged-box bound (floats per row BW, rows BH) of a tx x ty tile of variant
// v under map A: a subaperture's patch origin is the floor of an affine
// function of (u*p, v*p), so over a tile the origins spread by at most the
// map's stretch of the tile + 1; only the patch rows holding a weight are
// staged (at most ph_need of the PH), columns over the full patch width.
void tile_bound(const synim_affine& A, int p, const Variant& v, int tx, int ty, int ph_need,
                int* bw, int* bh) {
  const double sx = std::fabs(A.A[0][0]) * p * (tx - 1) + std::fabs(A.A[0][1]) * p * (ty - 1);
  const double sy = std::fabs(A.A[1][0]) * p * (tx - 1) + std::fabs(A.A[1][1]) * p * (ty - 1);
  *bw = ((int)std::floor(sx + 1e-6) + 1 + v.PW + 3 + 3) / 4 * 4;
  *bh = (int)std::floor(sy + 1e-6) + 1 + ph_need;
}

// Tile shapes of one variant for this geometry, cheapest first by the cost
// model: staged IF floats per subaperture (a partial 128-byte line counted at
// each row end), for tiles whose packed rows provably fit the stage buffers.
// pe: the subaperture span the patches must cover (w.p; larger when the
// plan repairs edges, whose sample window is wider).
int tiles_for_variant(const synim_wfs& w, const synim_affine& A, const Variant& v, Dims* out,
                      double* cost_out, int max_out, int pe = -1) {
  int pw_need, ph_need;
  patch_need(A, pe < 0 ? w.p : pe, &pw_need, &ph_need);
  if (v.PW < pw_need || v.PH() < ph_need) return 0;
  const int p = w.p;
  const long n_sub = (long)w.n_sub_x * w.n_sub_y;
  int n = 0;
  const int nslot_max = v.BLOCK / v.LPS;
  for (int ns = nslot_max; ns >= nslot_max / 4; ns /= 2)
    for (int tx = 1; tx <= ns; tx *= 2) {
      const int ty = ns / tx;
      if (tx * ty != ns) continue;   // slot s sits at (s % tx, s / tx) of its tile
      int BW, BH;
      tile_bound(A, p, v, tx, ty, ph_need, &BW, &BH);
      if ((long)BH * BW > v.cap_floats() || BH > MAX_TILE_ROWS) continue;
      const int ux = std::min(tx, w.n_sub_x), uy = std::min(ty, w.n_sub_y);
      const double fill = (double)(ux * uy) / ns;   // lanes with a subaperture
      const long tiles = (long)((w.n_sub_x + tx - 1) / tx) * ((w.n_sub_y + ty - 1) / ty);
      double cost = (double)(BW + 24) * BH / ((double)ux * uy) / fill;
      if (tiles * 8 < 64 && n_sub > 64) cost *= 1.5;   // too few tiles to spread
      // a packing twin ranks ahead of its one-actuator variant where the
      // tile bound leaves room for two actuators per stage, behind it
      // elsewhere (the exact rows may still leave room)
      if (v.PACK > 1) cost *= 2L * BH * BW <= v.cap_floats() ? 0.95 : 1.02;
      Dims d{};
      d.var = &v;
      d.PH = v.PH();
      d.PW = v.PW;
      d.TX = tx;
      d.TY = ty;
      d.NSLOT = ns;
      d.n_tiles_x = (w.n_sub_x + tx - 1) / tx;
      d.n_tiles = (int)tiles;
      d.BWmax = BW;
      d.BHmax = BH;
      int at = n;
      while (at > 0 && cost_out[at - 1] > cost) --at;
      if (at >= max_out) continue;
      for (int k = std::min(n, max_out - 1); k > at; --k) {
        out[k] = out[k - 1];
        cost_out[k] = cost_out[k - 1];
      }
      out[at] = d;
      cost_out[at] = cost;
      if (n < max_out) ++n;
    }
  return n;
}

int persistent_grid(StreamFn fn, int block);

// Every (variant, tile shape, schedule) that can run this geometry with the
// smallest weight patch that fits, cheapest first by the cost model.  The
// one-chunk-per-XCD schedule is offered for tile shapes with at most 5/4 as
// many tiles as an XCD has resident workgroups (known only with a device
// present).
int candidate_dims(const synim_wfs& w, const synim_affine& A, Dims* out, double* cost_out,
                   int max_out, int pe = -1) {
  int pw_need, ph_need;
  patch_need(A, pe < 0 ? w.p : pe, &pw_need, &ph_need);
  int best_area = INT_MAX;
  for (int i = 0; i < num_variants(); ++i)
    if (variants_table(nullptr)[i].PW >= pw_need && variants_table(nullptr)[i].PH() >= ph_need)
      best_area = std::min(best_area, variants_table(nullptr)[i].PW * variants_table(nullptr)[i].PH());
  if (best_area == INT_MAX) return 0;
  std::vector<std::pair<double, Dims>> all;
  for (int i = 0; i < num_variants(); ++i) {
    const Variant& v = variants_table(nullptr)[i];
    if (v.PW * v.PH() != best_area) continue;
    Dims tmp[64];
    double tc[64];
    const int m = tiles_for_variant(w, A, v, tmp, tc, 64, pe);
    const int G = persistent_grid(v.im4, v.BLOCK);
    for (int k = 0; k < m; ++k) {
      all.push_back({tc[k], tmp[k]});
      // empty tiles (outside the pupil) are skipped at once, so a few more
      // tiles than resident workgroups still start together
      if (G >= 8 && 4 * tmp[k].n_tiles <= 5 * (G / 8)) {
        // sync blocks of E actuators: E >= NST - 1 keeps the pipeline
        // prologue free of block entries
        const int e_min = std::max(2, v.NST - 1);
        const int es[4] = {e_min, std::max(4, e_min), std::max(8, e_min), 0};
        const double f[4] = {0.85, 0.86, 0.87, 0.9};
        for (int q = 0; q < 4; ++q) {
          if (q > 0 && q < 3 && es[q] == es[q - 1]) continue;
          Dims d = tmp[k];
          d.sched = SCHED_XCD;
          d.sync_every = es[q];
          all.push_back({f[q] * tc[k], d});
        }
      }
    }
  }
  std::stable_sort(all.begin(), all.end(),
                   [](const std::pair<double, Dims>& a, const std::pair<double, Dims>& b) {
                     return a.first < b.first;
                   });
  const int n = std::min((int)all.size(), max_out);
  for (int i = 0; i < n; ++i) {
    out[i] = all[i].second;
    cost_out[i] = all[i].first;
  }
  return n;
}

constexpr int MAX_CAND = 256;

// The configuration record of synim_im_config / synim_im_candidates.
void write_config(const Dims& d, int* o) {
  o[0] = d.var->BLOCK;
  o[1] = d.var->LPS;
  o[2] = d.PH;
  o[3] = d.PW;
  o[4] = d.TX;
  o[5] = d.TY;
  o[6] = d.var->NST;
  o[7] = d.sched == SCHED_XCD ? (d.sync_every > 0 ? d.sync_every : 1) : 0;
  o[8] = d.var->NJ4;
  o[9] = d.var->PACK;
}

// Autotune cache: geometry key -> (variant, tile shape) measured fastest.
struct TuneKey {
  int n_sub_x, n_sub_y, p, n_valid;
  long long a[4];   // the map's linear part, rounded to 1e-9
  bool operator==(const TuneKey& o) const {
    return n_sub_x == o.n_sub_x && n_sub_y == o.n_sub_y && p == o.p && n_valid == o.n_valid &&
           a[0] == o.a[0] && a[1] == o.a[1] && a[2] == o.a[2] && a[3] == o.a[3];
  }
};
struct TuneEntry {
  TuneKey key;
  int variant, TX, TY, NSLOT, sched, sync_every;
};
std::mutex g_tune_mu;
TuneEntry g_tune[256];
int g_tune_n = 0;

TuneKey tune_key(const synim_wfs& w, const synim_affine& A) {
  TuneKey k{w.n_sub_x, w.n_sub_y, w.p, w.n_valid, {}};
  for (int i = 0; i < 4; ++i) k.a[i] = std::llround(A.A[i / 2][i % 2] * 1e9);
  return k;
}

// The tuned configuration for this geometry if there is one, else the
// cost model's first choice.
int choose_dims(const synim_wfs& w, const synim_affine& A, Dims* d, int pe = -1) {
  Dims cand[MAX_CAND];
  double cost[MAX_CAND];
  const int n = candidate_dims(w, A, cand, cost, MAX_CAND, pe);
  if (n == 0) return SYNIM_E_UNSUPPORTED;
  *d = cand[0];
  const TuneKey key = tune_key(w, A);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int i = 0; i < g_tune_n; ++i)
    if (g_tune[i].key == key)
      for (int c = 0; c < n; ++c)
        if (cand[c].var == &variants_table(nullptr)[g_tune[i].variant] && cand[c].TX == g_tune[i].TX &&
            cand[c].TY == g_tune[i].TY && cand[c].NSLOT == g_tune[i].NSLOT &&
            cand[c].sched == g_tune[i].sched && cand[c].sync_every == g_tune[i].sync_every) {
          *d = cand[c];
          return SYNIM_OK;
        }
  return SYNIM_OK;
}

WsLayout layout(const synim_wfs& w, const Dims& d, int planes, bool repair = false) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  const size_t nv = (size_t)w.n_valid;
  L.status = take(16 * sizeof(int));
  L.counters = take(PLAN_COUNTER_INTS * sizeof(int));   // work items, sync blocks, finish
  L.scratch = take(64 * sizeof(float));
  L.origin = take(nv * sizeof(int2));
  L.hrows = take(nv * sizeof(int2));
  L.inv2nk = take(nv * sizeof(double));
  L.weights = take((size_t)planes * nv * 2 * d.PH * d.PW * sizeof(float));
  L.slot_kk = take((size_t)d.n_tiles * d.NSLOT * sizeof(int));
  L.tile_info = take((size_t)d.n_tiles * sizeof(int4));
  L.rows = take((size_t)d.n_tiles * d.BHmax * sizeof(int2));
  L.partials = take(planes > 1 ? (size_t)4 * GMAX_VJP * sizeof(double) : 0);
  const size_t rw = (size_t)sample_window(w.p, true);
  L.core = take(repair ? (size_t)(w.n_sub_x * w.p + 2) * (w.n_sub_y * w.p + 2) : 0);
  L.ceff = take(repair ? nv * rw * rw * 2 * sizeof(double) : 0);
  L.submask = take(nv * sizeof(unsigned long long));
  L.total = off;
  return L;
}

struct Plan {
  Dims d;
  WsLayout L;
  char* ws;
  int* status() const { return reinterpret_cast<int*>(ws + L.status); }
  int* counters() const { return reinterpret_cast<int*>(ws + L.counters); }
  float* scratch() const { return reinterpret_cast<float*>(ws + L.scratch); }
  int2* origin() const { return reinterpret_cast<int2*>(ws + L.origin); }
  int2* hrows() const { return reinterpret_cast<int2*>(ws + L.hrows); }
  double* inv2nk() const { return reinterpret_cast<double*>(ws + L.inv2nk); }
  float* weights() const { return reinterpret_cast<float*>(ws + L.weights); }
  int* slot_kk() const { return reinterpret_cast<int*>(ws + L.slot_kk); }
  int4* tile_info() const { return reinterpret_cast<int4*>(ws + L.tile_info); }
  int2* rows() const { return reinterpret_cast<int2*>(ws + L.rows); }
  double* partials() const { return reinterpret_cast<double*>(ws + L.partials); }
  uint8_t* core() const { return reinterpret_cast<uint8_t*>(ws + L.core); }
  double* ceff() const { return reinterpret_cast<double*>(ws + L.ceff); }
  unsigned long long* submask() const {
    return reinterpret_cast<unsigned long long*>(ws + L.submask);
  }
};

// Largest workspace any candidate configuration of this geometry needs, so a
// workspace sized once stays valid whatever the autotuner picks later.
size_t max_layout(const synim_wfs& w, const synim_affine& A, int planes, bool repair = false) {
  Dims cand[MAX_CAND];
  double cost[MAX_CAND];
  const int n = candidate_dims(w, A, cand, cost, MAX_CAND, repair ? w.p + 2 * REPAIR_PAD : -1);
  size_t m = 0;
  for (int i = 0; i < n; ++i) m = std::max(m, layout(w, cand[i], planes, repair).total);
  return m;
}

int build_plan_with(const synim_wfs& w, const synim_affine& A, const synim_affine* dA, int planes,
                    int H_in, int W_in, void* ws, size_t ws_bytes, hipStream_t st, Plan* P);
int enqueue_plan(const synim_wfs& w, const MapD& m, const MapD* m_dev, const Map4& dm, int planes,
                 int H_in, int W_in, const Plan& P, hipStream_t st);

// H_in, W_in: the IF grid the plan will stream, for the out-of-grid sample
// count (status word 2); 0 leaves it uncounted.
int build_plan(const synim_wfs& w, const synim_affine& A, const synim_affine* dA, int planes,
               int H_in, int W_in, void* ws, size_t ws_bytes, hipStream_t st, Plan* P) {
  int rc = choose_dims(w, A, &P->d);
  if (rc != SYNIM_OK) return rc;
  return build_plan_with(w, A, dA, planes, H_in, W_in, ws, ws_bytes, st, P);
}

int build_plan_with(const synim_wfs& w, const synim_affine& A, const synim_affine* dA, int planes,
                    int H_in, int W_in, void* ws, size_t ws_bytes, hipStream_t st, Plan* P) {
  P->L = layout(w, P->d, planes);
  if (!ws) return SYNIM_E_WORKSPACE;
  if (ws_bytes < P->L.total) return SYNIM_E_WORKSPACE;
  P->ws = static_cast<char*>(ws);
  const MapD m = to_map(A);
  const double det = m.a00 * m.a11 - m.a01 * m.a10;
  if (!(std::fabs(det) > 1e-12)) return SYNIM_E_PARAM;
  Map4 dm{};
  if (planes > 1)
    for (int j = 0; j < 4; ++j) dm.m[j] = to_map(dA[j]);
  return enqueue_plan(w, m, nullptr, dm, planes, H_in, W_in, *P, st);
}

// The plan job of one pair: its WFS, plan regions and kernel dimensions.
PlanJob make_job(const synim_wfs& w, const MapD& m, const MapD* m_dev, const Map4& dm,
                 const Map4* dm_dev, int planes, const Plan& P, int H_in, int W_in) {
  const Dims& d = P.d;
  PlanJob J{};
  J.m = m;
  J.dm = dm;
  J.m_dev = m_dev;
  J.dm_dev = dm_dev;
  J.valid = w.valid_idx;
  J.pupil = w.pupil;
  J.n_sub_x = w.n_sub_x;
  J.n_sub_y = w.n_sub_y;
  J.p = w.p;
  J.nv = w.n_valid;
  J.PH = d.PH;
  J.PW = d.PW;
  J.n_planes = planes;
  J.cap_floats = d.var->cap_floats();
  J.TX = d.TX;
  J.TY = d.TY;
  J.NSLOT = d.NSLOT;
  J.n_tiles_x = d.n_tiles_x;
  J.n_tiles = d.n_tiles;
  J.BHmax = d.BHmax;
  J.H_in = H_in;
  J.W_in = W_in;
  J.origin = P.origin();
  J.hrows = P.hrows();
  J.inv2nk = P.inv2nk();
  J.weights = P.weights();
  J.slot_kk = P.slot_kk();
  J.tile_info = P.tile_info();
  J.rows = P.rows();
  J.status = P.status();
  J.counters = P.counters();
  J.submask = w.p <= 8 ? P.submask() : nullptr;
  const double det = m.a00 * m.a11 - m.a01 * m.a10;
  J.minv = MapD{m.a11 / det, -m.a01 / det, -m.a10 / det, m.a00 / det, 0, 0};
  return J;
}

template <bool TABLE>
int enqueue_plan_kernels(const PlanJob& one, const PlanJob* jobs_dev, int n, int max_nv,
                         int max_e, int max_tiles, int planes, hipStream_t st,
                         bool tiles) {
  if (!TABLE && one.dm_mask) {
    // edge repair (single builds): strict core, then the effective coefficients
    const long cells = (long)(one.n_sub_x * one.p + 2) * (one.n_sub_y * one.p + 2);
    hipLaunchKernelGGL(plan_core_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st,
                       one);
    SYNIM_HIP_TRY(hipGetLastError());
    const int rw = sample_window(one.p, true);
    const long thr = (long)one.nv * rw * rw;
    hipLaunchKernelGGL(plan_ceff_kernel, dim3((unsigned)((thr + 255) / 256)), dim3(256), 0, st,
                       one);
    SYNIM_HIP_TRY(hipGetLastError());
  }
  for (int j0 = 0; j0 < n; j0 += 65535) {
    const int nj = std::min(65535, n - j0);
    const PlanJob* jt = TABLE ? jobs_dev + j0 : nullptr;
    hipLaunchKernelGGL(plan_subaps_kernel<TABLE>,
                       dim3((unsigned)(((long)max_nv * 64 + PLAN_SUBAPS_BLOCK - 1) / PLAN_SUBAPS_BLOCK),
                            nj),
                       dim3(PLAN_SUBAPS_BLOCK), 0, st, one, jt);
    SYNIM_HIP_TRY(hipGetLastError());
    const long nthr = (long)max_nv * max_e;
    const dim3 wgrid((unsigned)((nthr + PLAN_WEIGHTS_BLOCK - 1) / PLAN_WEIGHTS_BLOCK), nj);
    if (planes > 1)
      hipLaunchKernelGGL((plan_weights_kernel<true, TABLE>), wgrid, dim3(PLAN_WEIGHTS_BLOCK), 0,
                         st, one, jt);
    else
      hipLaunchKernelGGL((plan_weights_kernel<false, TABLE>), wgrid, dim3(PLAN_WEIGHTS_BLOCK), 0,
                         st, one, jt);
    SYNIM_HIP_TRY(hipGetLastError());
    if (!tiles) continue;
    hipLaunchKernelGGL(plan_rows_kernel<TABLE>, dim3(max_tiles, nj), dim3(256), 0, st, one, jt);
    SYNIM_HIP_TRY(hipGetLastError());
  }
  return SYNIM_OK;
}

// Enqueue the plan kernels for `n` jobs: one job by value (jobs_dev null) or
// a device table of n jobs (maxima give the grid extents).
// tiles = false: origins, row ranges and weights only (the batch's shared
// tiles replace the per-pair tile tables).
int enqueue_plans(const PlanJob& one, const PlanJob* jobs_dev, int n, int max_nv, int max_e,
                  int max_tiles, int planes, hipStream_t st, bool tiles = true) {
  if (jobs_dev) {
    hipLaunchKernelGGL(zero_job_status_kernel, dim3((n + 255) / 256), dim3(256), 0, st, jobs_dev,
                       n);
  } else {
    hipLaunchKernelGGL(zero_plan_kernel, dim3((PLAN_COUNTER_INTS + 255) / 256), dim3(256), 0,
                       st, one.status, one.counters, PLAN_COUNTER_INTS);
  }
  SYNIM_HIP_TRY(hipGetLastError());
  if (jobs_dev)
    return enqueue_plan_kernels<true>(one, jobs_dev, n, max_nv, max_e, max_tiles,
                                      planes, st, tiles);
  return enqueue_plan_kernels<false>(one, nullptr, 1, max_nv, max_e, max_tiles,
                                     planes, st, tiles);
}

int enqueue_plan(const synim_wfs& w, const MapD& m, const MapD* m_dev, const Map4& dm, int planes,
                 int H_in, int W_in, const Plan& P, hipStream_t st) {
  const PlanJob J = make_job(w, m, m_dev, dm, nullptr, planes, P, H_in, W_in);
  return enqueue_plans(J, nullptr, 1, J.nv, J.PH * J.PW, J.n_tiles, J.n_planes, st);
}

// Resident workgroups of a stream kernel on the current device (cached).
int persistent_grid(StreamFn fn, int block) {
  struct Entry {
    StreamFn fn;
    int dev, grid;
  };
  static Entry cache[64];
  static int n_cache = 0;
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  std::lock_guard<std::mutex> lk(mu);
  for (int i = 0; i < n_cache; ++i)
    if (cache[i].fn == fn && cache[i].dev == dev) return cache[i].grid;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn),
                                                   block, 0) != hipSuccess)
    return -1;
  int grid = std::max(8, (cus * std::max(1, per_cu) + 7) / 8 * 8);
  if (n_cache < 64) cache[n_cache++] = Entry{fn, dev, grid};
  return grid;
}

// Chunk length: enough (chunk, tile) items per workgroup for dynamic balance,
// chunks long enough to amortise each item's set-up, and no longer than
// CHUNK_MAX actuators: neighbouring tiles of a chunk start together and
// drift apart as they stream it, so short chunks keep their shared halo rows
// in L2 (measured on the ELT workload: 32 beats 64 by 8%, and 16-48 are
// within 3% of each other).
// A batch deals super-chunks of many small per-pair tiles, whose items are
// short already: there 64 measures best (MCAO workload: 14.1 ms against 14.7
// at 32).
constexpr int CHUNK_MAX = 32, CHUNK_MAX_BATCH = 64;
int chunk_for(long act_tiles, int G, int cap = CHUNK_MAX) {
  long chunk = (act_tiles + 4L * G - 1) / (4L * G);
  return (int)std::max(1L, std::min((long)cap, chunk));
}

// Chunks of a single-pair launch: as chunk_for asks, rounded up to a multiple
// of 8 so that every XCD queue holds the same number, the actuators split
// evenly over them (lengths differ by at most one).
int chunks_for(int n_act, int n_tiles, int G) {
  const long len = chunk_for((long)n_act * n_tiles, G);
  long nc = (n_act + len - 1) / len;
  nc = (nc + 7) / 8 * 8;
  return (int)std::min<long>(nc, n_act);
}

StreamFn pick_fn(const Variant& v, bool vec4, bool vjp, bool batch = false) {
  if (batch) return vec4 ? v.bim4 : v.bim1;
  return vjp ? (vec4 ? v.vjp4 : v.vjp1) : (vec4 ? v.im4 : v.im1);
}

// chunk > 0: chunks of that many actuators; chunk == 0: n_chunks even chunks
PairDesc pair_desc(const Plan& P, const float* ifs, int n_act, int H_in, int W_in, int nv,
                   float* out, int chunk, int n_chunks = 0) {
  PairDesc pd{};
  pd.ifs = ifs;
  pd.out = out;
  pd.origin = P.origin();
  pd.hrows = P.hrows();
  pd.weights = P.weights();
  pd.slot_kk = P.slot_kk();
  pd.tile_info = P.tile_info();
  pd.rows = P.rows();
  pd.n_act = n_act;
  pd.H_in = H_in;
  pd.W_in = W_in;
  pd.nv = nv;
  pd.n_tiles = P.d.n_tiles;
  pd.ns = P.d.NSLOT;
  pd.BHmax = P.d.BHmax;
  pd.chunk = chunk;
  pd.n_chunks = chunk > 0 ? (n_act + chunk - 1) / chunk : n_chunks;
  return pd;
}

int launch_stream(const Plan& P, const float* ifs, int n_act, int H_in, int W_in, int nv,
                  int plane0, int nplanes, float* out, const float* grad, hipStream_t st,
                  int* grid_out = nullptr) {
  const Dims& d = P.d;
  const Variant& v = *d.var;
  const bool vec4 = (W_in % 4 == 0) && ((reinterpret_cast<uintptr_t>(ifs) & 15) == 0);
  if ((long)H_in * W_in * 4 > INT_MAX) return SYNIM_E_SHAPE;   // 32-bit DMA offsets
  StreamFn fn = pick_fn(v, vec4, grad != nullptr);
  const int G = persistent_grid(fn, v.BLOCK);
  if (G < 0) return SYNIM_E_HIP;
  if (grad && G > GMAX_VJP) return SYNIM_E_SHAPE;
  StreamArgs g{};
  const int n_chunks = d.sched == SCHED_XCD ? std::min(8, n_act) : chunks_for(n_act, d.n_tiles, G);
  g.one = pair_desc(P, ifs, n_act, H_in, W_in, nv, out, 0, n_chunks);
  g.pairs = nullptr;
  g.counters = P.counters();
  g.scratch = P.scratch();
  g.plane0 = plane0;
  g.out_plane0 = plane0;
  g.grad = grad;
  g.partials = P.partials();
  g.sync_every = d.sched == SCHED_XCD ? d.sync_every : 0;
  g.sync_ctr = P.counters() + 8 * MAX_PLANES;
  g.n_active = P.status() + 1;
  // the plan cleared the counters, and every launch on it clears them as it
  // ends (its last workgroup)
  g.finish = P.counters() + FINISH_INT;
  g.n_counters = COUNTER_INTS;
  hipLaunchKernelGGL(fn, dim3((unsigned)G, 1, nplanes), dim3(v.BLOCK), 0, st, g);
  SYNIM_HIP_TRY(hipGetLastError());
  if (grid_out) *grid_out = G;
  return SYNIM_OK;
}

int check_common(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                 const synim_wfs* wfs) {
  if (!ifs || !A) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  if (n_act < 1 || H_in < 1 || W_in < 1) return SYNIM_E_SHAPE;
  if ((long)H_in * W_in > (long)INT_MAX / 4) return SYNIM_E_SHAPE;
  return SYNIM_OK;
}

}  // namespace
}  // namespace synim

using namespace synim;

extern "C" int synim_im_workspace(const synim_wfs* wfs, const synim_affine* A, int planes,
                                  size_t* bytes) {
  if (!wfs || !A || !bytes) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  if (planes != 1 && planes != 5) return SYNIM_E_PARAM;
  const size_t m = max_layout(*wfs, *A, planes);
  if (m == 0) return SYNIM_E_UNSUPPORTED;
  *bytes = m;
  return SYNIM_OK;
}

extern "C" int synim_im_autotune(const float* ifs, int n_act, int H_in, int W_in,
                                 const synim_affine* A, const synim_wfs* wfs, float* im, void* ws,
                                 size_t ws_bytes, int max_candidates, float* times_ms,
                                 int* n_tried, void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!im || !ws) return SYNIM_E_NULL;
  if (max_candidates < 1) return SYNIM_E_PARAM;
  hipStream_t st = (hipStream_t)stream;
  Dims cand[MAX_CAND];
  double cost[MAX_CAND];
  const int n = std::min(max_candidates, candidate_dims(*wfs, *A, cand, cost, MAX_CAND));
  if (n == 0) return SYNIM_E_UNSUPPORTED;
  hipEvent_t e0, e1;
  SYNIM_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SYNIM_E_HIP;
  }
  int best = -1;
  float best_ms = 1e30f;
  rc = SYNIM_OK;
  for (int c = 0; c < n && rc == SYNIM_OK; ++c) {
    Plan P{};
    P.d = cand[c];
    rc = build_plan_with(*wfs, *A, nullptr, 1, H_in, W_in, ws, ws_bytes, st, &P);
    if (rc != SYNIM_OK) break;
    rc = launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, st);   // warm
    if (rc != SYNIM_OK) break;
    const int reps = 3;
    if (hipEventRecord(e0, st) != hipSuccess) { rc = SYNIM_E_HIP; break; }
    for (int r = 0; r < reps && rc == SYNIM_OK; ++r)
      rc = launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, st);
    if (rc != SYNIM_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = SYNIM_E_HIP;
      break;
    }
    ms /= reps;
    if (times_ms) times_ms[c] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SYNIM_OK) return rc;
  if (n_tried) *n_tried = n;
  const TuneKey key = tune_key(*wfs, *A);
  TuneEntry e{key, (int)(cand[best].var - variants_table(nullptr)), cand[best].TX, cand[best].TY,
              cand[best].NSLOT, cand[best].sched, cand[best].sync_every};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int i = 0; i < g_tune_n; ++i)
    if (g_tune[i].key == key) {
      g_tune[i] = e;
      return SYNIM_OK;
    }
  if (g_tune_n < 256) g_tune[g_tune_n++] = e;
  return SYNIM_OK;
}

extern "C" int synim_im_config(const synim_wfs* wfs, const synim_affine* A, int* out) {
  if (!wfs || !A || !out) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  Dims d{};
  rc = choose_dims(*wfs, *A, &d);
  if (rc != SYNIM_OK) return rc;
  write_config(d, out);
  return SYNIM_OK;
}

extern "C" int synim_im_candidates(const synim_wfs* wfs, const synim_affine* A, int* out,
                                   int max_out, int* n_out) {
  if (!wfs || !A || !out || !n_out) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  Dims cand[MAX_CAND];
  double cost[MAX_CAND];
  const int n = std::min(max_out, candidate_dims(*wfs, *A, cand, cost, MAX_CAND));
  for (int i = 0; i < n; ++i) write_config(cand[i], out + SYNIM_CONFIG_INTS * i);
  *n_out = n;
  return SYNIM_OK;
}

extern "C" int synim_im_set_config(const synim_wfs* wfs, const synim_affine* A,
                                   const int* config) {
  if (!wfs || !A || !config) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  Dims cand[MAX_CAND];
  double cost[MAX_CAND];
  const int n = candidate_dims(*wfs, *A, cand, cost, MAX_CAND);
  for (int c = 0; c < n; ++c) {
    const Dims& d = cand[c];
    int mine[SYNIM_CONFIG_INTS];
    write_config(d, mine);
    if (!std::equal(mine, mine + SYNIM_CONFIG_INTS, config)) continue;
    const TuneKey key = tune_key(*wfs, *A);
    TuneEntry e{key, (int)(d.var - variants_table(nullptr)), d.TX, d.TY, d.NSLOT, d.sched, d.sync_every};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < g_tune_n; ++i)
      if (g_tune[i].key == key) {
        g_tune[i] = e;
        return SYNIM_OK;
      }
    if (g_tune_n < 256) g_tune[g_tune_n++] = e;
    return SYNIM_OK;
  }
  return SYNIM_E_UNSUPPORTED;
}

extern "C" void synim_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_n = 0;
}

namespace synim {
namespace {
// Autotune cache records: a header (format, variant-table signature, entry
// count), then per entry the geometry key (n_sub_x, n_sub_y, p, n_valid, the
// four rounded map entries as high/low 32-bit halves) and the configuration
// (variant index, TX, TY, NSLOT, schedule, sync blocks).
constexpr int TUNE_FORMAT = 1, TUNE_HEADER = 3, TUNE_ENTRY = 4 + 8 + 6;

// FNV-1a over every variant's parameters: a record names variants by their
// index in the table, so it is only valid for the same table.
int32_t variant_signature() {
  uint32_t h = 2166136261u;
  auto mix = [&](int v) {
    for (int b = 0; b < 4; ++b) {
      h ^= (uint32_t)((v >> (8 * b)) & 0xff);
      h *= 16777619u;
    }
  };
  const int n = num_variants();
  mix(n);
  for (int i = 0; i < n; ++i) {
    const Variant& v = variants_table(nullptr)[i];
    for (int x : {v.BLOCK, v.LPS, v.RPL, v.PW, v.NJ4, v.NST, v.PACK}) mix(x);
  }
  return (int32_t)h;
}
}  // namespace
}  // namespace synim

extern "C" int synim_autotune_export(int32_t* out, int cap, int* n_ints) {
  if (!n_ints) return SYNIM_E_NULL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int need = TUNE_HEADER + TUNE_ENTRY * g_tune_n;
  *n_ints = need;
  if (!out) return SYNIM_OK;
  if (cap < need) return SYNIM_E_SHAPE;
  out[0] = TUNE_FORMAT;
  out[1] = variant_signature();
  out[2] = g_tune_n;
  for (int i = 0; i < g_tune_n; ++i) {
    int32_t* o = out + TUNE_HEADER + TUNE_ENTRY * i;
    const TuneEntry& e = g_tune[i];
    o[0] = e.key.n_sub_x;
    o[1] = e.key.n_sub_y;
    o[2] = e.key.p;
    o[3] = e.key.n_valid;
    for (int j = 0; j < 4; ++j) {
      const uint64_t a = (uint64_t)e.key.a[j];
      o[4 + 2 * j] = (int32_t)(uint32_t)(a >> 32);
      o[5 + 2 * j] = (int32_t)(uint32_t)(a & 0xffffffffu);
    }
    o[12] = e.variant;
    o[13] = e.TX;
    o[14] = e.TY;
    o[15] = e.NSLOT;
    o[16] = e.sched;
    o[17] = e.sync_every;
  }
  return SYNIM_OK;
}

extern "C" int synim_autotune_import(const int32_t* in, int n_ints) {
  if (!in) return SYNIM_E_NULL;
  if (n_ints < TUNE_HEADER || in[0] != TUNE_FORMAT) return SYNIM_E_PARAM;
  const int n = in[2];
  if (n < 0 || n_ints != TUNE_HEADER + TUNE_ENTRY * n) return SYNIM_E_SHAPE;
  if (in[1] != variant_signature()) return SYNIM_E_UNSUPPORTED;
  std::vector<TuneEntry> es;
  for (int i = 0; i < n; ++i) {
    const int32_t* r = in + TUNE_HEADER + TUNE_ENTRY * i;
    TuneEntry e{};
    e.key.n_sub_x = r[0];
    e.key.n_sub_y = r[1];
    e.key.p = r[2];
    e.key.n_valid = r[3];
    for (int j = 0; j < 4; ++j)
      e.key.a[j] = (long long)(((uint64_t)(uint32_t)r[4 + 2 * j] << 32) | (uint32_t)r[5 + 2 * j]);
    e.variant = r[12];
    e.TX = r[13];
    e.TY = r[14];
    e.NSLOT = r[15];
    e.sched = r[16];
    e.sync_every = r[17];
    if (e.variant < 0 || e.variant >= num_variants() || e.TX < 1 || e.TY < 1 || e.NSLOT < 1 ||
        (e.sched != SCHED_DYNAMIC && e.sched != SCHED_XCD) || e.sync_every < 0)
      return SYNIM_E_PARAM;
    es.push_back(e);
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const TuneEntry& e : es) {
    int i = 0;
    while (i < g_tune_n && !(g_tune[i].key == e.key)) ++i;
    if (i < g_tune_n) g_tune[i] = e;
    else if (g_tune_n < 256) g_tune[g_tune_n++] = e;
    else return SYNIM_E_WORKSPACE;
  }
  return SYNIM_OK;
}

extern "C" int synim_im_build(const float* ifs, int n_act, int H_in, int W_in,
                              const synim_affine* A, const synim_wfs* wfs, float* im, void* ws,
                              size_t ws_bytes, void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!im) return SYNIM_E_NULL;
  hipStream_t st = (hipStream_t)stream;
  Plan P{};
  rc = build_plan(*wfs, *A, nullptr, 1, H_in, W_in, ws, ws_bytes, st, &P);
  if (rc != SYNIM_OK) return rc;
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, st);
}

// ------------------------------------------------- telescoping-sum engine
extern "C" int synim_im_build_tsum(const float* ifs, int n_act, int H_in, int W_in,
                                   const synim_affine* A, const synim_wfs* wfs, float* im,
                                   void* ws, size_t ws_bytes, void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!im || !ws) return SYNIM_E_NULL;
  hipStream_t st = (hipStream_t)stream;
  Plan P{};
  rc = choose_dims(*wfs, *A, &P.d);
  if (rc != SYNIM_OK) return rc;
  P.L = layout(*wfs, P.d, 1);
  if (ws_bytes < P.L.total) return SYNIM_E_WORKSPACE;
  P.ws = static_cast<char*>(ws);
  const MapD m = to_map(*A);
  const double det = m.a00 * m.a11 - m.a01 * m.a10;
  if (!(std::fabs(det) > 1e-12)) return SYNIM_E_PARAM;
  // no out-of-grid count: it is defined on the central-difference samples
  PlanJob J = make_job(*wfs, m, nullptr, Map4{}, nullptr, 1, P, 0, 0);
  J.engine = ENGINE_TSUM;
  rc = enqueue_plans(J, nullptr, 1, J.nv, J.PH * J.PW, J.n_tiles, 1, st);
  if (rc != SYNIM_OK) return rc;
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, st);
}

// ------------------------------------------------------- edge-repaired build
extern "C" int synim_im_repaired_workspace(const synim_wfs* wfs, const synim_affine* A,
                                           size_t* bytes) {
  if (!wfs || !A || !bytes) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  const size_t m = max_layout(*wfs, *A, 1, true);
  if (m == 0) return SYNIM_E_UNSUPPORTED;
  *bytes = m;
  return SYNIM_OK;
}

extern "C" int synim_im_build_repaired(const float* ifs, int n_act, int H_in, int W_in,
                                       const uint8_t* dm_mask, double threshold,
                                       const synim_affine* A, const synim_wfs* wfs, float* im,
                                       void* ws, size_t ws_bytes, void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!im || !dm_mask || !ws) return SYNIM_E_NULL;
  if (!(threshold > 0.0 && threshold <= 1.0)) return SYNIM_E_PARAM;
  hipStream_t st = (hipStream_t)stream;
  Plan P{};
  rc = choose_dims(*wfs, *A, &P.d, wfs->p + 2 * REPAIR_PAD);
  if (rc != SYNIM_OK) return rc;
  P.L = layout(*wfs, P.d, 1, true);
  if (ws_bytes < P.L.total) return SYNIM_E_WORKSPACE;
  P.ws = static_cast<char*>(ws);
  const MapD m = to_map(*A);
  const double det = m.a00 * m.a11 - m.a01 * m.a10;
  if (!(std::fabs(det) > 1e-12)) return SYNIM_E_PARAM;
  PlanJob J = make_job(*wfs, m, nullptr, Map4{}, nullptr, 1, P, H_in, W_in);
  J.dm_mask = dm_mask;
  J.thresh = threshold;
  J.core = P.core();
  J.ceff = P.ceff();
  rc = enqueue_plans(J, nullptr, 1, J.nv, J.PH * J.PW, J.n_tiles, 1, st);
  if (rc != SYNIM_OK) return rc;
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, st);
}

// ------------------------------------------------- build without allocation
// A fixed device array holds the plan of synim_im_build_noalloc, so that call
// needs no workspace and allocates nothing.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address is looked up once
// per device with hipGetSymbolAddress and only that address is passed on.
namespace {
constexpr size_t kNoallocBytes = (size_t)SYNIM_NOALLOC_WS_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];
constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocDevices] = {};

// Device address of this device's `scratch` (looked up on the first call).
int noalloc_scratch(void** out) {
  int dev = 0;
  SYNIM_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoallocDevices) return SYNIM_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    SYNIM_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SYNIM_E_HIP;
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return SYNIM_OK;
}
}  // namespace

extern "C" int synim_im_build_noalloc(const float* ifs, int n_act, int H_in, int W_in,
                                      const synim_affine* A, const synim_wfs* wfs, float* im,
                                      void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!im) return SYNIM_E_NULL;
  Plan P{};
  rc = choose_dims(*wfs, *A, &P.d);
  if (rc != SYNIM_OK) return rc;
  if (layout(*wfs, P.d, 1).total > kNoallocBytes) return SYNIM_E_WORKSPACE;
  void* ws = nullptr;
  rc = noalloc_scratch(&ws);
  if (rc != SYNIM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  rc = build_plan_with(*wfs, *A, nullptr, 1, H_in, W_in, ws, kNoallocBytes, st, &P);
  if (rc != SYNIM_OK) return rc;
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, st);
}

extern "C" int synim_im_jacobian(const float* ifs, int n_act, int H_in, int W_in,
                                 const synim_affine* A, const synim_affine* dA,
                                 const synim_wfs* wfs, float* im, float* dim, void* ws,
                                 size_t ws_bytes, void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!dA || !dim) return SYNIM_E_NULL;
  hipStream_t st = (hipStream_t)stream;
  Plan P{};
  rc = build_plan(*wfs, *A, dA, 5, H_in, W_in, ws, ws_bytes, st, &P);
  if (rc != SYNIM_OK) return rc;
  if (im) {
    rc = launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, st);
    if (rc != SYNIM_OK) return rc;
  }
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 1, 4, dim, nullptr, st);
}

extern "C" int synim_im_vjp(const float* ifs, int n_act, int H_in, int W_in,
                            const synim_affine* A, const synim_affine* dA, const synim_wfs* wfs,
                            const float* grad_im, double* grad_theta, void* ws, size_t ws_bytes,
                            void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!dA || !grad_im || !grad_theta) return SYNIM_E_NULL;
  hipStream_t st = (hipStream_t)stream;
  Plan P{};
  rc = build_plan(*wfs, *A, dA, 5, H_in, W_in, ws, ws_bytes, st, &P);
  if (rc != SYNIM_OK) return rc;
  int G = 0;
  rc = launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 1, 4, nullptr, grad_im, st, &G);
  if (rc != SYNIM_OK) return rc;
  hipLaunchKernelGGL(vjp_finalize_kernel, dim3(4), dim3(256), 0, st, P.partials(), G,
                     grad_theta);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

extern "C" int synim_im_plan(const synim_wfs* wfs, const synim_affine* A,
                             const synim_affine* dA, int planes, int H_in, int W_in, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!A) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  if (planes != 1 && planes != 5) return SYNIM_E_PARAM;
  if (planes == 5 && !dA) return SYNIM_E_NULL;
  if (H_in < 0 || W_in < 0 || (H_in == 0) != (W_in == 0)) return SYNIM_E_SHAPE;
  Plan P{};
  return build_plan(*wfs, *A, dA, planes, H_in, W_in, ws, ws_bytes, (hipStream_t)stream, &P);
}

extern "C" int synim_im_apply(const float* ifs, int n_act, int H_in, int W_in,
                              const synim_affine* A, const synim_wfs* wfs, int planes, int plane,
                              float* out, const void* ws, size_t ws_bytes, void* stream) {
  int rc = check_common(ifs, n_act, H_in, W_in, A, wfs);
  if (rc != SYNIM_OK) return rc;
  if (!out || !ws) return SYNIM_E_NULL;
  if ((planes != 1 && planes != 5) || plane < 0 || plane >= planes) return SYNIM_E_PARAM;
  Plan P{};
  rc = choose_dims(*wfs, *A, &P.d);
  if (rc != SYNIM_OK) return rc;
  P.L = layout(*wfs, P.d, planes);
  if (ws_bytes < P.L.total) return SYNIM_E_WORKSPACE;
  P.ws = static_cast<char*>(const_cast<void*>(ws));
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, plane, 1, out, nullptr,
                       (hipStream_t)stream);
}

extern "C" int synim_plan_status(const void* ws, int* host_out, void* stream) {
  if (!ws || !host_out) return SYNIM_E_NULL;
  SYNIM_HIP_TRY(hipMemcpyAsync(host_out, ws, sizeof(int), hipMemcpyDeviceToHost,
                               (hipStream_t)stream));
  SYNIM_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return SYNIM_OK;
}

extern "C" int synim_plan_oob(const void* ws, int64_t* host_count, void* stream) {
  if (!ws || !host_count) return SYNIM_E_NULL;
  int n = 0;
  SYNIM_HIP_TRY(hipMemcpyAsync(&n, static_cast<const int*>(ws) + 2, sizeof(int),
                               hipMemcpyDeviceToHost, (hipStream_t)stream));
  SYNIM_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  *host_count = n;
  return n > 0 ? SYNIM_E_OOB : SYNIM_OK;
}

// ------------------------------------------------------------------- batches
//
// Every (WFS, DM) pair of a multi-WFS system in one persistent launch (the
// paper's multi-WFS batch, Sec. 4.2): the pairs share one kernel variant, each
// pair keeps its own plan and tile shape, and DM-major super-chunks make the
// pairs that see a DM read each chunk of its IF stack side by side on one XCD.
// The maps live in device memory, so a captured graph replays after
// synim_batch_set_maps without re-capture.

struct synim_batch {
  std::vector<synim_wfs> wfs;
  std::vector<synim_dm> dms;
  std::vector<synim_pair> pairs;
  std::vector<int> group;        // pairs of one group share an IF stack (and its reads)
  int n_groups = 0;
  int planes = 1;                // 1: IM; 5: IM + 4 Jacobian planes (dmaps required)
  std::vector<int> order;        // pair indices sorted by group
  const Variant* var = nullptr;
  std::vector<Plan> plans;       // per pair (original index)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_maps = 0, off_pairs = 0, off_recs = 0, off_groups = 0, off_ctr = 0, off_scratch = 0;
  size_t off_jobs = 0, off_dmaps = 0;
  int max_nv = 0, max_e = 0, max_tiles = 0;
  int n_recs = 0;
  int rec_off[8] = {}, rec_cnt[8] = {}, xcd_items[8] = {};
  std::vector<SuperChunk> recs_host;   // to count the items of the first groups
  int G = 0;
  bool vec4 = true;
  MapD* staging = nullptr;       // pinned host copy of the maps
  hipEvent_t staged = nullptr;   // the last upload from `staging` has been read
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // Shared tiles (DM groups of several pairs): one set of tiles per group over
  // the IF grid, each holding the subapertures of every pair of the group
  // whose patches start in one cell of cell_x x cell_y pixels (see
  // build_shared).  The cells are fixed when the batch is bound; the exact
  // rows follow the maps on the device.
  bool shared = false;
  std::vector<std::vector<int>> valid_host;   // per WFS, copied once
  int cell_x = 0, cell_y = 0, jNS = 0, jBHmax = 0, n_jt = 0;
  std::vector<int> jslots_host;
  std::vector<int2> jgroups_host;
  std::vector<int2> jorigin_host;             // per slot of jslots_host: the binned origin
  size_t off_jslots = 0, off_jinfo = 0, off_jrows = 0, off_jgroups = 0, off_jstatus = 0;
  // A batch split by patch size (see batch_split): part k builds the pairs
  // part_idx[k] with a kernel variant of its own, in its own launch; the
  // batch itself then holds no tables.
  std::vector<synim_batch*> parts;
  std::vector<std::vector<int>> part_idx;
};

namespace synim {
namespace {

// Host estimate of a subaperture's patch origin: the floor of the map's
// minimum over the corners of the haloed window (the device takes the
// minimum over every sample; the two agree to within one pixel).
void host_origin(const MapD& m, int u, int v, int p, int* ox, int* oy) {
  double xmin = 1e300, ymin = 1e300;
  for (int cy = 0; cy < 2; ++cy)
    for (int cx = 0; cx < 2; ++cx) {
      const double x = u * p - 1 + cx * (p + 1), y = v * p - 1 + cy * (p + 1);
      xmin = std::min(xmin, m.a00 * x + m.a01 * y + m.b0);
      ymin = std::min(ymin, m.a10 * x + m.a11 * y + m.b1);
    }
  *ox = (int)std::floor(xmin);
  *oy = (int)std::floor(ymin);
}

// Margin (pixels) between a binned origin and the device's: host/device
// rounding (one pixel) plus one pixel of map drift before set_maps re-bins.
constexpr int SHARED_MARGIN = 2;

// Packs the subapertures of every pair of each DM group into shared tiles for
// variant v.  The slots of a group are ordered by the IF-space cell (cell_x x
// cell_y pixels) their patch origin falls in, then by origin, and taken in that
// order into tiles as long as a tile holds at most NSLOT subapertures and its
// staged box (origin spread + patch + the drift margin on every side, rows
// padded to 4 mod 8 floats) provably fits the stage buffers.  Tiles therefore
// come out nearly full: every lane of a tile runs the contraction whether its
// slot holds a subaperture or not, and the batch is bound by that arithmetic.
// The cell size is the one that minimises an estimate of the batch time: lane
// FMAs of all tiles plus the staged 128-byte lines at about 228 lane FMAs each
// (the ratio of the batch's FMA rate to its DMA streaming rate).
int build_shared(synim_batch* b, const Variant& v) {
  const int NS = v.BLOCK / v.LPS, PH = v.PH(), PW = v.PW, cap = v.cap_floats();
  const int np = (int)b->pairs.size();
  struct Sl {
    int pair, kk, ox, oy;
  };
  std::vector<std::vector<Sl>> per_group(b->n_groups);
  // slots name a pair by its position in group order (b->order): the pair
  // table and the plan jobs on the device are laid out that way
  for (int pos = 0; pos < np; ++pos) {
    const int i = b->order[pos];
    const synim_pair& pr = b->pairs[i];
    const synim_wfs& w = b->wfs[pr.wfs];
    const MapD m = to_map(pr.A);
    const std::vector<int>& valid = b->valid_host[pr.wfs];
    for (int kk = 0; kk < (int)valid.size(); ++kk) {
      const int k = valid[kk];
      int ox, oy;
      host_origin(m, k % w.n_sub_x, k / w.n_sub_x, w.p, &ox, &oy);
      per_group[b->group[i]].push_back(Sl{pos, kk, ox, oy});
    }
  }
  if (np >= (1 << 11)) return SYNIM_E_UNSUPPORTED;   // pair index field of a slot
  // staged-box bound of a tile whose origins span [x0, x1] x [y0, y1]: rows
  // at one pitch, the column span of the patches (drift margin on both sides,
  // ends at multiples of 4) rounded to 4 mod 8 floats (+ 4)
  auto box = [&](int x0, int x1, int y0, int y1, int* bw, int* bh) {
    *bw = (x1 - x0 + PW + 2 * SHARED_MARGIN + 3 + 3) / 4 * 4 + 4;
    *bh = y1 - y0 + PH + 2 * SHARED_MARGIN;
  };
  {
    int bw, bh;
    box(0, 0, 0, 0, &bw, &bh);
    if ((long)bw * bh > cap || bh > MAX_TILE_ROWS) return SYNIM_E_UNSUPPORTED;
  }
  auto order_by_cells = [&](std::vector<Sl>& sl, int cx, int cy) {
    std::stable_sort(sl.begin(), sl.end(), [&](const Sl& x, const Sl& y) {
      const int cxa = floor_div(x.ox, cx), cya = floor_div(x.oy, cy);
      const int cxb = floor_div(y.ox, cx), cyb = floor_div(y.oy, cy);
      if (cya != cyb) return cya < cyb;
      if (cxa != cxb) return cxa < cxb;
      if (x.oy != y.oy) return x.oy < y.oy;
      return x.ox < y.ox;
    });
  };
  // greedy packing of ordered slots; emit(begin, end, box width, box rows)
  auto pack = [&](const std::vector<Sl>& sl, auto&& emit) {
    size_t t0 = 0;
    int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    for (size_t i = 0; i < sl.size(); ++i) {
      if (i == t0) {
        x0 = x1 = sl[i].ox;
        y0 = y1 = sl[i].oy;
        continue;
      }
      const int nx0 = std::min(x0, sl[i].ox), nx1 = std::max(x1, sl[i].ox);
      const int ny0 = std::min(y0, sl[i].oy), ny1 = std::max(y1, sl[i].oy);
      int bw, bh;
      box(nx0, nx1, ny0, ny1, &bw, &bh);
      if (i - t0 >= (size_t)NS || (long)bw * bh > cap || bh > MAX_TILE_ROWS) {
        box(x0, x1, y0, y1, &bw, &bh);
        emit(t0, i, bw, bh);
        t0 = i;
        x0 = x1 = sl[i].ox;
        y0 = y1 = sl[i].oy;
      } else {
        x0 = nx0;
        x1 = nx1;
        y0 = ny0;
        y1 = ny1;
      }
    }
    if (t0 < sl.size()) {
      int bw, bh;
      box(x0, x1, y0, y1, &bw, &bh);
      emit(t0, sl.size(), bw, bh);
    }
  };
  static const int kCells[] = {8, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128};
  constexpr double kLineFmas = 228.0;
  const double fmas_per_tile = (double)NS * PH * PW * 2;
  double best = 1e300;
  int bx = 0, by = 0;
  for (int cx : kCells)
    for (int cy : kCells) {
      double cost = 0;
      for (auto sl : per_group) {
        order_by_cells(sl, cx, cy);
        pack(sl, [&](size_t, size_t, int bw, int bh) {
          cost += fmas_per_tile + kLineFmas * bh * (bw / 32.0 + 1.0);
        });
      }
      if (cost < best) {
        best = cost;
        bx = cx;
        by = cy;
      }
    }
  if (bx == 0) return SYNIM_E_UNSUPPORTED;
  b->cell_x = bx;
  b->cell_y = by;
  b->jNS = NS;
  b->jslots_host.clear();
  b->jorigin_host.clear();
  b->jgroups_host.assign(b->n_groups, make_int2(0, 0));
  int n_jt = 0, bh_max = 0;
  // Slot order within a tile.  The lanes of half a wave (32 / LPS slots) read
  // one column of their rows at the same time; a subaperture's rows, staged at
  // a pitch of 4 mod 8 floats, spread its lanes over the banks of one residue
  // mod 4, and that residue is its origin column's (the staged frame starts at
  // a multiple of 4).  The slots are therefore dealt to the half-wave groups
  // with the four residues as even as the tile's subapertures allow.
  const int HW = std::max(1, 32 / v.LPS);
  auto bank_order = [&](const Sl* in, size_t n) {
    std::vector<Sl> cls[4];
    for (size_t i = 0; i < n; ++i) cls[((in[i].ox % 4) + 4) % 4].push_back(in[i]);
    size_t next[4] = {0, 0, 0, 0};
    std::vector<Sl> out;
    out.reserve(n);
    while (out.size() < n) {
      int used[4] = {0, 0, 0, 0};
      for (int j = 0; j < HW && out.size() < n; ++j) {
        int best = -1;
        for (int c = 0; c < 4; ++c) {
          const size_t left = cls[c].size() - next[c];
          if (left == 0) continue;
          if (best < 0 || used[c] < used[best] ||
              (used[c] == used[best] && left > cls[best].size() - next[best]))
            best = c;
        }
        out.push_back(cls[best][next[best]++]);
        ++used[best];
      }
    }
    return out;
  };
  for (int gi = 0; gi < b->n_groups; ++gi) {
    std::vector<Sl> sl = per_group[gi];
    order_by_cells(sl, bx, by);
    b->jgroups_host[gi] = make_int2(n_jt, 0);
    pack(sl, [&](size_t t0, size_t t1, int, int bh) {
      const std::vector<Sl> ts = bank_order(sl.data() + t0, t1 - t0);
      for (int s = 0; s < NS; ++s) {
        if (s < (int)ts.size()) {
          b->jslots_host.push_back((ts[s].pair << 20) | ts[s].kk);
          b->jorigin_host.push_back(make_int2(ts[s].ox, ts[s].oy));
        } else {
          b->jslots_host.push_back(-1);
          b->jorigin_host.push_back(make_int2(INT_MIN, INT_MIN));
        }
      }
      bh_max = std::max(bh_max, bh);
      ++n_jt;
      ++b->jgroups_host[gi].y;
    });
  }
  // row tables sized for the most rows any tile can have (its narrowest box
  // at the stage capacity), so that re-packing for new maps keeps the layout
  int bw_min, bh_one;
  box(0, 0, 0, 0, &bw_min, &bh_one);
  b->jBHmax = std::max(bh_max, std::min(MAX_TILE_ROWS, cap / bw_min));
  b->n_jt = n_jt;
  return SYNIM_OK;
}

// Whether maps keep every binned subaperture within the margin its shared
// tile was sized for (else the tiles are rebuilt).
bool shared_maps_fit(const synim_batch* b, const synim_affine* maps) {
  for (size_t s = 0; s < b->jslots_host.size(); ++s) {
    const int e = b->jslots_host[s];
    if (e < 0) continue;
    const int i = b->order[e >> 20];
    const synim_pair& pr = b->pairs[i];
    const synim_wfs& w = b->wfs[pr.wfs];
    const int k = b->valid_host[pr.wfs][e & 0xFFFFF];
    int ox, oy;
    host_origin(to_map(maps[i]), k % w.n_sub_x, k / w.n_sub_x, w.p, &ox, &oy);
    const int2 o = b->jorigin_host[s];
    if (std::abs(ox - o.x) > SHARED_MARGIN - 1 || std::abs(oy - o.y) > SHARED_MARGIN - 1)
      return false;
  }
  return true;
}

// The batch's tables and the pairs' plans for kernel variant v, laid out in
// the workspace; returns the bytes needed (layout only if b->ws is null).
int batch_layout(synim_batch* b, const Variant& v, size_t* bytes) {
  const int np = (int)b->pairs.size();
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t at = off;
    off = align_up(off + n, 256);
    return at;
  };
  b->off_maps = take(np * sizeof(MapD));
  b->off_dmaps = take(b->planes > 1 ? np * sizeof(Map4) : 0);
  b->off_jobs = take(np * sizeof(PlanJob));
  b->off_pairs = take(np * sizeof(PairDesc));
  b->off_groups = take(b->n_groups * sizeof(int2));
  b->off_ctr = take(8 * MAX_PLANES * sizeof(int));   // one set of 8 per plane (grid z)
  b->off_scratch = take(64 * sizeof(float));
  // upper bound on the records: every DM chunk of length 1
  long max_recs = 0;
  for (int gi = 0; gi < b->n_groups; ++gi)
    for (int i = 0; i < np; ++i)
      if (b->group[i] == gi) {
        max_recs += b->dms[b->pairs[i].dm].n_act;
        break;
      }
  b->off_recs = take(max_recs * sizeof(SuperChunk));
  if (b->shared) {
    int rc = build_shared(b, v);
    if (rc != SYNIM_OK) return rc;
    // room for half as many tiles again, for re-binning after set_maps
    const size_t cap_jt = (size_t)b->n_jt + b->n_jt / 2 + 8;
    b->off_jslots = take(cap_jt * b->jNS * sizeof(int));
    b->off_jinfo = take(cap_jt * sizeof(int4));
    b->off_jrows = take(cap_jt * b->jBHmax * sizeof(int2));
    b->off_jgroups = take((size_t)b->n_groups * sizeof(int2));
    b->off_jstatus = take(16 * sizeof(int));
  }
  b->plans.assign(np, Plan{});
  for (int i = 0; i < np; ++i) {
    const synim_pair& pr = b->pairs[i];
    const synim_wfs& w = b->wfs[pr.wfs];
    Dims cand[64];
    double cost[64];
    if (tiles_for_variant(w, pr.A, v, cand, cost, 64) == 0) return SYNIM_E_UNSUPPORTED;
    Plan& P = b->plans[i];
    P.d = cand[0];
    P.L = layout(w, P.d, b->planes);
    const size_t at = take(P.L.total);
    P.ws = reinterpret_cast<char*>(at);   // offset until the workspace is bound
  }
  *bytes = off;
  return SYNIM_OK;
}

// Kernel variant for a batch: the smallest patch every pair fits, then the
// variant whose best tiles cost least summed over the pairs.
const Variant* batch_variant(const synim_batch* b, int rank) {
  int area_best = INT_MAX;
  for (int i = 0; i < num_variants(); ++i) {
    bool ok = true;
    for (const auto& pr : b->pairs) {
      int pw, ph;
      patch_need(pr.A, b->wfs[pr.wfs].p, &pw, &ph);
      if (variants_table(nullptr)[i].PW < pw || variants_table(nullptr)[i].PH() < ph) ok = false;
    }
    if (ok) area_best = std::min(area_best, variants_table(nullptr)[i].PW * variants_table(nullptr)[i].PH());
  }
  if (area_best == INT_MAX) return nullptr;
  std::vector<std::pair<double, int>> ranked;
  for (int i = 0; i < num_variants(); ++i) {
    const Variant& v = variants_table(nullptr)[i];
    if (v.PW * v.PH() != area_best) continue;
    double total = 0;
    bool ok = true;
    for (const auto& pr : b->pairs) {
      Dims c[64];
      double cost[64];
      if (tiles_for_variant(b->wfs[pr.wfs], pr.A, v, c, cost, 64) == 0) {
        ok = false;
        break;
      }
      total += cost[0] * b->wfs[pr.wfs].n_valid;
    }
    if (ok) ranked.push_back({total, i});
  }
  std::sort(ranked.begin(), ranked.end());
  if (rank >= (int)ranked.size()) return nullptr;
  return &variants_table(nullptr)[ranked[rank].second];
}

// Bind the layout of variant v to the workspace and upload the tables.
int batch_bind(synim_batch* b, const Variant& v, hipStream_t st) {
  size_t need = 0;
  int rc = batch_layout(b, v, &need);
  if (rc != SYNIM_OK) return rc;
  if (need > b->ws_bytes) return SYNIM_E_WORKSPACE;
  b->var = &v;
  const int np = (int)b->pairs.size();
  for (auto& P : b->plans) P.ws = b->ws + reinterpret_cast<size_t>(P.ws);
  b->vec4 = true;
  for (const auto& d : b->dms)
    if (d.W_in % 4 != 0 || (reinterpret_cast<uintptr_t>(d.ifs) & 15) != 0) b->vec4 = false;
  StreamFn fn = pick_fn(v, b->vec4, false, true);
  b->G = persistent_grid(fn, v.BLOCK);
  if (b->G < 0) return SYNIM_E_HIP;
  long act_tiles = 0;
  if (b->shared) {
    for (int gi = 0; gi < b->n_groups; ++gi)
      for (int i = 0; i < np; ++i)
        if (b->group[i] == gi) {
          act_tiles += (long)b->dms[b->pairs[i].dm].n_act * b->jgroups_host[gi].y;
          break;
        }
  } else {
    for (int i = 0; i < np; ++i)
      act_tiles += (long)b->dms[b->pairs[i].dm].n_act * b->plans[i].d.n_tiles;
  }
  const int chunk = chunk_for(act_tiles, b->G, CHUNK_MAX_BATCH);
  // pair table in DM order, groups, super-chunk records
  std::vector<PairDesc> pd(np);
  std::vector<int2> groups(b->n_groups, make_int2(0, 0));
  std::vector<int> group_nact(b->n_groups, 0);
  int at = 0;
  for (int gi = 0; gi < b->n_groups; ++gi) {
    groups[gi] = make_int2(at, 0);
    for (int i : b->order)
      if (b->group[i] == gi) {
        const synim_dm& dm = b->dms[b->pairs[i].dm];
        pd[at++] = pair_desc(b->plans[i], dm.ifs, dm.n_act, dm.H_in, dm.W_in,
                             b->wfs[b->pairs[i].wfs].n_valid, b->pairs[i].im, chunk);
        groups[gi].y++;
        group_nact[gi] = dm.n_act;
      }
  }
  std::vector<std::vector<SuperChunk>> per(8);
  long sc = 0;
  for (int gi = 0; gi < b->n_groups; ++gi) {
    if (groups[gi].y == 0) continue;
    int items = 0;
    if (b->shared)
      items = b->jgroups_host[gi].y;
    else
      for (int k = 0; k < groups[gi].y; ++k) items += pd[groups[gi].x + k].n_tiles;
    const int nch = (group_nact[gi] + chunk - 1) / chunk;
    for (int c = 0; c < nch; ++c, ++sc) {
      const int x = (int)(sc % 8);
      per[x].push_back(SuperChunk{0, gi, c, items});
    }
  }
  std::vector<SuperChunk> recs;
  for (int x = 0; x < 8; ++x) {
    b->rec_off[x] = (int)recs.size();
    b->rec_cnt[x] = (int)per[x].size();
    int acc = 0;
    for (auto r : per[x]) {
      r.item0 = acc;
      acc += r.items;
      recs.push_back(r);
    }
    b->xcd_items[x] = acc;
  }
  b->n_recs = (int)recs.size();
  b->recs_host = recs;
  std::vector<PlanJob> jobs(np);
  const MapD* maps_dev = reinterpret_cast<const MapD*>(b->ws + b->off_maps);
  b->max_nv = b->max_e = b->max_tiles = 0;
  // jobs in group order (the order of the pair table): shared-tile slots and
  // the group prefixes of batch_enqueue index them that way
  for (int pos = 0; pos < np; ++pos) {
    const int i = b->order[pos];
    const synim_pair& pr = b->pairs[i];
    const Map4* dmaps_dev =
        b->planes > 1 ? reinterpret_cast<const Map4*>(b->ws + b->off_dmaps) + i : nullptr;
    jobs[pos] = make_job(b->wfs[pr.wfs], to_map(pr.A), maps_dev + i, Map4{}, dmaps_dev,
                         b->planes, b->plans[i], b->dms[pr.dm].H_in, b->dms[pr.dm].W_in);
    b->max_nv = std::max(b->max_nv, jobs[pos].nv);
    b->max_e = std::max(b->max_e, jobs[pos].PH * jobs[pos].PW);
    b->max_tiles = std::max(b->max_tiles, jobs[pos].n_tiles);
  }
  SYNIM_HIP_TRY(hipMemcpyAsync(b->ws + b->off_jobs, jobs.data(), np * sizeof(PlanJob),
                               hipMemcpyHostToDevice, st));
  SYNIM_HIP_TRY(hipMemcpyAsync(b->ws + b->off_pairs, pd.data(), np * sizeof(PairDesc),
                               hipMemcpyHostToDevice, st));
  SYNIM_HIP_TRY(hipMemcpyAsync(b->ws + b->off_groups, groups.data(), groups.size() * sizeof(int2),
                               hipMemcpyHostToDevice, st));
  if (!recs.empty())
    SYNIM_HIP_TRY(hipMemcpyAsync(b->ws + b->off_recs, recs.data(),
                                 recs.size() * sizeof(SuperChunk), hipMemcpyHostToDevice, st));
  if (b->shared) {
    if (!b->jslots_host.empty())
      SYNIM_HIP_TRY(hipMemcpyAsync(b->ws + b->off_jslots, b->jslots_host.data(),
                                   b->jslots_host.size() * sizeof(int), hipMemcpyHostToDevice, st));
    SYNIM_HIP_TRY(hipMemcpyAsync(b->ws + b->off_jgroups, b->jgroups_host.data(),
                                 b->jgroups_host.size() * sizeof(int2), hipMemcpyHostToDevice,
                                 st));
  }
  SYNIM_HIP_TRY(hipStreamSynchronize(st));   // the host vectors go out of scope
  return SYNIM_OK;
}

// Enqueue plans and the stream launch for the pairs of the first n_groups
// groups (all by default): their records form a prefix of every XCD queue,
// since the records are dealt group-major, and their plan jobs a prefix of
// the job table, which is in group order.
int batch_enqueue(synim_batch* b, hipStream_t st, int n_groups = -1) {
  int np = (int)b->pairs.size();
  int items[8];
  for (int x = 0; x < 8; ++x) items[x] = b->xcd_items[x];
  if (n_groups >= 0 && n_groups < b->n_groups) {
    np = 0;
    for (int i = 0; i < (int)b->pairs.size(); ++i) np += b->group[i] < n_groups ? 1 : 0;
    for (int x = 0; x < 8; ++x) {
      int acc = 0;
      for (int r = 0; r < b->rec_cnt[x]; ++r) {
        const SuperChunk& rc = b->recs_host[b->rec_off[x] + r];
        if (rc.dm >= n_groups) break;
        acc += rc.items;
      }
      items[x] = acc;
    }
  }
  const PlanJob* jobs = reinterpret_cast<const PlanJob*>(b->ws + b->off_jobs);
  int rc = enqueue_plans(PlanJob{}, jobs, np, b->max_nv, b->max_e, b->max_tiles,
                         b->planes, st, !b->shared);
  if (rc != SYNIM_OK) return rc;
  StreamArgs g{};
  if (b->shared) {
    int* jstatus = reinterpret_cast<int*>(b->ws + b->off_jstatus);
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, jstatus, 16);
    SYNIM_HIP_TRY(hipGetLastError());
    if (b->n_jt > 0) {
      hipLaunchKernelGGL(plan_rows_shared_kernel, dim3((unsigned)b->n_jt), dim3(256), 0, st, jobs,
                         reinterpret_cast<const int*>(b->ws + b->off_jslots), b->n_jt, b->jNS,
                         b->var->PW, b->jBHmax, b->var->cap_floats(),
                         reinterpret_cast<int2*>(b->ws + b->off_jrows),
                         reinterpret_cast<int4*>(b->ws + b->off_jinfo), jstatus);
      SYNIM_HIP_TRY(hipGetLastError());
    }
    g.jslots = reinterpret_cast<const int*>(b->ws + b->off_jslots);
    g.jinfo = reinterpret_cast<const int4*>(b->ws + b->off_jinfo);
    g.jrows = reinterpret_cast<const int2*>(b->ws + b->off_jrows);
    g.jgroups = reinterpret_cast<const int2*>(b->ws + b->off_jgroups);
    g.jNS = b->jNS;
    g.jBHmax = b->jBHmax;
  }
  g.pairs = reinterpret_cast<const PairDesc*>(b->ws + b->off_pairs);
  g.recs = reinterpret_cast<const SuperChunk*>(b->ws + b->off_recs);
  g.groups = reinterpret_cast<const int2*>(b->ws + b->off_groups);
  for (int x = 0; x < 8; ++x) {
    g.rec_off[x] = b->rec_off[x];
    g.rec_cnt[x] = b->rec_cnt[x];
    g.xcd_items[x] = items[x];
  }
  g.counters = reinterpret_cast<int*>(b->ws + b->off_ctr);
  g.scratch = reinterpret_cast<float*>(b->ws + b->off_scratch);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, g.counters, 8 * b->planes);
  SYNIM_HIP_TRY(hipGetLastError());
  StreamFn fn = pick_fn(*b->var, b->vec4, false, true);
  hipLaunchKernelGGL(fn, dim3((unsigned)b->G, 1, b->planes), dim3(b->var->BLOCK), 0, st, g);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

void batch_drop_graph(synim_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

int batch_check(const synim_wfs* wfs, int n_wfs, const synim_dm* dms, int n_dm,
                const synim_pair* pairs, int n_pairs) {
  if (!wfs || !dms || !pairs) return SYNIM_E_NULL;
  if (n_wfs < 1 || n_dm < 1 || n_pairs < 1) return SYNIM_E_SHAPE;
  for (int i = 0; i < n_wfs; ++i) {
    int rc = validate_wfs(&wfs[i]);
    if (rc != SYNIM_OK) return rc;
  }
  for (int i = 0; i < n_dm; ++i) {
    if (!dms[i].ifs) return SYNIM_E_NULL;
    if (dms[i].n_act < 1 || dms[i].H_in < 1 || dms[i].W_in < 1) return SYNIM_E_SHAPE;
    if ((long)dms[i].H_in * dms[i].W_in * 4 > INT_MAX) return SYNIM_E_SHAPE;
  }
  for (int i = 0; i < n_pairs; ++i) {
    if (!pairs[i].im) return SYNIM_E_NULL;
    if (pairs[i].wfs < 0 || pairs[i].wfs >= n_wfs || pairs[i].dm < 0 || pairs[i].dm >= n_dm)
      return SYNIM_E_SHAPE;
  }
  return SYNIM_OK;
}

// group: nullptr groups the pairs by DM (pairs sharing a DM share its reads).
void batch_fill(synim_batch* b, const synim_wfs* wfs, int n_wfs, const synim_dm* dms, int n_dm,
                const synim_pair* pairs, int n_pairs, const int* group = nullptr,
                int n_groups = 0, int planes = 1) {
  b->wfs.assign(wfs, wfs + n_wfs);
  b->dms.assign(dms, dms + n_dm);
  b->pairs.assign(pairs, pairs + n_pairs);
  b->planes = planes;
  b->group.resize(n_pairs);
  for (int i = 0; i < n_pairs; ++i) b->group[i] = group ? group[i] : pairs[i].dm;
  b->n_groups = group ? n_groups : n_dm;
  b->order.resize(n_pairs);
  for (int i = 0; i < n_pairs; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return b->group[x] < b->group[y]; });
}

// Shared tiles when some DM group holds several single-plane pairs; the
// WFS valid lists come to the host for the binning.  (An earlier build of this
// path gave wrong values and a memory fault: its DMA instructions read their
// buffer resource one wait state after the v_readfirstlane that wrote it, where
// 5 are needed, so a DMA could stream from a stale or half-updated address.
// The DMA padding in the stream kernel removes that hazard, and a CPU test
// checks the wait states of every LDS DMA in the built assembly.)
constexpr bool kSharedTiles = true;
int batch_pick_shared(synim_batch* b) {
  b->shared = false;
  if (!kSharedTiles || b->planes != 1) return SYNIM_OK;
  std::vector<int> per(b->n_groups, 0);
  for (int gi : b->group) ++per[gi];
  bool any = false;
  for (int c : per) any = any || c > 1;
  if (!any) return SYNIM_OK;
  b->valid_host.assign(b->wfs.size(), {});
  for (size_t w = 0; w < b->wfs.size(); ++w) {
    b->valid_host[w].resize(b->wfs[w].n_valid);
    SYNIM_HIP_TRY(hipMemcpy(b->valid_host[w].data(), b->wfs[w].valid_idx,
                            b->wfs[w].n_valid * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  b->shared = true;
  return SYNIM_OK;
}

// Smallest patch (PW * PH) of the variant table that holds a pair's patches,
// 0 if none does.
int min_patch_area(const synim_affine& A, int p) {
  int pw, ph;
  patch_need(A, p, &pw, &ph);
  int best = 0;
  for (int i = 0; i < num_variants(); ++i) {
    const Variant& v = variants_table(nullptr)[i];
    if (v.PW >= pw && v.PH() >= ph && (best == 0 || v.PW * v.PH() < best)) best = v.PW * v.PH();
  }
  return best;
}

// Parts of an IM batch by patch size.  Every lane of a tile runs the whole
// patch of the batch's one kernel variant, sized for its most demanding pair;
// where the pairs' own smallest patches would cut those FMAs by at least
// kSplitGain (weighted by subapertures x actuators), the pairs are grouped by
// that smallest patch, smallest first, and each group becomes a batch of its
// own (its own variant, shared tiles and launch).  Only batches with shared
// tiles split (IM planes, some DM seen by several pairs); the parts of a DM
// then each stage its rows, so HBM reads them once per part.  Empty: no split.
constexpr double kSplitGain = 0.15;
std::vector<std::vector<int>> batch_split(const synim_wfs* wfs, const synim_dm* dms,
                                          const synim_pair* pairs, int n_pairs) {
  std::vector<int> per_dm(n_pairs, 0), area(n_pairs);
  bool several = false;
  for (int i = 0; i < n_pairs; ++i) several = several || ++per_dm[pairs[i].dm] > 1;
  if (!several) return {};
  int amax = 0;
  for (int i = 0; i < n_pairs; ++i) {
    area[i] = min_patch_area(pairs[i].A, wfs[pairs[i].wfs].p);
    if (area[i] == 0) return {};
    amax = std::max(amax, area[i]);
  }
  double whole = 0, split = 0;
  for (int i = 0; i < n_pairs; ++i) {
    const double w = (double)wfs[pairs[i].wfs].n_valid * dms[pairs[i].dm].n_act;
    whole += w * amax;
    split += w * area[i];
  }
  std::vector<int> areas(area);
  std::sort(areas.begin(), areas.end());
  areas.erase(std::unique(areas.begin(), areas.end()), areas.end());
  if (areas.size() < 2 || split > (1.0 - kSplitGain) * whole) return {};
  std::vector<std::vector<int>> out(areas.size());
  for (int i = 0; i < n_pairs; ++i)
    out[std::lower_bound(areas.begin(), areas.end(), area[i]) - areas.begin()].push_back(i);
  return out;
}

std::vector<synim_pair> pairs_of(const synim_pair* pairs, const std::vector<int>& idx) {
  std::vector<synim_pair> out;
  for (int i : idx) out.push_back(pairs[i]);
  return out;
}

int batch_workspace_whole(const synim_wfs* wfs, int n_wfs, const synim_dm* dms, int n_dm,
                          const synim_pair* pairs, int n_pairs, size_t* bytes) {
  synim_batch b;
  batch_fill(&b, wfs, n_wfs, dms, n_dm, pairs, n_pairs);
  int rc = batch_pick_shared(&b);
  if (rc != SYNIM_OK) return rc;
  size_t m = 0;
  for (int r = 0;; ++r) {
    const Variant* v = batch_variant(&b, r);
    if (!v) break;
    size_t need = 0;
    if (batch_layout(&b, *v, &need) == SYNIM_OK) m = std::max(m, need);
  }
  if (m == 0) return SYNIM_E_UNSUPPORTED;
  *bytes = m;
  return SYNIM_OK;
}

}  // namespace
}  // namespace synim

extern "C" int synim_batch_workspace(const synim_wfs* wfs, int n_wfs, const synim_dm* dms,
                                     int n_dm, const synim_pair* pairs, int n_pairs,
                                     size_t* bytes) {
  if (!bytes) return SYNIM_E_NULL;
  int rc = batch_check(wfs, n_wfs, dms, n_dm, pairs, n_pairs);
  if (rc != SYNIM_OK) return rc;
  const auto parts = batch_split(wfs, dms, pairs, n_pairs);
  if (parts.empty()) return batch_workspace_whole(wfs, n_wfs, dms, n_dm, pairs, n_pairs, bytes);
  size_t total = 0;
  for (const auto& idx : parts) {
    const std::vector<synim_pair> sub = pairs_of(pairs, idx);
    size_t m = 0;
    rc = batch_workspace_whole(wfs, n_wfs, dms, n_dm, sub.data(), (int)sub.size(), &m);
    if (rc != SYNIM_OK) return rc;
    total += align_up(m, 256);
  }
  *bytes = total;
  return SYNIM_OK;
}

extern "C" int synim_batch_create(const synim_wfs* wfs, int n_wfs, const synim_dm* dms, int n_dm,
                                  const synim_pair* pairs, int n_pairs, void* ws, size_t ws_bytes,
                                  void* stream, synim_batch** out) {
  if (!out || !ws) return SYNIM_E_NULL;
  *out = nullptr;
  int rc = batch_check(wfs, n_wfs, dms, n_dm, pairs, n_pairs);
  if (rc != SYNIM_OK) return rc;
  const auto parts = batch_split(wfs, dms, pairs, n_pairs);
  if (!parts.empty()) {
    // each part a whole batch on its own slice of the workspace
    synim_batch* b = new synim_batch;
    b->pairs.assign(pairs, pairs + n_pairs);
    b->part_idx = parts;
    size_t at = 0;
    for (const auto& idx : parts) {
      const std::vector<synim_pair> sub = pairs_of(pairs, idx);
      size_t m = 0;
      rc = batch_workspace_whole(wfs, n_wfs, dms, n_dm, sub.data(), (int)sub.size(), &m);
      synim_batch* part = nullptr;
      if (rc == SYNIM_OK && at + m > ws_bytes) rc = SYNIM_E_WORKSPACE;
      if (rc == SYNIM_OK)
        rc = synim_batch_create(wfs, n_wfs, dms, n_dm, sub.data(), (int)sub.size(),
                                static_cast<char*>(ws) + at, m, stream, &part);
      if (rc != SYNIM_OK) {
        synim_batch_destroy(b);
        return rc;
      }
      b->parts.push_back(part);
      at += align_up(m, 256);
    }
    *out = b;
    return SYNIM_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  synim_batch* b = new synim_batch;
  batch_fill(b, wfs, n_wfs, dms, n_dm, pairs, n_pairs);
  b->ws = static_cast<char*>(ws);
  b->ws_bytes = ws_bytes;
  rc = batch_pick_shared(b);
  const Variant* v = rc == SYNIM_OK ? batch_variant(b, 0) : nullptr;
  rc = rc != SYNIM_OK ? rc : v ? batch_bind(b, *v, st) : SYNIM_E_UNSUPPORTED;
  if (rc == SYNIM_OK && hipHostMalloc(reinterpret_cast<void**>(&b->staging),
                                      n_pairs * sizeof(MapD), hipHostMallocDefault) != hipSuccess)
    rc = SYNIM_E_HIP;
  if (rc == SYNIM_OK && hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess)
    rc = SYNIM_E_HIP;
  if (rc == SYNIM_OK) {
    std::vector<synim_affine> a(n_pairs);
    for (int i = 0; i < n_pairs; ++i) a[i] = pairs[i].A;
    rc = synim_batch_set_maps(b, a.data(), stream);
  }
  if (rc != SYNIM_OK) {
    synim_batch_destroy(b);
    return rc;
  }
  *out = b;
  return SYNIM_OK;
}

extern "C" int synim_batch_set_maps(synim_batch* b, const synim_affine* maps, void* stream) {
  if (!b || !maps) return SYNIM_E_NULL;
  if (!b->parts.empty()) {
    // every map is checked before any part takes its maps: a singular map, or
    // one whose patches outgrow its part's variant, leaves all parts as they
    // were
    for (size_t k = 0; k < b->parts.size(); ++k) {
      const synim_batch* part = b->parts[k];
      for (int i : b->part_idx[k]) {
        const double det =
            maps[i].A[0][0] * maps[i].A[1][1] - maps[i].A[0][1] * maps[i].A[1][0];
        if (!(std::fabs(det) > 1e-12)) return SYNIM_E_PARAM;
        int pw, ph;
        patch_need(maps[i], part->wfs[b->pairs[i].wfs].p, &pw, &ph);
        if (pw > part->var->PW || ph > part->var->PH()) return SYNIM_E_UNSUPPORTED;
      }
    }
    for (size_t k = 0; k < b->parts.size(); ++k) {
      std::vector<synim_affine> sub;
      for (int i : b->part_idx[k]) sub.push_back(maps[i]);
      const int rc = synim_batch_set_maps(b->parts[k], sub.data(), stream);
      if (rc != SYNIM_OK) return rc;
    }
    return SYNIM_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  const int np = (int)b->pairs.size();
  // the previous upload must have left the staging buffer before it is reused
  SYNIM_HIP_TRY(hipEventSynchronize(b->staged));
  for (int i = 0; i < np; ++i) {
    const double det = maps[i].A[0][0] * maps[i].A[1][1] - maps[i].A[0][1] * maps[i].A[1][0];
    if (!(std::fabs(det) > 1e-12)) return SYNIM_E_PARAM;
  }
  // The kernel variant (patch size) and each pair's tile shape were chosen for
  // the maps at creation.  A map whose patches no longer fit the variant needs
  // a new batch; one whose tiles outgrow their staged-box bound re-binds the
  // pair tables for the new maps (and drops a captured graph).
  bool rebind = false;
  if (b->var) {
    const Variant& v = *b->var;
    for (int i = 0; i < np; ++i) {
      const int p = b->wfs[b->pairs[i].wfs].p;
      int pw, ph;
      patch_need(maps[i], p, &pw, &ph);
      if (pw > v.PW || ph > v.PH()) return SYNIM_E_UNSUPPORTED;
      if (b->shared || (int)b->plans.size() != np) continue;
      const Dims& d = b->plans[i].d;
      int bw, bh;
      tile_bound(maps[i], p, v, d.TX, d.TY, ph, &bw, &bh);
      if (bh > d.BHmax || (long)bw * bh > v.cap_floats() || bh > MAX_TILE_ROWS) rebind = true;
    }
  }
  if (rebind) {
    for (int i = 0; i < np; ++i) b->pairs[i].A = maps[i];
    const int rc = batch_bind(b, *b->var, st);
    if (rc != SYNIM_OK) return rc;
    batch_drop_graph(b);
  } else if (b->shared && !shared_maps_fit(b, maps)) {
    // a subaperture moved past the margin of its shared tile: re-bin for the
    // new maps (a captured graph is captured again on the next run)
    for (int i = 0; i < np; ++i) b->pairs[i].A = maps[i];
    const int rc = batch_bind(b, *b->var, st);
    if (rc != SYNIM_OK) return rc;
    batch_drop_graph(b);
  }
  for (int i = 0; i < np; ++i) b->staging[i] = to_map(maps[i]);
  SYNIM_HIP_TRY(hipMemcpyAsync(b->ws + b->off_maps, b->staging, np * sizeof(MapD),
                               hipMemcpyHostToDevice, st));
  SYNIM_HIP_TRY(hipEventRecord(b->staged, st));
  return SYNIM_OK;
}

extern "C" int synim_batch_run(synim_batch* b, void* stream) {
  if (!b) return SYNIM_E_NULL;
  for (synim_batch* part : b->parts) {
    const int rc = synim_batch_run(part, stream);
    if (rc != SYNIM_OK) return rc;
  }
  if (!b->parts.empty()) return SYNIM_OK;
  return batch_enqueue(b, (hipStream_t)stream);
}

extern "C" int synim_batch_run_graph(synim_batch* b, void* stream) {
  if (!b) return SYNIM_E_NULL;
  if (!stream) return SYNIM_E_PARAM;   // capture needs an explicit stream
  for (synim_batch* part : b->parts) {   // one graph per part
    const int rc = synim_batch_run_graph(part, stream);
    if (rc != SYNIM_OK) return rc;
  }
  if (!b->parts.empty()) return SYNIM_OK;
  hipStream_t st = (hipStream_t)stream;
  if (!b->exec) {
    SYNIM_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = batch_enqueue(b, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != SYNIM_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc != SYNIM_OK ? rc : SYNIM_E_HIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      batch_drop_graph(b);
      return SYNIM_E_HIP;
    }
  }
  SYNIM_HIP_TRY(hipGraphLaunch(b->exec, st));
  return SYNIM_OK;
}

extern "C" int synim_batch_status(synim_batch* b, int* host_out, void* stream) {
  if (!b || !host_out) return SYNIM_E_NULL;
  if (!b->parts.empty()) {
    int v = 0;
    for (synim_batch* part : b->parts) {
      int x = 0;
      const int rc = synim_batch_status(part, &x, stream);
      if (rc != SYNIM_OK) return rc;
      v |= x;
    }
    *host_out = v;
    return SYNIM_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  std::vector<int> s(b->plans.size() + 1, 0);
  for (size_t i = 0; i < b->plans.size(); ++i)
    SYNIM_HIP_TRY(hipMemcpyAsync(&s[i], b->plans[i].status(), sizeof(int), hipMemcpyDeviceToHost,
                                 st));
  if (b->shared)
    SYNIM_HIP_TRY(hipMemcpyAsync(&s.back(), b->ws + b->off_jstatus, sizeof(int),
                                 hipMemcpyDeviceToHost, st));
  SYNIM_HIP_TRY(hipStreamSynchronize(st));
  int v = 0;
  for (int x : s) v |= x;
  *host_out = v;
  return SYNIM_OK;
}

extern "C" int synim_batch_oob(synim_batch* b, int64_t* host_count, void* stream) {
  if (!b || !host_count) return SYNIM_E_NULL;
  if (!b->parts.empty()) {
    int64_t t = 0;
    for (synim_batch* part : b->parts) {
      int64_t x = 0;
      const int rc = synim_batch_oob(part, &x, stream);
      if (rc != SYNIM_OK && rc != SYNIM_E_OOB) return rc;
      t += x;
    }
    *host_count = t;
    return t > 0 ? SYNIM_E_OOB : SYNIM_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  std::vector<int> n(b->plans.size(), 0);
  for (size_t i = 0; i < b->plans.size(); ++i)
    SYNIM_HIP_TRY(hipMemcpyAsync(&n[i], b->plans[i].status() + 2, sizeof(int),
                                 hipMemcpyDeviceToHost, st));
  SYNIM_HIP_TRY(hipStreamSynchronize(st));
  int64_t t = 0;
  for (int x : n) t += x;
  *host_count = t;
  return t > 0 ? SYNIM_E_OOB : SYNIM_OK;
}

extern "C" int synim_batch_autotune(synim_batch* b, int max_variants, float* times_ms,
                                    int* n_tried, void* stream) {
  if (!b) return SYNIM_E_NULL;
  if (max_variants < 1) return SYNIM_E_PARAM;
  if (!b->parts.empty()) {
    // each part keeps its own fastest variant; times_ms[r] = the parts' r-th
    // variants summed (a part with fewer variants adds its last time)
    std::vector<float> sum(max_variants, 0.f);
    int n_max = 0;
    for (synim_batch* part : b->parts) {
      std::vector<float> t(max_variants, 0.f);
      int n = 0;
      const int rc = synim_batch_autotune(part, max_variants, t.data(), &n, stream);
      if (rc != SYNIM_OK) return rc;
      for (int r = 0; r < max_variants; ++r) sum[r] += n > 0 ? t[std::min(r, n - 1)] : 0.f;
      n_max = std::max(n_max, n);
    }
    if (times_ms)
      for (int r = 0; r < n_max; ++r) times_ms[r] = sum[r];
    if (n_tried) *n_tried = n_max;
    return SYNIM_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  batch_drop_graph(b);
  hipEvent_t e0, e1;
  SYNIM_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SYNIM_E_HIP;
  }
  int best = -1, tried = 0, rc = SYNIM_OK;
  float best_ms = 1e30f;
  for (int r = 0; r < max_variants && rc == SYNIM_OK; ++r) {
    const Variant* v = batch_variant(b, r);
    if (!v) break;
    if (batch_bind(b, *v, st) != SYNIM_OK) continue;   // does not fit this workspace
    rc = batch_enqueue(b, st);
    if (rc != SYNIM_OK) break;
    const int reps = 3;
    if (hipEventRecord(e0, st) != hipSuccess) { rc = SYNIM_E_HIP; break; }
    for (int k = 0; k < reps && rc == SYNIM_OK; ++k) rc = batch_enqueue(b, st);
    float ms = 0.f;
    if (rc == SYNIM_OK && (hipEventRecord(e1, st) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = SYNIM_E_HIP;
    if (rc != SYNIM_OK) break;
    ms /= reps;
    if (times_ms) times_ms[tried] = ms;
    ++tried;
    if (ms < best_ms) {
      best_ms = ms;
      best = r;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SYNIM_OK) return rc;
  if (n_tried) *n_tried = tried;
  if (best < 0) return SYNIM_E_UNSUPPORTED;
  return batch_bind(b, *batch_variant(b, best), st);
}

extern "C" int synim_batch_config(const synim_batch* b, int* out6) {
  if (b && !b->parts.empty()) return synim_batch_config(b->parts[0], out6);
  if (!b || !out6 || !b->var) return SYNIM_E_NULL;
  out6[0] = b->var->BLOCK;
  out6[1] = b->var->LPS;
  out6[2] = b->var->NST;
  out6[3] = b->G;
  out6[4] = b->var->NJ4;
  out6[5] = b->var->PACK;
  return SYNIM_OK;
}

extern "C" int synim_batch_parts(const synim_batch* b, int* n_parts) {
  if (!b || !n_parts) return SYNIM_E_NULL;
  *n_parts = b->parts.empty() ? 1 : (int)b->parts.size();
  return SYNIM_OK;
}

extern "C" void synim_batch_destroy(synim_batch* b) {
  if (!b) return;
  for (synim_batch* part : b->parts) synim_batch_destroy(part);
  batch_drop_graph(b);
  if (b->staged) {
    (void)hipEventSynchronize(b->staged);
    (void)hipEventDestroy(b->staged);
  }
  if (b->staging) (void)hipHostFree(b->staging);
  delete b;
}

#include "misreg.inc"
