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
//   plan_tiles    groups subapertures into tiles and computes each tile's IF
//                 bounding box.
// Stream (FP32, the hot loop): each workgroup owns one tile and a chunk of
// actuators; its weights sit in registers, and every actuator's bounding box
// is read from HBM once (coalesced float4 rows, double-buffered through LDS)
// and contracted against the patches; partial sums of the LPS lanes that share
// a subaperture are combined with DPP.
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.hpp"

namespace synim {
namespace {

constexpr int BLOCK = 256;
constexpr int GMAX_VJP = 16384;   // max workgroups of a VJP launch (partials buffer)

struct Map4 {
  MapD m[4];
};

// ------------------------------------------------------------------ planning

__global__ void plan_subaps_kernel(MapD m, const int32_t* __restrict__ valid,
                                   const uint8_t* __restrict__ pupil, int n_sub_x, int p, int nv,
                                   int PH, int PW, int2* __restrict__ origin,
                                   double* __restrict__ inv2nk, int* __restrict__ status) {
  const int kk = blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= nv) return;
  const int k = valid[kk];
  const int u = k % n_sub_x, v = k / n_sub_x;
  const int W = n_sub_x * p;
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int y = v * p - 1; y <= v * p + p; ++y)
    for (int x = u * p - 1; x <= u * p + p; ++x) {
      double xs, ys;
      src_xy(m, x, y, xs, ys);
      xmin = fmin(xmin, xs);
      xmax = fmax(xmax, xs);
      ymin = fmin(ymin, ys);
      ymax = fmax(ymax, ys);
    }
  int nk = 0;
  for (int y = v * p; y < v * p + p; ++y)
    for (int x = u * p; x < u * p + p; ++x) nk += pupil[(size_t)y * W + x] ? 1 : 0;
  int ox = 0, oy = 0;
  if (fabs(xmin) < 1e9 && fabs(xmax) < 1e9 && fabs(ymin) < 1e9 && fabs(ymax) < 1e9) {
    ox = (int)floor(xmin);
    oy = (int)floor(ymin);
    // the last tap column is floor(xmax) + 1
    if ((int)floor(xmax) + 2 - ox > PW || (int)floor(ymax) + 2 - oy > PH) atomicOr(status, 1);
  } else {
    atomicOr(status, 1);
  }
  if (nk == 0) atomicOr(status, 4);
  origin[kk] = make_int2(ox, oy);
  inv2nk[kk] = nk > 0 ? 1.0 / (2.0 * nk) : 0.0;
}

__device__ __forceinline__ int in_sub(const uint8_t* __restrict__ pupil, int W, int x0, int y0,
                                      int p, int x, int y) {
  return (x >= x0 && x < x0 + p && y >= y0 && y < y0 + p && pupil[(size_t)y * W + x]) ? 1 : 0;
}

// One thread per (valid subaperture, patch entry).  Gathers, in a fixed
// order, every haloed-window sample q whose bilinear cell has this entry as a
// tap.  Weights layout: [plane][kk][component x|y][PH*PW].
__global__ void plan_weights_kernel(MapD m, MapD inv, double rx, double ry, Map4 dm, int n_planes,
                                    const int32_t* __restrict__ valid,
                                    const uint8_t* __restrict__ pupil, int n_sub_x, int p, int nv,
                                    int PH, int PW, const int2* __restrict__ origin,
                                    const double* __restrict__ inv2nk, float* __restrict__ weights,
                                    int* __restrict__ status) {
  const int E = PH * PW;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)nv * E) return;
  const int kk = (int)(gid / E);
  const int e = (int)(gid - (long)kk * E);
  const int r = e / PW, c = e - (e / PW) * PW;
  const int k = valid[kk];
  const int u = k % n_sub_x, v = k / n_sub_x;
  const int W = n_sub_x * p;
  const int2 o = origin[kk];
  const int X = o.x + c, Y = o.y + r;

  // candidate window: p_o = A^-1 (p_s - b) with p_s in [X-1, X+1) x [Y-1, Y+1)
  const double dx = (double)X - m.b0, dy = (double)Y - m.b1;
  const double qx = inv.a00 * dx + inv.a01 * dy;
  const double qy = inv.a10 * dx + inv.a11 * dy;
  const int xl = max(u * p - 1, (int)ceil(qx - rx)), xh = min(u * p + p, (int)floor(qx + rx));
  const int yl = max(v * p - 1, (int)ceil(qy - ry)), yh = min(v * p + p, (int)floor(qy + ry));
  const int sx0 = u * p, sy0 = v * p;

  double acc[5][2];
#pragma unroll
  for (int j = 0; j < 5; ++j) acc[j][0] = acc[j][1] = 0.0;
  for (int y = yl; y <= yh; ++y)
    for (int x = xl; x <= xh; ++x) {
      const int cx = in_sub(pupil, W, sx0, sy0, p, x - 1, y) - in_sub(pupil, W, sx0, sy0, p, x + 1, y);
      const int cy = in_sub(pupil, W, sx0, sy0, p, x, y - 1) - in_sub(pupil, W, sx0, sy0, p, x, y + 1);
      if (cx == 0 && cy == 0) continue;
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
  const double s = inv2nk[kk];
  for (int j = 0; j < n_planes; ++j) {
    float* w = weights + ((size_t)j * nv + kk) * 2 * E;
    w[e] = (float)(acc[j][0] * s);
    w[E + e] = (float)(acc[j][1] * s);
  }
  (void)status;
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

__global__ void plan_tiles_kernel(const int32_t* __restrict__ valid, int nv, int n_sub_x,
                                  int n_sub_y, int TX, int TY, int n_tiles_x, int n_tiles,
                                  const int2* __restrict__ origin, int PH, int PW, int BWmax,
                                  int BHmax, int* __restrict__ slot_kk, int4* __restrict__ bbox,
                                  int* __restrict__ status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int tu = t % n_tiles_x, tv = t / n_tiles_x;
  const int NS = TX * TY;
  int xmin = INT_MAX, ymin = INT_MAX, xmax = INT_MIN, ymax = INT_MIN;
  for (int s = 0; s < NS; ++s) {
    const int u = tu * TX + s % TX, v = tv * TY + s / TX;
    int kk = -1;
    if (u < n_sub_x && v < n_sub_y) kk = find_valid(valid, nv, v * n_sub_x + u);
    slot_kk[(size_t)t * NS + s] = kk;
    if (kk >= 0) {
      const int2 o = origin[kk];
      xmin = min(xmin, o.x);
      ymin = min(ymin, o.y);
      xmax = max(xmax, o.x);
      ymax = max(ymax, o.y);
    }
  }
  int4 bb = make_int4(0, 0, 0, 0);
  if (xmin != INT_MAX) {
    const int x0 = floor_div(xmin, 4) * 4;
    const int bw = ((xmax + PW - x0) + 3) / 4 * 4;
    const int bh = ymax + PH - ymin;
    if (bw > BWmax || bh > BHmax) {
      atomicOr(status, 2);   // tile skipped: its slopes stay unwritten
    } else {
      bb = make_int4(x0, ymin, bw, bh);
    }
  }
  bbox[t] = bb;
}

// ------------------------------------------------------------------ streaming

__device__ __forceinline__ float dpp_sum(float v, int lps) {
  // quad_perm [1,0,3,2] then [2,3,0,1]; for 8 lanes also row_half_mirror
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  if (lps == 8)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
  return v;
}

struct StreamArgs {
  const float* ifs;
  int n_act, H_in, W_in;
  const int2* origin;
  const float* weights;      // plane 0 base
  const int* slot_kk;
  const int4* bbox;
  int nv, n_tiles, chunk, n_chunks;
  int ns;                    // subapertures per tile (TX*TY <= BLOCK/LPS)
  int S;                     // LDS row stride (floats, multiple of 4)
  int BHmax;
  int vec_ok;                // IF rows are 16-byte aligned float4 rows
  int plane0;                // first weight plane handled (blockIdx.z adds to it)
  int out_plane0;            // weight plane that lands in out[0]
  float* out;                // [plane - out_plane0][n_act][2nv]
  const float* grad;         // VJP: [n_act][2nv]
  double* partials;          // VJP: [4][gridDim.x]
};

template <int LPS, int RPL, int PW, int NPF, bool VJP>
__global__ __launch_bounds__(BLOCK) void im_stream_kernel(StreamArgs g) {
  constexpr int PH = LPS * RPL;
  constexpr int E = PH * PW;
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);

  // XCD-aware mapping: consecutive workgroups go round-robin over the 8 XCDs,
  // so give each XCD a contiguous range of (chunk, tile) work; the tiles of one
  // actuator chunk then run side by side and share their halo rows in L2.
  const int G = gridDim.x;
  const int per = G / 8;
  const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int total = g.n_tiles * g.n_chunks;
  if (logical >= total) {
    if (VJP && threadIdx.x == 0)
      g.partials[(size_t)(g.plane0 + blockIdx.z - 1) * G + blockIdx.x] = 0.0;
    return;
  }
  const int chunk_id = logical / g.n_tiles;
  const int tile = logical - chunk_id * g.n_tiles;
  const int plane = g.plane0 + blockIdx.z;
  const int4 bb = g.bbox[tile];

  const int tid = threadIdx.x;
  const int slot = tid / LPS, q = tid % LPS;
  const int kk = (bb.z > 0 && slot < g.ns) ? g.slot_kk[(size_t)tile * g.ns + slot] : -1;

  double vacc = 0.0;
  if (bb.z > 0) {
    const int x0 = bb.x, y0 = bb.y, bw = bb.z, bh = bb.w;
    const int S = g.S;
    const int buf_stride = g.BHmax * S;

    float wx[RPL][PW], wy[RPL][PW];
    int lbase = 0;
    if (kk >= 0) {
      const int2 o = g.origin[kk];
      lbase = (o.y - y0 + q) * S + (o.x - x0);
      const float* W = g.weights + ((size_t)plane * g.nv + kk) * 2 * E;
#pragma unroll
      for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int c = 0; c < PW; ++c) {
          wx[i][c] = W[(q + LPS * i) * PW + c];
          wy[i][c] = W[E + (q + LPS * i) * PW + c];
        }
    } else {
#pragma unroll
      for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int c = 0; c < PW; ++c) wx[i][c] = wy[i][c] = 0.f;
    }

    // this thread's share of the bounding box: vectors tid + BLOCK*j
    const int vpr = bw >> 2;   // float4 per bbox row
    const int nvec = bh * vpr;
    int goff[NPF], loff[NPF], kind[NPF];
#pragma unroll
    for (int j = 0; j < NPF; ++j) {
      const int vi = tid + BLOCK * j;
      const int r = vi / vpr, cv = vi - (vi / vpr) * vpr;
      const int gy = y0 + r, gx = x0 + 4 * cv;
      loff[j] = r * S + 4 * cv;
      goff[j] = 0;
      if (vi >= nvec) {
        kind[j] = 0;
      } else if (g.vec_ok && gy >= 0 && gy < g.H_in && gx >= 0 && gx + 3 < g.W_in) {
        kind[j] = 1;
        goff[j] = gy * g.W_in + gx;
      } else {
        kind[j] = 2;   // partly or fully outside the IF grid, or unaligned rows
        goff[j] = gy * g.W_in + gx;
      }
    }
    const size_t plane_in = (size_t)g.H_in * g.W_in;
    const int a0 = chunk_id * g.chunk;
    const int a1 = min(g.n_act, a0 + g.chunk);

    float4 pf[NPF];
    auto fetch = [&](int a) {
      const float* F = g.ifs + (size_t)a * plane_in;
#pragma unroll
      for (int j = 0; j < NPF; ++j) {
        if (kind[j] == 1) {
          pf[j] = *reinterpret_cast<const float4*>(F + goff[j]);
        } else if (kind[j] == 2) {
          const int vi = tid + BLOCK * j;
          const int r = vi / vpr, cv = vi - (vi / vpr) * vpr;
          const int gy = y0 + r, gx = x0 + 4 * cv;
          float t[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int xx = gx + e;
            t[e] = (gy >= 0 && gy < g.H_in && xx >= 0 && xx < g.W_in)
                       ? F[(size_t)gy * g.W_in + xx]
                       : 0.f;
          }
          pf[j] = make_float4(t[0], t[1], t[2], t[3]);
        }
      }
    };

    if (a0 < a1) fetch(a0);
    for (int a = a0; a < a1; ++a) {
      float* buf = lds + ((a - a0) & 1) * buf_stride;
#pragma unroll
      for (int j = 0; j < NPF; ++j)
        if (kind[j]) *reinterpret_cast<float4*>(buf + loff[j]) = pf[j];
      __syncthreads();
      if (a + 1 < a1) fetch(a + 1);

      float sx = 0.f, sy = 0.f;
      const float* rowp = buf + lbase;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
#pragma unroll
        for (int c = 0; c < PW; ++c) {
          const float f = rowp[i * LPS * S + c];
          sx = __fmaf_rn(wx[i][c], f, sx);
          sy = __fmaf_rn(wy[i][c], f, sy);
        }
      }
      sx = dpp_sum(sx, LPS);
      sy = dpp_sum(sy, LPS);
      if (kk >= 0) {
        const size_t row = (size_t)a * 2 * g.nv;
        if (VJP) {
          if (q == 0) vacc += (double)g.grad[row + kk] * sx + (double)g.grad[row + g.nv + kk] * sy;
        } else {
          float* o = g.out + (size_t)(plane - g.out_plane0) * g.n_act * 2 * g.nv + row;
          if (q == 0) o[kk] = sx;
          if (q == 1) o[g.nv + kk] = sy;
        }
      }
    }
  }
  if (VJP) {
    // fixed-order block reduction of the per-lane accumulators
    __shared__ double red[BLOCK];
    __syncthreads();
    red[tid] = vacc;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) g.partials[(size_t)(plane - 1) * G + blockIdx.x] = red[0];
  }
}

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

using StreamFn = void (*)(StreamArgs);

struct Variant {
  int LPS, RPL, PW, NPF;
  StreamFn im, vjp;
};

#define SYNIM_VARIANT(L, R, W, N) \
  {L, R, W, N, im_stream_kernel<L, R, W, N, false>, im_stream_kernel<L, R, W, N, true>}

// ordered by cost: the first variant whose patch fits is used
const Variant kVariants[] = {
    SYNIM_VARIANT(4, 2, 8, 4),  SYNIM_VARIANT(4, 3, 10, 4), SYNIM_VARIANT(4, 3, 12, 4),
    SYNIM_VARIANT(8, 2, 12, 6), SYNIM_VARIANT(8, 2, 14, 6), SYNIM_VARIANT(8, 2, 16, 6),
    SYNIM_VARIANT(8, 3, 20, 8), SYNIM_VARIANT(8, 3, 24, 8),
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

struct Dims {
  const Variant* var;
  int PH, PW;
  int TX, TY, NSLOT, n_tiles_x, n_tiles;
  int BWmax, BHmax, S;
};

struct WsLayout {
  size_t status, origin, inv2nk, weights, slot_kk, bbox, partials, total;
};

int choose_dims(const synim_wfs& w, const synim_affine& A, Dims* d) {
  const double ax = std::fabs(A.A[0][0]) + std::fabs(A.A[0][1]);
  const double ay = std::fabs(A.A[1][0]) + std::fabs(A.A[1][1]);
  const int p = w.p;
  const int pw_need = (int)std::floor(ax * (p + 1) + 1e-7) + 3;
  const int ph_need = (int)std::floor(ay * (p + 1) + 1e-7) + 3;
  const Variant* var = nullptr;
  for (int i = 0; i < kNumVariants; ++i)
    if (kVariants[i].PW >= pw_need && kVariants[i].LPS * kVariants[i].RPL >= ph_need) {
      var = &kVariants[i];
      break;
    }
  if (!var) return SYNIM_E_UNSUPPORTED;
  const int nslot_max = BLOCK / var->LPS;
  const int PH = var->LPS * var->RPL, PW = var->PW;
  // tile shape: the TX x TY factorisation with the least staged IF area per
  // covered subaperture whose bounding box fits the prefetch registers; full
  // tiles (every lane busy) first, then half and quarter tiles for strongly
  // rotated or magnified maps
  int bt = -1, bns = 0, bBW = 0, bBH = 0;
  for (int ns = nslot_max; ns >= nslot_max / 4 && bt < 0; ns /= 2) {
    double best = 1e300;
    for (int tx = 1; tx <= ns; tx *= 2) {
      const int ty = ns / tx;
      const double wt = std::fabs(A.A[0][0]) * (tx * p + 1) + std::fabs(A.A[0][1]) * (ty * p + 1);
      const double ht = std::fabs(A.A[1][0]) * (tx * p + 1) + std::fabs(A.A[1][1]) * (ty * p + 1);
      const int BW = ((int)std::floor(wt + 1e-6) + PW + 4 + 3) / 4 * 4;
      const int BH = (int)std::floor(ht + 1e-6) + 1 + PH;
      if ((long)BH * (BW / 4) > (long)BLOCK * var->NPF) continue;
      const int ux = std::min(tx, w.n_sub_x), uy = std::min(ty, w.n_sub_y);
      const double cost = (double)BW * BH / ((double)ux * uy);
      if (cost < best) {
        best = cost;
        bt = tx;
        bns = ns;
        bBW = BW;
        bBH = BH;
      }
    }
  }
  if (bt < 0) return SYNIM_E_UNSUPPORTED;
  d->var = var;
  d->PH = PH;
  d->PW = PW;
  d->TX = bt;
  d->TY = bns / bt;
  d->NSLOT = bns;
  d->n_tiles_x = (w.n_sub_x + d->TX - 1) / d->TX;
  d->n_tiles = d->n_tiles_x * ((w.n_sub_y + d->TY - 1) / d->TY);
  d->BWmax = bBW;
  d->BHmax = bBH;
  d->S = bBW;
  return SYNIM_OK;
}

WsLayout layout(const synim_wfs& w, const Dims& d, int planes) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  const size_t nv = (size_t)w.n_valid;
  L.status = take(16 * sizeof(int));
  L.origin = take(nv * sizeof(int2));
  L.inv2nk = take(nv * sizeof(double));
  L.weights = take((size_t)planes * nv * 2 * d.PH * d.PW * sizeof(float));
  L.slot_kk = take((size_t)d.n_tiles * d.NSLOT * sizeof(int));
  L.bbox = take((size_t)d.n_tiles * sizeof(int4));
  L.partials = take(planes > 1 ? (size_t)4 * GMAX_VJP * sizeof(double) : 0);
  L.total = off;
  return L;
}

struct Plan {
  Dims d;
  WsLayout L;
  char* ws;
  int* status() const { return reinterpret_cast<int*>(ws + L.status); }
  int2* origin() const { return reinterpret_cast<int2*>(ws + L.origin); }
  double* inv2nk() const { return reinterpret_cast<double*>(ws + L.inv2nk); }
  float* weights() const { return reinterpret_cast<float*>(ws + L.weights); }
  int* slot_kk() const { return reinterpret_cast<int*>(ws + L.slot_kk); }
  int4* bbox() const { return reinterpret_cast<int4*>(ws + L.bbox); }
  double* partials() const { return reinterpret_cast<double*>(ws + L.partials); }
};

int build_plan(const synim_wfs& w, const synim_affine& A, const synim_affine* dA, int planes,
               void* ws, size_t ws_bytes, hipStream_t st, Plan* P) {
  int rc = choose_dims(w, A, &P->d);
  if (rc != SYNIM_OK) return rc;
  P->L = layout(w, P->d, planes);
  if (!ws) return SYNIM_E_WORKSPACE;
  if (ws_bytes < P->L.total) return SYNIM_E_WORKSPACE;
  P->ws = static_cast<char*>(ws);
  const Dims& d = P->d;
  const MapD m = to_map(A);
  const double det = m.a00 * m.a11 - m.a01 * m.a10;
  if (!(std::fabs(det) > 1e-12)) return SYNIM_E_PARAM;
  MapD inv{m.a11 / det, -m.a01 / det, -m.a10 / det, m.a00 / det, 0, 0};
  const double rx = std::fabs(inv.a00) + std::fabs(inv.a01) + 0.01;
  const double ry = std::fabs(inv.a10) + std::fabs(inv.a11) + 0.01;
  Map4 dm{};
  if (planes > 1)
    for (int j = 0; j < 4; ++j) dm.m[j] = to_map(dA[j]);

  SYNIM_HIP_TRY(hipMemsetAsync(P->status(), 0, 16 * sizeof(int), st));
  const int nv = w.n_valid;
  hipLaunchKernelGGL(plan_subaps_kernel, dim3((nv + 127) / 128), dim3(128), 0, st, m, w.valid_idx,
                     w.pupil, w.n_sub_x, w.p, nv, d.PH, d.PW, P->origin(), P->inv2nk(),
                     P->status());
  SYNIM_HIP_TRY(hipGetLastError());
  const long nthr = (long)nv * d.PH * d.PW;
  hipLaunchKernelGGL(plan_weights_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st,
                     m, inv, rx, ry, dm, planes, w.valid_idx, w.pupil, w.n_sub_x, w.p, nv, d.PH,
                     d.PW, P->origin(), P->inv2nk(), P->weights(), P->status());
  SYNIM_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(plan_tiles_kernel, dim3((d.n_tiles + 127) / 128), dim3(128), 0, st,
                     w.valid_idx, nv, w.n_sub_x, w.n_sub_y, d.TX, d.TY, d.n_tiles_x, d.n_tiles,
                     P->origin(), d.PH, d.PW, d.BWmax, d.BHmax, P->slot_kk(), P->bbox(),
                     P->status());
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

int default_chunk(int n_act, int n_tiles) {
  // aim for >= ~8 workgroups per CU (256 CUs) while keeping the per-workgroup
  // weight load amortised over as many actuators as possible
  const long target = 2048;
  long chunks = (target + n_tiles - 1) / n_tiles;
  int chunk = (int)std::max(1L, ((long)n_act + chunks - 1) / chunks);
  return std::min(chunk, 64);
}

int launch_stream(const Plan& P, const float* ifs, int n_act, int H_in, int W_in, int nv,
                  int plane0, int nplanes, float* out, const float* grad, int chunk,
                  hipStream_t st, int* grid_out = nullptr) {
  const Dims& d = P.d;
  StreamArgs g{};
  g.ifs = ifs;
  g.n_act = n_act;
  g.H_in = H_in;
  g.W_in = W_in;
  g.origin = P.origin();
  g.weights = P.weights();
  g.slot_kk = P.slot_kk();
  g.bbox = P.bbox();
  g.nv = nv;
  g.n_tiles = d.n_tiles;
  g.chunk = chunk;
  g.n_chunks = (n_act + chunk - 1) / chunk;
  g.ns = d.NSLOT;
  g.S = d.S;
  g.BHmax = d.BHmax;
  g.vec_ok = (W_in % 4 == 0) && ((reinterpret_cast<uintptr_t>(ifs) & 15) == 0);
  g.plane0 = plane0;
  g.out_plane0 = plane0;
  g.out = out;
  g.grad = grad;
  g.partials = P.partials();
  long total = (long)d.n_tiles * g.n_chunks;
  long G = (total + 7) / 8 * 8;
  if (G > INT_MAX) return SYNIM_E_SHAPE;
  if (grad && G > GMAX_VJP) return SYNIM_E_SHAPE;
  const size_t lds = (size_t)2 * d.BHmax * d.S * sizeof(float);
  if (lds > 160 * 1024) return SYNIM_E_UNSUPPORTED;
  StreamFn fn = grad ? d.var->vjp : d.var->im;
  if (lds > 64 * 1024)
    SYNIM_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(fn, dim3((unsigned)G, 1, nplanes), dim3(BLOCK), lds, st, g);
  SYNIM_HIP_TRY(hipGetLastError());
  if (grid_out) *grid_out = (int)G;
  return SYNIM_OK;
}

int check_common(const float* ifs, int n_act, int H_in, int W_in, const synim_affine* A,
                 const synim_wfs* wfs) {
  if (!ifs || !A) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  if (n_act < 1 || H_in < 1 || W_in < 1) return SYNIM_E_SHAPE;
  if ((long)H_in * W_in > (long)INT_MAX / 2) return SYNIM_E_SHAPE;
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
  Dims d{};
  rc = choose_dims(*wfs, *A, &d);
  if (rc != SYNIM_OK) return rc;
  *bytes = layout(*wfs, d, planes).total;
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
  rc = build_plan(*wfs, *A, nullptr, 1, ws, ws_bytes, st, &P);
  if (rc != SYNIM_OK) return rc;
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr,
                       default_chunk(n_act, P.d.n_tiles), st);
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
  rc = build_plan(*wfs, *A, dA, 5, ws, ws_bytes, st, &P);
  if (rc != SYNIM_OK) return rc;
  const int chunk = default_chunk(n_act, P.d.n_tiles);
  if (im) {
    rc = launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 0, 1, im, nullptr, chunk, st);
    if (rc != SYNIM_OK) return rc;
  }
  return launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 1, 4, dim, nullptr, chunk, st);
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
  rc = build_plan(*wfs, *A, dA, 5, ws, ws_bytes, st, &P);
  if (rc != SYNIM_OK) return rc;
  // keep the grid within the partials buffer: grow the chunk if needed
  int chunk = default_chunk(n_act, P.d.n_tiles);
  while ((long)P.d.n_tiles * ((n_act + chunk - 1) / chunk) > GMAX_VJP - 8) chunk *= 2;
  int G = 0;
  rc = launch_stream(P, ifs, n_act, H_in, W_in, wfs->n_valid, 1, 4, nullptr, grad_im, chunk, st,
                     &G);
  if (rc != SYNIM_OK) return rc;
  hipLaunchKernelGGL(vjp_finalize_kernel, dim3(4), dim3(256), 0, st, P.partials(), G,
                     grad_theta);
  SYNIM_HIP_TRY(hipGetLastError());
  return SYNIM_OK;
}

extern "C" int synim_im_plan(const synim_wfs* wfs, const synim_affine* A,
                             const synim_affine* dA, int planes, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!A) return SYNIM_E_NULL;
  int rc = validate_wfs(wfs);
  if (rc != SYNIM_OK) return rc;
  if (planes != 1 && planes != 5) return SYNIM_E_PARAM;
  if (planes == 5 && !dA) return SYNIM_E_NULL;
  Plan P{};
  return build_plan(*wfs, *A, dA, planes, ws, ws_bytes, (hipStream_t)stream, &P);
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
                       default_chunk(n_act, P.d.n_tiles), (hipStream_t)stream);
}

extern "C" int synim_plan_status(const void* ws, int* host_out, void* stream) {
  if (!ws || !host_out) return SYNIM_E_NULL;
  SYNIM_HIP_TRY(hipMemcpyAsync(host_out, ws, sizeof(int), hipMemcpyDeviceToHost,
                               (hipStream_t)stream));
  SYNIM_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return SYNIM_OK;
}
