// Internal helpers shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/synim.h"

namespace synim {

// FP64 inverse map p_s = A p_o + b, passed to kernels by value.
struct MapD {
  double a00, a01, a10, a11, b0, b1;
};

inline MapD to_map(const synim_affine& A) {
  return MapD{A.A[0][0], A.A[0][1], A.A[1][0], A.A[1][1], A.b[0], A.b[1]};
}

// Source coordinates of output pixel (x, y).  Every kernel that needs the
// coordinate of a pixel calls this one function, written with explicit fused
// multiply-adds, so all threads and kernels agree bit for bit on every floor
// decision.
__device__ __forceinline__ void src_xy(const MapD& m, int x, int y, double& xs, double& ys) {
  xs = __fma_rn(m.a01, (double)y, __fma_rn(m.a00, (double)x, m.b0));
  ys = __fma_rn(m.a11, (double)y, __fma_rn(m.a10, (double)x, m.b1));
}

#define SYNIM_HIP_TRY(expr)                              \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return SYNIM_E_HIP;            \
  } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Floor division for possibly negative integers.
__host__ __device__ inline int floor_div(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

int validate_wfs(const synim_wfs* wfs);

}  // namespace synim
