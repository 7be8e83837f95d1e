// Complex-product building blocks on the CDNA matrix cores: the real
// 16x16x4 MFMA in FP64 and FP32, and the lane layout of its 16x16 result.
// Operand layout (both types): A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k of a wave64.
#pragma once

#include <hip/hip_runtime.h>

namespace tdvp {

typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mf;
template <> struct Mf<double> {
  using acc = f64x4_t;
  using c2 = double2;
  static __device__ __forceinline__ acc mfma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of a 16x16 result block held by (lane, register r); column = lane % 16
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mf<float> {
  using acc = f32x4_t;
  using c2 = float2;
  static __device__ __forceinline__ acc mfma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// 1/sqrt(x) and 1/x for x > 0 in FP64 without the long division and square
// root sequences: the hardware estimate refined by two Newton steps (each
// squares the relative error), so the result is within a few ulp.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);      // 1 - x y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x, y, 1.0);          // 1 - x y
    y = fma(y, e, y);
  }
  return y;
}

}  // namespace tdvp
