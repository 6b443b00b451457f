// 16x16x4 matrix-core products in FP64 and FP32 (gfx950 MFMA builtins).
//
// D (16 x 16) += A (16 x 4) B (4 x 16) over a wavefront: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds four values of D in
// column l % 16, rows row(l, v), v = 0..3.  The lane layouts were read off a
// GPU probe of the builtins checked against a CPU product.
#pragma once

#include <hip/hip_runtime.h>

namespace ikr {

typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
template <> struct Mfma<double> {
  typedef mf64x4 acc;
  __device__ __forceinline__ static acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of result value v held by lane l (the column is l % 16)
  __device__ __forceinline__ static int row(int l, int v) { return 4 * v + (l >> 4); }
};
template <> struct Mfma<float> {
  typedef mf32x4 acc;
  __device__ __forceinline__ static acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

}  // namespace ikr
