// MFMA fragment helpers of the contraction kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace sbp {

// MFMA 16x16x4 wrappers.  Lane l holds A[l%16][k0 + l/16], B[k0 + l/16][l%16];
// accumulator register i of lane l holds D[row(l/16, i)][l%16] with
// row = l/16 + 4 i for v_mfma_f64_16x16x4f64 and 4 (l/16) + i for
// v_mfma_f32_16x16x4f32 (checked on gfx950).
template <typename T>
struct MF;
template <>
struct MF<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int kr, int i) { return kr + 4 * i; }
};
template <>
struct MF<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int kr, int i) { return 4 * kr + i; }
};

}  // namespace sbp
