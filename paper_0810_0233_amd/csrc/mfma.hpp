// mfma.hpp -- the 16x16x4 matrix-core instructions used by the M2L and batched
// near-field kernels, and their register layouts on gfx950.
//
// Operands: lane l supplies A[row l%16][k l/16] and B[k l/16][column l%16].
// Result: lane l holds column l%16; its item r is row 4 (l/16) + r for FP32
// and row l/16 + 4 r for FP64 (checked on the device by ccfmm_selftest_mfma).
#pragma once
#include <hip/hip_runtime.h>

namespace ccfmm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
struct Acc;
template <>
struct Acc<float> {
  using type = f32x4;
};
template <>
struct Acc<double> {
  using type = f64x4;
};

template <typename T>
__device__ __forceinline__ int acc_row(int kq, int r);
template <>
__device__ __forceinline__ int acc_row<float>(int kq, int r) {
  return 4 * kq + r;
}
template <>
__device__ __forceinline__ int acc_row<double>(int kq, int r) {
  return kq + 4 * r;
}

}  // namespace ccfmm
