// Matrix-core (MFMA) helpers for gfx950: one 16x16 output block per wave,
// K = 4 per instruction, in FP64 or FP32.
//
// Operand layout (both precisions): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]. Accumulator element j of lane l is
//   FP32: C[4 * (l / 16) + j][l % 16]
//   FP64: C[l / 16 + 4 * j][l % 16]
// (checked on the device against a host product).
#pragma once

#include <hip/hip_runtime.h>

namespace tls {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;

template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of accumulator element j held by lane l (column is l % 16)
  __device__ static inline int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};

template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int j) { return (lane >> 4) + 4 * j; }
};

}  // namespace tls
