// One 16 x 16 output tile of the 16x16x4 matrix-core instructions, in the
// precision of the factor T: FP64 operands and accumulation
// (v_mfma_f64_16x16x4f64) for double, FP32 (v_mfma_f32_16x16x4f32) for
// float.  Both take, from lane l, A(l % 16, l / 16) and B(l / 16, l % 16) of
// a 16 x 4 by 4 x 16 step; they leave their four results in different rows:
// element i of lane l is D(row(l, i), l % 16).
#pragma once

#include <hip/hip_runtime.h>

namespace riga {

typedef double mfma_v4d __attribute__((ext_vector_type(4)));
typedef float mfma_v4f __attribute__((ext_vector_type(4)));

template <class T>
struct Tile16;

template <>
struct Tile16<double> {
  mfma_v4d acc;
  __device__ __forceinline__ void zero() { acc = mfma_v4d{0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ void step(double a, double b) {
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  __device__ __forceinline__ double get(int i) const { return acc[i]; }
  __device__ static __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct Tile16<float> {
  mfma_v4f acc;
  __device__ __forceinline__ void zero() { acc = mfma_v4f{0.0f, 0.0f, 0.0f, 0.0f}; }
  __device__ __forceinline__ void step(double a, double b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, acc, 0, 0, 0);
  }
  __device__ __forceinline__ double get(int i) const { return (double)acc[i]; }
  __device__ static __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

}  // namespace riga
