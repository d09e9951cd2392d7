// Reductions over the 64 lanes of a wave through the data-parallel
// primitives of the ROCm device library (lane exchanges within the vector
// unit instead of round trips through the LDS crossbar).  Every lane of the
// wave must be active; every lane receives the result.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

extern "C" __device__ double __ockl_wfred_max_f64(double);
extern "C" __device__ double __ockl_wfred_add_f64(double);
extern "C" __device__ int __ockl_wfred_min_i32(int);

namespace riga {

__device__ __forceinline__ double wave_max(double v) { return __ockl_wfred_max_f64(v); }
// (a fixed summation order: the same inputs give the same sum every time)
__device__ __forceinline__ double wave_sum(double v) { return __ockl_wfred_add_f64(v); }
__device__ __forceinline__ int wave_min(int v) { return __ockl_wfred_min_i32(v); }

// The largest of the lanes' `v` and the smallest `idx` among the lanes
// holding it with idx >= 0 (-1 if none does): the same choice as scanning
// the candidates in index order and keeping the first strict maximum, for
// lanes that each kept their own first strict maximum over values > 0.
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
  const double best = wave_max(v);
  const int cand = (idx >= 0 && v == best) ? idx : INT_MAX;
  const int i = wave_min(cand);
  v = best;
  idx = i == INT_MAX ? -1 : i;
}

}  // namespace riga
