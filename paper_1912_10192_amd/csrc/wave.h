// wave.h -- wavefront (64-lane) reductions and counting used by the kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace grmhd {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// add one to ctr[value] for every active lane: one add per distinct value per wave, by
// the first lane holding that value (ctr may live in LDS or in global memory)
template <typename T>
__device__ __forceinline__ void wave_count(T* ctr, int value, bool active) {
  unsigned long long mask = __ballot(active);
  while (mask) {
    const int leader = __ffsll((long long)mask) - 1;
    const int v = __shfl(value, leader);
    const unsigned long long same = __ballot(active && value == v);
    if (lane_id() == leader) atomicAdd(&ctr[v], (T)__popcll(same));
    if (active && value == v) active = false;
    mask = __ballot(active);
  }
}

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ long long wave_sum(long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace grmhd
