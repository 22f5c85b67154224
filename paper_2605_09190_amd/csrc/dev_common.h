// dev_common.h - device helpers shared by the AQMP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aqmp {

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ __host__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Threads that cooperate on one quadtree node of size N: TPN threads per
// node (at most one 256-thread workgroup), NPW nodes per workgroup, PPT
// pixels per thread arranged as a PH x PW patch of the N x N block.
template <int N>
struct Geo {
  static constexpr int K = N * N;
  static constexpr int TPN = K < 256 ? K : 256;
  static constexpr int NPW = 256 / TPN;
  static constexpr int PPT = K / TPN;
  static constexpr int PH = PPT == 16 ? 4 : (PPT == 4 ? 2 : 1);
  static constexpr int PW = PPT / PH;
  static constexpr int PX = N / PW;   // patches per patch row
};

// Sum of v over the TPN threads of a node group, returned to every thread
// of the group.  Fixed butterfly order, then (TPN = 256) a fixed-order sum of
// the four wave totals: the result is bit-reproducible.  `scratch` must hold
// 4 doubles per group and the call must be reached by the whole workgroup.
template <int TPN>
__device__ inline double group_sum(double v, double* scratch) {
  constexpr int W = TPN < 64 ? TPN : 64;
#pragma unroll
  for (int off = 1; off < W; off <<= 1) v += __shfl_xor(v, off, 64);
  if constexpr (TPN > 64) {
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    v = (scratch[0] + scratch[1]) + (scratch[2] + scratch[3]);
  }
  return v;
}

// Same for an array of CNT doubles (each element reduced independently).
template <int TPN, int CNT>
__device__ inline void group_sum_n(double (&v)[CNT], double* scratch) {
  constexpr int W = TPN < 64 ? TPN : 64;
#pragma unroll
  for (int c = 0; c < CNT; ++c) {
#pragma unroll
    for (int off = 1; off < W; off <<= 1) v[c] += __shfl_xor(v[c], off, 64);
  }
  if constexpr (TPN > 64) {
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int c = 0; c < CNT; ++c) scratch[c * 4 + w] = v[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CNT; ++c)
      v[c] = (scratch[c * 4 + 0] + scratch[c * 4 + 1]) + (scratch[c * 4 + 2] + scratch[c * 4 + 3]);
  }
}

}  // namespace aqmp
