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

// ---------------------------------------------------------------------------
// Decoupled look-back for stable single-pass prefix sums.  A tile word holds a
// flag in its top two bits (1: tile aggregate published, 2: inclusive prefix
// published) and a 32-bit count.  Tiles are taken in ticket order, so a tile
// only waits on tiles held by workgroups that started before it.  Each wait
// is bounded; when the bound runs out *err is set and the (then wrong) sum is
// used, so every wave still finishes.
// ---------------------------------------------------------------------------
constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagInc = 2ull << 62;
constexpr int kSpinLimit = 1 << 24;

__device__ inline unsigned long long load_acq(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_rel(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-parallel look-back, called by all 64 lanes of one wave: publishes
// tile `tile`'s aggregate, then reads up to 64 predecessors per probe (lane i
// reads tile - 1 - i), stops at the nearest inclusive prefix, and publishes its
// own inclusive prefix.  Returns the exclusive prefix in every lane.
__device__ inline int lookback_wave(unsigned long long* tiles, int tile, int agg, int32_t* err) {
  const int lane = threadIdx.x & 63;
  if (tile == 0) {
    if (lane == 0) store_rel(&tiles[0], kFlagInc | (unsigned)agg);
    return 0;
  }
  if (lane == 0) store_rel(&tiles[tile], kFlagAgg | (unsigned)agg);
  int prefix = 0, end = tile, spins = 0;
  for (;;) {
    const int idx = end - 1 - lane;
    const unsigned long long v = idx >= 0 ? load_acq(&tiles[idx]) : (kFlagInc | 0ull);
    const unsigned fl = (unsigned)(v >> 62);
    const int val = (int)(unsigned)(v & 0xFFFFFFFFull);
    const unsigned long long inc = __ballot(fl == 2);
    const unsigned long long miss = __ballot(fl == 0);
    const unsigned long long upto = inc ? (inc & (~inc + 1ull)) : 0ull;   // lowest inclusive lane
    const unsigned long long need = inc ? (upto | (upto - 1ull)) : ~0ull;   // lanes that must be ready
    if (miss & need) {
      if (++spins > kSpinLimit) {
        if (lane == 0) atomicExch(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    int x = ((need >> lane) & 1ull) ? val : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
    prefix += x;
    if (inc) break;
    end -= 64;
    spins = 0;
  }
  if (lane == 0) store_rel(&tiles[tile], kFlagInc | (unsigned)(prefix + agg));
  return prefix;
}

// Whole-wave reductions with DPP row operations (quad swaps, row mirrors,
// row broadcasts 15 and 31), then a read of lane 63: a fixed order, so the
// results are bit-reproducible, and no LDS-crossbar round trips.
template <int CTRL, int RM>
__device__ inline unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, RM, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ inline unsigned long long lane63_u64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
#define AQMP_MAXSTEP(C, RM) { const unsigned long long o = dpp_u64<C, RM>(v); v = o > v ? o : v; }
  AQMP_MAXSTEP(0xB1, 0xF) AQMP_MAXSTEP(0x4E, 0xF) AQMP_MAXSTEP(0x141, 0xF)
  AQMP_MAXSTEP(0x140, 0xF) AQMP_MAXSTEP(0x142, 0xA) AQMP_MAXSTEP(0x143, 0xC)
#undef AQMP_MAXSTEP
  return lane63_u64(v);
}
// Orders the LDS writes of a wave's lanes before its later LDS reads by
// other lanes of the same wave (no workgroup barrier): the wave's LDS
// operations complete before it goes on.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline double wave_sum_f64(double d) {
#define AQMP_SUMSTEP(C, RM) { d += __longlong_as_double((long long)dpp_u64<C, RM>((unsigned long long)__double_as_longlong(d))); }
  AQMP_SUMSTEP(0xB1, 0xF) AQMP_SUMSTEP(0x4E, 0xF) AQMP_SUMSTEP(0x141, 0xF)
  AQMP_SUMSTEP(0x140, 0xF) AQMP_SUMSTEP(0x142, 0xA) AQMP_SUMSTEP(0x143, 0xC)
#undef AQMP_SUMSTEP
  return __longlong_as_double((long long)lane63_u64((unsigned long long)__double_as_longlong(d)));
}


}  // namespace aqmp
