// kernels_fused.hip - whole-level Matching Pursuit for small blocks (N <= 8).
//
// For N <= 8 the dictionary (M <= 128 atoms of K <= 64 pixels) fits in LDS
// even in FP64 (64 KB), while one MP step of one node is only K*M = 8192
// multiply-adds: a batched correlation launch per step would be all launch
// and latency.  Here one group of TPN = min(K, 64) lanes runs a node's whole
// pursuit (Section 2.2 steps (a)-(d), eq. (2)) without leaving the kernel:
//   r = unravel(block) (FP64, lane = pixel), stop test before every step;
//   c_a = <r, phi_a> for every atom in FP64 (the plain definition, dense);
//   i = argmax |c| (lowest index on ties), stop if max |c| = 0;
//   r <- r - c_i phi_i, ||r||^2, record (i, c_i).
// The residual stays in registers; atoms are formed in LDS once per
// workgroup from the FP64 1D tables (constant atom exactly 1/N).
#include "internal.h"
#include "dev_common.h"

namespace aqmp {

namespace {

template <int N>
struct FGeo {
  static constexpr int K = N * N;
  static constexpr int TPN = K < 64 ? K : 64;     // lanes per node (lane = pixel)
  static constexpr int NPW = 64 / TPN;             // nodes per wave
  static constexpr int MMAX = 2 * K;               // both families
  static constexpr int APL = MMAX / TPN;           // atom slots per lane
  static_assert(TPN == K, "one lane per pixel");
};

template <int TPN>
__device__ inline double grp_sum(double v) {
#pragma unroll
  for (int off = 1; off < TPN; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int N>
__global__ __launch_bounds__(256) void k_mp_fused(const JobDev* __restrict__ jobs, LevelDev lv,
                                                  const int32_t* __restrict__ count_ptr, int32_t lg, int32_t n_atoms,
                                                  const double* __restrict__ tab) {
  using G = FGeo<N>;
  constexpr int K = G::K, TPN = G::TPN;
  // Atoms transposed: sD[pixel][atom], so lane a reads consecutive words.
  __shared__ double sD[K * G::MMAX];
  // Per-node residual copy for broadcast reads during the correlation.
  __shared__ double sR[4 * G::NPW][K];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane / TPN, lt = lane % TPN;
  const double inv_n = 1.0 / N;
  for (int i = tid; i < K * G::MMAX; i += blockDim.x) {
    const int px = i / G::MMAX, a = i % G::MMAX;
    double v = 0.0;
    if (a < n_atoms) {
      const int f = a / K, q = (a % K) / N, p = a % N;
      const int y = px / N, x = px % N;
      v = (p == 0 && q == 0) ? inv_n : tab[(size_t)f * K + p * N + y] * tab[(size_t)f * K + q * N + x];
    }
    sD[i] = v;
  }
  __syncthreads();
  const int count = *count_ptr;
  double* rs = sR[w * G::NPW + g];
  const int stride = gridDim.x * 4 * G::NPW;
  for (int base = (blockIdx.x * 4 + w) * G::NPW; base < count; base += stride) {
    const int node = base + g;
    const bool valid = node < count;
    const int nd = valid ? node : base;
    const JobDev& jb = jobs[lv.job[nd]];
    const double eps2 = jb.eps2[lg];
    const int k = jb.k[lg];
    // gather (Algorithm 2: y = unravel(b))
    const int y = lt / N, x = lt % N;
    const int64_t idx = (int64_t)(lv.y0[nd] + y) * jb.row_stride + lv.x0[nd] + x;
    double r = jb.dtype == AQMP_F64 ? ((const double*)jb.img)[idx] : (double)((const float*)jb.img)[idx];
    double e = grp_sum<TPN>(r * r);
    int t = 0;
    uint8_t st = ST_RUN;
    for (;;) {
      if (e < eps2) { st = ST_ACC; break; }
      if (t >= k) { st = ST_SPARSE; break; }
      rs[lt] = r;                       // group-private; read back by the same group below
      __builtin_amdgcn_wave_barrier();
      double c[G::APL];
#pragma unroll
      for (int j = 0; j < G::APL; ++j) c[j] = 0.0;
#pragma unroll 8
      for (int p = 0; p < K; ++p) {
        const double rp = rs[p];
#pragma unroll
        for (int j = 0; j < G::APL; ++j) c[j] = fma(rp, sD[p * G::MMAX + lt + j * TPN], c[j]);
      }
      __builtin_amdgcn_wave_barrier();
      // arg-max over this lane's atoms, then over the group (lowest index on ties)
      double bm = -1.0;
      int bi = 0x7fffffff;
      double bc = 0.0;
#pragma unroll
      for (int j = 0; j < G::APL; ++j) {
        const int a = lt + j * TPN;
        const double m = fabs(c[j]);
        if (a < n_atoms && (m > bm || (m == bm && a < bi))) { bm = m; bi = a; bc = c[j]; }
      }
#pragma unroll
      for (int off = 1; off < TPN; off <<= 1) {
        const double om = __shfl_xor(bm, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        const double oc = __shfl_xor(bc, off, 64);
        if (om > bm || (om == bm && oi < bi)) { bm = om; bi = oi; bc = oc; }
      }
      if (bm == 0.0) { st = ST_ZERO; break; }
      r = fma(-bc, sD[lt * G::MMAX + bi], r);
      e = grp_sum<TPN>(r * r);
      if (valid && lt == 0) {
        const size_t slot = (size_t)nd * lv.kmax + t;
        lv.rec_idx[slot] = bi;
        lv.rec_coef[slot] = bc;
      }
      ++t;
    }
    if (valid && lt == 0) {
      lv.e[nd] = e;
      lv.t[nd] = t;
      lv.st[nd] = st;
    }
  }
}

}  // namespace

hipError_t launch_mp_fused(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t lg, int32_t n_atoms,
                           const double* tab, hipStream_t s) {
  switch (n) {
    case 4:
      hipLaunchKernelGGL(k_mp_fused<4>, dim3(256 * 4), dim3(256), 0, s, jobs, lv, count, lg, n_atoms, tab);
      break;
    case 8:
      hipLaunchKernelGGL(k_mp_fused<8>, dim3(256 * 2), dim3(256), 0, s, jobs, lv, count, lg, n_atoms, tab);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aqmp
