// kernels_gram.hip - Matching Pursuit through the Gram matrix (exact
// reformulation of Section 2.2, FP64 throughout), for N = 16, 32, 64.
//
// Every atom of D_N is an outer product of two rows of a 1D orthonormal table
// (Section 2.1), so
//   * the correlations of a block with all atoms of family f are the entries
//     of T_f Y T_f^T (two N x N products, O(N^3) per node instead of the
//     O(N^4) dense product), and
//   * after atom i is chosen with c_i = <r, phi_i>, the residual update
//     r <- r - c_i phi_i changes every correlation by the Gram column:
//     c_a <- c_a - c_i <phi_a, phi_i>, with
//     <phi_a, phi_i> = <T_fa[p_a], T_fi[p_i]> <T_fa[q_a], T_fi[q_i]>,
//     and the squared norm by e <- e - c_i^2 (phi_i has unit norm).
// The same-family part of that column is a Kronecker delta (each family is
// an orthonormal basis); the cross-family part is a product of two entries of
// the N x N table X[p][p'] = <T_0[p], T_1[p']>, built once with the
// dictionary with its row and column 0 exact (the constant rows are equal,
// every other row sums to zero).  So an MP step costs O(M) table lookups and
// FMAs, the residual itself is never formed, and the constant atoms (exactly
// 1/N) are handled exactly.
//
// k_gram_init: one workgroup per node: gather, ||y||^2, the first stop test,
// and the correlations (separable products in FP64), written to a per-node
// buffer.
// k_gram_iter: one workgroup per node: the whole pursuit (selection with
// the lowest index on ties, records, stop test of eq. (2)), correlations
// held in registers.
#include "internal.h"
#include "dev_common.h"

namespace aqmp {

namespace {

template <int N>
struct GramGeo {
  static constexpr int K = N * N;
  static constexpr int TB = N / 16;          // output block per thread (TB x TB)
  static constexpr int NP = N + 1;           // padded LDS row (doubles)
};

// Fixed-order sum over the workgroup (4 waves), result in every thread.
__device__ inline double wg_sum(double v, double* red) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

template <int N>
__global__ __launch_bounds__(256) void k_gram_init(const JobDev* __restrict__ jobs, LevelDev lv,
                                                   const int32_t* __restrict__ count_ptr, int32_t lg, int32_t nfam,
                                                   const double* __restrict__ tab, double* __restrict__ cbuf) {
  using G = GramGeo<N>;
  constexpr int K = G::K, TB = G::TB, NP = G::NP;
  __shared__ double sT[2][N][N];    // T_f[p][y]
  __shared__ double sY[N][NP];      // block pixels
  __shared__ double sZ[N][NP];      // T_f Y
  __shared__ double sRed[4];
  const int tid = threadIdx.x;
  for (int i = tid; i < nfam * K; i += 256) (&sT[0][0][0])[i] = tab[i];
  const int count = *count_ptr;
  const int b0 = tid / 16, b1 = tid % 16;   // this thread's output block
  const int M = nfam * K;
  for (int node = blockIdx.x; node < count; node += gridDim.x) {
    __syncthreads();   // sT ready / previous node done with sY, sZ
    const JobDev& jb = jobs[lv.job[node]];
    const int bx = lv.x0[node], by = lv.y0[node];
    double e = 0.0, s = 0.0;
    for (int i = tid; i < K; i += 256) {
      const int y = i / N, x = i % N;
      const int64_t idx = (int64_t)(by + y) * jb.row_stride + bx + x;
      const double v = jb.dtype == AQMP_F64 ? ((const double*)jb.img)[idx] : (double)((const float*)jb.img)[idx];
      sY[y][x] = v;
      e += v * v;
      s += v;
    }
    e = wg_sum(e, sRed);   // (its barriers also publish sY)
    s = wg_sum(s, sRed);
    if (tid == 0) {
      lv.e[node] = e;
      lv.t[node] = 0;
      uint8_t st = ST_RUN;
      if (e < jb.eps2[lg])
        st = ST_ACC;
      else if (jb.k[lg] <= 0)
        st = ST_SPARSE;
      lv.st[node] = st;
    }
    double* cn = cbuf + (size_t)node * M;
    for (int f = 0; f < nfam; ++f) {
      // Z = T_f Y (rows b0 TB.., columns b1 TB..)
      double z[TB][TB];
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) z[i][j] = 0.0;
      for (int y = 0; y < N; ++y) {
        double tv[TB], yv[TB];
#pragma unroll
        for (int i = 0; i < TB; ++i) tv[i] = sT[f][b0 * TB + i][y];
#pragma unroll
        for (int j = 0; j < TB; ++j) yv[j] = sY[y][b1 * TB + j];
#pragma unroll
        for (int i = 0; i < TB; ++i)
#pragma unroll
          for (int j = 0; j < TB; ++j) z[i][j] = fma(tv[i], yv[j], z[i][j]);
      }
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) sZ[b0 * TB + i][b1 * TB + j] = z[i][j];
      __syncthreads();
      // C[p][q] = sum_x Z[p][x] T_f[q][x] (p = b0 TB + i, q = b1 TB + j): atom f K + q N + p
      double c[TB][TB];
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) c[i][j] = 0.0;
      for (int x = 0; x < N; ++x) {
        double zv[TB], tv[TB];
#pragma unroll
        for (int i = 0; i < TB; ++i) zv[i] = sZ[b0 * TB + i][x];
#pragma unroll
        for (int j = 0; j < TB; ++j) tv[j] = sT[f][b1 * TB + j][x];
#pragma unroll
        for (int i = 0; i < TB; ++i)
#pragma unroll
          for (int j = 0; j < TB; ++j) c[i][j] = fma(zv[i], tv[j], c[i][j]);
      }
#pragma unroll
      for (int i = 0; i < TB; ++i)
#pragma unroll
        for (int j = 0; j < TB; ++j) {
          const int p = b0 * TB + i, q = b1 * TB + j;
          cn[f * K + q * N + p] = (p == 0 && q == 0) ? s / N : c[i][j];
        }
      __syncthreads();   // sZ is rewritten by the next family
    }
  }
}

template <int N>
__global__ __launch_bounds__(256) void k_gram_iter(const JobDev* __restrict__ jobs, LevelDev lv,
                                                   const int32_t* __restrict__ count_ptr, int32_t lg, int32_t nfam,
                                                   const double* __restrict__ xg, const double* __restrict__ cbuf) {
  constexpr int K = N * N;
  constexpr int APT = 2 * K / 256;      // atoms per thread (both families)
  constexpr int RW = 64;                // records held in registers between flushes
  constexpr int NP = N + 1;
  __shared__ double sX[N][NP];          // cross-family table X[p][p'] = <T_0[p], T_1[p']>
  __shared__ double sBc[2][4];          // per-wave best (signed) correlation, double-buffered
  __shared__ int sBi[2][4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (nfam == 2)
    for (int i = tid; i < K; i += 256) sX[i / N][i % N] = xg[i];
  __syncthreads();
  const int count = *count_ptr;
  const int M = nfam * K;
  // This thread's atoms a = tid + 256 j: p_a = tid mod N for every j (256 is
  // a multiple of N); q_a and the family depend on j only through 256 j.
  const int pa = tid % N;
  int ph = 0;
  for (int node = blockIdx.x; node < count; node += gridDim.x) {
    const JobDev& jb = jobs[lv.job[node]];
    const double eps2 = jb.eps2[lg];
    const int kmax = jb.k[lg];
    double e = lv.e[node];
    uint8_t st = lv.st[node];
    int t = 0;
    int rec_i = 0;
    double rec_c = 0.0;
    double c[APT];
    const double* cn = cbuf + (size_t)node * M;
#pragma unroll
    for (int j = 0; j < APT; ++j) {
      const int a = tid + 256 * j;
      c[j] = a < M ? cn[a] : 0.0;
    }
    const size_t rec0 = (size_t)node * lv.kmax;
    while (st == ST_RUN) {
      // arg-max |c|, lowest atom index among equal magnitudes
      double bc = 0.0;
      int bi = 0x7fffffff;
#pragma unroll
      for (int j = 0; j < APT; ++j) {
        const int a = tid + 256 * j;
        if (a < M && fabs(c[j]) > fabs(bc)) { bc = c[j]; bi = a; }
      }
      if (bi == 0x7fffffff) bi = tid;   // all zero: lowest own index
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double oc = __shfl_xor(bc, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (fabs(oc) > fabs(bc) || (fabs(oc) == fabs(bc) && oi < bi)) { bc = oc; bi = oi; }
      }
      if (lane == 0) { sBc[ph][w] = bc; sBi[ph][w] = bi; }
      __syncthreads();
      bc = sBc[ph][0];
      bi = sBi[ph][0];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        const double oc = sBc[ph][q];
        const int oi = sBi[ph][q];
        if (fabs(oc) > fabs(bc) || (fabs(oc) == fabs(bc) && oi < bi)) { bc = oc; bi = oi; }
      }
      ph ^= 1;
      if (bc == 0.0) { st = ST_ZERO; break; }
      if (tid == t % RW) { rec_i = bi; rec_c = bc; }
      // c_a <- c_a - c_i <phi_a, phi_i>: same family -> Kronecker delta
      // (orthonormal basis); other family -> X[p_a][p_i] X[q_a][q_i] (or
      // its transpose), which also covers the constant atoms exactly.
      const int fi = bi / K, pi = bi % N, qi = (bi % K) / N;
      const double vp = fi ? sX[pa][pi] : sX[pi][pa];
#pragma unroll
      for (int j = 0; j < APT; ++j) {
        const int a = tid + 256 * j;
        const int fa = a / K;
        if (fa == fi) {
          if (a == bi) c[j] = 0.0;
        } else if (a < M) {
          const int qa = (a % K) / N;
          const double vq = fi ? sX[qa][qi] : sX[qi][qa];
          c[j] = fma(-bc, vp * vq, c[j]);
        }
      }
      e = fma(-bc, bc, e);
      ++t;
      if (t % RW == 0 && tid < RW) {
        lv.rec_idx[rec0 + (t - RW) + tid] = rec_i;
        lv.rec_coef[rec0 + (t - RW) + tid] = rec_c;
      }
      if (e < eps2)
        st = ST_ACC;
      else if (t >= kmax)
        st = ST_SPARSE;
    }
    if (tid < t % RW) {
      lv.rec_idx[rec0 + (t - t % RW) + tid] = rec_i;
      lv.rec_coef[rec0 + (t - t % RW) + tid] = rec_c;
    }
    if (tid == 0) {
      lv.e[node] = e;
      lv.t[node] = t;
      lv.st[node] = st;
    }
  }
}

}  // namespace

hipError_t launch_mp_gram(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t lg, int32_t nfam,
                          const double* tab, const double* xg, double* cbuf, hipStream_t s) {
  if (nfam == 2 && !xg) return hipErrorInvalidValue;
  switch (n) {
    case 16:
      hipLaunchKernelGGL(k_gram_init<16>, dim3(2048), dim3(256), 0, s, jobs, lv, count, lg, nfam, tab, cbuf);
      hipLaunchKernelGGL(k_gram_iter<16>, dim3(2048), dim3(256), 0, s, jobs, lv, count, lg, nfam, xg, cbuf);
      break;
    case 32:
      hipLaunchKernelGGL(k_gram_init<32>, dim3(1024), dim3(256), 0, s, jobs, lv, count, lg, nfam, tab, cbuf);
      hipLaunchKernelGGL(k_gram_iter<32>, dim3(1024), dim3(256), 0, s, jobs, lv, count, lg, nfam, xg, cbuf);
      break;
    case 64:
      hipLaunchKernelGGL(k_gram_init<64>, dim3(256), dim3(256), 0, s, jobs, lv, count, lg, nfam, tab, cbuf);
      hipLaunchKernelGGL(k_gram_iter<64>, dim3(512), dim3(256), 0, s, jobs, lv, count, lg, nfam, xg, cbuf);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aqmp
