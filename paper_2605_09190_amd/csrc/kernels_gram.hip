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
// k_gram_init: gather, ||y||^2, the first stop test, and the correlations of
// every node as two FP64 matrix-core products per family (Z^T = Y^T T_f^T,
// then C^T = T_f Z^T), written to a per-node buffer.  N / 16 waves per node,
// each owning one 16-wide strip of the row index p.
// k_gram_pursuit: the whole pursuit of every node (selection with the lowest
// index on ties, records, stop test of eq. (2)) with the correlations held
// in registers: one wave per node for N <= 32, four for N = 64.
#include "internal.h"
#include "dev_common.h"

namespace aqmp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// LDS index of element (row, col) of an N x N FP64 tile.  The matrix-core
// operands are read as four rows of 16 consecutive doubles; for N >= 32 the
// odd rows swap their 16-column halves so that two such rows fall on
// different banks.
template <int N>
__device__ inline int sw(int row, int col) {
  if constexpr (N >= 32)
    return row * N + (col ^ ((row & 1) << 4));
  else
    return row * N + col;
}

// v_mfma_f64_16x16x4_f64: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; it holds D[l / 16 + 4 r][l % 16], r = 0..3.
__device__ inline d4 mfma64(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

template <int N, int NFAM>
struct InitGeo {
  static constexpr int K = N * N;
  static constexpr int M = NFAM * K;
  static constexpr int WPN = N / 16;        // waves per node
  static constexpr int GPW = 4 / WPN;       // nodes per workgroup
  static constexpr int TPN = 64 * WPN;      // threads per node
  static constexpr int T = N / 16;          // 16 x 16 output tiles along x (or p)
  static constexpr int KS = N / 4;          // k-steps of one product
};

// Wave wn of a node owns the 16-row strip s0 = 16 wn of the 1D tables.  It
// computes Z^T[x][p] for p in its strip (first product, all x) and C^T[q][p]
// for q in its strip (second product, all p).  Both products read the same
// table entries T_f[s0 + l % 16][4 ks + l / 16] (the B operand of the first,
// the A operand of the second), which the lane keeps in registers for the
// whole kernel; only Y and Z^T go through LDS.
template <int N, int NFAM>
__global__ __launch_bounds__(256) void k_gram_init(const JobDev* __restrict__ jobs, LevelDev lv,
                                                   const int32_t* __restrict__ count_ptr, int32_t lg,
                                                   const double* __restrict__ tab, double* __restrict__ cbuf) {
  using G = InitGeo<N, NFAM>;
  constexpr int K = G::K, M = G::M, WPN = G::WPN, GPW = G::GPW, TPN = G::TPN, T = G::T, KS = G::KS;
  __shared__ double sY[GPW][K];             // sY[g][sw(y, x)] = pixel (y, x)
  __shared__ double sZt[GPW][K];            // sZt[g][sw(x, p)] = (T_f Y)[p][x]
  __shared__ double sRed[GPW][WPN][2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = tid / TPN, tn = tid % TPN, wn = tn >> 6;
  const int s0 = 16 * wn;
  const int li = lane & 15, lk = lane >> 4;
  double tr[NFAM][KS];
#pragma unroll
  for (int f = 0; f < NFAM; ++f)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) tr[f][ks] = tab[(size_t)f * K + (s0 + li) * N + 4 * ks + lk];
  const int count = *count_ptr;
  for (int base = blockIdx.x * GPW; base < count; base += gridDim.x * GPW) {
    const int node = base + g;
    const bool live = node < count;
    double e = 0.0, s = 0.0;
    const JobDev* jb = nullptr;
    if (live) {
      jb = &jobs[lv.job[node]];
      const int bx = lv.x0[node], by = lv.y0[node];
#pragma unroll
      for (int i0 = 0; i0 < K; i0 += TPN) {
        const int i = i0 + tn;
        const int y = i / N, x = i % N;
        const double v = job_pixel(*jb, by + y, bx + x);
        sY[g][sw<N>(y, x)] = v;
        e = fma(v, v, e);
        s += v;
      }
    }
    e = wave_sum_f64(e);
    s = wave_sum_f64(s);
    if (lane == 0) {
      sRed[g][wn][0] = e;
      sRed[g][wn][1] = s;
    }
    __syncthreads();   // sY, sRed ready
    if (live) {
      e = sRed[g][0][0];
      s = sRed[g][0][1];
#pragma unroll
      for (int q = 1; q < WPN; ++q) {
        e += sRed[g][q][0];
        s += sRed[g][q][1];
      }
      if (tn == 0) {
        lv.e[node] = e;
        lv.t[node] = 0;
        uint8_t st = ST_RUN;
        if (e < jb->eps2[lg])
          st = ST_ACC;
        else if (jb->k[lg] <= 0)
          st = ST_SPARSE;
        lv.st[node] = st;
      }
    }
    double* cn = cbuf + (size_t)node * M;
#pragma unroll
    for (int f = 0; f < NFAM; ++f) {
      // Z^T[x][p] = sum_y Y[y][x] T_f[p][y], p in this wave's strip
      d4 acc[T];
#pragma unroll
      for (int tx = 0; tx < T; ++tx) acc[tx] = d4{0.0, 0.0, 0.0, 0.0};
      if (live) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + lk;
#pragma unroll
          for (int tx = 0; tx < T; ++tx) acc[tx] = mfma64(sY[g][sw<N>(k, 16 * tx + li)], tr[f][ks], acc[tx]);
        }
      }
      __syncthreads();   // the previous family's second product is done with sZt
      if (live) {
#pragma unroll
        for (int tx = 0; tx < T; ++tx)
#pragma unroll
          for (int r = 0; r < 4; ++r) sZt[g][sw<N>(16 * tx + lk + 4 * r, s0 + li)] = acc[tx][r];
      }
      __syncthreads();   // Z^T complete
      if (live) {
        // C^T[q][p] = sum_x T_f[q][x] Z^T[x][p], q in this wave's strip
#pragma unroll
        for (int tp = 0; tp < T; ++tp) acc[tp] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + lk;
#pragma unroll
          for (int tp = 0; tp < T; ++tp) acc[tp] = mfma64(tr[f][ks], sZt[g][sw<N>(k, 16 * tp + li)], acc[tp]);
        }
        // atom f K + q N + p; the constant atom (p = q = 0) is exactly 1/N
#pragma unroll
        for (int tp = 0; tp < T; ++tp)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = s0 + lk + 4 * r, pp = 16 * tp + li;
            cn[f * K + q * N + pp] = (q == 0 && pp == 0) ? s / N : acc[tp][r];
          }
      }
    }
    // The next round's gather writes sY: every wave has passed the barriers
    // after its last read of sY (first product of the last family).
  }
}

template <int N, int NFAM>
struct PurGeo {
  static constexpr int K = N * N;
  static constexpr int M = NFAM * K;
  static constexpr int TPN = N == 64 ? 256 : 64;   // threads per node
  static constexpr int WPN = TPN / 64;
  static constexpr int APT = M / TPN;              // atoms per thread
  static constexpr int NPW = 256 / TPN;            // nodes per workgroup
};

// Best atom of a wave: largest |c|, lowest atom index among equal
// magnitudes; the result is uniform across the wave.  |c| is non-negative,
// so its bit pattern orders like its value.
__device__ inline void wave_best(double bc, int bi, double& wbc, int& wbi) {
  const unsigned long long mb = (unsigned long long)__double_as_longlong(fabs(bc));
  const unsigned long long m = wave_max_u64(mb);
  unsigned long long ball = __ballot(mb == m);
  int best = 0x7fffffff, L = 0;
  while (ball) {
    const int l = __builtin_ctzll(ball);
    const int cand = __builtin_amdgcn_readlane(bi, l);
    if (cand < best) {
      best = cand;
      L = l;
    }
    ball &= ball - 1;
  }
  const long long v = __double_as_longlong(bc);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), L);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), L);
  wbc = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  wbi = best;
}

// Largest |v[j]| of a register array and its position, lowest j among equal
// magnitudes (pairwise tree: the left operand always holds lower positions).
template <int A>
__device__ inline void lane_best(const double (&c)[A], double& bc, int& bj) {
  double v[A];
  int ix[A];
#pragma unroll
  for (int j = 0; j < A; ++j) {
    v[j] = c[j];
    ix[j] = j;
  }
#pragma unroll
  for (int w = 1; w < A; w *= 2)
#pragma unroll
    for (int i = 0; i + w < A; i += 2 * w) {
      const bool take = fabs(v[i + w]) > fabs(v[i]);
      v[i] = take ? v[i + w] : v[i];
      ix[i] = take ? ix[i + w] : ix[i];
    }
  bc = v[0];
  bj = ix[0];
}

template <int N, int NFAM>
__global__ __launch_bounds__(256) void k_gram_pursuit(const JobDev* __restrict__ jobs, LevelDev lv,
                                                      const int32_t* __restrict__ count_ptr, int32_t* next, int32_t lg,
                                                      const double* __restrict__ xg, const double* __restrict__ cbuf) {
  using G = PurGeo<N, NFAM>;
  constexpr int K = G::K, M = G::M, TPN = G::TPN, WPN = G::WPN, APT = G::APT, NPW = G::NPW;
  constexpr int AF = APT / NFAM;          // atoms per thread per family
  constexpr int RW = 64;                  // records held in registers between flushes
  constexpr int NX = NFAM == 2 ? N : 1;
  __shared__ double sX[NX][NX + 1];       // X[p][p'] = <T_0[p], T_1[p']>
  __shared__ double sBc[2][4];            // per-wave best, double-buffered (N = 64)
  __shared__ int sBi[2][4];
  __shared__ int sNode[2];                // node handed to the workgroup (N = 64), double-buffered
  const int tid = threadIdx.x, lane = tid & 63;
  const int tn = tid % TPN, wn = tn >> 6;
  if constexpr (NFAM == 2)
    for (int i = tid; i < K; i += 256) sX[i / N][i % N] = xg[i];
  __syncthreads();
  const int count = *count_ptr;
  // This thread's atoms: a = tn + TPN j.  TPN is a multiple of N, so p_a =
  // tn mod N for every j, q_a = (tn / N + (TPN / N) j) mod N and the family
  // is j / AF.
  const int pa = tn % N;
  const int qb = tn / N;
  int ph = 0, np = 0;
  // Nodes are handed out one at a time from a counter: their pursuits differ
  // in length by up to k steps, and neighbouring node indices (the same
  // block in the channels of one image) tend to be long together.
  for (;;) {
    // N = 64: one thread fetches, the workgroup reads the value after the
    // barrier.  Smaller blocks (one wave per node, short pursuits): a fixed
    // grid-stride assignment, since a fetch per node would cost more than
    // the imbalance it removes.
    int node;
    if constexpr (NPW == 1) {
      if (tid == 0) sNode[np] = atomicAdd(next, 1);
      __syncthreads();
      node = sNode[np];
      np ^= 1;
    } else {
      node = (blockIdx.x + gridDim.x * np) * NPW + (tid >> 6);
      ++np;
    }
    if (node >= count) break;
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
    for (int j = 0; j < APT; ++j) c[j] = cn[tn + TPN * j];
    const size_t rec0 = (size_t)node * lv.kmax;
    while (st == ST_RUN) {
      // this thread's best (ascending j is ascending atom index)
      double bc;
      int bj;
      lane_best(c, bc, bj);
      int bi = tn + TPN * bj;
      wave_best(bc, bi, bc, bi);
      if constexpr (WPN > 1) {
        if (lane == 0) {
          sBc[ph][wn] = bc;
          sBi[ph][wn] = bi;
        }
        __syncthreads();
        bc = sBc[ph][0];
        bi = sBi[ph][0];
#pragma unroll
        for (int q = 1; q < WPN; ++q) {
          const double oc = sBc[ph][q];
          const int oi = sBi[ph][q];
          if (fabs(oc) > fabs(bc) || (fabs(oc) == fabs(bc) && oi < bi)) {
            bc = oc;
            bi = oi;
          }
        }
        ph ^= 1;
      }
      if (bc == 0.0) {
        st = ST_ZERO;
        break;
      }
      if (tn == t % RW) {
        rec_i = bi;
        rec_c = bc;
      }
      // c_a <- c_a - c_i <phi_a, phi_i>.  Across families the Gram entry is
      // X[p_a][p_i] X[q_a][q_i] (or its transpose), exact for the constant
      // atoms.  Within the chosen atom's family it is a Kronecker delta, so
      // only c_i changes, to zero: c_j += z s_j with z = -c_i on the thread
      // holding it (0 elsewhere) and s_j = [j = j_i] a scalar 0 or 1 gives
      // exactly 0 there and leaves every other value unchanged, at one FMA
      // per atom.
      const int fi = bi / K, pi = bi % N, qi = (bi % K) / N;
      const double z = (tn == bi % TPN) ? -bc : 0.0;
      const int jsel = __builtin_amdgcn_readfirstlane(bi / TPN);
      if constexpr (NFAM == 2) {
        if (fi == 0) {
          const double bv = -bc * sX[pi][pa];
#pragma unroll
          for (int j = 0; j < AF; ++j) c[j] = fma(z, j == jsel ? 1.0 : 0.0, c[j]);
#pragma unroll
          for (int j = AF; j < APT; ++j) {
            const int qa = (qb + (TPN / N) * j) % N;
            c[j] = fma(bv, sX[qi][qa], c[j]);
          }
        } else {
          const double bv = -bc * sX[pa][pi];
#pragma unroll
          for (int j = 0; j < AF; ++j) {
            const int qa = (qb + (TPN / N) * j) % N;
            c[j] = fma(bv, sX[qa][qi], c[j]);
          }
#pragma unroll
          for (int j = AF; j < APT; ++j) c[j] = fma(z, j == jsel ? 1.0 : 0.0, c[j]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < APT; ++j) c[j] = fma(z, j == jsel ? 1.0 : 0.0, c[j]);
      }
      e = fma(-bc, bc, e);
      ++t;
      if (t % RW == 0 && tn < RW) {
        lv.rec_idx[rec0 + (t - RW) + tn] = rec_i;
        lv.rec_coef[rec0 + (t - RW) + tn] = rec_c;
      }
      if (e < eps2)
        st = ST_ACC;
      else if (t >= kmax)
        st = ST_SPARSE;
    }
    if (tn < t % RW) {
      lv.rec_idx[rec0 + (t - t % RW) + tn] = rec_i;
      lv.rec_coef[rec0 + (t - t % RW) + tn] = rec_c;
    }
    if (tn == 0) {
      lv.e[node] = e;
      lv.t[node] = t;
      lv.st[node] = st;
    }
  }
}

// ---------------------------------------------------------------------------
// Small blocks (N = 4, 8): one group of K = N^2 lanes per node (a whole wave
// at N = 8, a row of 16 lanes at N = 4), lane = pixel for the gather and
// lane = (p, q) for the atoms, one atom per family per lane.  The
// correlations come from the separable sum sum_y T_f[p][y] sum_x T_f[q][x]
// Y[y][x]; the pursuit then runs on the Gram updates as above.  Selection
// reductions stay inside the group (DPP row operations; the wave-wide form
// at N = 8): the largest |c|, then the lowest atom index among the lanes
// holding it, then that lane's c.
// ---------------------------------------------------------------------------
template <int LPN>
__device__ inline unsigned long long grp_max_u64(unsigned long long v) {
  if constexpr (LPN == 64) {
    return wave_max_u64(v);
  } else {
    static_assert(LPN == 16, "groups of 16 or 64 lanes");
#define AQMP_GMAX(C) { const unsigned long long o = dpp_u64<C, 0xF>(v); v = o > v ? o : v; }
    AQMP_GMAX(0xB1) AQMP_GMAX(0x4E) AQMP_GMAX(0x141) AQMP_GMAX(0x140)
#undef AQMP_GMAX
    return v;
  }
}
template <int LPN>
__device__ inline double grp_sum_f64(double d) {
  if constexpr (LPN == 64) {
    return wave_sum_f64(d);
  } else {
#define AQMP_GSUM(C) { d += __longlong_as_double((long long)dpp_u64<C, 0xF>((unsigned long long)__double_as_longlong(d))); }
    AQMP_GSUM(0xB1) AQMP_GSUM(0x4E) AQMP_GSUM(0x141) AQMP_GSUM(0x140)
#undef AQMP_GSUM
    return d;
  }
}
// Minimum of non-negative 32-bit values over the group (lanes that a row
// operation leaves without a source keep their own value).
template <int CTRL, int RM>
__device__ inline int dpp_keep(int v) { return __builtin_amdgcn_update_dpp(v, v, CTRL, RM, 0xF, false); }
template <int LPN>
__device__ inline int grp_min_i32(int v) {
#define AQMP_GMIN(C, RM) { const int o = dpp_keep<C, RM>(v); v = o < v ? o : v; }
  AQMP_GMIN(0xB1, 0xF) AQMP_GMIN(0x4E, 0xF) AQMP_GMIN(0x141, 0xF) AQMP_GMIN(0x140, 0xF)
  if constexpr (LPN == 64) {
    AQMP_GMIN(0x142, 0xA) AQMP_GMIN(0x143, 0xC)
    v = __builtin_amdgcn_readlane(v, 63);
  }
#undef AQMP_GMIN
  return v;
}

template <int N, int NFAM>
__global__ __launch_bounds__(256) void k_gram_small(const JobDev* __restrict__ jobs, LevelDev lv,
                                                    const int32_t* __restrict__ count_ptr, int32_t lg,
                                                    const double* __restrict__ tab, const double* __restrict__ xg) {
  constexpr int K = N * N;
  constexpr int LPN = K;                 // lanes per node
  constexpr int GPW = 64 / LPN;          // nodes per wave
  constexpr int NG = 4 * GPW;            // nodes per workgroup
  constexpr int NX = NFAM == 2 ? N : 1;
  __shared__ double sT[NFAM][K];         // T_f[p][y] at [f][p N + y]
  __shared__ double sX[NX][NX + 1];      // X[p][p'] = <T_0[p], T_1[p']>
  __shared__ double sY[NG][K];           // the node's pixels (group-private)
  const int tid = threadIdx.x, lane = tid & 63;
  const int grp = (tid >> 6) * GPW + lane / LPN, lt = lane % LPN;
  for (int i = tid; i < NFAM * K; i += 256) (&sT[0][0])[i] = tab[i];
  if constexpr (NFAM == 2)
    for (int i = tid; i < K; i += 256) sX[i / N][i % N] = xg[i];
  __syncthreads();
  const int count = *count_ptr;
  const int pa = lt % N, qa = lt / N;    // this lane's atoms f K + lt
  for (int node = blockIdx.x * NG + grp; node < count; node += gridDim.x * NG) {
    const JobDev& jb = jobs[lv.job[node]];
    const double eps2 = jb.eps2[lg];
    const int kmax = jb.k[lg];
    const double v = job_pixel(jb, lv.y0[node] + qa, lv.x0[node] + pa);   // pixel (lt / N, lt % N)
    sY[grp][lt] = v;
    __builtin_amdgcn_wave_barrier();     // group-private: the wave's own writes are seen by its reads
    double e = grp_sum_f64<LPN>(v * v);
    const double s = grp_sum_f64<LPN>(v);
    uint8_t st = ST_RUN;
    if (e < eps2)
      st = ST_ACC;
    else if (kmax <= 0)
      st = ST_SPARSE;
    double c[NFAM];
#pragma unroll
    for (int f = 0; f < NFAM; ++f) {
      double acc = 0.0;
#pragma unroll
      for (int y = 0; y < N; ++y) {
        double u = 0.0;
#pragma unroll
        for (int x = 0; x < N; ++x) u = fma(sT[f][qa * N + x], sY[grp][y * N + x], u);
        acc = fma(sT[f][pa * N + y], u, acc);
      }
      c[f] = lt == 0 ? s / N : acc;
    }
    __builtin_amdgcn_wave_barrier();     // sY is rewritten by the next node
    int t = 0, rec_i = 0;
    double rec_c = 0.0;
    const size_t rec0 = (size_t)node * lv.kmax;
    while (st == ST_RUN) {
      double bc = c[0];
      int bi = lt;
      if constexpr (NFAM == 2) {
        const bool take = fabs(c[1]) > fabs(bc);
        bc = take ? c[1] : bc;
        bi = take ? K + lt : bi;
      }
      const unsigned long long mb = (unsigned long long)__double_as_longlong(fabs(bc));
      const unsigned long long m = grp_max_u64<LPN>(mb);
      bi = grp_min_i32<LPN>(mb == m ? bi : 0x7fffffff);
      if (m == 0ull) {
        st = ST_ZERO;
        break;
      }
      bc = grp_sum_f64<LPN>((lt == bi % K) ? (bi >= K ? c[NFAM - 1] : c[0]) : 0.0);
      if (lt == t % LPN) {
        rec_i = bi;
        rec_c = bc;
      }
      const int fi = bi / K, pi = bi % N, qi = (bi % K) / N;
      // same family: only c_i changes (to zero); other family: X products
#pragma unroll
      for (int f = 0; f < NFAM; ++f) {
        if (f == fi) {
          c[f] = (lt == bi % K) ? 0.0 : c[f];
        } else if constexpr (NFAM == 2) {
          const double g = fi ? sX[pa][pi] * sX[qa][qi] : sX[pi][pa] * sX[qi][qa];
          c[f] = fma(-bc, g, c[f]);
        }
      }
      e = fma(-bc, bc, e);
      ++t;
      if (t % LPN == 0) {
        lv.rec_idx[rec0 + (t - LPN) + lt] = rec_i;
        lv.rec_coef[rec0 + (t - LPN) + lt] = rec_c;
      }
      if (e < eps2)
        st = ST_ACC;
      else if (t >= kmax)
        st = ST_SPARSE;
    }
    if (lt < t % LPN) {
      lv.rec_idx[rec0 + (t - t % LPN) + lt] = rec_i;
      lv.rec_coef[rec0 + (t - t % LPN) + lt] = rec_c;
    }
    if (lt == 0) {
      lv.e[node] = e;
      lv.t[node] = t;
      lv.st[node] = st;
    }
  }
}

// ---------------------------------------------------------------------------
// Orthogonal Matching Pursuit (the solver of the authors' implementation,
// Section 2.2): the selection of MP, then every selected coefficient re-fit by
// least squares, x_S = argmin ||y - D_S x||.  Computed in correlation space
// with the same Gram structure:
//   * L = the inverse of the Cholesky factor of the selected atoms' Gram
//     matrix G_SS (lower triangular, in LDS), one new row per step: with
//     g = G_{S,i} and w = L g, d = sqrt(1 - w.w), the row is (-w^T L, 1) / d;
//   * z = L D_S^T y grows by z_t = (<y, phi_i> - w.z) / d, so
//     ||r||^2 = ||y||^2 - ||z||^2 drops by z_t^2, and x_S = L^T z;
//   * c = D^T r = c0 - G_{:,S} x_S: within a family the Gram column is a
//     Kronecker delta (the selected atoms' own correlations are exactly zero,
//     r being orthogonal to them), across families the X products.
// One workgroup per node at every N (the per-step solves are small and
// serial), nodes handed out from a counter.  c0 = D^T y comes from
// k_gram_init for N >= 16 and is computed here for N <= 8.
// ---------------------------------------------------------------------------
template <int N, int NFAM>
struct OmpGeo {
  static constexpr int K = N * N;
  static constexpr int M = NFAM * K;
  static constexpr bool SMALL = N <= 8;                // K <= 64: one wave, lane k holds atom (f, k) of each family, c0 computed here
  // threads per node: one wave at N <= 16 (its workgroup barriers are the
  // wave's own ordering), two waves at N = 32, eight at N = 64 (two 16 x 16
  // tiles per wave and family at either)
  static constexpr int NT = N <= 16 ? 64 : (N == 32 ? 128 : 512);
  // N >= 16 (MF): a family's N x N grid of (p, q) is cut into 16 x 16 tiles,
  // TPW consecutive tiles per wave; a lane holds, per tile, the four atoms of
  // the FP64 MFMA output layout: p = 16 tp + lane / 16 + 4 r,
  // q = 16 tq + lane % 16, as j = f AF + 4 i + r, so the cross-family refresh
  // is a rank-4 MFMA update per four selected atoms.  The atom index grows
  // with j, so the per-thread arg-max keeps the lowest index on ties.
  static constexpr bool MF = !SMALL;
  static constexpr int NT16 = N / 16;                  // tiles per row of a family's grid
  static constexpr int TPW = MF ? NT16 * NT16 / (NT / 64) : 1;   // tiles per wave per family
  static constexpr int AF = MF ? 4 * TPW : 1;          // atoms per thread per family
  static constexpr int APT = SMALL ? NFAM : NFAM * AF;
  // a wave's tiles cover the grid once and lie in one tile row (so that the
  // atom index grows with j); at most eight waves (the per-wave best slots)
  static_assert(!MF || (TPW * (NT / 64) == NT16 * NT16 && NT16 % TPW == 0), "tile split");
  static_assert(NT <= 512, "per-wave slots");
  __device__ static int atom(int tid, int j) {
    if constexpr (SMALL) return tid < K ? j * K + tid : M;   // lanes past K hold no atom
    const int f = j / AF, rem = j % AF, i = rem / 4, r = rem % 4, l = tid & 63;
    const int t = (tid >> 6) * TPW + i, tp = t / NT16, tq = t % NT16;
    return f * K + (16 * tq + (l & 15)) * N + 16 * tp + (l >> 4) + 4 * r;
  }
  __device__ static int owner(int a) {
    if constexpr (SMALL) return a % K;
    const int q = (a % K) / N, p = a % N, t = (p / 16) * NT16 + q / 16;
    return 64 * (t / TPW) + 16 * ((p % 16) % 4) + q % 16;
  }
  __device__ static int slot(int a) {
    if constexpr (SMALL) return a / K;
    const int q = (a % K) / N, p = a % N, t = (p / 16) * NT16 + q / 16;
    return (a / K) * AF + 4 * (t % TPW) + (p % 16) / 4;
  }
};

template <int N, int NFAM>
__global__ __launch_bounds__((OmpGeo<N, NFAM>::NT)) void k_omp(const JobDev* __restrict__ jobs, LevelDev lv,
                                             const int32_t* __restrict__ count_ptr, int32_t* next, int32_t lg,
                                             const double* __restrict__ tab, const double* __restrict__ xg,
                                             const double* __restrict__ cbuf, int kcap) {
  using G = OmpGeo<N, NFAM>;
  constexpr int K = G::K, M = G::M, APT = G::APT, AF = G::AF;
  constexpr bool SMALL = G::SMALL;
  constexpr int KC = kOmpMaxAtoms;
  constexpr int NX = NFAM == 2 ? N : 1;
  __shared__ double sX[NX][NX + 1];                    // X[p][p'] = <T_0[p], T_1[p']>
  __shared__ double sT[SMALL ? NFAM : 1][SMALL ? K : 1];
  __shared__ double sY[SMALL ? K : 1];
  // L = chol(G_SS)^-1, lower triangular, kcap x (kcap + 1) doubles sized at
  // launch by the largest k of the level (smaller k: more workgroups per CU)
  extern __shared__ double sLdyn[];
  const int ldl = kcap + 1;
  __shared__ int sS[KC];                               // selected atoms in order
  __shared__ double sXc[KC], sG[KC], sW[KC];           // x_S, g, w
  // the selected atoms split by family, in selection order: p | q << 8 and x
  __shared__ int sPQ[NFAM][KC];
  __shared__ double sXF[NFAM][KC];
  __shared__ int sNF[NFAM];
  __shared__ double sBc[2][8];                         // per-wave best c
  __shared__ int sBi[2][8];
  __shared__ double sScal[2];                          // dependence flag, new ||r||^2
  __shared__ double sRed[2];
  __shared__ int sNode[2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if constexpr (NFAM == 2)
    for (int i = tid; i < K; i += G::NT) sX[i / N][i % N] = xg[i];
  if constexpr (SMALL)
    for (int i = tid; i < NFAM * K; i += G::NT) (&sT[0][0])[i] = tab[i];
  __syncthreads();
  const int count = *count_ptr;
  const int pa = tid % N;                              // p of the thread's atom (N <= 8)
  int ph = 0, np = 0;
  for (;;) {
    if (tid == 0) sNode[np] = atomicAdd(next, 1);
    __syncthreads();
    const int node = sNode[np];
    np ^= 1;
    if (node >= count) break;
    const JobDev& jb = jobs[lv.job[node]];
    const double eps2 = jb.eps2[lg];
    const int kmax = jb.k[lg];
    double e;
    uint8_t st;
    // c: the current correlations <r, phi_a> of the thread's atoms.  Small
    // blocks recompute them from c0 = D^T y each step; larger ones update
    // them in place (see the refresh).
    double c0[SMALL ? APT : 1], c[APT];
    if constexpr (SMALL) {
      // gather (pixel k in thread k), ||y||^2, sum y, first stop test, c0
      double v = 0.0;
      if (tid < K) {
        v = job_pixel(jb, lv.y0[node] + tid / N, lv.x0[node] + tid % N);
        sY[tid] = v;
      }
      if (wv == 0) {
        const double ee = wave_sum_f64(v * v), ss = wave_sum_f64(v);
        if (lane == 0) {
          sRed[0] = ee;
          sRed[1] = ss;
        }
      }
      __syncthreads();
      e = sRed[0];
      const double ssum = sRed[1];
      st = e < eps2 ? ST_ACC : (kmax <= 0 ? ST_SPARSE : ST_RUN);
#pragma unroll
      for (int f = 0; f < APT; ++f) {   // the lane's atom (f, p = tid % N, q = tid / N)
        double acc = 0.0;
        if (tid < K) {
          const int q = tid / N;
#pragma unroll
          for (int y = 0; y < N; ++y) {
            double u = 0.0;
#pragma unroll
            for (int x = 0; x < N; ++x) u = fma(sT[f][q * N + x], sY[y * N + x], u);
            acc = fma(sT[f][pa * N + y], u, acc);
          }
          if (tid == 0) acc = ssum / N;
        }
        c0[f] = acc;
        c[f] = acc;
      }
    } else {
      e = lv.e[node];
      st = lv.st[node];
      const double* cn = cbuf + (size_t)node * M;
#pragma unroll
      for (int j = 0; j < APT; ++j) c[j] = cn[G::atom(tid, j)];
    }
    uint32_t selm = 0;   // bit j: the thread's atom j is selected
    int t = 0;
    while (st == ST_RUN) {
      // (1) arg-max |c| (lowest index on ties); selected atoms hold exact
      // zeros.
      double bc;
      int bj;
      lane_best(c, bc, bj);
      int bi = G::atom(tid, bj);
      if (bi >= M) bi = M;   // threads without atoms (N <= 8) hold c = 0
      wave_best(bc, bi, bc, bi);
      if (lane == 0) {
        sBc[ph][wv] = bc;
        sBi[ph][wv] = bi;
      }
      __syncthreads();
      bc = sBc[ph][0];
      bi = sBi[ph][0];
#pragma unroll
      for (int q = 1; q < G::NT / 64; ++q) {
        const double oc = sBc[ph][q];
        const int oi = sBi[ph][q];
        if (fabs(oc) > fabs(bc) || (fabs(oc) == fabs(bc) && oi < bi)) {
          bc = oc;
          bi = oi;
        }
      }
      ph ^= 1;
      if (bc == 0.0) {
        st = ST_ZERO;
        break;
      }
      // (2)-(5) in wave 0 (t <= 64 lanes), synchronised within the wave:
      // g_r = <phi_{S_r}, phi_i>; w = L g; d = sqrt(1 - w.w);
      // z_t = <y, q_t> = <r, phi_i> / d (q_t, the new orthonormal direction,
      // is phi_i minus its projection on the selected atoms, over d, and r
      // is orthogonal to those); the new row t of L, (-w^T L, 1) / d;
      // x_S = L^T z updated in place, dx = z_t L[t][:] (x_r += dx_r,
      // x_t = dx_t); the selected atoms listed per family with dx (with x
      // for small blocks) for the refresh.
      if (wv == 0) {
        const int fi = bi / K, pi = bi % N, qi = (bi % K) / N;
        const bool act = lane < t;
        int as = bi;
        double g = 0.0;
        if (act) {
          as = sS[lane];
          if constexpr (NFAM == 2) {
            const int fs = as / K, ps = as % N, qs = (as % K) / N;
            if (fs != fi) g = fi == 0 ? sX[pi][ps] * sX[qi][qs] : sX[ps][pi] * sX[qs][qi];
          }
        }
        sG[lane] = g;
        wave_sync();
        double wr = 0.0;
        if (act) {
#pragma unroll 4
          for (int cc = 0; cc <= lane; ++cc) wr = fma(sLdyn[lane * ldl + cc], sG[cc], wr);
        }
        sW[lane] = wr;
        const double s1 = wave_sum_f64(wr * wr);
        const double d2 = 1.0 - s1;
        const bool dep = !(d2 > 1e-24);   // chosen atom (numerically) in the span of the selected ones
        double enew = e;
        if (!dep) {
          const double d = sqrt(d2);
          const double invd = 1.0 / d;
          const double zt = bc / d;
          enew = fma(-zt, zt, e);
          wave_sync();
          double lr = invd, dx = zt * invd, xn = dx;
          if (act) {
            double acc = 0.0;
#pragma unroll 4
            for (int r = lane; r < t; ++r) acc = fma(sW[r], sLdyn[r * ldl + lane], acc);
            lr = -acc * invd;
            dx = zt * lr;
            xn = sXc[lane] + dx;
          }
          const bool in = lane <= t;
          if (in) {
            sLdyn[t * ldl + lane] = lr;
            sXc[lane] = xn;
          }
          if (lane == 0) {
            sS[t] = bi;
          }
          if constexpr (NFAM == 2) {
            const int f = as / K;
            const unsigned long long m1 = __ballot(in && f == 1), m0 = __ballot(in && f == 0);
            const unsigned long long below = (1ull << lane) - 1ull;
            if (in) {
              const int rk = __popcll((f ? m1 : m0) & below);
              sPQ[f][rk] = (as % N) | (((as % K) / N) << 8);
              sXF[f][rk] = SMALL ? xn : dx;
            }
            if (lane == 0) {
              sNF[0] = __popcll(m0);
              sNF[1] = __popcll(m1);
            }
          }
        }
        if (lane == 0) {
          sScal[0] = dep ? 1.0 : 0.0;
          sScal[1] = enew;
        }
      }
      __syncthreads();
      if (sScal[0] != 0.0) {
        st = ST_ZERO;
        break;
      }
      e = sScal[1];
      if (tid == G::owner(bi)) selm |= 1u << G::slot(bi);
      ++t;
      if (e < eps2)
        st = ST_ACC;
      else if (t >= kmax)
        st = ST_SPARSE;
      if (st != ST_RUN) break;
      // (6) refresh: small blocks c = c0 - G_{:,S} x_S, larger ones
      // c -= G_{:,S} dx (c = c0 - G x at every step either way)
      if constexpr (SMALL) {
#pragma unroll
        for (int f = 0; f < APT; ++f) c[f] = c0[f];
      }
      if constexpr (NFAM == 2 && SMALL) {
        // each of the lane's atoms takes the other family's selections, in
        // selection order, with their current coefficients
        const int qa = tid / N;
        if (tid < K) {
#pragma unroll
          for (int fs = 0; fs < 2; ++fs) {
            const int fa = 1 - fs;
            for (int k = 0; k < sNF[fs]; ++k) {
              const int pq = sPQ[fs][k];
              const int ps = pq & 255, qs = pq >> 8;
              const double g = fs == 0 ? sX[ps][pa] * sX[qs][qa] : sX[pa][ps] * sX[qa][qs];
              c[fa] = fma(-sXF[fs][k], g, c[fa]);
            }
          }
        }
      } else if constexpr (NFAM == 2 && G::MF) {
        // Each family's atoms take the other family's selections, four at a
        // time as one rank-4 FP64 MFMA update per 16 x 16 tile:
        // C[p][q] += A[p][k] B[k][q] with A = -dx_k X(p part), B = X(q part)
        // (lane: A[lane % 16][lane / 16], B[lane / 16][lane % 16]).
        constexpr int TPW = G::TPW, NT16 = G::NT16;
        const int lk = lane >> 4, li = lane & 15;
#pragma unroll
        for (int fs = 0; fs < 2; ++fs) {
          const int ns = sNF[fs];
          const int fa = 1 - fs;   // the family whose atoms change
          for (int kb = 0; kb < ns; kb += 4) {
            const int k = kb + lk;
            const bool ok = k < ns;
            const int pq = ok ? sPQ[fs][k] : 0;
            const double xs = ok ? sXF[fs][k] : 0.0;
            const int ps = pq & 255, qs = pq >> 8;
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
              const int tt = wv * TPW + i, tp = tt / NT16, tq = tt % NT16;
              // family-1 atoms: X[ps][p] X[qs][q]; family-0 atoms: X[p][ps] X[q][qs]
              const double av = -xs * (fs == 0 ? sX[ps][16 * tp + li] : sX[16 * tp + li][ps]);
              const double bv = fs == 0 ? sX[qs][16 * tq + li] : sX[16 * tq + li][qs];
              const int j0 = fa * G::AF + 4 * i;
              d4 cv = d4{c[j0], c[j0 + 1], c[j0 + 2], c[j0 + 3]};
              cv = mfma64(av, bv, cv);
              c[j0] = cv[0];
              c[j0 + 1] = cv[1];
              c[j0 + 2] = cv[2];
              c[j0 + 3] = cv[3];
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < APT; ++j) c[j] = ((selm >> j) & 1u) ? 0.0 : c[j];
    }
    // records: the atoms in selection order with their final coefficients
    if (tid < t) {
      lv.rec_idx[(size_t)node * lv.kmax + tid] = sS[tid];
      lv.rec_coef[(size_t)node * lv.kmax + tid] = sXc[tid];
    }
    if (tid == 0) {
      lv.e[node] = e;
      lv.t[node] = t;
      lv.st[node] = st;
    }
  }
}

}  // namespace

hipError_t launch_gram_init(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t lg, int32_t nfam,
                            const double* tab, double* cbuf, hipStream_t s) {
  if (nfam != 1 && nfam != 2) return hipErrorInvalidValue;
#define AQMP_GINIT(NN, GRID)                                                                                  \
  case NN:                                                                                                    \
    if (nfam == 2)                                                                                            \
      hipLaunchKernelGGL((k_gram_init<NN, 2>), dim3(GRID), dim3(256), 0, s, jobs, lv, count, lg, tab, cbuf); \
    else                                                                                                      \
      hipLaunchKernelGGL((k_gram_init<NN, 1>), dim3(GRID), dim3(256), 0, s, jobs, lv, count, lg, tab, cbuf); \
    break;
  switch (n) {
    AQMP_GINIT(16, 2048)
    AQMP_GINIT(32, 1024)
    AQMP_GINIT(64, 512)
    default:
      return hipErrorInvalidValue;
  }
#undef AQMP_GINIT
  return hipGetLastError();
}

hipError_t launch_gram_pursuit(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next, int32_t lg,
                               int32_t nfam, const double* tab, const double* xg, const double* cbuf, hipStream_t s) {
  if (nfam == 2 && !xg) return hipErrorInvalidValue;
  if (nfam != 1 && nfam != 2) return hipErrorInvalidValue;
#define AQMP_GSMALL(NN, GRID)                                                                                  \
  case NN:                                                                                                     \
    if (nfam == 2)                                                                                             \
      hipLaunchKernelGGL((k_gram_small<NN, 2>), dim3(GRID), dim3(256), 0, s, jobs, lv, count, lg, tab, xg);   \
    else                                                                                                       \
      hipLaunchKernelGGL((k_gram_small<NN, 1>), dim3(GRID), dim3(256), 0, s, jobs, lv, count, lg, tab, xg);   \
    break;
#define AQMP_GPUR(NN, GRID)                                                                                    \
  case NN:                                                                                                     \
    if (nfam == 2)                                                                                             \
      hipLaunchKernelGGL((k_gram_pursuit<NN, 2>), dim3(GRID), dim3(256), 0, s, jobs, lv, count, next, lg, xg, \
                         cbuf);                                                                                \
    else                                                                                                       \
      hipLaunchKernelGGL((k_gram_pursuit<NN, 1>), dim3(GRID), dim3(256), 0, s, jobs, lv, count, next, lg, xg, \
                         cbuf);                                                                                \
    break;
  switch (n) {
    AQMP_GSMALL(4, 1024)
    AQMP_GSMALL(8, 2048)
    AQMP_GPUR(16, 2048)
    AQMP_GPUR(32, 2048)
    AQMP_GPUR(64, 1024)
    default:
      return hipErrorInvalidValue;
  }
#undef AQMP_GSMALL
#undef AQMP_GPUR
  return hipGetLastError();
}

hipError_t launch_omp_pursuit(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next, int32_t lg,
                              int32_t nfam, const double* tab, const double* xg, const double* cbuf, int32_t kmax,
                              hipStream_t s) {
  if (nfam == 2 && !xg) return hipErrorInvalidValue;
  if (nfam != 1 && nfam != 2) return hipErrorInvalidValue;
  if (kmax > kOmpMaxAtoms) return hipErrorInvalidValue;
  const int kcap = kmax < 1 ? 1 : kmax;
  int dev = 0, n_cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t smem = sizeof(double) * (size_t)kcap * (kcap + 1);
  // Nodes come from a counter, so the grid is as many workgroups as fit on
  // the device at once (registers and LDS decide; more would only start
  // after the work is gone).
#define AQMP_OMP_F(NN, FF)                                                                                     \
  {                                                                                                            \
    int per_cu = 0;                                                                                            \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_omp<NN, FF>, OmpGeo<NN, FF>::NT, smem) !=     \
            hipSuccess ||                                                                                      \
        per_cu < 1)                                                                                            \
      per_cu = 1;                                                                                              \
    hipLaunchKernelGGL((k_omp<NN, FF>), dim3(n_cus * per_cu), dim3(OmpGeo<NN, FF>::NT), smem, s, jobs, lv,  \
                       count, next, lg, tab, xg, cbuf, kcap);                                                  \
  }
#define AQMP_OMP(NN)             \
  case NN:                       \
    if (nfam == 2)               \
      AQMP_OMP_F(NN, 2)          \
    else                         \
      AQMP_OMP_F(NN, 1)          \
    break;
  switch (n) {
    AQMP_OMP(4)
    AQMP_OMP(8)
    AQMP_OMP(16)
    AQMP_OMP(32)
    AQMP_OMP(64)
    default:
      return hipErrorInvalidValue;
  }
#undef AQMP_OMP
#undef AQMP_OMP_F
  return hipGetLastError();
}

}  // namespace aqmp
