// kernels_fused.hip - whole-level Matching Pursuit for small blocks: the dense
// FP64 pursuit (N <= 8, the FP32 form and N = 4), and the BF16 MFMA pursuits
// of the BF16 form at N = 8 and N = 16.
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
    double r = job_pixel(jb, lv.y0[nd] + y, lv.x0[nd] + x);
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

// ---------------------------------------------------------------------------
// Whole-level pursuit for N = 16 in the BF16 form.  At N = 16 one MP step of
// a node is 262 K multiply-adds: a batched launch per step is mostly launch
// latency and dependent memory chains.  One workgroup takes 32 nodes through
// their whole pursuit (Section 2.2 steps (a)-(d), eq. (2)) with every array
// in LDS:
//   C   correlation of all 512 atoms with the 32 BF16 residuals by MFMA
//       (32x32x16, FP32 accumulation, pixel order as in the batched kernels);
//       the A operand is generated in registers from the FP32 1D tables,
//       bf16(T32_f[p][y] * T32_f[q][x]), the canonical BF16 atom;
//   E   each wave keeps, per node, the best 8 keys of its 128 atoms
//       (branch-free sorting networks, as in the batched epilogue);
//   M   the four wave lists are merged into the node's 8 candidates, ordered
//       by (|c| key, lower atom), the same ranking as the batched path;
//   S   one thread per (node, candidate) re-scores in FP64 against the FP32
//       residual, separably (Section 2.1 outer product);
//   A   arg-max (lowest atom on ties), rank-1 update in FP64 rounded to FP32,
//       ||r||^2 in FP64, record (i, c_i), stop test of eq. (2).
// Up to 32 MP steps run inside the kernel; a node that stops keeps its slot
// (its correlation is still computed, its state no longer changes).
// ---------------------------------------------------------------------------
constexpr int kP16N = 16, kP16K = 256, kP16G = 32;   // block size, pixels, nodes per workgroup
constexpr int kP8Nodes = 16;                          // nodes per wave of the N = 8 BF16 pursuit
constexpr int kP16RS = kP16K + 4;                     // padded FP32 residual row (floats)
constexpr int kP16AC = 3;                             // A tiles whose fragments stay in registers

typedef __bf16 p16_bf16x8 __attribute__((ext_vector_type(8)));
typedef float p16_f32x16 __attribute__((ext_vector_type(16)));

__device__ inline void p16_cx(uint32_t& a, uint32_t& b) {
  const uint32_t hi = a > b ? a : b;
  b = a > b ? b : a;
  a = hi;
}
__device__ inline void p16_sort8(uint32_t (&v)[8]) {
  p16_cx(v[0], v[1]); p16_cx(v[2], v[3]); p16_cx(v[4], v[5]); p16_cx(v[6], v[7]);
  p16_cx(v[0], v[2]); p16_cx(v[1], v[3]); p16_cx(v[4], v[6]); p16_cx(v[5], v[7]);
  p16_cx(v[1], v[2]); p16_cx(v[5], v[6]);
  p16_cx(v[0], v[4]); p16_cx(v[1], v[5]); p16_cx(v[2], v[6]); p16_cx(v[3], v[7]);
  p16_cx(v[2], v[4]); p16_cx(v[3], v[5]);
  p16_cx(v[1], v[2]); p16_cx(v[3], v[4]); p16_cx(v[5], v[6]);
}
template <class T>
__device__ inline void p16_cxT(T& a, T& b) {
  const T hi = a > b ? a : b;
  b = a > b ? b : a;
  a = hi;
}
// a, b descending -> a = top 8 of both, descending (bitonic merge)
template <class T>
__device__ inline void p16_merge8(T (&a)[8], const T (&b)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = a[i] > b[7 - i] ? a[i] : b[7 - i];
  p16_cxT(a[0], a[4]); p16_cxT(a[1], a[5]); p16_cxT(a[2], a[6]); p16_cxT(a[3], a[7]);
  p16_cxT(a[0], a[2]); p16_cxT(a[1], a[3]); p16_cxT(a[4], a[6]); p16_cxT(a[5], a[7]);
  p16_cxT(a[0], a[1]); p16_cxT(a[2], a[3]); p16_cxT(a[4], a[5]); p16_cxT(a[6], a[7]);
}

// 16-byte chunk c (8 pixels) of node row nl in the swizzled BF16 residual.
__device__ inline int p16_chunk(int nl, int c) { return nl * 32 + (c ^ (nl & 15)); }

__global__ __launch_bounds__(256, 1) void k_pursuit16_bf16(const JobDev* __restrict__ jobs, LevelDev lv,
                                                           const int32_t* __restrict__ count_ptr, int32_t lg,
                                                           int32_t n_atoms, int32_t nfam,
                                                           const double* __restrict__ tab,
                                                           const float* __restrict__ tabT32) {
  constexpr int N = kP16N, K = kP16K, G = kP16G;
  __shared__ __attribute__((aligned(16))) float sR[G][kP16RS];   // FP32 residual
  __shared__ __attribute__((aligned(16))) uint4 sB[G * 32];  // BF16 residual, 32 chunks per node
  __shared__ __attribute__((aligned(16))) double sTab[2][N][N];  // FP64 tables [f][p][y]
  __shared__ float sT32[2][N][N];                            // FP32 tables [f][y][p]
  __shared__ uint32_t sKey[4][G][8];
  __shared__ __attribute__((aligned(16))) int sCand[G][8];
  __shared__ __attribute__((aligned(16))) double sC[G][8];
  __shared__ double sE[G], sEps[G];
  __shared__ int sSt[G], sT[G], sKmax[G];
  // records of the current 32-step window, flushed to global after it
  constexpr int RW = 32;
  __shared__ int sRecIdx[G][RW];
  __shared__ double sRecCoef[G][RW];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < nfam * K; i += 256) {
    (&sTab[0][0][0])[i] = tab[i];
    (&sT32[0][0][0])[i] = tabT32[i];
  }
  __syncthreads();
  const double inv_n = 1.0 / N;
  const int count = *count_ptr;

  // Correlation geometry: wave w holds atoms [128 w, 128 w + 128); lane row
  // 32 ma + rr is atom (fam, p = rr & 15, q = 8 (w & 1) + 2 ma + (rr >> 4)).
  const int rr = lane & 31, hh = lane >> 5;
  const int fam = min(w >> 1, nfam - 1);
  const bool fam_ok = (w >> 1) < nfam;
  float tq[4][8];
#pragma unroll
  for (int ma = 0; ma < 4; ++ma) {
    const int q = 8 * (w & 1) + 2 * ma + (rr >> 4);
#pragma unroll
    for (int j = 0; j < 8; ++j) tq[ma][j] = sT32[fam][8 * hh + j][q];
  }
  const float* tpcol = &sT32[fam][0][rr & 15];   // T32_f[p][y] at tpcol[y * N]
  // The A fragments do not change between steps or groups: those of the
  // first kP16AC tiles are generated once and held in registers, the others
  // each step.
  constexpr int AC = kP16AC;
  p16_bf16x8 afc[N][AC];
#pragma unroll
  for (int kk = 0; kk < N; ++kk) {
    const float tpk = tpcol[kk * N];
#pragma unroll
    for (int ma = 0; ma < AC; ++ma)
#pragma unroll
      for (int j = 0; j < 8; ++j) afc[kk][ma][j] = (__bf16)(tpk * tq[ma][j]);
  }
  // Keys: the 23 bits of |c| that the batched path ranks on (exponent and 15
  // mantissa bits), then 511 - atom: the same order as its 64-bit keys.
  // 511 - atom of accumulator (ma, r) = lb - (32 ma + 8 (r >> 2) + (r & 3)).
  const uint32_t lb = 511u - (uint32_t)(128 * w + 4 * hh);

  // Update / gather geometry: thread = (node nl, part): 32 pixels, rows 2 part, 2 part + 1.
  const int nl = tid >> 3, part = tid & 7;

  for (int g0 = blockIdx.x * G; g0 < count; g0 += gridDim.x * G) {
    // ---- gather (Algorithm 2: y = unravel(b)) and the first stop test ----
    {
      const int node = g0 + nl;
      const bool valid = node < count;
      const int nd = valid ? node : g0;
      const JobDev& jb = jobs[lv.job[nd]];
      const int bx = lv.x0[nd], by = lv.y0[nd];
      double e = 0.0;
      const JobDev jl = jb;   // one copy of the job's fields in registers
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
        const int y = 2 * part + dy;
        float f[N];
        double pv[N];
        job_pixels<N>(jl, by + y, bx, pv);
#pragma unroll
        for (int x = 0; x < N; ++x) {
          const double v = pv[x];
          f[x] = (float)v;
          e += v * v;
        }
#pragma unroll
        for (int x = 0; x < N; ++x) sR[nl][y * N + x] = valid ? f[x] : 0.f;
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
          p16_bf16x8 b;
#pragma unroll
          for (int j = 0; j < 8; ++j) b[j] = (__bf16)(valid ? f[8 * c2 + j] : 0.f);
          sB[p16_chunk(nl, 2 * y + c2)] = __builtin_bit_cast(uint4, b);
        }
      }
      e += __shfl_xor(e, 1, 64);
      e += __shfl_xor(e, 2, 64);
      e += __shfl_xor(e, 4, 64);
      if (part == 0) {
        uint8_t st = ST_RUN;
        if (!valid)
          st = ST_SPARSE;
        else if (e < jb.eps2[lg])
          st = ST_ACC;
        else if (jb.k[lg] <= 0)
          st = ST_SPARSE;
        sE[nl] = e;
        sEps[nl] = jb.eps2[lg];
        sKmax[nl] = jb.k[lg];
        sT[nl] = 0;
        sSt[nl] = st;
      }
    }
    bool any = __syncthreads_or(part == 0 && sSt[nl] == ST_RUN);
    int step = 0;   // MP steps made in this group (every running node makes one per step)

    while (any) {
      // ---- C: correlation (MFMA) ----
      p16_f32x16 acc[4];
#pragma unroll
      for (int ma = 0; ma < 4; ++ma)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[ma][r] = 0.f;
#pragma unroll
      for (int kk = 0; kk < N; ++kk) {   // k-step kk = pixel row y
        const p16_bf16x8 bf = __builtin_bit_cast(p16_bf16x8, sB[p16_chunk(rr, 2 * kk + hh)]);
        const float tpk = tpcol[kk * N];
#pragma unroll
        for (int ma = 0; ma < 4; ++ma) {
          p16_bf16x8 af;
          if (ma < AC) {
            af = afc[kk][ma < AC ? ma : 0];
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) af[j] = (__bf16)(tpk * tq[ma][j]);
          }
          acc[ma] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf, acc[ma], 0, 0, 0);
        }
      }
      // ---- E: this wave's best 8 keys per node (node = rr) ----
      {
        uint32_t top[8];
#pragma unroll
        for (int gi = 0; gi < 8; ++gi) {
          const int ma = gi >> 1;
          uint32_t v[8];
#pragma unroll
          for (int e8 = 0; e8 < 8; ++e8) {
            const int r = 8 * (gi & 1) + e8;
            const uint32_t bits = __float_as_uint(acc[ma][r]);
            v[e8] = ((bits & 0x7FFFFF00u) << 1) | (lb - (uint32_t)(32 * ma + 8 * (r >> 2) + (r & 3)));
          }
          p16_sort8(v);
          if (gi == 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) top[j] = v[j];
          } else {
            p16_merge8(top, v);
          }
        }
        uint32_t other[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) other[j] = __shfl_xor(top[j], 32, 64);
        p16_merge8(top, other);
        if (lane < 32) {
#pragma unroll
          for (int j = 0; j < 8; ++j) sKey[w][rr][j] = fam_ok ? top[j] : 0u;
        }
      }
      __syncthreads();
      // ---- M: the node's 8 candidates (wave 0: lane half hh merges waves 2 hh, 2 hh + 1) ----
      if (w == 0) {
        uint32_t top[8], v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          top[j] = sKey[2 * hh][rr][j];
          v[j] = sKey[2 * hh + 1][rr][j];
        }
        p16_merge8(top, v);
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = __shfl_xor(top[j], 32, 64);
        p16_merge8(top, v);
        if (lane < 32) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const unsigned atom = 511u - (top[j] & 0x1FFu);
            sCand[rr][j] = (top[j] != 0u && atom < (unsigned)n_atoms) ? (int)atom : -1;
          }
        }
      }
      __syncthreads();
      // ---- S: FP64 re-score, thread = (node nl, candidate part) ----
      {
        const int atom = sCand[nl][part];
        double c = 0.0;
        if (sSt[nl] == ST_RUN && atom >= 0) {
          const int f = atom / K, q = (atom % K) / N, p = atom % N;
          const bool dc = (p == 0 && q == 0);
          double tqx[N], tpy[N];
          const double2* qrow = (const double2*)&sTab[f][q][0];
          const double2* prow = (const double2*)&sTab[f][p][0];
#pragma unroll
          for (int i = 0; i < N / 2; ++i) {
            const double2 u = qrow[i], v = prow[i];
            tqx[2 * i] = dc ? 1.0 : u.x;
            tqx[2 * i + 1] = dc ? 1.0 : u.y;
            tpy[2 * i] = v.x;
            tpy[2 * i + 1] = v.y;
          }
          const float4* rrow = (const float4*)&sR[nl][0];
#pragma unroll 4
          for (int y = 0; y < N; ++y) {
            float rv[N];
#pragma unroll
            for (int i = 0; i < N / 4; ++i) {
              const float4 t4 = rrow[y * (N / 4) + i];
              rv[4 * i] = t4.x; rv[4 * i + 1] = t4.y; rv[4 * i + 2] = t4.z; rv[4 * i + 3] = t4.w;
            }
            double sum = 0.0;
#pragma unroll
            for (int x = 0; x < N; ++x) sum = fma((double)rv[x], tqx[x], sum);
            c = dc ? c + sum : fma(tpy[y], sum, c);
          }
          if (dc) c *= inv_n;
        }
        sC[nl][part] = c;
      }
      __syncthreads();
      // ---- A: arg-max, update, norm, record, stop test ----
      {
        const bool run = sSt[nl] == ST_RUN;
        int cd[8];
        double cv[8];
        {
          const int4* cp = (const int4*)&sCand[nl][0];
          const double2* vp = (const double2*)&sC[nl][0];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int4 t4 = cp[i];
            cd[4 * i] = t4.x; cd[4 * i + 1] = t4.y; cd[4 * i + 2] = t4.z; cd[4 * i + 3] = t4.w;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double2 t2 = vp[i];
            cv[2 * i] = t2.x; cv[2 * i + 1] = t2.y;
          }
        }
        // arg-max |c| over the valid candidates, lowest atom on ties
        int batom = -1;
        double bmag = -1.0, bc = 0.0;
#pragma unroll
        for (int ci = 0; ci < 8; ++ci) {
          const double m = fabs(cv[ci]);
          const bool better = cd[ci] >= 0 && (batom < 0 || m > bmag || (m == bmag && cd[ci] < batom));
          batom = better ? cd[ci] : batom;
          bmag = better ? m : bmag;
          bc = better ? cv[ci] : bc;
        }
        const bool zero = (batom < 0 || bmag == 0.0);
        const int atom = zero ? 0 : batom;
        const double coef = zero ? 0.0 : bc;
        double e = 0.0;
        if (run && !zero) {
          const int f = atom / K, q = (atom % K) / N, p = atom % N;
          const bool dc = (p == 0 && q == 0);
          double tqx[N];
          const double2* qrow = (const double2*)&sTab[f][q][0];
#pragma unroll
          for (int i = 0; i < N / 2; ++i) {
            const double2 u = qrow[i];
            tqx[2 * i] = u.x;
            tqx[2 * i + 1] = u.y;
          }
          float rv[2][N];
          float4* rrow = (float4*)&sR[nl][0];
#pragma unroll
          for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int i = 0; i < N / 4; ++i) {
              const float4 t4 = rrow[(2 * part + dy) * (N / 4) + i];
              rv[dy][4 * i] = t4.x; rv[dy][4 * i + 1] = t4.y; rv[dy][4 * i + 2] = t4.z; rv[dy][4 * i + 3] = t4.w;
            }
          double eh[2] = {0.0, 0.0};
#pragma unroll
          for (int dy = 0; dy < 2; ++dy) {
            const int y = 2 * part + dy;
            const double ty = sTab[f][p][y];
            float rn[N];
#pragma unroll
            for (int x = 0; x < N; ++x) {
              const double phi = dc ? inv_n : ty * tqx[x];
              rn[x] = (float)fma(-coef, phi, (double)rv[dy][x]);
              eh[dy] = fma((double)rn[x], (double)rn[x], eh[dy]);
            }
#pragma unroll
            for (int i = 0; i < N / 4; ++i) rrow[y * (N / 4) + i] = make_float4(rn[4 * i], rn[4 * i + 1], rn[4 * i + 2], rn[4 * i + 3]);
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2) {
              p16_bf16x8 b;
#pragma unroll
              for (int j = 0; j < 8; ++j) b[j] = (__bf16)rn[8 * c2 + j];
              sB[p16_chunk(nl, 2 * y + c2)] = __builtin_bit_cast(uint4, b);
            }
          }
          e = eh[0] + eh[1];
        }
        e += __shfl_xor(e, 1, 64);
        e += __shfl_xor(e, 2, 64);
        e += __shfl_xor(e, 4, 64);
        bool still = false;
        if (part == 0 && run) {
          const int t = sT[nl];
          if (zero) {
            sSt[nl] = ST_ZERO;
          } else {
            sRecIdx[nl][t % RW] = atom;
            sRecCoef[nl][t % RW] = coef;
            uint8_t st = ST_RUN;
            if (e < sEps[nl])
              st = ST_ACC;
            else if (t + 1 >= sKmax[nl])
              st = ST_SPARSE;
            sE[nl] = e;
            sT[nl] = t + 1;
            sSt[nl] = st;
            still = st == ST_RUN;
          }
        }
        any = __syncthreads_or(still);
        // every RW steps (all running nodes share the step count) and at the
        // end, the window's records go to global memory
        ++step;
        if (step % RW == 0 || !any) {
          const int base = (step - 1) / RW * RW;
          for (int i = tid; i < G * RW; i += 256) {
            const int n2 = i / RW, j = i % RW, ts = base + j;
            if (g0 + n2 < count && ts < sT[n2]) {
              const size_t slot = (size_t)(g0 + n2) * lv.kmax + ts;
              lv.rec_idx[slot] = sRecIdx[n2][j];
              lv.rec_coef[slot] = sRecCoef[n2][j];
            }
          }
          __syncthreads();
        }
      }
    }
    // ---- node state for the split test ----
    if (tid < G && g0 + tid < count) {
      lv.e[g0 + tid] = sE[tid];
      lv.t[g0 + tid] = sT[tid];
      lv.st[g0 + tid] = (uint8_t)sSt[tid];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Whole-level pursuit for N = 8 in the BF16 form.  One wave takes G <= 16
// nodes through their whole pursuit (Section 2.2 steps (a)-(d), eq. (2)),
// with no workgroup barrier: the waves of a workgroup are independent.
// Lane l serves node l % 16 and holds rows 2 (l / 16), 2 (l / 16) + 1 of its
// FP32 residual in registers for the whole pursuit.
//   C  correlation of all M <= 128 atoms with the G BF16 residuals by
//      v_mfma_f32_16x16x32_bf16 (A = 16 atoms x 32 pixels, B = 32 pixels x
//      16 nodes, FP32 accumulation; output row 4 (l / 16) + r, column
//      l % 16).  The BF16 atoms never change, so the wave builds all 16 A
//      fragments (8 atom tiles x 2 pixel halves) once, in registers: atom
//      a = 16 ma + row, family a / 64, q = (a % 64) / 8, p = a % 8, value
//      bf16(fl32(T_f[p][y]) fl32(T_f[q][x])), constant atom exactly 1/8.  The
//      B fragments (BF16 residual rows) go through LDS;
//   E  each lane ranks the 32 correlations it holds of its node (4 per atom
//      tile) as 32-bit keys (|c| bits, then 127 - atom: a larger key is a
//      larger |c|, then the lower atom), keeps its best 8 with sorting
//      networks and merges them with the node's other three lanes;
//   S  FP64 re-score of the 8 candidates: each lane sums over its own 16
//      pixels (sum_y T[p][y] sum_x r[y][x] T[q][x], the table rows read from
//      LDS in one batch), then the node's four lanes add their partials;
//   A  arg-max (lowest atom on ties), rank-1 update of the lane's pixels in
//      FP64 rounded to FP32, ||r||^2 in FP64, record (i, c_i) straight to
//      memory, stop test.
// ---------------------------------------------------------------------------
typedef __bf16 p8_bf16x8 __attribute__((ext_vector_type(8)));
typedef float p8_f32x4 __attribute__((ext_vector_type(4)));

// Sum over the four lanes l % 16 + 16 j of a node (a fixed order: the
// partner 16 lanes away, then the partner 32 lanes away).
__device__ inline double quad_sum(double v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

template <int G>
__global__ __launch_bounds__(256) void k_pursuit8_bf16(const JobDev* __restrict__ jobs, LevelDev lv,
                                                       const int32_t* __restrict__ count_ptr, int32_t n_atoms,
                                                       int32_t nfam, const double* __restrict__ tab,
                                                       const float* __restrict__ tabT32) {
  constexpr int N = 8, K = 64;
  static_assert(G >= 1 && G <= 16, "at most 16 nodes per wave (the B operand's columns)");
  __shared__ __attribute__((aligned(16))) double sTab[2][N][N];   // [f][p][y] FP64
  __shared__ float sT32[2][N][N];                                 // [f][y][p] FP32
  __shared__ __attribute__((aligned(16))) uint4 sB[4][N][16];     // BF16 residual rows [wave][row][node]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < nfam * K; i += 256) {
    (&sTab[0][0][0])[i] = tab[i];
    (&sT32[0][0][0])[i] = tabT32[i];
  }
  __syncthreads();
  const int count = *count_ptr;
  const int c = lane & 15, quad = lane >> 4;      // node column, lane group of the node
  const int y0 = 2 * quad;                        // the lane's rows y0, y0 + 1
  const double inv_n = 1.0 / N;

  // A fragments: tile ma (16 atoms), pixel half kh (rows 4 kh .. 4 kh + 3).
  p8_bf16x8 afr[8][2];
#pragma unroll
  for (int ma = 0; ma < 8; ++ma) {
    const int a = 16 * ma + c;
    const int f = a / K, q = (a % K) / N, p = a % N;
    const bool ok = a < n_atoms;
    const int ff = ok ? f : 0;
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      const int y = 4 * kh + quad;
      const float tpy = sT32[ff][y][p];
      p8_bf16x8 v;
#pragma unroll
      for (int x = 0; x < N; ++x) {
        const float prod = (p == 0 && q == 0) ? 0.125f : tpy * sT32[ff][x][q];
        v[x] = (__bf16)(ok ? prod : 0.f);
      }
      afr[ma][kh] = v;
    }
  }
  // atom of accumulator element r of tile ma: 16 ma + 4 quad + r
  const uint32_t kb = 127u - (uint32_t)(4 * quad);

  const int ngroups = (count + G - 1) / G;
  for (int grp = blockIdx.x * 4 + w; grp < ngroups; grp += gridDim.x * 4) {
    const int g0 = grp * G;
    const int node = g0 + c;
    const bool mine = c < G && node < count;      // a real node behind this lane's column
    // ---- gather (Algorithm 2: y = unravel(b)), the lane's two rows ----
    float rr[2][N];
    double eps2 = 0.0, e = 0.0;
    int kmax = 0, t = 0;
    uint8_t st = ST_SPARSE;
    {
      const int nd = mine ? node : g0;
      const JobDev& jb = jobs[lv.job[nd]];
      const int bx = lv.x0[nd], by = lv.y0[nd];
      double ep = 0.0;
      const JobDev jl = jb;   // one copy of the job's fields in registers
      double pv[2][N];
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) job_pixels<N>(jl, by + y0 + dy, bx, pv[dy]);
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
        p8_bf16x8 b;
#pragma unroll
        for (int x = 0; x < N; ++x) {
          const double v = mine ? pv[dy][x] : 0.0;
          rr[dy][x] = (float)v;
          ep += v * v;
          b[x] = (__bf16)rr[dy][x];
        }
        sB[w][y0 + dy][c] = __builtin_bit_cast(uint4, b);
      }
      e = quad_sum(ep);
      eps2 = jb.eps2[3];
      kmax = jb.k[3];
      if (mine) st = e < eps2 ? ST_ACC : (kmax <= 0 ? ST_SPARSE : ST_RUN);
    }
    wave_sync();
    while (__ballot(st == ST_RUN) != 0ull) {
      // ---- C: correlation of every atom with the G residuals ----
      p8_f32x4 acc[8];
#pragma unroll
      for (int ma = 0; ma < 8; ++ma) acc[ma] = p8_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kh = 0; kh < 2; ++kh) {
        const p8_bf16x8 bf = __builtin_bit_cast(p8_bf16x8, sB[w][4 * kh + quad][c]);
#pragma unroll
        for (int ma = 0; ma < 8; ++ma)
          acc[ma] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[ma][kh], bf, acc[ma], 0, 0, 0);
      }
      // ---- E: the node's best 8 keys ----
      uint32_t top[8];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        uint32_t v[8];
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) {
          const int ma = 2 * g + (e8 >> 2), r = e8 & 3;
          const uint32_t bits = __float_as_uint(acc[ma][r]) & 0x7FFFFF80u;
          const uint32_t atom_low = kb - (uint32_t)(16 * ma + r);     // 127 - atom
          v[e8] = (16 * ma + 4 * quad + r < n_atoms) ? (bits | atom_low) : 0u;
        }
        p16_sort8(v);
        if (g == 0) {
#pragma unroll
          for (int j = 0; j < 8; ++j) top[j] = v[j];
        } else {
          p16_merge8(top, v);
        }
      }
#pragma unroll
      for (int sh = 16; sh <= 32; sh <<= 1) {
        uint32_t o[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = __shfl_xor(top[j], sh, 64);
        p16_merge8(top, o);
      }
      // ---- S: FP64 re-score of the 8 candidates on the lane's 16 pixels ----
      double rd[2][N];
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int x = 0; x < N; ++x) rd[dy][x] = (double)rr[dy][x];
      int cand[8];
      double cv[8];
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        // table rows of four candidates, read before any arithmetic
        double tq[4][N], tp[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = 4 * half + i;
          const int at = top[j] != 0u ? (int)(127u - (top[j] & 0x7Fu)) : -1;
          cand[j] = at;
          const int aa = at < 0 ? 0 : at;
          const int f = aa / K, q = (aa % K) / N, p = aa % N;
          const double2* qr = (const double2*)&sTab[f][q][0];
#pragma unroll
          for (int x2 = 0; x2 < N / 2; ++x2) {
            const double2 u = qr[x2];
            tq[i][2 * x2] = u.x;
            tq[i][2 * x2 + 1] = u.y;
          }
          const double2 pr = *(const double2*)&sTab[f][p][y0];
          tp[i][0] = pr.x;
          tp[i][1] = pr.y;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = 4 * half + i;
          const int aa = cand[j] < 0 ? 0 : cand[j];
          const bool dc = (aa % K) == 0;            // p = q = 0: the constant atom
          double part = 0.0;
#pragma unroll
          for (int dy = 0; dy < 2; ++dy) {
            double sx = 0.0;
#pragma unroll
            for (int x = 0; x < N; ++x) sx = fma(rd[dy][x], dc ? 1.0 : tq[i][x], sx);
            part = dc ? part + sx : fma(tp[i][dy], sx, part);
          }
          cv[j] = dc ? part * inv_n : part;
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) cv[j] = quad_sum(cv[j]);
      // ---- A: arg-max (lowest atom on ties), update, norm, record, stop ----
      int best = -1;
      double bmag = -1.0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double m = fabs(cv[j]);
        const bool better = cand[j] >= 0 && (best < 0 || m > bmag || (m == bmag && cand[j] < cand[best < 0 ? 0 : best]));
        if (better) {
          best = j;
          bmag = m;
        }
      }
      const bool zero = best < 0 || bmag == 0.0;
      int atom = 0;
      double coef = 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j == best) {
          atom = cand[j];
          coef = cv[j];
        }
      const bool run = st == ST_RUN;
      double en = 0.0;
      if (run && !zero) {
        const int f = atom / K, q = (atom % K) / N, p = atom % N;
        const bool dc = (p == 0 && q == 0);
        double tqx[N];
        const double2* qr = (const double2*)&sTab[f][q][0];
#pragma unroll
        for (int x2 = 0; x2 < N / 2; ++x2) {
          const double2 u = qr[x2];
          tqx[2 * x2] = u.x;
          tqx[2 * x2 + 1] = u.y;
        }
        const double2 pr = *(const double2*)&sTab[f][p][y0];
        const double tpy[2] = {pr.x, pr.y};
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          p8_bf16x8 b;
#pragma unroll
          for (int x = 0; x < N; ++x) {
            const double phi = dc ? inv_n : tpy[dy] * tqx[x];
            rr[dy][x] = (float)fma(-coef, phi, rd[dy][x]);
            en = fma((double)rr[dy][x], (double)rr[dy][x], en);
            b[x] = (__bf16)rr[dy][x];
          }
          sB[w][y0 + dy][c] = __builtin_bit_cast(uint4, b);
        }
      }
      en = quad_sum(en);
      if (run) {
        if (zero) {
          st = ST_ZERO;
        } else {
          if (quad == 0) {
            const size_t slot = (size_t)node * lv.kmax + t;
            lv.rec_idx[slot] = atom;
            lv.rec_coef[slot] = coef;
          }
          e = en;
          ++t;
          st = e < eps2 ? ST_ACC : (t >= kmax ? ST_SPARSE : ST_RUN);
        }
      }
      wave_sync();   // the new BF16 rows are in LDS before the next correlation reads them
    }
    if (mine && quad == 0) {
      lv.e[node] = e;
      lv.t[node] = t;
      lv.st[node] = st;
    }
    wave_sync();   // the next group overwrites this group's rows
  }
}

}  // namespace

hipError_t launch_pursuit16_bf16(const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t n_atoms, int32_t nfam,
                                 const double* tab, const float* tabT32, hipStream_t s) {
  hipLaunchKernelGGL(k_pursuit16_bf16, dim3(512), dim3(256), 0, s, jobs, lv, count, 4, n_atoms, nfam, tab, tabT32);
  return hipGetLastError();
}

hipError_t launch_pursuit8_bf16(const JobDev* jobs, LevelDev lv, const int32_t* count, int64_t cap, int32_t n_atoms,
                                int32_t nfam, const double* tab, const float* tabT32, hipStream_t s) {
  constexpr int G = kP8Nodes;
  int64_t groups = (cap + G - 1) / G;
  int64_t wgs = (groups + 3) / 4;
  if (wgs > 4096) wgs = 4096;
  if (wgs < 1) wgs = 1;
  hipLaunchKernelGGL(k_pursuit8_bf16<G>, dim3((unsigned)wgs), dim3(256), 0, s, jobs, lv, count, n_atoms, nfam, tab,
                     tabT32);
  return hipGetLastError();
}

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
