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
// a node is 131 K multiply-adds: a batched launch per step would be mostly
// launch latency and dependent memory chains.  Here one workgroup of eight
// waves runs 16 node slots through their whole pursuits (Section 2.2 steps
// (a)-(d), eq. (2)) with every array in LDS or registers:
//   C  correlation of all 512 atoms with the 16 BF16 residuals by
//      v_mfma_f32_16x16x32_bf16 (A = 16 atoms x 32 pixels, B = 32 pixels x
//      16 slots, FP32 accumulation, pixel order as in the batched kernels).
//      Wave w holds atoms f = w / 4, q = 4 (w % 4) + ma (ma < 4), all p: the
//      canonical BF16 atoms bf16(T32_f[p][y] T32_f[q][x]), generated once
//      per kernel into registers (32 fragments);
//   E  each lane ranks its 16 correlations of one slot as 32-bit keys (|c|
//      bits, then 511 - atom), keeps the best 8 with sorting networks and
//      merges them with the slot's other three lanes of the wave;
//   M  the slot's eight wave lists are merged into its 8 candidates (the
//      same ranking as the batched path);
//   S  FP64 re-score of the candidates against the FP32 residual,
//      separably (Section 2.1 outer product): a slot is one DPP row of 16
//      lanes, lane = a 4 x 4 pixel patch, and the eight candidate sums are
//      reduced over the row by exchanging halves of the list;
//   A  arg-max (lowest atom on ties), rank-1 update of the lane's patch in
//      FP64 rounded to FP32, ||r||^2 in FP64, record (i, c_i), stop test.
// A slot whose node stops takes the next node of the level (the first
// gridDim.x * 16 nodes are dealt out in order, the rest come from a
// counter), so stopped nodes cost no MFMA columns while work remains and
// one wave of workgroups covers the whole level.  Every reduction is a
// butterfly over XOR partners, so the lanes of a slot hold bit-identical
// sums and take the same decisions.
// ---------------------------------------------------------------------------
constexpr int kP16N = 16, kP16K = 256;
constexpr int kP16Slots = 16;                  // node slots per workgroup (the B operand's columns)
constexpr int kP16Waves = 8;                   // 64 atoms per wave
constexpr int kP16RowB = 2 * kP16K + 16;       // bytes per slot in the BF16 residual (padded)
constexpr int kP8Nodes = 16;                   // nodes per wave of the N = 8 BF16 pursuit

typedef __bf16 p16_bf16x8 __attribute__((ext_vector_type(8)));
typedef float p16_f32x4 __attribute__((ext_vector_type(4)));

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

// Lane exchanges inside a DPP row of 16 lanes, all XOR partners: row_ror:8
// (lane ^ 8), row_half_mirror (lane ^ 7 within eight), quad_perm [2,3,0,1]
// (lane ^ 2) and [1,0,3,2] (lane ^ 1).
constexpr int kDppX8 = 0x128, kDppX7 = 0x141, kDppX2 = 0x4E, kDppX1 = 0xB1;
template <int CTRL>
__device__ inline uint32_t p16_dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline double p16_dppf64(double v) {
  return __longlong_as_double((long long)dpp_u64<CTRL, 0xF>((unsigned long long)__double_as_longlong(v)));
}
// Sum over the 16 lanes of a row; a butterfly, so every lane of the row gets
// the same bits.
__device__ inline double p16_row_sum(double v) {
  v += p16_dppf64<kDppX8>(v);
  v += p16_dppf64<kDppX7>(v);
  v += p16_dppf64<kDppX2>(v);
  v += p16_dppf64<kDppX1>(v);
  return v;
}

// Per-slot state, uniform over the slot's 16 lanes.
struct P16Slot {
  int node;       // node of the level, -1 when none is left for this slot
  int t, kmax;
  double eps2, e;
  bool run;
};

// Loads node `node` into the lane's 4 x 4 patch (FP64 values of the FP32
// residual), the slot's BF16 row, and makes the first stop test; a node
// that stops at once gets its final state here.
__device__ __attribute__((always_inline)) inline void p16_load_node(const JobDev* __restrict__ jobs, const LevelDev& lv, int lg, int node,
                                     int yq, int xq, int li, char* sBrow, double (&rd)[4][4], P16Slot& s) {
  const int jidx = lv.job[node];
  const int bx = lv.x0[node], by = lv.y0[node];
  const JobDev jl = jobs[jidx];
  double pv[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) job_pixels<4>(jl, by + 4 * yq + i, bx + 4 * xq, pv[i]);
  double ep[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ep[i] = 0.0;
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    bf16x4 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float f = (float)pv[i][j];
      rd[i][j] = (double)f;
      ep[i] = fma(pv[i][j], pv[i][j], ep[i]);
      b[j] = (__bf16)f;
    }
    *(bf16x4*)(sBrow + ((4 * yq + i) * kP16N + 4 * xq) * 2) = b;
  }
  s.node = node;
  s.e = p16_row_sum((ep[0] + ep[1]) + (ep[2] + ep[3]));
  s.eps2 = jobs[jidx].eps2[lg];
  s.kmax = jobs[jidx].k[lg];
  s.t = 0;
  uint8_t st = ST_RUN;
  if (s.e < s.eps2)
    st = ST_ACC;
  else if (s.kmax <= 0)
    st = ST_SPARSE;
  s.run = st == ST_RUN;
  if (!s.run && li == 0) {
    lv.e[node] = s.e;
    lv.t[node] = 0;
    lv.st[node] = st;
  }
}

// Fills the wave's stopped slots from the level's nodes until each runs or
// none are left: node blockIdx.x * 16 + slot first, then nodes from the
// counter.  The loop and the lane exchange are uniform over the wave.
__device__ __attribute__((always_inline)) inline void p16_refill(
    const JobDev* __restrict__ jobs, const LevelDev& lv, int lg, int count, int32_t* next, int queue0, int slot,
    int yq, int xq, int li, char* sBrow, double (&rd)[4][4], P16Slot& s, bool& first, bool& dry) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    const bool need = !s.run && !dry;
    if (__ballot(need) == 0ull) break;
    int idx = 0;
    if (need && li == 0) idx = first ? (int)blockIdx.x * kP16Slots + slot : queue0 + atomicAdd(next, 1);
    idx = __shfl(idx, lane & ~15, 64);
    if (need) {
      if (idx < count) {
        p16_load_node(jobs, lv, lg, idx, yq, xq, li, sBrow, rd, s);
      } else {
        dry = true;
        s.node = -1;
      }
    }
    first = false;
  }
}

__global__ __launch_bounds__(kP16Waves * 64, 1) void k_pursuit16_bf16(
    const JobDev* __restrict__ jobs, LevelDev lv, const int32_t* __restrict__ count_ptr,
    int32_t* __restrict__ next, int32_t lg, int32_t n_atoms, int32_t nfam, const double* __restrict__ tab,
    const float* __restrict__ tabT32) {
  constexpr int N = kP16N, K = kP16K, NS = kP16Slots, NT = kP16Waves * 64;
  __shared__ __attribute__((aligned(16))) char sB[NS * kP16RowB];       // BF16 residual per slot
  __shared__ __attribute__((aligned(16))) uint32_t sKey[kP16Waves][NS][8];
  __shared__ __attribute__((aligned(16))) double sTab[2][N][N];         // FP64 T_f[k][n]
  __shared__ float sT32[2][N][N];                                       // FP32 [f][n][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < nfam * K; i += NT) {
    (&sTab[0][0][0])[i] = tab[i];
    (&sT32[0][0][0])[i] = tabT32[i];
  }
  for (int i = tid; i < NS * kP16RowB / 16; i += NT) ((uint4*)sB)[i] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  const int count = *count_ptr;
  const double inv_n = 1.0 / N;

  // ---- correlation geometry: wave w, family w / 4, q = 4 (w % 4) + ma ----
  const int c16 = lane & 15, quad = lane >> 4;
  const bool fam_ok = (w >> 2) < nfam;
  const int fam = fam_ok ? (w >> 2) : 0;
  const int qb = 4 * (w & 3);
  // A fragment (tile ma, k-step ks): row p = c16, pixels 32 ks + 8 quad + j,
  // i.e. y = 2 ks + quad / 2, x = 8 (quad % 2) + j.
  p16_bf16x8 afr[4][8];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    const int y = 2 * ks + (quad >> 1), x0 = 8 * (quad & 1);
    const float tp = sT32[fam][y][c16];
#pragma unroll
    for (int ma = 0; ma < 4; ++ma)
#pragma unroll
      for (int j = 0; j < 8; ++j) afr[ma][ks][j] = (__bf16)(tp * sT32[fam][x0 + j][qb + ma]);
  }
  // 511 - atom of accumulator (ma, r): atom = 256 f + 16 (qb + ma) + 4 quad + r
  const uint32_t lb = 511u - (uint32_t)(256 * (w >> 2) + 16 * qb + 4 * quad);

  // ---- slot geometry: waves 0-3 own the slots, four per wave (a DPP row each) ----
  const bool owner = w < NS / 4;
  const int slot = 4 * w + quad;
  const int li = c16, yq = li >> 2, xq = li & 3;
  char* sBrow = sB + (owner ? slot : 0) * kP16RowB;
  P16Slot s{-1, 0, 0, 0.0, 0.0, false};
  double rd[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) rd[i][j] = 0.0;
  const int queue0 = gridDim.x * NS;   // nodes below this are dealt out in order
  bool first = true, dry = false;

  if (owner) p16_refill(jobs, lv, lg, count, next, queue0, slot, yq, xq, li, sBrow, rd, s, first, dry);
  first = false;
  bool any = __syncthreads_or(s.run);

  while (any) {
    // ---- C: correlation of the wave's 64 atoms with the 16 slots ----
    p16_f32x4 acc[4];
#pragma unroll
    for (int ma = 0; ma < 4; ++ma) acc[ma] = p16_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const p16_bf16x8 bf = *(const p16_bf16x8*)(sB + c16 * kP16RowB + 64 * ks + 16 * quad);
#pragma unroll
      for (int ma = 0; ma < 4; ++ma) acc[ma] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[ma][ks], bf, acc[ma], 0, 0, 0);
    }
    // ---- E: the wave's best 8 keys of slot c16 ----
    {
      uint32_t top[8], v[8];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) {
          const int ma = 2 * g + (e8 >> 2), r = e8 & 3;
          const uint32_t bits = __float_as_uint(acc[ma][r]);
          v[e8] = ((bits & 0x7FFFFF00u) << 1) | (lb - (uint32_t)(16 * ma + r));
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
      for (int j = 0; j < 8; ++j) v[j] = __shfl_xor(top[j], 16, 64);
      p16_merge8(top, v);
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = __shfl_xor(top[j], 32, 64);
      p16_merge8(top, v);
      if (quad == 0) {
        uint4* kp = (uint4*)&sKey[w][c16][0];
        kp[0] = fam_ok ? make_uint4(top[0], top[1], top[2], top[3]) : make_uint4(0u, 0u, 0u, 0u);
        kp[1] = fam_ok ? make_uint4(top[4], top[5], top[6], top[7]) : make_uint4(0u, 0u, 0u, 0u);
      }
    }
    __syncthreads();
    if (owner) {
      if (s.run) {
        // ---- M: the slot's 8 candidates from the eight wave lists ----
        uint32_t top[8], v[8];
        {
          const uint4* kp = (const uint4*)&sKey[li & 7][slot][0];
          const uint4 k0 = kp[0], k1 = kp[1];
          top[0] = k0.x; top[1] = k0.y; top[2] = k0.z; top[3] = k0.w;
          top[4] = k1.x; top[5] = k1.y; top[6] = k1.z; top[7] = k1.w;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p16_dpp32<kDppX7>(top[j]);
        p16_merge8(top, v);
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p16_dpp32<kDppX1>(top[j]);
        p16_merge8(top, v);
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p16_dpp32<kDppX2>(top[j]);
        p16_merge8(top, v);
        int cand[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const unsigned at = 511u - (top[j] & 0x1FFu);
          cand[j] = (top[j] != 0u && at < (unsigned)n_atoms) ? (int)at : -1;
        }
        // ---- S: FP64 re-score, the lane's patch, then the row sums ----
        double part[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int at = cand[j] < 0 ? 0 : cand[j];
          const int f = at >> 8, q = (at >> 4) & 15, p = at & 15;
          const bool dc = (at & 255) == 0;
          const double2 q0 = *(const double2*)&sTab[f][q][4 * xq];
          const double2 q1 = *(const double2*)&sTab[f][q][4 * xq + 2];
          const double2 p0 = *(const double2*)&sTab[f][p][4 * yq];
          const double2 p1 = *(const double2*)&sTab[f][p][4 * yq + 2];
          const double tq[4] = {dc ? 1.0 : q0.x, dc ? 1.0 : q0.y, dc ? 1.0 : q1.x, dc ? 1.0 : q1.y};
          const double tp[4] = {dc ? 1.0 : p0.x, dc ? 1.0 : p0.y, dc ? 1.0 : p1.x, dc ? 1.0 : p1.y};
          double sy[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            sy[i] = rd[i][0] * tq[0];
#pragma unroll
            for (int x = 1; x < 4; ++x) sy[i] = fma(rd[i][x], tq[x], sy[i]);
          }
          const double pt = fma(tp[0], sy[0], tp[1] * sy[1]) + fma(tp[2], sy[2], tp[3] * sy[3]);
          part[j] = cand[j] < 0 ? 0.0 : (dc ? pt * inv_n : pt);
        }
        // halves of the list go to the partner 8, 7 (within eight), 2 lanes
        // away, then one plain sum: lane bits 3, 2, 1 name the candidate
        const bool b3 = li & 8, b2 = li & 4, b1 = li & 2;
        double h4[4], h2[2];
#pragma unroll
        for (int j = 0; j < 4; ++j) h4[j] = (b3 ? part[j + 4] : part[j]) + p16_dppf64<kDppX8>(b3 ? part[j] : part[j + 4]);
#pragma unroll
        for (int j = 0; j < 2; ++j) h2[j] = (b2 ? h4[j + 2] : h4[j]) + p16_dppf64<kDppX7>(b2 ? h4[j] : h4[j + 2]);
        double c = (b1 ? h2[1] : h2[0]) + p16_dppf64<kDppX2>(b1 ? h2[0] : h2[1]);
        c += p16_dppf64<kDppX1>(c);
        const int jj = (b3 ? 4 : 0) + (b2 ? 2 : 0) + (b1 ? 1 : 0);
        int at = -1;
#pragma unroll
        for (int j = 0; j < 8; ++j) at = jj == j ? cand[j] : at;
        // ---- A: arg-max over the row (lowest atom on ties) ----
        double mag = at >= 0 ? fabs(c) : -1.0;
#define AQMP_P16_ARGMAX(CTRL)                                                            \
  {                                                                                      \
    const double om = p16_dppf64<CTRL>(mag), oc = p16_dppf64<CTRL>(c);                   \
    const int oa = (int)p16_dpp32<CTRL>((uint32_t)at);                                   \
    const bool take = om > mag || (om == mag && oa < at);                                \
    mag = take ? om : mag;                                                               \
    c = take ? oc : c;                                                                   \
    at = take ? oa : at;                                                                 \
  }
        AQMP_P16_ARGMAX(kDppX8) AQMP_P16_ARGMAX(kDppX7) AQMP_P16_ARGMAX(kDppX2)
#undef AQMP_P16_ARGMAX
        const bool zero = at < 0 || mag == 0.0;
        if (zero) {
          s.run = false;
          if (li == 0) {
            lv.e[s.node] = s.e;
            lv.t[s.node] = s.t;
            lv.st[s.node] = ST_ZERO;
          }
        } else {
          // rank-1 update of the patch, ||r||^2, record, stop test
          const int f = at >> 8, q = (at >> 4) & 15, p = at & 15;
          const bool dc = (at & 255) == 0;
          const double2 q0 = *(const double2*)&sTab[f][q][4 * xq];
          const double2 q1 = *(const double2*)&sTab[f][q][4 * xq + 2];
          const double2 p0 = *(const double2*)&sTab[f][p][4 * yq];
          const double2 p1 = *(const double2*)&sTab[f][p][4 * yq + 2];
          const double tq[4] = {q0.x, q0.y, q1.x, q1.y};
          const double tp[4] = {p0.x, p0.y, p1.x, p1.y};
          double eh[4];
          typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            bf16x4 b;
            eh[i] = 0.0;
#pragma unroll
            for (int x = 0; x < 4; ++x) {
              const double phi = dc ? inv_n : tp[i] * tq[x];
              const float rn = (float)fma(-c, phi, rd[i][x]);
              rd[i][x] = (double)rn;
              eh[i] = fma(rd[i][x], rd[i][x], eh[i]);
              b[x] = (__bf16)rn;
            }
            *(bf16x4*)(sBrow + ((4 * yq + i) * N + 4 * xq) * 2) = b;
          }
          const double en = p16_row_sum((eh[0] + eh[1]) + (eh[2] + eh[3]));
          if (li == 0) {
            const size_t rs = (size_t)s.node * lv.kmax + s.t;
            lv.rec_idx[rs] = at;
            lv.rec_coef[rs] = c;
          }
          s.t += 1;
          s.e = en;
          uint8_t st = ST_RUN;
          if (en < s.eps2)
            st = ST_ACC;
          else if (s.t >= s.kmax)
            st = ST_SPARSE;
          if (st != ST_RUN) {
            s.run = false;
            if (li == 0) {
              lv.e[s.node] = s.e;
              lv.t[s.node] = s.t;
              lv.st[s.node] = st;
            }
          }
        }
      }
      p16_refill(jobs, lv, lg, count, next, queue0, slot, yq, xq, li, sBrow, rd, s, first, dry);
    }
    any = __syncthreads_or(s.run);
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

hipError_t launch_pursuit16_bf16(const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next, int64_t cap,
                                 int32_t n_atoms, int32_t nfam, const double* tab, const float* tabT32, hipStream_t s) {
  // Slots take nodes until none are left, so the grid is as many workgroups
  // as are resident at once (at most one per 16 nodes of the level).
  int dev = 0, n_cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pursuit16_bf16, kP16Waves * 64, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int64_t wgs = (cap + kP16Slots - 1) / kP16Slots;
  if (wgs > (int64_t)n_cus * per_cu) wgs = (int64_t)n_cus * per_cu;
  if (wgs < 1) wgs = 1;
  hipLaunchKernelGGL(k_pursuit16_bf16, dim3((unsigned)wgs), dim3(kP16Waves * 64), 0, s, jobs, lv, count, next, 4,
                     n_atoms, nfam, tab, tabT32);
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
