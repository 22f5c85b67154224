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
// Whole-level pursuit for N = 8 and N = 16 in the BF16 form.  At these sizes
// one MP step of a node is 8 K (N = 8) or 131 K (N = 16) multiply-adds: a
// batched launch per step would be mostly launch latency and dependent
// memory chains.  Here one workgroup runs 16 node slots through their whole
// pursuits (Section 2.2 steps (a)-(d), eq. (2)) with every array in LDS or
// registers:
//   C  correlation of all M = 2 N^2 atoms with the 16 BF16 residuals by
//      v_mfma_f32_16x16x32_bf16 (A = 16 atoms x 32 pixels, B = 32 pixels x
//      16 slots, FP32 accumulation, pixel order as in the batched kernels).
//      The atoms are split evenly over the waves; tile ma of wave w holds
//      the 16 atoms a' = base_w + 16 ma + row of family f_w (q = a' / N,
//      p = a' % N), the canonical BF16 atoms bf16(T32_f[p][y] T32_f[q][x])
//      (the constant atom exactly 1/N), generated once per kernel into
//      registers;
//   E  each lane ranks its correlations of one slot as 32-bit keys (|c|
//      bits, then the inverse atom index), keeps the best 8 with sorting
//      networks and merges them with the slot's other lanes of the wave;
//   M  the slot's wave lists are merged into its 8 candidates;
//   S  FP64 re-score of the candidates against the FP32 residual,
//      separably (Section 2.1 outer product): lane = a patch of 4-pixel row
//      pieces of one slot, two candidates at a time in key order, each sum
//      reduced over the slot's lanes, stopping once the candidates' bounds
//      fall below the best re-scored value;
//   A  arg-max (lowest atom on ties), rank-1 update of the lane's patch in
//      FP64 rounded to FP32, ||r||^2 in FP64, record (i, c_i), stop test.
// A slot whose node stops takes the next node of the level (the first
// gridDim.x * 16 nodes are dealt out in order, the rest come from a
// counter, up to two fetches per step), so stopped nodes cost no MFMA
// columns while work remains and one wave of workgroups covers the level.
// Every reduction is a butterfly over XOR partners, so the lanes of a slot
// hold bit-identical sums and take the same decisions.
// ---------------------------------------------------------------------------
constexpr int kPSlots = 16;   // node slots per workgroup (the B operand's columns)

template <int N_>
struct PGeo {
  static constexpr int N = N_, K = N * N, M = 2 * K;
  static constexpr int W = N == 16 ? 8 : 4;         // waves per workgroup
  static constexpr int NT = 64 * W;
  static constexpr int AW = M / W;                  // atoms per wave
  static constexpr int MA = AW / 16;                // atom tiles per wave
  static constexpr int WPF = W / 2;                 // waves per family
  static constexpr int KS = K / 32;                 // MFMA k-steps
  static constexpr int LPS = NT / kPSlots;          // lanes per slot
  static constexpr int SPW = 64 / LPS;              // slots per wave
  static constexpr int PR = K / LPS / 4;            // rows of 4 pixels per lane
  static constexpr int XQ = N / 4;                  // 4-pixel pieces per row
  static constexpr int IB = N == 16 ? 9 : 7;        // bits of the atom index in a key
  static constexpr int ROWB = 2 * K + 16;           // bytes per slot in the BF16 residual (padded)
  // The update takes the chosen atom's table entries kept from its
  // re-score (at N = 16 the registers are not there: 255 VGPRs and a slower
  // schedule; it reads them from LDS again)
  static constexpr bool KEEP_ROWS = N == 8;
  static_assert(MA * 16 * W == M && KS * 32 == K, "whole tiles");
  static_assert(LPS == 8 || LPS == 16 || LPS == 32, "a slot is half a DPP row, one or two rows");
  static_assert(PR * 4 * LPS == K && PR >= 1, "whole patches");
  static_assert((1 << IB) == M, "key index width");
};

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
// a, b descending -> a = top 8 of both, descending (bitonic merge)
__device__ inline void p16_merge8(uint32_t (&a)[8], const uint32_t (&b)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = a[i] > b[7 - i] ? a[i] : b[7 - i];
  p16_cx(a[0], a[4]); p16_cx(a[1], a[5]); p16_cx(a[2], a[6]); p16_cx(a[3], a[7]);
  p16_cx(a[0], a[2]); p16_cx(a[1], a[3]); p16_cx(a[4], a[6]); p16_cx(a[5], a[7]);
  p16_cx(a[0], a[1]); p16_cx(a[2], a[3]); p16_cx(a[4], a[5]); p16_cx(a[6], a[7]);
}

// Lane exchanges between XOR partners inside the lanes of a slot: the DPP
// row operations row_ror:8 (lane ^ 8), row_half_mirror (lane ^ 7 within
// eight), quad_perm [2,3,0,1] (lane ^ 2) and [1,0,3,2] (lane ^ 1).
constexpr int kDppX8 = 0x128, kDppX7 = 0x141, kDppX2 = 0x4E, kDppX1 = 0xB1;
template <int CTRL>
__device__ inline uint32_t p16_x32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
// Lanes l and l ^ X (X = 16: v_permlane16_swap, rows of 16 lanes; X = 32:
// v_permlane32_swap, halves of the wave), both VALU, no LDS round trip.  A
// register swapped against a copy of itself leaves the value of the lower
// lane of each pair in p and that of the upper lane in q, in both lanes of
// the pair.
template <int X>
__device__ inline void p_pair(uint32_t v, uint32_t& p, uint32_t& q) {
  if constexpr (X == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    p = r[0];
    q = r[1];
  } else {
    static_assert(X == 32, "pairs at distance 16 or 32");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    p = r[0];
    q = r[1];
  }
}
// v(l) + v(l ^ 16), the same bits in both lanes
__device__ inline double p_pair_sum16(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  uint32_t p0, q0, p1, q1;
  p_pair<16>((uint32_t)u, p0, q0);
  p_pair<16>((uint32_t)(u >> 32), p1, q1);
  return __longlong_as_double((long long)(((unsigned long long)p1 << 32) | p0)) +
         __longlong_as_double((long long)(((unsigned long long)q1 << 32) | q0));
}
template <int CTRL>
__device__ inline double p16_xf64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = p16_x32<CTRL>((uint32_t)u), hi = p16_x32<CTRL>((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Sum over the LPS lanes of a slot; a butterfly, so every lane of the slot
// gets the same bits.
template <int LPS>
__device__ inline double p_slot_sum(double v) {
  if constexpr (LPS == 32) v = p_pair_sum16(v);
  if constexpr (LPS >= 16) v += p16_xf64<kDppX8>(v);
  v += p16_xf64<kDppX7>(v);
  v += p16_xf64<kDppX2>(v);
  v += p16_xf64<kDppX1>(v);
  return v;
}

// Two slot sums at once (the same operations on each as p_slot_sum).
template <int LPS>
__device__ inline void p_slot_sum2(double& a, double& b) {
  if constexpr (LPS == 32) {
    a = p_pair_sum16(a);
    b = p_pair_sum16(b);
  }
  if constexpr (LPS >= 16) {
    const double ta = p16_xf64<kDppX8>(a), tb = p16_xf64<kDppX8>(b);
    a += ta;
    b += tb;
  }
  {
    const double ta = p16_xf64<kDppX7>(a), tb = p16_xf64<kDppX7>(b);
    a += ta;
    b += tb;
  }
  {
    const double ta = p16_xf64<kDppX2>(a), tb = p16_xf64<kDppX2>(b);
    a += ta;
    b += tb;
  }
  {
    const double ta = p16_xf64<kDppX1>(a), tb = p16_xf64<kDppX1>(b);
    a += ta;
    b += tb;
  }
}

// BF16 copies of four FP32 values, each rounded to nearest even from the
// FP32 value.  The empty asm hides where the FP32 values came from; without
// it the compiler folds an FP64 -> FP32 -> BF16 pair of roundings into one
// FP64 -> BF16 rounding (round to odd, then to BF16: eight more
// instructions per value).
typedef __bf16 p_bf16x4 __attribute__((ext_vector_type(4)));
__device__ inline p_bf16x4 p_to_bf16x4(float a, float b, float c, float d) {
  __asm__("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
  p_bf16x4 r;
  r[0] = (__bf16)a;
  r[1] = (__bf16)b;
  r[2] = (__bf16)c;
  r[3] = (__bf16)d;
  return r;
}

// Per-slot state, uniform over the slot's lanes.
struct PSlot {
  int node;       // node of the level, -1 when none is left for this slot
  int t, kmax;
  double eps2, e;
  bool run;
};

// Lane li of a slot holds the pixels y = PR yq + i (i < PR), x = 4 xq + j
// (j < 4), yq = li / XQ, xq = li % XQ.
//
// Loads node `node` into the lane's patch (FP64 values of the FP32
// residual) and the slot's BF16 row, and makes the first stop test; a node
// that stops at once gets its final state here.
template <class G>
__device__ __attribute__((always_inline)) inline void p_load_node(const JobDev* __restrict__ jobs,
                                                                  const LevelDev& lv, int lg, int node, int yq,
                                                                  int xq, int li, char* sBrow,
                                                                  double (&rd)[G::PR][4], PSlot& s) {
  const int jidx = lv.job[node];
  const int bx = lv.x0[node], by = lv.y0[node];
  const JobDev jl = jobs[jidx];
  double pv[G::PR][4];
#pragma unroll
  for (int i = 0; i < G::PR; ++i) job_pixels<4>(jl, by + G::PR * yq + i, bx + 4 * xq, pv[i]);
  double ep = 0.0;
#pragma unroll
  for (int i = 0; i < G::PR; ++i) {
    double ei = 0.0;
    float f[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      f[j] = (float)pv[i][j];
      rd[i][j] = (double)f[j];
      ei = fma(pv[i][j], pv[i][j], ei);
    }
    ep += ei;
    *(p_bf16x4*)(sBrow + ((G::PR * yq + i) * G::N + 4 * xq) * 2) = p_to_bf16x4(f[0], f[1], f[2], f[3]);
  }
  s.node = node;
  s.e = p_slot_sum<G::LPS>(ep);
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

// One fetch for each of the wave's stopped slots: the slot leader takes the
// next node from the counter, the lanes of the slot receive it and load it.
// Straight-line code, no loop: a cross-lane exchange inside a loop whose exit
// depends on an atomic result let the compiler's structurised control flow
// run lanes of one slot out of step.  A slot whose new node stops at once
// tries again at the next fetch.  The counter only grows, so once one slot
// of the workgroup has found it past the level's end (flag *wg_dry in LDS),
// the others stop asking it.
template <class G>
__device__ __attribute__((always_inline)) inline void p_fetch(
    const JobDev* __restrict__ jobs, const LevelDev& lv, int lg, int count, int32_t* next, int queue0, int yq,
    int xq, int li, char* sBrow, double (&rd)[G::PR][4], PSlot& s, bool& dry, int* wg_dry) {
  // most steps no slot of the wave is looking for a node (uniform branch)
  if (__ballot(!s.run && !dry) == 0ull) return;
  const int lane = threadIdx.x & 63, lead = lane & ~(G::LPS - 1);
  // the leader's decision, taken by the whole slot
  const bool need = __shfl((int)(!s.run && !dry), lead, 64) != 0;
  int idx = count;
  if (need && li == 0 && __hip_atomic_load(wg_dry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
    idx = queue0 + atomicAdd(next, 1);
    if (idx >= count) __hip_atomic_store(wg_dry, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  idx = __shfl(idx, lead, 64);
  if (need) {
    if (idx < count) {
      p_load_node<G>(jobs, lv, lg, idx, yq, xq, li, sBrow, rd, s);
    } else {
      dry = true;
      s.node = -1;
    }
  }
}

// Whether v holds for some lane of the workgroup: one flag word per wave in
// LDS, one barrier.  Successive calls alternate between the two flag rows
// (par), so a row is written again only after a later barrier that every
// wave reaches after reading it.
template <int W>
__device__ __attribute__((always_inline)) inline bool p_wg_any(bool v, uint32_t (&flags)[2][W], int par) {
  const bool wv = __ballot(v) != 0ull;
  if ((threadIdx.x & 63) == 0) flags[par][threadIdx.x >> 6] = wv ? 1u : 0u;
  __syncthreads();
  uint32_t r = 0u;
#pragma unroll
  for (int i = 0; i < W; ++i) r |= flags[par][i];
  return r != 0u;
}

template <int N>
__global__ __launch_bounds__(PGeo<N>::NT) void k_pursuit_bf16(
    const JobDev* __restrict__ jobs, LevelDev lv, const int32_t* __restrict__ count_ptr,
    int32_t* __restrict__ next, int32_t lg, int32_t n_atoms, int32_t nfam, const double* __restrict__ tab,
    const float* __restrict__ tabT32) {
  using G = PGeo<N>;
  constexpr int K = G::K, NS = kPSlots, NT = G::NT, MA = G::MA, KS = G::KS, LPS = G::LPS;
  __shared__ __attribute__((aligned(16))) char sB[NS * G::ROWB];        // BF16 residual per slot
  __shared__ __attribute__((aligned(16))) uint32_t sKey[G::W][NS][8];
  __shared__ __attribute__((aligned(16))) double sTab[2][N][N];         // FP64 T_f[k][n]
  __shared__ float sT32[2][N][N];                                       // FP32 [f][n][k]
  __shared__ __attribute__((aligned(16))) uint32_t sAny[2][G::W];       // p_wg_any flags
  __shared__ int sDry;                                                  // the counter is past the end
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) sDry = 0;
  for (int i = tid; i < nfam * K; i += NT) {
    (&sTab[0][0][0])[i] = tab[i];
    (&sT32[0][0][0])[i] = tabT32[i];
  }
  for (int i = tid; i < NS * G::ROWB / 16; i += NT) ((uint4*)sB)[i] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  const int count = *count_ptr;
  const double inv_n = 1.0 / N;

  // ---- correlation geometry ----
  const int c16 = lane & 15, quad = lane >> 4;
  const int fw = w / G::WPF;                  // the wave's family
  const bool fam_ok = fw < nfam;
  const int fam = fam_ok ? fw : 0;
  const int abase = (w % G::WPF) * G::AW;     // first atom of the wave within its family
  // A fragment (tile ma, k-step ks): row = c16, pixels 32 ks + 8 quad + j
  p16_bf16x8 afr[MA][KS];
#pragma unroll
  for (int ma = 0; ma < MA; ++ma) {
    const int a = abase + 16 * ma + c16, q = a / N, p = a % N;
    const bool dc = a == 0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int px0 = 32 * ks + 8 * quad, y = px0 / N, x0 = px0 % N;
      const float tp = sT32[fam][y][p];
#pragma unroll
      for (int j = 0; j < 8; ++j) afr[ma][ks][j] = (__bf16)(dc ? (float)inv_n : tp * sT32[fam][x0 + j][q]);
    }
  }
  // (M - 1) - atom of accumulator (ma, r): atom = K f + abase + 16 ma + 4 quad + r
  const uint32_t lb = (uint32_t)(G::M - 1) - (uint32_t)(K * fw + abase + 4 * quad);

  // ---- slot geometry: wave w owns slots SPW w .. SPW w + SPW - 1 ----
  const int slot = G::SPW * w + lane / LPS;
  const int li = lane % LPS, yq = li / G::XQ, xq = li % G::XQ;
  char* sBrow = sB + slot * G::ROWB;
  PSlot s{-1, 0, 0, 0.0, 0.0, false};
  double rd[G::PR][4];
#pragma unroll
  for (int i = 0; i < G::PR; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) rd[i][j] = 0.0;
  // Node blockIdx.x * 16 + slot first (no exchange needed), then nodes from
  // the counter, starting after the first gridDim.x * 16.
  const int queue0 = gridDim.x * NS;
  bool dry = false;
  {
    const int idx0 = (int)blockIdx.x * NS + slot;
    if (idx0 < count)
      p_load_node<G>(jobs, lv, lg, idx0, yq, xq, li, sBrow, rd, s);
    else
      dry = true;
  }
  p_fetch<G>(jobs, lv, lg, count, next, queue0, yq, xq, li, sBrow, rd, s, dry, &sDry);
  int par = 0;
  bool any = p_wg_any<G::W>(s.run || !dry, sAny, par);

  while (any) {
    // ---- C: correlation of the wave's atoms with the 16 slots ----
    p16_f32x4 acc[MA];
#pragma unroll
    for (int ma = 0; ma < MA; ++ma) acc[ma] = p16_f32x4{0.f, 0.f, 0.f, 0.f};
    // Tiles in pairs, pair by pair, so the keys of one pair (E) can be
    // ranked while the next pair's MFMAs run.
#pragma unroll
    for (int g = 0; g < MA / 2; ++g)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const p16_bf16x8 bf = *(const p16_bf16x8*)(sB + c16 * G::ROWB + 64 * ks + 16 * quad);
        acc[2 * g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[2 * g][ks], bf, acc[2 * g], 0, 0, 0);
        acc[2 * g + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[2 * g + 1][ks], bf, acc[2 * g + 1], 0, 0, 0);
      }
    // ---- E: the wave's best 8 keys of slot c16 ----
    {
      constexpr uint32_t kMask = ~((1u << G::IB) - 1u);
      uint32_t top[8], v[8];
#pragma unroll
      for (int g = 0; g < MA / 2; ++g) {
#pragma unroll
        for (int e8 = 0; e8 < 8; ++e8) {
          const int ma = 2 * g + (e8 >> 2), r = e8 & 3;
          const uint32_t bits = __float_as_uint(acc[ma][r]);
          v[e8] = ((bits << 1) & kMask) | (lb - (uint32_t)(16 * ma + r));
        }
        p16_sort8(v);
        if (g == 0) {
#pragma unroll
          for (int j = 0; j < 8; ++j) top[j] = v[j];
        } else {
          p16_merge8(top, v);
        }
      }
      // the lists of lanes l ^ 16 and l ^ 32 (the same slot column)
      uint32_t u[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) p_pair<16>(top[j], u[j], v[j]);
      p16_merge8(u, v);
#pragma unroll
      for (int j = 0; j < 8; ++j) p_pair<32>(u[j], top[j], v[j]);
      p16_merge8(top, v);
      if (quad == 0) {
        uint4* kp = (uint4*)&sKey[w][c16][0];
        kp[0] = fam_ok ? make_uint4(top[0], top[1], top[2], top[3]) : make_uint4(0u, 0u, 0u, 0u);
        kp[1] = fam_ok ? make_uint4(top[4], top[5], top[6], top[7]) : make_uint4(0u, 0u, 0u, 0u);
      }
    }
    __syncthreads();
    if (s.run) {
      // ---- M: the slot's 8 candidates from the W wave lists ----
      uint32_t top[8], v[8];
      {
        const uint4* kp = (const uint4*)&sKey[li & (G::W - 1)][slot][0];
        const uint4 k0 = kp[0], k1 = kp[1];
        top[0] = k0.x; top[1] = k0.y; top[2] = k0.z; top[3] = k0.w;
        top[4] = k1.x; top[5] = k1.y; top[6] = k1.z; top[7] = k1.w;
      }
      if constexpr (G::W == 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p16_x32<kDppX7>(top[j]);
        p16_merge8(top, v);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = p16_x32<kDppX1>(top[j]);
      p16_merge8(top, v);
      if constexpr (G::W >= 4) {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p16_x32<kDppX2>(top[j]);
        p16_merge8(top, v);
      }
      int cand[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const unsigned at = (unsigned)(G::M - 1) - (top[j] & (unsigned)(G::M - 1));
        cand[j] = (top[j] != 0u && at < (unsigned)n_atoms) ? (int)at : -1;
      }
      // ---- S + A: FP64 re-score on the lane's patch and the slot sums,
      // in key order, with the arg-max (lowest atom on ties).  The BF16
      // correlation behind a key is within (2^-8 + K 2^-24) ||r|| of the
      // FP64 value (BF16 atoms and residual, each within 2^-9 relative,
      // products exact in FP32, FP32 sums); delta = 2^-7 ||r|| is nearly
      // twice that bound.  A candidate whose key bound
      // plus delta is below the best re-scored |c| can neither be the
      // arg-max nor tie it, and no later candidate (smaller keys) can either,
      // so the choice is the one the re-score of all eight makes.  ||r|| is
      // taken in FP32 (one instruction instead of the FP64 square root's
      // refinement), clamped from below and raised by 2^-16, so that delta
      // is never below 2^-7 ||r||.
      const double delta = 0.0078125 * (double)(__builtin_sqrtf(fmaxf((float)s.e, 1e-30f)) * 1.0000153f);
      double dcpart = 0.0;   // the constant atoms are exactly 1/N
#pragma unroll
      for (int i = 0; i < G::PR; ++i) dcpart += (rd[i][0] + rd[i][1]) + (rd[i][2] + rd[i][3]);
      dcpart *= inv_n;
      constexpr uint32_t kFMask = 0x7FFFFFFFu & ~((1u << (G::IB - 1)) - 1u);
      constexpr uint32_t kFUlp = 1u << (G::IB - 1);
      double mag = -1.0, c = 0.0;
      int at = -1;
      bool live = true;
      // The FP64 table entries of atom a on the lane's patch: T_f[q][x] for
      // its four columns, T_f[p][y] for its PR rows.
      struct Rows {
        double q[4], t[G::PR];
      };
      auto rows = [&](int a) -> Rows {
        const int f = a / K, q = (a % K) / N, p = a % N;
        const double2 q0 = *(const double2*)&sTab[f][q][4 * xq];
        const double2 q1 = *(const double2*)&sTab[f][q][4 * xq + 2];
        Rows r;
        r.q[0] = q0.x;
        r.q[1] = q0.y;
        r.q[2] = q1.x;
        r.q[3] = q1.y;
        if constexpr (G::PR == 2) {
          const double2 p0 = *(const double2*)&sTab[f][p][2 * yq];
          r.t[0] = p0.x;
          r.t[1] = p0.y;
        } else {
          r.t[0] = sTab[f][p][yq];
        }
        return r;
      };
      // The lane's part of candidate a's FP64 correlation.
      auto part = [&](int a, const Rows& r) -> double {
        if ((a % K) == 0) return dcpart;
        double pt = 0.0;
#pragma unroll
        for (int i = 0; i < G::PR; ++i) {
          const double sy = fma(rd[i][0], r.q[0], rd[i][1] * r.q[1]) + fma(rd[i][2], r.q[2], rd[i][3] * r.q[3]);
          pt = i == 0 ? r.t[0] * sy : fma(r.t[i], sy, pt);
        }
        return pt;
      };
      Rows br{};   // the rows of the best candidate so far (KEEP_ROWS)
      // Candidates two at a time (two slot sums in flight together); the
      // bound test is made on the first of each pair.  Re-scoring the second
      // even when its bound has fallen below mag changes nothing: its |c| is
      // then below mag, so it is not taken, and every later bound is smaller.
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const int a0 = cand[j], a1 = cand[j + 1];
        const double ub = (double)__uint_as_float(((top[j] >> 1) & kFMask) + kFUlp) + delta;
        live = live && a0 >= 0 && ub >= mag;
        if (__ballot(live) != 0ull) {   // uniform: some slot of the wave needs this pair
          const int b0 = a0 < 0 ? 0 : a0, b1 = a1 < 0 ? 0 : a1;
          const Rows r0 = rows(b0), r1 = rows(b1);
          double c0 = part(b0, r0), c1 = part(b1, r1);
          p_slot_sum2<LPS>(c0, c1);
          const double m0 = fabs(c0), m1 = fabs(c1);
          if (live && (m0 > mag || (m0 == mag && a0 < at))) {
            mag = m0;
            c = c0;
            at = a0;
            if constexpr (G::KEEP_ROWS) br = r0;
          }
          if (live && a1 >= 0 && (m1 > mag || (m1 == mag && a1 < at))) {
            mag = m1;
            c = c1;
            at = a1;
            if constexpr (G::KEEP_ROWS) br = r1;
          }
        }
      }
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
        const bool dc = (at % K) == 0;
        if constexpr (!G::KEEP_ROWS) br = rows(at);
        const double* tq = br.q;
        const double* tp = br.t;
        double eh = 0.0;
#pragma unroll
        for (int i = 0; i < G::PR; ++i) {
          float rn[4];
          double ei = 0.0;
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            const double phi = dc ? inv_n : tp[i] * tq[x];
            rn[x] = (float)fma(-c, phi, rd[i][x]);
            rd[i][x] = (double)rn[x];
            ei = fma(rd[i][x], rd[i][x], ei);
          }
          eh += ei;
          *(p_bf16x4*)(sBrow + ((G::PR * yq + i) * N + 4 * xq) * 2) = p_to_bf16x4(rn[0], rn[1], rn[2], rn[3]);
        }
        const double en = p_slot_sum<LPS>(eh);
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
    p_fetch<G>(jobs, lv, lg, count, next, queue0, yq, xq, li, sBrow, rd, s, dry, &sDry);
    p_fetch<G>(jobs, lv, lg, count, next, queue0, yq, xq, li, sBrow, rd, s, dry, &sDry);
    par ^= 1;
    any = p_wg_any<G::W>(s.run || !dry, sAny, par);
  }
}
}  // namespace

namespace {
template <int N>
hipError_t launch_pursuit_n(const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next, int64_t cap,
                            int32_t lg, int32_t n_atoms, int32_t nfam, const double* tab, const float* tabT32,
                            hipStream_t s) {
  using G = PGeo<N>;
  // Slots take nodes until none are left, so the grid is as many workgroups
  // as are resident at once (at most one per 16 nodes of the level).
  int dev = 0, n_cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pursuit_bf16<N>, G::NT, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int64_t wgs = (cap + kPSlots - 1) / kPSlots;
  if (wgs > (int64_t)n_cus * per_cu) wgs = (int64_t)n_cus * per_cu;
  if (wgs < 1) wgs = 1;
  hipLaunchKernelGGL(k_pursuit_bf16<N>, dim3((unsigned)wgs), dim3(G::NT), 0, s, jobs, lv, count, next, lg, n_atoms,
                     nfam, tab, tabT32);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_pursuit_bf16(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next,
                               int64_t cap, int32_t n_atoms, int32_t nfam, const double* tab, const float* tabT32,
                               hipStream_t s) {
  switch (n) {
    case 8: return launch_pursuit_n<8>(jobs, lv, count, next, cap, 3, n_atoms, nfam, tab, tabT32, s);
    case 16: return launch_pursuit_n<16>(jobs, lv, count, next, cap, 4, n_atoms, nfam, tab, tabT32, s);
    default: return hipErrorInvalidValue;
  }
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
