// kernels_mp.hip - per-node Matching Pursuit kernels: gathering a block into
// its residual, the candidate re-score / coefficient / rank-1 update / norm
// step of MP (Section 2.2, steps (b)-(c) and eq. (2)), and the decoder of
// Algorithm 3.
//
// Layout: the residual of node slot i is r32[i * N*N + y*N + x] (row-major
// pixels of the block; the correlation sums over pixels, so the dictionary
// uses the same order).  Atom a = f*N*N + q*N + p has the 2D shape
// T_f[p][y] * T_f[q][x]; the constant atom (p = q = 0) is exactly 1/N.
#include "internal.h"
#include "dev_common.h"

namespace aqmp {

namespace {

// Pixels of thread `lt` in its node: rows y0..y0+PH-1, columns x0..x0+PW-1.
template <int N>
__device__ inline void patch_origin(int lt, int& y0, int& x0) {
  using G = Geo<N>;
  y0 = (lt / G::PX) * G::PH;
  x0 = (lt % G::PX) * G::PW;
}

// ---------------------------------------------------------------------------
// Gather: residual r = unravel(block) (Algorithm 2, y := unravel(b)), its
// squared norm in FP64 and the stop test before the first iteration.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_gather(StepArgs a, const int32_t* count_ptr) {
  using G = Geo<N>;
  constexpr int K = G::K;
  __shared__ double s_red[G::NPW][4];
  const int count = *count_ptr;
  const int g = threadIdx.x / G::TPN, lt = threadIdx.x % G::TPN;
  const int lg = a.lg;
  for (int base = blockIdx.x * G::NPW; base < count; base += gridDim.x * G::NPW) {
    const int i = base + g;
    const bool valid = i < count;
    const int node = valid ? i : 0;
    const JobDev& jb = a.jobs[a.lv.job[node]];
    const int bx = a.lv.x0[node], by = a.lv.y0[node];
    int py, px;
    patch_origin<N>(lt, py, px);
    float* r = a.r32 + (size_t)node * K;
    double e = 0.0;
    // a patch row of PW pixels: one FP32 and one BF16 vector store
    typedef float f32v __attribute__((ext_vector_type(G::PW)));
    typedef uint16_t u16v __attribute__((ext_vector_type(G::PW)));
    // every load of the patch is issued before the first is used
    const JobDev jl = jb;
    double pv[G::PH][G::PW];
#pragma unroll
    for (int dy = 0; dy < G::PH; ++dy) job_pixels<G::PW>(jl, by + py + dy, bx + px, pv[dy]);
#pragma unroll
    for (int dy = 0; dy < G::PH; ++dy) {
      f32v fv;
      u16v bv;
#pragma unroll
      for (int dx = 0; dx < G::PW; ++dx) {
        const double v = pv[dy][dx];
        fv[dx] = (float)v;
        bv[dx] = f32_to_bf16(fv[dx]);
        e += v * v;
      }
      const int o = (py + dy) * N + px;
      if (valid) {
        *(f32v*)(r + o) = fv;
        if (a.r16) *(u16v*)(a.r16 + (size_t)node * K + o) = bv;
      }
    }
    e = group_sum<G::TPN>(e, s_red[g]);
    if (valid && lt == 0) {
      a.lv.e[node] = e;
      a.lv.t[node] = 0;
      uint8_t st = ST_RUN;
      if (e < jb.eps2[lg])
        st = ST_ACC;
      else if (jb.k[lg] <= 0)
        st = ST_SPARSE;
      a.lv.st[node] = st;
    }
  }
}

// ---------------------------------------------------------------------------
// Select/update: one MP iteration for every active node after the
// correlation pass has left each node's best keys per atom tile.
//   1. merge the keys into the kCand best candidates;
//   2. re-score them in FP64 against the FP32 residual (this is also the
//      coefficient <r, phi_i> of the chosen atom);
//   3. i = argmax |c| (lowest atom index on ties); stop if max |c| = 0;
//   4. r <- r - c_i phi_i (FP64 arithmetic, stored in FP32), ||r||^2 in FP64;
//   5. record (i, c_i), t <- t + 1, stop test of eq. (2).
// With about one active node per SIMD at the large block sizes, the time of
// a step is the length of one node's chain of dependent loads and FP64
// arithmetic, so a node is split over WPN waves: wave h of a node owns rows
// [h N / WPN, (h + 1) N / WPN) of the block, each lane a PH x PW patch.  The
// partial candidate sums and squared norms of a node's waves meet in LDS and
// are added in wave order, so every wave of a node sees the same totals.  A
// workgroup holds NPG nodes; all of them take the same barriers (positions
// past the active count take part without work).  Each wave merges the
// node's keys itself (no barrier) with two 32-bit wave maxima per candidate
// (high word = |c| bits, then the low word = ~atom among the lanes holding
// that high word), the same order as the 64-bit keys.  The candidates' 1D
// table rows a wave needs (its p-rows, all q-rows) are staged in its LDS
// slice with one coalesced load.
// The nodes still running form the next step's active list: the lead wave of
// each node slot holds its survivors in registers (one per lane; the launch
// gives a slot at most 64 positions), and after the loop the workgroup
// appends them with a single atomic.  The list order then varies from run to
// run; no result depends on it, since every node's arithmetic is independent
// of its list position.
// ---------------------------------------------------------------------------
// Measured on the 2048 x 2048 x 3 encode: one wave per node is fastest at
// every block size (two or four waves per node at N = 64 took 0.82-0.84 ms
// per encode instead of 0.72: more barriers, redundant key merges and twice
// the appends), and 4 (N = 64) or 8 nodes per workgroup, i.e. per append.
template <int N>
struct SelCfg {
  static constexpr int WPN = 1;                 // waves per node
  static constexpr int NPG = N >= 64 ? 4 : 8;   // nodes per workgroup
};

template <int N, int WPN>
struct SGeo {
  static constexpr int K = N * N;
  static constexpr int PW = N / 8;              // columns per lane
  static constexpr int PH = N / (8 * WPN);      // rows per lane
  static constexpr int ROWS = N / WPN;          // rows per wave
  static_assert(PW >= 1 && PH >= 1, "at least one pixel per lane");
  static constexpr int NKEYL = 4;               // keys per lane (<= 256 keys per node)
  static_assert(kCand * N % 64 == 0 && kCand * ROWS % 64 == 0, "whole waves of table entries");
};

__device__ inline uint32_t wave_max_u32(uint32_t v) {
#define AQMP_MAXSTEP32(C, RM) { const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, C, RM, 0xF, false); v = o > v ? o : v; }
  AQMP_MAXSTEP32(0xB1, 0xF) AQMP_MAXSTEP32(0x4E, 0xF) AQMP_MAXSTEP32(0x141, 0xF)
  AQMP_MAXSTEP32(0x140, 0xF) AQMP_MAXSTEP32(0x142, 0xA) AQMP_MAXSTEP32(0x143, 0xC)
#undef AQMP_MAXSTEP32
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

template <int N>
__global__ __launch_bounds__(64 * SelCfg<N>::WPN * SelCfg<N>::NPG, 2) void k_select(StepArgs a) {
  constexpr int WPN = SelCfg<N>::WPN, NPG = SelCfg<N>::NPG, W = WPN * NPG;
  using G = SGeo<N, WPN>;
  constexpr int K = G::K, PH = G::PH, PW = G::PW, KPL = G::NKEYL;
  // per wave and candidate: the p-row over the wave's rows, the whole q-row
  // (FP64 tables)
  __shared__ double sP[W][kCand][G::ROWS];
  __shared__ double sQ[W][kCand][N];
  __shared__ double sPart[NPG][kCand][WPN];
  __shared__ double sE[NPG][WPN];
  const int count = *a.act_count;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int slot = w / WPN, h = w % WPN;         // node slot, wave of the node
  const int lg = a.lg;
  const int nkeys = a.n_atom_tiles * kTopR;
  const double inv_n = 1.0 / N;
  const int ry = (lane >> 3) * PH;               // patch row inside the wave's rows
  const int py = h * G::ROWS + ry;               // patch row inside the block
  const int px = (lane & 7) * PW;
  const int stride = gridDim.x * NPG;
  typedef float f32v __attribute__((ext_vector_type(PW)));
  int held = -1, n_held = 0;   // survivors of this slot (lead wave), lane j holds the j-th
  // The trip count is uniform over the workgroup (barriers inside); slots past
  // the active count take part without work.
  for (int base = blockIdx.x * NPG; base < count; base += stride) {
    const int pos = base + slot;
    const bool valid = pos < count;               // uniform over the node's waves
    int node = 0, t = 0, kk = 0, jidx = 0;
    double eps2 = 0.0, eold = 0.0;
    int cand[kCand];
    uint32_t khi[kCand];   // |c| bits of each candidate's key (15 mantissa bits)
    // the re-score's choice (one wave per node)
    int r_bat = -1, r_bsel = 0;
    double r_bmag = -1.0, r_bc = 0.0;
    double rv[PH][PW];
    double c[kCand];
#pragma unroll
    for (int ci = 0; ci < kCand; ++ci) {
      cand[ci] = -1;
      c[ci] = 0.0;
    }
    if (valid) {
      // The node and its keys (which depend only on the position) are
      // loaded together: one round trip, the key loads unconditional (a
      // clamped index) so that nothing waits between them.
      node = a.act[pos];
      unsigned long long k[KPL];
      const unsigned long long* kp = a.keys + (size_t)pos * nkeys;
#pragma unroll
      for (int j = 0; j < KPL; ++j) {
        const int idx = lane + j * 64;
        const unsigned long long v = kp[idx < nkeys ? idx : nkeys - 1];
        k[j] = idx < nkeys ? v : 0ull;
      }
      // all five loads in flight before anything waits for one of them
      __builtin_amdgcn_sched_barrier(0);
      t = a.lv.t[node];
      jidx = a.lv.job[node];
      eold = a.lv.e[node];
      const float* r = a.r32 + (size_t)node * K;
#pragma unroll
      for (int dy = 0; dy < PH; ++dy) {
        const f32v v = *(const f32v*)(r + (py + dy) * N + px);
#pragma unroll
        for (int dx = 0; dx < PW; ++dx) rv[dy][dx] = (double)v[dx];
      }

      // 1. the kCand best keys: each lane sorts its own keys, then each
      // round takes the wave maximum of the lane heads (high word, then low
      // word among the lanes holding that high word) and pops it.
#pragma unroll
      for (int p0 = 0; p0 < KPL; ++p0)
#pragma unroll
        for (int p1 = 0; p1 < KPL - 1 - p0; ++p1)
          if (k[p1] < k[p1 + 1]) {
            const unsigned long long tt = k[p1];
            k[p1] = k[p1 + 1];
            k[p1 + 1] = tt;
          }
#pragma unroll
      for (int rr = 0; rr < kCand; ++rr) {
        const uint32_t hi = (uint32_t)(k[0] >> 32), lo = (uint32_t)k[0];
        const uint32_t mhi = wave_max_u32(hi);
        const uint32_t mlo = wave_max_u32(hi == mhi ? lo : 0u);
        const bool nonempty = (mhi | mlo) != 0u;
        if (nonempty && hi == mhi && lo == mlo) {
#pragma unroll
          for (int j = 0; j < KPL - 1; ++j) k[j] = k[j + 1];
          k[KPL - 1] = 0ull;
        }
        const unsigned at = 0xFFFFFFFFu - mlo;
        cand[rr] = (nonempty && at < (unsigned)a.n_atoms) ? (int)at : -1;
        khi[rr] = mhi;
      }

      // Stage the candidates' table rows this wave needs: for every
      // candidate its p-row over the wave's rows and its whole q-row; all
      // loads are issued before the first LDS write (one memory round trip).
      constexpr int NQ = kCand * N / 64, NP = kCand * G::ROWS / 64;
      double sq[NQ], sp[NP];
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const int e2 = lane + 64 * i, ci = e2 / N, col = e2 % N;
        int at = -1;
#pragma unroll
        for (int c2 = 0; c2 < kCand; ++c2)
          if (c2 * N <= 64 * i + 63 && (c2 + 1) * N > 64 * i && ci == c2) at = cand[c2];
        const int f = at / K, q = (at % K) / N;
        sq[i] = at >= 0 ? a.tab[(size_t)f * K + q * N + col] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const int e2 = lane + 64 * i, ci = e2 / G::ROWS, col = e2 % G::ROWS;
        int at = -1;
#pragma unroll
        for (int c2 = 0; c2 < kCand; ++c2)
          if (c2 * G::ROWS <= 64 * i + 63 && (c2 + 1) * G::ROWS > 64 * i && ci == c2) at = cand[c2];
        const int f = at / K, p = at % N;
        sp[i] = at >= 0 ? a.tab[(size_t)f * K + p * N + h * G::ROWS + col] : 0.0;
      }
      // the stop test's inputs share the table rows' round trip; held in
      // scalar registers (uniform per node), the end of the step waits for
      // no load
      {
        const double e2v = a.jobs[jidx].eps2[lg];
        const int kv = a.jobs[jidx].k[lg];
        const unsigned long long eb = (unsigned long long)__double_as_longlong(e2v);
        const unsigned elo = __builtin_amdgcn_readfirstlane((int)(unsigned)eb);
        const unsigned ehi = __builtin_amdgcn_readfirstlane((int)(unsigned)(eb >> 32));
        eps2 = __longlong_as_double((long long)(((unsigned long long)ehi << 32) | elo));
        kk = __builtin_amdgcn_readfirstlane(kv);
      }
#pragma unroll
      for (int i = 0; i < NQ; ++i) (&sQ[w][0][0])[lane + 64 * i] = sq[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) (&sP[w][0][0])[lane + 64 * i] = sp[i];
      __builtin_amdgcn_wave_barrier();

      // 2. FP64 re-score of the candidates: this lane's patch, row sums kept
      // apart so that the FMA chains are short.
      auto part_of = [&](int ci) -> double {
        const int at = cand[ci];
        double part = 0.0;
        if (at >= 0) {
          const int q = (at % K) / N, p = at % N;
          double sr[PH];
          if (p == 0 && q == 0) {
#pragma unroll
            for (int dy = 0; dy < PH; ++dy) {
              sr[dy] = 0.0;
#pragma unroll
              for (int dx = 0; dx < PW; ++dx) sr[dy] += rv[dy][dx];
            }
#pragma unroll
            for (int dy = 0; dy < PH; ++dy) part += sr[dy];
            part *= inv_n;
          } else {
#pragma unroll
            for (int dy = 0; dy < PH; ++dy) {
              sr[dy] = 0.0;
#pragma unroll
              for (int dx = 0; dx < PW; ++dx) sr[dy] = fma(rv[dy][dx], sQ[w][ci][px + dx], sr[dy]);
            }
#pragma unroll
            for (int dy = 0; dy < PH; ++dy) part = fma(sP[w][ci][ry + dy], sr[dy], part);
          }
        }
        return part;
      };
      if constexpr (WPN == 1) {
        // Candidates in key order, two at a time, with the arg-max (lowest
        // atom on ties).  The BF16 correlation behind a key is within
        // (2^-8 + K 2^-24) ||r|| of the FP64 value (BF16 atoms and residual,
        // each within 2^-9 relative, products exact in FP32, FP32 sums), and
        // the key's |c| bits are truncated to 15 mantissa bits, so its bits
        // plus one unit in the last kept place, plus delta = 2^-7 ||r||,
        // bound the FP64 |c| from above.  A pair whose first candidate's
        // bound is below the best re-scored |c| is skipped with every later
        // one: none of them can be the arg-max or tie it, so the choice is
        // the one the re-score of all eight makes.  ||r|| is taken in FP32,
        // clamped from below and raised by 2^-16 (never below the FP64 one).
        const double delta = 0.0078125 * (double)(__builtin_sqrtf(fmaxf((float)eold, 1e-30f)) * 1.0000153f);
        bool live = true;
#pragma unroll
        for (int j = 0; j < kCand; j += 2) {
          const double ub = (double)__uint_as_float(khi[j] + 0x100u) + delta;
          live = live && cand[j] >= 0 && ub >= r_bmag;
          if (live) {   // the same in every lane of the wave
            const double c0 = wave_sum_f64(part_of(j)), c1 = wave_sum_f64(part_of(j + 1));
            const double m0 = fabs(c0), m1 = fabs(c1);
            if (m0 > r_bmag || (m0 == r_bmag && cand[j] < r_bat)) {
              r_bmag = m0;
              r_bc = c0;
              r_bat = cand[j];
              r_bsel = j;
            }
            if (cand[j + 1] >= 0 && (m1 > r_bmag || (m1 == r_bmag && cand[j + 1] < r_bat))) {
              r_bmag = m1;
              r_bc = c1;
              r_bat = cand[j + 1];
              r_bsel = j + 1;
            }
          }
        }
      } else {
#pragma unroll
        for (int ci = 0; ci < kCand; ++ci) {
          c[ci] = wave_sum_f64(part_of(ci));
          // one candidate at a time: keeps the scheduler from holding every
          // candidate's table entries in registers at once
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // the node's candidate totals (a barrier when a node spans several waves)
#pragma unroll
    for (int ci = 0; ci < kCand; ++ci) {
      if constexpr (WPN > 1) {
        if (valid && lane == 0) sPart[slot][ci][h] = c[ci];
      }
    }
    if constexpr (WPN > 1) {
      __syncthreads();
#pragma unroll
      for (int ci = 0; ci < kCand; ++ci) {
        double v = sPart[slot][ci][0];
#pragma unroll
        for (int hh = 1; hh < WPN; ++hh) v += sPart[slot][ci][hh];
        c[ci] = v;
      }
    }
    bool zero = true;
    int atom = 0;
    double coef = 0.0;
    double ew = 0.0;
    if (valid) {
      // 3. arg-max over the re-scored candidates, lowest atom index on ties
      // (the running best carried by value: no indexed array reads); one
      // wave per node made it with the re-score.
      int bat = r_bat, bsel = r_bsel;
      double bmag = r_bmag, bc = r_bc;
      if constexpr (WPN > 1) {
#pragma unroll
        for (int ci = 0; ci < kCand; ++ci) {
          const int at = cand[ci];
          const double m = fabs(c[ci]);
          const bool take = at >= 0 && (bat < 0 || m > bmag || (m == bmag && at < bat));
          bat = take ? at : bat;
          bmag = take ? m : bmag;
          bc = take ? c[ci] : bc;
          bsel = take ? ci : bsel;
        }
      }
      zero = (bat < 0 || bmag == 0.0);
      atom = bat < 0 ? 0 : bat;
      coef = bc;

      // 4. rank-1 update of this wave's rows and their squared norm.
      if (!zero) {
        const int q = (atom % K) / N, p = atom % N;
        const bool dc = (p == 0 && q == 0);
        float* rw = a.r32 + (size_t)node * K;
        // the chosen atom's rows, read once (the constant atom is exactly
        // 1/N: inv_n times 1)
        double ty[PH], tx[PW];
#pragma unroll
        for (int dy = 0; dy < PH; ++dy) ty[dy] = sP[w][bsel][ry + dy];
#pragma unroll
        for (int dx = 0; dx < PW; ++dx) tx[dx] = sQ[w][bsel][px + dx];
#pragma unroll
        for (int dy = 0; dy < PH; ++dy) ty[dy] = dc ? inv_n : ty[dy];
#pragma unroll
        for (int dx = 0; dx < PW; ++dx) tx[dx] = dc ? 1.0 : tx[dx];
        double eh[PH];
#pragma unroll
        for (int dy = 0; dy < PH; ++dy) {
          f32v rn;
          eh[dy] = 0.0;
#pragma unroll
          for (int dx = 0; dx < PW; ++dx) {
            const double phi = ty[dy] * tx[dx];
            rn[dx] = (float)fma(-coef, phi, rv[dy][dx]);
            eh[dy] = fma((double)rn[dx], (double)rn[dx], eh[dy]);
          }
          const int o = (py + dy) * N + px;
          // Non-temporal stores: the residual is not read again in this
          // launch, and stores that do not stay dirty in L2 leave less to
          // write back when the launch ends (measured: the select steps
          // 0.971 -> 0.909 ms per encode, the correlations reading the
          // residual from memory instead +0.017 ms).
          __builtin_nontemporal_store(rn, (f32v*)(rw + o));
          if (a.r16) {
            // PW BF16 values, each rounded to nearest even from the FP32
            // value (integer rounding of the FP32 bits: written as a plain
            // conversion, the compiler folds the FP64 -> FP32 -> BF16 pair
            // of roundings into one FP64 -> BF16 rounding, eight more
            // instructions per value), as one vector store.
            typedef uint16_t u16v __attribute__((ext_vector_type(PW)));
            u16v pk;
#pragma unroll
            for (int dx = 0; dx < PW; ++dx) pk[dx] = f32_to_bf16(rn[dx]);
            __builtin_nontemporal_store(pk, (u16v*)(a.r16 + (size_t)node * K + o));
          }
        }
#pragma unroll
        for (int dy = 0; dy < PH; ++dy) ew += eh[dy];
        ew = wave_sum_f64(ew);
      }
    }
    // the node's squared norm (uniform: zero is uniform over the node's waves)
    double e = 0.0;
    if constexpr (WPN > 1) {
      if (valid && lane == 0) sE[slot][h] = ew;
      __syncthreads();   // also: the table rows are consumed before the next position
      if (valid && !zero) {
        e = sE[slot][0];
#pragma unroll
        for (int hh = 1; hh < WPN; ++hh) e += sE[slot][hh];
      }
    } else {
      e = ew;
      __builtin_amdgcn_wave_barrier();   // table rows consumed before the next position overwrites them
    }
    if (valid) {
      // 5. record and stop test (a zero correlation stops without a record).
      // Every input of the test is uniform over the node's waves.
      uint8_t st = ST_ZERO;
      if (!zero) {
        st = ST_RUN;
        if (e < eps2)
          st = ST_ACC;
        else if (t + 1 >= kk)
          st = ST_SPARSE;
      }
      if (h == 0) {
        if (lane == 0) {
          if (!zero) {
            const size_t rs = (size_t)node * a.lv.kmax + t;
            a.lv.rec_idx[rs] = atom;
            a.lv.rec_coef[rs] = coef;
            a.lv.t[node] = t + 1;
            a.lv.e[node] = e;
          }
          a.lv.st[node] = st;
        }
        if (st == ST_RUN) {
          if (lane == n_held) held = node;
          ++n_held;
        }
      }
    }
  }
  if (a.next_act == nullptr) return;   // uniform: the level's last step
  __shared__ int s_held[NPG], s_base;
  if (h == 0 && lane == 0) s_held[slot] = n_held;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
#pragma unroll
    for (int j = 0; j < NPG; ++j) tot += s_held[j];
    s_base = tot > 0 ? atomicAdd(a.next_count, tot) : 0;
    if (blockIdx.x == 0) *a.clear_count = 0;
  }
  __syncthreads();
  if (h == 0) {
    int off = s_base;
    for (int j = 0; j < slot; ++j) off += s_held[j];
    if (lane < n_held) a.next_act[off + lane] = held;
  }
}

// ---------------------------------------------------------------------------
// Decoder (Algorithm 3): every leaf of `job` at this level writes
// sum_t c_t phi_{i_t} at its position.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_decode(const JobDev* jobs, LevelDev lv, const int32_t* count_ptr,
                                                int32_t job, const double* tab, double step, void* out,
                                                int32_t dtype, int64_t row_stride) {
  using G = Geo<N>;
  constexpr int K = G::K;
  const int count = *count_ptr;
  const int g = threadIdx.x / G::TPN, lt = threadIdx.x % G::TPN;
  const double inv_n = 1.0 / N;
  for (int base = blockIdx.x * G::NPW; base < count; base += gridDim.x * G::NPW) {
    const int i = base + g;
    if (i >= count) continue;
    if (lv.job[i] != job || (lv.st[i] & ST_SPLIT)) continue;
    int py, px;
    patch_origin<N>(lt, py, px);
    double acc[G::PH][G::PW];
#pragma unroll
    for (int dy = 0; dy < G::PH; ++dy)
#pragma unroll
      for (int dx = 0; dx < G::PW; ++dx) acc[dy][dx] = 0.0;
    const int na = lv.t[i];
    for (int s = 0; s < na; ++s) {
      const size_t slot = (size_t)i * lv.kmax + s;
      const int atom = lv.rec_idx[slot];
      const double c0 = lv.rec_coef[slot];
      const double coef = step > 0.0 ? rint(c0 / step) * step : c0;
      const int f = atom / K, q = (atom % K) / N, p = atom % N;
      const double* tf = tab + (size_t)f * K;
      const bool dc = (p == 0 && q == 0);
#pragma unroll
      for (int dy = 0; dy < G::PH; ++dy) {
        const double ty = tf[p * N + py + dy];
#pragma unroll
        for (int dx = 0; dx < G::PW; ++dx) {
          const double phi = dc ? inv_n : ty * tf[q * N + px + dx];
          acc[dy][dx] = fma(coef, phi, acc[dy][dx]);
        }
      }
    }
    // Pixels of the padding (past the image) are not written.
    const int bx = lv.x0[i], by = lv.y0[i];
    const int w = jobs[job].w, h = jobs[job].h;
#pragma unroll
    for (int dy = 0; dy < G::PH; ++dy) {
      const int y = by + py + dy;
      const int64_t row = (int64_t)y * row_stride + bx + px;
#pragma unroll
      for (int dx = 0; dx < G::PW; ++dx) {
        if (y >= h || bx + px + dx >= w) continue;
        if (dtype == AQMP_F64)
          ((double*)out)[row + dx] = acc[dy][dx];
        else
          ((float*)out)[row + dx] = (float)acc[dy][dx];
      }
    }
  }
}

template <int N>
int grid_for(int per_cu) {
  return 256 * per_cu;
}

}  // namespace

#define AQMP_DISPATCH_N(n, CALL)         \
  switch (n) {                           \
    case 4: { constexpr int NN = 4; CALL; } break;   \
    case 8: { constexpr int NN = 8; CALL; } break;   \
    case 16: { constexpr int NN = 16; CALL; } break; \
    case 32: { constexpr int NN = 32; CALL; } break; \
    case 64: { constexpr int NN = 64; CALL; } break; \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_gather(int n, const StepArgs& a, const int32_t* count, hipStream_t s) {
  AQMP_DISPATCH_N(n, hipLaunchKernelGGL(k_gather<NN>, dim3(grid_for<NN>(8)), dim3(256), 0, s, a, count));
  return hipGetLastError();
}

template <int N>
static void launch_select_n(const StepArgs& a, int64_t cap, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  // 4096 node slots, and at most 64 positions per slot: one register per
  // lane of the slot's lead wave holds a survivor.
  constexpr int NPG = SelCfg<N>::NPG, W = SelCfg<N>::WPN * NPG;
  int64_t g = 4096 / NPG;
  if (g * NPG * 64 < cap) g = (cap + 64 * NPG - 1) / (64 * NPG);
  launch_timed(k_select<N>, dim3((unsigned)g), dim3(64 * W), s, e0, e1, a);
}

hipError_t launch_select(int n, const StepArgs& a, int64_t cap, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  switch (n) {
    case 16: launch_select_n<16>(a, cap, s, ev0, ev1); break;
    case 32: launch_select_n<32>(a, cap, s, ev0, ev1); break;
    case 64: launch_select_n<64>(a, cap, s, ev0, ev1); break;
    default: return hipErrorInvalidValue;   // smaller levels run the fused pursuit
  }
  return hipGetLastError();
}

hipError_t launch_decode(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t job,
                         int32_t nfam, const double* tab, double step, void* out, int32_t dtype, int64_t row_stride,
                         hipStream_t s) {
  (void)nfam;
  AQMP_DISPATCH_N(n, hipLaunchKernelGGL(k_decode<NN>, dim3(grid_for<NN>(4)), dim3(256), 0, s, jobs, lv,
                                        count, job, tab, step, out, dtype, row_stride));
  return hipGetLastError();
}

}  // namespace aqmp
