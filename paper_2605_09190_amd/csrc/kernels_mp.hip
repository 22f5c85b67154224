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
#pragma unroll
    for (int dy = 0; dy < G::PH; ++dy) {
      f32v fv;
      u16v bv;
#pragma unroll
      for (int dx = 0; dx < G::PW; ++dx) {
        const double v = job_pixel(jb, by + py + dy, bx + px + dx);
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

// Lane groups of the select kernel: TPN lanes (at most one wave) per node,
// each lane owning a PH x PW patch of the block.
template <int N>
struct WGeo {
  static constexpr int K = N * N;
  static constexpr int TPN = K < 64 ? K : 64;
  static constexpr int NPI = 64 / TPN;               // nodes per wave per iteration
  static constexpr int PPT = K / TPN;
  static constexpr int PH = PPT == 64 ? 8 : (PPT == 16 ? 4 : (PPT == 4 ? 2 : 1));
  static constexpr int PW = PPT / PH;
  static constexpr int PX = N / PW;
};

// ---------------------------------------------------------------------------
// Select/update: one MP iteration for every active node after the
// correlation pass has left each node's best keys per atom tile.
//   1. merge the keys into the kCand best candidates;
//   2. re-score them in FP64 against the FP32 residual (this is also the
//      coefficient <r, phi_i> of the chosen atom);
//   3. i = argmax |c| (lowest atom index on ties); stop if max |c| = 0;
//   4. r <- r - c_i phi_i (FP64 arithmetic, stored in FP32), ||r||^2 in FP64;
//   5. record (i, c_i), t <- t + 1, stop test of eq. (2).
// One wave per node (N >= 16); positions are walked grid-stride.  The
// candidates' 1D table rows are staged in the wave's LDS slice with one
// coalesced load, so nothing after the merge waits on global memory.
// The nodes still running form the next step's active list: each wave holds
// its survivors in registers (one per lane; the launch gives every wave at
// most 64 positions), and after the loop the workgroup (4 or 8 waves)
// appends them with a single atomic.  The list order then varies from run to
// run; no result depends on it, since every node's arithmetic is independent
// of its list position.
// ---------------------------------------------------------------------------
// Waves (nodes) per workgroup: 8 where the staging fits in LDS, so that one
// atomic appends the survivors of 8 nodes.
template <int N>
constexpr int sel_waves() { return N >= 64 ? 4 : 8; }

template <int N>
__global__ __launch_bounds__(64 * sel_waves<N>()) void k_select(StepArgs a) {
  constexpr int W = sel_waves<N>();
  using G = WGeo<N>;
  constexpr int K = G::K, TPN = G::TPN;
  static_assert(TPN == 64, "one wave per node");
  constexpr int KPL = 4;                   // keys per lane (<= 256 keys)
  // per wave: rows [cand][0 = p row, 1 = q row][N] of the FP64 tables
  __shared__ double sT[W][kCand][2][N];
  const int count = *a.act_count;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lg = a.lg;
  const int nkeys = a.n_atom_tiles * kTopR;
  const double inv_n = 1.0 / N;
  const int py = (lane / G::PX) * G::PH;
  const int px = (lane % G::PX) * G::PW;
  const int stride = gridDim.x * W;
  int held = -1, n_held = 0;   // survivors of this wave, lane j holds the j-th
  for (int pos = blockIdx.x * W + w; pos < count; pos += stride) {
    // The keys depend only on the position: their loads go out first.
    unsigned long long k[KPL];
    const unsigned long long* kp = a.keys + (size_t)pos * nkeys;
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
      const int idx = lane + j * 64;
      k[j] = idx < nkeys ? kp[idx] : 0ull;
    }
    const int node = a.act[pos];
    const JobDev& jb = a.jobs[a.lv.job[node]];
    const int t = a.lv.t[node];
    float* r = a.r32 + (size_t)node * K;
    float rv[G::PH][G::PW];
#pragma unroll
    for (int dy = 0; dy < G::PH; ++dy)
#pragma unroll
      for (int dx = 0; dx < G::PW; ++dx) rv[dy][dx] = r[(py + dy) * N + px + dx];

    // 1. top kCand keys over the node's per-tile lists.
#pragma unroll
    for (int p0 = 0; p0 < KPL; ++p0)
#pragma unroll
      for (int p1 = 0; p1 < KPL - 1 - p0; ++p1)
        if (k[p1] < k[p1 + 1]) {
          const unsigned long long tt = k[p1];
          k[p1] = k[p1 + 1];
          k[p1 + 1] = tt;
        }
    int cand[kCand];
#pragma unroll
    for (int rr = 0; rr < kCand; ++rr) {
      const unsigned long long mx = wave_max_u64(k[0]);
      if (mx != 0ull && k[0] == mx) {
#pragma unroll
        for (int j = 0; j < KPL - 1; ++j) k[j] = k[j + 1];
        k[KPL - 1] = 0ull;
      }
      const unsigned atom = 0xFFFFFFFFu - (unsigned)(mx & 0xFFFFFFFFull);
      cand[rr] = (mx != 0ull && atom < (unsigned)a.n_atoms) ? (int)atom : -1;
    }

    // Stage the candidates' table rows: 2 * kCand rows of N doubles, all
    // loads issued before the first LDS write (one memory round trip).
    constexpr int NSTG = kCand * 2 * N / 64;
    static_assert(kCand * 2 * N % 64 == 0, "whole waves of table entries");
    double stg[NSTG];
#pragma unroll
    for (int i = 0; i < NSTG; ++i) {
      const int e = lane + 64 * i;
      const int ci = e / (2 * N), which = (e / N) & 1, col = e % N;
      int at = cand[0];
#pragma unroll
      for (int c2 = 1; c2 < kCand; ++c2)
        if (ci == c2) at = cand[c2];
      double v = 0.0;
      if (at >= 0) {
        const int f = at / K, q = (at % K) / N, p = at % N;
        v = a.tab[(size_t)f * K + (which ? q : p) * N + col];
      }
      stg[i] = v;
    }
#pragma unroll
    for (int i = 0; i < NSTG; ++i) {
      const int e = lane + 64 * i;
      sT[w][e / (2 * N)][(e / N) & 1][e % N] = stg[i];
    }
    __builtin_amdgcn_wave_barrier();

    // 2. FP64 re-score of the candidates on this lane's patch.
    double c[kCand];
#pragma unroll
    for (int ci = 0; ci < kCand; ++ci) {
      const int atom = cand[ci];
      double part = 0.0;
      if (atom >= 0) {
        const int q = (atom % K) / N, p = atom % N;
        if (p == 0 && q == 0) {
          double s = 0.0;
#pragma unroll
          for (int dy = 0; dy < G::PH; ++dy)
#pragma unroll
            for (int dx = 0; dx < G::PW; ++dx) s += (double)rv[dy][dx];
          part = s * inv_n;
        } else {
#pragma unroll
          for (int dy = 0; dy < G::PH; ++dy) {
            double s = 0.0;
#pragma unroll
            for (int dx = 0; dx < G::PW; ++dx) s = fma((double)rv[dy][dx], sT[w][ci][1][px + dx], s);
            part = fma(sT[w][ci][0][py + dy], s, part);
          }
        }
      }
      c[ci] = wave_sum_f64(part);
    }

    // 3. arg-max over the re-scored candidates, lowest atom index on ties.
    int best = -1;
    double bmag = -1.0;
#pragma unroll
    for (int ci = 0; ci < kCand; ++ci) {
      const int atom = cand[ci];
      if (atom < 0) continue;
      const double m = fabs(c[ci]);
      if (best < 0 || m > bmag || (m == bmag && atom < cand[best])) {
        best = ci;
        bmag = m;
      }
    }
    const bool zero = (best < 0 || bmag == 0.0);
    int atom = 0, bsel = 0;
    double coef = 0.0;
#pragma unroll
    for (int ci = 0; ci < kCand; ++ci)
      if (ci == best) {
        atom = cand[ci];
        coef = c[ci];
        bsel = ci;
      }

    // 4. rank-1 update and the new squared norm.
    double e = 0.0;
    if (!zero) {
      const int q = (atom % K) / N, p = atom % N;
      const bool dc = (p == 0 && q == 0);
#pragma unroll
      for (int dy = 0; dy < G::PH; ++dy) {
        const double ty = sT[w][bsel][0][py + dy];
        float rn[G::PW];
#pragma unroll
        for (int dx = 0; dx < G::PW; ++dx) {
          const double phi = dc ? inv_n : ty * sT[w][bsel][1][px + dx];
          rn[dx] = (float)fma(-coef, phi, (double)rv[dy][dx]);
          e = fma((double)rn[dx], (double)rn[dx], e);
        }
        const int o = (py + dy) * N + px;
#pragma unroll
        for (int dx = 0; dx < G::PW; ++dx) r[o + dx] = rn[dx];
        if (a.r16) {
          // PW BF16 values (round to nearest even) as one vector store
          typedef __bf16 bf16v __attribute__((ext_vector_type(G::PW)));
          bf16v pk;
#pragma unroll
          for (int dx = 0; dx < G::PW; ++dx) pk[dx] = (__bf16)rn[dx];
          *(bf16v*)(a.r16 + (size_t)node * K + o) = pk;
        }
      }
      e = wave_sum_f64(e);
    }
    __builtin_amdgcn_wave_barrier();   // table rows consumed before the next node overwrites them

    // 5. record and stop test (a zero correlation stops without a record).
    // Every input of the test is uniform over the wave.
    uint8_t st = ST_ZERO;
    if (!zero) {
      st = ST_RUN;
      if (e < jb.eps2[lg])
        st = ST_ACC;
      else if (t + 1 >= jb.k[lg])
        st = ST_SPARSE;
    }
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
  if (a.next_act == nullptr) return;   // uniform: the level's last step
  __shared__ int s_held[W], s_base;
  if (lane == 0) s_held[w] = n_held;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) tot += s_held[j];
    s_base = tot > 0 ? atomicAdd(a.next_count, tot) : 0;
    if (blockIdx.x == 0) *a.clear_count = 0;
  }
  __syncthreads();
  int off = s_base;
  for (int j = 0; j < w; ++j) off += s_held[j];
  if (lane < n_held) a.next_act[off + lane] = held;
}

// ---------------------------------------------------------------------------
// Decoder (Algorithm 3): every leaf of `job` at this level writes
// sum_t c_t phi_{i_t} at its position.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_decode(const JobDev* jobs, LevelDev lv, const int32_t* count_ptr,
                                                int32_t job, const double* tab, void* out, int32_t dtype,
                                                int64_t row_stride) {
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
      const double coef = lv.rec_coef[slot];
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
static void launch_select_n(const StepArgs& a, int64_t cap, hipStream_t s) {
  // 4096 waves, and at most 64 positions per wave: one register per lane
  // holds a survivor.
  constexpr int W = sel_waves<N>();
  int64_t g = 4096 / W;
  if (g * W * 64 < cap) g = (cap + 64 * W - 1) / (64 * W);
  hipLaunchKernelGGL(k_select<N>, dim3((unsigned)g), dim3(64 * W), 0, s, a);
}

hipError_t launch_select(int n, const StepArgs& a, int64_t cap, hipStream_t s) {
  switch (n) {
    case 16: launch_select_n<16>(a, cap, s); break;
    case 32: launch_select_n<32>(a, cap, s); break;
    case 64: launch_select_n<64>(a, cap, s); break;
    default: return hipErrorInvalidValue;   // smaller levels run the fused pursuit
  }
  return hipGetLastError();
}

hipError_t launch_decode(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t job,
                         int32_t nfam, const double* tab, void* out, int32_t dtype, int64_t row_stride,
                         hipStream_t s) {
  (void)nfam;
  AQMP_DISPATCH_N(n, hipLaunchKernelGGL(k_decode<NN>, dim3(grid_for<NN>(4)), dim3(256), 0, s, jobs, lv,
                                        count, job, tab, out, dtype, row_stride));
  return hipGetLastError();
}

}  // namespace aqmp
