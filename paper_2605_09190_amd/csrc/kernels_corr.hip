// kernels_corr.hip - the batched correlation of every active node's residual
// with every atom of D_N (MP step (b): c_a = <r, phi_a> for all a), as an
// MFMA contraction, fused with a per-node top-R selection so that the
// correlations never reach HBM.
//
// Contraction: C^T[atom][node] = sum_k D[atom][k] * X[node][k], K = N*N,
// with D stored atom-major ([M_pad][K], K contiguous) and the residuals X
// node-major ([slot][K]).  Rows of X are gathered through the active list.
// A workgroup owns a BA (atoms) x BB (nodes) tile and streams K through a
// double-buffered LDS stage of BK.  Four waves split the tile WA x WB; each
// wave holds MA x MB accumulators of the 32x32 MFMA shape, so every lane owns
// one node column and 16 atom rows per accumulator.
//
// Epilogue: each lane keeps the R best |c| of its node among its atoms as
// 32-bit keys (|c| bits with the low byte replaced by 255 - local atom, so a
// plain unsigned max prefers larger |c| and then the lower atom); the two
// half-waves and the WA waves are merged, and the R keys of every (node,
// atom tile) go out as 64-bit keys ((|c| bits) << 32 | ~atom).  The key keeps
// 15 mantissa bits of |c|: it only ranks candidates for the FP64 re-score.
#include <type_traits>

#include "internal.h"
#include "dev_common.h"

namespace aqmp {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int BA_, int BB_, int BK_, int WA_, int WB_>
struct Cfg {
  static constexpr int BA = BA_, BB = BB_, BK = BK_, WA = WA_, WB = WB_;
  static constexpr int WTA = BA / WA, WTB = BB / WB;     // wave tile
  static constexpr int MA = WTA / 32, MB = WTB / 32;     // 32x32 blocks per wave
  static_assert(WA * WB == 4, "four waves");
  static_assert(MA >= 1 && MB >= 1 && BA <= 256, "tile shape");
};

// Persistent tile walk with an XCD-aware order: workgroup b runs on XCD
// b % 8; each XCD takes a contiguous chunk of the atom-major tile order, so
// the workgroups of one XCD share the same few dictionary tiles in its L2.
struct TileWalk {
  int ntiles, chunk, xcd, slot, per;
  __device__ TileWalk(int nt) : ntiles(nt) {
    xcd = blockIdx.x & 7;
    slot = blockIdx.x >> 3;
    per = gridDim.x >> 3;
    chunk = (nt + 7) >> 3;
  }
  __device__ int tile(int j) const { return xcd * chunk + j; }
};

__device__ inline void insert_key(uint32_t* top, uint32_t v, int R) {
  for (int j = 0; j < R; ++j) {
    const uint32_t hi = top[j] > v ? top[j] : v;
    v = top[j] > v ? v : top[j];
    top[j] = hi;
  }
}

// Shared epilogue: accumulators -> per (node, atom tile) top-R keys.
template <class C>
__device__ inline void epilogue(f32x16 (&acc)[C::MA][C::MB], uint32_t* sK, int a0, int a_tile,
                                int n_atom_tiles, int b0, int count, unsigned long long* keys) {
  constexpr int R = kTopR;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wa = w % C::WA, wb = w / C::WA;
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb) {
    uint32_t top[R];
#pragma unroll
    for (int j = 0; j < R; ++j) top[j] = 0u;
#pragma unroll
    for (int ma = 0; ma < C::MA; ++ma) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int loc = wa * C::WTA + ma * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const uint32_t bits = __float_as_uint(fabsf(acc[ma][mb][r]));
        const uint32_t key = (bits & 0xFFFFFF00u) | (uint32_t)(255 - loc);
        if (key > top[R - 1]) insert_key(top, key, R);
      }
    }
    // merge with the other half-wave (same node, other atom rows)
    uint32_t other[R];
#pragma unroll
    for (int j = 0; j < R; ++j) other[j] = __shfl_xor(top[j], 32, 64);
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (other[j] > top[R - 1]) insert_key(top, other[j], R);
    if (lane < 32) {
      const int nl = wb * C::WTB + mb * 32 + lane;
#pragma unroll
      for (int j = 0; j < R; ++j) sK[(wa * C::BB + nl) * R + j] = top[j];
    }
  }
  __syncthreads();
  for (int nl = tid; nl < C::BB; nl += 256) {
    const int pos = b0 + nl;
    if (pos >= count) continue;
    uint32_t top[R];
#pragma unroll
    for (int j = 0; j < R; ++j) top[j] = sK[nl * R + j];
    for (int q = 1; q < C::WA; ++q)
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t v = sK[(q * C::BB + nl) * R + j];
        if (v > top[R - 1]) insert_key(top, v, R);
      }
    unsigned long long* out = keys + ((size_t)pos * n_atom_tiles + a_tile) * R;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint32_t atom = (uint32_t)a0 + (255u - (top[j] & 0xFFu));
      out[j] = ((unsigned long long)(top[j] & 0xFFFFFF00u) << 32) | (unsigned long long)(0xFFFFFFFFu - atom);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// BF16 x BF16 -> FP32 (v_mfma_f32_32x32x16_bf16).
//
// Pipeline per K stage s (LDS buffer s & 1):
//   issue the global loads of stage s + 2 into register set s & 1;
//   compute stage s, reading the operand fragments of sub-step kk + 1 from
//   LDS while the MFMAs of sub-step kk run;
//   store register set (s + 1) & 1 (stage s + 1, loaded one stage earlier)
//   into LDS buffer (s + 1) & 1; one barrier.
// Rows of X past the active count are read from the last active row (their
// results are never written), so no load is predicated.
// ---------------------------------------------------------------------------
template <class C, int K>
struct Bf16Tile {
  static constexpr int BK = C::BK, LDA = BK + 8;   // +16 B per row against bank conflicts
  static constexpr int CPR = BK / 8;               // 16-byte chunks per row
  static constexpr int NCA = C::BA * CPR, NCB = C::BB * CPR;
  static constexpr int CA = (NCA + 255) / 256, CB = (NCB + 255) / 256;
  static constexpr bool FULLA = NCA % 256 == 0, FULLB = NCB % 256 == 0;
  static constexpr int NST = K / BK;
  static_assert(K % BK == 0, "K must be a whole number of stages");
};

template <class C, class T>
struct Bf16Regs {
  uint4 a[T::CA], b[T::CB];
};

template <class C, class T>
__device__ inline void bf16_gload(Bf16Regs<C, T>& r, const uint16_t* const* ga, const uint16_t* const* gb, int s) {
#pragma unroll
  for (int i = 0; i < T::CA; ++i)
    if (T::FULLA || ga[i]) r.a[i] = *(const uint4*)(ga[i] + s * T::BK);
#pragma unroll
  for (int i = 0; i < T::CB; ++i)
    if (T::FULLB || gb[i]) r.b[i] = *(const uint4*)(gb[i] + s * T::BK);
}

template <class C, class T>
__device__ inline void bf16_lstore(const Bf16Regs<C, T>& r, uint16_t* sa, uint16_t* sb, const int* la, const int* lb) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < T::CA; ++i)
    if (T::FULLA || tid + 256 * i < T::NCA) *(uint4*)&sa[la[i]] = r.a[i];
#pragma unroll
  for (int i = 0; i < T::CB; ++i)
    if (T::FULLB || tid + 256 * i < T::NCB) *(uint4*)&sb[lb[i]] = r.b[i];
}

template <class C, class T>
__device__ inline void bf16_compute(f32x16 (&acc)[C::MA][C::MB], const uint16_t* sa, const uint16_t* sb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wa = w % C::WA, wb = w / C::WA;
  const uint16_t* pa = sa + (wa * C::WTA + (lane & 31)) * T::LDA + (lane >> 5) * 8;
  const uint16_t* pb = sb + (wb * C::WTB + (lane & 31)) * T::LDA + (lane >> 5) * 8;
  bf16x8 fa[2][C::MA], fb[2][C::MB];
#pragma unroll
  for (int ma = 0; ma < C::MA; ++ma) fa[0][ma] = *(const bf16x8*)(pa + ma * 32 * T::LDA);
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb) fb[0][mb] = *(const bf16x8*)(pb + mb * 32 * T::LDA);
#pragma unroll
  for (int kk = 0; kk < T::BK / 16; ++kk) {
    const int cur = kk & 1, nxt = cur ^ 1;
    if (kk + 1 < T::BK / 16) {
#pragma unroll
      for (int ma = 0; ma < C::MA; ++ma) fa[nxt][ma] = *(const bf16x8*)(pa + ma * 32 * T::LDA + (kk + 1) * 16);
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb) fb[nxt][mb] = *(const bf16x8*)(pb + mb * 32 * T::LDA + (kk + 1) * 16);
    }
#pragma unroll
    for (int ma = 0; ma < C::MA; ++ma)
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb)
        acc[ma][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[cur][ma], fb[cur][mb], acc[ma][mb], 0, 0, 0);
  }
}

template <int N, class C>
__global__ __launch_bounds__(256, 1) void k_corr_bf16(const uint16_t* __restrict__ D,
                                                      const uint16_t* __restrict__ X,
                                                      const int32_t* __restrict__ act,
                                                      const int32_t* __restrict__ act_count,
                                                      unsigned long long* __restrict__ keys,
                                                      int n_atom_tiles) {
  constexpr int K = N * N;
  using T = Bf16Tile<C, K>;
  constexpr int NST = T::NST;
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][C::BA * T::LDA];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][C::BB * T::LDA];
  __shared__ uint32_t sK[C::WA * C::BB * kTopR];

  const int count = *act_count;
  const int ntB = (count + C::BB - 1) / C::BB;
  const int ntiles = n_atom_tiles * ntB;
  const int tid = threadIdx.x;
  TileWalk walk(ntiles);
  for (int j = walk.slot; j < walk.chunk; j += walk.per) {
    const int tile = walk.tile(j);
    if (tile >= ntiles) break;
    const int a_tile = tile / ntB, b_tile = tile % ntB;
    const int a0 = a_tile * C::BA, b0 = b_tile * C::BB;

    const uint16_t* ga[T::CA];
    const uint16_t* gb[T::CB];
    int la[T::CA], lb[T::CB];
#pragma unroll
    for (int i = 0; i < T::CA; ++i) {
      const int c = tid + 256 * i, row = c / T::CPR, kc = c % T::CPR;
      ga[i] = (T::FULLA || c < T::NCA) ? D + (size_t)(a0 + row) * K + kc * 8 : nullptr;
      la[i] = row * T::LDA + kc * 8;
    }
#pragma unroll
    for (int i = 0; i < T::CB; ++i) {
      const int c = tid + 256 * i, row = c / T::CPR, kc = c % T::CPR;
      const int pos = min(b0 + row, count - 1);
      gb[i] = (T::FULLB || c < T::NCB) ? X + (size_t)act[pos] * K + kc * 8 : nullptr;
      lb[i] = row * T::LDA + kc * 8;
    }

    f32x16 acc[C::MA][C::MB];
#pragma unroll
    for (int ma = 0; ma < C::MA; ++ma)
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[ma][mb][r] = 0.f;

    Bf16Regs<C, T> r0, r1;
    bf16_gload<C, T>(r0, ga, gb, 0);
    if (NST > 1) bf16_gload<C, T>(r1, ga, gb, 1);
    bf16_lstore<C, T>(r0, sA[0], sB[0], la, lb);
    __syncthreads();
    // Two stages per trip so that the register sets are compile-time.
    for (int s = 0; s < NST; s += 2) {
      if (s + 2 < NST) bf16_gload<C, T>(r0, ga, gb, s + 2);
      bf16_compute<C, T>(acc, sA[0], sB[0]);
      if (s + 1 < NST) bf16_lstore<C, T>(r1, sA[1], sB[1], la, lb);
      __syncthreads();
      if (s + 1 >= NST) break;
      if (s + 3 < NST) bf16_gload<C, T>(r1, ga, gb, s + 3);
      bf16_compute<C, T>(acc, sA[1], sB[1]);
      if (s + 2 < NST) bf16_lstore<C, T>(r0, sA[0], sB[0], la, lb);
      __syncthreads();
    }
    epilogue<C>(acc, sK, a0, a_tile, n_atom_tiles, b0, count, keys);
  }
}

// ---------------------------------------------------------------------------
// BF16, large blocks (N >= 16): direct-to-LDS loads and a three-stage ring.
//
// Tile 256 atoms x 128 nodes, BK = 64 (128-byte rows).  Each global load
// (global_load_lds_dwordx4) moves 16 bytes per lane straight into LDS, 1 KB
// per wave instruction (8 rows); no staging registers, so three stages stay
// in flight: at stage s the loads of stage s + 2 are issued while stage s is
// computed.  Row r keeps its 16-byte chunk c at slot c ^ f(r) with
// f(r) = (r & 7) ^ ((r >> 3) & 1): the 8 or 16 rows read together by one
// LDS phase hit distinct banks.  Waits are explicit (vmcnt per wave, then a
// raw barrier), because a full workgroup fence would drain the ring.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

// Geometry of the direct-to-LDS kernel for a stage depth BK (64 or 32).
template <int BK_>
struct DmaGeo {
  static constexpr int BA = 256, BB = 128, BK = BK_, WA = 2, WB = 2;
  static constexpr int WTA = BA / WA, WTB = BB / WB, MA = WTA / 32, MB = WTB / 32;
  static constexpr int ROWB = BK * 2;              // bytes per LDS row
  static constexpr int CPR = ROWB / 16;            // 16-byte chunks per row
  static constexpr int RPB = 1024 / ROWB;          // rows per 1 KB block (one wave DMA)
  static constexpr int A_BYTES = BA * ROWB, B_BYTES = BB * ROWB;
  static constexpr int A_INS = BA / RPB / 4, B_INS = BB / RPB / 4;   // DMA per wave per stage
  static constexpr int INS = A_INS + B_INS;
  static_assert(A_INS % 2 == 0, "block parity of a wave's first block is even");
  using C = Cfg<BA, BB, BK, WA, WB>;
  // Slot swizzle of row r: the rows one LDS phase reads (8 rows of a 128-byte
  // phase or 16 rows of a 256-byte phase) land in distinct banks.
  __device__ static int swz(int r) {
    if constexpr (BK == 64) return (r & 7) ^ ((r >> 3) & 1);
    else return ((r >> 1) ^ (r >> 2)) & 3;
  }
};

// vmcnt(n) with the other counters left alone (gfx9 encoding).
#define AQMP_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(((n) & 0xF) | (0x7 << 4) | (0xF << 8) | ((((n) >> 4) & 0x3) << 14))

template <class G>
struct DmaPtrs {
  const char* a_lane[2];     // A: this lane's address in even / odd blocks (stage 0)
  const char* b_lane[G::B_INS];
};

template <class G, int K>
__device__ inline void dma_issue(const DmaPtrs<G>& p, char* sa, char* sb, int s) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t kofs = (size_t)s * G::BK * 2;
#pragma unroll
  for (int i = 0; i < G::A_INS; ++i) {
    const int blk = w * G::A_INS + i;
    const char* g = p.a_lane[i & 1] + (size_t)i * G::RPB * K * 2 + kofs;
    __builtin_amdgcn_global_load_lds((gbl_void_t*)g, (lds_void_t*)(sa + blk * 1024), 16, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < G::B_INS; ++i) {
    const int blk = w * G::B_INS + i;
    __builtin_amdgcn_global_load_lds((gbl_void_t*)(p.b_lane[i] + kofs), (lds_void_t*)(sb + blk * 1024), 16, 0, 0);
  }
}

template <class G>
__device__ inline void dma_compute(f32x16 (&acc)[G::MA][G::MB], const char* sa, const char* sb,
                                   const int (&off)[G::BK / 16]) {
  const int w = threadIdx.x >> 6;
  const int wa = w % G::WA, wb = w / G::WA;
  const char* pa = sa + wa * G::WTA * G::ROWB;
  const char* pb = sb + wb * G::WTB * G::ROWB;
  bf16x8 fa[2][G::MA], fb[2][G::MB];
#pragma unroll
  for (int ma = 0; ma < G::MA; ++ma) fa[0][ma] = *(const bf16x8*)(pa + ma * 32 * G::ROWB + off[0]);
#pragma unroll
  for (int mb = 0; mb < G::MB; ++mb) fb[0][mb] = *(const bf16x8*)(pb + mb * 32 * G::ROWB + off[0]);
#pragma unroll
  for (int kk = 0; kk < G::BK / 16; ++kk) {
    const int cur = kk & 1, nxt = cur ^ 1;
    if (kk + 1 < G::BK / 16) {
#pragma unroll
      for (int ma = 0; ma < G::MA; ++ma) fa[nxt][ma] = *(const bf16x8*)(pa + ma * 32 * G::ROWB + off[kk + 1]);
#pragma unroll
      for (int mb = 0; mb < G::MB; ++mb) fb[nxt][mb] = *(const bf16x8*)(pb + mb * 32 * G::ROWB + off[kk + 1]);
    }
#pragma unroll
    for (int ma = 0; ma < G::MA; ++ma)
#pragma unroll
      for (int mb = 0; mb < G::MB; ++mb)
        acc[ma][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[cur][ma], fb[cur][mb], acc[ma][mb], 0, 0, 0);
  }
}

template <int N, int BK, int MINB>
__global__ __launch_bounds__(256, MINB) void k_corr_bf16_dma(const uint16_t* __restrict__ D,
                                                             const uint16_t* __restrict__ X,
                                                             const int32_t* __restrict__ act,
                                                             const int32_t* __restrict__ act_count,
                                                             unsigned long long* __restrict__ keys,
                                                             int n_atom_tiles) {
  using G = DmaGeo<BK>;
  constexpr int K = N * N;
  constexpr int NST = K / BK;
  static_assert(K % BK == 0 && NST >= 1, "stages");
  __shared__ __attribute__((aligned(1024))) char sA0[G::A_BYTES];
  __shared__ __attribute__((aligned(1024))) char sA1[G::A_BYTES];
  __shared__ __attribute__((aligned(1024))) char sA2[G::A_BYTES];
  __shared__ __attribute__((aligned(1024))) char sB0[G::B_BYTES];
  __shared__ __attribute__((aligned(1024))) char sB1[G::B_BYTES];
  __shared__ __attribute__((aligned(1024))) char sB2[G::B_BYTES];
  static_assert(G::WA * G::BB * kTopR * 4 <= G::A_BYTES, "epilogue scratch fits one A buffer");
  uint32_t* sK = (uint32_t*)sA0;   // epilogue scratch, after the ring drains

  const int count = *act_count;
  const int ntB = (count + G::BB - 1) / G::BB;
  const int ntiles = n_atom_tiles * ntB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int fr = G::swz(lane & 31);   // MFMA rows of this lane: row & 31 == lane & 31
  int off[G::BK / 16];
#pragma unroll
  for (int kk = 0; kk < G::BK / 16; ++kk) off[kk] = (lane & 31) * G::ROWB + (((2 * kk + (lane >> 5)) ^ fr) << 4);
  const int drow = lane / G::CPR, dslot = lane % G::CPR;   // DMA: row within block, slot
  TileWalk walk(ntiles);
  for (int j = walk.slot; j < walk.chunk; j += walk.per) {
    const int tile = walk.tile(j);
    if (tile >= ntiles) break;
    const int a_tile = tile / ntB, b_tile = tile % ntB;
    const int a0 = a_tile * G::BA, b0 = b_tile * G::BB;
    DmaPtrs<G> p;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int gc = dslot ^ G::swz(par * G::RPB + drow);
      p.a_lane[par] = (const char*)(D + (size_t)(a0 + w * G::A_INS * G::RPB + drow) * K + gc * 8);
    }
#pragma unroll
    for (int i = 0; i < G::B_INS; ++i) {
      const int row = (w * G::B_INS + i) * G::RPB + drow;
      const int gc = dslot ^ G::swz(row);
      const int pos = min(b0 + row, count - 1);
      p.b_lane[i] = (const char*)(X + (size_t)act[pos] * K + gc * 8);
    }
    f32x16 acc[G::MA][G::MB];
#pragma unroll
    for (int ma = 0; ma < G::MA; ++ma)
#pragma unroll
      for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[ma][mb][r] = 0.f;

    __syncthreads();   // previous tile's epilogue is done with sK (= sA0)
    dma_issue<G, K>(p, sA0, sB0, 0);
    if constexpr (NST > 1) dma_issue<G, K>(p, sA1, sB1, 1);
    // Steady state: every stage waits for its own loads (the next stage's
    // stay in flight), passes the barrier, issues stage s + 2 and computes.
    // Three stages per trip so that the buffers are compile-time.
    constexpr int FULL = NST > 2 ? NST - 2 : 0;    // stages that issue a load
    constexpr int TRIPS = FULL / 3;
    for (int t = 0; t < TRIPS; ++t) {
      const int s = 3 * t;
      AQMP_WAIT_VM(G::INS);
      __builtin_amdgcn_s_barrier();
      dma_issue<G, K>(p, sA2, sB2, s + 2);
      dma_compute<G>(acc, sA0, sB0, off);
      AQMP_WAIT_VM(G::INS);
      __builtin_amdgcn_s_barrier();
      dma_issue<G, K>(p, sA0, sB0, s + 3);
      dma_compute<G>(acc, sA1, sB1, off);
      AQMP_WAIT_VM(G::INS);
      __builtin_amdgcn_s_barrier();
      dma_issue<G, K>(p, sA1, sB1, s + 4);
      dma_compute<G>(acc, sA2, sB2, off);
    }
    // Tail: the last (at most four) stages, all decisions compile-time.
    constexpr int S0 = 3 * TRIPS;
#define AQMP_DMA_TAIL(I, SA, SB, NA, NB)                                    \
    if constexpr (S0 + (I) < NST) {                                         \
      if constexpr (S0 + (I) + 1 < NST) AQMP_WAIT_VM(G::INS);               \
      else AQMP_WAIT_VM(0);                                                 \
      __builtin_amdgcn_s_barrier();                                         \
      if constexpr (S0 + (I) + 2 < NST) dma_issue<G, K>(p, NA, NB, S0 + (I) + 2); \
      dma_compute<G>(acc, SA, SB, off);                                     \
    }
    AQMP_DMA_TAIL(0, sA0, sB0, sA2, sB2)
    AQMP_DMA_TAIL(1, sA1, sB1, sA0, sB0)
    AQMP_DMA_TAIL(2, sA2, sB2, sA1, sB1)
    AQMP_DMA_TAIL(3, sA0, sB0, sA2, sB2)
    static_assert(NST - S0 <= 4, "tail covers the remaining stages");
#undef AQMP_DMA_TAIL
    __syncthreads();   // all waves done reading the ring before sK reuses sA0
    epilogue<typename G::C>(acc, sK, a0, a_tile, n_atom_tiles, b0, count, keys);
  }
}

// ---------------------------------------------------------------------------
// FP32 x FP32 -> FP32 (v_mfma_f32_32x32x2f32).  Inside a BK stage the lane
// half h consumes k in [h*BK/2, (h+1)*BK/2) one MFMA at a time, so a lane
// reads its operands as contiguous 16-byte chunks (A and B use the same k
// order, which is all the contraction needs).
// ---------------------------------------------------------------------------
template <int N, class C>
__global__ __launch_bounds__(256, 1) void k_corr_f32(const float* __restrict__ D, const float* __restrict__ X,
                                                     const int32_t* __restrict__ act,
                                                     const int32_t* __restrict__ act_count,
                                                     unsigned long long* __restrict__ keys,
                                                     int n_atom_tiles) {
  constexpr int K = N * N;
  constexpr int BK = C::BK, LDA = BK + 4;
  constexpr int CPR = BK / 4;
  constexpr int NCA = C::BA * CPR, NCB = C::BB * CPR;    // chunks per stage
  constexpr int CA = (NCA + 255) / 256, CB = (NCB + 255) / 256;
  __shared__ __attribute__((aligned(16))) float sA[2][C::BA * LDA];
  __shared__ __attribute__((aligned(16))) float sB[2][C::BB * LDA];
  __shared__ uint32_t sK[C::WA * C::BB * kTopR];

  const int count = *act_count;
  const int ntB = (count + C::BB - 1) / C::BB;
  const int ntiles = n_atom_tiles * ntB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wa = w % C::WA, wb = w / C::WA;
  constexpr int nst = K / BK;
  static_assert(K % BK == 0, "K must be a whole number of stages");
  TileWalk walk(ntiles);
  for (int j = walk.slot; j < walk.chunk; j += walk.per) {
    const int tile = walk.tile(j);
    if (tile >= ntiles) break;
    const int a_tile = tile / ntB, b_tile = tile % ntB;
    const int a0 = a_tile * C::BA, b0 = b_tile * C::BB;

    const float* ga[CA];
    const float* gb[CB];
    int la[CA], lb[CB];
#pragma unroll
    for (int i = 0; i < CA; ++i) {
      const int c = tid + 256 * i, row = c / CPR, kc = c % CPR;
      ga[i] = c < NCA ? D + (size_t)(a0 + row) * K + kc * 4 : nullptr;
      la[i] = row * LDA + kc * 4;
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int c = tid + 256 * i, row = c / CPR, kc = c % CPR;
      const int pos = b0 + row;
      gb[i] = (c < NCB && pos < count) ? X + (size_t)act[pos] * K + kc * 4 : nullptr;
      lb[i] = row * LDA + kc * 4;
    }
    float4 ra[CA], rb[CB];
    auto gload = [&](int s) {
#pragma unroll
      for (int i = 0; i < CA; ++i) ra[i] = ga[i] ? *(const float4*)(ga[i] + s * BK) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int i = 0; i < CB; ++i) rb[i] = gb[i] ? *(const float4*)(gb[i] + s * BK) : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int i = 0; i < CA; ++i)
        if (tid + 256 * i < NCA) *(float4*)&sA[buf][la[i]] = ra[i];
#pragma unroll
      for (int i = 0; i < CB; ++i)
        if (tid + 256 * i < NCB) *(float4*)&sB[buf][lb[i]] = rb[i];
    };

    f32x16 acc[C::MA][C::MB];
#pragma unroll
    for (int ma = 0; ma < C::MA; ++ma)
#pragma unroll
      for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[ma][mb][r] = 0.f;

    gload(0);
    lstore(0);
    __syncthreads();
    const int hk = (lane >> 5) * (BK / 2);
    for (int s = 0; s < nst; ++s) {
      const int buf = s & 1;
      if (s + 1 < nst) gload(s + 1);
#pragma unroll
      for (int kc = 0; kc < BK / 8; ++kc) {
        float4 af[C::MA], bfr[C::MB];
#pragma unroll
        for (int ma = 0; ma < C::MA; ++ma)
          af[ma] = *(const float4*)&sA[buf][(wa * C::WTA + ma * 32 + (lane & 31)) * LDA + hk + kc * 4];
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb)
          bfr[mb] = *(const float4*)&sB[buf][(wb * C::WTB + mb * 32 + (lane & 31)) * LDA + hk + kc * 4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int ma = 0; ma < C::MA; ++ma)
#pragma unroll
            for (int mb = 0; mb < C::MB; ++mb) {
              const float x = e == 0 ? af[ma].x : e == 1 ? af[ma].y : e == 2 ? af[ma].z : af[ma].w;
              const float y = e == 0 ? bfr[mb].x : e == 1 ? bfr[mb].y : e == 2 ? bfr[mb].z : bfr[mb].w;
              acc[ma][mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, acc[ma][mb], 0, 0, 0);
            }
      }
      if (s + 1 < nst) lstore(buf ^ 1);
      __syncthreads();
    }
    epilogue<C>(acc, sK, a0, a_tile, n_atom_tiles, b0, count, keys);
  }
}

using CfgBig = Cfg<256, 128, 64, 2, 2>;     // N >= 16, BF16
using CfgNarrow = Cfg<256, 32, 64, 4, 1>;   // N = 16, 32, BF16, narrow node tiles
using CfgNarrow8 = Cfg<128, 32, 64, 4, 1>;  // N = 8, BF16, narrow node tiles
using CfgMid = Cfg<128, 128, 64, 2, 2>;     // N = 8, BF16
using CfgSmall = Cfg<32, 256, 16, 1, 4>;    // N = 4, BF16
using CfgBigF = Cfg<256, 128, 32, 2, 2>;    // N >= 16, FP32
using CfgMidF = Cfg<128, 128, 32, 2, 2>;    // N = 8, FP32
using CfgSmallF = Cfg<32, 256, 16, 1, 4>;   // N = 4, FP32

constexpr int kCorrGrid = 256;   // one persistent workgroup per CU
constexpr int kDefaultVariant = 2;

}  // namespace

int corr_atom_tile(int n) { return n >= 16 ? 256 : (n == 8 ? 128 : 32); }

int corr_grid(int, int) { return kCorrGrid; }

// Correlation kernel variants (BF16); 0 picks the default.
//   1: direct-to-LDS, BK 64, three stages, one workgroup per CU (N >= 16);
//   2: direct-to-LDS, BK 32, three stages, two workgroups per CU (N >= 16);
//   3: register-staged loads, BK 64, 256 x 128 tiles;
//   4: as 2 for N = 64; register-staged narrow node tiles (32 nodes) for
//      N <= 32, so that the few nodes x atoms of the small levels still
//      spread over every CU.
template <int N>
static void launch_corr_n(int precision, int variant, const void* atoms, const StepArgs& a, int nat, hipStream_t s) {
  using CB = typename std::conditional<(N >= 16), CfgBig, typename std::conditional<(N == 8), CfgMid, CfgSmall>::type>::type;
  using CF = typename std::conditional<(N >= 16), CfgBigF, typename std::conditional<(N == 8), CfgMidF, CfgSmallF>::type>::type;
  if (variant == 0) variant = kDefaultVariant;
  if constexpr (N <= 32 && N >= 8) {
    if (precision == AQMP_PREC_BF16 && variant == 4) {
      using CN = typename std::conditional<(N == 8), CfgNarrow8, CfgNarrow>::type;
      hipLaunchKernelGGL((k_corr_bf16<N, CN>), dim3(2 * kCorrGrid), dim3(256), 0, s, (const uint16_t*)atoms, a.r16,
                         a.act, a.act_count, a.keys, nat);
      return;
    }
  }
  if (variant == 4) variant = 2;
  if (precision == AQMP_PREC_BF16) {
    if constexpr (N >= 16) {
      if (variant == 1)
        hipLaunchKernelGGL((k_corr_bf16_dma<N, 64, 1>), dim3(kCorrGrid), dim3(256), 0, s, (const uint16_t*)atoms,
                           a.r16, a.act, a.act_count, a.keys, nat);
      else if (variant == 2)
        hipLaunchKernelGGL((k_corr_bf16_dma<N, 32, 2>), dim3(2 * kCorrGrid), dim3(256), 0, s, (const uint16_t*)atoms,
                           a.r16, a.act, a.act_count, a.keys, nat);
      else
        hipLaunchKernelGGL((k_corr_bf16<N, CB>), dim3(kCorrGrid), dim3(256), 0, s, (const uint16_t*)atoms, a.r16,
                           a.act, a.act_count, a.keys, nat);
    } else {
      hipLaunchKernelGGL((k_corr_bf16<N, CB>), dim3(kCorrGrid), dim3(256), 0, s, (const uint16_t*)atoms, a.r16,
                         a.act, a.act_count, a.keys, nat);
    }
  } else {
    hipLaunchKernelGGL((k_corr_f32<N, CF>), dim3(kCorrGrid), dim3(256), 0, s, (const float*)atoms, a.r32, a.act,
                       a.act_count, a.keys, nat);
  }
}

hipError_t launch_corr(int n, int precision, int variant, const void* dict_atoms, const StepArgs& a,
                       int32_t m_pad, hipStream_t s) {
  const int nat = m_pad / corr_atom_tile(n);
  switch (n) {
    case 4: launch_corr_n<4>(precision, variant, dict_atoms, a, nat, s); break;
    case 8: launch_corr_n<8>(precision, variant, dict_atoms, a, nat, s); break;
    case 16: launch_corr_n<16>(precision, variant, dict_atoms, a, nat, s); break;
    case 32: launch_corr_n<32>(precision, variant, dict_atoms, a, nat, s); break;
    case 64: launch_corr_n<64>(precision, variant, dict_atoms, a, nat, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aqmp
