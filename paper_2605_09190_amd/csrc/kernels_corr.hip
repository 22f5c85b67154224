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

// Compare-exchange keeping the larger key first.
__device__ inline void cx(uint32_t& a, uint32_t& b) {
  const uint32_t hi = a > b ? a : b;
  b = a > b ? b : a;
  a = hi;
}

// Batcher's odd-even merge sort of eight keys, descending (19 exchanges).
__device__ inline void sort8_desc(uint32_t (&v)[8]) {
  cx(v[0], v[1]); cx(v[2], v[3]); cx(v[4], v[5]); cx(v[6], v[7]);
  cx(v[0], v[2]); cx(v[1], v[3]); cx(v[4], v[6]); cx(v[5], v[7]);
  cx(v[1], v[2]); cx(v[5], v[6]);
  cx(v[0], v[4]); cx(v[1], v[5]); cx(v[2], v[6]); cx(v[3], v[7]);
  cx(v[2], v[4]); cx(v[3], v[5]);
  cx(v[1], v[2]); cx(v[3], v[4]); cx(v[5], v[6]);
}

// a, b sorted descending -> a = the eight largest of both, descending: the
// pairwise maximum of a and reversed b is bitonic and holds the top eight;
// a bitonic merger (distances 4, 2, 1) sorts it.
__device__ inline void merge8_desc(uint32_t (&a)[8], const uint32_t (&b)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = a[i] > b[7 - i] ? a[i] : b[7 - i];
  cx(a[0], a[4]); cx(a[1], a[5]); cx(a[2], a[6]); cx(a[3], a[7]);
  cx(a[0], a[2]); cx(a[1], a[3]); cx(a[4], a[6]); cx(a[5], a[7]);
  cx(a[0], a[1]); cx(a[2], a[3]); cx(a[4], a[5]); cx(a[6], a[7]);
}

// Shared epilogue: accumulators -> per (node, atom tile) top-R keys.  Branch
// free: every lane sorts its keys of a node column in groups of eight and
// merges the groups, then the two half-waves and the WA waves are merged.
// Keys are unique (they carry the atom), so the result is the exact top R.
template <class C>
__device__ inline void epilogue(f32x16 (&acc)[C::MA][C::MB], uint32_t* sK, int a0, int a_tile,
                                int n_atom_tiles, int b0, int count, unsigned long long* keys) {
  constexpr int R = kTopR;
  static_assert(R == 8, "the sorting networks handle eight keys");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wa = w % C::WA, wb = w / C::WA;
  // 255 - local atom of accumulator (ma, r) = lb - (32 ma + 8 (r >> 2) + (r & 3))
  const uint32_t lb = 255u - (uint32_t)(wa * C::WTA + 4 * (lane >> 5));
#pragma unroll
  for (int mb = 0; mb < C::MB; ++mb) {
    uint32_t top[R];
#pragma unroll
    for (int g = 0; g < 2 * C::MA; ++g) {
      const int ma = g >> 1;
      uint32_t v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int r = 8 * (g & 1) + e;
        const uint32_t bits = __float_as_uint(acc[ma][mb][r]);
        v[e] = (bits & 0x7FFFFF00u) | (lb - (uint32_t)(32 * ma + 8 * (r >> 2) + (r & 3)));
      }
      sort8_desc(v);
      if (g == 0) {
#pragma unroll
        for (int j = 0; j < R; ++j) top[j] = v[j];
      } else {
        merge8_desc(top, v);
      }
    }
    // merge with the other half-wave (same node, other atom rows)
    uint32_t other[R];
#pragma unroll
    for (int j = 0; j < R; ++j) other[j] = __shfl_xor(top[j], 32, 64);
    merge8_desc(top, other);
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
#pragma unroll
    for (int q = 1; q < C::WA; ++q) {
      uint32_t v[R];
#pragma unroll
      for (int j = 0; j < R; ++j) v[j] = sK[(q * C::BB + nl) * R + j];
      merge8_desc(top, v);
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
// lgkmcnt(0) and vmcnt(n) together (gfx9 encoding, expcnt left alone).
#define AQMP_WAIT_VM_LGKM0(n) __builtin_amdgcn_s_waitcnt(((n) & 0xF) | (0x7 << 4) | ((((n) >> 4) & 0x3) << 14))

// DMA addressing: buffer loads with an SGPR resource per operand, a 32-bit
// per-lane byte offset (one VGPR each) and a wave-uniform SGPR offset for the
// row block and the k stage.  Out-of-range offsets read zeros, never fault.
constexpr int kBufWord3 = 0x00020000;   // raw buffer, 32-bit data format (gfx9)

template <class G>
struct DmaPtrs {
  const void* a_base;              // dictionary, all atoms
  const void* b_base;              // residual buffer
  int32_t a_bytes;                 // dictionary extent in bytes
  uint32_t a_sofs;                 // byte offset of this wave's first A row block (uniform)
  uint32_t a_off[2];               // lane offset in even / odd blocks
  uint32_t b_off[G::B_INS];        // lane offset of its node row per block
};

// One 16-byte-per-lane buffer load into LDS (lane l lands at lds + 16 l).
// Kept out of the templates: the host pass of the HIP compiler mishandles the
// buffer-resource builtins inside function template specializations that are
// reached from more than one call site.
__device__ inline void lds_dma16(const void* base, int bytes, char* lds, int voff, int soff) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kBufWord3);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)lds, 16, voff, soff, 0, 0);
}

template <class G, int K>
__device__ inline void dma_issue(const DmaPtrs<G>& p, char* sa, char* sb, int s) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kofs = s * G::BK * 2;
#pragma unroll
  for (int i = 0; i < G::A_INS; ++i) {
    const int blk = w * G::A_INS + i;
    lds_dma16(p.a_base, p.a_bytes, sa + blk * 1024, (int)p.a_off[i & 1], (int)p.a_sofs + i * G::RPB * K * 2 + kofs);
  }
#pragma unroll
  for (int i = 0; i < G::B_INS; ++i) {
    const int blk = w * G::B_INS + i;
    lds_dma16(p.b_base, (int)0xFFFFFFFFu, sb + blk * 1024, (int)p.b_off[i], kofs);
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
    const int wu = __builtin_amdgcn_readfirstlane(w);
    p.a_base = D;
    p.b_base = X;
    p.a_bytes = n_atom_tiles * G::BA * K * 2;
    p.a_sofs = (uint32_t)((a0 + wu * G::A_INS * G::RPB) * K * 2);
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int gc = dslot ^ G::swz(par * G::RPB + drow);
      p.a_off[par] = (uint32_t)((drow * K + gc * 8) * 2);
    }
#pragma unroll
    for (int i = 0; i < G::B_INS; ++i) {
      const int row = (w * G::B_INS + i) * G::RPB + drow;
      const int gc = dslot ^ G::swz(row);
      const int pos = min(b0 + row, count - 1);
      p.b_off[i] = (uint32_t)(((size_t)act[pos] * K + gc * 8) * 2);
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
// BF16, N = 32 and 64: atoms generated in registers (no dictionary traffic).
//
// Atom (f, p, q) is the outer product of rows p and q of the 1D table T_f, so
// its BF16 value at pixel (y, x) is RNE(fl32(T32_f[p][y] * T32_f[q][x])), the
// canonical BF16 dictionary (T32 = the FP64 table rounded to FP32; for the
// constant atom the product rounds to exactly 1/N in BF16).  A lane's MFMA
// rows keep the same (p, q) over the whole K loop: it holds the T32_f[q][x]
// values it needs in registers and reads T32_f[p][y] from LDS once per
// stage, then builds each 8-value A fragment with 8 multiplies and 4 packed
// conversions while the MFMAs of the previous k-step run.  A stage is 64
// pixels: one row at N = 64, two rows at N = 32.  Only the residual tile goes
// through LDS (direct-to-LDS buffer loads, four-buffer ring, the barrier
// that publishes stage s + 1 inside the last k-step of stage s).  The node
// tile is 32 MB nodes, MB picked per launch from the node count so that the
// tiles fill the workgroups in as few rounds as possible.  Same k order and
// epilogue as the other forms: the keys are bit-identical.
// ---------------------------------------------------------------------------
constexpr int kGenRing = 4;      // residual stages in LDS (prefetch distance 3)
constexpr int kGenMBMax = 7;     // node tile = 32 MB nodes, MB <= 7

// Geometry for block size N and a node tile of 32 MB nodes: tile 256 atoms x
// 32 MB nodes, BK = 64, the four waves side by side along the atoms (64
// atoms x 32 MB nodes each), so a wave makes only the A fragments of its own
// rows: 2 per k-step, shared by MB MFMAs.
template <int N_, int MB_>
struct GenGeo {
  static constexpr int N = N_, K = N * N;
  static constexpr int BA = 256, BB = 32 * MB_, BK = 64, WA = 4, WB = 1;
  static constexpr int WTA = BA / WA, WTB = BB / WB, MA = WTA / 32, MB = WTB / 32;
  static constexpr int ROWB = BK * 2, CPR = ROWB / 16, RPB = 1024 / ROWB;
  static constexpr int B_BYTES = BB * ROWB;
  static constexpr int B_INS = BB / RPB / 4;   // = MB loads per wave per stage
  static constexpr int RPS = BK / N;           // pixel rows per stage
  static constexpr int XPL = N >= 64 ? 32 : N / 2;   // distinct x per lane
  static constexpr bool QSHARED = N >= 64;     // both of a lane's rows share q
  static constexpr int NQ = QSHARED ? 1 : MA;
  static_assert(N == 32 || N == 64, "generated atoms for N = 32, 64");
  using C = Cfg<BA, BB, BK, WA, WB>;
  __device__ static int swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }
  // x index (into the lane's XPL values) of element j of k-step KK
  __device__ static constexpr int xi(int kk) { return ((kk * 16) % N) / 16 * 8; }
  __device__ static constexpr int row(int kk) { return (kk * 16) / N; }   // row within the stage
};
constexpr int kGenBufBytes = 32 * kGenMBMax * 128;   // one ring buffer (28 KB)

template <class G>
struct GenFrag {
  bf16x8 a[2][G::MA];
  bf16x8 b[2][G::MB];
};

// B fragments of k-step KK into parity slot P.
template <class G, int KK, int P>
__device__ inline void gen_read_b(GenFrag<G>& f, const char* sb, const int (&off)[4]) {
#pragma unroll
  for (int mb = 0; mb < G::MB; ++mb) f.b[P][mb] = *(const bf16x8*)(sb + mb * 32 * G::ROWB + off[KK]);
  __builtin_amdgcn_sched_barrier(0);   // the reads go out a whole k-step before their MFMAs
}

// A fragments of k-step KK for the row factors tp[ma][row in stage].
template <class G, int KK, int P>
__device__ inline void gen_make_a(GenFrag<G>& f, const float (&tp)[G::MA][G::RPS], const float (&tq)[G::NQ][G::XPL]) {
#pragma unroll
  for (int ma = 0; ma < G::MA; ++ma) {
    bf16x8 v;
    const int qi = G::QSHARED ? 0 : ma;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (__bf16)(tp[ma][G::row(KK)] * tq[qi][G::xi(KK) + j]);
    f.a[P][ma] = v;
  }
}

template <class G, int KK>
__device__ inline void gen_mfma(f32x16 (&acc)[G::MA][G::MB], const GenFrag<G>& f) {
  constexpr int P = KK & 1;
#pragma unroll
  for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
    for (int ma = 0; ma < G::MA; ++ma)
      acc[ma][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[P][ma], f.b[P][mb], acc[ma][mb], 0, 0, 0);
}

// Residual rows of stage s: loads [first, first + cnt) of the wave's B_INS.
template <class G>
__device__ inline void gen_dma(const DmaPtrs<G>& p, char* sb, int s, int first, int cnt) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kofs = s * G::BK * 2;
#pragma unroll
  for (int i = 0; i < G::B_INS; ++i)
    if (i >= first && i < first + cnt)
      lds_dma16(p.b_base, (int)0xFFFFFFFFu, sb + (w * G::B_INS + i) * 1024, (int)p.b_off[i], kofs);
}

// Row factors T32_f[p_ma][y] of the rows of stage s.
template <class G>
__device__ inline void gen_row_factors(float (&tp)[G::MA][G::RPS], const float* sTf, const int (&pl)[G::MA], int s) {
#pragma unroll
  for (int ma = 0; ma < G::MA; ++ma)
#pragma unroll
    for (int r = 0; r < G::RPS; ++r) tp[ma][r] = sTf[(s * G::RPS + r) * G::N + pl[ma]];
}

// One stage s computed from cb.  DMA: the loads of stage s_dma go to db,
// spread over the first two k-steps.  NEXT: stage s + 1 follows in nb; its
// loads are complete once at most VMN of this wave's loads are outstanding
// (loads complete in order), and its first fragments are made here, under
// the last MFMAs of stage s.
template <class G, bool DMA, bool NEXT, int VMN>
__device__ inline void gen_stage(f32x16 (&acc)[G::MA][G::MB], GenFrag<G>& f, const DmaPtrs<G>& p, const float* sTf,
                                 const int (&pl)[G::MA], const float (&tq)[G::NQ][G::XPL], float (&tp)[G::MA][G::RPS],
                                 const char* cb, const char* nb, char* db, int s, int s_dma, const int (&off)[4]) {
  constexpr int H1 = (G::B_INS + 1) / 2;
  gen_read_b<G, 1, 1>(f, cb, off);
  gen_make_a<G, 1, 1>(f, tp, tq);
  if constexpr (DMA) gen_dma<G>(p, db, s_dma, 0, H1);
  gen_mfma<G, 0>(acc, f);
  gen_read_b<G, 2, 0>(f, cb, off);
  gen_make_a<G, 2, 0>(f, tp, tq);
  if constexpr (DMA) gen_dma<G>(p, db, s_dma, H1, G::B_INS - H1);
  gen_mfma<G, 1>(acc, f);
  gen_read_b<G, 3, 1>(f, cb, off);
  gen_make_a<G, 3, 1>(f, tp, tq);
  float tpn[G::MA][G::RPS];
  if constexpr (NEXT) gen_row_factors<G>(tpn, sTf, pl, s + 1);
  gen_mfma<G, 2>(acc, f);
  if constexpr (NEXT) {
    // every wave is done reading cb before any wave passes, so loads issued
    // after this barrier may overwrite it
    AQMP_WAIT_VM_LGKM0(VMN);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ma = 0; ma < G::MA; ++ma)
#pragma unroll
      for (int r = 0; r < G::RPS; ++r) tp[ma][r] = tpn[ma][r];
    gen_read_b<G, 0, 0>(f, nb, off);
    gen_make_a<G, 0, 0>(f, tp, tq);
  }
  gen_mfma<G, 3>(acc, f);
}

// The ring buffers are separate LDS arrays: the compiler then knows that a
// load into one buffer cannot feed a read of another, and does not wait for
// the loads in flight before every fragment read.
struct GenRing {
  char* r0;
  char* r1;
  char* r2;
  char* r3;
  template <int I>
  __device__ char* buf() const {
    static_assert(kGenRing == 4, "four ring buffers");
    if constexpr (I == 0) return r0;
    else if constexpr (I == 1) return r1;
    else if constexpr (I == 2) return r2;
    else return r3;
  }
};

template <class G>
struct GenLane {
  const float* sTf;
  int pl[G::MA];
  float tq[G::NQ][G::XPL];
};

// Stages S .. NST - 1 with every decision at compile time.
template <class G, int NST, int S>
__device__ inline void gen_tail(f32x16 (&acc)[G::MA][G::MB], GenFrag<G>& f, const DmaPtrs<G>& p,
                                const GenLane<G>& ln, const GenRing& rg, float (&tp)[G::MA][G::RPS],
                                const int (&off)[4]) {
  if constexpr (S < NST) {
    constexpr int NB = kGenRing;
    constexpr bool DMA = S + NB - 1 < NST;
    constexpr bool NEXT = S + 1 < NST;
    constexpr int AHEAD = (NST - 2 - S) < (NB - 2) ? (NST - 2 - S) : (NB - 2);
    constexpr int VMN = NEXT ? G::B_INS * (AHEAD > 0 ? AHEAD : 0) : 0;
    gen_stage<G, DMA, NEXT, VMN>(acc, f, p, ln.sTf, ln.pl, ln.tq, tp, rg.template buf<S % NB>(),
                                 rg.template buf<(S + 1) % NB>(), rg.template buf<(S + NB - 1) % NB>(), S, S + NB - 1,
                                 off);
    gen_tail<G, NST, S + 1>(acc, f, p, ln, rg, tp, off);
  }
}

// NB consecutive steady-state stages s0 + I (s0 a multiple of NB).
template <class G, int I>
__device__ inline void gen_trip(f32x16 (&acc)[G::MA][G::MB], GenFrag<G>& f, const DmaPtrs<G>& p,
                                const GenLane<G>& ln, const GenRing& rg, float (&tp)[G::MA][G::RPS],
                                const int (&off)[4], int s0) {
  if constexpr (I < kGenRing) {
    constexpr int NB = kGenRing;
    gen_stage<G, true, true, G::B_INS * (NB - 2)>(acc, f, p, ln.sTf, ln.pl, ln.tq, tp, rg.template buf<I>(),
                                                   rg.template buf<(I + 1) % NB>(),
                                                   rg.template buf<(I + NB - 1) % NB>(), s0 + I, s0 + I + NB - 1,
                                                   off);
    gen_trip<G, I + 1>(acc, f, p, ln, rg, tp, off, s0);
  }
}

// The FP32 tables (nfam N x N, 1 KB blocks) into sT by direct-to-LDS loads,
// block c = 4 i + wave, issued at kernel entry: no registers, and their
// round trip overlaps that of the first tile's active-list loads.
template <int N>
__device__ inline void gen_table_dma(const float* tabT32, int nfam, float* sT) {
  constexpr int MAXB = 2 * N * N * 4 / 1024;   // blocks of both families
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nb = nfam * N * N * 4 / 1024;
#pragma unroll
  for (int i = 0; i < MAXB / 4; ++i) {
    const int c = 4 * i + w;
    if (c < nb) lds_dma16(tabT32, nb * 1024, (char*)sT + c * 1024, lane * 16, c * 1024);
  }
}

// Every tile of one launch with node tiles of 32 MB nodes.
template <int N, int MB>
__device__ void gen_tiles(const uint16_t* __restrict__ X, const int32_t* __restrict__ act, int count,
                          unsigned long long* __restrict__ keys, int n_atom_tiles, int nfam, const float* sT,
                          const GenRing& rg) {
  using G = GenGeo<N, MB>;
  constexpr int K = G::K, NST = K / G::BK, NB = kGenRing;
  static_assert(NST >= NB, "ring shorter than the K loop");
  static_assert(G::B_BYTES <= kGenBufBytes, "stage fits a ring buffer");
  static_assert(G::WA * G::BB * kTopR * 4 <= kGenBufBytes, "epilogue scratch fits one ring buffer");
  uint32_t* sK = (uint32_t*)rg.r0;
  const int ntB = (count + G::BB - 1) / G::BB;
  const int ntiles = n_atom_tiles * ntB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wa = w, rr = lane & 31, hh = lane >> 5;
  const int fr = G::swz(rr);
  int off[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) off[kk] = rr * G::ROWB + (((2 * kk + hh) ^ fr) << 4);
  const int drow = lane / G::CPR, dslot = lane % G::CPR;
  TileWalk walk(ntiles);
  for (int j = walk.slot; j < walk.chunk; j += walk.per) {
    const int tile = walk.tile(j);
    if (tile >= ntiles) break;
    // node-major order: the workgroups of one XCD share a residual tile in
    // its L2 (the atoms cost no memory traffic here)
    const int a_tile = tile % n_atom_tiles, b_tile = tile / n_atom_tiles;
    const int a0 = a_tile * G::BA, b0 = b_tile * G::BB;
    DmaPtrs<G> p;
    p.b_base = X;
#pragma unroll
    for (int i = 0; i < G::B_INS; ++i) {
      const int row = (w * G::B_INS + i) * G::RPB + drow;
      const int gc = dslot ^ G::swz(row);
      const int pos = min(b0 + row, count - 1);
      p.b_off[i] = (uint32_t)(((size_t)act[pos] * K + gc * 8) * 2);
    }
    // The table blocks (loaded before the active-list entries, and loads
    // complete in order) have landed in every wave; the previous tile's
    // epilogue is done with sK (= buffer 0).
    AQMP_WAIT_VM(G::B_INS);
    __syncthreads();
    // Rows of this lane: atom a0 + 64 wa + 32 ma + rr of family fam, i.e.
    // q = qb + (64 wa + 32 ma + rr) / N, p = (64 wa + 32 ma + rr) % N.
    GenLane<G> ln;
    const int fam = min(a0 / K, nfam - 1);
    const int qb = (a0 % K) / N;
    ln.sTf = sT + fam * K;
    int ql[G::MA];
#pragma unroll
    for (int ma = 0; ma < G::MA; ++ma) {
      const int ri = 64 * wa + 32 * ma + rr;
      ql[ma] = qb + ri / N;
      ln.pl[ma] = ri % N;
    }
#pragma unroll
    for (int qi = 0; qi < G::NQ; ++qi)
#pragma unroll
      for (int kk = 0; kk < (G::XPL / 8); ++kk)
#pragma unroll
        for (int e = 0; e < 8; ++e) ln.tq[qi][kk * 8 + e] = ln.sTf[(kk * 16 + 8 * hh + e) * N + ql[qi]];
    float tp[G::MA][G::RPS];
    gen_row_factors<G>(tp, ln.sTf, ln.pl, 0);
    f32x16 acc[G::MA][G::MB];
#pragma unroll
    for (int ma = 0; ma < G::MA; ++ma)
#pragma unroll
      for (int mb = 0; mb < G::MB; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[ma][mb][r] = 0.f;
    GenFrag<G> f;

    gen_dma<G>(p, rg.template buf<0>(), 0, 0, G::B_INS);
    gen_dma<G>(p, rg.template buf<1>(), 1, 0, G::B_INS);
    gen_dma<G>(p, rg.template buf<2>(), 2, 0, G::B_INS);
    AQMP_WAIT_VM(G::B_INS * (NB - 2));
    __builtin_amdgcn_s_barrier();
    gen_read_b<G, 0, 0>(f, rg.template buf<0>(), off);
    gen_make_a<G, 0, 0>(f, tp, ln.tq);
    constexpr int FULL = NST - (NB - 1);      // stages that issue a load
    constexpr int TRIPS = FULL / NB;
    for (int t = 0; t < TRIPS; ++t) gen_trip<G, 0>(acc, f, p, ln, rg, tp, off, t * NB);
    gen_tail<G, NST, TRIPS * NB>(acc, f, p, ln, rg, tp, off);
    __syncthreads();   // all waves done reading the ring before sK reuses buffer 0
    epilogue<typename G::C>(acc, sK, a0, a_tile, n_atom_tiles, b0, count, keys);
  }
}

// Node-tile width for this launch: the fewest 32-node block-rounds over the
// workgroups (rounds x MB), ties to the wider tile.  Every workgroup computes
// the same value from the count.
__device__ inline int gen_pick_mb(int count, int n_atom_tiles, int wgs, int mb_min, int mb_max) {
  int best = mb_max, best_cost = 0x7fffffff;
  for (int mb = mb_max; mb >= mb_min; --mb) {
    const int tiles = n_atom_tiles * ((count + 32 * mb - 1) / (32 * mb));
    const int cost = ((tiles + wgs - 1) / wgs) * mb;
    if (cost < best_cost) {
      best_cost = cost;
      best = mb;
    }
  }
  return best;
}

template <int N>
__global__ __launch_bounds__(256, 1) void k_corr_bf16_gen(const float* __restrict__ tabT32, int nfam,
                                                          const uint16_t* __restrict__ X,
                                                          const int32_t* __restrict__ act,
                                                          const int32_t* __restrict__ act_count,
                                                          unsigned long long* __restrict__ keys, int n_atom_tiles,
                                                          int tile_range) {
  constexpr int K = N * N;
  __shared__ __attribute__((aligned(1024))) char sR0[kGenBufBytes];
  __shared__ __attribute__((aligned(1024))) char sR1[kGenBufBytes];
  __shared__ __attribute__((aligned(1024))) char sR2[kGenBufBytes];
  __shared__ __attribute__((aligned(1024))) char sR3[kGenBufBytes];
  __shared__ __attribute__((aligned(16))) float sT[2 * K];   // [f][y][p] = fl32(T_f[p][y])
  gen_table_dma<N>(tabT32, nfam, sT);
  const int count = *act_count;
  if (count <= 0) {
    AQMP_WAIT_VM(0);   // no load into LDS outlives the workgroup
    return;
  }
  const GenRing rg{sR0, sR1, sR2, sR3};
  // node-tile range: the tuned one when given, else 3..7 (N = 64), 1..7 (N = 32)
  const int mb_lo = tile_range ? (tile_range & 0xF) : (N == 64 ? 3 : 1);
  const int mb_hi = tile_range ? (tile_range >> 4) : kGenMBMax;
  if constexpr (N == 64) {
    switch (gen_pick_mb(count, n_atom_tiles, gridDim.x, mb_lo, mb_hi)) {
      case 1: gen_tiles<N, 1>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 2: gen_tiles<N, 2>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 3: gen_tiles<N, 3>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 4: gen_tiles<N, 4>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 5: gen_tiles<N, 5>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 6: gen_tiles<N, 6>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      default: gen_tiles<N, 7>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
    }
  } else {
    switch (gen_pick_mb(count, n_atom_tiles, gridDim.x, mb_lo, mb_hi)) {
      case 1: gen_tiles<N, 1>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 2: gen_tiles<N, 2>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 3: gen_tiles<N, 3>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 4: gen_tiles<N, 4>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 5: gen_tiles<N, 5>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      case 6: gen_tiles<N, 6>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
      default: gen_tiles<N, 7>(X, act, count, keys, n_atom_tiles, nfam, sT, rg); break;
    }
  }
  AQMP_WAIT_VM(0);   // a workgroup without a tile still waits for its table loads
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
using CfgMid = Cfg<128, 128, 64, 2, 2>;     // N = 8, BF16
using CfgSmall = Cfg<32, 256, 16, 1, 4>;    // N = 4, BF16
using CfgBigF = Cfg<256, 128, 32, 2, 2>;    // N >= 16, FP32
using CfgMidF = Cfg<128, 128, 32, 2, 2>;    // N = 8, FP32
using CfgSmallF = Cfg<32, 256, 16, 1, 4>;   // N = 4, FP32

constexpr int kCorrGrid = 256;   // one persistent workgroup per CU
// Default BF16 kernel per block size (measured): generated atoms at N = 32
// and 64; two workgroups per CU at N = 16 (used by the step-by-step path),
// where K (four stages) is too short for one workgroup's pipeline fill.
constexpr int default_variant(int n) { return n >= 32 ? 6 : 2; }

}  // namespace

int corr_atom_tile(int n) { return n >= 16 ? 256 : (n == 8 ? 128 : 32); }

int corr_grid(int, int) { return kCorrGrid; }

// Correlation kernel variants (BF16); 0 picks the default.  All sum the same
// products in the same order, so the keys are bit-identical.
//   2: direct-to-LDS loads, BK 32, three stages, two workgroups per CU
//      (N >= 16; the default of the step-by-step N = 16 level);
//   3: register-staged loads, BK 64, 256 x 128 tiles (every N; the form
//      used when a residual buffer exceeds the 32-bit offsets of the
//      direct-to-LDS loads);
//   6: atoms generated in registers (N = 32, 64; the default there).
// Numbers 1, 4 and 5 named forms that never won a timing (one workgroup per
// CU with BK 64, narrow register-staged tiles, a two-operand software
// pipeline) and were removed; they are rejected.
template <int N>
static void launch_corr_n(int precision, int variant, const void* atoms, const StepArgs& a, int nat, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1) {
  using CB = typename std::conditional<(N >= 16), CfgBig, typename std::conditional<(N == 8), CfgMid, CfgSmall>::type>::type;
  using CF = typename std::conditional<(N >= 16), CfgBigF, typename std::conditional<(N == 8), CfgMidF, CfgSmallF>::type>::type;
  if (variant == 0) variant = default_variant(N);
  if (precision == AQMP_PREC_BF16) {
    if constexpr (N >= 16) {
      if (variant == 6 && N >= 32)
        launch_timed((k_corr_bf16_gen<(N >= 32 ? N : 32)>), dim3(kCorrGrid), dim3(256), s, e0, e1, a.tabT32,
                           a.nfam, a.r16, a.act, a.act_count, a.keys, nat, (int)a.corr_tile);
      else if (variant == 2)
        launch_timed((k_corr_bf16_dma<N, 32, 2>), dim3(2 * kCorrGrid), dim3(256), s, e0, e1, (const uint16_t*)atoms,
                           a.r16, a.act, a.act_count, a.keys, nat);
      else
        launch_timed((k_corr_bf16<N, CB>), dim3(kCorrGrid), dim3(256), s, e0, e1, (const uint16_t*)atoms, a.r16,
                           a.act, a.act_count, a.keys, nat);
    } else {
      launch_timed((k_corr_bf16<N, CB>), dim3(kCorrGrid), dim3(256), s, e0, e1, (const uint16_t*)atoms, a.r16,
                         a.act, a.act_count, a.keys, nat);
    }
  } else {
    launch_timed((k_corr_f32<N, CF>), dim3(kCorrGrid), dim3(256), s, e0, e1, (const float*)atoms, a.r32, a.act,
                       a.act_count, a.keys, nat);
  }
}

const char* corr_kernel_name(int n, int precision, int variant) {
  if (n < AQMP_MIN_N || n > AQMP_MAX_N || (n & (n - 1))) return "";
  if (!corr_variant_valid(variant)) return "";
  if (precision != AQMP_PREC_FP32 && precision != AQMP_PREC_BF16) return "";
  static const char* const fused[] = {"", "", "k_mp_fused<4>", "k_mp_fused<8>"};
  if (n == 8 && precision == AQMP_PREC_BF16) return "k_pursuit8_bf16<16>";
  if (n <= kFusedMaxN) return fused[ilog2(n)];
  static const char* const f32[] = {"k_corr_f32<16>", "k_corr_f32<32>", "k_corr_f32<64>"};
  const int li = ilog2(n) - 4;
  if (precision == AQMP_PREC_FP32) return f32[li];
  if (variant == 0) variant = default_variant(n);
  static const char* const v2[] = {"k_corr_bf16_dma<16,32,2>", "k_corr_bf16_dma<32,32,2>", "k_corr_bf16_dma<64,32,2>"};
  static const char* const v3[] = {"k_corr_bf16<16>", "k_corr_bf16<32>", "k_corr_bf16<64>"};
  if (variant == 2) return v2[li];
  if (variant == 6) return n == 64 ? "k_corr_bf16_gen<64>" : (n == 32 ? "k_corr_bf16_gen<32>" : v3[li]);
  return v3[li];
}

hipError_t launch_corr(int n, int precision, int variant, const void* dict_atoms, const StepArgs& a,
                       int32_t m_pad, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const int nat = m_pad / corr_atom_tile(n);
  switch (n) {
    case 4: launch_corr_n<4>(precision, variant, dict_atoms, a, nat, s, ev0, ev1); break;
    case 8: launch_corr_n<8>(precision, variant, dict_atoms, a, nat, s, ev0, ev1); break;
    case 16: launch_corr_n<16>(precision, variant, dict_atoms, a, nat, s, ev0, ev1); break;
    case 32: launch_corr_n<32>(precision, variant, dict_atoms, a, nat, s, ev0, ev1); break;
    case 64: launch_corr_n<64>(precision, variant, dict_atoms, a, nat, s, ev0, ev1); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aqmp
