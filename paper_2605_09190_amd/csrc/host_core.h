// host_core.h - the host-only parts of the library that need no device: the
// 1D transform tables of the dictionaries (Section 2.1) and the bitstream
// writer (encoder step (ii), Section 2.3).  Plain C++17 with no HIP header,
// so that the CPU tests can also build these files on their own with the
// address and undefined-behaviour sanitizers.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace aqmp {

// DCT-II rows: t[k*n + m] = alpha_k cos(pi/n (m + 1/2) k), alpha_0 = sqrt(1/n),
// alpha_k = sqrt(2/n).  t holds n*n doubles.
void dct_table(int n, double* t);

// Orthonormal Haar rows by the two-scale recursion H_1 = [1],
// H_2m = [H_m (x) (1, 1); I_m (x) (1, -1)] / sqrt(2); n a power of two,
// t holds n*n doubles.
void haar_table(int n, double* t);

// One node of a channel's quadtree in depth-first order.  A split node
// carries no atoms in the stream; a leaf's atoms are idx[0..n_atoms) with
// FP64 coefficients coef[0..n_atoms).
struct StreamNode {
  int32_t n;
  bool split;
  int32_t n_atoms;
  const int32_t* idx;
  const double* coef;
};

struct StreamChannel {
  const StreamNode* nodes;
  size_t count;
};

struct StreamHeader {
  int families;  // dictionary family mask
  uint32_t w, h;
  int n_min, n_max;  // powers of two
};

// The uncompressed stream: the 20-byte header ("AQMP", version 1, family
// mask, coefficient format, channel count, width, height, log2 N_min,
// log2 N_max, count width, quantised-value width), the binary32 step when
// step > 0 (coefficient format 1), then per channel the node, leaf and atom
// counts (u32 each), the split flags of the nodes with N > N_min (bit i of
// byte i/8), the leaves' atom counts (u8, or u16 when one exceeds 255), the
// atom indices (u16) and the coefficients: binary32 (format 0) or
// q = round-half-to-even(c / d) with d the step rounded to binary32, as
// int16 when every |q| <= 32767, else int32 (format 1).  All little-endian.
// Returns AQMP_OK or AQMP_E_INVALID with the reason in *err; raw is then
// unchanged.
int stream_write(const StreamHeader& hd, const StreamChannel* ch, int n_ch, double step,
                 std::vector<uint8_t>& raw, std::string* err);

// zlib stream (DEFLATE) of raw at the given level (0..9).  Returns AQMP_OK
// or AQMP_E_NOMEM.
int stream_deflate(const std::vector<uint8_t>& raw, int level, std::vector<uint8_t>& z);

// Upper bound of stream_deflate's output size for raw_bytes of input.
size_t stream_deflate_bound(size_t raw_bytes);

}  // namespace aqmp
