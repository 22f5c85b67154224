// host_core.cpp - transform tables and the bitstream writer (no device code).
#include "host_core.h"

#include <zlib.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "aqmp.h"

namespace aqmp {

void dct_table(int n, double* t) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < n; ++k) {
    const double alpha = k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
    for (int m = 0; m < n; ++m) t[(size_t)k * n + m] = alpha * std::cos(pi / n * (m + 0.5) * k);
  }
}

void haar_table(int n, double* t) {
  std::vector<double> h(1, 1.0);
  int m = 1;
  const double s2 = std::sqrt(2.0);
  while (m < n) {
    const int m2 = 2 * m;
    std::vector<double> g((size_t)m2 * m2, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        g[(size_t)i * m2 + 2 * j] = h[(size_t)i * m + j] / s2;
        g[(size_t)i * m2 + 2 * j + 1] = h[(size_t)i * m + j] / s2;
      }
    for (int i = 0; i < m; ++i) {
      g[(size_t)(m + i) * m2 + 2 * i] = 1.0 / s2;
      g[(size_t)(m + i) * m2 + 2 * i + 1] = -1.0 / s2;
    }
    h.swap(g);
    m = m2;
  }
  std::memcpy(t, h.data(), sizeof(double) * (size_t)n * n);
}

namespace {

template <class T>
void put(std::vector<uint8_t>& b, T v) {
  uint8_t tmp[sizeof(T)];
  std::memcpy(tmp, &v, sizeof(T));
  b.insert(b.end(), tmp, tmp + sizeof(T));
}

int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}

int fail(std::string* err, const char* msg) {
  if (err) *err = msg;
  return AQMP_E_INVALID;
}

}  // namespace

int stream_write(const StreamHeader& hd, const StreamChannel* ch, int n_ch, double step,
                 std::vector<uint8_t>& raw, std::string* err) {
  if (n_ch < 1 || n_ch > 255 || !ch) return fail(err, "1..255 channels per stream");
  if (!(step >= 0.0) || !std::isfinite(step)) return fail(err, "step must be finite and >= 0");
  const int lmin = log2_exact(hd.n_min), lmax = log2_exact(hd.n_max);
  if (lmin < 0 || lmax < 0 || lmin > lmax || lmax > 255) return fail(err, "block range must be powers of two");
  if (hd.families < 0 || hd.families > 255) return fail(err, "family mask out of range");
  const bool quant = step > 0.0;
  const float step32 = (float)step;
  const double d = (double)step32;
  if (quant && !(d > 0.0)) return fail(err, "step rounds to zero in binary32");
  // widths: atom counts and quantised values, over the leaves of every channel
  int max_count = 0;
  double big = 0.0;
  for (int c = 0; c < n_ch; ++c) {
    if (ch[c].count && !ch[c].nodes) return fail(err, "null node list");
    if (ch[c].count > 0xffffffffu) return fail(err, "too many nodes in a channel");
    for (size_t i = 0; i < ch[c].count; ++i) {
      const StreamNode& nd = ch[c].nodes[i];
      if (nd.split) continue;
      if (nd.n_atoms < 0 || nd.n_atoms > 65535) return fail(err, "leaf atom count out of range");
      if (nd.n_atoms && (!nd.idx || !nd.coef)) return fail(err, "null atom list");
      max_count = std::max(max_count, nd.n_atoms);
      for (int t = 0; t < nd.n_atoms; ++t) {
        if (nd.idx[t] < 0 || nd.idx[t] > 65535) return fail(err, "atom index out of range");
        if (!std::isfinite(nd.coef[t])) return fail(err, "coefficient not finite");
        if (quant) big = std::max(big, std::fabs(std::nearbyint(nd.coef[t] / d)));
      }
    }
  }
  if (big > 2147483647.0) return fail(err, "step too small for 32-bit quantised values");
  const int cb = max_count > 255 ? 2 : 1;
  const int qb = quant ? (big <= 32767.0 ? 2 : 4) : 0;
  std::vector<uint8_t> b;
  b.insert(b.end(), {'A', 'Q', 'M', 'P'});
  put<uint8_t>(b, 1);
  put<uint8_t>(b, (uint8_t)hd.families);
  put<uint8_t>(b, quant ? 1 : 0);
  put<uint8_t>(b, (uint8_t)n_ch);
  put<uint32_t>(b, hd.w);
  put<uint32_t>(b, hd.h);
  put<uint8_t>(b, (uint8_t)lmin);
  put<uint8_t>(b, (uint8_t)lmax);
  put<uint8_t>(b, (uint8_t)cb);
  put<uint8_t>(b, (uint8_t)qb);
  if (quant) put<float>(b, step32);
  for (int c = 0; c < n_ch; ++c) {
    const StreamNode* nodes = ch[c].nodes;
    const size_t cnt = ch[c].count;
    uint32_t n_leaves = 0, n_atoms = 0;
    std::vector<uint8_t> bits;
    size_t nbits = 0;
    for (size_t i = 0; i < cnt; ++i) {
      if (nodes[i].n > hd.n_min) {
        if (nbits % 8 == 0) bits.push_back(0);
        if (nodes[i].split) bits.back() |= (uint8_t)(1u << (nbits % 8));
        ++nbits;
      }
      if (!nodes[i].split) {
        ++n_leaves;
        n_atoms += (uint32_t)nodes[i].n_atoms;
      }
    }
    put<uint32_t>(b, (uint32_t)cnt);
    put<uint32_t>(b, n_leaves);
    put<uint32_t>(b, n_atoms);
    b.insert(b.end(), bits.begin(), bits.end());
    for (size_t i = 0; i < cnt; ++i)
      if (!nodes[i].split) {
        if (cb == 1)
          put<uint8_t>(b, (uint8_t)nodes[i].n_atoms);
        else
          put<uint16_t>(b, (uint16_t)nodes[i].n_atoms);
      }
    for (size_t i = 0; i < cnt; ++i)
      if (!nodes[i].split)
        for (int t = 0; t < nodes[i].n_atoms; ++t) put<uint16_t>(b, (uint16_t)nodes[i].idx[t]);
    for (size_t i = 0; i < cnt; ++i)
      if (!nodes[i].split)
        for (int t = 0; t < nodes[i].n_atoms; ++t) {
          if (!quant) {
            put<float>(b, (float)nodes[i].coef[t]);
          } else {
            const double q = std::nearbyint(nodes[i].coef[t] / d);
            if (qb == 2)
              put<int16_t>(b, (int16_t)q);
            else
              put<int32_t>(b, (int32_t)q);
          }
        }
  }
  raw.swap(b);
  return AQMP_OK;
}

size_t stream_deflate_bound(size_t raw_bytes) { return (size_t)compressBound((uLong)raw_bytes); }

int stream_deflate(const std::vector<uint8_t>& raw, int level, std::vector<uint8_t>& z) {
  if (level < 0 || level > 9) return AQMP_E_INVALID;
  uLongf bound = compressBound((uLong)raw.size());
  std::vector<uint8_t> o(bound);
  if (compress2(o.data(), &bound, raw.data(), (uLong)raw.size(), level) != Z_OK) return AQMP_E_NOMEM;
  o.resize(bound);
  z.swap(o);
  return AQMP_OK;
}

}  // namespace aqmp
