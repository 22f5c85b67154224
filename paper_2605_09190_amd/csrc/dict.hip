// dict.hip - dictionaries D_N (Section 2.1; Section 2.3 and Appendix A: a DCT
// basis concatenated with a Haar basis, one dictionary per block size).
//
// The 1D tables are computed on the host in FP64 (host_core.cpp):
//   DCT-II:  C[k][m] = alpha_k cos(pi/N (m + 1/2) k), alpha_0 = sqrt(1/N),
//            alpha_k = sqrt(2/N) (Section 2.1);
//   Haar:    H_1 = [1], H_2m = [H_m (x) (1, 1); I_m (x) (1, -1)] / sqrt(2)
//            (orthonormal, rows from the constant to the finest wavelets).
// Atom a = f N^2 + q N + p is T_f[p][y] T_f[q][x] (outer product of two 1D
// rows, Section 2.1); the constant atom of every family is exactly 1/N so
// that the two copies of it tie exactly in every precision.  The device keeps
// the FP64 tables (re-score, update, decode) and the atoms in FP32 (the FP64
// product rounded once) and BF16 (the FP32 product of the FP32-rounded table
// entries, rounded to BF16), atom-major with pixels row-major, padded with
// zero atoms to a whole number of correlation tiles.
#include <cmath>
#include <cstring>
#include <vector>

#include "dev_common.h"
#include "host_core.h"
#include "host_util.h"
#include "internal.h"

namespace aqmp {

static double atom_value(const aqmp_dict::Level& L, int a, int y, int x) {
  const int n = L.n, k = L.k;
  const int f = a / k, q = (a % k) / n, p = a % n;
  if (p == 0 && q == 0) return 1.0 / n;
  const double* t = L.h_tab.data() + (size_t)f * k;
  return t[p * n + y] * t[q * n + x];
}

// BF16 atom value: the FP32 product of the two table entries rounded to FP32,
// then rounded to BF16 (DC atoms exactly 1/N).  Kernels that build atoms from
// the tables on the fly compute exactly this.
static uint16_t atom_bf16(const aqmp_dict::Level& L, int a, int y, int x) {
  const int n = L.n, k = L.k;
  const int f = a / k, q = (a % k) / n, p = a % n;
  if (p == 0 && q == 0) return f32_to_bf16(1.0f / (float)n);
  const double* t = L.h_tab.data() + (size_t)f * k;
  const float v = (float)t[p * n + y] * (float)t[q * n + x];
  return f32_to_bf16(v);
}

static void free_level(aqmp_dict::Level& L) {
  if (L.d_tab) dev_free(L.d_tab, sizeof(double) * L.h_tab.size());
  if (L.d_tabT32) dev_free(L.d_tabT32, sizeof(float) * L.h_tab.size());
  if (L.d_xg) dev_free(L.d_xg, sizeof(double) * L.k);
  if (L.d_f32) dev_free(L.d_f32, sizeof(float) * (size_t)L.m_pad * L.k);
  if (L.d_bf16) dev_free(L.d_bf16, sizeof(uint16_t) * (size_t)L.m_pad * L.k);
  L = aqmp_dict::Level();
}

void dictionary_free(aqmp_dict* d) {
  if (!d) return;
  for (auto& L : d->lv) free_level(L);
  delete d;
}

int dictionary_build(int n_min, int n_max, uint32_t families, hipStream_t s, aqmp_dict** out) {
  if (!out) AQMP_FAIL(AQMP_E_INVALID, "aqmp_dictionary_build: out is null");
  *out = nullptr;
  auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  if (!pow2(n_min) || !pow2(n_max) || n_min < AQMP_MIN_N || n_max > AQMP_MAX_N || n_min > n_max)
    AQMP_FAIL(AQMP_E_INVALID, "aqmp_dictionary_build: need powers of two 4 <= n_min <= n_max <= 64");
  if (families == 0 || (families & ~(uint32_t)(AQMP_DCT | AQMP_HAAR)))
    AQMP_FAIL(AQMP_E_INVALID, "aqmp_dictionary_build: families must be AQMP_DCT and/or AQMP_HAAR");
  aqmp_dict* d = new (std::nothrow) aqmp_dict();
  if (!d) AQMP_FAIL(AQMP_E_NOMEM, "aqmp_dictionary_build: host allocation failed");
  d->n_min = n_min;
  d->n_max = n_max;
  d->families = families;
  d->nfam = ((families & AQMP_DCT) ? 1 : 0) + ((families & AQMP_HAAR) ? 1 : 0);
  for (int n = n_min; n <= n_max; n *= 2) {
    aqmp_dict::Level& L = d->lv[ilog2(n)];
    L.n = n;
    L.k = n * n;
    L.m = d->nfam * L.k;
    const int tile = corr_atom_tile(n);
    L.m_pad = (L.m + tile - 1) / tile * tile;
    L.h_tab.assign((size_t)d->nfam * L.k, 0.0);
    int f = 0;
    if (families & AQMP_DCT) dct_table(n, L.h_tab.data() + (size_t)(f++) * L.k);
    if (families & AQMP_HAAR) haar_table(n, L.h_tab.data() + (size_t)(f++) * L.k);
    std::vector<float> a32((size_t)L.m_pad * L.k, 0.0f);
    std::vector<uint16_t> a16((size_t)L.m_pad * L.k, 0);
    for (int a = 0; a < L.m; ++a)
      for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
          const size_t o = (size_t)a * L.k + y * n + x;
          a32[o] = (float)atom_value(L, a, y, x);
          a16[o] = atom_bf16(L, a, y, x);
        }
    std::vector<float> tT(L.h_tab.size());
    for (int fm = 0; fm < d->nfam; ++fm)
      for (int y = 0; y < n; ++y)
        for (int pp = 0; pp < n; ++pp)
          tT[(size_t)fm * L.k + y * n + pp] = (float)L.h_tab[(size_t)fm * L.k + pp * n + y];
    // Cross-family table of the Gram form: X[p][p'] = <T_0[p], T_1[p']>.
    // Both constant rows equal 1/sqrt(N) and every other row of either table
    // sums to zero, so row and column 0 are set exactly.
    std::vector<double> xg;
    if (d->nfam == 2) {
      xg.assign(L.k, 0.0);
      for (int p0 = 0; p0 < n; ++p0)
        for (int p1 = 0; p1 < n; ++p1) {
          long double acc = 0.0L;
          for (int y = 0; y < n; ++y)
            acc += (long double)L.h_tab[(size_t)p0 * n + y] * (long double)L.h_tab[(size_t)L.k + p1 * n + y];
          xg[(size_t)p0 * n + p1] = (p0 == 0 || p1 == 0) ? ((p0 == 0 && p1 == 0) ? 1.0 : 0.0) : (double)acc;
        }
    }
    int rc = dev_alloc((void**)&L.d_tab, sizeof(double) * L.h_tab.size());
    if (rc == AQMP_OK) rc = dev_alloc((void**)&L.d_tabT32, sizeof(float) * tT.size());
    if (rc == AQMP_OK && !xg.empty()) rc = dev_alloc((void**)&L.d_xg, sizeof(double) * xg.size());
    if (rc == AQMP_OK) rc = dev_alloc((void**)&L.d_f32, sizeof(float) * a32.size());
    if (rc == AQMP_OK) rc = dev_alloc((void**)&L.d_bf16, sizeof(uint16_t) * a16.size());
    if (rc != AQMP_OK) {
      dictionary_free(d);
      return rc;
    }
    L.have = true;
    hipError_t e = hipMemcpyAsync(L.d_tab, L.h_tab.data(), sizeof(double) * L.h_tab.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(L.d_f32, a32.data(), sizeof(float) * a32.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(L.d_bf16, a16.data(), sizeof(uint16_t) * a16.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(L.d_tabT32, tT.data(), sizeof(float) * tT.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && L.d_xg)
      e = hipMemcpyAsync(L.d_xg, xg.data(), sizeof(double) * xg.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      dictionary_free(d);
      AQMP_FAIL(AQMP_E_HIP, std::string("aqmp_dictionary_build: upload failed: ") + hipGetErrorString(e));
    }
  }
  *out = d;
  return AQMP_OK;
}

int dictionary_atoms(const aqmp_dict* d, int n, int* m_out) {
  if (!d || !m_out) AQMP_FAIL(AQMP_E_INVALID, "aqmp_dictionary_atoms: null argument");
  if (n < 1 || (n & (n - 1)) || n > AQMP_MAX_N || !d->lv[ilog2(n)].have)
    AQMP_FAIL(AQMP_E_NODICT, "aqmp_dictionary_atoms: block size not in the dictionary");
  *m_out = d->lv[ilog2(n)].m;
  return AQMP_OK;
}

int dictionary_copy(const aqmp_dict* d, int n, double* host_out) {
  if (!d || !host_out) AQMP_FAIL(AQMP_E_INVALID, "aqmp_dictionary_copy: null argument");
  if (n < 1 || (n & (n - 1)) || n > AQMP_MAX_N || !d->lv[ilog2(n)].have)
    AQMP_FAIL(AQMP_E_NODICT, "aqmp_dictionary_copy: block size not in the dictionary");
  const aqmp_dict::Level& L = d->lv[ilog2(n)];
  for (int a = 0; a < L.m; ++a)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) host_out[(size_t)a * L.k + (size_t)x * n + y] = atom_value(L, a, y, x);
  return AQMP_OK;
}

}  // namespace aqmp
