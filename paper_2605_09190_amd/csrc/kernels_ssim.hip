// kernels_ssim.hip - SSIM of two planes (Section 3's quality measure).
//
// SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
// C1 = (0.01 L)^2, C2 = (0.03 L)^2.
//   global : moments of the whole planes (population); the kernel returns the
//            five plane sums per workgroup, the host finishes the formula.
//   window7: the formula on every 7 x 7 window inside the plane (uniform
//            weights, sample moments), averaged over the windows.  A
//            workgroup stages a 38 x 38 input tile of both planes in LDS (FP64)
//            and evaluates 32 x 32 windows, four per thread.
// Both write one FP64 partial per workgroup; the host adds them in a fixed
// order, so the result is reproducible.
#include "internal.h"

namespace aqmp {

namespace {

constexpr int kTile = 32, kWin = 7, kHalo = kWin - 1, kIn = kTile + kHalo;

__device__ inline double load(const void* p, int dtype, int64_t stride, int y, int x) {
  const int64_t i = (int64_t)y * stride + x;
  return dtype == AQMP_F64 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_ssim_window(const void* a, int64_t sa, const void* b, int64_t sb, int dtype,
                                                     int w, int h, double c1, double c2, double* partial) {
  __shared__ double sx[kIn][kIn + 1], sy[kIn][kIn + 1];
  __shared__ double red[4];
  const int ow = w - kHalo, oh = h - kHalo;   // windows per row / column
  const int tx0 = blockIdx.x * kTile, ty0 = blockIdx.y * kTile;
  for (int i = threadIdx.x; i < kIn * kIn; i += 256) {
    const int yy = i / kIn, xx = i % kIn;
    const int gy = ty0 + yy, gx = tx0 + xx;
    const bool in = gy < h && gx < w;
    sx[yy][xx] = in ? load(a, dtype, sa, gy, gx) : 0.0;
    sy[yy][xx] = in ? load(b, dtype, sb, gy, gx) : 0.0;
  }
  __syncthreads();
  const double n = kWin * kWin, inv_n = 1.0 / n, inv_n1 = 1.0 / (n - 1.0);
  double acc = 0.0;
  const int lx = threadIdx.x % kTile;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ly = threadIdx.x / kTile + 8 * q;
    if (tx0 + lx >= ow || ty0 + ly >= oh) continue;
    double s_x = 0, s_y = 0, s_xx = 0, s_yy = 0, s_xy = 0;
#pragma unroll
    for (int dy = 0; dy < kWin; ++dy)
#pragma unroll
      for (int dx = 0; dx < kWin; ++dx) {
        const double u = sx[ly + dy][lx + dx], v = sy[ly + dy][lx + dx];
        s_x += u;
        s_y += v;
        s_xx = fma(u, u, s_xx);
        s_yy = fma(v, v, s_yy);
        s_xy = fma(u, v, s_xy);
      }
    const double mx = s_x * inv_n, my = s_y * inv_n;
    const double vx = (s_xx - s_x * mx) * inv_n1, vy = (s_yy - s_y * my) * inv_n1;
    const double cxy = (s_xy - s_x * my) * inv_n1;
    acc += ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2));
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_ssim_moments(const void* a, int64_t sa, const void* b, int64_t sb, int dtype,
                                                      int w, int h, double* partial) {
  __shared__ double red[4];
  double s[5] = {0, 0, 0, 0, 0};
  const int64_t total = (int64_t)w * h;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int y = (int)(i / w), x = (int)(i % w);
    const double u = load(a, dtype, sa, y, x), v = load(b, dtype, sb, y, x);
    s[0] += u;
    s[1] += v;
    s[2] = fma(u, u, s[2]);
    s[3] = fma(v, v, s[3]);
    s[4] = fma(u, v, s[4]);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double r = block_sum(s[k], red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * 5 + k] = r;
  }
}

}  // namespace

hipError_t launch_ssim(const aqmp_image& x, const aqmp_image& y, int mode, double c1, double c2, double* partial,
                       int* n_partial, hipStream_t s) {
  if (mode == AQMP_SSIM_WINDOW7) {
    const dim3 grid((x.w - kHalo + kTile - 1) / kTile, (x.h - kHalo + kTile - 1) / kTile);
    *n_partial = (int)(grid.x * grid.y);
    hipLaunchKernelGGL(k_ssim_window, grid, dim3(256), 0, s, x.dev_ptr, x.row_stride, y.dev_ptr, y.row_stride,
                       x.dtype, x.w, x.h, c1, c2, partial);
  } else {
    *n_partial = kSsimMomentBlocks;
    hipLaunchKernelGGL(k_ssim_moments, dim3(kSsimMomentBlocks), dim3(256), 0, s, x.dev_ptr, x.row_stride,
                       y.dev_ptr, y.row_stride, x.dtype, x.w, x.h, partial);
  }
  return hipGetLastError();
}

}  // namespace aqmp

// ---------------------------------------------------------------------------
// Host entry: validates, launches, and finishes the mean on the host.
// ---------------------------------------------------------------------------
#include "host_util.h"

namespace aqmp {

int ssim_planes(const aqmp_image* x, const aqmp_image* y, int mode, double data_range, double* out, hipStream_t s) {
  if (!x || !y || !out) AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: null argument");
  if (!x->dev_ptr || !y->dev_ptr) AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: plane without data");
  if (x->w != y->w || x->h != y->h || x->dtype != y->dtype)
    AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: the planes need one size and one dtype");
  if (x->dtype != AQMP_F32 && x->dtype != AQMP_F64) AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: bad dtype");
  if (x->row_stride < x->w || y->row_stride < y->w) AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: row stride too small");
  if (mode != AQMP_SSIM_GLOBAL && mode != AQMP_SSIM_WINDOW7) AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: bad mode");
  if (mode == AQMP_SSIM_WINDOW7 ? (x->w < 7 || x->h < 7) : (x->w < 1 || x->h < 1))
    AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: plane too small for the mode");
  if (!(data_range > 0.0) || !std::isfinite(data_range)) AQMP_FAIL(AQMP_E_INVALID, "aqmp_ssim: bad data_range");
  const double c1 = (0.01 * data_range) * (0.01 * data_range), c2 = (0.03 * data_range) * (0.03 * data_range);
  const size_t cap = mode == AQMP_SSIM_WINDOW7
                         ? (size_t)((x->w - 6 + 31) / 32) * (size_t)((x->h - 6 + 31) / 32)
                         : (size_t)kSsimMomentBlocks * 5;
  double* d_part = nullptr;
  int rc = dev_alloc((void**)&d_part, cap * sizeof(double));
  if (rc != AQMP_OK) return rc;
  int np = 0;
  hipError_t e = launch_ssim(*x, *y, mode, c1, c2, d_part, &np, s);
  std::vector<double> h(mode == AQMP_SSIM_WINDOW7 ? (size_t)np : (size_t)np * 5);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d_part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(d_part, cap * sizeof(double));
  if (e != hipSuccess) AQMP_FAIL(AQMP_E_HIP, std::string("aqmp_ssim: ") + hipGetErrorString(e));
  if (mode == AQMP_SSIM_WINDOW7) {
    double sum = 0.0;
    for (double v : h) sum += v;
    *out = sum / ((double)(x->w - 6) * (double)(x->h - 6));
  } else {
    double m[5] = {0, 0, 0, 0, 0};
    for (int b = 0; b < np; ++b)
      for (int k = 0; k < 5; ++k) m[k] += h[(size_t)b * 5 + k];
    const double n = (double)x->w * (double)x->h;
    const double mx = m[0] / n, my = m[1] / n;
    const double vx = m[2] / n - mx * mx, vy = m[3] / n - my * my, cxy = m[4] / n - mx * my;
    *out = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2));
  }
  return AQMP_OK;
}

}  // namespace aqmp
