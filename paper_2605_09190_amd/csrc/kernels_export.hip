// kernels_export.hip - a code's visited nodes gathered on the device in the
// canonical order of its readers (export, statistics, bitstream): job, then
// top-level block in raster order, then depth-first with the children of a
// node in TL, TR, BL, BR order (Alg. 2 recursion).  Depth-first order inside
// a top-level block is the order of (Morton code of the node's corner,
// larger node first), so one radix sort of a 64-bit key per node gives it.
// The host then reads three dense arrays (node records, atom indices,
// coefficients) instead of every level's fixed-stride record slots.
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "internal.h"
#include "dev_common.h"

namespace aqmp {

namespace {

// Morton code of a corner inside its top-level block: x in the even bits,
// so TL < TR < BL < BR at every level.
__device__ inline uint32_t corner_morton(uint32_t x, uint32_t y) {
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < kExportCornerBits; ++b) m |= (((x >> b) & 1u) << (2 * b)) | (((y >> b) & 1u) << (2 * b + 1));
  return m;
}

// Flat node id -> its segment (level of a pass), by binary search over the
// segments' first flat ids.
__device__ inline int seg_of(const ExportSeg* segs, int nseg, uint32_t fid) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].flat_base <= fid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One key and one flat id per visited node, appended in any order (the sort
// fixes the order); totals[0] counts nodes, totals[1] their MP iterations.
__global__ __launch_bounds__(256) void k_export_keys(const ExportSeg* segs, const ExportJob* jx,
                                                     unsigned long long* keys, uint32_t* vals,
                                                     unsigned long long* totals) {
  const ExportSeg sg = segs[blockIdx.y];
  const int count = *sg.count;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int base = blockIdx.x * 256; base < count; base += gridDim.x * 256) {
    const int i = base + (int)threadIdx.x;
    const bool v = i < count;
    unsigned long long key = 0;
    int t = 0;
    if (v) {
      const int job = sg.L.job[i];
      const ExportJob j = jx[job];
      const int x0 = sg.L.x0[i], y0 = sg.L.y0[i];
      const long long top = j.top_base + (long long)(y0 / j.nm) * j.cols + x0 / j.nm;
      key = ((unsigned long long)top << kExportLowBits) |
            ((unsigned long long)corner_morton((uint32_t)(x0 % j.nm), (uint32_t)(y0 % j.nm)) << 3) |
            (unsigned long long)(7 - sg.lg);
      t = sg.L.t[i];
    }
    const unsigned long long m = __ballot(v);
    const int rank = __popcll(m & below);
    int tsum = t;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) tsum += __shfl_xor(tsum, d, 64);
    unsigned long long slot = 0;
    if (lane == 0 && m) {
      slot = atomicAdd(&totals[0], (unsigned long long)__popcll(m));
      atomicAdd(&totals[1], (unsigned long long)tsum);
    }
    slot = __shfl(slot, 0, 64);
    if (v) {
      keys[slot + rank] = key;
      vals[slot + rank] = sg.flat_base + (uint32_t)i;
    }
  }
}

// Atom counts in sorted order (the scan's input).
__global__ __launch_bounds__(256) void k_export_counts(const ExportSeg* segs, int nseg, const uint32_t* vals,
                                                       int64_t n, int64_t* t_out) {
  for (int64_t p = blockIdx.x * 256ll + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
    const uint32_t fid = vals[p];
    const ExportSeg& sg = segs[seg_of(segs, nseg, fid)];
    t_out[p] = sg.L.t[fid - sg.flat_base];
  }
}

// One wave per node in sorted order: its record, then its atoms at the
// scanned offset.
__global__ __launch_bounds__(256) void k_export_write(const ExportSeg* segs, int nseg, const uint32_t* vals,
                                                      const int64_t* off, int64_t n, aqmp_leaf* out,
                                                      int32_t* idx, double* coef) {
  const int lane = threadIdx.x & 63;
  for (int64_t p = blockIdx.x * 4ll + (threadIdx.x >> 6); p < n; p += (int64_t)gridDim.x * 4) {
    const uint32_t fid = vals[p];
    const ExportSeg& sg = segs[seg_of(segs, nseg, fid)];
    const int64_t i = fid - sg.flat_base;
    const int t = sg.L.t[i];
    const int64_t o = off[p];
    if (lane == 0) {
      aqmp_leaf r;
      r.job = sg.L.job[i];
      r.x0 = sg.L.x0[i];
      r.y0 = sg.L.y0[i];
      r.n = 1 << sg.lg;
      r.n_atoms = t;
      r.flags = (sg.L.st[i] & ST_SPLIT) ? 1 : 0;
      r.atom_off = o;
      r.resid_sq = sg.L.e[i];
      out[p] = r;
    }
    const size_t rs = (size_t)i * sg.L.kmax;
    for (int r = lane; r < t; r += 64) {
      idx[o + r] = sg.L.rec_idx[rs + r];
      coef[o + r] = sg.L.rec_coef[rs + r];
    }
  }
}

int grid_1d(int64_t items, int per_block) {
  const int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

}  // namespace

hipError_t launch_export_keys(const ExportSeg* segs, int nseg, int64_t max_cap, const ExportJob* jx,
                              unsigned long long* keys, uint32_t* vals, unsigned long long* totals, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  const dim3 grid(grid_1d(max_cap, 256), nseg);
  hipLaunchKernelGGL(k_export_keys, grid, dim3(256), 0, s, segs, jx, keys, vals, totals);
  return hipGetLastError();
}

hipError_t export_sort(void* tmp, size_t& tmp_bytes, unsigned long long* keys, unsigned long long* keys_out,
                       uint32_t* vals, uint32_t* vals_out, int64_t n, int end_bit, hipStream_t s) {
  return rocprim::radix_sort_pairs(tmp, tmp_bytes, keys, keys_out, vals, vals_out, (size_t)n, 0u,
                                   (unsigned)end_bit, s);
}

hipError_t export_scan(void* tmp, size_t& tmp_bytes, const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return rocprim::exclusive_scan(tmp, tmp_bytes, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s);
}

hipError_t launch_export_counts(const ExportSeg* segs, int nseg, const uint32_t* vals, int64_t n, int64_t* t_out,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_counts, dim3(grid_1d(n, 256)), dim3(256), 0, s, segs, nseg, vals, n, t_out);
  return hipGetLastError();
}

hipError_t launch_export_write(const ExportSeg* segs, int nseg, const uint32_t* vals, const int64_t* off, int64_t n,
                               aqmp_leaf* out, int32_t* idx, double* coef, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_write, dim3(grid_1d(n, 4)), dim3(256), 0, s, segs, nseg, vals, off, n, out, idx,
                     coef);
  return hipGetLastError();
}

}  // namespace aqmp
