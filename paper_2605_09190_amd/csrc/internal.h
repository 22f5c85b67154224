// internal.h - structures shared by the host orchestration and the kernels
// of the AQMP encoder library.  Not part of the public ABI (see aqmp.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "aqmp.h"

namespace aqmp {

// Node status byte.  The low two bits say why MP stopped (or that it is still
// running); ST_SPLIT is set by the split pass.
enum : uint8_t {
  ST_RUN = 0,       // MP continues at the next step
  ST_ACC = 1,       // stopped: ||r||^2 < eps_N^2 (eq. (2), accuracy)
  ST_SPARSE = 2,    // stopped: k_N iterations made (eq. (2), sparsity)
  ST_ZERO = 3,      // stopped: the largest |correlation| is exactly zero
  ST_SPLIT = 0x10,  // node refined into its four quadrants
};

constexpr int kLevels = 7;        // log2(N) for N = 1 .. 64
constexpr int kCand = AQMP_CANDIDATES;
constexpr int kTopR = 8;          // keys kept per node per atom tile
constexpr int kScanTile = 1024;   // items per block of the stable scans
constexpr int kFusedMaxN = 8;     // levels up to this size run the fused per-node pursuit
constexpr int kBranches = 4;      // parallel graph branches of the concurrent schedule
constexpr int kOmpMaxAtoms = AQMP_OMP_MAX_ATOMS;   // OMP: selected atoms per node (LDS factor size)
constexpr int kSsimMomentBlocks = 1024;   // workgroups of the whole-plane SSIM moments

// Kernel launch, with start/end events recorded by the dispatch when given.
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                         Args... args) {
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev0, ev1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

inline int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Per-job table read by the kernels.  eps2 and k are indexed by log2(N).
struct JobDev {
  const void* img;
  int32_t dtype;
  int32_t w, h;
  int32_t n_min, n_max;
  int32_t split_rule;
  int64_t row_stride;
  double eps2[kLevels];
  int32_t k[kLevels];
  int32_t pad;
};

// Pixel (y, x) of a job's plane in FP64.  Blocks tile the plane padded up
// to a multiple of N_max; rows and columns past the image repeat its last
// row and column (edge replication).
__device__ inline double job_pixel(const JobDev& jb, int y, int x) {
  y = y < jb.h ? y : jb.h - 1;
  x = x < jb.w ? x : jb.w - 1;
  const int64_t idx = (int64_t)y * jb.row_stride + x;
  return jb.dtype == AQMP_F64 ? ((const double*)jb.img)[idx] : (double)((const float*)jb.img)[idx];
}

// Host checks of one parameter set (AQMP_E_INVALID with tag + reason), and
// the per-job table entry the kernels read for a plane and a parameter set.
int check_params(const aqmp_params& p, const std::string& tag);
JobDev make_jobdev(const aqmp_image& im, const aqmp_params& p);

// Pixels (y, x0 .. x0 + W - 1) of a job's plane in FP64, edge-replicated
// like job_pixel.  The sample type is tested once and the W loads are
// independent, so they are all in flight together.
template <int W>
__device__ inline void job_pixels(const JobDev& jb, int y, int x0, double (&v)[W]) {
  const int yy = y < jb.h ? y : jb.h - 1;
  const int64_t row = (int64_t)yy * jb.row_stride;
  int xs[W];
#pragma unroll
  for (int j = 0; j < W; ++j) xs[j] = x0 + j < jb.w ? x0 + j : jb.w - 1;
  if (jb.dtype == AQMP_F64) {
    const double* p = (const double*)jb.img + row;
#pragma unroll
    for (int j = 0; j < W; ++j) v[j] = p[xs[j]];
  } else {
    const float* p = (const float*)jb.img + row;
#pragma unroll
    for (int j = 0; j < W; ++j) v[j] = (double)p[xs[j]];
  }
}

// Device-side arrays of one quadtree level (block size N = 1 << lg).  The
// node arrays are shared by all passes; a pass owns [base, base + cap).
struct LevelDev {
  int32_t* job;
  int32_t* x0;
  int32_t* y0;
  double* e;        // ||r||^2 after the last iteration (FP64)
  int32_t* t;       // iterations made
  uint8_t* st;      // ST_* status
  int32_t* rec_idx;   // [node * kmax + t] selected atom
  double* rec_coef;   // [node * kmax + t] FP64 coefficient
  int32_t kmax;
};

// Per-pass counters in device memory.
struct Counters {
  int32_t count[kLevels];   // nodes present at each level
  int32_t act[3];           // active-list lengths (rotating: in, out, cleared)
  int32_t scan_error;       // set if a bounded scan wait ran out
  int32_t next[kLevels];    // work counter of the dynamically scheduled kernels per level
};

// Look-back scan bookkeeping: one 64-bit word per tile plus two counters.
// The last block of every scan launch restores it to zero.
struct ScanState {
  unsigned long long* tiles;
  int32_t* ticket;   // [0] tile ticket, [1] blocks done
  int32_t ntiles_max;
};

// Arguments of the per-step kernels of one level.
struct StepArgs {
  const JobDev* jobs;
  LevelDev lv;            // already offset by the pass base
  int32_t lg;             // log2(N)
  int32_t n_atoms;        // M (real atoms; the correlation pads to its tile)
  int32_t nfam;
  const double* tab;      // FP64 1D tables [nfam][N][N]
  const float* tabT32;    // the same rounded to FP32 and transposed, [nfam][pixel][row]
  float* r32;             // residual [node][N*N] FP32, row-major pixels
  uint16_t* r16;          // BF16 shadow of r32 (null in the FP32 form)
  const int32_t* act;     // active list (node slots within the pass)
  const int32_t* act_count;
  unsigned long long* keys;   // [pos][atom tile][kTopR]
  int32_t n_atom_tiles;
  // The select step appends the nodes still running to next_act (any
  // order; zero on entry) and zeroes clear_count, the counter the step
  // after the next one appends to.  next_act is null on a level's last step.
  int32_t* next_act;
  int32_t* next_count;
  int32_t* clear_count;
  // Node-tile range of the generated-atom correlation: lo | hi << 4, 0 =
  // the kernel's own range.
  int32_t corr_tile;
};

// ---------------------------------------------------------------------------
// Launch wrappers (defined in the kernel translation units).
// ---------------------------------------------------------------------------
hipError_t launch_init_counts(Counters* c, const int32_t* ntop_dev, hipStream_t s);
// p[0] = v and p[1 .. n-1] = 0, by a fill kernel.
hipError_t launch_head_zero_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_gather(int n, const StepArgs& a, const int32_t* count, hipStream_t s);
hipError_t launch_compact(const int32_t* in_list, const int32_t* in_count, const uint8_t* st,
                          int32_t* out_list, int32_t* out_count, int32_t* clear_count, int64_t cap,
                          ScanState ss, int32_t* err, hipStream_t s);
// Split test and child emission of one level.  A node whose job index is not
// below n_jobs is not split and sets *err.
hipError_t launch_split_emit(const JobDev* jobs, int32_t n_jobs, LevelDev parent, const int32_t* parent_count,
                             LevelDev child, int32_t child_ntop, int32_t* child_count,
                             int32_t lg, int64_t cap, ScanState ss, int32_t* err, hipStream_t s);
// ev0 / ev1, when given, are recorded by the dispatch itself at the kernel's
// start and end (hipExtLaunchKernel), so their elapsed time is the kernel's
// execution time without the launch gap.
hipError_t launch_corr(int n, int precision, int variant, const void* dict_atoms, const StepArgs& a,
                       int32_t m_pad, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_select(int n, const StepArgs& a, int64_t cap, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
hipError_t launch_mp_fused(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t lg, int32_t n_atoms,
                           const double* tab, hipStream_t s);
// Whole-level BF16 pursuit of a level of N = 8 or 16 (next: the level's
// node counter, zero on entry; cap: the level's node capacity).
hipError_t launch_pursuit_bf16(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next,
                               int64_t cap, int32_t n_atoms, int32_t nfam, const double* tab, const float* tabT32,
                               hipStream_t s);
// Gram and OMP forms (FP64).  For N >= 16 launch_gram_init writes the
// correlations of every node of the level to cbuf ([node][nfam * n * n]) and
// sets its ||y||^2 and first stop test; the pursuit launches then take each
// node through its whole MP (Gram updates) or OMP (least-squares refits);
// for N <= 8 the pursuit launch does everything.  `next` is a zero-
// initialised work counter the pursuits hand out nodes from.
hipError_t launch_gram_init(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t lg, int32_t nfam,
                            const double* tab, double* cbuf, hipStream_t s);
hipError_t launch_gram_pursuit(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next, int32_t lg,
                               int32_t nfam, const double* tab, const double* xg, const double* cbuf, hipStream_t s);
// kmax: the largest k among the level's jobs (at most kOmpMaxAtoms); it
// sizes the factor in LDS.
hipError_t launch_omp_pursuit(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t* next, int32_t lg,
                              int32_t nfam, const double* tab, const double* xg, const double* cbuf, int32_t kmax,
                              hipStream_t s);
// SSIM partials: one FP64 per workgroup (window7) or five plane sums per
// workgroup (global); *n_partial receives the workgroup count.
hipError_t launch_ssim(const aqmp_image& x, const aqmp_image& y, int mode, double c1, double c2, double* partial,
                       int* n_partial, hipStream_t s);
int ssim_planes(const aqmp_image* x, const aqmp_image* y, int mode, double data_range, double* out, hipStream_t s);
// step > 0: every coefficient is replaced by its quantised value
// rint(c / step) * step first (the stream's coefficient format 1).
hipError_t launch_decode(int n, const JobDev* jobs, LevelDev lv, const int32_t* count, int32_t job,
                         int32_t nfam, const double* tab, double step, void* out, int32_t dtype,
                         int64_t row_stride, hipStream_t s);

// Device gather of a code's visited nodes in canonical order.  Sort key of a
// node: global top-level block ordinal << kExportLowBits | Morton code of its
// corner inside that block << 3 | (7 - log2 N).
constexpr int kExportCornerBits = 6;                       // corner coordinates < 64
constexpr int kExportLowBits = 2 * kExportCornerBits + 3;
struct ExportSeg {          // one level of one pass
  LevelDev L;               // offset by the pass base
  const int32_t* count;     // nodes present (device)
  int32_t lg;
  uint32_t flat_base;       // first flat node id of the segment
};
struct ExportJob {
  long long top_base;       // global ordinal of the job's first top-level block
  int32_t nm;               // N_max of the job
  int32_t cols;             // top-level blocks per row of the padded plane
};
hipError_t launch_export_keys(const ExportSeg* segs, int nseg, int64_t max_cap, const ExportJob* jx,
                              unsigned long long* keys, uint32_t* vals, unsigned long long* totals, hipStream_t s);
hipError_t export_sort(void* tmp, size_t& tmp_bytes, unsigned long long* keys, unsigned long long* keys_out,
                       uint32_t* vals, uint32_t* vals_out, int64_t n, int end_bit, hipStream_t s);
hipError_t export_scan(void* tmp, size_t& tmp_bytes, const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
hipError_t launch_export_counts(const ExportSeg* segs, int nseg, const uint32_t* vals, int64_t n, int64_t* t_out,
                                hipStream_t s);
hipError_t launch_export_write(const ExportSeg* segs, int nseg, const uint32_t* vals, const int64_t* off, int64_t n,
                               aqmp_leaf* out, int32_t* idx, double* coef, hipStream_t s);

// Name of the correlation kernel launch_corr runs (or the fused pursuit for
// n <= kFusedMaxN); "" when the combination is invalid.
const char* corr_kernel_name(int n, int precision, int variant);
// The BF16 correlation variants the library has: 0 (default), 2, 3, 6.
inline bool corr_variant_valid(int v) { return v == 0 || v == 2 || v == 3 || v == 6; }

// Tile geometry of the correlation kernel per block size (atoms per tile).
int corr_atom_tile(int n);
int corr_grid(int n, int precision);

}  // namespace aqmp

// Opaque public handles.
struct aqmp_dict {
  int n_min, n_max;
  uint32_t families;
  int nfam;
  struct Level {
    bool have = false;
    int n = 0, k = 0, m = 0, m_pad = 0;
    std::vector<double> h_tab;     // [nfam][n][n]
    double* d_tab = nullptr;
    float* d_tabT32 = nullptr;     // [nfam][y][p] = fl32(T_f[p][y])
    double* d_xg = nullptr;        // [n][n] <T_0[p], T_1[p']> (two families only)
    float* d_f32 = nullptr;        // [m_pad][k]
    uint16_t* d_bf16 = nullptr;    // [m_pad][k]
  } lv[aqmp::kLevels];
};
