// kernels_tree.hip - the quadtree worklist on the device: stable stream
// compaction of the active nodes and split/child emission (Algorithm 2).
// All of it is integer work with a fixed result: a single-pass prefix sum
// with decoupled look-back keeps the original order of the kept items.
#include "internal.h"
#include "dev_common.h"

namespace aqmp {

namespace {

// One launch = one stable scan over op.count() items with 0/1 keep flags.
// Blocks take tiles in ticket order, so a block only ever waits on tiles
// owned by blocks that started before it.  Every wait is bounded; when a
// bound runs out the scan reports it through *err and continues (its output
// is then wrong, and the host turns the flag into an error).  The last block
// to finish clears the tile words and the tickets for the next launch.
template <class Op>
__device__ void stable_scan(Op& op, ScanState ss, int32_t* err) {
  __shared__ int s_tile, s_prefix, s_last;
  __shared__ int s_wsum[4];
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = atomicAdd(&ss.ticket[0], 1);
  __syncthreads();
  const int tile = s_tile;
  const int n = op.count();
  const int ntiles = (n + kScanTile - 1) / kScanTile;
  if (tile < ntiles) {
    const int base = tile * kScanTile + tid * 4;
    int f[4];
    int loc = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = base + j;
      f[j] = (i < n) ? op.keep(i) : 0;
      loc += f[j];
    }
    const int lane = tid & 63, w = tid >> 6;
    int x = loc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) s_wsum[w] = x;
    __syncthreads();
    int wpre = 0;
    for (int j = 0; j < w; ++j) wpre += s_wsum[j];
    const int agg = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    const int excl = wpre + x - loc;
    if (w == 0) {
      const int pre = lookback_wave(ss.tiles, tile, agg, err);
      if (lane == 0) s_prefix = pre;
    }
    __syncthreads();
    int pos = s_prefix + excl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (f[j]) op.emit(base + j, pos++);
    }
    if (tile == ntiles - 1 && tid == 0) op.total(s_prefix + agg);
  } else if (tile == 0 && tid == 0) {
    op.total(0);   // n == 0: nothing kept
  }
  // Completion count; the last block resets the shared scan state.
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const int done = atomicAdd(&ss.ticket[1], 1);
    s_last = (done == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (s_last) {
    const int used = ntiles > (int)gridDim.x ? ntiles : (int)gridDim.x;
    for (int i = tid; i < used && i < ss.ntiles_max; i += blockDim.x) ss.tiles[i] = 0ull;
    if (tid == 0) {
      ss.ticket[0] = 0;
      ss.ticket[1] = 0;
    }
  }
}

struct CompactOp {
  const int32_t* in_list;   // null = identity (item i is node i)
  const int32_t* in_count;
  const uint8_t* st;
  int32_t* out_list;
  int32_t* out_count;
  int32_t* clear;           // optional counter set to zero with the total
  __device__ int count() const { return *in_count; }
  __device__ int node(int i) const { return in_list ? in_list[i] : i; }
  __device__ int keep(int i) const { return st[node(i)] == ST_RUN ? 1 : 0; }
  __device__ void emit(int i, int pos) const { out_list[pos] = node(i); }
  __device__ void total(int t) const {
    *out_count = t;
    if (clear) *clear = 0;
  }
};

struct SplitOp {
  const JobDev* jobs;
  int32_t n_jobs;
  int32_t* bad;             // set when a node names a job outside the table
  LevelDev parent;
  const int32_t* parent_count;
  LevelDev child;
  int32_t child_ntop;
  int32_t* child_count;
  int32_t lg;
  __device__ int count() const { return *parent_count; }
  // Algorithm 2: refine when N > N_min and the node failed the test of its
  // split rule; the node's own atoms are then discarded by the exporter.
  __device__ int keep(int i) const {
    const int jb = parent.job[i];
    if ((unsigned)jb >= (unsigned)n_jobs) {
      atomicExch(bad, 1);
      return 0;
    }
    const JobDev& j = jobs[jb];
    const int n = 1 << lg;
    int s = 0;
    if (n > j.n_min) {
      if (j.split_rule == AQMP_SPLIT_R1)
        s = parent.e[i] >= j.eps2[lg];
      else
        s = parent.t[i] >= j.k[lg];
    }
    if (s) parent.st[i] = (uint8_t)(parent.st[i] | ST_SPLIT);
    return s;
  }
  // Children are the four quadrants of the original block, TL, TR, BL, BR.
  __device__ void emit(int i, int pos) const {
    const int h = 1 << (lg - 1);
    const int jb = parent.job[i], x = parent.x0[i], y = parent.y0[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = child_ntop + 4 * pos + q;
      child.job[c] = jb;
      child.x0[c] = x + (q & 1) * h;
      child.y0[c] = y + (q >> 1) * h;
    }
  }
  __device__ void total(int t) const { *child_count = child_ntop + 4 * t; }
};

__global__ __launch_bounds__(256) void k_compact(CompactOp op, ScanState ss, int32_t* err) {
  stable_scan(op, ss, err);
}

__global__ __launch_bounds__(256) void k_split_emit(SplitOp op, ScanState ss, int32_t* err) {
  stable_scan(op, ss, err);
}

// Word 0 = v, words 1 .. n-1 = 0: one thread per word.
__global__ __launch_bounds__(256) void k_head_zero_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = i == 0 ? v : 0u;
}

__global__ void k_init_counts(Counters* c, const int32_t* ntop) {
  const int i = threadIdx.x;
  if (i < kLevels) {
    c->count[i] = ntop[i];
    c->next[i] = 0;
  }
  if (i < 3) c->act[i] = 0;
  if (i == 0) c->scan_error = 0;
}

}  // namespace

hipError_t launch_init_counts(Counters* c, const int32_t* ntop_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_init_counts, dim3(1), dim3(64), 0, s, c, ntop_dev);
  return hipGetLastError();
}

hipError_t launch_head_zero_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  hipLaunchKernelGGL(k_head_zero_u32, dim3((unsigned)b), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

static int scan_blocks(int64_t cap) {
  int64_t b = (cap + kScanTile - 1) / kScanTile;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_compact(const int32_t* in_list, const int32_t* in_count, const uint8_t* st,
                          int32_t* out_list, int32_t* out_count, int32_t* clear_count, int64_t cap,
                          ScanState ss, int32_t* err, hipStream_t s) {
  CompactOp op{in_list, in_count, st, out_list, out_count, clear_count};
  hipLaunchKernelGGL(k_compact, dim3(scan_blocks(cap)), dim3(256), 0, s, op, ss, err);
  return hipGetLastError();
}

hipError_t launch_split_emit(const JobDev* jobs, int32_t n_jobs, LevelDev parent, const int32_t* parent_count,
                             LevelDev child, int32_t child_ntop, int32_t* child_count,
                             int32_t lg, int64_t cap, ScanState ss, int32_t* err, hipStream_t s) {
  SplitOp op{jobs, n_jobs, err, parent, parent_count, child, child_ntop, child_count, lg};
  hipLaunchKernelGGL(k_split_emit, dim3(scan_blocks(cap)), dim3(256), 0, s, op, ss, err);
  return hipGetLastError();
}

}  // namespace aqmp
