// worklist.hip - the integer steps of the quadtree worklist as calls of their
// own: the active-list compaction (the nodes whose pursuit goes on, Section
// 2.2 step (d)) and the split test with child emission (Algorithm 2).  They
// run the encoder's own scan kernels (kernels_tree.hip) on caller arrays, so
// that the integer work can be checked bit for bit on its own.
#include <mutex>
#include <string>
#include <vector>

#include "host_util.h"
#include "internal.h"

namespace aqmp {

namespace {

constexpr int64_t kWorklistMaxItems = (int64_t)1 << 28;

// Scan state of one call in one device block: four int32 (item count, the
// two tickets, the error flag), then the look-back tile words.
struct ScanBlock {
  int32_t* hdr = nullptr;
  ScanState ss{};
};

size_t scan_block_bytes(int64_t n) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  return 16 + 8 * (size_t)(ntiles + 2);
}

ScanBlock scan_block_at(void* p, int64_t n) {
  ScanBlock b;
  b.hdr = (int32_t*)p;
  b.ss.tiles = (unsigned long long*)((char*)p + 16);
  b.ss.ticket = b.hdr + 1;
  b.ss.ntiles_max = (int32_t)((n + kScanTile - 1) / kScanTile + 2);
  return b;
}

// Sets the item count and zeroes the rest of the block with one fill kernel,
// runs `launch`, reads the error flag back after the stream has drained.
// On a failed HIP call the stream is drained before returning, so the caller
// may release the block.
template <class F>
int run_scan(ScanBlock b, size_t bytes, int64_t n, hipStream_t s, const char* who, F launch) {
  int32_t err = 0;
  hipError_t e = launch_head_zero_u32((uint32_t*)b.hdr, (int64_t)(bytes / 4), (uint32_t)n, s);
  if (e == hipSuccess) e = launch(b);
  if (e == hipSuccess) e = hipMemcpyAsync(&err, b.hdr + 3, sizeof(err), hipMemcpyDeviceToHost, s);
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) AQMP_FAIL(AQMP_E_HIP, std::string(who) + ": " + hipGetErrorString(e));
  if (err)
    AQMP_FAIL(AQMP_E_HIP, std::string(who) + ": a bounded device wait ran out or a node names a parameter set "
                                             "outside the table");
  return AQMP_OK;
}

}  // namespace

int check_compact(const uint8_t* st, int64_t n, const int32_t* out, const int32_t* count, int64_t max_items,
                  const char* who) {
  if (n < 0 || n > max_items)
    AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": n must be in [0, " + std::to_string(max_items) + "]");
  if (!count || (n > 0 && (!st || !out))) AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": null argument");
  return AQMP_OK;
}

int compact_with(void* scratch, const uint8_t* st, int64_t n, int32_t* out, int32_t* count, hipStream_t s,
                 const char* who) {
  const ScanBlock b = scan_block_at(scratch, n);
  return run_scan(b, scan_block_bytes(n), n, s, who, [&](ScanBlock sb) {
    return launch_compact(nullptr, sb.hdr, st, out, count, nullptr, n, sb.ss, sb.hdr + 3, s);
  });
}

size_t compact_scratch_bytes(int64_t n) { return scan_block_bytes(n); }

int worklist_compact(const uint8_t* st, int64_t n, int32_t* out, int32_t* count, hipStream_t s) {
  const char* who = "aqmp_worklist_compact";
  int rc = check_compact(st, n, out, count, kWorklistMaxItems, who);
  if (rc != AQMP_OK) return rc;
  void* p = nullptr;
  const size_t bytes = scan_block_bytes(n);
  rc = dev_alloc(&p, bytes);
  if (rc != AQMP_OK) return rc;
  rc = compact_with(p, st, n, out, count, s, who);
  dev_free(p, bytes);
  return rc;
}

// ---------------------------------------------------------------------------
// Compaction without allocation.  The scan state lives in `scratch`, a
// file-scope device array of a fixed size (each device the library runs on
// holds its own copy until the process ends), sized for up to
// kNoAllocMaxItems items.  Host code never passes the array's name to a
// kernel: on the host it is a stand-in, not a device address.  The device
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, and kept in g_scratch_dev.  Calls on one device share the
// array, so calls that overlap on one device race; every call clears the
// part it uses before its scan.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxItems = (int64_t)1 << 24;
constexpr size_t kNoAllocBytes = (16 + 8 * (size_t)(kNoAllocMaxItems / kScanTile + 2) + 255) / 256 * 256;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static int scratch_for_current_device(void** out) {
  int dev = -1;
  AQMP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) AQMP_FAIL(AQMP_E_INVALID, "aqmp_worklist_compact_noalloc: device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      AQMP_FAIL(AQMP_E_HIP, std::string("aqmp_worklist_compact_noalloc: hipGetSymbolAddress: ") +
                                hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return AQMP_OK;
}

int worklist_compact_noalloc(const uint8_t* st, int64_t n, int32_t* out, int32_t* count, hipStream_t s) {
  const char* who = "aqmp_worklist_compact_noalloc";
  if (n > kNoAllocMaxItems)
    AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": n = " + std::to_string(n) + " exceeds the static scan state (at most " +
                                  std::to_string(kNoAllocMaxItems) + " items)");
  int rc = check_compact(st, n, out, count, kNoAllocMaxItems, who);
  if (rc != AQMP_OK) return rc;
  void* p = nullptr;
  rc = scratch_for_current_device(&p);
  if (rc != AQMP_OK) return rc;
  return compact_with(p, st, n, out, count, s, who);
}

int worklist_split(const aqmp_params* prm, int n_prm, int n, const int32_t* node_prm, const int32_t* x0,
                   const int32_t* y0, const double* e, const int32_t* t, int64_t n_nodes, int32_t child_base,
                   uint8_t* st, int32_t* child_prm, int32_t* child_x0, int32_t* child_y0, int32_t* child_count,
                   hipStream_t s) {
  const char* who = "aqmp_worklist_split";
  if (!prm || n_prm < 1) AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": no parameter sets");
  for (int i = 0; i < n_prm; ++i) {
    const int rc = check_params(prm[i], std::string(who) + ": params " + std::to_string(i) + ": ");
    if (rc != AQMP_OK) return rc;
  }
  if (n < 2 * AQMP_MIN_N || n > AQMP_MAX_N || (n & (n - 1)))
    AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": n must be a power of two in [8, 64]");
  if (n_nodes < 0 || n_nodes > kWorklistMaxItems)
    AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": n_nodes must be in [0, " + std::to_string(kWorklistMaxItems) + "]");
  if (child_base < 0 || (int64_t)child_base + 4 * n_nodes > (int64_t)INT32_MAX)
    AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": child_base + 4 n_nodes must fit in int32");
  if (!child_count || (n_nodes > 0 && (!node_prm || !x0 || !y0 || !e || !t || !st || !child_prm || !child_x0 ||
                                       !child_y0)))
    AQMP_FAIL(AQMP_E_INVALID, std::string(who) + ": null argument");
  std::vector<JobDev> table(n_prm);
  const aqmp_image none{};
  for (int i = 0; i < n_prm; ++i) table[i] = make_jobdev(none, prm[i]);
  const size_t scan_bytes = scan_block_bytes(n_nodes);
  const size_t bytes = scan_bytes + sizeof(JobDev) * table.size();
  void* p = nullptr;
  int rc = dev_alloc(&p, bytes);
  if (rc != AQMP_OK) return rc;
  JobDev* djobs = (JobDev*)((char*)p + scan_bytes);   // scan_bytes is a multiple of 8
  const hipError_t ce = hipMemcpyAsync(djobs, table.data(), sizeof(JobDev) * table.size(), hipMemcpyHostToDevice, s);
  if (ce != hipSuccess) {
    dev_free(p, bytes);
    AQMP_FAIL(AQMP_E_HIP, std::string(who) + ": upload failed: " + hipGetErrorString(ce));
  }
  LevelDev parent{};
  parent.job = const_cast<int32_t*>(node_prm);
  parent.x0 = const_cast<int32_t*>(x0);
  parent.y0 = const_cast<int32_t*>(y0);
  parent.e = const_cast<double*>(e);
  parent.t = const_cast<int32_t*>(t);
  parent.st = st;
  LevelDev child{};
  child.job = child_prm;
  child.x0 = child_x0;
  child.y0 = child_y0;
  const int lg = ilog2(n);
  const ScanBlock b = scan_block_at(p, n_nodes);
  rc = run_scan(b, scan_bytes, n_nodes, s, who, [&](ScanBlock sb) {
    return launch_split_emit(djobs, n_prm, parent, sb.hdr, child, child_base, child_count, lg, n_nodes, sb.ss,
                             sb.hdr + 3, s);
  });
  dev_free(p, bytes);
  return rc;
}

}  // namespace aqmp
