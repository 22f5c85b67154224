// api.hip - the extern "C" entry points declared in aqmp.h: argument
// marshalling, error state and the device allocation cap.  Every computation
// runs in the kernels behind encode.hip / dict.hip.
#include <atomic>
#include <cstdlib>
#include <string>

#include "host_util.h"
#include "internal.h"

namespace aqmp {

int dictionary_build(int n_min, int n_max, uint32_t families, hipStream_t s, aqmp_dict** out);
void dictionary_free(aqmp_dict* d);
int dictionary_atoms(const aqmp_dict* d, int n, int* m_out);
int dictionary_copy(const aqmp_dict* d, int n, double* host_out);
int encode(const aqmp_dict* d, const aqmp_image* imgs, int n_imgs, const aqmp_params* prm, int n_prm,
           const aqmp_job* jobs, int n_jobs, const aqmp_options* opt, hipStream_t s, aqmp_code** out);
int reencode(aqmp_code* c, const aqmp_image* imgs, int n_imgs, hipStream_t s);
void code_free(aqmp_code* c);
int code_stats(const aqmp_code* c, aqmp_stats* s);
int code_timing(const aqmp_code* c, aqmp_timing* t);
int code_sizes(const aqmp_code* c, int64_t* n_leaves, int64_t* n_atoms);
int code_pack(const aqmp_code* c, const int32_t* jobs, int n_jobs, int level, double step, uint8_t* out,
              int64_t capacity, int64_t* size_out);
int code_export(const aqmp_code* c, bool leaves_only, aqmp_leaf* leaves, int32_t* atom_idx, double* coef,
                int64_t cap_leaves, int64_t cap_atoms);
int decode(const aqmp_dict* d, const aqmp_code* c, int job, double step, void* out, int dtype, int64_t row_stride,
           hipStream_t s);
int worklist_compact(const uint8_t* st, int64_t n, int32_t* out, int32_t* count, hipStream_t s);
int worklist_compact_noalloc(const uint8_t* st, int64_t n, int32_t* out, int32_t* count, hipStream_t s);
int worklist_split(const aqmp_params* prm, int n_prm, int n, const int32_t* node_prm, const int32_t* x0,
                   const int32_t* y0, const double* e, const int32_t* t, int64_t n_nodes, int32_t child_base,
                   uint8_t* st, int32_t* child_prm, int32_t* child_x0, int32_t* child_y0, int32_t* child_count,
                   hipStream_t s);

namespace {
thread_local std::string g_error;
std::atomic<long long> g_bytes{0};

long long byte_cap() {
  static const long long cap = [] {
    const char* v = std::getenv("AQMP_MAX_DEVICE_BYTES");
    return v ? std::atoll(v) : 0LL;
  }();
  return cap;
}
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }
const char* last_error() { return g_error.c_str(); }

int dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  const long long cap = byte_cap();
  if (cap > 0 && g_bytes.load() + (long long)bytes > cap) {
    set_error("device allocation of " + std::to_string(bytes) + " bytes exceeds AQMP_MAX_DEVICE_BYTES");
    return AQMP_E_NOMEM;
  }
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    return AQMP_E_NOMEM;
  }
  g_bytes += (long long)bytes;
  return AQMP_OK;
}

void dev_free(void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  g_bytes -= (long long)bytes;
}

}  // namespace aqmp

using namespace aqmp;

#define AQMP_ENTRY(expr)       \
  do {                         \
    clear_error();             \
    try {                      \
      return (expr);           \
    } catch (...) {            \
      set_error("internal error"); \
      return AQMP_E_NOMEM;     \
    }                          \
  } while (0)

extern "C" {

int aqmp_dictionary_build(int n_min, int n_max, uint32_t families, void* hip_stream, aqmp_dict** out) {
  AQMP_ENTRY(dictionary_build(n_min, n_max, families, (hipStream_t)hip_stream, out));
}

void aqmp_dictionary_free(aqmp_dict* d) {
  try {
    dictionary_free(d);
  } catch (...) {
  }
}

int aqmp_dictionary_atoms(const aqmp_dict* d, int n, int* m_out) { AQMP_ENTRY(dictionary_atoms(d, n, m_out)); }

int aqmp_dictionary_copy(const aqmp_dict* d, int n, double* host_out) {
  AQMP_ENTRY(dictionary_copy(d, n, host_out));
}

int aqmp_encode(const aqmp_dict* d, const aqmp_image* imgs, int n_imgs, const aqmp_params* prm, int n_prm,
                const aqmp_job* jobs, int n_jobs, const aqmp_options* opt, void* hip_stream, aqmp_code** out) {
  AQMP_ENTRY(encode(d, imgs, n_imgs, prm, n_prm, jobs, n_jobs, opt, (hipStream_t)hip_stream, out));
}

int aqmp_reencode(aqmp_code* c, const aqmp_image* imgs, int n_imgs, void* hip_stream) {
  AQMP_ENTRY(reencode(c, imgs, n_imgs, (hipStream_t)hip_stream));
}

int aqmp_code_sizes(const aqmp_code* c, int64_t* n_leaves, int64_t* n_atoms) {
  AQMP_ENTRY(code_sizes(c, n_leaves, n_atoms));
}

int aqmp_code_export(const aqmp_code* c, aqmp_leaf* leaves, int32_t* atom_idx, double* coef, int64_t cap_leaves,
                     int64_t cap_atoms) {
  AQMP_ENTRY(code_export(c, true, leaves, atom_idx, coef, cap_leaves, cap_atoms));
}

int aqmp_ssim(const aqmp_image* x, const aqmp_image* y, int mode, double data_range, double* out,
              void* hip_stream) {
  AQMP_ENTRY(ssim_planes(x, y, mode, data_range, out, (hipStream_t)hip_stream));
}

int aqmp_code_pack(const aqmp_code* c, const int32_t* jobs, int n_jobs, int level, uint8_t* out, int64_t capacity,
                   int64_t* size_out) {
  AQMP_ENTRY(code_pack(c, jobs, n_jobs, level, 0.0, out, capacity, size_out));
}

int aqmp_code_pack_quantized(const aqmp_code* c, const int32_t* jobs, int n_jobs, int level, double step,
                             uint8_t* out, int64_t capacity, int64_t* size_out) {
  AQMP_ENTRY(code_pack(c, jobs, n_jobs, level, step, out, capacity, size_out));
}

int aqmp_code_export_nodes(const aqmp_code* c, aqmp_leaf* nodes, int32_t* atom_idx, double* coef, int64_t cap_nodes,
                           int64_t cap_atoms) {
  AQMP_ENTRY(code_export(c, false, nodes, atom_idx, coef, cap_nodes, cap_atoms));
}

int aqmp_code_stats(const aqmp_code* c, aqmp_stats* s) { AQMP_ENTRY(code_stats(c, s)); }

int aqmp_code_timing(const aqmp_code* c, aqmp_timing* t) { AQMP_ENTRY(code_timing(c, t)); }

void aqmp_code_free(aqmp_code* c) {
  try {
    code_free(c);
  } catch (...) {
  }
}

int aqmp_decode(const aqmp_dict* d, const aqmp_code* c, int job, void* dev_out, int dtype, int64_t row_stride,
                void* hip_stream) {
  AQMP_ENTRY(decode(d, c, job, 0.0, dev_out, dtype, row_stride, (hipStream_t)hip_stream));
}

int aqmp_decode_quantized(const aqmp_dict* d, const aqmp_code* c, int job, double step, void* dev_out, int dtype,
                          int64_t row_stride, void* hip_stream) {
  AQMP_ENTRY(decode(d, c, job, step, dev_out, dtype, row_stride, (hipStream_t)hip_stream));
}

int aqmp_worklist_compact(const uint8_t* dev_status, int64_t n, int32_t* dev_out, int32_t* dev_count,
                          void* hip_stream) {
  AQMP_ENTRY(worklist_compact(dev_status, n, dev_out, dev_count, (hipStream_t)hip_stream));
}

int aqmp_worklist_compact_noalloc(const uint8_t* dev_status, int64_t n, int32_t* dev_out, int32_t* dev_count,
                                  void* hip_stream) {
  AQMP_ENTRY(worklist_compact_noalloc(dev_status, n, dev_out, dev_count, (hipStream_t)hip_stream));
}

int aqmp_worklist_split(const aqmp_params* prm, int n_prm, int n, const int32_t* dev_node_prm, const int32_t* dev_x0,
                        const int32_t* dev_y0, const double* dev_e, const int32_t* dev_t, int64_t n_nodes,
                        int32_t child_base, uint8_t* dev_status, int32_t* dev_child_prm, int32_t* dev_child_x0,
                        int32_t* dev_child_y0, int32_t* dev_child_count, void* hip_stream) {
  AQMP_ENTRY(worklist_split(prm, n_prm, n, dev_node_prm, dev_x0, dev_y0, dev_e, dev_t, n_nodes, child_base,
                            dev_status, dev_child_prm, dev_child_x0, dev_child_y0, dev_child_count,
                            (hipStream_t)hip_stream));
}

const char* aqmp_last_error(void) { return last_error(); }

const char* aqmp_corr_kernel(int n, int precision, int corr_variant) {
  // the N = 8 level of the BF16 form is the whole-level MFMA pursuit
  const char* name = aqmp::corr_kernel_name(n, precision, corr_variant);
  if (n == 8 && precision == AQMP_PREC_BF16 && name[0] != '\0') return "k_pursuit_bf16<8>";
  return name;
}

}  // extern "C"
