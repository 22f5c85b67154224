// encode.hip - host orchestration of the AQMP encoder (Algorithms 1-2):
// planning, device buffers, the level-synchronous launch sequence, the HIP
// graph of the batched schedule, result export and the decoder launch.
//
// Launch sequence of one pass (a set of jobs coded together):
//   init counts; for each block size N from the largest to the smallest:
//     gather the level's nodes -> residuals, norms, first stop test;
//     compact the running nodes into the active list;
//     k_N times: correlation + top-R keys (MFMA), select/update (FP64)
//                that appends the still-running nodes to the next list;
//     split test, stable scan, emit the children into the next level.
// All data-dependent counts live in device memory: kernels read them and
// idle when there is no work, so the sequence is fixed and can be captured
// once as a graph.  The batched schedule runs every job in one pass (one
// launch per MP step for every image, channel and parameter set); the plain
// schedule runs one pass per job, stream-ordered without a graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>


#include "host_core.h"
#include "host_util.h"
#include "internal.h"

namespace aqmp {

struct PassPlan {
  int j0 = 0, j1 = 0;                 // jobs [j0, j1)
  int64_t base[kLevels] = {};          // first node slot of the pass per level
  int64_t cap[kLevels] = {};           // node capacity per level
  int32_t ntop[kLevels] = {};          // top-level nodes per level
  int32_t kmax[kLevels] = {};          // MP steps launched per level
  int lg_hi = 0, lg_lo = 0;
};

// A node copied back to the host, with its place in the canonical order.
struct HostNode {
  aqmp_leaf leaf;
  const int32_t* idx;
  const double* coef;
};

// Grow-only device (or pinned host) buffer of a code's result gather.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace aqmp

struct aqmp_code {
  const aqmp_dict* dict = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  aqmp_options opt{};
  std::vector<aqmp_image> imgs;
  std::vector<aqmp_params> prm;
  std::vector<aqmp_job> jobs;
  std::vector<aqmp::JobDev> hjobs;
  std::vector<aqmp::JobDev> hjobs_dev;   // what djobs holds (empty: not uploaded yet)
  aqmp::JobDev* djobs = nullptr;
  std::vector<aqmp::PassPlan> passes;
  aqmp::Counters* dcnt = nullptr;      // one per pass
  int32_t* dntop = nullptr;            // [pass][kLevels]
  int64_t cap_total[aqmp::kLevels] = {};
  int32_t kmax_total[aqmp::kLevels] = {};
  aqmp::LevelDev lv[aqmp::kLevels] = {};
  // Working buffers of a pass (residuals, keys, active lists, scan state).
  // Passes that run one after another share one set; passes captured as
  // parallel graph branches get one set each.
  struct Work {
    float* r32 = nullptr;
    uint16_t* r16 = nullptr;
    unsigned long long* keys = nullptr;
    int32_t* act[2] = {nullptr, nullptr};
    double* cbuf = nullptr;          // Gram form: FP64 correlations [node][M]
    aqmp::ScanState ss{};
  };
  std::vector<Work> work;            // indexed by pass % work.size()
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  struct Alloc {
    void* p;
    size_t bytes;
  };
  std::vector<Alloc> allocs;
  int64_t steps_launched = 0;
  bool wide_residual = false;        // BF16 residual buffer of 4 GiB or more
  // Timing events (AQMP_OPT_TIMING): per level of every pass a start/end
  // pair; per MP step the start and end of the correlation (a, b) and of the
  // select/update launch (c, d), recorded by the dispatches themselves.  The
  // Gram and OMP solvers' levels use a, b, c around their two launches.
  struct LevelEv {
    int lg;
    hipEvent_t start, end;
  };
  struct StepEv {
    int lg;
    hipEvent_t a, b, c, d;
  };
  std::vector<LevelEv> lev;
  std::vector<StepEv> sev;
  size_t lev_pos = 0, sev_pos = 0;
  // Every visited node of the last encode in canonical order, gathered on
  // the device and copied back on the first read (stats, export, pack), kept
  // until the next encode.
  bool nodes_ok = false;
  std::vector<aqmp::HostNode> nodes;   // records and atoms point into `pinned`
  aqmp::DevBuf pinned;                 // page-locked host copy of ex_out
  // Device side of the gather: segment and job tables (built once), keys,
  // flat ids, scan and output buffers (grown as needed).
  bool ex_ready = false;
  int ex_nseg = 0;
  int ex_end_bit = 0;
  int64_t ex_max_cap = 0;
  aqmp::ExportSeg* d_ex_segs = nullptr;
  aqmp::ExportJob* d_ex_jobs = nullptr;
  // ex_out: node records, then atom indices, then coefficients (8-byte aligned)
  aqmp::DevBuf ex_keys, ex_keys2, ex_vals, ex_vals2, ex_tot, ex_tmp, ex_t, ex_off, ex_out;
};

namespace aqmp {

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static int k_of(const aqmp_params& p, int lg) {
  const int k = p.k_per_level[lg];
  return k >= 0 ? k : p.max_atoms;
}

int check_params(const aqmp_params& p, const std::string& tag) {
  if (!pow2(p.n_min) || !pow2(p.n_max) || p.n_min < AQMP_MIN_N || p.n_max > AQMP_MAX_N || p.n_min > p.n_max)
    AQMP_FAIL(AQMP_E_INVALID, tag + "need powers of two 4 <= n_min <= n_max <= 64");
  if (!(p.tol >= 0.0) || !std::isfinite(p.tol)) AQMP_FAIL(AQMP_E_INVALID, tag + "tol must be finite and >= 0");
  if (p.tol_mode != AQMP_TOL_RMS && p.tol_mode != AQMP_TOL_ABS) AQMP_FAIL(AQMP_E_INVALID, tag + "bad tol_mode");
  if (p.split_rule != AQMP_SPLIT_R1 && p.split_rule != AQMP_SPLIT_R2)
    AQMP_FAIL(AQMP_E_INVALID, tag + "bad split_rule");
  if (p.max_atoms < 0 || p.max_atoms > AQMP_MAX_ATOMS) AQMP_FAIL(AQMP_E_INVALID, tag + "max_atoms out of range");
  for (int l = 0; l < kLevels; ++l)
    if (p.k_per_level[l] < -1 || p.k_per_level[l] > AQMP_MAX_ATOMS)
      AQMP_FAIL(AQMP_E_INVALID, tag + "k_per_level out of range");
  return AQMP_OK;
}

JobDev make_jobdev(const aqmp_image& im, const aqmp_params& p) {
  JobDev j{};
  j.img = im.dev_ptr;
  j.dtype = im.dtype;
  j.w = im.w;
  j.h = im.h;
  j.row_stride = im.row_stride;
  j.n_min = p.n_min;
  j.n_max = p.n_max;
  j.split_rule = p.split_rule;
  for (int l = 0; l < kLevels; ++l) {
    const double n = (double)(1 << l);
    const double eps = p.tol_mode == AQMP_TOL_RMS ? p.tol * n : p.tol;
    j.eps2[l] = eps * eps;
    j.k[l] = k_of(p, l);
  }
  return j;
}

namespace {

// Image extent rounded up to a multiple of the top-level block size: the
// blocks tile the padded plane (edge replication, see job_pixel).
int64_t padded(int v, int n) { return ((int64_t)v + n - 1) / n * n; }

int validate(const aqmp_dict* d, const aqmp_image* imgs, int n_imgs, const aqmp_params* prm, int n_prm,
             const aqmp_job* jobs, int n_jobs, const aqmp_options* opt) {
  if (!d) AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: dictionary is null");
  if (n_imgs < 1 || !imgs) AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: no images");
  if (n_prm < 1 || !prm) AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: no parameter sets");
  if (n_jobs < 1 || !jobs) AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: no jobs");
  if (opt) {
    if (opt->precision != AQMP_PREC_FP32 && opt->precision != AQMP_PREC_BF16)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: bad precision");
    if (opt->schedule != AQMP_SCHED_PLAIN && opt->schedule != AQMP_SCHED_BATCHED &&
        opt->schedule != AQMP_SCHED_CONCURRENT)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: bad schedule");
    if (opt->flags & ~(AQMP_OPT_TIMING | AQMP_OPT_STEPWISE))
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: unknown option flags");
    if (!corr_variant_valid(opt->corr_variant))
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: bad corr_variant (0, 2, 3 or 6)");
    if (opt->corr_variant_levels & ~0x7FFFF00u)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: corr_variant_levels has bits outside the block sizes 4..64");
    for (int lg = 2; lg <= 6; ++lg)
      if (!corr_variant_valid((int)((opt->corr_variant_levels >> (4 * lg)) & 0xFu)))
        AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: bad corr_variant_levels entry for N = " + std::to_string(1 << lg));
    if (opt->solver != AQMP_SOLVER_DENSE && opt->solver != AQMP_SOLVER_GRAM && opt->solver != AQMP_SOLVER_OMP)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: bad solver");
    if (opt->corr_tile_levels & ~0xFFFFu)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: corr_tile_levels has bits outside the block sizes 32, 64");
    for (int b = 0; b < 2; ++b) {
      const uint32_t v = (opt->corr_tile_levels >> (8 * b)) & 0xFFu, lo = v & 0xFu, hi = v >> 4;
      if (v && !(lo >= 1 && lo <= hi && hi <= 7))
        AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: bad corr_tile_levels entry for N = " + std::to_string(32 << b));
    }
  }
  for (int i = 0; i < n_imgs; ++i) {
    const aqmp_image& im = imgs[i];
    if (!im.dev_ptr) AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: image " + std::to_string(i) + " has no data");
    if (im.dtype != AQMP_F32 && im.dtype != AQMP_F64)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: image " + std::to_string(i) + " has a bad dtype");
    if (im.w < 1 || im.h < 1 || im.row_stride < im.w)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: image " + std::to_string(i) + " has a bad shape or stride");
  }
  for (int i = 0; i < n_prm; ++i) {
    const aqmp_params& p = prm[i];
    const std::string tag = "aqmp_encode: params " + std::to_string(i) + ": ";
    const int rc = check_params(p, tag);
    if (rc != AQMP_OK) return rc;
    for (int n = p.n_min; n <= p.n_max; n *= 2) {
      if (!d->lv[ilog2(n)].have)
        AQMP_FAIL(AQMP_E_NODICT, tag + "the dictionary has no block size " + std::to_string(n));
      const int kl = p.k_per_level[ilog2(n)] >= 0 ? p.k_per_level[ilog2(n)] : p.max_atoms;
      if (opt && opt->solver == AQMP_SOLVER_OMP && kl > AQMP_OMP_MAX_ATOMS)
        AQMP_FAIL(AQMP_E_INVALID, tag + "OMP supports at most " + std::to_string(AQMP_OMP_MAX_ATOMS) +
                                      " atoms per node (k = " + std::to_string(kl) + ")");
    }
  }
  for (int i = 0; i < n_jobs; ++i) {
    const aqmp_job& j = jobs[i];
    if (j.image < 0 || j.image >= n_imgs || j.params < 0 || j.params >= n_prm)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: job " + std::to_string(i) + " refers to a missing image or params");
  }
  return AQMP_OK;
}

int alloc(aqmp_code* c, void** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  const int rc = dev_alloc(p, bytes);
  if (rc == AQMP_OK) c->allocs.push_back({*p, bytes});
  return rc;
}

void plan_pass(const aqmp_code* c, int j0, int j1, PassPlan& pp) {
  pp.j0 = j0;
  pp.j1 = j1;
  pp.lg_hi = 0;
  pp.lg_lo = kLevels;
  for (int j = j0; j < j1; ++j) {
    const aqmp_image& im = c->imgs[c->jobs[j].image];
    const aqmp_params& p = c->prm[c->jobs[j].params];
    const int hi = ilog2(p.n_max), lo = ilog2(p.n_min);
    pp.lg_hi = std::max(pp.lg_hi, hi);
    pp.lg_lo = std::min(pp.lg_lo, lo);
    const int64_t wp = padded(im.w, p.n_max), hp = padded(im.h, p.n_max);
    for (int l = lo; l <= hi; ++l) {
      const int64_t n = 1 << l;
      pp.cap[l] += (wp / n) * (hp / n);
      pp.kmax[l] = std::max(pp.kmax[l], k_of(p, l));
    }
    pp.ntop[hi] += (int32_t)((wp >> hi) * (hp >> hi));
  }
}

// Top-level nodes of a pass at one level: jobs in order, blocks in raster order.
void top_nodes(const aqmp_code* c, const PassPlan& pp, int lg, std::vector<int32_t>& job,
               std::vector<int32_t>& x0, std::vector<int32_t>& y0) {
  const int n = 1 << lg;
  for (int j = pp.j0; j < pp.j1; ++j) {
    const aqmp_image& im = c->imgs[c->jobs[j].image];
    const aqmp_params& p = c->prm[c->jobs[j].params];
    if (p.n_max != n) continue;
    for (int y = 0; y < padded(im.h, n); y += n)
      for (int x = 0; x < padded(im.w, n); x += n) {
        job.push_back(j);
        x0.push_back(x);
        y0.push_back(y);
      }
  }
}

LevelDev level_at(const aqmp_code* c, int lg, int64_t base) {
  LevelDev L = c->lv[lg];
  L.job += base;
  L.x0 += base;
  L.y0 += base;
  L.e += base;
  L.t += base;
  L.st += base;
  L.rec_idx += base * L.kmax;
  L.rec_coef += base * L.kmax;
  return L;
}

void free_code(aqmp_code* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->done) (void)hipEventDestroy(c->done);
  // (destroying a null event would leave an error for the next HIP call to report)
  auto destroy = [](hipEvent_t ev) {
    if (ev) (void)hipEventDestroy(ev);
  };
  for (auto& e : c->lev) destroy(e.start), destroy(e.end);
  for (auto& e : c->sev) destroy(e.a), destroy(e.b), destroy(e.c), destroy(e.d);
  for (auto& a : c->allocs) dev_free(a.p, a.bytes);
  for (DevBuf* b : {&c->ex_keys, &c->ex_keys2, &c->ex_vals, &c->ex_vals2, &c->ex_tot, &c->ex_tmp, &c->ex_t,
                    &c->ex_off, &c->ex_out})
    if (b->p) dev_free(b->p, b->bytes);
  if (c->pinned.p) (void)hipHostFree(c->pinned.p);
  delete c;
}

// Levels that run without per-step launches: N <= kFusedMaxN in both forms
// (dense FP64 pursuit), N = 16 in the BF16 form (whole-level MFMA pursuit),
// and every level of the Gram solver.
static bool whole_level(const aqmp_code* c, int n) {
  if (n <= kFusedMaxN || c->opt.solver != AQMP_SOLVER_DENSE) return true;
  return n == 16 && c->opt.precision == AQMP_PREC_BF16 && !(c->opt.flags & AQMP_OPT_STEPWISE);
}

int build_plan(aqmp_code* c) {
  const int nj = (int)c->jobs.size();
  c->hjobs.resize(nj);
  for (int j = 0; j < nj; ++j) c->hjobs[j] = make_jobdev(c->imgs[c->jobs[j].image], c->prm[c->jobs[j].params]);
  if (c->opt.schedule == AQMP_SCHED_BATCHED) {
    c->passes.resize(1);
    plan_pass(c, 0, nj, c->passes[0]);
  } else if (c->opt.schedule == AQMP_SCHED_CONCURRENT) {
    // Up to kBranches groups of consecutive jobs, balanced by pixel count.
    const int nb = std::min(nj, kBranches);
    int64_t total = 0;
    for (int j = 0; j < nj; ++j) total += (int64_t)c->imgs[c->jobs[j].image].w * c->imgs[c->jobs[j].image].h;
    int j0 = 0;
    int64_t acc = 0;
    for (int b = 0; b < nb; ++b) {
      int j1 = j0;
      const int64_t target = total * (b + 1) / nb;
      while (j1 < nj && (j1 == j0 || acc < target) && nj - j1 > nb - b - 1) {
        acc += (int64_t)c->imgs[c->jobs[j1].image].w * c->imgs[c->jobs[j1].image].h;
        ++j1;
      }
      if (b == nb - 1) j1 = nj;
      c->passes.emplace_back();
      plan_pass(c, j0, j1, c->passes.back());
      j0 = j1;
    }
  } else {
    c->passes.resize(nj);
    for (int j = 0; j < nj; ++j) plan_pass(c, j, j + 1, c->passes[j]);
  }
  // Level arrays: the passes are laid out one after the other.
  const size_t nwork = c->opt.schedule == AQMP_SCHED_CONCURRENT ? c->passes.size() : 1;
  std::vector<int64_t> max_r(nwork, 0), max_keys(nwork, 0), max_cap(nwork, 0), max_cbuf(nwork, 0);
  for (size_t pi = 0; pi < c->passes.size(); ++pi) {
    auto& pp = c->passes[pi];
    const size_t wi = pi % nwork;
    for (int l = 0; l < kLevels; ++l) {
      pp.base[l] = c->cap_total[l];
      c->cap_total[l] += pp.cap[l];
      c->kmax_total[l] = std::max(c->kmax_total[l], pp.kmax[l]);
      const int64_t n = 1 << l;
      if (pp.cap[l] == 0) continue;
      const aqmp_dict::Level& D = c->dict->lv[l];
      max_r[wi] = std::max(max_r[wi], pp.cap[l] * n * n);
      max_keys[wi] = std::max(max_keys[wi], pp.cap[l] * (D.m_pad / corr_atom_tile((int)n)) * kTopR);
      max_cap[wi] = std::max(max_cap[wi], pp.cap[l]);
      if (c->opt.solver != AQMP_SOLVER_DENSE && n > kFusedMaxN)
        max_cbuf[wi] = std::max(max_cbuf[wi], pp.cap[l] * D.m);
      c->steps_launched += pp.kmax[l];
    }
  }
#define ALLOC(ptr, bytes)                                      \
  do {                                                         \
    const int rc_ = alloc(c, (void**)&(ptr), (size_t)(bytes)); \
    if (rc_ != AQMP_OK) return rc_;                            \
  } while (0)
  for (int l = 0; l < kLevels; ++l) {
    const int64_t cap = c->cap_total[l];
    if (cap == 0) continue;
    LevelDev& L = c->lv[l];
    L.kmax = std::max(1, c->kmax_total[l]);
    ALLOC(L.job, cap * 4);
    ALLOC(L.x0, cap * 4);
    ALLOC(L.y0, cap * 4);
    ALLOC(L.e, cap * 8);
    ALLOC(L.t, cap * 4);
    ALLOC(L.st, cap);
    ALLOC(L.rec_idx, cap * L.kmax * 4);
    ALLOC(L.rec_coef, cap * L.kmax * 8);
  }
  // The direct-to-LDS correlation addresses residual rows with 32-bit byte
  // offsets; larger passes use the register-staged kernel instead.
  for (size_t wi = 0; wi < nwork; ++wi)
    if (max_r[wi] * 2 >= (int64_t)1 << 32) c->wide_residual = true;
  c->work.resize(nwork);
  for (size_t wi = 0; wi < nwork; ++wi) {
    aqmp_code::Work& wk = c->work[wi];
    if (c->opt.solver != AQMP_SOLVER_DENSE) {
      // No per-step launches: no residual, key or active-list buffers.
      ALLOC(wk.cbuf, max_cbuf[wi] * 8);
    } else {
      ALLOC(wk.r32, max_r[wi] * 4);
      if (c->opt.precision == AQMP_PREC_BF16) ALLOC(wk.r16, max_r[wi] * 2);
      ALLOC(wk.keys, max_keys[wi] * 8);
      ALLOC(wk.act[0], max_cap[wi] * 4);
      ALLOC(wk.act[1], max_cap[wi] * 4);
    }
    // Tile words of the look-back scans: one per scan tile of kScanTile
    // items and at least one per workgroup of a scan launch (both far below
    // this bound).
    wk.ss.ntiles_max = (int32_t)(max_cap[wi] / 4 + 2);
    ALLOC(wk.ss.tiles, sizeof(unsigned long long) * wk.ss.ntiles_max);
    ALLOC(wk.ss.ticket, sizeof(int32_t) * 2);
  }
  ALLOC(c->djobs, sizeof(JobDev) * nj);
  ALLOC(c->dcnt, sizeof(Counters) * c->passes.size());
  ALLOC(c->dntop, sizeof(int32_t) * kLevels * c->passes.size());
#undef ALLOC
  hipStream_t s = c->stream;
  for (auto& wk : c->work) {
    AQMP_HIP(hipMemsetAsync(wk.ss.tiles, 0, sizeof(unsigned long long) * wk.ss.ntiles_max, s));
    AQMP_HIP(hipMemsetAsync(wk.ss.ticket, 0, sizeof(int32_t) * 2, s));
  }
  AQMP_HIP(hipMemsetAsync(c->dcnt, 0, sizeof(Counters) * c->passes.size(), s));
  // Static top-level node lists.
  std::vector<int32_t> ntop_all(kLevels * c->passes.size(), 0);
  for (size_t pi = 0; pi < c->passes.size(); ++pi) {
    const PassPlan& pp = c->passes[pi];
    for (int l = 0; l < kLevels; ++l) {
      ntop_all[pi * kLevels + l] = pp.ntop[l];
      if (!pp.ntop[l]) continue;
      std::vector<int32_t> job, x0, y0;
      top_nodes(c, pp, l, job, x0, y0);
      const int64_t b = pp.base[l];
      AQMP_HIP(hipMemcpyAsync(c->lv[l].job + b, job.data(), 4 * job.size(), hipMemcpyHostToDevice, s));
      AQMP_HIP(hipMemcpyAsync(c->lv[l].x0 + b, x0.data(), 4 * x0.size(), hipMemcpyHostToDevice, s));
      AQMP_HIP(hipMemcpyAsync(c->lv[l].y0 + b, y0.data(), 4 * y0.size(), hipMemcpyHostToDevice, s));
      AQMP_HIP(hipStreamSynchronize(s));
    }
  }
  AQMP_HIP(hipMemcpyAsync(c->dntop, ntop_all.data(), 4 * ntop_all.size(), hipMemcpyHostToDevice, s));
  AQMP_HIP(hipStreamSynchronize(s));
  AQMP_HIP(hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
  if (c->opt.flags & AQMP_OPT_TIMING) {
    for (const auto& pp : c->passes)
      for (int l = pp.lg_hi; l >= pp.lg_lo; --l) {
        if (pp.cap[l] == 0) continue;
        aqmp_code::LevelEv le{l, nullptr, nullptr};
        AQMP_HIP(hipEventCreate(&le.start));
        AQMP_HIP(hipEventCreate(&le.end));
        c->lev.push_back(le);
        if (whole_level(c, 1 << l)) {
          // Gram and OMP levels with N >= 16: one event triple around the
          // initial-correlation and pursuit launches.
          if (c->opt.solver != AQMP_SOLVER_DENSE && (1 << l) > kFusedMaxN) {
            aqmp_code::StepEv se{l, nullptr, nullptr, nullptr, nullptr};
            AQMP_HIP(hipEventCreate(&se.a));
            AQMP_HIP(hipEventCreate(&se.b));
            AQMP_HIP(hipEventCreate(&se.c));
            c->sev.push_back(se);
          }
          continue;
        }
        for (int t = 0; t < pp.kmax[l]; ++t) {
          aqmp_code::StepEv se{l, nullptr, nullptr, nullptr, nullptr};
          AQMP_HIP(hipEventCreate(&se.a));
          AQMP_HIP(hipEventCreate(&se.b));
          AQMP_HIP(hipEventCreate(&se.c));
          AQMP_HIP(hipEventCreate(&se.d));
          c->sev.push_back(se);
        }
      }
  }
  return AQMP_OK;
}

#define AQMP_LAUNCH(call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) AQMP_FAIL(AQMP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int enqueue_pass(aqmp_code* c, size_t pi, hipStream_t s) {
  const PassPlan& pp = c->passes[pi];
  aqmp_code::Work& wk = c->work[pi % c->work.size()];
  Counters* cnt = c->dcnt + pi;
  const aqmp_dict* d = c->dict;
  AQMP_LAUNCH(launch_init_counts(cnt, c->dntop + pi * kLevels, s));
  for (int l = pp.lg_hi; l >= pp.lg_lo; --l) {
    if (pp.cap[l] == 0) continue;
    const int n = 1 << l;
    const aqmp_dict::Level& D = d->lv[l];
    StepArgs a{};
    a.jobs = c->djobs;
    a.lv = level_at(c, l, pp.base[l]);
    a.lg = l;
    a.n_atoms = D.m;
    a.nfam = d->nfam;
    a.tab = D.d_tab;
    a.tabT32 = D.d_tabT32;
    a.r32 = wk.r32;
    a.r16 = c->opt.precision == AQMP_PREC_BF16 ? wk.r16 : nullptr;
    a.keys = wk.keys;
    a.n_atom_tiles = D.m_pad / corr_atom_tile(n);
    int32_t* count = &cnt->count[l];
    const bool timing = (c->opt.flags & AQMP_OPT_TIMING) != 0;
    const aqmp_code::LevelEv* le = timing ? &c->lev[c->lev_pos++] : nullptr;
    if (le) AQMP_HIP(hipEventRecord(le->start, s));
    if (whole_level(c, n)) {
      // Small blocks: each node's whole pursuit in one launch.
      if (c->opt.solver != AQMP_SOLVER_DENSE) {
        const aqmp_code::StepEv* se = timing && n > kFusedMaxN ? &c->sev[c->sev_pos++] : nullptr;
        if (se) AQMP_HIP(hipEventRecord(se->a, s));
        if (n > kFusedMaxN)
          AQMP_LAUNCH(launch_gram_init(n, c->djobs, a.lv, count, l, d->nfam, D.d_tab, wk.cbuf, s));
        if (se) AQMP_HIP(hipEventRecord(se->b, s));
        if (c->opt.solver == AQMP_SOLVER_OMP)
          AQMP_LAUNCH(launch_omp_pursuit(n, c->djobs, a.lv, count, &cnt->next[l], l, d->nfam, D.d_tab, D.d_xg,
                                         wk.cbuf, pp.kmax[l], s));
        else
          AQMP_LAUNCH(launch_gram_pursuit(n, c->djobs, a.lv, count, &cnt->next[l], l, d->nfam, D.d_tab, D.d_xg,
                                          wk.cbuf, s));
        if (se) AQMP_HIP(hipEventRecord(se->c, s));
      } else if (n == 8 && c->opt.precision == AQMP_PREC_BF16)
        AQMP_LAUNCH(launch_pursuit_bf16(8, c->djobs, a.lv, count, &cnt->next[l], pp.cap[l], D.m, d->nfam, D.d_tab,
                                        D.d_tabT32, s));
      else if (n <= kFusedMaxN)
        AQMP_LAUNCH(launch_mp_fused(n, c->djobs, a.lv, count, l, D.m, D.d_tab, s));
      else
        AQMP_LAUNCH(launch_pursuit_bf16(16, c->djobs, a.lv, count, &cnt->next[l], pp.cap[l], D.m, d->nfam, D.d_tab,
                                        D.d_tabT32, s));
      if (l > pp.lg_lo && pp.cap[l - 1] > 0)
        AQMP_LAUNCH(launch_split_emit(c->djobs, (int32_t)c->jobs.size(), a.lv, count, level_at(c, l - 1, pp.base[l - 1]), pp.ntop[l - 1],
                                      &cnt->count[l - 1], l, pp.cap[l], wk.ss, &cnt->scan_error, s));
      if (le) AQMP_HIP(hipEventRecord(le->end, s));
      continue;
    }
    AQMP_LAUNCH(launch_gather(n, a, count, s));
    // Step t reads list t % 2 with counter t % 3 and appends to list
    // (t + 1) % 2 with counter (t + 1) % 3, which must be zero: the initial
    // compaction clears counter 1, and step t clears counter (t + 2) % 3.
    AQMP_LAUNCH(launch_compact(nullptr, count, a.lv.st, wk.act[0], &cnt->act[0], &cnt->act[1], pp.cap[l],
                               wk.ss, &cnt->scan_error, s));
    const void* atoms = c->opt.precision == AQMP_PREC_BF16 ? (const void*)D.d_bf16 : (const void*)D.d_f32;
    for (int t = 0; t < pp.kmax[l]; ++t) {
      a.act = wk.act[t & 1];
      a.act_count = &cnt->act[t % 3];
      const bool more = t + 1 < pp.kmax[l];
      a.next_act = more ? wk.act[(t + 1) & 1] : nullptr;
      a.next_count = &cnt->act[(t + 1) % 3];
      a.clear_count = &cnt->act[(t + 2) % 3];
      const aqmp_code::StepEv* se = timing ? &c->sev[c->sev_pos++] : nullptr;
      a.corr_tile = l >= 5 ? (int32_t)((c->opt.corr_tile_levels >> (8 * (l - 5))) & 0xFFu) : 0;
      const int lv_var = (int)((c->opt.corr_variant_levels >> (4 * l)) & 0xFu);
      const int variant = c->wide_residual ? 3 : (lv_var ? lv_var : c->opt.corr_variant);
      AQMP_LAUNCH(launch_corr(n, c->opt.precision, variant, atoms, a, D.m_pad, s, se ? se->a : nullptr,
                              se ? se->b : nullptr));
      AQMP_LAUNCH(launch_select(n, a, pp.cap[l], s, se ? se->c : nullptr, se ? se->d : nullptr));
    }
    if (l > pp.lg_lo && pp.cap[l - 1] > 0)
      AQMP_LAUNCH(launch_split_emit(c->djobs, (int32_t)c->jobs.size(), a.lv, count, level_at(c, l - 1, pp.base[l - 1]), pp.ntop[l - 1],
                                    &cnt->count[l - 1], l, pp.cap[l], wk.ss, &cnt->scan_error, s));
    if (le) AQMP_HIP(hipEventRecord(le->end, s));
  }
  return AQMP_OK;
}

int run(aqmp_code* c, hipStream_t s) {
  c->lev_pos = c->sev_pos = 0;
  c->nodes_ok = false;
  // The job table goes to the device only when it differs from what is
  // there (a re-encode of the same images changes nothing in it).
  if (c->hjobs_dev.size() != c->hjobs.size() ||
      std::memcmp(c->hjobs_dev.data(), c->hjobs.data(), sizeof(JobDev) * c->hjobs.size()) != 0) {
    AQMP_HIP(hipMemcpyAsync(c->djobs, c->hjobs.data(), sizeof(JobDev) * c->hjobs.size(), hipMemcpyHostToDevice, s));
    c->hjobs_dev = c->hjobs;
  }
  // HIP events recorded inside a graph cannot be timed, so a timed encode
  // issues the same launch sequence directly on the stream.
  if (c->opt.schedule != AQMP_SCHED_PLAIN && !(c->opt.flags & AQMP_OPT_TIMING)) {
    if (!c->gexec) {
      // Capture on a private stream (the caller's may be the null stream,
      // which cannot be captured); the graph is launched on the caller's.
      hipStream_t cs = nullptr;
      AQMP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        AQMP_FAIL(AQMP_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
      }
      int rc = AQMP_OK;
      std::vector<hipStream_t> br;
      std::vector<hipEvent_t> evs;
      if (c->passes.size() == 1) {
        rc = enqueue_pass(c, 0, cs);
      } else {
        // Parallel branches: fork from the capture stream, one pass per
        // branch, join back.
        hipEvent_t fork = nullptr;
        e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) {
          evs.push_back(fork);
          e = hipEventRecord(fork, cs);
        }
        for (size_t pi = 0; pi < c->passes.size() && e == hipSuccess && rc == AQMP_OK; ++pi) {
          hipStream_t bs = nullptr;
          e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking);
          if (e != hipSuccess) break;
          br.push_back(bs);
          e = hipStreamWaitEvent(bs, fork, 0);
          if (e != hipSuccess) break;
          rc = enqueue_pass(c, pi, bs);
          if (rc != AQMP_OK) break;
          hipEvent_t join = nullptr;
          e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
          if (e != hipSuccess) break;
          evs.push_back(join);
          e = hipEventRecord(join, bs);
          if (e == hipSuccess) e = hipStreamWaitEvent(cs, join, 0);
        }
        if (e != hipSuccess && rc == AQMP_OK) {
          set_error(std::string("graph branches: ") + hipGetErrorString(e));
          rc = AQMP_E_HIP;
        }
      }
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);
      for (auto bs : br) (void)hipStreamDestroy(bs);
      for (auto ev : evs) (void)hipEventDestroy(ev);
      (void)hipStreamDestroy(cs);
      if (rc != AQMP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) AQMP_FAIL(AQMP_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      c->graph = g;
      AQMP_HIP(hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
    }
    AQMP_HIP(hipGraphLaunch(c->gexec, s));
  } else {
    for (size_t pi = 0; pi < c->passes.size(); ++pi) {
      const int rc = enqueue_pass(c, pi, s);
      if (rc != AQMP_OK) return rc;
    }
  }
  c->stream = s;
  AQMP_HIP(hipEventRecord(c->done, s));
  return AQMP_OK;
}

int ensure(DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return AQMP_OK;
  if (b.p) dev_free(b.p, b.bytes);
  b.p = nullptr;
  b.bytes = 0;
  const size_t nb = std::max<size_t>(bytes + bytes / 4, 256);
  const int rc = dev_alloc(&b.p, nb);
  if (rc != AQMP_OK) return rc;
  b.bytes = nb;
  return AQMP_OK;
}

int ensure_pinned(DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return AQMP_OK;
  if (b.p) AQMP_HIP(hipHostFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  const size_t nb = std::max<size_t>(bytes + bytes / 4, 256);
  AQMP_HIP(hipHostMalloc(&b.p, nb, hipHostMallocDefault));
  b.bytes = nb;
  return AQMP_OK;
}

// Segment table (one entry per level of every pass) and job table of the
// device gather; built on the first read of a code.
int export_tables(aqmp_code* c) {
  std::vector<ExportSeg> segs;
  uint64_t flat = 0;
  int64_t max_cap = 0;
  for (size_t pi = 0; pi < c->passes.size(); ++pi) {
    const PassPlan& pp = c->passes[pi];
    for (int l = pp.lg_hi; l >= pp.lg_lo; --l) {
      if (pp.cap[l] == 0) continue;
      ExportSeg sg;
      sg.L = level_at(c, l, pp.base[l]);
      sg.count = &c->dcnt[pi].count[l];
      sg.lg = l;
      sg.flat_base = (uint32_t)flat;
      segs.push_back(sg);
      flat += (uint64_t)pp.cap[l];
      max_cap = std::max<int64_t>(max_cap, pp.cap[l]);
    }
  }
  if (flat >= (1ull << 32) || segs.size() > 65535)
    AQMP_FAIL(AQMP_E_CAPACITY, "aqmp_code: too many node slots for the result gather");
  std::vector<ExportJob> jx(c->jobs.size());
  long long tops = 0;
  for (size_t j = 0; j < c->jobs.size(); ++j) {
    const int nm = c->prm[c->jobs[j].params].n_max;
    const aqmp_image& im = c->imgs[c->jobs[j].image];
    jx[j].top_base = tops;
    jx[j].nm = nm;
    jx[j].cols = (int32_t)(padded(im.w, nm) / nm);
    tops += (long long)jx[j].cols * (padded(im.h, nm) / nm);
  }
  int bits = 1;
  while (bits < 63 && (1ll << bits) < tops) ++bits;
  if (bits + kExportLowBits > 64) AQMP_FAIL(AQMP_E_CAPACITY, "aqmp_code: too many top-level blocks for the result gather");
  c->ex_end_bit = bits + kExportLowBits;
  c->ex_nseg = (int)segs.size();
  c->ex_max_cap = max_cap;
  if (!segs.empty()) {
    const int rc1 = alloc(c, (void**)&c->d_ex_segs, sizeof(ExportSeg) * segs.size());
    if (rc1 != AQMP_OK) return rc1;
    const int rc2 = alloc(c, (void**)&c->d_ex_jobs, sizeof(ExportJob) * jx.size());
    if (rc2 != AQMP_OK) return rc2;
    AQMP_HIP(hipMemcpy(c->d_ex_segs, segs.data(), sizeof(ExportSeg) * segs.size(), hipMemcpyHostToDevice));
    AQMP_HIP(hipMemcpy(c->d_ex_jobs, jx.data(), sizeof(ExportJob) * jx.size(), hipMemcpyHostToDevice));
    int rc = ensure(c->ex_keys, sizeof(unsigned long long) * flat);
    if (rc == AQMP_OK) rc = ensure(c->ex_vals, sizeof(uint32_t) * flat);
    if (rc == AQMP_OK) rc = ensure(c->ex_tot, 2 * sizeof(unsigned long long));
    if (rc != AQMP_OK) return rc;
  }
  c->ex_ready = true;
  return AQMP_OK;
}

#define AQMP_ENSURE(buf, bytes)                 \
  do {                                          \
    const int rc_ = ensure((buf), (bytes));     \
    if (rc_ != AQMP_OK) return rc_;             \
  } while (0)

// Gathers every visited node on the device in canonical order (job, top-level
// block in raster order, then depth-first: Morton order of the corner, the
// larger node first) and copies three dense arrays back: node records, atom
// indices, coefficients.
int collect_all(aqmp_code* c) {
  hipStream_t s = c->stream;
  AQMP_HIP(hipStreamSynchronize(s));
  std::vector<Counters> cnt(c->passes.size());
  AQMP_HIP(hipMemcpy(cnt.data(), c->dcnt, sizeof(Counters) * cnt.size(), hipMemcpyDeviceToHost));
  for (size_t pi = 0; pi < cnt.size(); ++pi) {
    if (cnt[pi].scan_error) AQMP_FAIL(AQMP_E_HIP, "aqmp_encode: a device scan exceeded its bounded wait");
    for (int l = 0; l < kLevels; ++l)
      if (cnt[pi].count[l] > c->passes[pi].cap[l])
        AQMP_FAIL(AQMP_E_HIP, "aqmp_encode: level count exceeds its capacity");
  }
  c->nodes.clear();
  if (!c->ex_ready) {
    const int rc = export_tables(c);
    if (rc != AQMP_OK) return rc;
  }
  if (c->ex_nseg == 0) return AQMP_OK;
  auto* keys = (unsigned long long*)c->ex_keys.p;
  auto* vals = (uint32_t*)c->ex_vals.p;
  auto* tot = (unsigned long long*)c->ex_tot.p;
  AQMP_HIP(hipMemsetAsync(tot, 0, 2 * sizeof(unsigned long long), s));
  AQMP_HIP(launch_export_keys(c->d_ex_segs, c->ex_nseg, c->ex_max_cap, c->d_ex_jobs, keys, vals, tot, s));
  unsigned long long ht[2] = {0, 0};
  AQMP_HIP(hipMemcpyAsync(ht, tot, sizeof(ht), hipMemcpyDeviceToHost, s));
  AQMP_HIP(hipStreamSynchronize(s));
  const int64_t n = (int64_t)ht[0], na = (int64_t)ht[1];
  if (n == 0) return AQMP_OK;
  AQMP_ENSURE(c->ex_keys2, sizeof(unsigned long long) * n);
  AQMP_ENSURE(c->ex_vals2, sizeof(uint32_t) * n);
  AQMP_ENSURE(c->ex_t, sizeof(int64_t) * n);
  AQMP_ENSURE(c->ex_off, sizeof(int64_t) * n);
  auto* keys2 = (unsigned long long*)c->ex_keys2.p;
  auto* vals2 = (uint32_t*)c->ex_vals2.p;
  auto* tcount = (int64_t*)c->ex_t.p;
  auto* off = (int64_t*)c->ex_off.p;
  size_t sort_bytes = 0, scan_bytes = 0;
  AQMP_HIP(export_sort(nullptr, sort_bytes, keys, keys2, vals, vals2, n, c->ex_end_bit, s));
  AQMP_HIP(export_scan(nullptr, scan_bytes, tcount, off, n, s));
  AQMP_ENSURE(c->ex_tmp, std::max(sort_bytes, scan_bytes));
  sort_bytes = scan_bytes = c->ex_tmp.bytes;
  AQMP_HIP(export_sort(c->ex_tmp.p, sort_bytes, keys, keys2, vals, vals2, n, c->ex_end_bit, s));
  AQMP_HIP(launch_export_counts(c->d_ex_segs, c->ex_nseg, vals2, n, tcount, s));
  AQMP_HIP(export_scan(c->ex_tmp.p, scan_bytes, tcount, off, n, s));
  // one output block, one copy into page-locked memory
  const size_t idx_at = sizeof(aqmp_leaf) * n;
  const size_t coef_at = idx_at + (sizeof(int32_t) * na + 7) / 8 * 8;
  const size_t total = coef_at + sizeof(double) * na;
  AQMP_ENSURE(c->ex_out, total);
  {
    const int rc = ensure_pinned(c->pinned, total);
    if (rc != AQMP_OK) return rc;
  }
  char* dout = (char*)c->ex_out.p;
  AQMP_HIP(launch_export_write(c->d_ex_segs, c->ex_nseg, vals2, off, n, (aqmp_leaf*)dout, (int32_t*)(dout + idx_at),
                               (double*)(dout + coef_at), s));
  AQMP_HIP(hipMemcpyAsync(c->pinned.p, dout, total, hipMemcpyDeviceToHost, s));
  AQMP_HIP(hipStreamSynchronize(s));
  const char* hout = (const char*)c->pinned.p;
  const aqmp_leaf* rec = (const aqmp_leaf*)hout;
  const int32_t* idx = (const int32_t*)(hout + idx_at);
  const double* coef = (const double*)(hout + coef_at);
  c->nodes.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    HostNode& h = c->nodes[i];
    h.leaf = rec[i];
    h.idx = idx + h.leaf.atom_off;
    h.coef = coef + h.leaf.atom_off;
  }
  return AQMP_OK;
}

#undef AQMP_ENSURE

// The code's visited nodes (or leaves) in canonical order; the device copy is
// made once per encode.
int collect(const aqmp_code* cc, bool leaves_only, std::vector<HostNode>& out) {
  aqmp_code* c = const_cast<aqmp_code*>(cc);   // the cache is not part of the code's observable state
  if (!c->nodes_ok) {
    const int rc = collect_all(c);
    if (rc != AQMP_OK) return rc;
    c->nodes_ok = true;
  }
  out.clear();
  for (const auto& h : c->nodes)
    if (!(leaves_only && (h.leaf.flags & 1))) out.push_back(h);
  return AQMP_OK;
}

}  // namespace

int encode(const aqmp_dict* d, const aqmp_image* imgs, int n_imgs, const aqmp_params* prm, int n_prm,
           const aqmp_job* jobs, int n_jobs, const aqmp_options* opt, hipStream_t s, aqmp_code** out) {
  if (!out) AQMP_FAIL(AQMP_E_INVALID, "aqmp_encode: out is null");
  *out = nullptr;
  int rc = validate(d, imgs, n_imgs, prm, n_prm, jobs, n_jobs, opt);
  if (rc != AQMP_OK) return rc;
  aqmp_code* c = new (std::nothrow) aqmp_code();
  if (!c) AQMP_FAIL(AQMP_E_NOMEM, "aqmp_encode: host allocation failed");
  c->dict = d;
  c->stream = s;
  if (opt) c->opt = *opt;
  else c->opt.precision = AQMP_PREC_FP32, c->opt.schedule = AQMP_SCHED_PLAIN;
  c->imgs.assign(imgs, imgs + n_imgs);
  c->prm.assign(prm, prm + n_prm);
  c->jobs.assign(jobs, jobs + n_jobs);
  rc = build_plan(c);
  if (rc == AQMP_OK) rc = run(c, s);
  if (rc != AQMP_OK) {
    const std::string msg = last_error();
    free_code(c);
    set_error(msg);
    return rc;
  }
  *out = c;
  return AQMP_OK;
}

int reencode(aqmp_code* c, const aqmp_image* imgs, int n_imgs, hipStream_t s) {
  if (!c || !imgs) AQMP_FAIL(AQMP_E_INVALID, "aqmp_reencode: null argument");
  if (n_imgs != (int)c->imgs.size()) AQMP_FAIL(AQMP_E_INVALID, "aqmp_reencode: image count differs");
  for (int i = 0; i < n_imgs; ++i) {
    const aqmp_image& a = imgs[i];
    const aqmp_image& b = c->imgs[i];
    if (!a.dev_ptr || a.dtype != b.dtype || a.w != b.w || a.h != b.h || a.row_stride < a.w)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_reencode: image " + std::to_string(i) + " differs in type or shape");
  }
  // Wait for any earlier use of the buffers on another stream.
  if (c->stream != s) AQMP_HIP(hipStreamWaitEvent(s, c->done, 0));
  c->imgs.assign(imgs, imgs + n_imgs);
  for (size_t j = 0; j < c->jobs.size(); ++j) {
    c->hjobs[j].img = c->imgs[c->jobs[j].image].dev_ptr;
    c->hjobs[j].row_stride = c->imgs[c->jobs[j].image].row_stride;
  }
  return run(c, s);
}

void code_free(aqmp_code* c) { free_code(c); }

int code_stats(const aqmp_code* c, aqmp_stats* s) {
  if (!c || !s) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_stats: null argument");
  std::vector<HostNode> nodes;
  const int rc = collect(c, false, nodes);
  if (rc != AQMP_OK) return rc;
  std::memset(s, 0, sizeof(*s));
  for (const auto& h : nodes) {
    const int l = ilog2(h.leaf.n);
    s->nodes[l]++;
    s->iters_level[l] += h.leaf.n_atoms;
    s->iters_executed += h.leaf.n_atoms;
    if (!(h.leaf.flags & 1)) {
      s->leaves[l]++;
      s->iters_emitted += h.leaf.n_atoms;
    }
  }
  s->steps_launched = c->steps_launched;
  return AQMP_OK;
}

int code_timing(const aqmp_code* c, aqmp_timing* t) {
  if (!c || !t) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_timing: null argument");
  if (!(c->opt.flags & AQMP_OPT_TIMING)) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_timing: encode made without timing");
  AQMP_HIP(hipStreamSynchronize(c->stream));
  std::memset(t, 0, sizeof(*t));
  float ms = 0.f;
  for (const auto& e : c->lev) {
    AQMP_HIP(hipEventElapsedTime(&ms, e.start, e.end));
    t->level_ms[e.lg] += ms;
  }
  for (const auto& e : c->sev) {
    AQMP_HIP(hipEventElapsedTime(&ms, e.a, e.b));
    t->corr_ms[e.lg] += ms;
    AQMP_HIP(hipEventElapsedTime(&ms, e.d ? e.c : e.b, e.d ? e.d : e.c));
    t->select_ms[e.lg] += ms;
    t->steps[e.lg] += 1;
  }
  return AQMP_OK;
}

int code_sizes(const aqmp_code* c, int64_t* n_leaves, int64_t* n_atoms) {
  if (!c || !n_leaves || !n_atoms) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_sizes: null argument");
  aqmp_stats s;
  const int rc = code_stats(c, &s);
  if (rc != AQMP_OK) return rc;
  *n_leaves = 0;
  for (int l = 0; l < kLevels; ++l) *n_leaves += s.leaves[l];
  *n_atoms = s.iters_emitted;
  return AQMP_OK;
}

int code_export(const aqmp_code* c, bool leaves_only, aqmp_leaf* leaves, int32_t* atom_idx, double* coef,
                int64_t cap_leaves, int64_t cap_atoms) {
  if (!c || !leaves || !atom_idx || !coef) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_export: null argument");
  std::vector<HostNode> nodes;
  const int rc = collect(c, leaves_only, nodes);
  if (rc != AQMP_OK) return rc;
  int64_t na = 0;
  for (const auto& h : nodes) na += h.leaf.n_atoms;
  if ((int64_t)nodes.size() > cap_leaves || na > cap_atoms)
    AQMP_FAIL(AQMP_E_CAPACITY, "aqmp_code_export: need " + std::to_string(nodes.size()) + " records and " +
                                   std::to_string(na) + " atoms");
  int64_t off = 0;
  for (size_t i = 0; i < nodes.size(); ++i) {
    aqmp_leaf L = nodes[i].leaf;
    L.atom_off = off;
    std::memcpy(atom_idx + off, nodes[i].idx, sizeof(int32_t) * L.n_atoms);
    std::memcpy(coef + off, nodes[i].coef, sizeof(double) * L.n_atoms);
    off += L.n_atoms;
    leaves[i] = L;
  }
  return AQMP_OK;
}

// ---------------------------------------------------------------------------
// Bitstream (encoder step (iii), Section 2.3): the sparse vectors of every
// channel, then a lossless DEFLATE pass.  The byte layout is stream_write's
// (host_core.h); here the nodes of each packed job are taken in the
// canonical depth-first order (top-level blocks in raster order over the
// padded plane, children TL, TR, BL, BR).
// ---------------------------------------------------------------------------
int code_pack(const aqmp_code* c, const int32_t* jobs, int n_jobs, int level, double step, uint8_t* out,
              int64_t capacity, int64_t* size_out) {
  if (!c || !jobs || !size_out) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_pack: null argument");
  if (n_jobs < 1 || n_jobs > 255) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_pack: 1..255 channels per stream");
  if (level < -1 || level > 9) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_pack: level must be -1 (raw) or 0..9");
  const int nj = (int)c->jobs.size();
  for (int i = 0; i < n_jobs; ++i)
    if (jobs[i] < 0 || jobs[i] >= nj) AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_pack: job out of range");
  const aqmp_image& im0 = c->imgs[c->jobs[jobs[0]].image];
  const aqmp_params& p0 = c->prm[c->jobs[jobs[0]].params];
  for (int i = 1; i < n_jobs; ++i) {
    const aqmp_image& im = c->imgs[c->jobs[jobs[i]].image];
    const aqmp_params& p = c->prm[c->jobs[jobs[i]].params];
    if (im.w != im0.w || im.h != im0.h || p.n_min != p0.n_min || p.n_max != p0.n_max)
      AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_pack: the channels of a stream need one size and one block range");
  }
  std::vector<HostNode> nodes;
  const int rc = collect(c, false, nodes);
  if (rc != AQMP_OK) return rc;
  std::vector<std::vector<StreamNode>> sn(n_jobs);
  std::vector<StreamChannel> ch(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    // the job's nodes are contiguous in the canonical order
    auto lo = std::lower_bound(nodes.begin(), nodes.end(), jobs[i],
                               [](const HostNode& a, int32_t j) { return a.leaf.job < j; });
    auto hi = std::lower_bound(lo, nodes.end(), jobs[i] + 1,
                               [](const HostNode& a, int32_t j) { return a.leaf.job < j; });
    sn[i].reserve((size_t)(hi - lo));
    for (auto it = lo; it != hi; ++it)
      sn[i].push_back(StreamNode{it->leaf.n, (it->leaf.flags & 1) != 0, it->leaf.n_atoms, it->idx, it->coef});
    ch[i] = StreamChannel{sn[i].data(), sn[i].size()};
  }
  const StreamHeader hd{(int)c->dict->families, (uint32_t)im0.w, (uint32_t)im0.h, p0.n_min, p0.n_max};
  std::vector<uint8_t> raw;
  std::string why;
  if (stream_write(hd, ch.data(), n_jobs, step, raw, &why) != AQMP_OK)
    AQMP_FAIL(AQMP_E_INVALID, "aqmp_code_pack: " + why);
  const std::vector<uint8_t>* res = &raw;
  std::vector<uint8_t> z;
  if (level >= 0) {
    if (!out) {
      *size_out = (int64_t)stream_deflate_bound(raw.size());
      return AQMP_OK;
    }
    if (stream_deflate(raw, level, z) != AQMP_OK) AQMP_FAIL(AQMP_E_NOMEM, "aqmp_code_pack: DEFLATE failed");
    res = &z;
  }
  *size_out = (int64_t)res->size();
  if (!out) return AQMP_OK;
  if (capacity < (int64_t)res->size()) AQMP_FAIL(AQMP_E_CAPACITY, "aqmp_code_pack: output buffer too small");
  std::copy(res->begin(), res->end(), out);
  return AQMP_OK;
}

int decode(const aqmp_dict* d, const aqmp_code* c, int job, double step, void* out, int dtype, int64_t row_stride,
           hipStream_t s) {
  if (!d || !c || !out) AQMP_FAIL(AQMP_E_INVALID, "aqmp_decode: null argument");
  if (!(step >= 0.0) || !std::isfinite(step)) AQMP_FAIL(AQMP_E_INVALID, "aqmp_decode: step must be finite and >= 0");
  if (step > 0.0 && !((double)(float)step > 0.0)) AQMP_FAIL(AQMP_E_INVALID, "aqmp_decode: step rounds to zero in binary32");
  if (d != c->dict) AQMP_FAIL(AQMP_E_INVALID, "aqmp_decode: code was made with another dictionary");
  if (job < 0 || job >= (int)c->jobs.size()) AQMP_FAIL(AQMP_E_INVALID, "aqmp_decode: job out of range");
  if (dtype != AQMP_F32 && dtype != AQMP_F64) AQMP_FAIL(AQMP_E_INVALID, "aqmp_decode: bad dtype");
  if (row_stride < c->imgs[c->jobs[job].image].w) AQMP_FAIL(AQMP_E_INVALID, "aqmp_decode: row stride too small");
  AQMP_HIP(hipStreamWaitEvent(s, c->done, 0));
  size_t pi = 0;
  while (pi < c->passes.size() && !(job >= c->passes[pi].j0 && job < c->passes[pi].j1)) ++pi;
  const PassPlan& pp = c->passes[pi];
  for (int l = pp.lg_hi; l >= pp.lg_lo; --l) {
    if (pp.cap[l] == 0) continue;
    AQMP_LAUNCH(launch_decode(1 << l, c->djobs, level_at(c, l, pp.base[l]), &c->dcnt[pi].count[l], job, d->nfam,
                              d->lv[l].d_tab, step > 0.0 ? (double)(float)step : 0.0, out, dtype, row_stride, s));
  }
  return AQMP_OK;
}

}  // namespace aqmp
