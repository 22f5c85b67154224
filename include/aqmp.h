/*
 * aqmp.h - C ABI of the MI355X (gfx950) AQMP encoder.
 *
 * AQMP (Adaptive Quadtree Matching Pursuit, arXiv 2605.09190) codes every
 * channel of an image as a quadtree of square blocks.  Each block is
 * approximated by greedy Matching Pursuit over a dictionary of unit-norm 2D
 * atoms; a block whose residual misses the accuracy target after k
 * iterations is split into its four quadrants, down to a minimum size.
 *
 * Conventions shared by every entry point:
 *   - Return value: AQMP_OK (0) or a negative AQMP_E_* code.  Nothing throws
 *     or aborts across this boundary.  aqmp_last_error() gives a message for
 *     the calling thread's last failure.  On failure no output handle is
 *     created and caller buffers are left untouched.
 *   - "device" pointers are HIP device memory of the current device;
 *     "host" pointers are ordinary host memory.  The caller owns every
 *     buffer it passes in; the library owns the handles it returns.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Encode and decode are stream-ordered and asynchronous.
 *   - Same inputs give bit-identical outputs: all reductions have a fixed
 *     order, and no result depends on the order of the active-node list
 *     (which the select step builds by atomic append).
 *   - A handle may be used by one thread at a time.  The first read of a
 *     code after an encode (sizes, stats, export, pack) sorts its visited
 *     nodes into canonical order on the device, on the encode stream, and
 *     copies them once into page-locked host memory owned by the handle;
 *     later reads use that copy until the next encode of that code.
 *   - Block sizes N are powers of two with 4 <= N <= 64.
 *
 * Pixel and atom layout.  A block b of size N is the N x N sub-matrix of a
 * channel, b[i][j] with i the row and j the column.  The paper flattens a
 * block by concatenating its columns (Appendix A): element (i, j) sits at
 * position j*N + i of the flattened vector.  For family f (0 = DCT, 1 = Haar
 * when both are built) and frequencies (p, q), atom a = f*N*N + q*N + p is
 * the 2D block A[i][j] = T_f[p][i] * T_f[q][j] (outer product of two 1D
 * basis rows, Section 2.1), where T_0 is the orthonormal DCT-II matrix of
 * Section 2.1 and T_1 the orthonormal Haar matrix.  The constant atom of each
 * family is exactly 1/N.  M_N = (number of families) * N * N.
 */
#ifndef AQMP_H
#define AQMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
  AQMP_OK = 0,
  AQMP_E_INVALID = -1,   /* null pointer, bad enum, n not a power of two,
                            n_min > n_max, tol < 0, k out of range ...     */
  AQMP_E_SHAPE = -2,     /* reserved (non-multiple sizes are padded)      */
  AQMP_E_NODICT = -3,    /* the dictionary lacks a block size the jobs use */
  AQMP_E_NOMEM = -4,     /* device or host allocation failed, or the
                            AQMP_MAX_DEVICE_BYTES environment cap is hit   */
  AQMP_E_HIP = -5,       /* a HIP runtime call failed                      */
  AQMP_E_CAPACITY = -6   /* caller's output buffer too small               */
};

/* ---- enumerations ------------------------------------------------------ */
enum { AQMP_DCT = 1, AQMP_HAAR = 2 };             /* dictionary families   */
enum { AQMP_F32 = 0, AQMP_F64 = 1 };              /* sample types          */
enum { AQMP_TOL_RMS = 0, AQMP_TOL_ABS = 1 };      /* tolerance modes       */
enum { AQMP_SPLIT_R1 = 0, AQMP_SPLIT_R2 = 1 };    /* split rules           */
enum { AQMP_PREC_FP32 = 0, AQMP_PREC_BF16 = 1 };  /* correlation precision */
enum { AQMP_SCHED_PLAIN = 0, AQMP_SCHED_BATCHED = 1, AQMP_SCHED_CONCURRENT = 2 };

#define AQMP_MIN_N 4
#define AQMP_MAX_N 64
#define AQMP_MAX_ATOMS 256     /* largest k (iterations per node)          */
#define AQMP_CANDIDATES 8      /* candidates re-scored per MP iteration    */
#define AQMP_OMP_MAX_ATOMS 64  /* largest k with AQMP_SOLVER_OMP            */

typedef struct aqmp_dict aqmp_dict;
typedef struct aqmp_code aqmp_code;

/* One channel plane: h rows of w samples, sample (row y, column x) at
 * dev_ptr[y * row_stride + x].  Device memory, read-only, owned by the
 * caller and valid until the encode's stream work has completed. */
typedef struct {
  const void* dev_ptr;
  int32_t dtype;          /* AQMP_F32 or AQMP_F64 */
  int32_t w, h;
  int64_t row_stride;     /* in samples, >= w */
} aqmp_image;

/* Parameters of the problem statement (Section 2.3): accuracy tolerance,
 * sparsity, admissible block sizes.
 *   tol_mode AQMP_TOL_RMS: eps_N = tol * N (residual RMS <= tol per block);
 *   tol_mode AQMP_TOL_ABS: eps_N = tol at every level (Algorithm 2 passes
 *                          the same eps to the children).
 * A node stops when ||r||^2 < eps_N^2 or after k_N iterations (eq. (2)),
 * checked before every iteration.  k_N = k_per_level[log2 N] when that entry
 * is >= 0, else max_atoms.  0 <= k_N <= AQMP_MAX_ATOMS.
 *   split_rule AQMP_SPLIT_R1: split when N > n_min and ||r||^2 >= eps_N^2
 *                             after MP (accuracy not met);
 *   split_rule AQMP_SPLIT_R2: split when N > n_min and k_N iterations ran
 *                             (the pseudocode's ||x||_0 >= k test). */
typedef struct {
  double tol;
  int32_t tol_mode;
  int32_t max_atoms;
  int32_t n_min, n_max;
  int32_t split_rule;
  int32_t k_per_level[7];   /* index log2(N); -1 = use max_atoms */
} aqmp_params;

/* One job = one channel plane coded under one parameter set (Algorithm 1's
 * loop over channels; a hyperparameter trial is another job on the same
 * plane). */
typedef struct {
  int32_t image;
  int32_t params;
} aqmp_job;

enum { AQMP_OPT_TIMING = 1, AQMP_OPT_STEPWISE = 2 };   /* aqmp_options.flags */

enum { AQMP_SOLVER_DENSE = 0, AQMP_SOLVER_GRAM = 1, AQMP_SOLVER_OMP = 2 };   /* aqmp_options.solver */

typedef struct {
  int32_t precision;   /* AQMP_PREC_FP32: FP32 MFMA correlation;
                          AQMP_PREC_BF16: BF16 MFMA, FP32 accumulate.
                          Both re-score the AQMP_CANDIDATES best atoms in
                          FP64 and take the coefficient and the stop/split
                          test in FP64. */
  int32_t schedule;    /* AQMP_SCHED_PLAIN: jobs one after another,
                          stream-ordered launches;
                          AQMP_SCHED_BATCHED: every job in one pass,
                          captured once as a HIP graph and replayed;
                          AQMP_SCHED_CONCURRENT: the jobs split into up to
                          four groups of consecutive jobs, each group one
                          pass, captured as parallel branches of one graph
                          so that their launches overlap. */
  int32_t flags;       /* AQMP_OPT_TIMING: time every launch of an MP step
                          with HIP events that the dispatch itself records at
                          the kernel's start and end (see
                          aqmp_code_timing).  Events cannot be timed inside
                          a graph, so a timed batched encode issues the same
                          launches directly on the stream.
                          AQMP_OPT_STEPWISE: run the N = 16 level of the
                          BF16 form one MP step per launch (correlation
                          and select) instead of the whole-level
                          pursuit; same method, for comparison. */
  int32_t corr_variant;  /* tuning: 0 = library default; 2, 3 or 6 force
                            one family of BF16 correlation kernels (results
                            are identical, only speed differs): 2 direct-
                            to-LDS loads, two workgroups per CU (N >= 16);
                            3 register-staged loads (every N); 6 atoms
                            generated in registers (N = 32, 64; other N
                            take 3).  Other values are AQMP_E_INVALID. */
  int32_t solver;      /* AQMP_SOLVER_DENSE: every MP step correlates the
                          residual with all M atoms (Section 2.2, eq. (1)),
                          in the precision above.
                          AQMP_SOLVER_GRAM: the same MP, computed exactly
                          through the dictionary's structure: the
                          correlations of y as separable products
                          T_f Y T_f^T, then per step c <- c - c_i G[:, i]
                          and ||r||^2 <- ||r||^2 - c_i^2, all in FP64
                          (precision and corr_variant do not apply; levels
                          with N <= 8 run the dense FP64 pursuit as in the
                          dense solver).  A labelled variant: the paper
                          states the dense correlation.
                          AQMP_SOLVER_OMP: Orthogonal Matching Pursuit, the
                          solver the authors' implementation ran (Section
                          2.2): MP's selection, then all selected
                          coefficients re-fit by least squares each step
                          (FP64, Cholesky-updated; records hold the final
                          coefficients in selection order).  k may not
                          exceed AQMP_OMP_MAX_ATOMS; precision and
                          corr_variant do not apply. */
  uint32_t corr_variant_levels;  /* tuning, per block size: bits 4 lg .. 4 lg + 3
                                    hold the BF16 correlation variant (0, 2, 3, 6) for
                                    N = 2^lg, 2 <= lg <= 6; a zero nibble takes
                                    corr_variant.  An autotuner fills it from
                                    timed encodes of the caller's workload. */
  uint32_t corr_tile_levels;     /* tuning of the generated-atom correlation
                                    (variant 6, N = 32 and 64): the node tile of
                                    a launch is 32 MB nodes, MB chosen from the
                                    active-node count inside [lo, hi].  Byte
                                    8 (lg - 5) holds lo in its low nibble and hi
                                    in its high nibble for N = 2^lg; a zero byte
                                    takes the library's range (3..7 at N = 64,
                                    1..7 at N = 32); 1 <= lo <= hi <= 7.  Results
                                    do not depend on it. */
  int32_t reserved;
} aqmp_options;

/* A leaf of the quadtree (or, from aqmp_code_export_nodes, any visited
 * node).  Its atoms are atom_idx[atom_off .. atom_off + n_atoms) with
 * coefficients coef[...] in MP order.  flags bit 0: the node was split. */
typedef struct {
  int32_t job;
  int32_t x0, y0, n;
  int32_t n_atoms;
  int32_t flags;
  int64_t atom_off;
  double resid_sq;          /* ||r||^2 when MP stopped (FP64) */
} aqmp_leaf;

typedef struct {
  int64_t nodes[7];         /* visited nodes per log2(N)                    */
  int64_t leaves[7];        /* leaves per log2(N)                           */
  int64_t iters_level[7];   /* MP iterations executed per log2(N)           */
  int64_t iters_executed;   /* MP iterations, nodes later split included    */
  int64_t iters_emitted;    /* MP iterations kept in leaves                 */
  int64_t steps_launched;   /* MP steps issued (levels x k)                 */
} aqmp_stats;

/* Device time of the last encode, per log2(N), from HIP events (only with
 * AQMP_OPT_TIMING): correlation and select times are kernel execution times
 * (start and end recorded by each dispatch); level times span the level's
 * launches on the stream. */
typedef struct {
  double corr_ms[7];        /* correlation + top-R key launches (Gram and
                               OMP solvers, N >= 16: the initial-
                               correlation launch)                         */
  double select_ms[7];      /* re-score / update / norm launches (Gram and
                               OMP solvers, N >= 16: the pursuit launch)    */
  double level_ms[7];       /* whole level: gather .. split/emit            */
  int64_t steps[7];         /* MP steps timed (Gram and OMP solvers: one
                               per level)                                   */
} aqmp_timing;

/* ---- dictionaries (Section 2.1; Section 2.3 "D_N assumed available") --- */

/* Builds D_N for every N = n_min, 2 n_min, ..., n_max (4 <= N <= 64) with the
 * given families (AQMP_DCT | AQMP_HAAR, DCT first).  The 1D tables are
 * computed in FP64 on the host; the device keeps the FP64 tables and the
 * atoms rounded to FP32 and to BF16.  *out is owned by the library; free it
 * with aqmp_dictionary_free.  Synchronous (returns when uploaded). */
int aqmp_dictionary_build(int n_min, int n_max, uint32_t families,
                          void* hip_stream, aqmp_dict** out);

/* Null-safe. */
void aqmp_dictionary_free(aqmp_dict* d);

/* Number of atoms M_N of block size n; AQMP_E_NODICT if n was not built. */
int aqmp_dictionary_atoms(const aqmp_dict* d, int n, int* m_out);

/* Copies D_N in FP64 to host memory as an N^2 x M column-major matrix:
 * element (flattened pixel j*N + i, atom a) at host_out[a * N*N + j*N + i].
 * host_out must hold N*N*M doubles. */
int aqmp_dictionary_copy(const aqmp_dict* d, int n, double* host_out);

/* ---- encoder (Algorithms 1-2, MP of Section 2.2) ----------------------- */

/* Encodes n_jobs jobs.  Every image, parameter set and job is validated on
 * the host first (AQMP_E_INVALID, AQMP_E_NODICT).  A plane whose width or
 * height is not a multiple of the job's n_max is tiled as if padded up to
 * the next multiple by repeating its last row and column; the padding's
 * blocks are coded like the others and aqmp_decode writes only the image's
 * own pixels.  The call
 * allocates the code's device buffers (worst case for these shapes), then
 * enqueues the encode on hip_stream and returns; *out is valid once that
 * stream's work has completed (the aqmp_code_* readers synchronise it).
 * The images must stay valid until then.  The returned handle keeps its
 * buffers (and, for the batched schedule, its graph) for aqmp_reencode. */
int aqmp_encode(const aqmp_dict* d,
                const aqmp_image* imgs, int n_imgs,
                const aqmp_params* prm, int n_prm,
                const aqmp_job* jobs, int n_jobs,
                const aqmp_options* opt, void* hip_stream, aqmp_code** out);

/* Runs the same encode again on new planes of the same count, types and
 * shapes (device pointers and strides may change), on hip_stream, reusing
 * the handle's buffers and graph.  Previous results are overwritten. */
int aqmp_reencode(aqmp_code* c, const aqmp_image* imgs, int n_imgs, void* hip_stream);

/* Synchronises the encode stream, then reports the number of leaves and of
 * atoms kept in leaves. */
int aqmp_code_sizes(const aqmp_code* c, int64_t* n_leaves, int64_t* n_atoms);

/* Copies the leaves in canonical order (job, then top-level blocks in raster
 * order, then depth-first TL, TR, BL, BR) with their atoms to host buffers.
 * AQMP_E_CAPACITY (nothing written) if cap_leaves or cap_atoms is too small. */
int aqmp_code_export(const aqmp_code* c, aqmp_leaf* leaves, int32_t* atom_idx,
                     double* coef, int64_t cap_leaves, int64_t cap_atoms);

/* Like aqmp_code_export, but for every visited node (split nodes included,
 * flags bit 0 set, with the atoms MP chose before the split was decided).
 * Sizes: aqmp_code_stats (sum of nodes[] and iters_executed). */
int aqmp_code_export_nodes(const aqmp_code* c, aqmp_leaf* nodes, int32_t* atom_idx,
                           double* coef, int64_t cap_nodes, int64_t cap_atoms);

int aqmp_code_stats(const aqmp_code* c, aqmp_stats* s);

/* ---- quality (Section 3) ------------------------------------------------ */

enum { AQMP_SSIM_GLOBAL = 0, AQMP_SSIM_WINDOW7 = 1 };

/* SSIM of two device planes of one size and dtype (Section 3's equation,
 * C1 = (0.01 L)^2, C2 = (0.03 L)^2 with L = data_range).  AQMP_SSIM_GLOBAL:
 * the equation with the means, variances and covariance of the whole planes
 * (population moments).  AQMP_SSIM_WINDOW7: the equation on every 7 x 7
 * window inside the planes (uniform weights, sample moments), averaged over
 * the windows; planes of at least 7 x 7.  Enqueued on hip_stream, then
 * synchronised; *out (host) receives the value.  Allocates a small device
 * buffer per call. */
int aqmp_ssim(const aqmp_image* x, const aqmp_image* y, int mode, double data_range,
              double* out, void* hip_stream);

/* ---- bitstream (encoder step (iii), Section 2.3; CR of Section 3) ------- */

/* Packs the given jobs, as the channels of one image (same plane size and
 * block range), into the AQMP bitstream and compresses it with DEFLATE
 * (zlib compress2 at `level` 0..9; -1 leaves the stream uncompressed).
 * Format (version 1, little-endian): header "AQMP", u8 version, u8
 * families, u8 coefficient format (0 = binary32; 1 = quantised, see
 * aqmp_code_pack_quantized), u8 channels, u32 width, u32 height, u8 log2
 * N_min, u8 log2 N_max, u8 bytes per atom count, u8 0 (format 0);
 * then per channel, nodes in depth-first order (top-level blocks in raster
 * order over the padded plane, children TL, TR, BL, BR): u32 nodes, u32
 * leaves, u32 atoms, the split flags of the nodes with N > N_min (one bit
 * each, LSB first), the atom count of every leaf, the u16 index of every
 * atom, the binary32 coefficient of every atom.  The compression rate of
 * Section 3 is (width x height x channels bytes of 8-bit samples) / size.
 * out == NULL: *size_out receives the exact raw size (level -1) or an upper
 * bound of the compressed size.  Otherwise out (host memory, capacity bytes)
 * receives the stream and *size_out its size; AQMP_E_CAPACITY if it does
 * not fit.  Synchronises the encode stream. */
int aqmp_code_pack(const aqmp_code* c, const int32_t* jobs, int n_jobs, int level,
                   uint8_t* out, int64_t capacity, int64_t* size_out);

/* aqmp_code_pack with the coefficients quantised (coefficient format 1):
 * the lossy part of encoder step (ii), Section 2.3, which the paper does not
 * specify; this uniform scalar quantiser is the library's reading.  With d
 * the step rounded to binary32, each coefficient c is stored as the integer
 * q = round-half-to-even(c / d), computed in FP64; the decoder's value is
 * q * d, within d / 2 of c.  Format 1 differs from format 0 in: the
 * coefficient format byte is 1, the header's last byte is the integer width
 * (2 when every |q| <= 32767, else 4), the binary32 step d follows the
 * 20-byte header, and the coefficients are signed little-endian integers of
 * that width.  step > 0, finite; AQMP_E_INVALID if a |q| exceeds 2^31 - 1.
 * step = 0 gives exactly aqmp_code_pack's stream. */
int aqmp_code_pack_quantized(const aqmp_code* c, const int32_t* jobs, int n_jobs, int level, double step,
                             uint8_t* out, int64_t capacity, int64_t* size_out);

/* Synchronises the encode stream and sums the per-launch event times of the
 * last encode or re-encode.  AQMP_E_INVALID if the code was not made with
 * AQMP_OPT_TIMING. */
int aqmp_code_timing(const aqmp_code* c, aqmp_timing* t);

/* Null-safe; waits for the handle's stream work first. */
void aqmp_code_free(aqmp_code* c);

/* ---- decoder (Algorithm 3) --------------------------------------------- */

/* Writes job's reconstruction sum_t c_t phi_{i_t} of every leaf, placed at
 * its (x0, y0), into dev_out (device, dtype AQMP_F32 or AQMP_F64, h rows of
 * w samples of the job's plane, row stride row_stride samples); no clipping.
 * Samples outside every leaf are not written (leaves tile the plane).
 * Stream-ordered on hip_stream, after the encode's stream work. */
int aqmp_decode(const aqmp_dict* d, const aqmp_code* c, int job,
                void* dev_out, int dtype, int64_t row_stride, void* hip_stream);

/* aqmp_decode with every coefficient replaced by its quantised value q * d
 * (d = step rounded to binary32, q as in aqmp_code_pack_quantized): the
 * image a decoder of the format 1 stream reconstructs.  step > 0, finite;
 * step = 0 is aqmp_decode. */
int aqmp_decode_quantized(const aqmp_dict* d, const aqmp_code* c, int job, double step, void* dev_out, int dtype,
                          int64_t row_stride, void* hip_stream);

/* ---- the integer worklist steps on their own ----------------------------
 * The encoder's active-list compaction and split/emit kernels, applied to
 * caller arrays, so that this integer work can be checked bit for bit.  Both
 * calls allocate a small device scan state per call (a few bytes per 1024
 * items), run on hip_stream, and synchronise it before returning. */

/* Active list (Section 2.2 step (d): the nodes whose pursuit has not stopped
 * go on).  dev_status: n node status bytes (device), 0 = running, any other
 * value = stopped.  Writes to dev_out (device, room for n int32), in
 * increasing order, every i in [0, n) with dev_status[i] == 0, and their
 * number to *dev_count (device int32).  dev_out past the count is not
 * written.  0 <= n <= 2^28.  AQMP_E_HIP if a bounded device wait ran out. */
int aqmp_worklist_compact(const uint8_t* dev_status, int64_t n, int32_t* dev_out, int32_t* dev_count,
                          void* hip_stream);

/* aqmp_worklist_compact without any device allocation, for callers that
 * cannot allocate (code that runs while other work is being captured, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, result
 * and errors; n may not exceed 2^24 (AQMP_E_INVALID beyond that).  The scan
 * state is a fixed array of about 128 KiB of device memory inside the library, one
 * per device, held until the process ends and cleared by every call before
 * use.  Calls on one device share it: calls that overlap on one device
 * (other threads, or other streams before this one has returned) race.
 * Synchronises hip_stream before returning. */
int aqmp_worklist_compact_noalloc(const uint8_t* dev_status, int64_t n, int32_t* dev_out, int32_t* dev_count,
                                  void* hip_stream);

/* Split test and child emission of one quadtree level of block size n
 * (Algorithm 2: a block that misses its target is refined into the four
 * quadrants of its original pixels).  Node i (0 <= i < n_nodes) uses the
 * parameter set prm[dev_node_prm[i]] (host array prm of n_prm sets); it is
 * split when n > n_min and, under AQMP_SPLIT_R1, dev_e[i] (its ||r||^2 after
 * MP) >= eps_n^2, or under AQMP_SPLIT_R2, dev_t[i] (its iterations) >= k_n,
 * with eps_n and k_n as in aqmp_params.  For a split node, bit 4 (0x10) of
 * dev_status[i] is set (the other bits are kept), and its four children,
 * of size n/2, in the order top-left, top-right, bottom-left, bottom-right,
 * go to positions child_base + 4 p .. child_base + 4 p + 3 of dev_child_prm
 * (the node's parameter set), dev_child_x0 and dev_child_y0, where p counts
 * the split nodes before i.  *dev_child_count receives child_base + 4 x (split
 * nodes).  All node and child arrays are device memory; the child arrays
 * need room for child_base + 4 n_nodes entries; entries before child_base and
 * past the count are not written.  n is a power of two in [8, 64],
 * 0 <= n_nodes <= 2^28.  AQMP_E_HIP if a node names a parameter set outside
 * [0, n_prm) (that node is not split) or a bounded device wait ran out. */
int aqmp_worklist_split(const aqmp_params* prm, int n_prm, int n, const int32_t* dev_node_prm, const int32_t* dev_x0,
                        const int32_t* dev_y0, const double* dev_e, const int32_t* dev_t, int64_t n_nodes,
                        int32_t child_base, uint8_t* dev_status, int32_t* dev_child_prm, int32_t* dev_child_x0,
                        int32_t* dev_child_y0, int32_t* dev_child_count, void* hip_stream);

/* Message for the calling thread's last failure ("" if none). */
const char* aqmp_last_error(void);

/* Name of the correlation kernel (MP step (b) of Section 2.2, c = D^T r) that
 * an encode runs for block size n with the given precision (AQMP_PREC_*) and
 * aqmp_options.corr_variant (0 = library default), e.g. for labelling
 * profiles.  Static string owned by the library; "" for an invalid
 * combination (n not a power of two in [AQMP_MIN_N, AQMP_MAX_N], unknown
 * precision or variant).  Levels with n <= 8 run the fused per-level pursuit
 * instead; their name is returned for those n. */
const char* aqmp_corr_kernel(int n, int precision, int corr_variant);

#ifdef __cplusplus
}
#endif
#endif /* AQMP_H */
