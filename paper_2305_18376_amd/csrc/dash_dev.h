// Layouts shared by the host core (dash_host.cpp) and the gfx950 kernels
// (dash_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace dash {

constexpr int kBlock = 256;           // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxR = 32;             // rank limit: one wave64 owns an R x R factorisation
constexpr int kMaxJ = 256;            // column limit: a row of Y_k is <= 4 floats per lane
constexpr double kPivotRel = 1e-12;   // Cholesky pivot threshold relative to max diagonal
constexpr double kEigCutoff = 1e-12;  // pseudo-inverse / inverse-sqrt eigenvalue cutoff
constexpr int kReportRing = 64;       // pinned report slots (updates in flight)
constexpr int kMaxChunks = 4096;      // bound on sweep chunks (partials memory)
constexpr int kWaveWarps = 8;         // waves per workgroup of the wave sweep
constexpr int kWaveMaxSlices = 4;     // default schedule: the wave sweep while each wave holds at most this many slices
constexpr int kChunksPerRGroup = 16;  // first-level reduction fan-in

// Per-update descriptor block, written by the host into pinned memory and
// copied to the device by a fetch kernel once per update:
//   StepHeader | int32 chunk_gptr[n_chunks+1] | Group groups[n_groups] | Item items[n_items]
// Groups are sorted by slice (ingest order within a slice); chunk c covers
// slices [c*chunk, (c+1)*chunk) and its groups start at chunk_gptr[c].  Items
// list the touched slices, most rows first.
struct StepHeader {
  int32_t K;          // slices after the update
  int32_t K_prev;     // slices before it (ids >= K_prev are new)
  int32_t n_groups;   // row groups, sorted by slice
  int32_t n_chunks;   // slice chunks of the sweep (one workgroup each)
  int32_t chunk;      // slices per chunk
  int32_t n_rgroups;  // first-level reduction groups of chunk partials
  int32_t chunks_per_rgroup;
  int32_t n_items;    // touched slices (split sweep: the row stage's work items)
  int64_t step;       // 1-based index of this update (the committed index for evaluations)
  int64_t M;          // rows in the update
  void *report;       // device-visible pointer to this update's pinned report slot
  int32_t n_chunks2;  // split sweep: solve-stage chunks (chunk2 slices each)
  int32_t chunk2;     // a sweep chunk is (chunk / chunk2) solve chunks
  int32_t seq;        // enqueue sequence number (never reused, rolled-back updates included)
  int32_t force_fail; // 1: the commit check treats this update as non-finite (injected failure)
};

// One touched slice of an update: its row groups are groups[g0 .. g1).
struct Item {
  int32_t slice, g0, g1, rows;
};

struct Group {        // contiguous rows of one slice, in the caller's buffer
  const float *src;   // nrows x J, row-major
  int64_t out_row;    // first row of U_new (ingest order)
  int32_t nrows;
  int32_t slice;
};

// Device-resident control block.
struct Ctl {
  int32_t gcur;       // which of the two W / V-bundle buffers is committed
  int32_t poison;     // set once an update failed: later in-flight updates do not commit
  int32_t ok;         // factors of the update in progress are finite
  int32_t pad;
  double loss, fit, sum_n;
};

// Layout of one pinned report slot (mirrors dash_update_report plus a flag).
struct Report {
  int64_t step, rows;
  int32_t K, committed;
  double fit, loss, sum_n;
  uint64_t t_start, t_end;   // device realtime clock (100 MHz) at the update's first and last launch
  double te;                 // tensor-level error of the update (anomaly scores on)
  int32_t n_anomalies;       // slices flagged by the slice-level threshold
  int32_t done;
};
constexpr double kRealtimeMHz = 100.0;

// One "V bundle": everything a pass needs from V, double-buffered.
//   V64  [J][R]  float64 master
//   VtV  [R][R]  float64 V^T V
//   piv  [R]     float64 elimination pivots of V^T V (the squares of its Cholesky
//                diagonal; all 0 when V^T V failed the acceptance rule)
//   Vt32 [R][J]  float32 V^T   (for c_k = diag(Y_k V))
//   P32  [J][R]  float32 V (V^T V)^{-1}  (Lemma 1 projector; pseudo-inverse if singular)
struct VBundleView {
  double *V64, *VtV, *piv;
  float *Vt32, *P32;
};

__host__ __device__ inline int64_t vb_bytes(int J, int R) {
  int64_t b = (int64_t)J * R * 8 + (int64_t)R * R * 8 + (int64_t)R * 8 + (int64_t)R * J * 4 +
              (int64_t)J * R * 4;
  return (b + 255) / 256 * 256;
}

__host__ __device__ inline VBundleView vb_view(char *base, int J, int R) {
  VBundleView v;
  v.V64 = (double *)base;
  v.VtV = v.V64 + (int64_t)J * R;
  v.piv = v.VtV + (int64_t)R * R;
  v.Vt32 = (float *)(v.piv + R);
  v.P32 = v.Vt32 + (int64_t)R * J;
  return v;
}

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Floats per slice of the Y state: R*J rounded up to whole wave64 rows (the
// padding stays zero), so wave-wide loads and stores need no bounds checks.
__host__ __device__ inline int y_stride(int J, int R) { return (R * J + 63) / 64 * 64; }

// Size of one sweep partial: F^T (R*J), G (R*R), sum n.
__host__ __device__ inline int partial_len(int J, int R) { return R * J + R * R + 1; }

// Arguments of the pass kernels (by value).
struct PassArgs {
  int J, R;
  int ys;              // floats per slice of Y (y_stride)
  double lambda, log2_lambda;
  int pass;            // 0-based ALS pass within the update
  int last_pass;       // this pass writes U_new and commits
  int mode;            // 0: update pass, 1: evaluate the committed state (fit only)
  int64_t K_cap;
  const StepHeader *hdr;
  const int32_t *chunk_gptr;   // [n_chunks+1]
  const Group *groups;
  float *Y;            // [2][K_cap][ys]: R x J row-major, zero padded
  uint16_t *Yc;        // mixed precision: compensation of Y as BF16 bits (same layout), else NULL
  float *Dc;           // mixed precision: compensation of D, else NULL
  float *D;            // [2][K_cap][R][R]
  double *n;           // [2][K_cap]
  uint8_t *cur;        // [2][K_cap] buffer of Y/D/n holding each slice (by gcur)
  int32_t *tlast;      // [2][K_cap] update index of the slice's last fold (by gcur)
  double *W;           // [2][K_cap][R]
  char *vb;            // 2 V bundles
  int64_t vb_stride;
  Ctl *ctl;
  float *U_out;        // [M_cap][R]
  double *partials;    // [n_chunks][partial_len]
  double *gpart;       // [n_rgroups][partial_len]
  int32_t *counters;   // [kMaxChunks + 1] arrival tickets (the last one: all groups), zero between launches
  int fuse;            // the last workgroup to arrive runs the final phase in the same launch
  int mixed;           // 1: Lemma 1 and the row accumulation on BF16 MFMA (FP32 sums)
  int stamp_start;     // 1: the first pass's workgroup 0 stamps the report's start time
  int lds_bytes;       // dynamic LDS of the sweep launch
  // split sweep (row stage, solve stage, F stage, final phase)
  const Item *items;   // [n_items] touched slices, heaviest first
  double *cbuf;        // [K_cap][R] c_k of the touched slices of the current pass
  double *part2;       // [n_chunks2][R*R + 1] solve-stage partials (G, sum n)
  int32_t *tag;        // [K_cap] seq of the update that last touched the slice
  int32_t *queue;      // row-stage counters (zero between launches): [0] work queue,
                       // [1] deferred slices, [2] their work queue
  int32_t *slow_list;  // [K_cap] items deferred to Lemma 1's pseudo-inverse form
  int32_t *solve_defer;   // [n_chunks2] slices of a solve chunk deferred to the pseudo-inverse
  int lagged;          // DASH_STATS_LAGGED: Algorithm 1's recursions for c_k, F, G
  double *cst;         // lagged: [2][K_cap][R] stored c_k (buffer by cur)
  double *FG;          // lagged: [2][R*J + R*R] F^T then G (buffer by gcur)
  int defer_done;      // 1: the final phase leaves the report's done flag to the anomaly scores
  int pre_reduced;     // 1: the group partials were summed into group 0 before the final phase
};

// Buffers of the anomaly scores (dash_anomaly): per touched slice of the last
// scored update se, flag, slice id ([G_cap] each, in item order), per slice a
// ring of its previous errors ([K_cap][window]) and their count, a ticket.
struct AnomalyArgs {
  float *se;
  int32_t *flag;
  int32_t *sid;
  float *hist;
  int32_t *hcnt;
  int32_t *ticket;
  int window;
};
int launch_slice_errors(const PassArgs &a, const AnomalyArgs &x, int n_blocks, hipStream_t s);

// One workgroup of a launch that serves several contexts (a serving tick): the
// context's pass arguments (device copy) and the workgroup's index among that
// context's workgroups.  Launches for one context pass no map: workgroup i of
// the launch is its workgroup i.
struct BlockMap {
  const PassArgs *args;
  int32_t local;
  int32_t pad;
};

// A kernel's view of its PassArgs in device memory: the constant address space
// tells the compiler the fields never change during the launch, so it loads
// each where it is used (scalar loads it may repeat) instead of holding a copy
// of the whole block in registers.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) PassArgs CPassArgs;
#else
typedef const PassArgs CPassArgs;
#endif

// Kernel variants of the sweep: one fused launch with one wave per slice, or
// the split sweep (row stage, solve stage, F stage, final phase).
enum { kPassWave = 0, kPassSplit = 1 };

// Arguments of the initial-decomposition kernels (PARAFAC2-ALS, Sec. 3.2.1).
struct InitArgs {
  int J, R, K;
  int ys;              // Y slice stride (y_stride)
  int64_t K_cap;
  const int64_t *row_ptr;   // device [K+1]
  const float *X;      // device [row_ptr[K] x J]
  float *Y;            // state Y [2][K_cap][ys]: buffer 1 holds (X_k V)^T X_k, buffer 0 Y_k
  float *D;            // state D [2][K_cap][R*R]: buffer 0 holds Pi_k
  double *Dh;          // [K][R*R] (X_k V)^T X_k V in FP64 (its rank decides P_k's retained eigenspace)
  double *n;           // state n [K_cap] (buffer 0)
  double *W;           // state W [K_cap][R] (buffer 0)
  double *V64;         // V, J x R (the committed bundle's V)
  double *H;           // R x R
  double *WtW;         // R x R
  double *VtV;         // R x R
  double *Mwinv;       // ((H^T H) * (V^T V))^{-1}, R x R
  double *part;        // chunk partials [n_chunks][plen]
  int plen;            // max(2 R^2, J R) + 2
  int chunk;           // slices per chunk
  int n_chunks;
  double *result;      // [0] loss, [1] sum of n_k
};

int init_gram_chunks(int J);
int launch_init_gram(int J, int64_t N, int n_gc, const float *X, double *part, double *Gm, hipStream_t s);
int launch_sym_eig(int n, double *A, double *Z, double *evals, hipStream_t s);
int launch_top_vectors(int J, int R, const double *evals, const double *Z, double *V64, hipStream_t s);
int launch_init_start(const InitArgs &a, hipStream_t s);
int launch_init_iteration(const InitArgs &a, hipStream_t s);
int launch_init_handoff(const InitArgs &a, hipStream_t s);

// Launchers (dash_kernels.hip).
// Default sweep variant for (J, R, precision, stats mode): kPassWave or kPassSplit.
int pass_variant(int J, int R, int precision, int lagged);
// Slices per workgroup for a variant and slice count.
int pass_chunk(int variant, int K, int n_cu);
int launch_pass(const PassArgs &a, int variant, int n_chunks, hipStream_t s);
// Split sweep launchers (dash_split.hip).  Row stage: n_blocks persistent
// workgroups pulling touched slices from a.queue, then a small launch for the
// slices whose Lemma 1 system needs the pseudo-inverse; solve stage: n_chunks2
// workgroups; F stage: n_chunks workgroups (each sums its solve chunks' G, n
// and arrives at the two-level reduction; the final phase is a separate launch).
// The kernels read their arguments from device memory: `args` (a context's
// PassArgs, device copy) with map = NULL, or map[n_blocks] (several contexts
// of one kernel class: a = the host copy of any of them, for the template
// choice).  The row stage's deferred-slice launch takes kSlowBlocks
// workgroups per context.
constexpr int kSlowBlocks = 32;
// lds: dynamic LDS of the launch (0: the layout of a; a launch for several
// contexts passes the largest of theirs).
int launch_split_rows(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s,
                      size_t lds = 0);
int launch_split_rows_slow(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks,
                           hipStream_t s, size_t lds = 0);
int split_rows_blocks_per_cu(int J, int R, int mixed);
int launch_split_solve(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s,
                       size_t lds = 0);
int launch_split_fsum(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s,
                      size_t lds = 0);
int launch_finish_dev(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, int mode,
                      hipStream_t s, size_t lds = 0);
// The group partials summed into group 0 (one thread per partial entry).
int reduce_groups_blocks(int J, int R);
int launch_reduce_groups(const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s);
// One launch over workgroups of contexts of every class (a server tick): the
// solve stage, the exact-mode F stage and the final phase (mode 0), each
// workgroup running the instantiation of its own context's R (and J).  lds:
// the largest dynamic LDS among the members.
size_t split_rows_lds(int J, int R, int mixed);
size_t split_solve_lds(int J, int R);
size_t split_fsum_lds(int J, int R, int lagged);
size_t finish_dev_lds(int J, int R);
// Kernel classes (launches that may share contexts): equal keys, one launch.
int split_rows_class(int J, int R, int mixed);
int split_solve_class(int R);
int split_fsum_class(int J, int R, int lagged, int mixed);
int finish_class(int R);
// Copy bytes (a multiple of 16 not required) from a device-visible pinned host
// block to device memory with a kernel on stream s.
int launch_fetch(const char *src_mapped, char *dst, size_t bytes, void *report, hipStream_t s);
// The fetch kernel's arguments and grid for bytes (for rewriting a graph node).
struct FetchArgs {
  const void *src, *src_tail;
  void *dst, *dst_tail;
  int64_t n16;
  int tail;
  void *report;   // Report of the update (its start time is written), or NULL
  unsigned grid;
};
FetchArgs fetch_args(const char *src_mapped, char *dst, size_t bytes, void *report);
// One copy of a batched fetch: src (device view of pinned host memory) to
// dst, bytes a multiple of 16; report (or NULL) gets its start time.
struct FetchJob {
  const char *src;
  char *dst;
  int64_t bytes;
  void *report;
};
// Copy every job of jobs[0 .. n_jobs) in one launch; jobs is itself read
// through its device view (pinned host memory).  max_bytes: the largest job.
int launch_fetch_list(const FetchJob *jobs_mapped, int n_jobs, int64_t max_bytes, hipStream_t s);
// LDS of the row stage's deferred-slice kernel.
size_t split_rows_slow_lds(int J, int R);
// The solve stage's deferred systems (those that failed the acceptance rule):
// one workgroup per solve chunk, most of which find nothing to do.
int launch_split_solve_fix(const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s, size_t lds);
// Name of the kernel instantiation a split-sweep stage launches for arguments
// a (stage: 0 rows, 1 deferred slices, 2 solve, 3 F, 4 group reduction, 5
// final phase), e.g. "k_solve<16>"; written into buf (n bytes).
void split_kernel_name(int stage, const PassArgs &a, char *buf, size_t n);
// Dynamic LDS of a sweep launch that also runs the final phase, or 0 when the
// two do not fit one workgroup.
size_t fused_pass_lds(int variant, int J, int R);
// Final phase of a pass (one workgroup): mode 0 after an update sweep (Lemma 3,
// next-pass operands, commit on the last pass), 1 builds the committed V bundle
// from its V64, 2 evaluates the fit after an evaluation sweep.
int launch_finish(const PassArgs &a, int mode, hipStream_t s);
int launch_accum_given_u(int J, int R, int K, const int64_t *row_ptr_dev, const float *X,
                         const float *U, float *Y, float *D, double *n, hipStream_t s);  // Y stride y_stride
int launch_v_from_f32(int J, int R, const float *V, char *vb_committed, hipStream_t s);
int launch_w_from_f32(int R, int K, const float *W, double *Wc, hipStream_t s);
int launch_export_state(int J, int R, int K, int64_t step, double lambda, const float *Y,
                        const float *D, const double *n, const uint8_t *cur, const int32_t *tlast,
                        int64_t K_cap, double *Yo, double *Do, double *no, const uint16_t *Yc, const float *Dc,
                        hipStream_t s);
int launch_gather_state(int J, int R, int K, const float *Y, const float *D, const double *n,
                        const uint8_t *cur, int64_t K_cap, float *Yo, float *Do, double *no,
                        hipStream_t s);
int launch_gather_carry(int J, int R, int K, const uint16_t *Yc, const float *Dc, const uint8_t *cur, int64_t K_cap,
                        float *Yo, float *Do, hipStream_t s);
int launch_to_f32(const double *src, float *dst, int64_t count, hipStream_t s);

}  // namespace dash
