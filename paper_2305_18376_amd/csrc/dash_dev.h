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
constexpr double kWCutoff = 1e-12;    // 1/w := 0 below this fraction of max|w|
constexpr int kReportRing = 64;       // pinned report slots (updates in flight)

// Per-update descriptor block, written by the host into pinned memory and
// copied to the device once per update (one hipMemcpyAsync).
struct StepHeader {
  int32_t K;          // slices after the update
  int32_t K_prev;     // slices before it (ids >= K_prev are new)
  int32_t n_touched;  // slices that received rows
  int32_t n_groups;   // row groups (ingest calls x groups), sorted by slice
  int32_t n_chunks;   // slice chunks of the sweep
  int32_t chunk;      // slices per chunk
  int32_t n_rgroups;  // first-level reduction groups of chunk partials
  int32_t chunks_per_rgroup;
  int64_t step;       // 1-based index of this update
  int64_t M;          // rows in the update
  void *report;       // device-visible pointer to this update's pinned report slot
};

struct Touched {      // one slice that received rows; its groups are [g_begin, g_end)
  int32_t slice, g_begin, g_end, pad;
};

struct Group {        // contiguous rows of one slice, in the caller's buffer
  const float *src;   // nrows x J, row-major
  int64_t out_row;    // first row of U_new (ingest order)
  int32_t nrows, pad;
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
  int32_t done, pad;
};

// One "V bundle": everything a pass needs from V, double-buffered.
//   V64  [J][R]  float64 master
//   VtV  [R][R]  float64 V^T V
//   Vt32 [R][J]  float32 V^T   (for c_k = diag(Y_k V))
//   P32  [J][R]  float32 V (V^T V)^{-1}  (Lemma 1 projector)
struct VBundleView {
  double *V64, *VtV;
  float *Vt32, *P32;
};

__host__ __device__ inline int64_t vb_bytes(int J, int R) {
  int64_t b = (int64_t)J * R * 8 + (int64_t)R * R * 8 + (int64_t)R * J * 4 + (int64_t)J * R * 4;
  return (b + 255) / 256 * 256;
}

__host__ __device__ inline VBundleView vb_view(char *base, int J, int R) {
  VBundleView v;
  v.V64 = (double *)base;
  v.VtV = v.V64 + (int64_t)J * R;
  v.Vt32 = (float *)(v.VtV + (int64_t)R * R);
  v.P32 = v.Vt32 + (int64_t)R * J;
  return v;
}

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Size of one sweep partial: F^T (R*J), G (R*R), sum n.
__host__ __device__ inline int partial_len(int J, int R) { return R * J + R * R + 1; }

// Arguments of the fused pass kernel (by value).
struct PassArgs {
  int J, R;
  double lambda;
  int pass;            // 0-based ALS pass within the update
  int write_u;         // write U_new rows (last pass)
  int mode;            // 0: update pass, 1: evaluate F/G with current W (no solve, no writes)
  int64_t K_cap;
  const StepHeader *hdr;
  const int32_t *chunk_tptr;   // [n_chunks+1] first touched entry per chunk
  const Touched *touched;
  const Group *groups;
  float *Y;            // [2][K_cap][R][J]
  float *D;            // [2][K_cap][R][R]
  double *n;           // [2][K_cap]
  uint8_t *cur;        // [K_cap] committed buffer of Y/D/n per slice
  int32_t *tlast;      // [K_cap] step of the last commit of the slice
  double *W;           // [2][K_cap][R]
  char *vb;            // 2 V bundles
  int64_t vb_stride;
  Ctl *ctl;
  float *U_out;        // [M_cap][R]
  double *partials;    // [n_chunks][partial_len]
};

// Launchers (dash_kernels.hip).
int launch_pass(const PassArgs &a, int n_chunks, hipStream_t s);
int launch_reduce(const double *partials, double *gpart, const StepHeader *hdr, int plen,
                  int n_chunks, int n_rgroups, int chunks_per_rgroup, hipStream_t s);
// mode 0: reduce + V = F G^{-1} + prep of next bundle + fit; mode 1: prep bundle from V64 of
// the committed bundle (init/set_state); mode 2: fit only (F, G from partials, V committed).
int launch_solve(int J, int R, const double *gpart, int n_rgroups, char *vb, int64_t vb_stride,
                 Ctl *ctl, int mode, hipStream_t s);
int launch_commit(const StepHeader *hdr, const Touched *touched, uint8_t *cur, int32_t *tlast,
                  Ctl *ctl, int n_touched, hipStream_t s);
int launch_accum_given_u(int J, int R, int K, const int64_t *row_ptr_dev, const float *X,
                         const float *U, float *Y, float *D, double *n, hipStream_t s);
int launch_v_from_f32(int J, int R, const float *V, char *vb_committed, hipStream_t s);
int launch_w_from_f32(int R, int K, const float *W, double *Wc, hipStream_t s);
int launch_export_state(int J, int R, int K, int64_t step, double lambda, const float *Y,
                        const float *D, const double *n, const uint8_t *cur, const int32_t *tlast,
                        int64_t K_cap, double *Yo, double *Do, double *no, hipStream_t s);
int launch_gather_state(int J, int R, int K, const float *Y, const float *D, const double *n,
                        const uint8_t *cur, int64_t K_cap, float *Yo, float *Do, double *no,
                        hipStream_t s);
int launch_to_f32(const double *src, float *dst, int64_t count, hipStream_t s);

}  // namespace dash
