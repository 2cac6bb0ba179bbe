// Internal to libdash: the context (every device buffer and the host view of
// a decomposition) and the host steps that dash_host.cpp and dash_server.cpp
// share.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <string>
#include <vector>

#include "dash.h"
#include "dash_dev.h"

namespace dash {

constexpr int kStages = 4;             // pinned descriptor blocks in rotation
constexpr int kMaxChunks2 = 8192;      // bound on solve-stage chunks of the split sweep
constexpr int kServeCUs = 16;          // compute units a served stream's schedule plans for
constexpr int kServeSolveCUs = 64;     // the same, for its solve chunks
constexpr int64_t kServeChunkBytes = 512 << 10;   // Y bytes of a served stream's F-stage chunk

struct PendingGroup {
  int32_t slice;
  const float *src;
  int64_t nrows;
  int64_t out_row;
};

struct InFlight {
  int64_t step;
  int32_t K_prev, K_after;
  int64_t rows;
  int slot;
  int cand;        // autotuning candidate the update ran with, or -1
  double bytes;    // its algorithmic bytes (the autotuner's cost unit)
  int n_items;     // slices that received rows
  bool scored;     // anomaly scores were computed
};

// How an update is launched: sweep variant, slices per wave (or workgroup)
// relative to the default, and whether the final phase rides in the sweep.
struct Schedule {
  int variant;
  int spread;   // 1: the default chunking; 2: twice the slices per chunk
  int fuse;
  int solve_div = 1;   // split sweep: solve chunks 1/solve_div of the default (more, shorter)
};

}  // namespace dash


// the C ABI's opaque context (global namespace, as dash.h declares it)
using namespace dash;

struct dash_ctx {
  dash_config cfg{};
  int J = 0, R = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool served = false;   // a server's stream: launched in the server's batched ticks
  int32_t fail_next = 0; // dash_debug_fail_next: the site whose next call fails (0: none)
  bool server_ingest = false;   // the server is staging a request (dash_ingest_* allowed)
  std::string err;
  int64_t K_cap = 0, M_cap = 0, G_cap = 0, N_init_cap = 0;
  // device state
  float *Y = nullptr;
  uint16_t *Yc = nullptr;   // compensation words of Y (BF16 bits) and D (mixed precision only)
  float *Dc = nullptr;
  float *D = nullptr;
  double *n = nullptr;
  uint8_t *cur = nullptr;
  int32_t *tlast = nullptr;
  double *W = nullptr;
  char *vb = nullptr;
  int64_t vb_stride = 0;
  Ctl *ctl = nullptr;
  float *U_out = nullptr;
  double *partials = nullptr;
  double *gpart = nullptr;
  int32_t *counters = nullptr;
  // split sweep
  double *cbuf = nullptr;    // [K_cap][R] c_k of touched slices
  double *part2 = nullptr;   // [kMaxChunks2][R*R+1]
  int32_t *tag = nullptr;    // [K_cap]
  int32_t *queue = nullptr;  // row-stage counters [4]
  int32_t *slow_list = nullptr;   // [K_cap] deferred row-stage items (and solve-stage systems)
  int32_t *solve_defer = nullptr; // [min(K_cap, kMaxChunks2)] deferred systems per solve chunk
  double *cst = nullptr;     // lagged: [2][K_cap][R]
  double *FG = nullptr;      // lagged: [2][R*J + R*R]
  int32_t seq = 0;           // enqueue sequence (never reused)
  int rows_blocks = 0;       // row-stage workgroups per launch
  size_t off_items = 0;      // descriptor offset of the items of the update being built
  int n_items = 0, n_chunks2 = 0, chunk2 = 0;
  // anomaly scores (dash_anomaly)
  int anom_window = 0;
  AnomalyArgs anom{};
  std::deque<double> te_hist;   // te of committed scored updates (the last anom_window)
  int anom_n_last = -1;         // slices scored by the last committed scored update
  int64_t *d_rowptr = nullptr;
  char *dstep[kStages] = {nullptr, nullptr, nullptr, nullptr};   // device copies of the stages
  char *hstage_dev[kStages] = {nullptr, nullptr, nullptr, nullptr};   // device view of the pinned stages
  bool desc_fetch = true;   // true: copy each descriptor to device memory first; false: kernels read it in place
  size_t off_args = 0, off_gptr = 0, off_groups = 0, step_bytes = 0;   // descriptor layout
  int variant = kPassWave;
  bool variant_forced = false;   // the wave sweep at every K (a test override)
  Schedule sched{kPassWave, 1, 1};         // current schedule
  // autotuning (dash_autotune): candidates tried in turn over the next updates,
  // each scored by device time per algorithmic byte; the best is kept
  std::vector<Schedule> tune_cands;
  std::vector<double> tune_us, tune_bytes;
  std::vector<int> tune_n;
  int tune_per = 0, tune_next = 0;
  bool tuned = false;
  std::string tune_cache;    // JSON-lines file of tuned schedules ("" = none)
  std::string tune_key;      // key of the update shape being tuned
  bool tune_from_cache = false;
  int fused_lds = 0;   // > 0: the sweep launch runs the final phase too (its dynamic LDS)
  int n_cu = 0;   // compute units of the device
  // pinned
  char *hstage[kStages] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t stage_ev[kStages] = {nullptr, nullptr, nullptr, nullptr};
  bool stage_used[kStages] = {false, false, false, false};
  int stage_next = 0;
  Report *hreport = nullptr;
  Report *dreport = nullptr;
  // host-side view of the state
  bool initialized = false;
  int32_t K = 0;          // committed slices
  int64_t step = 0;       // committed updates
  int64_t m_last = 0;     // rows of the last committed update
  int32_t K_enq = 0;      // slices after the last enqueued update
  int64_t step_enq = 0;
  int32_t K_pending = 0;  // including staged new slices
  std::vector<PendingGroup> pending;
  int64_t rows_pending = 0;
  std::deque<InFlight> inflight;
  // graph mode: an update's launches (descriptor fetch, n_iter sweeps, final
  // phases) replayed from an instantiated graph whose kernel-node parameters
  // (grid sizes, descriptor pointers) are rewritten for every update.  One
  // graph per descriptor stage: a stage is reused only after the update that
  // last used it has completed, so no graph is rewritten while in flight.
  bool graph_on = false;
  hipGraph_t graph[kStages] = {};
  hipGraphExec_t gexec[kStages] = {};
  std::vector<hipGraphNode_t> gnodes[kStages];      // kernel nodes in launch order
  std::vector<hipKernelNodeParams> gparams[kStages];   // their captured parameters
  Schedule gsched{-1, 0, 0};                // the schedule the graphs were captured with
  bool spans_on = false;                   // collect every reaped update's device span
  std::vector<float> spans;                // spans (ms) of the reaped updates
  int chunk_override = 0;
  std::vector<int> order;  // scratch
  // profiling: event pairs around launches, folded into stats on read
  bool profiling = false;   // events around this update's launches
  int prof_every = 0;       // > 0: profile the updates whose index is a multiple of it
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;  // kind per recorded pair
  int ev_used = 0;           // pairs recorded since the last fold
  dash_profile_stats prof{};
};

namespace dash {

// An update whose descriptor has been written (build_update) but whose kernels
// are not yet enqueued: the stage it sits in and the launch sizes.
struct BuiltUpdate {
  int stage = 0;           // descriptor stage
  size_t bytes = 0;        // descriptor bytes to bring to the device
  const char *dblk = nullptr;   // device address the kernels read it from
  int nch = 0;             // F-stage (or sweep) chunks
  int n_chunks2 = 0;       // solve-stage chunks (split sweep)
  int n_items = 0;         // slices that received rows
  int64_t step = 0;
  int slot = 0;            // report slot
  int cand = -1;           // autotuning candidate
  bool scored = false;
  void *report = nullptr;  // device address of the report
  int K = 0;               // slices after the update
  int64_t rows = 0;        // rows it consumes
};

dash_status fail(dash_ctx *c, dash_status s, const char *fmt, ...);
// true when the next descriptor stage can be rewritten without waiting
bool stage_free(dash_ctx *c);
// Write the descriptor of the staged rows into the next stage (waits for it
// when it is still in use).  Nothing is enqueued.
dash_status build_update(dash_ctx *c, BuiltUpdate *b);
// After an update's kernels are enqueued: in-flight record, staging cleared.
void account_update(dash_ctx *c, const BuiltUpdate &b);
PassArgs base_args_at(const dash_ctx *c, const char *d);
const PassArgs *args_dev(const dash_ctx *c, const char *d, int p);
int64_t context_footprint(const dash_config *cfg);
// dash_create with a given HIP stream; served = true fixes the schedule a
// served stream runs with (split sweep, chunking independent of the device
// and of other streams).
dash_status create_context(const dash_config *cfg, hipStream_t stream, bool served, dash_ctx **out);
// dash_init in parts: argument checks, the size of its device workspace (in
// doubles), and the initialisation itself on a given workspace (synchronous:
// the workspace is free again when it returns).
dash_status init_check(dash_ctx *c, int32_t K, const int64_t *row_ptr, const float *X);
// Whether p points to device memory; the initial row_ptr as host memory (a
// device array is copied into tmp and p redirected there).
bool on_device(const void *p);
dash_status host_row_ptr(dash_ctx *c, const int64_t *&p, int32_t K, std::vector<int64_t> &tmp);
size_t init_workspace_doubles(const dash_ctx *c, int32_t K, bool has_v0);
dash_status init_with_workspace(dash_ctx *c, int32_t K, const int64_t *row_ptr, const float *X, const float *V0,
                                dash_init_report *report, double *ws);

}  // namespace dash
