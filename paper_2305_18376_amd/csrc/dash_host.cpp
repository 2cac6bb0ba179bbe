// Host core of libdash: the C ABI of include/dash.h.
//
// Owns every device buffer (allocated once in dash_create), validates and
// stages ingested row groups (metadata on the host, rows left in the caller's
// device buffers), builds the per-update descriptor block and enqueues the
// kernel sequence of dash_kernels.hip.  Updates are transactional: kernels
// write the next state beside the committed one and k_commit switches to it
// only if the update's factors are finite.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "dash_ctx.h"

using namespace dash;

namespace dash {

dash_status fail(dash_ctx *c, dash_status s, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIP_OR_FAIL(c, expr)                                                          \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((c), DASH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_OR_FAIL(c, expr)                                                        \
  do {                                                                                 \
    int e_ = (expr);                                                                   \
    if (e_ != 0)                                                                       \
      return fail((c), DASH_E_DEVICE, "%s failed: %s", #expr,                          \
                  hipGetErrorString((hipError_t)e_));                                  \
  } while (0)

// float -> BF16 bits, rounded to nearest even (the compensation words of Y)
inline uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T>
hipError_t dalloc(T **p, size_t bytes) {
  return hipMalloc((void **)p, bytes < 256 ? 256 : bytes);
}

// Split sweep chunking: F-stage chunks of c3 slices (about two workgroups per
// CU), solve-stage chunks of c2 slices (about eight per CU); c3 is a multiple
// of c2 so that every F-stage chunk sums whole solve chunks.
void split_chunks(const dash_ctx *c, int K, int *c3_out, int *c2_out) {
  const int n = std::max(1, c->n_cu);
  int c3 = std::max(1, (K + 2 * n - 1) / (2 * n));
  // a served stream shares the device: F chunks of about kServeChunkBytes of
  // Y each, whatever the slice size
  if (c->served) c3 = std::max(1, (int)(kServeChunkBytes / (4 * (int64_t)y_stride(c->J, c->R))));
  if (c->chunk_override > 0) c3 = c->chunk_override;
  c3 *= c->sched.spread;
  // solve chunks: two workgroups per CU (one resident round), a multiple of
  // the workgroup's four waves; a served stream plans them for the whole
  // device (short chunks: its latency, not its own throughput, matters)
  const int ns = (c->served ? kServeSolveCUs : n) * std::max(1, c->sched.solve_div);
  int c2 = std::max(1, std::min(c3, (K + 2 * ns - 1) / (2 * ns)));
  c2 = (c2 + 3) / 4 * 4;
  while ((K + c2 - 1) / c2 > kMaxChunks2) c2 += 4;
  c3 = std::max(c3, c2);
  c3 = (c3 + c2 - 1) / c2 * c2;
  while ((K + c3 - 1) / c3 > kMaxChunks) c3 += c2;
  *c3_out = c3;
  *c2_out = c2;
}

int choose_chunk(const dash_ctx *c, int K) {
  if (c->sched.variant == kPassSplit) {
    int c3, c2;
    split_chunks(c, K, &c3, &c2);
    return c3;
  }
  if (c->chunk_override > 0) {
    int ch = c->chunk_override;
    while ((K + ch - 1) / ch > kMaxChunks) ++ch;
    return ch;
  }
  int ch = pass_chunk(c->sched.variant, K, c->n_cu);
  ch *= c->sched.spread;
  int out = std::max(1, std::min(ch, K));
  while ((K + out - 1) / out > kMaxChunks) ++out;
  return out;
}

StepHeader *stage_header(char *blk) { return (StepHeader *)blk; }

enum { kProfPass = 0, kProfReduce, kProfSolve, kProfCommit, kProfUpload };
constexpr int kProfPairs = 1024;

// Fold recorded event pairs into the stats (the stream must be idle).
hipError_t prof_fold(dash_ctx *c) {
  for (int i = 0; i < c->ev_used; ++i) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]);
    if (e != hipSuccess) return e;
    switch (c->ev_kind[i]) {
      case kProfPass: c->prof.pass_launches++; c->prof.pass_ms += ms; break;
      case kProfReduce: c->prof.reduce_launches++; c->prof.reduce_ms += ms; break;
      case kProfSolve: c->prof.solve_launches++; c->prof.solve_ms += ms; break;
      case kProfCommit: c->prof.commit_launches++; c->prof.commit_ms += ms; break;
      default: c->prof.upload_launches++; c->prof.upload_ms += ms; break;
    }
  }
  c->ev_used = 0;
  return hipSuccess;
}

// Open / close a timed region around one launch (no-ops unless profiling).
hipError_t prof_begin(dash_ctx *c, int kind) {
  if (!c->profiling) return hipSuccess;
  if (c->ev_used == kProfPairs) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = prof_fold(c);
    if (e != hipSuccess) return e;
  }
  c->ev_kind[c->ev_used] = kind;
  return hipEventRecord(c->ev[2 * c->ev_used], c->stream);
}

hipError_t prof_end(dash_ctx *c) {
  if (!c->profiling) return hipSuccess;
  hipError_t e = hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream);
  c->ev_used++;
  return e;
}

// Wait until a pinned descriptor block can be rewritten.
hipError_t take_stage(dash_ctx *c, int *idx) {
  const int s = c->stage_next;
  c->stage_next = (c->stage_next + 1) % kStages;
  if (c->stage_used[s]) {
    hipError_t e = hipEventSynchronize(c->stage_ev[s]);
    if (e != hipSuccess) return e;
  }
  *idx = s;
  return hipSuccess;
}

// Bring stage s (bytes) to the device: a fetch kernel on the compute stream
// reads the pinned block through its device mapping, so the update's kernels
// follow it on the same queue without a copy-engine round trip.  The block is
// free for the host again once stage_ev[s] has completed.
hipError_t upload_stage(dash_ctx *c, int s, size_t bytes, bool profile, void *report) {
  hipError_t e = hipSuccess;
  if (!c->desc_fetch) return e;   // the kernels read the pinned block in place (see stage_done)
  if (profile) e = prof_begin(c, kProfUpload);
  if (e == hipSuccess) e = (hipError_t)launch_fetch(c->hstage_dev[s], c->dstep[s], bytes, report, c->stream);
  if (e == hipSuccess && profile) e = prof_end(c);
  if (e == hipSuccess) e = hipEventRecord(c->stage_ev[s], c->stream);
  c->stage_used[s] = true;
  return e;
}

// After the kernels of an update that read stage s in place: the host may
// rewrite the block once they have run.
hipError_t stage_done(dash_ctx *c, int s) {
  if (c->desc_fetch) return hipSuccess;
  c->stage_used[s] = true;
  return hipEventRecord(c->stage_ev[s], c->stream);
}

// Pass arguments of the update whose descriptor block sits at device address d.
PassArgs base_args_at(const dash_ctx *c, const char *d);

PassArgs base_args(const dash_ctx *c, int s) {
  return base_args_at(c, c->desc_fetch ? c->dstep[s] : c->hstage_dev[s]);
}

PassArgs base_args_at(const dash_ctx *c, const char *d) {
  PassArgs a{};
  a.J = c->J;
  a.R = c->R;
  a.ys = y_stride(c->J, c->R);
  a.lambda = c->cfg.lambda;
  a.log2_lambda = std::log2(c->cfg.lambda);
  a.K_cap = c->K_cap;
  a.hdr = (const StepHeader *)d;
  a.chunk_gptr = (const int32_t *)(d + c->off_gptr);
  a.groups = (const Group *)(d + c->off_groups);
  a.Y = c->Y;
  a.D = c->D;
  a.Yc = c->Yc;
  a.Dc = c->Dc;
  a.n = c->n;
  a.cur = c->cur;
  a.tlast = c->tlast;
  a.W = c->W;
  a.vb = c->vb;
  a.vb_stride = c->vb_stride;
  a.ctl = c->ctl;
  a.U_out = c->U_out;
  a.partials = c->partials;
  a.gpart = c->gpart;
  a.counters = c->counters;
  const int flds = c->sched.fuse ? (int)fused_pass_lds(c->sched.variant, c->J, c->R) : 0;
  a.fuse = flds > 0 ? 1 : 0;
  a.mixed = c->cfg.precision == DASH_PREC_MIXED ? 1 : 0;
  a.stamp_start = c->desc_fetch ? 0 : 1;
  a.lds_bytes = flds;
  a.items = (const Item *)(d + c->off_items);
  a.cbuf = c->cbuf;
  a.part2 = c->part2;
  a.tag = c->tag;
  a.queue = c->queue;
  a.slow_list = c->slow_list;
  a.solve_defer = c->solve_defer;
  a.lagged = c->cfg.stats_mode == DASH_STATS_LAGGED ? 1 : 0;
  a.cst = c->cst;
  a.FG = c->FG;
  a.defer_done = c->anom_window > 0 ? 1 : 0;
  return a;
}

// The anomaly-score fields of a reaped update's report: te from the device,
// its moving threshold over this context's previous te (host).
void score_report(dash_ctx *c, const InFlight &f, const Report &r, dash_update_report *out) {
  out->te = 0.0;
  out->te_threshold = 0.0;
  out->te_anomaly = 0;
  out->n_anomalies = 0;
  if (!f.scored || !r.committed) return;
  out->te = r.te;
  out->n_anomalies = r.n_anomalies;
  double thr = INFINITY;
  const size_t n = c->te_hist.size();
  if (n > 0) {
    double mean = 0.0, var = 0.0;
    for (double v : c->te_hist) mean += v;
    mean /= (double)n;
    for (double v : c->te_hist) var += (v - mean) * (v - mean);
    thr = mean + std::sqrt(var / (double)n);
  }
  out->te_threshold = thr;
  out->te_anomaly = r.te > thr ? 1 : 0;
  c->te_hist.push_back(r.te);
  while ((int)c->te_hist.size() > c->anom_window) c->te_hist.pop_front();
  c->anom_n_last = f.n_items;
}

// Device address of the pass arguments of pass p in the descriptor at d.
const PassArgs *args_dev(const dash_ctx *c, const char *d, int p) {
  return (const PassArgs *)(d + c->off_args) + p;
}

// Write the pass arguments of every pass into the descriptor block (host
// copy blk, device address d) for the split sweep's kernels.
void write_pass_args(const dash_ctx *c, char *blk, const char *d, int mode) {
  PassArgs *pa = (PassArgs *)(blk + c->off_args);
  const int n = mode == 0 ? c->cfg.n_iter : 1;
  for (int p = 0; p < n; ++p) {
    PassArgs a = base_args_at(c, d);
    a.fuse = 0;
    a.mode = mode;
    a.pass = p;
    a.last_pass = (mode == 0 && p == n - 1) ? 1 : 0;
    a.pre_reduced = 1;
    pa[p] = a;
  }
}

// The launches of one split-sweep pass: row stage (and its deferred slices),
// solve stage, F stage, final phase.  a: host copy of the pass's arguments,
// ad: their device copy.
dash_status enqueue_split_pass(dash_ctx *c, const PassArgs &a, const PassArgs *ad, int n_items, int n_chunks2,
                               int n_chunks) {
  if (a.mode == 0 && n_items > 0) {
    HIP_OR_FAIL(c, prof_begin(c, kProfPass));
    LAUNCH_OR_FAIL(c, launch_split_rows(a, ad, nullptr, std::min(n_items, c->rows_blocks), c->stream));
    LAUNCH_OR_FAIL(c, launch_split_rows_slow(a, ad, nullptr, kSlowBlocks, c->stream));
    HIP_OR_FAIL(c, prof_end(c));
  }
  HIP_OR_FAIL(c, prof_begin(c, kProfSolve));
  LAUNCH_OR_FAIL(c, launch_split_solve(a, ad, nullptr, n_chunks2, c->stream));
  LAUNCH_OR_FAIL(c, launch_split_solve_fix(ad, nullptr, n_chunks2, c->stream, split_solve_lds(c->J, c->R)));
  HIP_OR_FAIL(c, prof_end(c));
  HIP_OR_FAIL(c, prof_begin(c, kProfReduce));
  LAUNCH_OR_FAIL(c, launch_split_fsum(a, ad, nullptr, n_chunks, c->stream));
  HIP_OR_FAIL(c, prof_end(c));
  LAUNCH_OR_FAIL(c, launch_reduce_groups(ad, nullptr, reduce_groups_blocks(c->J, c->R), c->stream));
  HIP_OR_FAIL(c, prof_begin(c, kProfCommit));
  LAUNCH_OR_FAIL(c, launch_finish_dev(a, ad, nullptr, 1, a.mode == 0 ? 0 : 2, c->stream));
  HIP_OR_FAIL(c, prof_end(c));
  return DASH_OK;
}

// Enqueue an evaluation sweep of the committed state (F, G with the committed
// W) and its fit, over K slices.
dash_status enqueue_eval(dash_ctx *c, int K) {
  int s;
  HIP_OR_FAIL(c, take_stage(c, &s));
  char *blk = c->hstage[s];
  StepHeader *h = stage_header(blk);
  const int ch = choose_chunk(c, K);
  const int nch = (K + ch - 1) / ch;
  int c3 = ch, c2 = ch;
  if (c->sched.variant == kPassSplit) split_chunks(c, K, &c3, &c2);
  std::memset(h, 0, sizeof *h);
  h->K = K;
  h->K_prev = K;
  h->n_groups = 0;
  h->n_chunks = nch;
  h->chunk = ch;
  h->chunks_per_rgroup = kChunksPerRGroup;
  h->n_rgroups = (nch + kChunksPerRGroup - 1) / kChunksPerRGroup;
  h->step = c->step;
  h->M = 0;
  h->report = nullptr;
  h->n_items = 0;
  h->chunk2 = c2;
  h->n_chunks2 = (K + c2 - 1) / c2;
  h->seq = ++c->seq;
  int32_t *gptr = (int32_t *)(blk + c->off_gptr);
  for (int i = 0; i <= nch; ++i) gptr[i] = 0;
  const size_t bytes = c->off_gptr + sizeof(int32_t) * (nch + 1);
  c->off_items = c->off_groups;
  const char *d = c->desc_fetch ? c->dstep[s] : c->hstage_dev[s];
  if (c->sched.variant == kPassSplit) write_pass_args(c, blk, d, 1);
  HIP_OR_FAIL(c, upload_stage(c, s, bytes, false, nullptr));
  PassArgs a = base_args(c, s);
  a.pass = 0;
  a.last_pass = 0;
  a.mode = 1;
  if (c->sched.variant == kPassSplit) {
    a.fuse = 0;
    if (dash_status st = enqueue_split_pass(c, a, args_dev(c, d, 0), 0, h->n_chunks2, nch)) return st;
  } else {
    LAUNCH_OR_FAIL(c, launch_pass(a, c->sched.variant, nch, c->stream));
    if (!a.fuse) LAUNCH_OR_FAIL(c, launch_finish(a, 2, c->stream));
  }
  HIP_OR_FAIL(c, stage_done(c, s));
  return DASH_OK;
}

dash_status enqueue_prep(dash_ctx *c) {
  PassArgs a = base_args(c, 0);   // reads no descriptor
  LAUNCH_OR_FAIL(c, launch_finish(a, 1, c->stream));
  return DASH_OK;
}

// Committed-buffer index 0 for everything; slices [0, K) last folded at update tl.
dash_status reset_device_state(dash_ctx *c, int32_t K, int32_t tl) {
  HIP_OR_FAIL(c, hipMemsetAsync(c->cur, 0, (size_t)(2 * c->K_cap), c->stream));
  if (c->Yc) {
    HIP_OR_FAIL(c, hipMemsetAsync(c->Yc, 0, sizeof(uint16_t) * 2 * c->K_cap * y_stride(c->J, c->R), c->stream));
    HIP_OR_FAIL(c, hipMemsetAsync(c->Dc, 0, sizeof(float) * 2 * c->K_cap * c->R * c->R, c->stream));
  }
  if (tl == 0) {
    HIP_OR_FAIL(c, hipMemsetAsync(c->tlast, 0, sizeof(int32_t) * std::max<int32_t>(K, 1), c->stream));
  } else {
    std::vector<int32_t> t(std::max<int32_t>(K, 1), tl);
    if (K > 0) HIP_OR_FAIL(c, hipMemcpy(c->tlast, t.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice));
  }
  Ctl ctl{};
  ctl.gcur = 0;
  ctl.ok = 1;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return DASH_OK;
}

dash_status validate_ptr(dash_ctx *c, const int64_t *ptr, int64_t n, bool nonempty) {
  if (!ptr) return fail(c, DASH_E_INVALID_ARG, "row_ptr is NULL");
  if (ptr[0] < 0) return fail(c, DASH_E_INVALID_ARG, "row_ptr[0] < 0");
  for (int64_t i = 0; i < n; ++i) {
    if (ptr[i + 1] < ptr[i]) return fail(c, DASH_E_INVALID_ARG, "row_ptr decreases at %lld", (long long)i);
    if (nonempty && ptr[i + 1] == ptr[i])
      return fail(c, DASH_E_INVALID_ARG, "group %lld has no rows", (long long)i);
  }
  return DASH_OK;
}

// Device bytes a context with this configuration allocates at creation.
int64_t context_footprint(const dash_config *cfg) {
  const int64_t R = cfg->R, Kc = cfg->max_slices;
  const int64_t YS = y_stride(cfg->J, cfg->R);
  const int64_t n_chunks_cap = std::min<int64_t>(Kc, kMaxChunks);
  const int64_t plen = partial_len(cfg->J, cfg->R);
  const int64_t G_cap = cfg->max_groups_per_update + Kc;
  auto al = [](int64_t b) { return (b < 256 ? 256 : b + 255) / 256 * 256; };
  const size_t off_gptr = align_up(align_up(sizeof(StepHeader), 64) + sizeof(PassArgs) * cfg->n_iter, 64);
  const int64_t step_bytes = (int64_t)align_up(
      align_up(align_up(off_gptr + sizeof(int32_t) * (n_chunks_cap + 1), 64) + sizeof(Group) * G_cap, 64) +
          sizeof(Item) * G_cap, 256);
  const int64_t carry = cfg->precision == DASH_PREC_MIXED ? al(2 * 2 * Kc * YS) + al(4 * 2 * Kc * R * R) : 0;
  const int64_t lag = cfg->stats_mode == DASH_STATS_LAGGED
                          ? al(8 * 2 * Kc * R) + al(8 * 2 * ((int64_t)cfg->J * R + R * R)) : 0;
  const int64_t split = al(8 * Kc * R) + al(8 * std::min<int64_t>(Kc, kMaxChunks2) * (R * R + 1)) +
                        al(4 * Kc) + al(16) + al(4 * Kc) + al(4 * std::min<int64_t>(Kc, kMaxChunks2));
  return carry + lag + split + al(4 * 2 * Kc * YS) + al(4 * 2 * Kc * R * R) + al(8 * 2 * Kc) + al(2 * Kc) + al(4 * 2 * Kc) +
         al(8 * 2 * Kc * R) + al(2 * (int64_t)vb_bytes(cfg->J, cfg->R)) + al(sizeof(Ctl)) +
         al(4 * cfg->max_rows_per_update * R) + al(8 * n_chunks_cap * plen) +
         al(8 * ((n_chunks_cap + kChunksPerRGroup - 1) / kChunksPerRGroup) * plen) +
         al(4 * (kMaxChunks + 1)) + al(8 * (Kc + 1)) + kStages * al(step_bytes);
}

// Device time of an update from its report's realtime stamps (microseconds).
double device_us(const Report &r) {
  return (r.t_end > r.t_start && r.t_start) ? (double)(r.t_end - r.t_start) / kRealtimeMHz : 0.0;
}

// The autotuner's cache: one JSON object per line,
//   {"key": "<shape>", "variant": v, "spread": s, "fuse": f, "solve_div": d, "ns_per_kb": x}
// keyed by the device architecture, J, R, precision, statistics mode, passes,
// the mean rows per touched slice (log2 bucket) and the slice count (log2
// bucket) of the update the tuning started on.
std::string tune_key_of(const dash_ctx *c) {
  int touched = 0;
  int last = -1;
  std::vector<int> ids;
  ids.reserve(c->pending.size());
  for (const PendingGroup &g : c->pending) ids.push_back(g.slice);
  std::sort(ids.begin(), ids.end());
  for (int id : ids)
    if (id != last) {
      ++touched;
      last = id;
    }
  const double mean = touched ? (double)c->rows_pending / touched : 0.0;
  const int mb = (int)std::floor(std::log2(1.0 + mean));
  const int kb = (int)std::floor(std::log2(1.0 + (double)c->K_pending));
  char buf[160];
  std::snprintf(buf, sizeof buf, "gfx950/J%d/R%d/p%d/s%d/i%d/m%d/k%d", c->J, c->R, (int)c->cfg.precision,
                (int)c->cfg.stats_mode, (int)c->cfg.n_iter, mb, kb);
  return buf;
}

bool tune_cache_lookup(const dash_ctx *c, const std::string &key, Schedule *out) {
  FILE *fp = std::fopen(c->tune_cache.c_str(), "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, fp)) {
    char k[200];
    Schedule s{};
    double x = 0.0;
    if (std::sscanf(line, "{\"key\": \"%199[^\"]\", \"variant\": %d, \"spread\": %d, \"fuse\": %d, \"solve_div\": %d, \"ns_per_kb\": %lf}",
                    k, &s.variant, &s.spread, &s.fuse, &s.solve_div, &x) == 6 &&
        key == k && (s.variant == kPassWave || s.variant == kPassSplit) && s.spread >= 1 && s.solve_div >= 1) {
      *out = s;   // the last entry of a key wins
      found = true;
    }
  }
  std::fclose(fp);
  // a cached wave schedule only where the wave sweep applies to this context
  if (found && out->variant == kPassWave && c->variant != kPassWave) return false;
  if (found && out->fuse && fused_pass_lds(out->variant, c->J, c->R) == 0) out->fuse = 0;
  return found;
}

void tune_cache_store(const dash_ctx *c, const std::string &key, const Schedule &s, double ns_per_kb) {
  std::vector<std::string> keep;
  if (FILE *fp = std::fopen(c->tune_cache.c_str(), "r")) {
    char line[512];
    const std::string tag = "{\"key\": \"" + key + "\"";
    while (std::fgets(line, sizeof line, fp))
      if (std::strncmp(line, tag.c_str(), tag.size()) != 0) keep.push_back(line);
    std::fclose(fp);
  }
  const std::string tmp = c->tune_cache + ".tmp";
  FILE *fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return;
  for (const std::string &l : keep) std::fputs(l.c_str(), fp);
  std::fprintf(fp, "{\"key\": \"%s\", \"variant\": %d, \"spread\": %d, \"fuse\": %d, \"solve_div\": %d, \"ns_per_kb\": %.4f}\n",
               key.c_str(), s.variant, s.spread, s.fuse, s.solve_div, ns_per_kb);
  std::fclose(fp);
  std::rename(tmp.c_str(), c->tune_cache.c_str());
}

// Fold one reaped update into the autotuner's scores; once every candidate has
// run tune_per times, keep the one with the least device time per byte.
void tune_account(dash_ctx *c, const InFlight &f, const Report &r) {
  if (f.cand < 0 || c->tuned || f.cand >= (int)c->tune_cands.size()) return;
  const double us = device_us(r);
  if (us <= 0.0) return;
  c->tune_us[f.cand] += us;
  c->tune_bytes[f.cand] += f.bytes;
  c->tune_n[f.cand] += 1;
  for (int n : c->tune_n)
    if (n < c->tune_per) return;
  int best = 0;
  for (int i = 1; i < (int)c->tune_cands.size(); ++i)
    if (c->tune_us[i] / c->tune_bytes[i] < c->tune_us[best] / c->tune_bytes[best]) best = i;
  c->sched = c->tune_cands[best];
  c->tuned = true;
  if (!c->tune_cache.empty() && !c->tune_key.empty())
    tune_cache_store(c, c->tune_key, c->sched, 1e3 * c->tune_us[best] / (c->tune_bytes[best] / 1024.0));
}

void graph_reset(dash_ctx *c) {
  c->gsched = Schedule{-1, 0, 0};
  for (int s = 0; s < kStages; ++s) {
    if (c->gexec[s]) (void)hipGraphExecDestroy(c->gexec[s]);
    if (c->graph[s]) (void)hipGraphDestroy(c->graph[s]);
    c->gexec[s] = nullptr;
    c->graph[s] = nullptr;
    c->gnodes[s].clear();
    c->gparams[s].clear();
  }
}

// Enqueue the launches of one update (stage s, descriptor bytes, nch chunks)
// as a graph.  The first call captures the update's launches -- fetch, then per
// pass the fused sweep [and final phase], or the split sweep's row, solve, F
// and final-phase launches -- and instantiates them; later calls rewrite every
// kernel node's grid and arguments for this update and relaunch the same
// executable graph.
dash_status graph_update(dash_ctx *c, int s, size_t bytes, int nch, void *report, int n_items, int n_chunks2) {
  const int n_iter = c->cfg.n_iter;
  const bool split = c->sched.variant == kPassSplit;
  PassArgs base = base_args(c, s);
  base.mode = 0;
  if (split) base.fuse = 0;
  std::vector<PassArgs> args(n_iter, base);
  for (int p = 0; p < n_iter; ++p) {
    args[p].pass = p;
    args[p].last_pass = (p == n_iter - 1) ? 1 : 0;
  }
  FetchArgs fa = fetch_args(c->hstage_dev[s], c->dstep[s], bytes, report);
  const size_t per_pass = split ? 7 : (base.fuse ? 1 : 2);
  const size_t expect = 1 + (size_t)n_iter * per_pass;
  if (!c->gexec[s]) {
    HIP_OR_FAIL(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int e = launch_fetch(c->hstage_dev[s], c->dstep[s], bytes, report, c->stream);
    for (int p = 0; p < n_iter && !e; ++p) {
      if (split) {
        const PassArgs *ad = args_dev(c, c->dstep[s], p);
        e = launch_split_rows(args[p], ad, nullptr, std::min(n_items, c->rows_blocks), c->stream);
        if (!e) e = launch_split_rows_slow(args[p], ad, nullptr, kSlowBlocks, c->stream);
        if (!e) e = launch_split_solve(args[p], ad, nullptr, n_chunks2, c->stream);
        if (!e) e = launch_split_solve_fix(ad, nullptr, n_chunks2, c->stream, split_solve_lds(c->J, c->R));
        if (!e) e = launch_split_fsum(args[p], ad, nullptr, nch, c->stream);
        if (!e) e = launch_reduce_groups(ad, nullptr, reduce_groups_blocks(c->J, c->R), c->stream);
        if (!e) e = launch_finish_dev(args[p], ad, nullptr, 1, 0, c->stream);
      } else {
        e = launch_pass(args[p], c->sched.variant, nch, c->stream);
        if (!e && !base.fuse) e = launch_finish(args[p], 0, c->stream);
      }
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->stream, &g);
    if (e || ee != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, DASH_E_DEVICE, "graph capture failed (%d, %s)", e, hipGetErrorString(ee));
    }
    c->graph[s] = g;
    size_t count = 0;
    HIP_OR_FAIL(c, hipGraphGetNodes(g, nullptr, &count));
    std::vector<hipGraphNode_t> nodes(count);
    HIP_OR_FAIL(c, hipGraphGetNodes(g, nodes.data(), &count));
    // the captured nodes form one chain: order them from the root
    std::vector<hipGraphNode_t> chain;
    hipGraphNode_t cur = nullptr;
    for (auto nd : nodes) {
      size_t ndep = 0;
      HIP_OR_FAIL(c, hipGraphNodeGetDependencies(nd, nullptr, &ndep));
      if (ndep == 0) cur = nd;
    }
    while (cur) {
      chain.push_back(cur);
      size_t nd = 0;
      HIP_OR_FAIL(c, hipGraphNodeGetDependentNodes(cur, nullptr, &nd));
      if (nd != 1) break;
      hipGraphNode_t nx = nullptr;
      HIP_OR_FAIL(c, hipGraphNodeGetDependentNodes(cur, &nx, &nd));
      cur = nx;
    }
    if (chain.size() != expect || count != expect) {
      (void)hipGraphDestroy(g);
      c->graph[s] = nullptr;
      return fail(c, DASH_E_DEVICE, "captured graph has %zu nodes, expected %zu", count, expect);
    }
    c->gnodes[s] = chain;
    c->gparams[s].resize(chain.size());
    for (size_t i = 0; i < chain.size(); ++i)
      HIP_OR_FAIL(c, hipGraphKernelNodeGetParams(chain[i], &c->gparams[s][i]));
    HIP_OR_FAIL(c, hipGraphInstantiate(&c->gexec[s], g, nullptr, nullptr, 0));
  } else {
    if (c->gnodes[s].size() != expect) return fail(c, DASH_E_DEVICE, "graph does not match the schedule");
    auto set = [&](size_t i, unsigned grid, void **params) -> hipError_t {
      hipKernelNodeParams kp = c->gparams[s][i];
      kp.gridDim = dim3(grid);
      kp.kernelParams = params;
      return hipGraphExecKernelNodeSetParams(c->gexec[s], c->gnodes[s][i], &kp);
    };
    size_t i = 0;
    void *fargs[] = {&fa.src, &fa.dst, &fa.n16, &fa.src_tail, &fa.dst_tail, &fa.tail, &fa.report};
    HIP_OR_FAIL(c, set(i++, fa.grid, fargs));
    int mode0 = 0;
    const BlockMap *nomap = nullptr;
    for (int p = 0; p < n_iter; ++p) {
      void *pargs[] = {&args[p]};
      void *fin[] = {&args[p], &mode0};
      if (split) {
        // the split kernels read their arguments from the stage's fixed
        // descriptor slot: only the grids change
        const PassArgs *ad = args_dev(c, c->dstep[s], p);
        void *dargs[] = {&ad, &nomap};
        void *dfin[] = {&ad, &nomap, &mode0};
        HIP_OR_FAIL(c, set(i++, (unsigned)std::min(n_items, c->rows_blocks), dargs));
        HIP_OR_FAIL(c, set(i++, (unsigned)kSlowBlocks, dargs));
        HIP_OR_FAIL(c, set(i++, (unsigned)n_chunks2, dargs));
        HIP_OR_FAIL(c, set(i++, (unsigned)n_chunks2, dargs));
        HIP_OR_FAIL(c, set(i++, (unsigned)nch, dargs));
        HIP_OR_FAIL(c, set(i++, (unsigned)reduce_groups_blocks(c->J, c->R), dargs));
        HIP_OR_FAIL(c, set(i++, 1u, dfin));
      } else {
        HIP_OR_FAIL(c, set(i++, (unsigned)nch, pargs));
        if (!base.fuse) HIP_OR_FAIL(c, set(i++, 1u, fin));
      }
    }
  }
  HIP_OR_FAIL(c, hipGraphLaunch(c->gexec[s], c->stream));
  // the pinned block and this stage's graph are free again once the whole update ran
  HIP_OR_FAIL(c, hipEventRecord(c->stage_ev[s], c->stream));
  c->stage_used[s] = true;
  return DASH_OK;
}

dash_status read_ctl(dash_ctx *c, Ctl *out) {
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  HIP_OR_FAIL(c, hipMemcpy(out, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  return DASH_OK;
}

}  // namespace dash

extern "C" {

void dash_config_default(dash_config *cfg, int32_t J, int32_t R) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->J = J;
  cfg->R = R;
  cfg->lambda = 0.7;
  cfg->n_iter = 1;
  cfg->init_max_iter = 10;
  cfg->init_tol = 1e-10;
  cfg->precision = DASH_PREC_FP32;
  cfg->stats_mode = DASH_STATS_EXACT;
  cfg->max_slices = 65536;
  cfg->max_rows_per_update = 1 << 20;
  cfg->max_groups_per_update = 65536;
  cfg->max_init_rows = 4 << 20;
  cfg->device = 0;
  cfg->stream = nullptr;
}

dash_status dash_profile(dash_ctx *c, int32_t enable) {
  if (!c) return DASH_E_INVALID_ARG;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (enable && c->ev.empty()) {
    c->ev.resize(2 * kProfPairs, nullptr);
    c->ev_kind.resize(kProfPairs, 0);
    // timing-only events: no system-scope fence, so they do not write back and
    // invalidate the caches around the launches they bracket
    for (auto &e : c->ev) HIP_OR_FAIL(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  if (c->ev_used) HIP_OR_FAIL(c, prof_fold(c));
  c->ev_used = 0;
  c->prof = dash_profile_stats{};
  c->prof_every = enable > 0 ? enable : 0;
  c->profiling = false;
  return DASH_OK;
}

dash_status dash_profile_read(dash_ctx *c, dash_profile_stats *out) {
  if (!c || !out) return DASH_E_INVALID_ARG;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  HIP_OR_FAIL(c, prof_fold(c));
  *out = c->prof;
  return DASH_OK;
}

const char *dash_status_string(dash_status s) {
  switch (s) {
    case DASH_OK: return "ok";
    case DASH_E_INVALID_ARG: return "invalid argument";
    case DASH_E_OUT_OF_MEMORY: return "out of memory";
    case DASH_E_BAD_STATE: return "bad state";
    case DASH_E_CAPACITY: return "capacity exceeded";
    case DASH_E_NUMERIC: return "non-finite factors (update rolled back)";
    case DASH_E_DEVICE: return "HIP runtime error";
    case DASH_E_IO: return "checkpoint I/O error";
  }
  return "unknown status";
}

const char *dash_last_error(const dash_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"

namespace dash {

dash_status create_context(const dash_config *cfg, hipStream_t stream, bool served, dash_ctx **out) {
  if (!cfg || !out) return DASH_E_INVALID_ARG;
  *out = nullptr;
  if (cfg->J < 1 || cfg->J > kMaxJ || cfg->R < 1 || cfg->R > kMaxR) return DASH_E_INVALID_ARG;
  if (!(cfg->lambda > 0.0 && cfg->lambda <= 1.0) || cfg->n_iter < 1 || cfg->init_max_iter < 0)
    return DASH_E_INVALID_ARG;
  if (cfg->max_slices < 1 || cfg->max_slices > (int64_t)1 << 30 || cfg->max_rows_per_update < 1 ||
      cfg->max_groups_per_update < 1 || cfg->max_init_rows < 0)
    return DASH_E_INVALID_ARG;
  if ((cfg->precision != DASH_PREC_FP32 && cfg->precision != DASH_PREC_MIXED) ||
      (cfg->stats_mode != DASH_STATS_EXACT && cfg->stats_mode != DASH_STATS_LAGGED))
    return DASH_E_INVALID_ARG;
  dash_ctx *c = new (std::nothrow) dash_ctx();
  if (!c) return DASH_E_OUT_OF_MEMORY;
  c->cfg = *cfg;
  c->J = cfg->J;
  c->R = cfg->R;
  c->K_cap = cfg->max_slices;
  c->M_cap = cfg->max_rows_per_update;
  c->G_cap = cfg->max_groups_per_update + c->K_cap;  // new slices are groups too
  c->N_init_cap = cfg->max_init_rows;
  c->served = served;
  c->variant = pass_variant(cfg->J, cfg->R, cfg->precision, cfg->stats_mode == DASH_STATS_LAGGED);
  if (const char *e = std::getenv("DASH_VARIANT")) {
    if (std::atoi(e) == kPassSplit) c->variant = kPassSplit;
    else if (std::atoi(e) == kPassWave && c->variant == kPassWave) c->variant_forced = true;
  }
  if (served) c->variant = kPassSplit;   // the batched launches of a server tick run the split sweep
  c->fused_lds = served ? 0 : (int)fused_pass_lds(c->variant, cfg->J, cfg->R);
  if (const char *e = std::getenv("DASH_FUSE"))
    if (std::atoi(e) == 0) c->fused_lds = 0;
  c->sched = Schedule{c->variant, 1, c->fused_lds > 0 ? 1 : 0};
  if (!served) {
    if (const char *e = std::getenv("DASH_DESC_FETCH")) c->desc_fetch = std::atoi(e) != 0;
    if (const char *e = std::getenv("DASH_CHUNK")) c->chunk_override = std::atoi(e);
  }
  auto bail = [&](dash_status s) {
    dash_destroy(c);
    return s;
  };
  if (hipSetDevice(cfg->device) != hipSuccess) return bail(DASH_E_DEVICE);
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess)
    return bail(DASH_E_DEVICE);
  // a served stream plans its chunks for a fixed share of the device, so that
  // its reductions have the same order whatever else the server runs
  if (served) c->n_cu = std::min(c->n_cu, kServeCUs);
  // persistent row-stage workgroups: as many as can be resident
  c->rows_blocks = std::max(1, c->n_cu) *
                   std::max(1, split_rows_blocks_per_cu(cfg->J, cfg->R, cfg->precision == DASH_PREC_MIXED));
  if (stream) {
    c->stream = stream;
  } else {
    // a blocking stream: ordered after the work of the null stream, on which
    // callers that name no stream produce the rows they ingest
    if (hipStreamCreate(&c->stream) != hipSuccess) return bail(DASH_E_DEVICE);
    c->own_stream = true;
  }
  const int64_t J = c->J, R = c->R, Kc = c->K_cap;
  const int64_t n_chunks_cap = std::min<int64_t>(Kc, kMaxChunks);
  const int64_t plen = partial_len(c->J, c->R);
  c->vb_stride = vb_bytes(c->J, c->R);
  const int64_t YS = y_stride(c->J, c->R);
  bool ok = dalloc(&c->Y, sizeof(float) * 2 * Kc * YS) == hipSuccess &&
            dalloc(&c->D, sizeof(float) * 2 * Kc * R * R) == hipSuccess &&
            dalloc(&c->n, sizeof(double) * 2 * Kc) == hipSuccess &&
            dalloc(&c->cur, (size_t)(2 * Kc)) == hipSuccess &&
            dalloc(&c->tlast, sizeof(int32_t) * 2 * Kc) == hipSuccess &&
            dalloc(&c->W, sizeof(double) * 2 * Kc * R) == hipSuccess &&
            dalloc(&c->vb, (size_t)(2 * c->vb_stride)) == hipSuccess &&
            dalloc(&c->ctl, sizeof(Ctl)) == hipSuccess &&
            dalloc(&c->U_out, sizeof(float) * c->M_cap * R) == hipSuccess &&
            dalloc(&c->partials, sizeof(double) * n_chunks_cap * plen) == hipSuccess &&
            dalloc(&c->gpart, sizeof(double) * ((n_chunks_cap + kChunksPerRGroup - 1) / kChunksPerRGroup) * plen) == hipSuccess &&
            dalloc(&c->counters, sizeof(int32_t) * (kMaxChunks + 1)) == hipSuccess &&
            dalloc(&c->d_rowptr, sizeof(int64_t) * (Kc + 1)) == hipSuccess &&
            dalloc(&c->cbuf, sizeof(double) * Kc * R) == hipSuccess &&
            dalloc(&c->part2, sizeof(double) * std::min<int64_t>(Kc, kMaxChunks2) * (R * R + 1)) == hipSuccess &&
            dalloc(&c->tag, sizeof(int32_t) * Kc) == hipSuccess &&
            dalloc(&c->queue, sizeof(int32_t) * 4) == hipSuccess &&
            dalloc(&c->slow_list, sizeof(int32_t) * Kc) == hipSuccess &&
            dalloc(&c->solve_defer, sizeof(int32_t) * std::min<int64_t>(Kc, kMaxChunks2)) == hipSuccess;
  if (ok && cfg->stats_mode == DASH_STATS_LAGGED)
    ok = dalloc(&c->cst, sizeof(double) * 2 * Kc * R) == hipSuccess &&
         dalloc(&c->FG, sizeof(double) * 2 * (J * R + R * R)) == hipSuccess;
  if (ok && cfg->precision == DASH_PREC_MIXED)
    ok = dalloc(&c->Yc, sizeof(uint16_t) * 2 * Kc * YS) == hipSuccess &&
         dalloc(&c->Dc, sizeof(float) * 2 * Kc * R * R) == hipSuccess;
  if (!ok) return bail(DASH_E_OUT_OF_MEMORY);
  c->off_args = align_up(sizeof(StepHeader), 64);
  c->off_gptr = align_up(c->off_args + sizeof(PassArgs) * cfg->n_iter, 64);
  c->off_groups = align_up(c->off_gptr + sizeof(int32_t) * (n_chunks_cap + 1), 64);
  c->off_items = c->off_groups;
  c->step_bytes = align_up(align_up(c->off_groups + sizeof(Group) * c->G_cap, 64) + sizeof(Item) * c->G_cap, 256);
  for (int s = 0; s < kStages; ++s) {
    if (dalloc(&c->dstep[s], c->step_bytes) != hipSuccess) return bail(DASH_E_OUT_OF_MEMORY);
    if (hipHostMalloc((void **)&c->hstage[s], c->step_bytes, hipHostMallocMapped) != hipSuccess)
      return bail(DASH_E_OUT_OF_MEMORY);
    if (hipHostGetDevicePointer((void **)&c->hstage_dev[s], c->hstage[s], 0) != hipSuccess)
      return bail(DASH_E_DEVICE);
    if (hipEventCreateWithFlags(&c->stage_ev[s], hipEventDisableTiming) != hipSuccess)
      return bail(DASH_E_DEVICE);
  }
  if (hipHostMalloc((void **)&c->hreport, sizeof(Report) * kReportRing, hipHostMallocMapped) != hipSuccess)
    return bail(DASH_E_OUT_OF_MEMORY);

  std::memset(c->hreport, 0, sizeof(Report) * kReportRing);
  if (hipHostGetDevicePointer((void **)&c->dreport, c->hreport, 0) != hipSuccess) return bail(DASH_E_DEVICE);
  if (hipMemsetAsync(c->Y, 0, sizeof(float) * 2 * Kc * YS, c->stream) != hipSuccess ||
      hipMemsetAsync(c->cur, 0, (size_t)(2 * Kc), c->stream) != hipSuccess ||
      (c->Yc && hipMemsetAsync(c->Yc, 0, sizeof(uint16_t) * 2 * Kc * YS, c->stream) != hipSuccess) ||
      (c->Dc && hipMemsetAsync(c->Dc, 0, sizeof(float) * 2 * Kc * R * R, c->stream) != hipSuccess) ||
      hipMemsetAsync(c->tlast, 0, sizeof(int32_t) * 2 * Kc, c->stream) != hipSuccess ||
      hipMemsetAsync(c->counters, 0, sizeof(int32_t) * (kMaxChunks + 1), c->stream) != hipSuccess ||
      hipMemsetAsync(c->tag, 0, sizeof(int32_t) * Kc, c->stream) != hipSuccess ||
      hipMemsetAsync(c->queue, 0, sizeof(int32_t) * 4, c->stream) != hipSuccess ||
      (c->cst && hipMemsetAsync(c->cst, 0, sizeof(double) * 2 * Kc * R, c->stream) != hipSuccess) ||
      (c->FG && hipMemsetAsync(c->FG, 0, sizeof(double) * 2 * (J * R + R * R), c->stream) != hipSuccess) ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(DASH_E_DEVICE);
  {
    Ctl ctl{};
    ctl.ok = 1;
    if (hipMemcpy(c->ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice) != hipSuccess) return bail(DASH_E_DEVICE);
  }
  c->pending.reserve(1024);
  *out = c;
  return DASH_OK;
}

}  // namespace dash

extern "C" {

dash_status dash_create(const dash_config *cfg, dash_ctx **out) {
  if (!cfg || !out) return DASH_E_INVALID_ARG;
  return create_context(cfg, (hipStream_t)cfg->stream, false, out);
}

dash_status dash_destroy(dash_ctx *c) {
  if (!c) return DASH_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->Y);
  (void)hipFree(c->D);
  (void)hipFree(c->Yc);
  (void)hipFree(c->Dc);
  (void)hipFree(c->n);
  (void)hipFree(c->cur);
  (void)hipFree(c->tlast);
  (void)hipFree(c->W);
  (void)hipFree(c->vb);
  (void)hipFree(c->ctl);
  (void)hipFree(c->U_out);
  (void)hipFree(c->partials);
  (void)hipFree(c->gpart);
  (void)hipFree(c->counters);
  (void)hipFree(c->d_rowptr);
  (void)hipFree(c->cbuf);
  (void)hipFree(c->part2);
  (void)hipFree(c->tag);
  (void)hipFree(c->queue);
  (void)hipFree(c->slow_list);
  (void)hipFree(c->solve_defer);
  (void)hipFree(c->cst);
  (void)hipFree(c->FG);
  (void)hipFree(c->anom.se);
  (void)hipFree(c->anom.flag);
  (void)hipFree(c->anom.sid);
  (void)hipFree(c->anom.hist);
  (void)hipFree(c->anom.hcnt);
  (void)hipFree(c->anom.ticket);
  for (int s = 0; s < kStages; ++s) {
    (void)hipFree(c->dstep[s]);
    if (c->hstage[s]) (void)hipHostFree(c->hstage[s]);
    if (c->stage_ev[s]) (void)hipEventDestroy(c->stage_ev[s]);
  }
  if (c->hreport) (void)hipHostFree(c->hreport);
  graph_reset(c);
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return DASH_OK;
}

dash_status dash_get_dims(const dash_ctx *c, dash_dims *d) {
  if (!c || !d) return DASH_E_INVALID_ARG;
  d->J = c->J;
  d->R = c->R;
  d->K = c->K;
  d->K_pending = c->K_pending;
  d->step = c->step;
  d->m_last = c->m_last;
  d->rows_pending = c->rows_pending;
  d->initialized = c->initialized ? 1 : 0;
  return DASH_OK;
}

dash_status dash_init_from_factors(dash_ctx *c, int32_t K, const int64_t *row_ptr, const float *X,
                                   const float *U, const float *W, const float *V) {
  if (!c) return DASH_E_INVALID_ARG;
  if (c->initialized) return fail(c, DASH_E_BAD_STATE, "context already initialised");
  if (K < 1) return fail(c, DASH_E_INVALID_ARG, "K must be >= 1");
  if (K > c->K_cap) return fail(c, DASH_E_CAPACITY, "K=%d exceeds max_slices", K);
  if (!X || !U || !W || !V) return fail(c, DASH_E_INVALID_ARG, "NULL factor or data pointer");
  std::vector<int64_t> rp_host;
  if (dash_status s = dash::host_row_ptr(c, row_ptr, K, rp_host)) return s;
  if (dash_status s = validate_ptr(c, row_ptr, K, true)) return s;
  if (row_ptr[0] != 0) return fail(c, DASH_E_INVALID_ARG, "row_ptr[0] must be 0");
  if (dash_status s = reset_device_state(c, K, 0)) return s;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_rowptr, row_ptr, sizeof(int64_t) * (K + 1),
                                hipMemcpyHostToDevice, c->stream));
  LAUNCH_OR_FAIL(c, launch_accum_given_u(c->J, c->R, K, c->d_rowptr, X, U, c->Y, c->D, c->n, c->stream));
  LAUNCH_OR_FAIL(c, launch_w_from_f32(c->R, K, W, c->W, c->stream));
  LAUNCH_OR_FAIL(c, launch_v_from_f32(c->J, c->R, V, c->vb, c->stream));
  if (dash_status s = enqueue_prep(c)) return s;
  c->step = 0;
  if (dash_status s = enqueue_eval(c, K)) return s;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->initialized = true;
  c->K = c->K_enq = c->K_pending = K;
  c->step = c->step_enq = 0;
  c->m_last = 0;
  c->pending.clear();
  c->rows_pending = 0;
  return DASH_OK;
}

}  // extern "C"

namespace dash {

// Whether p points to device memory.  Host memory the runtime does not know
// may fail the query; that error is cleared here so that no later call
// reports it.
bool on_device(const void *p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

// The initial decomposition's row_ptr as host memory (the host plans the
// passes from it): a device array of K + 1 entries is copied into tmp once the
// context's stream is idle, and p then points there.
dash_status host_row_ptr(dash_ctx *c, const int64_t *&p, int32_t K, std::vector<int64_t> &tmp) {
  if (!p || K < 1 || !on_device(p)) return DASH_OK;
  tmp.resize((size_t)K + 1);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  HIP_OR_FAIL(c, hipMemcpy(tmp.data(), p, sizeof(int64_t) * ((size_t)K + 1), hipMemcpyDeviceToHost));
  p = tmp.data();
  return DASH_OK;
}

dash_status init_check(dash_ctx *c, int32_t K, const int64_t *row_ptr, const float *X) {
  if (!c) return DASH_E_INVALID_ARG;
  if (c->initialized) return fail(c, DASH_E_BAD_STATE, "context already initialised");
  if (K < 1) return fail(c, DASH_E_INVALID_ARG, "K must be >= 1");
  if (K > c->K_cap) return fail(c, DASH_E_CAPACITY, "K=%d exceeds max_slices", K);
  if (!X) return fail(c, DASH_E_INVALID_ARG, "X is NULL");
  if (dash_status s = validate_ptr(c, row_ptr, K, true)) return s;
  if (row_ptr[0] != 0) return fail(c, DASH_E_INVALID_ARG, "row_ptr[0] must be 0");
  if (row_ptr[K] > c->N_init_cap)
    return fail(c, DASH_E_CAPACITY, "%lld initial rows exceed max_init_rows", (long long)row_ptr[K]);
  return DASH_OK;
}

size_t init_workspace_doubles(const dash_ctx *c, int32_t K, bool has_v0) {
  const int J = c->J, R = c->R, RR = R * R;
  const int chunk = std::max(1, (K + 1023) / 1024);
  const int n_chunks = (K + chunk - 1) / chunk;
  const int plen = std::max(2 * RR, J * R) + 2;
  const int n_gc = init_gram_chunks(J);
  return (size_t)2 * J * J + J + (size_t)(has_v0 ? 0 : n_gc) * J * J + 4 * (size_t)RR + (size_t)n_chunks * plen +
         2 + (size_t)K * RR;
}

dash_status init_with_workspace(dash_ctx *c, int32_t K, const int64_t *row_ptr, const float *X, const float *V0,
                                dash_init_report *report, double *ws) {
  const int64_t N = row_ptr[K];
  if (dash_status s = reset_device_state(c, K, 0)) return s;
  HIP_OR_FAIL(c, hipMemcpyAsync(c->d_rowptr, row_ptr, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice,
                                c->stream));
  const int J = c->J, R = c->R, RR = R * R;
  const int chunk = std::max(1, (K + 1023) / 1024);
  const int n_chunks = (K + chunk - 1) / chunk;
  const int plen = std::max(2 * RR, J * R) + 2;
  const int n_gc = init_gram_chunks(J);
  double *Gm = ws, *Z = Gm + (size_t)J * J, *evals = Z + (size_t)J * J;
  double *gpart = evals + J;
  double *small = gpart + (size_t)(V0 ? 0 : n_gc) * J * J;
  InitArgs a{};
  a.J = J;
  a.R = R;
  a.K = K;
  a.ys = y_stride(J, R);
  a.K_cap = c->K_cap;
  a.row_ptr = c->d_rowptr;
  a.X = X;
  a.Y = c->Y;
  a.D = c->D;
  a.n = c->n;
  a.W = c->W;
  a.V64 = vb_view(c->vb, J, R).V64;   // the committed bundle (generation 0)
  a.H = small;
  a.WtW = small + RR;
  a.VtV = small + 2 * RR;
  a.Mwinv = small + 3 * RR;
  a.part = small + 4 * RR;
  a.plen = plen;
  a.chunk = chunk;
  a.n_chunks = n_chunks;
  a.result = a.part + (size_t)n_chunks * plen;
  a.Dh = a.result + 2;
  if (V0) {
    LAUNCH_OR_FAIL(c, launch_v_from_f32(J, R, V0, c->vb, c->stream));
  } else {
    LAUNCH_OR_FAIL(c, launch_init_gram(J, N, n_gc, X, gpart, Gm, c->stream));
    LAUNCH_OR_FAIL(c, launch_sym_eig(J, Gm, Z, evals, c->stream));
    LAUNCH_OR_FAIL(c, launch_top_vectors(J, R, evals, Z, a.V64, c->stream));
  }
  LAUNCH_OR_FAIL(c, launch_init_start(a, c->stream));
  const int max_iter = std::max(1, c->cfg.init_max_iter);
  double prev = 0.0, loss = 0.0, sum_n = 0.0;
  int iters = 0;
  for (int it = 1; it <= max_iter; ++it) {
    LAUNCH_OR_FAIL(c, launch_init_iteration(a, c->stream));
    double res[2];
    HIP_OR_FAIL(c, hipMemcpyAsync(res, a.result, sizeof res, hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    iters = it;
    loss = res[0];
    sum_n = res[1];
    if (!std::isfinite(loss)) return fail(c, DASH_E_NUMERIC, "non-finite loss in initial iteration %d", it);
    if (it > 1 && std::fabs(prev - loss) <= c->cfg.init_tol * std::fabs(loss)) break;
    prev = loss;
  }
  LAUNCH_OR_FAIL(c, launch_init_handoff(a, c->stream));
  if (dash_status s = enqueue_prep(c)) return s;
  c->step = 0;
  if (dash_status s = enqueue_eval(c, K)) return s;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->initialized = true;
  c->K = c->K_enq = c->K_pending = K;
  c->step = c->step_enq = 0;
  c->m_last = 0;
  c->pending.clear();
  c->rows_pending = 0;
  if (report) {
    report->iters = iters;
    report->loss = loss;
    report->fit = sum_n > 0.0 ? 1.0 - std::sqrt(std::max(0.0, loss)) / std::sqrt(sum_n) : 1.0;
  }
  return DASH_OK;
}

}  // namespace dash

extern "C" {

dash_status dash_init(dash_ctx *c, int32_t K, const int64_t *row_ptr, const float *X, const float *V0,
                      dash_init_report *report) {
  if (!c) return DASH_E_INVALID_ARG;
  std::vector<int64_t> rp_host;
  if (!c->initialized && K >= 1 && K <= c->K_cap)
    if (dash_status s = host_row_ptr(c, row_ptr, K, rp_host)) return s;
  if (dash_status s = init_check(c, K, row_ptr, X)) return s;
  // the initialisation's scratch lives for this call only
  const size_t ws_doubles = init_workspace_doubles(c, K, V0 != nullptr);
  double *ws = nullptr;
  if (c->fail_next == DASH_SITE_INIT_ALLOC) {
    c->fail_next = 0;
    return fail(c, DASH_E_OUT_OF_MEMORY, "initialisation scratch (%zu doubles): injected failure", ws_doubles);
  }
  if (hipMalloc((void **)&ws, ws_doubles * sizeof(double)) != hipSuccess)
    return fail(c, DASH_E_OUT_OF_MEMORY, "initialisation scratch (%zu doubles)", ws_doubles);
  const dash_status s = init_with_workspace(c, K, row_ptr, X, V0, report, ws);
  if (s == DASH_OK) {
    (void)hipFree(ws);
  } else {
    // kernels may still read it: free once the stream is idle
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(ws);
  }
  return s;
}

dash_status dash_ingest_rows(dash_ctx *c, int32_t n, const int32_t *slice_id, const int64_t *row_ptr,
                             const float *rows) {
  if (!c) return DASH_E_INVALID_ARG;
  if (c->served && !c->server_ingest)
    return fail(c, DASH_E_BAD_STATE, "a served stream takes rows through dash_server_submit");
  if (!c->initialized) return fail(c, DASH_E_BAD_STATE, "context not initialised");
  if (n < 0) return fail(c, DASH_E_INVALID_ARG, "n < 0");
  if (n == 0) return DASH_OK;
  if (c->fail_next == DASH_SITE_INGEST) {
    c->fail_next = 0;
    return fail(c, DASH_E_CAPACITY, "dash_ingest_rows: injected failure, nothing staged");
  }
  if (!slice_id) return fail(c, DASH_E_INVALID_ARG, "slice_id is NULL");
  if (dash_status s = validate_ptr(c, row_ptr, n, false)) return s;
  const int64_t add = row_ptr[n] - row_ptr[0];
  if (add > 0 && !rows) return fail(c, DASH_E_INVALID_ARG, "rows is NULL");
  int64_t ng = 0;
  for (int32_t g = 0; g < n; ++g) {
    if (slice_id[g] < 0 || slice_id[g] >= c->K_pending)
      return fail(c, DASH_E_INVALID_ARG, "slice_id[%d]=%d out of range [0,%d)", g, slice_id[g], c->K_pending);
    if (row_ptr[g + 1] > row_ptr[g]) ++ng;
  }
  if (c->rows_pending + add > c->M_cap)
    return fail(c, DASH_E_CAPACITY, "rows per update would exceed %lld", (long long)c->M_cap);
  if ((int64_t)c->pending.size() + ng > c->G_cap)
    return fail(c, DASH_E_CAPACITY, "row groups per update would exceed %lld", (long long)c->G_cap);
  for (int32_t g = 0; g < n; ++g) {
    const int64_t m = row_ptr[g + 1] - row_ptr[g];
    if (m == 0) continue;
    c->pending.push_back({slice_id[g], rows + row_ptr[g] * c->J, m, c->rows_pending});
    c->rows_pending += m;
  }
  return DASH_OK;
}

dash_status dash_ingest_slices(dash_ctx *c, int32_t L, const int64_t *row_ptr, const float *rows,
                               int32_t *first_id) {
  if (!c) return DASH_E_INVALID_ARG;
  if (c->served && !c->server_ingest)
    return fail(c, DASH_E_BAD_STATE, "a served stream takes rows through dash_server_submit");
  if (!c->initialized) return fail(c, DASH_E_BAD_STATE, "context not initialised");
  if (L < 0) return fail(c, DASH_E_INVALID_ARG, "L < 0");
  if (first_id) *first_id = c->K_pending;
  if (L == 0) return DASH_OK;
  if (c->fail_next == DASH_SITE_INGEST) {
    c->fail_next = 0;
    return fail(c, DASH_E_CAPACITY, "dash_ingest_slices: injected failure, nothing staged");
  }
  if (dash_status s = validate_ptr(c, row_ptr, L, true)) return s;
  if (!rows) return fail(c, DASH_E_INVALID_ARG, "rows is NULL");
  const int64_t add = row_ptr[L] - row_ptr[0];
  if ((int64_t)c->K_pending + L > c->K_cap)
    return fail(c, DASH_E_CAPACITY, "slices would exceed max_slices=%lld", (long long)c->K_cap);
  if (c->rows_pending + add > c->M_cap)
    return fail(c, DASH_E_CAPACITY, "rows per update would exceed %lld", (long long)c->M_cap);
  if ((int64_t)c->pending.size() + L > c->G_cap)
    return fail(c, DASH_E_CAPACITY, "row groups per update would exceed %lld", (long long)c->G_cap);
  for (int32_t l = 0; l < L; ++l) {
    const int64_t m = row_ptr[l + 1] - row_ptr[l];
    c->pending.push_back({c->K_pending + l, rows + row_ptr[l] * c->J, m, c->rows_pending});
    c->rows_pending += m;
  }
  c->K_pending += L;
  return DASH_OK;
}

dash_status dash_debug_fail_next(dash_ctx *c, int32_t site) {
  if (!c) return DASH_E_INVALID_ARG;
  if (site < DASH_SITE_NONE || site > DASH_SITE_INIT_ALLOC)
    return fail(c, DASH_E_INVALID_ARG, "dash_debug_fail_next: unknown site %d", site);
  c->fail_next = site;
  return DASH_OK;
}

}  // extern "C"

namespace dash {

bool stage_free(dash_ctx *c) {
  const int s = c->stage_next;
  return !c->stage_used[s] || hipEventQuery(c->stage_ev[s]) == hipSuccess;
}

dash_status build_update(dash_ctx *c, BuiltUpdate *bu) {
  const int K = c->K_pending, Kp = c->K_enq;
  int cand = -1;
  if (!c->tune_cands.empty() && !c->tuned) {
    cand = c->tune_next % (int)c->tune_cands.size();
    c->tune_next++;
    c->sched = c->tune_cands[cand];
  }
  const int ch = choose_chunk(c, K);
  const int nch = (K + ch - 1) / ch;
  int s;
  HIP_OR_FAIL(c, take_stage(c, &s));
  char *blk = c->hstage[s];
  StepHeader *h = stage_header(blk);
  int32_t *gptr = (int32_t *)(blk + c->off_gptr);
  Group *grp = (Group *)(blk + c->off_groups);
  // groups sorted by slice, ingest order kept within a slice
  const int ng = (int)c->pending.size();
  bool sorted = true;
  for (int g = 1; g < ng; ++g)
    if (c->pending[g].slice < c->pending[g - 1].slice) {
      sorted = false;
      break;
    }
  c->order.resize(ng);
  for (int g = 0; g < ng; ++g) c->order[g] = g;
  if (!sorted)
    std::stable_sort(c->order.begin(), c->order.end(),
                     [&](int x, int y) { return c->pending[x].slice < c->pending[y].slice; });
  for (int i = 0; i < ng; ++i) {
    const PendingGroup &pg = c->pending[c->order[i]];
    grp[i].src = pg.src;
    grp[i].out_row = pg.out_row;
    grp[i].nrows = (int32_t)pg.nrows;
    grp[i].slice = pg.slice;
  }
  int gi = 0;
  for (int cidx = 0; cidx <= nch; ++cidx) {
    const int first = cidx * ch;
    while (gi < ng && grp[gi].slice < first) ++gi;
    gptr[cidx] = gi;
  }
  // the touched slices (split sweep's row stage), most rows first
  const bool split = c->sched.variant == kPassSplit;
  int n_items = 0, c3 = ch, c2 = ch;
  c->off_items = align_up(c->off_groups + sizeof(Group) * ng, 64);
  if (split) split_chunks(c, K, &c3, &c2);
  {
    Item *items = (Item *)(blk + c->off_items);
    for (int g = 0; g < ng;) {
      int e = g, rows = 0;
      while (e < ng && grp[e].slice == grp[g].slice) rows += grp[e++].nrows;
      items[n_items++] = Item{grp[g].slice, g, e, rows};
      g = e;
    }
    std::stable_sort(items, items + n_items, [](const Item &x, const Item &y) { return x.rows > y.rows; });
  }
  const int64_t step = c->step_enq + 1;
  const int slot = (int)(step % kReportRing);
  std::memset(h, 0, sizeof *h);
  h->K = K;
  h->K_prev = Kp;
  h->n_groups = ng;
  h->n_chunks = nch;
  h->chunk = ch;
  h->chunks_per_rgroup = kChunksPerRGroup;
  h->n_rgroups = (nch + kChunksPerRGroup - 1) / kChunksPerRGroup;
  h->step = step;
  h->M = c->rows_pending;
  h->report = (void *)(c->dreport + slot);
  h->n_items = n_items;
  h->chunk2 = c2;
  h->n_chunks2 = (K + c2 - 1) / c2;
  h->seq = ++c->seq;
  if (c->fail_next == DASH_SITE_COMMIT) {
    h->force_fail = 1;
    c->fail_next = 0;
  }
  c->hreport[slot].done = 0;
  c->hreport[slot].t_start = c->hreport[slot].t_end = 0;
  const char *dblk = c->desc_fetch ? c->dstep[s] : c->hstage_dev[s];
  if (split) write_pass_args(c, blk, dblk, 0);
  bu->stage = s;
  bu->bytes = c->off_items + sizeof(Item) * n_items;
  bu->dblk = dblk;
  bu->nch = nch;
  bu->n_chunks2 = h->n_chunks2;
  bu->n_items = n_items;
  bu->step = step;
  bu->slot = slot;
  bu->cand = cand;
  bu->scored = c->anom_window > 0;
  bu->report = h->report;
  bu->K = K;
  bu->rows = c->rows_pending;
  return DASH_OK;
}

void account_update(dash_ctx *c, const BuiltUpdate &b) {
  const Group *grp = (const Group *)(c->hstage[b.stage] + c->off_groups);
  const int ng = (int)c->pending.size();
  int touched = 0;
  for (int g = 0; g < ng; ++g)
    if (g == 0 || grp[g].slice != grp[g - 1].slice) ++touched;
  const int K = c->K_pending;
  const double J = c->J, R = c->R, M = (double)c->rows_pending, Kt = (double)touched;
  const double bytes = c->cfg.n_iter * (M * J * 4 + M * R * 4 + K * (R * J * 4 + R * R * 4 + 8 + R * 8) +
                                        Kt * (R * J * 4 + R * R * 4 + 8) + K * R * 8);
  c->inflight.push_back({b.step, c->K_enq, K, c->rows_pending, b.slot, b.cand, bytes, b.n_items, b.scored});
  c->K_enq = K;
  c->step_enq = b.step;
  c->pending.clear();
  c->rows_pending = 0;
}

}  // namespace dash

extern "C" {

dash_status dash_update_async(dash_ctx *c) {
  if (!c) return DASH_E_INVALID_ARG;
  if (!c->initialized) return fail(c, DASH_E_BAD_STATE, "context not initialised");
  if (c->served) return fail(c, DASH_E_BAD_STATE, "a served stream is updated by its server's ticks");
  if (c->rows_pending == 0) return DASH_OK;  // empty update: no-op, no forgetting
  if (c->fail_next == DASH_SITE_LAUNCH) {
    c->fail_next = 0;
    return fail(c, DASH_E_DEVICE, "injected launch failure: nothing enqueued, the staged rows stay staged");
  }
  if ((int)c->inflight.size() >= kReportRing - 1) {
    dash_status s = dash_wait(c, nullptr);
    if (s != DASH_OK) return s;
  }
  // a tuning run about to start: a cached schedule for this shape ends it at once
  if (!c->tune_cands.empty() && !c->tuned && c->tune_next == 0 && c->tune_key.empty()) {
    c->tune_key = tune_key_of(c);
    Schedule cached{};
    if (!c->tune_cache.empty() && tune_cache_lookup(c, c->tune_key, &cached)) {
      c->sched = cached;
      c->tuned = true;
      c->tune_from_cache = true;
    }
  }
  // The default schedule of a context the wave sweep fits: that sweep while
  // each wave holds at most kWaveMaxSlices slices, the split sweep beyond
  // (faster there on this device, and its F sums stay FP64 throughout).  A
  // tuned or cached schedule is left as it is.
  if (c->variant == kPassWave && !c->variant_forced && c->tune_cands.empty()) {
    const int slots = kWaveWarps * std::max(1, c->n_cu);
    const bool wave = c->K_pending <= kWaveMaxSlices * slots;
    c->sched.variant = wave ? kPassWave : kPassSplit;
    c->sched.fuse = (wave && c->fused_lds > 0) ? 1 : 0;
  }
  BuiltUpdate b;
  if (dash_status st = build_update(c, &b)) return st;
  const int s = b.stage, nch = b.nch, n_items = b.n_items;
  const bool split = c->sched.variant == kPassSplit;
  c->profiling = c->prof_every > 0 && b.step % c->prof_every == 0;
  const bool tuning = !c->tune_cands.empty() && !c->tuned;
  const bool scored = b.scored;
  if (c->graph_on && !c->profiling && c->desc_fetch && !tuning && !scored) {
    if (c->gsched.variant != c->sched.variant || c->gsched.spread != c->sched.spread ||
        c->gsched.fuse != c->sched.fuse) {
      // captured for another schedule: drop the graphs once nothing runs them
      HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
      graph_reset(c);
      c->gsched = c->sched;
    }
    if (dash_status st = graph_update(c, s, b.bytes, nch, b.report, n_items, b.n_chunks2)) return st;
  } else {
    HIP_OR_FAIL(c, upload_stage(c, s, b.bytes, true, b.report));
    PassArgs a = base_args(c, s);
    a.mode = 0;
    for (int p = 0; p < c->cfg.n_iter; ++p) {
      a.pass = p;
      a.last_pass = (p == c->cfg.n_iter - 1) ? 1 : 0;
      if (split) {
        a.fuse = 0;
        if (dash_status st = enqueue_split_pass(c, a, args_dev(c, b.dblk, p), n_items, b.n_chunks2, nch)) return st;
        continue;
      }
      HIP_OR_FAIL(c, prof_begin(c, kProfPass));
      LAUNCH_OR_FAIL(c, launch_pass(a, c->sched.variant, nch, c->stream));
      HIP_OR_FAIL(c, prof_end(c));
      if (!a.fuse) {
        HIP_OR_FAIL(c, prof_begin(c, kProfSolve));
        LAUNCH_OR_FAIL(c, launch_finish(a, 0, c->stream));
        HIP_OR_FAIL(c, prof_end(c));
      }
    }
    if (scored) {
      // Definitions 1-2 with the committed factors; this kernel publishes the report
      a.last_pass = 1;
      LAUNCH_OR_FAIL(c, launch_slice_errors(a, c->anom, std::min(std::max(n_items, 1), 2 * std::max(1, c->n_cu)),
                                            c->stream));
    }
  }
  HIP_OR_FAIL(c, stage_done(c, s));
  if (c->profiling) c->prof.updates++;
  c->profiling = false;
  account_update(c, b);
  return DASH_OK;
}

dash_status dash_wait(dash_ctx *c, dash_update_report *rep) {
  if (!c) return DASH_E_INVALID_ARG;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  dash_status st = DASH_OK;
  bool failed = false;
  int64_t failed_step = 0;
  while (!c->inflight.empty()) {
    const InFlight f = c->inflight.front();
    c->inflight.pop_front();
    const Report &r = c->hreport[f.slot];
    if (c->spans_on) c->spans.push_back((float)(device_us(r) * 1e-3));
    if (r.committed) tune_account(c, f, r);
    if (!failed && r.committed) {
      c->K = f.K_after;
      c->step = f.step;
      c->m_last = f.rows;
      dash_update_report tmp{};
      score_report(c, f, r, &tmp);
      if (rep) {
        rep->step = r.step;
        rep->rows = r.rows;
        rep->K = r.K;
        rep->committed = 1;
        rep->fit = r.fit;
        rep->loss = r.loss;
        rep->sum_n = r.sum_n;
        rep->device_us = device_us(r);
        rep->te = tmp.te;
        rep->te_threshold = tmp.te_threshold;
        rep->te_anomaly = tmp.te_anomaly;
        rep->n_anomalies = tmp.n_anomalies;
      }
    } else if (!failed) {
      failed = true;
      failed_step = f.step;
      if (rep) {
        rep->step = f.step;
        rep->rows = f.rows;
        rep->K = f.K_prev;
        rep->committed = 0;
        rep->fit = r.fit;
        rep->loss = r.loss;
        rep->sum_n = r.sum_n;
        rep->device_us = device_us(r);
        rep->te = rep->te_threshold = 0.0;
        rep->te_anomaly = rep->n_anomalies = 0;
      }
    }
  }
  if (failed) {
    // discard the failed update and everything enqueued after it
    Ctl ctl;
    HIP_OR_FAIL(c, hipMemcpy(&ctl, c->ctl, sizeof ctl, hipMemcpyDeviceToHost));
    ctl.poison = 0;
    HIP_OR_FAIL(c, hipMemcpy(c->ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice));
    c->K_enq = c->K_pending = c->K;
    c->step_enq = c->step;
    c->m_last = 0;
    c->pending.clear();
    c->rows_pending = 0;
    st = fail(c, DASH_E_NUMERIC, "update %lld produced non-finite factors; rolled back",
              (long long)failed_step);
  }
  return st;
}

dash_status dash_poll(dash_ctx *c, dash_update_report *reps, int32_t cap, int32_t *n_done) {
  if (!c || !n_done || cap < 0 || (cap > 0 && !reps)) return DASH_E_INVALID_ARG;
  *n_done = 0;
  while (!c->inflight.empty() && *n_done < cap) {
    const InFlight f = c->inflight.front();
    const Report &r = c->hreport[f.slot];
    // the final phase writes the report, then (after a system-scope fence) done
    if (!__atomic_load_n(&r.done, __ATOMIC_ACQUIRE)) break;
    if (!r.committed) {
      // the rollback needs the stream idle: drain like dash_wait, report the failed update
      dash_update_report last{};
      const dash_status st = dash_wait(c, &last);
      reps[(*n_done)++] = last;
      return st;
    }
    c->inflight.pop_front();
    if (c->spans_on) c->spans.push_back((float)(device_us(r) * 1e-3));
    tune_account(c, f, r);
    c->K = f.K_after;
    c->step = f.step;
    c->m_last = f.rows;
    dash_update_report &o = reps[(*n_done)++];
    o.step = r.step;
    o.rows = r.rows;
    o.K = r.K;
    o.committed = 1;
    o.fit = r.fit;
    o.loss = r.loss;
    o.sum_n = r.sum_n;
    o.device_us = device_us(r);
    score_report(c, f, r, &o);
  }
  return DASH_OK;
}

dash_status dash_anomaly(dash_ctx *c, int32_t window) {
  if (!c || window < 0) return DASH_E_INVALID_ARG;
  if (dash_status s = dash_wait(c, nullptr)) return s;
  AnomalyArgs &x = c->anom;
  (void)hipFree(x.se);
  (void)hipFree(x.flag);
  (void)hipFree(x.sid);
  (void)hipFree(x.hist);
  (void)hipFree(x.hcnt);
  (void)hipFree(x.ticket);
  x = AnomalyArgs{};
  c->anom_window = 0;
  c->te_hist.clear();
  c->anom_n_last = -1;
  if (window == 0) return DASH_OK;
  const bool ok = dalloc(&x.se, sizeof(float) * c->G_cap) == hipSuccess &&
                  dalloc(&x.flag, sizeof(int32_t) * c->G_cap) == hipSuccess &&
                  dalloc(&x.sid, sizeof(int32_t) * c->G_cap) == hipSuccess &&
                  dalloc(&x.hist, sizeof(float) * c->K_cap * window) == hipSuccess &&
                  dalloc(&x.hcnt, sizeof(int32_t) * c->K_cap) == hipSuccess &&
                  dalloc(&x.ticket, sizeof(int32_t)) == hipSuccess;
  if (!ok) {
    (void)dash_anomaly(c, 0);
    return fail(c, DASH_E_OUT_OF_MEMORY, "anomaly-score buffers");
  }
  HIP_OR_FAIL(c, hipMemsetAsync(x.hcnt, 0, sizeof(int32_t) * c->K_cap, c->stream));
  HIP_OR_FAIL(c, hipMemsetAsync(x.ticket, 0, sizeof(int32_t), c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  x.window = window;
  c->anom_window = window;
  return DASH_OK;
}

dash_status dash_get_slice_errors(dash_ctx *c, int32_t *slice, float *se, int32_t *flag, int32_t cap, int32_t *n) {
  if (!c || !n || cap < 0 || (cap > 0 && (!slice || !se || !flag))) return DASH_E_INVALID_ARG;
  if (c->anom_window == 0) return fail(c, DASH_E_BAD_STATE, "anomaly scores are off");
  if (dash_status s = dash_wait(c, nullptr)) return s;
  *n = 0;
  const int m = c->anom_n_last;
  if (m <= 0) return DASH_OK;
  std::vector<float> s_se(m);
  std::vector<int32_t> s_fl(m), s_id(m);
  HIP_OR_FAIL(c, hipMemcpy(s_se.data(), c->anom.se, sizeof(float) * m, hipMemcpyDeviceToHost));
  HIP_OR_FAIL(c, hipMemcpy(s_fl.data(), c->anom.flag, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  HIP_OR_FAIL(c, hipMemcpy(s_id.data(), c->anom.sid, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return s_id[x] < s_id[y]; });
  const int out = std::min(m, cap);
  for (int i = 0; i < out; ++i) {
    slice[i] = s_id[ord[i]];
    se[i] = s_se[ord[i]];
    flag[i] = s_fl[ord[i]];
  }
  *n = out;
  return DASH_OK;
}

dash_status dash_autotune(dash_ctx *c, int32_t trials) {
  if (!c || trials < 0) return DASH_E_INVALID_ARG;
  c->tune_cands.clear();
  c->tune_us.clear();
  c->tune_bytes.clear();
  c->tune_n.clear();
  c->tune_next = 0;
  c->tuned = false;
  c->tune_key.clear();
  c->tune_from_cache = false;
  const int fl = (int)fused_pass_lds(c->variant, c->J, c->R);
  c->sched = Schedule{c->variant, 1, fl > 0 ? 1 : 0};
  if (trials == 0) return DASH_OK;
  std::vector<int> variants{c->variant};
  if (c->variant == kPassWave) variants.push_back(kPassSplit);
  for (int v : variants)
    for (int spread : {1, 2})
      for (int fuse : {1, 0})
        for (int sd : {1, 4}) {
          if (fuse && fused_pass_lds(v, c->J, c->R) == 0) continue;
          if (sd > 1 && v != kPassSplit) continue;   // solve chunks exist in the split sweep only
          c->tune_cands.push_back(Schedule{v, spread, fuse, sd});
        }
  c->tune_us.assign(c->tune_cands.size(), 0.0);
  c->tune_bytes.assign(c->tune_cands.size(), 0.0);
  c->tune_n.assign(c->tune_cands.size(), 0);
  c->tune_per = trials;
  return DASH_OK;
}

dash_status dash_autotune_read(dash_ctx *c, dash_schedule *out) {
  if (!c || !out) return DASH_E_INVALID_ARG;
  out->variant = c->sched.variant;
  out->spread = c->sched.spread;
  out->fused = c->sched.fuse;
  out->solve_div = c->sched.solve_div;
  out->from_cache = c->tune_from_cache ? 1 : 0;
  out->tuned = c->tuned ? 1 : 0;
  out->candidates = (int32_t)c->tune_cands.size();
  out->ns_per_kb = 0.0;
  for (size_t i = 0; i < c->tune_cands.size(); ++i) {
    const Schedule &k = c->tune_cands[i];
    if (k.variant == c->sched.variant && k.spread == c->sched.spread && k.fuse == c->sched.fuse &&
        k.solve_div == c->sched.solve_div && c->tune_bytes[i] > 0)
      out->ns_per_kb = 1e3 * c->tune_us[i] / (c->tune_bytes[i] / 1024.0);
  }
  return DASH_OK;
}

dash_status dash_autotune_cache(dash_ctx *c, const char *path) {
  if (!c) return DASH_E_INVALID_ARG;
  c->tune_cache = path ? path : "";
  return DASH_OK;
}

dash_status dash_graph(dash_ctx *c, int32_t enable) {
  if (!c) return DASH_E_INVALID_ARG;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  graph_reset(c);
  c->graph_on = enable != 0;
  return DASH_OK;
}

dash_status dash_spans(dash_ctx *c, int32_t enable) {
  if (!c) return DASH_E_INVALID_ARG;
  c->spans.clear();
  c->spans_on = enable != 0;
  return DASH_OK;
}

dash_status dash_spans_read(dash_ctx *c, float *ms, int32_t cap, int32_t *n) {
  if (!c || !n || cap < 0 || (cap > 0 && !ms)) return DASH_E_INVALID_ARG;
  *n = (int32_t)std::min<size_t>((size_t)cap, c->spans.size());
  std::copy(c->spans.begin(), c->spans.begin() + *n, ms);
  return DASH_OK;
}

dash_status dash_footprint(const dash_config *cfg, int64_t *bytes) {
  if (!cfg || !bytes) return DASH_E_INVALID_ARG;
  if (cfg->J < 1 || cfg->J > kMaxJ || cfg->R < 1 || cfg->R > kMaxR || cfg->max_slices < 1 ||
      cfg->max_rows_per_update < 1 || cfg->max_groups_per_update < 1)
    return DASH_E_INVALID_ARG;
  *bytes = context_footprint(cfg);
  return DASH_OK;
}

dash_status dash_update(dash_ctx *c, dash_update_report *rep) {
  if (!c) return DASH_E_INVALID_ARG;
  if (!c->initialized) return fail(c, DASH_E_BAD_STATE, "context not initialised");
  if (c->rows_pending == 0 && c->inflight.empty()) {
    if (rep) {
      Ctl ctl;
      if (dash_status s = read_ctl(c, &ctl)) return s;
      rep->step = c->step;
      rep->rows = 0;
      rep->K = c->K;
      rep->committed = 1;
      rep->fit = ctl.fit;
      rep->loss = ctl.loss;
      rep->sum_n = ctl.sum_n;
    }
    return DASH_OK;
  }
  if (dash_status s = dash_update_async(c)) return s;
  return dash_wait(c, rep);
}

dash_status dash_get_factors(dash_ctx *c, float *V, float *W, float *U_new, int64_t *m_last) {
  if (!c) return DASH_E_INVALID_ARG;
  if (!c->initialized) return fail(c, DASH_E_BAD_STATE, "context not initialised");
  if (dash_status s = dash_wait(c, nullptr)) return s;
  Ctl ctl;
  if (dash_status s = read_ctl(c, &ctl)) return s;
  const VBundleView v = vb_view(c->vb + (int64_t)ctl.gcur * c->vb_stride, c->J, c->R);
  if (V) LAUNCH_OR_FAIL(c, launch_to_f32(v.V64, V, (int64_t)c->J * c->R, c->stream));
  if (W) LAUNCH_OR_FAIL(c, launch_to_f32(c->W + (int64_t)ctl.gcur * c->K_cap * c->R, W, (int64_t)c->K * c->R, c->stream));
  if (U_new && c->m_last > 0)
    HIP_OR_FAIL(c, hipMemcpyAsync(U_new, c->U_out, sizeof(float) * c->m_last * c->R,
                                  hipMemcpyDeviceToDevice, c->stream));
  if (m_last) *m_last = c->m_last;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  return DASH_OK;
}

dash_status dash_get_state(dash_ctx *c, double *V, double *W, double *Y, double *D, double *n) {
  if (!c) return DASH_E_INVALID_ARG;
  if (!c->initialized) return fail(c, DASH_E_BAD_STATE, "context not initialised");
  if (dash_status s = dash_wait(c, nullptr)) return s;
  Ctl ctl;
  if (dash_status s = read_ctl(c, &ctl)) return s;
  const int64_t K = c->K, J = c->J, R = c->R;
  const VBundleView v = vb_view(c->vb + (int64_t)ctl.gcur * c->vb_stride, c->J, c->R);
  if (V) HIP_OR_FAIL(c, hipMemcpy(V, v.V64, sizeof(double) * J * R, hipMemcpyDeviceToHost));
  if (W) HIP_OR_FAIL(c, hipMemcpy(W, c->W + (int64_t)ctl.gcur * c->K_cap * R, sizeof(double) * K * R, hipMemcpyDeviceToHost));
  if (Y || D || n) {
    double *dY = nullptr, *dD = nullptr, *dn = nullptr;
    if (dalloc(&dY, sizeof(double) * K * R * J) != hipSuccess || dalloc(&dD, sizeof(double) * K * R * R) != hipSuccess ||
        dalloc(&dn, sizeof(double) * K) != hipSuccess) {
      (void)hipFree(dY);
      (void)hipFree(dD);
      (void)hipFree(dn);
      return fail(c, DASH_E_OUT_OF_MEMORY, "export buffers");
    }
    int e = launch_export_state(c->J, c->R, c->K, c->step, c->cfg.lambda, c->Y, c->D, c->n,
                                c->cur + (int64_t)ctl.gcur * c->K_cap, c->tlast + (int64_t)ctl.gcur * c->K_cap,
                                c->K_cap, dY, dD, dn, c->Yc, c->Dc, c->stream);
    hipError_t he = (hipError_t)e;
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he == hipSuccess && Y) he = hipMemcpy(Y, dY, sizeof(double) * K * R * J, hipMemcpyDeviceToHost);
    if (he == hipSuccess && D) he = hipMemcpy(D, dD, sizeof(double) * K * R * R, hipMemcpyDeviceToHost);
    if (he == hipSuccess && n) he = hipMemcpy(n, dn, sizeof(double) * K, hipMemcpyDeviceToHost);
    (void)hipFree(dY);
    (void)hipFree(dD);
    (void)hipFree(dn);
    if (he != hipSuccess) return fail(c, DASH_E_DEVICE, "state export: %s", hipGetErrorString(he));
  }
  return DASH_OK;
}

dash_status dash_set_state(dash_ctx *c, int32_t K, const double *V, const double *W, const double *Y,
                           const double *D, const double *n) {
  if (!c) return DASH_E_INVALID_ARG;
  if (K < 1) return fail(c, DASH_E_INVALID_ARG, "K must be >= 1");
  if (K > c->K_cap) return fail(c, DASH_E_CAPACITY, "K=%d exceeds max_slices", K);
  if (!V || !W || !Y || !D || !n) return fail(c, DASH_E_INVALID_ARG, "NULL state array");
  if (dash_status s = dash_wait(c, nullptr)) return s;
  const int64_t J = c->J, R = c->R;
  const int64_t tl = c->step;
  if (dash_status s = reset_device_state(c, K, (int32_t)tl)) return s;
  // the state is stored in float32 (Y, D) and float64 (n, W, V); the cast is the
  // only host-side arithmetic (a mixed-precision context also keeps the
  // remainder of the cast as its compensation word)
  std::vector<float> f((size_t)std::max<int64_t>(K * R * J, K * R * R)), lo(c->Yc ? f.size() : 0);
  std::vector<uint16_t> lob(c->Yc ? (size_t)(K * R * J) : 0);
  for (int64_t i = 0; i < K * R * J; ++i) {
    f[i] = (float)Y[i];
    if (c->Yc) lob[i] = bf16_bits((float)(Y[i] - (double)f[i]));
  }
  HIP_OR_FAIL(c, hipMemcpy2D(c->Y, sizeof(float) * y_stride(c->J, c->R), f.data(), sizeof(float) * R * J,
                             sizeof(float) * R * J, (size_t)K, hipMemcpyHostToDevice));
  if (c->Yc)
    HIP_OR_FAIL(c, hipMemcpy2D(c->Yc, sizeof(uint16_t) * y_stride(c->J, c->R), lob.data(), sizeof(uint16_t) * R * J,
                               sizeof(uint16_t) * R * J, (size_t)K, hipMemcpyHostToDevice));
  for (int64_t i = 0; i < K * R * R; ++i) {
    f[i] = (float)D[i];
    if (c->Dc) lo[i] = (float)(D[i] - (double)f[i]);
  }
  HIP_OR_FAIL(c, hipMemcpy(c->D, f.data(), sizeof(float) * K * R * R, hipMemcpyHostToDevice));
  if (c->Dc) HIP_OR_FAIL(c, hipMemcpy(c->Dc, lo.data(), sizeof(float) * K * R * R, hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(c->n, n, sizeof(double) * K, hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(c->W, W, sizeof(double) * K * R, hipMemcpyHostToDevice));
  const VBundleView v = vb_view(c->vb, c->J, c->R);
  HIP_OR_FAIL(c, hipMemcpy(v.V64, V, sizeof(double) * J * R, hipMemcpyHostToDevice));
  if (dash_status s = enqueue_prep(c)) return s;
  if (dash_status s = enqueue_eval(c, K)) return s;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->initialized = true;
  c->K = c->K_enq = c->K_pending = K;
  c->step_enq = c->step;
  c->m_last = 0;
  c->pending.clear();
  c->rows_pending = 0;
  return DASH_OK;
}

namespace {
// Checkpoint file: header, then the raw committed state exactly as the device
// holds it (float32 Y_k and D_k without the pending lambda^dt, float64 n_k,
// W and V, int32 t_k; a mixed-precision context appends the compensation
// words of Y_k and D_k and sets `carry`), so that a restored context continues
// bit for bit.
struct CkptHeader {
  char magic[8];
  int32_t J, R, K, carry;
  int64_t step;
  double lambda;
};
}  // namespace

dash_status dash_save(dash_ctx *c, const char *path) {
  if (!c || !path) return DASH_E_INVALID_ARG;
  if (!c->initialized) return fail(c, DASH_E_BAD_STATE, "context not initialised");
  if (dash_status s = dash_wait(c, nullptr)) return s;
  Ctl ctl;
  if (dash_status s = read_ctl(c, &ctl)) return s;
  const int64_t K = c->K, J = c->J, R = c->R;
  std::vector<float> Y(K * R * J), D(K * R * R);
  std::vector<double> n(K), W(K * R), V(J * R);
  std::vector<int32_t> tl(K);
  float *dY = nullptr, *dD = nullptr;
  double *dn = nullptr;
  if (dalloc(&dY, sizeof(float) * K * R * J) != hipSuccess || dalloc(&dD, sizeof(float) * K * R * R) != hipSuccess ||
      dalloc(&dn, sizeof(double) * K) != hipSuccess) {
    (void)hipFree(dY);
    (void)hipFree(dD);
    (void)hipFree(dn);
    return fail(c, DASH_E_OUT_OF_MEMORY, "checkpoint buffers");
  }
  hipError_t he = (hipError_t)launch_gather_state(c->J, c->R, c->K, c->Y, c->D, c->n,
                                                  c->cur + (int64_t)ctl.gcur * c->K_cap, c->K_cap, dY, dD, dn,
                                                  c->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  if (he == hipSuccess) he = hipMemcpy(Y.data(), dY, sizeof(float) * Y.size(), hipMemcpyDeviceToHost);
  if (he == hipSuccess) he = hipMemcpy(D.data(), dD, sizeof(float) * D.size(), hipMemcpyDeviceToHost);
  if (he == hipSuccess) he = hipMemcpy(n.data(), dn, sizeof(double) * n.size(), hipMemcpyDeviceToHost);
  std::vector<float> Yc(c->Yc ? Y.size() : 0), Dc(c->Dc ? D.size() : 0);
  if (c->Yc && he == hipSuccess) {
    // the carry arrays share the layout of Y and D (Y's widened from BF16)
    he = (hipError_t)launch_gather_carry(c->J, c->R, c->K, c->Yc, c->Dc, c->cur + (int64_t)ctl.gcur * c->K_cap,
                                         c->K_cap, dY, dD, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he == hipSuccess) he = hipMemcpy(Yc.data(), dY, sizeof(float) * Yc.size(), hipMemcpyDeviceToHost);
    if (he == hipSuccess) he = hipMemcpy(Dc.data(), dD, sizeof(float) * Dc.size(), hipMemcpyDeviceToHost);
  }
  (void)hipFree(dY);
  (void)hipFree(dD);
  (void)hipFree(dn);
  const VBundleView v = vb_view(c->vb + (int64_t)ctl.gcur * c->vb_stride, c->J, c->R);
  if (he == hipSuccess) he = hipMemcpy(V.data(), v.V64, sizeof(double) * V.size(), hipMemcpyDeviceToHost);
  if (he == hipSuccess)
    he = hipMemcpy(W.data(), c->W + (int64_t)ctl.gcur * c->K_cap * R, sizeof(double) * W.size(), hipMemcpyDeviceToHost);
  if (he == hipSuccess)
    he = hipMemcpy(tl.data(), c->tlast + (int64_t)ctl.gcur * c->K_cap, sizeof(int32_t) * K, hipMemcpyDeviceToHost);
  if (he != hipSuccess) return fail(c, DASH_E_DEVICE, "checkpoint read-back: %s", hipGetErrorString(he));
  FILE *fp = std::fopen(path, "wb");
  if (!fp) return fail(c, DASH_E_IO, "cannot open %s", path);
  CkptHeader h{};
  std::memcpy(h.magic, "DASHCKP2", 8);
  h.J = c->J;
  h.R = c->R;
  h.K = c->K;
  h.step = c->step;
  h.lambda = c->cfg.lambda;
  h.carry = c->Yc ? 1 : 0;
  bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1 && std::fwrite(Y.data(), 4, Y.size(), fp) == Y.size() &&
            std::fwrite(D.data(), 4, D.size(), fp) == D.size() && std::fwrite(n.data(), 8, n.size(), fp) == n.size() &&
            std::fwrite(W.data(), 8, W.size(), fp) == W.size() && std::fwrite(V.data(), 8, V.size(), fp) == V.size() &&
            std::fwrite(tl.data(), 4, tl.size(), fp) == tl.size() &&
            std::fwrite(Yc.data(), 4, Yc.size(), fp) == Yc.size() && std::fwrite(Dc.data(), 4, Dc.size(), fp) == Dc.size();
  ok = (std::fclose(fp) == 0) && ok;
  return ok ? DASH_OK : fail(c, DASH_E_IO, "short write to %s", path);
}

dash_status dash_load(dash_ctx *c, const char *path) {
  if (!c || !path) return DASH_E_INVALID_ARG;
  FILE *fp = std::fopen(path, "rb");
  if (!fp) return fail(c, DASH_E_IO, "cannot open %s", path);
  CkptHeader h{};
  if (std::fread(&h, sizeof h, 1, fp) != 1 || std::memcmp(h.magic, "DASHCKP2", 8) != 0) {
    std::fclose(fp);
    return fail(c, DASH_E_IO, "%s is not a checkpoint", path);
  }
  if (h.J != c->J || h.R != c->R || h.K < 1 || h.K > c->K_cap || h.lambda != c->cfg.lambda) {
    std::fclose(fp);
    return fail(c, DASH_E_INVALID_ARG, "checkpoint (J=%d R=%d K=%d lambda=%g) does not fit the context", h.J, h.R,
                h.K, h.lambda);
  }
  const int64_t K = h.K, J = h.J, R = h.R;
  std::vector<float> Y(K * R * J), D(K * R * R);
  std::vector<double> n(K), W(K * R), V(J * R);
  std::vector<int32_t> tl(K);
  if (h.carry != 0 && h.carry != 1) {
    std::fclose(fp);
    return fail(c, DASH_E_IO, "%s: bad carry flag", path);
  }
  std::vector<float> Yc(h.carry ? Y.size() : 0), Dc(h.carry ? D.size() : 0);
  bool ok = std::fread(Y.data(), 4, Y.size(), fp) == Y.size() && std::fread(D.data(), 4, D.size(), fp) == D.size() &&
            std::fread(n.data(), 8, n.size(), fp) == n.size() && std::fread(W.data(), 8, W.size(), fp) == W.size() &&
            std::fread(V.data(), 8, V.size(), fp) == V.size() && std::fread(tl.data(), 4, tl.size(), fp) == tl.size() &&
            std::fread(Yc.data(), 4, Yc.size(), fp) == Yc.size() && std::fread(Dc.data(), 4, Dc.size(), fp) == Dc.size();
  std::fclose(fp);
  if (!ok) return fail(c, DASH_E_IO, "short read from %s", path);
  if (dash_status s = dash_wait(c, nullptr)) return s;
  if (dash_status s = reset_device_state(c, (int32_t)K, 0)) return s;
  HIP_OR_FAIL(c, hipMemcpy2D(c->Y, sizeof(float) * y_stride(c->J, c->R), Y.data(), sizeof(float) * R * J,
                             sizeof(float) * R * J, (size_t)K, hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(c->D, D.data(), sizeof(float) * D.size(), hipMemcpyHostToDevice));
  if (c->Yc && h.carry) {   // a float32 context drops the words; a mixed one without them starts at zero
    std::vector<uint16_t> yb(Yc.size());
    for (size_t i = 0; i < Yc.size(); ++i) yb[i] = bf16_bits(Yc[i]);
    HIP_OR_FAIL(c, hipMemcpy2D(c->Yc, sizeof(uint16_t) * y_stride(c->J, c->R), yb.data(), sizeof(uint16_t) * R * J,
                               sizeof(uint16_t) * R * J, (size_t)K, hipMemcpyHostToDevice));
    HIP_OR_FAIL(c, hipMemcpy(c->Dc, Dc.data(), sizeof(float) * Dc.size(), hipMemcpyHostToDevice));
  }
  HIP_OR_FAIL(c, hipMemcpy(c->n, n.data(), sizeof(double) * n.size(), hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(c->W, W.data(), sizeof(double) * W.size(), hipMemcpyHostToDevice));
  HIP_OR_FAIL(c, hipMemcpy(c->tlast, tl.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice));
  const VBundleView v = vb_view(c->vb, c->J, c->R);
  HIP_OR_FAIL(c, hipMemcpy(v.V64, V.data(), sizeof(double) * V.size(), hipMemcpyHostToDevice));
  if (dash_status s = enqueue_prep(c)) return s;
  c->step = h.step;
  if (dash_status s = enqueue_eval(c, (int32_t)K)) return s;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->initialized = true;
  c->K = c->K_enq = c->K_pending = (int32_t)K;
  c->step_enq = c->step;
  c->m_last = 0;
  c->pending.clear();
  c->rows_pending = 0;
  return DASH_OK;
}


}  // extern "C"
