// Serving layer of libdash (dash_server_* in include/dash.h): many independent
// streams -- each its own irregular tensor, decomposed by its own context
// (Problem 1 per stream) -- on one device.
//
// Clients submit row requests at any time; a tick cuts, for every admitted
// stream with submitted rows, one update from the requests it has so far and
// runs all of those updates together: one descriptor fetch for the whole
// tick, then each stage of the split sweep (row stage, deferred slices, solve,
// F stage, group reduction, final phase) as one launch per kernel class
// (template instantiation), whose workgroups a block map hands to the
// streams.  A stream's workgroup count and chunking in every stage depend on
// the stream alone, and every sum is taken in a fixed order within the stream,
// so its results are bit for bit the same alone and in any mix.
//
// Admission is by device footprint against the server's budget; a stream that
// does not fit may wait in a FIFO queue and is admitted when closes free the
// budget.  dash_server_start runs the tick/poll loop on a host thread of its
// own: a tick is launched as soon as rows are waiting and no tick is in
// flight, or beside the one in flight once every open stream has rows
// waiting, so requests that arrive while the GPU works join the next tick
// (continuous batching) and a second tick in flight is a full one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "dash_ctx.h"

using namespace dash;

namespace {

constexpr int kTickStages = 4;        // pinned launch tables in rotation
constexpr int kMaxServed = 4096;      // stream ids
constexpr int kTicksInFlight = 2;     // loop mode: ticks on the device at once
constexpr int kAuxStreams = 3;        // extra streams: kernel classes of one stage run side by side

double now_us() {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  std::vector<int32_t> slice_id;
  std::vector<int64_t> row_ptr;
  const float *rows = nullptr;
  std::vector<int64_t> new_ptr;
  const float *new_rows = nullptr;
  hipEvent_t ready = nullptr;   // recorded on the producer's stream, or none
  double t_submit = 0.0;
  int64_t n_rows = 0;           // rows of existing and new slices
  int64_t n_groups = 0;         // non-empty row groups plus new slices
};

struct Cut {
  double t_first;          // submit time of the update's first request
  int64_t last_request;    // the last request it consumed
};

enum { kStateClosed = 0, kStateQueued = 1, kStateOpen = 2 };

struct Stream {
  int state = kStateClosed;
  dash_ctx *ctx = nullptr;
  dash_config cfg{};
  int64_t footprint = 0;
  int32_t K_sub = -1;               // slices after every submitted request
  std::deque<Request> requests;     // submitted, not yet in an update
  std::deque<Cut> cuts;             // updates in flight
};

struct TickBuf {
  char *host = nullptr;    // pinned launch table: fetch jobs, then block maps
  char *hdev = nullptr;    // its device view
  char *dev = nullptr;     // device copy of the block maps
  size_t cap = 0;
  hipEvent_t ev = nullptr;   // the tick that last used it has completed
  bool used = false;
};

// One stream's update in the tick being built.
struct Sel {
  int32_t sid;
  dash_ctx *c;
  BuiltUpdate b;
  Cut cut;
};

// One launch of the tick: a stage's kernel class over its streams.
struct Launch {
  int group;          // launches of one (pass, stage): independent of each other
  int stage;          // 0 rows, 1 deferred slices, 2 solve, 3 F, 4 group reduction, 5 final phase
  PassArgs rep;       // a member's host arguments (the class is read from them)
  size_t map_off;     // byte offset of its block map in the table
  int n_blocks;
  size_t lds;         // the largest member's dynamic LDS
  double bytes;       // algorithmic bytes of its members' work
};

// A timed launch waiting for its events to be read.
struct ProfRec {
  hipEvent_t a, b;
  int entry;          // index into the per-kernel statistics
  double bytes;
};

// Algorithmic bytes one stage must move for one stream's update: 4 bytes per
// Y_k / D_k entry in float32; in the mixed path 6 per Y_k entry (float32
// value, BF16 compensation word) and 8 per D_k entry.
double stage_bytes(int stage, const dash_ctx *c, const BuiltUpdate &b) {
  const double J = c->J, R = c->R, M = (double)b.rows, K = b.K, Kt = b.n_items;
  const bool mx = c->cfg.precision == DASH_PREC_MIXED;
  const double yb = mx ? 6.0 : 4.0, db = mx ? 8.0 : 4.0;   // bytes per Y / D entry (BF16 / float32 carry)
  switch (stage) {
    case 0: return M * J * 4 + M * R * 4 + Kt * (2 * (R * J * yb + R * R * db) + 16 + R * 8);
    case 1: return 0.0;   // deferred slices: counted with the row stage
    case 2: return (K - Kt) * R * J * 4 + K * R * R * db + K * (2 * R * 8 + 8) + Kt * R * 8;
    case 3: return K * R * J * 4 + K * R * 8;
    case 4: return ((double)b.nch / kChunksPerRGroup + 1) * (R * J + R * R) * 8;
    default: return 2 * (R * J + R * R) * 8;
  }
}

}  // namespace

struct dash_server {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t aux[kAuxStreams] = {};   // a stage's further kernel classes, joined back by events
  int64_t budget = 0, used = 0;
  std::vector<Stream> streams;
  std::deque<int32_t> admit_queue;
  std::mutex mu;
  std::condition_variable cv;
  std::thread loop;
  bool running = false, stop = false;
  int tick_us = 0;
  double last_tick = 0.0;
  TickBuf tb[kTickStages];
  int tb_next = 0;
  std::deque<hipEvent_t> ticks_in_flight;
  std::vector<hipEvent_t> ev_pool;
  std::deque<dash_server_report> done;   // finished updates not yet polled
  dash_status loop_err = DASH_OK;
  int64_t next_request = 1;
  dash_server_stats stats{};
  std::string err;
  // profiling: HIP events around every launch of every prof_every-th tick
  int prof_every = 0;
  int64_t prof_ticks = 0;
  std::vector<ProfRec> prof_pending;
  std::vector<dash_kernel_stat> prof_stats;
  std::vector<hipEvent_t> tev_pool;   // timing events
};

namespace {

hipEvent_t take_event(dash_server *srv) {
  if (!srv->ev_pool.empty()) {
    hipEvent_t e = srv->ev_pool.back();
    srv->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void free_tick_bufs(dash_server *srv) {
  for (auto &t : srv->tb) {
    if (t.host) (void)hipHostFree(t.host);
    if (t.dev) (void)hipFree(t.dev);
    t.host = t.hdev = t.dev = nullptr;
    t.cap = 0;
    t.used = false;
  }
}

// A launch table of at least `bytes`, free for the host to rewrite.
dash_status take_tick_buf(dash_server *srv, size_t bytes, TickBuf **out) {
  if (bytes > srv->tb[srv->tb_next].cap) {
    // grow every table once nothing in flight reads them
    if (hipStreamSynchronize(srv->stream) != hipSuccess) return DASH_E_DEVICE;
    free_tick_bufs(srv);
    const size_t cap = std::max<size_t>(2 * bytes, 1 << 20);
    for (auto &t : srv->tb) {
      if (hipHostMalloc((void **)&t.host, cap, hipHostMallocMapped) != hipSuccess ||
          hipHostGetDevicePointer((void **)&t.hdev, t.host, 0) != hipSuccess ||
          hipMalloc((void **)&t.dev, cap) != hipSuccess)
        return DASH_E_OUT_OF_MEMORY;
      if (!t.ev && hipEventCreateWithFlags(&t.ev, hipEventDisableTiming) != hipSuccess) return DASH_E_DEVICE;
      t.cap = cap;
    }
  }
  TickBuf *t = &srv->tb[srv->tb_next];
  srv->tb_next = (srv->tb_next + 1) % kTickStages;
  if (t->used && hipEventSynchronize(t->ev) != hipSuccess) return DASH_E_DEVICE;
  *out = t;
  return DASH_OK;
}

// The server's HIP stream, made at the first admission: a blocking stream, so
// that the updates are ordered after work on the null stream (rows produced
// there by callers that name no stream).
dash_status ensure_stream(dash_server *srv) {
  if (srv->stream) return DASH_OK;
  if (hipSetDevice(srv->device) != hipSuccess || hipStreamCreate(&srv->stream) != hipSuccess) return DASH_E_DEVICE;
  for (auto &a : srv->aux)
    if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess) return DASH_E_DEVICE;
  return DASH_OK;
}

// Admit queued streams in arrival order while the head fits the budget.
void admit(dash_server *srv) {
  while (!srv->admit_queue.empty()) {
    const int32_t sid = srv->admit_queue.front();
    Stream &st = srv->streams[sid];
    if (srv->used + st.footprint > srv->budget) break;
    srv->admit_queue.pop_front();
    dash_ctx *ctx = nullptr;
    st.cfg.stream = srv->stream;
    if (create_context(&st.cfg, srv->stream, true, &ctx) != DASH_OK) {
      st = Stream{};   // could not be created: the id is closed
      continue;
    }
    st.ctx = ctx;
    st.state = kStateOpen;
    srv->used += st.footprint;
  }
}

// Finished updates of every stream into srv->done.
dash_status collect(dash_server *srv) {
  dash_status first = DASH_OK;
  const double t = now_us();
  for (size_t id = 0; id < srv->streams.size(); ++id) {
    Stream &st = srv->streams[id];
    if (st.state != kStateOpen || st.cuts.empty()) continue;
    dash_update_report reps[kReportRing];
    int32_t got = 0;
    const dash_status s = dash_poll(st.ctx, reps, kReportRing, &got);
    for (int32_t i = 0; i < got && !st.cuts.empty(); ++i) {
      dash_server_report o{};
      o.stream = (int32_t)id;
      o.committed = reps[i].committed;
      o.step = reps[i].step;
      o.rows = reps[i].rows;
      o.fit = reps[i].fit;
      o.latency_us = t - st.cuts.front().t_first;
      o.last_request = st.cuts.front().last_request;
      o.device_us = reps[i].device_us;
      st.cuts.pop_front();
      srv->done.push_back(o);
      srv->stats.updates += 1;
      srv->stats.rows += o.rows;
    }
    if (s != DASH_OK) {
      // rolled back: the stream's later updates in flight are gone too
      for (const Cut &c : st.cuts) {
        dash_server_report o{};
        o.stream = (int32_t)id;
        o.committed = 0;
        o.latency_us = t - c.t_first;
        o.last_request = c.last_request;
        srv->done.push_back(o);
      }
      st.cuts.clear();
      if (first == DASH_OK) first = s;
    }
  }
  while (!srv->ticks_in_flight.empty() && hipEventQuery(srv->ticks_in_flight.front()) == hipSuccess) {
    srv->ev_pool.push_back(srv->ticks_in_flight.front());
    srv->ticks_in_flight.pop_front();
  }
  return first;
}

// Move the stream's requests that fit one update into its context.
dash_status stage_requests(dash_server *srv, Stream &st, Cut *cut, int *n_req) {
  dash_ctx *c = st.ctx;
  *n_req = 0;
  while (!st.requests.empty()) {
    Request &q = st.requests.front();
    if (c->rows_pending + q.n_rows > c->M_cap || (int64_t)c->pending.size() + q.n_groups > c->G_cap) break;
    if (q.ready) {
      if (hipStreamWaitEvent(srv->stream, q.ready, 0) != hipSuccess) return DASH_E_DEVICE;
      srv->ev_pool.push_back(q.ready);
      q.ready = nullptr;
    }
    const int32_t n_new = (int32_t)q.new_ptr.size() - 1;
    const int32_t ng = (int32_t)q.slice_id.size();
    c->server_ingest = true;
    dash_status s = DASH_OK;
    if (n_new > 0) s = dash_ingest_slices(c, n_new, q.new_ptr.data(), q.new_rows, nullptr);
    if (s == DASH_OK && ng > 0) s = dash_ingest_rows(c, ng, q.slice_id.data(), q.row_ptr.data(), q.rows);
    c->server_ingest = false;
    if (s != DASH_OK) return s;
    if (*n_req == 0) cut->t_first = q.t_submit;
    cut->last_request = q.id;
    ++*n_req;
    st.requests.pop_front();
  }
  return DASH_OK;
}

hipEvent_t take_timing_event(dash_server *srv) {
  if (!srv->tev_pool.empty()) {
    hipEvent_t e = srv->tev_pool.back();
    srv->tev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Read the timed launches' events into the statistics (the stream is idle).
dash_status prof_fold(dash_server *srv) {
  for (const ProfRec &p : srv->prof_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) return DASH_E_DEVICE;
    dash_kernel_stat &st = srv->prof_stats[p.entry];
    st.launches += 1;
    st.ms += ms;
    st.bytes += p.bytes;
    srv->tev_pool.push_back(p.a);
    srv->tev_pool.push_back(p.b);
  }
  srv->prof_pending.clear();
  return DASH_OK;
}

int prof_entry(dash_server *srv, const char *name) {
  for (size_t i = 0; i < srv->prof_stats.size(); ++i)
    if (std::strncmp(srv->prof_stats[i].name, name, sizeof srv->prof_stats[i].name) == 0) return (int)i;
  dash_kernel_stat st{};
  std::snprintf(st.name, sizeof st.name, "%s", name);
  srv->prof_stats.push_back(st);
  return (int)srv->prof_stats.size() - 1;
}

void append_map(std::vector<BlockMap> &maps, const PassArgs *ad, int n) {
  for (int l = 0; l < n; ++l) maps.push_back(BlockMap{ad, l, n});
}

// Cut and launch one tick.  Caller holds srv->mu.
dash_status run_tick(dash_server *srv, int32_t *launched) {
  std::vector<Sel> sel;
  dash_status first = DASH_OK;
  for (size_t id = 0; id < srv->streams.size(); ++id) {
    Stream &st = srv->streams[id];
    if (st.state != kStateOpen || st.requests.empty() || !st.ctx->initialized) continue;
    dash_ctx *c = st.ctx;
    // at most kStages updates of a stream in flight: it waits for the next tick
    if (!stage_free(c) || (int)c->inflight.size() >= kReportRing - 1) continue;
    Cut cut{0.0, 0};
    int n_req = 0;
    dash_status s = stage_requests(srv, st, &cut, &n_req);
    if (s == DASH_OK && c->rows_pending == 0) continue;
    BuiltUpdate b;
    if (s == DASH_OK) s = build_update(c, &b);
    if (s != DASH_OK) {
      c->pending.clear();
      c->rows_pending = 0;
      c->K_pending = c->K_enq;
      if (first == DASH_OK) first = s;
      continue;
    }
    sel.push_back(Sel{(int32_t)id, c, b, cut});
  }
  if (launched) *launched = (int32_t)sel.size();
  if (sel.empty()) return first;

  // launch table: fetch jobs (one per stream, one for the block maps), maps
  std::vector<BlockMap> maps;
  std::vector<Launch> launches;
  int max_iter = 1, n_group = 0;
  for (const Sel &x : sel) max_iter = std::max(max_iter, x.c->cfg.n_iter);
  for (int p = 0; p < max_iter; ++p) {
    for (int stage = 0; stage < 6; ++stage, ++n_group) {
      // classes in order of first appearance (deterministic)
      std::vector<std::pair<int, std::vector<int>>> classes;
      for (int i = 0; i < (int)sel.size(); ++i) {
        const dash_ctx *c = sel[i].c;
        if (p >= c->cfg.n_iter) continue;
        if (stage <= 1 && sel[i].b.n_items == 0) continue;
        const int mixed = c->cfg.precision == DASH_PREC_MIXED;
        const int lagged = c->cfg.stats_mode == DASH_STATS_LAGGED;
        int key = 0;
        switch (stage) {
          case 0: key = split_rows_class(c->J, c->R, mixed); break;
          case 1: key = mixed; break;
          // one launch per kernel instantiation (they differ in registers and
          // occupancy), the classes of a stage side by side
          case 2: key = split_solve_class(c->R); break;
          case 3: key = split_fsum_class(c->J, c->R, lagged, mixed); break;
          case 4: key = 0; break;
          default: key = finish_class(c->R); break;
        }
        auto it = std::find_if(classes.begin(), classes.end(), [&](const auto &e) { return e.first == key; });
        if (it == classes.end()) {
          classes.push_back({key, {}});
          it = classes.end() - 1;
        }
        it->second.push_back(i);
      }
      for (const auto &cl : classes) {
        Launch L{};
        L.group = n_group;
        L.stage = stage;
        L.map_off = maps.size();
        L.n_blocks = 0;
        L.lds = 0;
        L.bytes = 0.0;
        for (int i : cl.second) {
          const dash_ctx *c = sel[i].c;
          const BuiltUpdate &b = sel[i].b;
          const PassArgs *ad = args_dev(c, b.dblk, p);
          const int mixed = c->cfg.precision == DASH_PREC_MIXED;
          const int lagged = c->cfg.stats_mode == DASH_STATS_LAGGED;
          int n = 0;
          size_t lds = 0;
          switch (stage) {
            case 0: n = std::min(b.n_items, c->rows_blocks); lds = split_rows_lds(c->J, c->R, mixed); break;
            case 1: n = kSlowBlocks; lds = split_rows_slow_lds(c->J, c->R); break;
            case 2: n = b.n_chunks2; lds = split_solve_lds(c->J, c->R); break;
            case 3: n = b.nch; lds = split_fsum_lds(c->J, c->R, lagged); break;
            case 4: n = reduce_groups_blocks(c->J, c->R); break;
            default: n = 1; lds = finish_dev_lds(c->J, c->R); break;
          }
          append_map(maps, ad, n);
          L.n_blocks += n;
          L.bytes += stage_bytes(stage, c, b);
          L.lds = std::max(L.lds, lds);
        }
        PassArgs a = base_args_at(sel[cl.second[0]].c, sel[cl.second[0]].b.dblk);
        a.mode = 0;
        a.pass = p;
        a.fuse = 0;
        L.rep = a;
        launches.push_back(L);
      }
    }
  }
  const int n_jobs = (int)sel.size() + 1;
  const size_t off_maps = align_up(sizeof(FetchJob) * n_jobs, 256);
  const size_t map_bytes = align_up(sizeof(BlockMap) * maps.size(), 16);
  TickBuf *tb = nullptr;
  if (dash_status s = take_tick_buf(srv, off_maps + map_bytes, &tb)) return s;
  FetchJob *jobs = (FetchJob *)tb->host;
  int64_t max_bytes = (int64_t)map_bytes;
  for (size_t i = 0; i < sel.size(); ++i) {
    const dash_ctx *c = sel[i].c;
    const int s = sel[i].b.stage;
    const int64_t bytes = (int64_t)align_up(sel[i].b.bytes, 16);   // stages are 256-byte multiples
    jobs[i] = FetchJob{c->hstage_dev[s], c->dstep[s], bytes, sel[i].b.report};
    max_bytes = std::max(max_bytes, bytes);
  }
  std::memcpy(tb->host + off_maps, maps.data(), sizeof(BlockMap) * maps.size());
  jobs[sel.size()] = FetchJob{tb->hdev + off_maps, tb->dev + off_maps, (int64_t)map_bytes, nullptr};
  const BlockMap *dmaps = (const BlockMap *)(tb->dev + off_maps);

  hipStream_t s0 = srv->stream;
  auto dev_fail = [&](int e) {
    srv->err = std::string("tick launch failed: ") + hipGetErrorString((hipError_t)e);
    return DASH_E_DEVICE;
  };
  if (int e = launch_fetch_list((const FetchJob *)tb->hdev, n_jobs, max_bytes, s0)) return dev_fail(e);
  for (const Sel &x : sel) {
    // the stage's pinned block is free again once the fetch has run
    if (hipEventRecord(x.c->stage_ev[x.b.stage], s0) != hipSuccess) return DASH_E_DEVICE;
    x.c->stage_used[x.b.stage] = true;
  }
  const bool timed = srv->prof_every > 0 && srv->stats.ticks % srv->prof_every == 0;
  if (timed && srv->prof_pending.size() > 4096) {
    if (hipStreamSynchronize(s0) != hipSuccess) return DASH_E_DEVICE;
    if (dash_status st = prof_fold(srv)) return st;
  }
  // the launches of one group run side by side: the first on the tick's
  // stream, the others on the extra streams after an event, joined back
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  for (size_t li = 0; li < launches.size(); ++li) {
    const Launch &L = launches[li];
    const bool first = li == 0 || launches[li - 1].group != L.group;
    const bool last = li + 1 == launches.size() || launches[li + 1].group != L.group;
    int slot = 0;   // position within the group
    for (size_t q = li; q > 0 && launches[q - 1].group == L.group; --q) ++slot;
    if (first && !last) {
      fork = take_event(srv);
      if (!fork || hipEventRecord(fork, s0) != hipSuccess) return DASH_E_DEVICE;
    }
    hipStream_t s = slot == 0 ? s0 : srv->aux[(slot - 1) % kAuxStreams];
    if (slot > 0 && hipStreamWaitEvent(s, fork, 0) != hipSuccess) return DASH_E_DEVICE;
    const BlockMap *m = dmaps + L.map_off;
    ProfRec pr{nullptr, nullptr, 0, L.bytes};
    if (timed) {
      char name[48];
      split_kernel_name(L.stage, L.rep, name, sizeof name);
      pr.entry = prof_entry(srv, name);
      pr.a = take_timing_event(srv);
      pr.b = take_timing_event(srv);
      if (!pr.a || !pr.b || hipEventRecord(pr.a, s) != hipSuccess) return DASH_E_DEVICE;
    }
    int e = 0;
    switch (L.stage) {
      case 0: e = launch_split_rows(L.rep, nullptr, m, L.n_blocks, s, L.lds); break;
      case 1: e = launch_split_rows_slow(L.rep, nullptr, m, L.n_blocks, s, L.lds); break;
      case 2:
        e = launch_split_solve(L.rep, nullptr, m, L.n_blocks, s, L.lds);
        if (!e) e = launch_split_solve_fix(nullptr, m, L.n_blocks, s, L.lds);
        break;
      case 3: e = launch_split_fsum(L.rep, nullptr, m, L.n_blocks, s, L.lds); break;
      case 4: e = launch_reduce_groups(nullptr, m, L.n_blocks, s); break;
      default: e = launch_finish_dev(L.rep, nullptr, m, L.n_blocks, 0, s, L.lds); break;
    }
    if (e) return dev_fail(e);
    if (timed) {
      if (hipEventRecord(pr.b, s) != hipSuccess) return DASH_E_DEVICE;
      srv->prof_pending.push_back(pr);
    }
    if (slot > 0) {
      hipEvent_t j = take_event(srv);
      if (!j || hipEventRecord(j, s) != hipSuccess) return DASH_E_DEVICE;
      joins.push_back(j);
    }
    if (last) {
      for (hipEvent_t j : joins) {
        if (hipStreamWaitEvent(s0, j, 0) != hipSuccess) return DASH_E_DEVICE;
        srv->ev_pool.push_back(j);   // the wait holds the state it was given
      }
      joins.clear();
      if (fork) srv->ev_pool.push_back(fork);
      fork = nullptr;
    }
  }
  hipStream_t s = s0;
  if (timed) srv->prof_ticks += 1;
  for (const Sel &x : sel) {
    if (!x.b.scored) continue;
    // anomaly scores of a stream that has them on (Definitions 1-2)
    PassArgs a = base_args_at(x.c, x.b.dblk);
    a.mode = 0;
    a.last_pass = 1;
    const int grid = std::min(std::max(x.b.n_items, 1), 2 * std::max(1, x.c->n_cu));
    if (int e = launch_slice_errors(a, x.c->anom, grid, s)) return dev_fail(e);
  }
  if (hipEventRecord(tb->ev, s) != hipSuccess) return DASH_E_DEVICE;
  tb->used = true;
  hipEvent_t done = take_event(srv);
  if (!done || hipEventRecord(done, s) != hipSuccess) return DASH_E_DEVICE;
  srv->ticks_in_flight.push_back(done);
  for (const Sel &x : sel) {
    account_update(x.c, x.b);
    srv->streams[x.sid].cuts.push_back(x.cut);
  }
  srv->stats.ticks += 1;
  srv->stats.launches += (int64_t)launches.size() + 1;
  srv->last_tick = now_us();
  return first;
}

bool has_requests(const dash_server *srv) {
  for (const Stream &st : srv->streams)
    if (st.state == kStateOpen && !st.requests.empty()) return true;
  return false;
}

// Open streams, and those with submitted rows that a tick could cut now.
void ready_count(const dash_server *srv, int *open, int *ready) {
  *open = *ready = 0;
  for (const Stream &st : srv->streams) {
    if (st.state != kStateOpen) continue;
    ++*open;
    if (!st.requests.empty() && st.ctx->initialized) ++*ready;
  }
}

void loop_main(dash_server *srv) {
  std::unique_lock<std::mutex> lk(srv->mu);
  while (!srv->stop) {
    dash_status s = collect(srv);
    if (s != DASH_OK && srv->loop_err == DASH_OK) srv->loop_err = s;
    // a tick starts when none is in flight, or beside the one in flight when
    // every open stream is ready (a stream's update costs work in proportion
    // to its slices whatever its rows, so under load ticks should carry every
    // stream; requests never wait for an idle device)
    const bool due = srv->tick_us <= 0 || now_us() - srv->last_tick >= (double)srv->tick_us;
    int open = 0, ready = 0;
    ready_count(srv, &open, &ready);
    const int inflight = (int)srv->ticks_in_flight.size();
    if (due && ready > 0 && (inflight == 0 || (inflight < kTicksInFlight && ready >= open))) {
      s = run_tick(srv, nullptr);
      if (s != DASH_OK && srv->loop_err == DASH_OK) srv->loop_err = s;
    }
    // wake on a submit, or soon to see completions
    const bool busy = !srv->ticks_in_flight.empty();
    srv->cv.wait_for(lk, std::chrono::microseconds(busy ? 20 : 500));
  }
}

}  // namespace

extern "C" {

dash_status dash_server_create(int32_t device, int64_t budget_bytes, dash_server **out) {
  if (!out || budget_bytes < 0) return DASH_E_INVALID_ARG;
  *out = nullptr;
  dash_server *srv = new (std::nothrow) dash_server();
  if (!srv) return DASH_E_OUT_OF_MEMORY;
  srv->device = device;
  srv->budget = budget_bytes;
  *out = srv;   // the device is first touched by the first admission
  return DASH_OK;
}

dash_status dash_server_stop(dash_server *srv) {
  if (!srv) return DASH_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->running) return DASH_OK;
    srv->stop = true;
  }
  srv->cv.notify_all();
  srv->loop.join();
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->running = false;
  srv->stop = false;
  return DASH_OK;
}

dash_status dash_server_destroy(dash_server *srv) {
  if (!srv) return DASH_OK;
  (void)dash_server_stop(srv);
  if (srv->stream) (void)hipStreamSynchronize(srv->stream);
  for (auto &st : srv->streams) {
    for (auto &q : st.requests)
      if (q.ready) srv->ev_pool.push_back(q.ready);
    if (st.ctx) dash_destroy(st.ctx);
  }
  free_tick_bufs(srv);
  for (auto &t : srv->tb)
    if (t.ev) (void)hipEventDestroy(t.ev);
  for (auto e : srv->ticks_in_flight) srv->ev_pool.push_back(e);
  for (auto e : srv->ev_pool) (void)hipEventDestroy(e);
  for (const ProfRec &p : srv->prof_pending) {
    srv->tev_pool.push_back(p.a);
    srv->tev_pool.push_back(p.b);
  }
  for (auto e : srv->tev_pool) (void)hipEventDestroy(e);
  for (auto a : srv->aux)
    if (a) (void)hipStreamDestroy(a);
  if (srv->stream) (void)hipStreamDestroy(srv->stream);
  delete srv;
  return DASH_OK;
}

dash_status dash_server_open(dash_server *srv, const dash_config *cfg, int32_t queue, int32_t *stream) {
  if (!srv || !cfg || !stream) return DASH_E_INVALID_ARG;
  int64_t fp = 0;
  if (dash_status s = dash_footprint(cfg, &fp)) return s;
  std::lock_guard<std::mutex> lk(srv->mu);
  const bool fits = srv->admit_queue.empty() && srv->used + fp <= srv->budget;
  if (!fits && (!queue || fp > srv->budget)) return DASH_E_CAPACITY;
  int32_t id = -1;
  for (size_t i = 0; i < srv->streams.size(); ++i)
    if (srv->streams[i].state == kStateClosed) {
      id = (int32_t)i;
      break;
    }
  if (id < 0) {
    if ((int)srv->streams.size() >= kMaxServed) return DASH_E_CAPACITY;
    srv->streams.emplace_back();
    id = (int32_t)srv->streams.size() - 1;
  }
  Stream &st = srv->streams[id];
  st = Stream{};
  st.cfg = *cfg;
  st.cfg.device = srv->device;
  st.footprint = fp;
  if (fits) {
    if (dash_status s = ensure_stream(srv)) {
      st = Stream{};
      return s;
    }
    st.cfg.stream = srv->stream;
    dash_ctx *ctx = nullptr;
    if (dash_status s = create_context(&st.cfg, srv->stream, true, &ctx)) {
      st = Stream{};
      return s;
    }
    st.ctx = ctx;
    st.state = kStateOpen;
    srv->used += fp;
  } else {
    st.state = kStateQueued;
    srv->admit_queue.push_back(id);
  }
  *stream = id;
  return DASH_OK;
}

dash_status dash_server_state(dash_server *srv, int32_t stream, int32_t *state) {
  if (!srv || !state) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  *state = (stream >= 0 && stream < (int32_t)srv->streams.size()) ? srv->streams[stream].state : kStateClosed;
  return DASH_OK;
}

dash_status dash_server_close(dash_server *srv, int32_t stream) {
  if (!srv) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (stream < 0 || stream >= (int32_t)srv->streams.size() || srv->streams[stream].state == kStateClosed)
    return DASH_E_INVALID_ARG;
  Stream &st = srv->streams[stream];
  if (st.state == kStateQueued) {
    srv->admit_queue.erase(std::find(srv->admit_queue.begin(), srv->admit_queue.end(), stream));
    st = Stream{};
    admit(srv);
    return DASH_OK;
  }
  // its updates in flight finish and are reported; unsent requests are dropped
  if (hipStreamSynchronize(srv->stream) != hipSuccess) return DASH_E_DEVICE;
  (void)collect(srv);
  for (auto &q : st.requests)
    if (q.ready) srv->ev_pool.push_back(q.ready);
  dash_destroy(st.ctx);
  srv->used -= st.footprint;
  st = Stream{};
  admit(srv);
  return DASH_OK;
}

dash_ctx *dash_server_context(dash_server *srv, int32_t stream) {
  if (!srv) return nullptr;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (stream < 0 || stream >= (int32_t)srv->streams.size()) return nullptr;
  return srv->streams[stream].ctx;
}

dash_status dash_server_submit(dash_server *srv, int32_t stream, int32_t n_groups, const int32_t *slice_id,
                               const int64_t *row_ptr, const float *rows, int32_t n_new, const int64_t *new_ptr,
                               const float *new_rows, void *producer, int64_t *request, int32_t *first_new_id) {
  if (!srv || n_groups < 0 || n_new < 0) return DASH_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (stream < 0 || stream >= (int32_t)srv->streams.size()) return DASH_E_INVALID_ARG;
  Stream &st = srv->streams[stream];
  if (st.state != kStateOpen || !st.ctx->initialized) {
    srv->err = "stream not open or not initialised";
    return DASH_E_BAD_STATE;
  }
  dash_ctx *c = st.ctx;
  if (st.K_sub < 0) st.K_sub = c->K_pending;
  Request q;
  int64_t n_rows = 0, ng = 0;
  if (n_new > 0) {
    if (!new_ptr || !new_rows) return DASH_E_INVALID_ARG;
    for (int32_t l = 0; l < n_new; ++l)
      if (new_ptr[l + 1] <= new_ptr[l] || new_ptr[l] < 0) return DASH_E_INVALID_ARG;
    if ((int64_t)st.K_sub + n_new > c->K_cap) return DASH_E_CAPACITY;
    q.new_ptr.assign(new_ptr, new_ptr + n_new + 1);
    q.new_rows = new_rows;
    n_rows += new_ptr[n_new] - new_ptr[0];
    ng += n_new;
  }
  if (n_groups > 0) {
    if (!slice_id || !row_ptr || row_ptr[0] < 0) return DASH_E_INVALID_ARG;
    for (int32_t g = 0; g < n_groups; ++g) {
      if (row_ptr[g + 1] < row_ptr[g]) return DASH_E_INVALID_ARG;
      if (slice_id[g] < 0 || slice_id[g] >= st.K_sub + n_new) return DASH_E_INVALID_ARG;
      if (row_ptr[g + 1] > row_ptr[g]) ++ng;
    }
    if (row_ptr[n_groups] > row_ptr[0] && !rows) return DASH_E_INVALID_ARG;
    q.slice_id.assign(slice_id, slice_id + n_groups);
    q.row_ptr.assign(row_ptr, row_ptr + n_groups + 1);
    q.rows = rows;
    n_rows += row_ptr[n_groups] - row_ptr[0];
  }
  if (n_rows > c->M_cap || ng > c->G_cap) return DASH_E_CAPACITY;
  if (producer) {
    q.ready = take_event(srv);
    if (!q.ready || hipEventRecord(q.ready, (hipStream_t)producer) != hipSuccess) return DASH_E_DEVICE;
  }
  q.id = srv->next_request++;
  q.t_submit = now_us();
  q.n_rows = n_rows;
  q.n_groups = ng;
  if (first_new_id) *first_new_id = st.K_sub;
  st.K_sub += n_new;
  if (request) *request = q.id;
  st.requests.push_back(std::move(q));
  lk.unlock();
  srv->cv.notify_one();
  return DASH_OK;
}

dash_status dash_server_tick(dash_server *srv, int32_t *launched) {
  if (!srv) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  return run_tick(srv, launched);
}

dash_status dash_server_poll(dash_server *srv, int32_t wait, dash_server_report *out, int32_t cap,
                             int32_t *n) {
  if (!srv || !n || cap < 0 || (cap > 0 && !out)) return DASH_E_INVALID_ARG;
  *n = 0;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (wait && !srv->running && srv->stream && hipStreamSynchronize(srv->stream) != hipSuccess)
    return DASH_E_DEVICE;
  dash_status st = srv->running ? DASH_OK : collect(srv);
  if (st == DASH_OK && srv->loop_err != DASH_OK) {
    st = srv->loop_err;
    srv->loop_err = DASH_OK;
  }
  while (!srv->done.empty() && *n < cap) {
    out[(*n)++] = srv->done.front();
    srv->done.pop_front();
  }
  return st;
}

dash_status dash_server_start(dash_server *srv, int32_t tick_us) {
  if (!srv || tick_us < 0) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->running) return DASH_E_BAD_STATE;
  srv->tick_us = tick_us;
  srv->stop = false;
  srv->running = true;
  try {
    srv->loop = std::thread(loop_main, srv);
  } catch (...) {
    srv->running = false;
    return DASH_E_OUT_OF_MEMORY;
  }
  return DASH_OK;
}

dash_status dash_server_drain(dash_server *srv, int32_t timeout_ms) {
  if (!srv) return DASH_E_INVALID_ARG;
  const double t_end = now_us() + 1e3 * (double)timeout_ms;
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      if (!srv->stream) return DASH_OK;   // nothing was ever admitted
      if (!srv->running) {
        // no loop: tick until every request is in an update, then wait
        while (has_requests(srv)) {
          int32_t n = 0;
          if (dash_status s = run_tick(srv, &n)) return s;
          if (n == 0 && hipStreamSynchronize(srv->stream) != hipSuccess) return DASH_E_DEVICE;
          (void)collect(srv);
        }
        if (hipStreamSynchronize(srv->stream) != hipSuccess) return DASH_E_DEVICE;
        return collect(srv);
      }
      bool idle = !has_requests(srv) && srv->ticks_in_flight.empty();
      for (const Stream &st : srv->streams) idle = idle && st.cuts.empty();
      if (idle) return DASH_OK;
    }
    if (timeout_ms >= 0 && now_us() > t_end) return DASH_E_BAD_STATE;
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
}

dash_status dash_server_get_stats(dash_server *srv, dash_server_stats *out) {
  if (!srv || !out) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  out->budget = srv->budget;
  out->used = srv->used;
  out->queued = (int32_t)srv->admit_queue.size();
  int32_t open = 0;
  for (const Stream &st : srv->streams) open += st.state == kStateOpen ? 1 : 0;
  out->open = open;
  return DASH_OK;
}

dash_status dash_server_profile(dash_server *srv, int32_t every) {
  if (!srv || every < 0) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stream && hipStreamSynchronize(srv->stream) != hipSuccess) return DASH_E_DEVICE;
  if (dash_status s = prof_fold(srv)) return s;
  srv->prof_every = every;
  srv->prof_stats.clear();
  srv->prof_ticks = 0;
  return DASH_OK;
}

dash_status dash_server_profile_read(dash_server *srv, dash_kernel_stat *out, int32_t cap, int32_t *n,
                                     int64_t *ticks) {
  if (!srv || !n || cap < 0 || (cap > 0 && !out)) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stream && hipStreamSynchronize(srv->stream) != hipSuccess) return DASH_E_DEVICE;
  if (dash_status s = prof_fold(srv)) return s;
  *n = (int32_t)std::min<size_t>(srv->prof_stats.size(), (size_t)cap);
  for (int32_t i = 0; i < *n; ++i) out[i] = srv->prof_stats[i];
  if (ticks) *ticks = srv->prof_ticks;
  return DASH_OK;
}

const char *dash_server_last_error(dash_server *srv) {
  if (!srv) return "";
  std::lock_guard<std::mutex> lk(srv->mu);
  return srv->err.c_str();
}

}  // extern "C"
