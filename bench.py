"""Benchmark of the streaming PARAFAC2 update on one MI355X.

Default (--workload serve): the serving workload in mixed precision -- 64
independent streams (J ~ U{32,64,128,256}, R ~ U{8,16,32}, K0 ~ U{500..5000},
lambda = 0.95), rows arriving as Poisson processes of 2000 rows/s per stream
to Zipf(1.2)-popular slices plus 2 new slices/s of U{1..60} rows, cut into
25 ms requests, served by one DashServer (200 GB admission budget) whose loop
thread batches every stream's pending requests into one tick.  A "step" is
one tick.  Three phases on the same streams: an open-loop replay at the
arrival times (p50/p99 latency from a request's submit to its update's
commit), a closed-loop run with eight requests in flight per stream (the
headline rows/s: every row of the phase over its wall time, inputs resident
in HBM), and a 2 GB-budget run in which streams wait for admission.  The
sampled streams' per-update fits are checked against the FP64 oracle fed the
same cuts, which is also timed on the host (the CPU baseline).

--workload mid | batch_r10 | batch_r20 | precision: one stream (one context),
a "step" is one update over a batch resident in HBM; warm-up updates run
blocking and are checked against the oracle, the timed updates run back to
back.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ingested rows/sec at fit within 1e-3 of FP64 oracle; p50/p99 update latency"
HBM_PEAK_GBS = 8000.0


WORKLOAD_TEXT = {
    "mid": "mid dual-way stream: K0=2000 slices, I_k lognormal(median 800, clip 100..4000), "
           "J=88, R=10, +U{1..20} rows/slice and +20 slices per update, lambda=0.95, 1 ALS pass",
    "batch_r10": "batching stream: K0=20000 slices, J=128, R=10, per update truncated-Zipf(1.2) rows per slice "
                 "(0..200, mean 21.4) and 20 new slices, lambda=0.95, 1 ALS pass",
    "batch_r20": "batching stream: K0=20000 slices, J=128, R=20, per update truncated-Zipf(1.2) rows per slice "
                 "(0..200, mean 21.4) and 20 new slices, lambda=0.95, 1 ALS pass",
    "precision": "precision stream: K0=20000 slices, J=256, R=32, Student-t(3) rows and noise, column scales "
                 "10^U[-3,3], Zipf(1.2) arrivals, lambda=0.95, 1 ALS pass",
}


def state_entry_bytes(words):
    """Bytes per Y_k and per D_k entry: float32 (words = 1), or the mixed
    path's float32 word plus its compensation word (BF16 for Y, float32 for
    D)."""
    return (4, 4) if words == 1 else (6, 8)


def algorithmic_bytes(M, K, K_t, J, R, words=1):
    """Bytes one update pass must move (the per-pass model of the design notes):
    new rows read, U_new written, every slice's Y_k (value words) / D_k / n_k /
    W row read, touched slices' Y_k / D_k / n_k written, every W row written.
    `words` = 2: the mixed path, whose touched slices move their compensation
    words too (state_entry_bytes)."""
    yb, db = state_entry_bytes(words)
    return (M * J * 4 + M * R * 4
            + K * (R * J * 4 + R * R * db + 8 + R * 8)
            + K_t * (R * J * yb + R * R * db + 8)
            + K * R * 8)


KERNEL_SOURCES = ("dash_dev.h", "dash_math.h", "dash_tiles.h", "dash_kernels.hip", "dash_split.hip")


def rows_stage_bytes(M, K_t, J, R, words=1):
    """Bytes the split sweep's row stage must move: the new rows read, U_new
    written, and each touched slice's Y_k / D_k read and the folded ones
    written (bytes per entry as state_entry_bytes), its n_k read and written
    and its c_k written."""
    yb, db = state_entry_bytes(words)
    return M * J * 4 + M * R * 4 + K_t * (2 * (R * J * yb + R * R * db) + 16 + R * 8)


def _source_digest():
    """SHA-256 over the device sources of the update kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_18376_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(kernel, workload, algorithmic_per_launch=None):
    """HBM bytes per dispatch of `kernel` from the committed byte-counter
    summary (profiles/<kernel>_<workload>_counters.md): the summary's
    traffic-to-algorithmic ratio times this run's algorithmic bytes per launch
    when given (a serving launch's size depends on the tick), else its bytes
    per dispatch; None when that summary is missing or was taken on a
    different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != _source_digest():
        return None
    try:
        if algorithmic_per_launch:
            return float(vals["traffic_over_algorithmic"]) * float(algorithmic_per_launch)
        return float(vals["traffic_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed updates (mid: 90, batch/precision: 20); serve: ignored (the phases are timed)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up updates (mid: 10, others: 3)")
    ap.add_argument("--workload", default="serve", choices=["serve", "mid", "batch_r10", "batch_r20", "precision"],
                    help="serve (default) is the serving workload; the others run one stream (the batching and "
                         "precision ones with shorter initial slices: the per-update cost does not depend on them)")
    ap.add_argument("--precision", default=None, choices=["fp32", "mixed"],
                    help="default: mixed for serve, fp32 otherwise")
    ap.add_argument("--open-seconds", type=float, default=8.0, help="serve: open-loop replay length")
    ap.add_argument("--closed-seconds", type=float, default=4.0,
                    help="serve: stream time replayed closed-loop after the open-loop phase")
    ap.add_argument("--streams", type=int, default=64, help="serve: number of streams")
    ap.add_argument("--closed-depth", type=int, default=8, help="serve: requests in flight per stream, closed loop")
    ap.add_argument("--no-queue", action="store_true", help="serve: skip the 2 GB admission-queue run")
    ap.add_argument("--study", default=None, choices=["cycle", "lambda", "static", "lagged"],
                    help="instead of the benchmark: time per update against the update cycle, the errors against "
                         "lambda, the streaming update against a static recompute, or the exact statistics "
                         "against the lagged recursions (prints its own JSON line)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="N > 0: the warm-up updates try every launch schedule N times and keep the fastest")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: replay each update's launches from one HIP graph; 0: launch directly")
    ap.add_argument("--sample-every", type=int, default=10,
                    help="time the kernels of every N-th update with HIP events (events perturb "
                         "the launches they bracket, so the others run undisturbed)")
    ap.add_argument("--oracle-seconds", type=float, default=25.0,
                    help="bound on the FP64 oracle replay (CPU baseline and fit check)")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed region, one plain device copy of this many MiB "
                         "(reference dispatch for hardware byte counters)")
    ap.add_argument("--pcie", action="store_true",
                    help="single stream: after the timed region, the same number of further updates whose rows "
                         "are first copied from pinned host memory (reported as pcie_inclusive)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the update would shard by slice with one all-reduce of F, G per pass).", file=sys.stderr)
        sys.exit(2)

    if args.study:
        return study_main(args)
    if args.workload == "serve":
        if args.precision is None:
            args.precision = "mixed"
        return serve_main(args)
    if args.precision is None:
        args.precision = "fp32"

    import torch
    from paper_2305_18376_amd.dash import Dash
    from paper_2305_18376_amd.synth import make_workload

    big = args.workload != "mid"
    W_ = args.warmup if args.warmup is not None else (3 if big else 10)
    if args.autotune > 0:
        W_ = max(W_, 8 * args.autotune + 2)   # at most 8 candidate schedules
    K_ = args.steps if args.steps is not None else (20 if big else 90)
    n_total = W_ + K_
    n_pcie = K_ if args.pcie else 0
    if big:
        # initial slices of log-normal length median 24 (the update cost depends on K, not on them)
        wl = make_workload(args.workload, n_steps=n_total + n_pcie, median=24, lo=1, hi=200)
        wl.init_len = np.maximum(wl.init_len, wl.R + 1)
    else:
        wl = make_workload("mid", n_steps=max(100, n_total + n_pcie))
    t0 = time.time()
    ptr, X, U = wl.init_data(want_u=True)
    batches = [wl.step(s) for s in range(1, n_total + 1)]
    pcie_batches = [wl.step(s) for s in range(n_total + 1, n_total + n_pcie + 1)]
    t_gen = time.time() - t0

    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    from paper_2305_18376_amd.dash import PREC_FP32, PREC_MIXED
    max_rows = max(64 * 1024, max(b.M for b in batches + pcie_batches) + 1)
    max_groups = max(8192, max(b.n_groups + b.n_new for b in batches + pcie_batches) + 1)
    g = Dash(wl.J, wl.R, lam=wl.lam, n_iter=wl.n_iter, max_slices=wl.K_max + 64,
             max_rows=max_rows, max_groups=max_groups,
             precision=PREC_MIXED if args.precision == "mixed" else PREC_FP32)
    Xd, Ud = to(X), to(U)
    g.init_from_factors(ptr, Xd, Ud, to(wl.W[: wl.K0]), to(wl.V))
    g.graph(bool(args.graph))
    if args.autotune > 0:
        g.autotune(args.autotune)
    del Xd, Ud
    dbat = []
    for b in batches:
        dbat.append((b.row_ids, b.row_ptr, to(b.rows), b.new_ptr, to(b.new_rows)))
    torch.cuda.synchronize()

    def stage(i):
        rid, rptr, rows, nptr, nrows = dbat[i]
        g.ingest_rows(rid, rptr, rows)
        g.ingest_slices(nptr, nrows)

    # warm-up: blocking updates, fits kept for the oracle check
    gpu_fits = []
    for i in range(W_):
        stage(i)
        gpu_fits.append(g.update()["fit"])

    # timed region: K updates enqueued back to back, bracketed by a full
    # synchronisation on both sides (the library works on its own stream, so
    # the interval is taken on the host clock: whole-job time, host included)
    g.profile(args.sample_every)
    g.spans(True)   # per-update device spans with timing-only events (p50 / p99)
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    for i in range(K_):
        stage(W_ + i)
        g.update_async()
    last = g.wait()
    torch.cuda.synchronize()
    h1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    if args.copy_mb > 0:
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dev_ms = (h1 - h0) * 1e3
    lat = g.spans_read()
    g.spans(False)
    rows = sum(batches[W_ + i].M for i in range(K_))
    value = rows / (dev_ms / 1e3)

    # algorithmic bytes of the sampled (event-timed) passes; update index s = W_ + i + 1
    # the dominant kernel: the fused sweep (wave variant: the whole update's
    # bytes) or the split sweep's row stage (its own bytes); its launches are
    # the "pass" events of the sampled updates
    sched = g.schedule()
    split = sched["variant"] != 0
    kernel = "k_pass_wave" if not split else "k_rows"
    words = 2 if args.precision == "mixed" else 1
    bytes_pass, bytes_all, n_sampled = 0, 0, 0
    for i in range(K_):
        b = batches[W_ + i]
        s = W_ + i + 1
        nb = algorithmic_bytes(b.M, wl.K_at(s), b.n_groups + b.n_new, wl.J, wl.R, words=words) * wl.n_iter
        bytes_all += nb
        if args.sample_every > 0 and s % args.sample_every == 0:
            bytes_pass += (rows_stage_bytes(b.M, b.n_groups + b.n_new, wl.J, wl.R, words) * wl.n_iter
                           if split else nb)
            n_sampled += wl.n_iter
    pass_ms = prof["pass_ms"]
    achieved = bytes_pass / (pass_ms / 1e3) / 1e9 if pass_ms > 0 else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": K_,
        "warmup": W_,
        "ms_per_step": dev_ms / K_,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16-mfma/f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "K_final": wl.K_at(n_total), "rows_timed": rows},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "note": "per-update device span, back-to-back updates"},
        "kernel_us_avg": {k: (1e3 * prof[k + "_ms"] / prof[k + "_launches"]) if prof[k + "_launches"] else None
                          for k in ("pass", "solve", "reduce", "commit", "upload")},
        "launch": "hip graph (node parameters rewritten per update)" if args.graph else "direct",
        "schedule": sched,
        "kernel_timing": f"HIP events around the launches of every {args.sample_every}-th update "
                         f"({prof['updates']} sampled)",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
                     "kernel": kernel, "algorithmic_bytes_per_step": bytes_all / K_,
                     "algorithmic_bytes_per_launch": bytes_pass / n_sampled if n_sampled else None,
                     "avg_launch_us": 1e3 * pass_ms / n_sampled if n_sampled else None,
                     "launches": n_sampled,
                     "timing": f"HIP events around the row stage (and its deferred-slice launch) of every "
                               f"{args.sample_every}-th update" if split else
                               f"HIP events around the sweep of every {args.sample_every}-th update"},
        "final_fit": last["fit"],
        "gen_s": t_gen,
    }

    tr = counter_traffic(kernel, args.workload + ("" if args.precision == "fp32" else "_mixed"),
                         out["roofline"].get("algorithmic_bytes_per_launch"))
    out["roofline"]["traffic"] = tr
    if pcie_batches:
        out["pcie_inclusive"] = pcie_phase(g, pcie_batches, dev)
    if not args.no_oracle:
        out["fit_check"], out["cpu_baseline"] = oracle_leg(wl, ptr, X, U, batches, gpu_fits, last["fit"],
                                                           args.oracle_seconds)
    print(json.dumps(out), flush=True)


def oracle_leg(wl, ptr, X, U, batches, gpu_fits, gpu_final_fit, budget_s):
    """The FP64 oracle replays the same stream from the start (single-threaded
    BLAS) for at most budget_s seconds of update time: its fits are compared
    with the GPU's blocking warm-up updates and, when the replay reaches the end
    of the stream, with the GPU's final fit; its update rate is the CPU
    baseline."""
    from threadpoolctl import threadpool_limits
    from oracle.dash_oracle import DashOracle
    with threadpool_limits(limits=1):
        o = DashOracle(wl.J, wl.R, wl.lam, n_iter=wl.n_iter)
        slices = [X[ptr[k]:ptr[k + 1]] for k in range(wl.K0)]
        o.init_from_factors(slices, [U[ptr[k]:ptr[k + 1]] for k in range(wl.K0)], wl.W[: wl.K0], wl.V)
        fits, secs, rows = [], 0.0, 0
        for b in batches:
            t = time.perf_counter()
            r = o.update(b.groups(), b.new_slices())
            secs += time.perf_counter() - t
            rows += b.M
            fits.append(r.fit)
            if secs >= budget_s:
                break
    n = len(fits)
    d = [abs(a - b) for a, b in zip(gpu_fits, fits)]
    complete = n == len(batches)
    if complete:
        d.append(abs(gpu_final_fit - fits[-1]))
    fit_check = {"updates_compared": len(d), "oracle_updates": n, "final_fit_compared": complete,
                 "max_abs_dfit": max(d) if d else None, "oracle_fit_last": fits[-1] if fits else None,
                 "within_1e-3": bool(d and max(d) <= 1e-3)}
    cpu = {"value": rows / secs if secs > 0 else None, "unit": "rows/s", "cores": 1, "kind": "oracle",
           "sample": f"updates 1..{n} of the same stream replayed by the FP64 numpy oracle "
                     f"(1 BLAS thread): {rows} rows in {secs:.1f} s"}
    return fit_check, cpu


SERVE_WORKLOAD = ("serving: {n} streams, J~U{{32,64,128,256}}, R~U{{8,16,32}}, K0~U{{500..5000}} slices "
                  "(initial slices log-normal median 24, clip [R+1,200], shorter than the median-500 law: the "
                  "update cost depends on the slice count, not on the rows that built them), lambda=0.95, "
                  "Poisson 2000 rows/s/stream to Zipf(1.2)-popular slices + Poisson 2 new slices/s of U{{1..60}} "
                  "rows, 25 ms requests, admission budget 200 GB; open loop {to:g} s at the arrival times, closed "
                  "loop over the next {tc:g} s of stream time with {qd} requests in flight per stream")


def _merge_cut(st, reqs):
    """The rows of several requests of one stream as one update (ingest order)."""
    groups, news = [], []
    for q in reqs:
        for l in range(len(q.new_ptr) - 1):
            news.append(st.new_rows[q.n0 + q.new_ptr[l]:q.n0 + q.new_ptr[l + 1]])
        for g in range(len(q.row_ids)):
            groups.append((int(q.row_ids[g]), st.rows[q.r0 + q.row_ptr[g]:q.r0 + q.row_ptr[g + 1]]))
    return groups, news


def serve_oracle_leg(streams, cuts, gpu_fits, sample, budget_s):
    """The FP64 oracle replays sampled streams with the server's cuts: its fit
    after every update is compared with the update's reported fit; the replay
    (one BLAS thread, then all threads) is the CPU baseline."""
    import platform
    from threadpoolctl import threadpool_limits
    from oracle.dash_oracle import DashOracle
    res = {"streams": [], "max_abs_dfit": 0.0, "updates_compared": 0}
    cpu = {}
    for label, limit, share in (("1 thread", 1, 0.6), ("all threads", None, 0.4)):
        rows_tot, secs_tot = 0, 0.0
        for i in sample:
            st = streams[i]
            with threadpool_limits(limits=limit):
                o = DashOracle(st.J, st.R, st.lam)
                p = st.init_ptr
                o.init_from_factors([st.init_X[p[k]:p[k + 1]] for k in range(st.K0)],
                                    [st.init_U[p[k]:p[k + 1]] for k in range(st.K0)], st.W[: st.K0], st.V)
                secs, n = 0.0, 0
                for c, f in zip(cuts[i], gpu_fits[i]):
                    groups, news = _merge_cut(st, c)
                    t = time.perf_counter()
                    r = o.update(groups, news)
                    secs += time.perf_counter() - t
                    rows_tot += sum(x.shape[0] for _, x in groups) + sum(x.shape[0] for x in news)
                    n += 1
                    if limit == 1:
                        d = abs(r.fit - f)
                        res["max_abs_dfit"] = max(res["max_abs_dfit"], d)
                        res["updates_compared"] += 1
                    if secs >= budget_s * share / len(sample):
                        break
            secs_tot += secs
            if limit == 1:
                res["streams"].append({"stream": i, "J": st.J, "R": st.R, "K0": st.K0, "updates": n})
        cores = limit if limit else (os.cpu_count() or 1)
        cpu[label] = {"value": rows_tot / secs_tot if secs_tot > 0 else None, "threads": cores,
                      "rows": rows_tot, "seconds": secs_tot}
    res["within_1e-3"] = bool(res["updates_compared"] > 0 and res["max_abs_dfit"] <= 1e-3)
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    best = cpu["all threads"]
    cpu_line = {"value": best["value"], "unit": "rows/s", "cores": best["threads"], "kind": "oracle",
                "cpu_model": model, "nproc": os.cpu_count(), "single_thread": cpu["1 thread"]["value"],
                "sample": f"the FP64 numpy oracle replaying the first updates of streams {list(sample)} with the "
                          f"server's cuts: {cpu['1 thread']['rows']} rows in {cpu['1 thread']['seconds']:.1f} s on 1 "
                          f"BLAS thread, {best['rows']} rows in {best['seconds']:.1f} s on {best['threads']}"}
    return res, cpu_line


def _json_default(o):
    if isinstance(o, np.generic):
        return o.item()
    raise TypeError(type(o).__name__)


def serve_main(args):
    import torch
    from paper_2305_18376_amd.dash import DashServer, PREC_FP32, PREC_MIXED
    from paper_2305_18376_amd.synth import serving_streams
    prec = PREC_MIXED if args.precision == "mixed" else PREC_FP32
    T_open, T_closed, n_streams = args.open_seconds, args.closed_seconds, args.streams
    t0 = time.time()
    streams = serving_streams(n_streams, seconds=T_open + T_closed)
    t_gen = time.time() - t0
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    M_CAP, G_CAP = 16384, 8192
    kw_of = lambda st: dict(lam=st.lam, precision=prec, max_slices=st.K_max + 8, max_rows=M_CAP, max_groups=G_CAP)
    srv = DashServer(200 << 30)
    sids, drows, dnew = [], [], []
    for st in streams:
        sid = srv.open(st.J, st.R, **kw_of(st))
        srv.context(sid).init_from_factors(st.init_ptr, to(st.init_X), to(st.init_U), to(st.W[: st.K0]),
                                           to(st.V))
        sids.append(sid)
        drows.append(to(st.rows))
        dnew.append(to(st.new_rows))
    torch.cuda.synchronize()
    idx_of_sid = {sid: i for i, sid in enumerate(sids)}
    req_of = {}          # (sid, request id) -> request index
    sent = [[] for _ in streams]   # request ids in submit order
    reports = []

    # every request's C arguments, prepared before the timed phases (the row
    # buffers stay alive in drows / dnew for the whole run)
    import ctypes as C
    from paper_2305_18376_amd.dash import lib as _lib
    L, hsrv = _lib(), srv._h
    cargs = []
    for i, st in enumerate(streams):
        rb, nb, J4 = drows[i].data_ptr(), dnew[i].data_ptr(), 4 * st.J
        per = []
        for q in st.requests:
            ng, nn = len(q.row_ids), len(q.new_ptr) - 1
            per.append((sids[i], ng, q.row_ids.ctypes.data if ng else None, q.row_ptr.ctypes.data if ng else None,
                        rb + q.r0 * J4 if ng else None, nn, q.new_ptr.ctypes.data if nn else None,
                        nb + q.n0 * J4 if nn else None))
        cargs.append(per)
    rid_box = C.c_int64()
    rid_ref = C.byref(rid_box)

    def submit(i, qi):
        a = cargs[i][qi]
        st = L.dash_server_submit(hsrv, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], None, rid_ref, None)
        if st != 0:
            raise RuntimeError(f"dash_server_submit: status {st}")
        rid = rid_box.value
        req_of[(sids[i], rid)] = qi
        sent[i].append(rid)
        return rid

    def collect():
        got = srv.poll()
        reports.extend(got)
        return got

    # warm-up: the first 0.2 s of every stream, then drain
    srv.start(0)
    warm = sorted((q.t, i, qi) for i, st in enumerate(streams) for qi, q in enumerate(st.requests) if q.t < 0.2)
    for _, i, qi in warm:
        submit(i, qi)
    srv.drain(120000)
    collect()
    n_warm_reports = len(reports)

    # open loop: each request submitted at its arrival time
    sched = sorted((q.t, i, qi) for i, st in enumerate(streams) for qi, q in enumerate(st.requests)
                   if 0.2 <= q.t < T_open)
    st_warm = srv.stats()
    lag = []
    h0 = time.perf_counter()
    t_base = sched[0][0] if sched else 0.0
    last_poll = h0
    for t, i, qi in sched:
        target = h0 + (t - t_base)
        now = time.perf_counter()
        if target > now:
            time.sleep(target - now)
        lag.append(time.perf_counter() - target)
        submit(i, qi)
        if time.perf_counter() - last_poll > 0.005:
            collect()
            last_poll = time.perf_counter()
    srv.drain(120000)
    h1 = time.perf_counter()
    collect()
    open_reps = reports[n_warm_reports:]
    open_lat = np.array([r["latency_us"] for r in open_reps]) / 1e3 if open_reps else np.zeros(1)
    open_rows = sum(r["rows"] for r in open_reps)
    st_open = srv.stats()

    # closed loop: QD requests in flight per stream, profiled every N-th tick
    todo = [[qi for qi, q in enumerate(st.requests) if q.t >= T_open] for st in streams]
    nxt = [0] * n_streams
    inflight = [0] * n_streams
    done_upto = [0] * n_streams      # index into sent[i] of the first request not yet consumed
    n_before = len(reports)
    srv.profile(args.sample_every)
    h2 = time.perf_counter()
    QD = args.closed_depth
    for i in range(n_streams):
        while inflight[i] < QD and nxt[i] < len(todo[i]):
            submit(i, todo[i][nxt[i]])
            nxt[i] += 1
            inflight[i] += 1
    remaining = sum(len(t) for t in todo)
    consumed = 0
    while consumed < remaining:
        got = collect()
        if not got:
            time.sleep(50e-6)
            continue
        for r in got:
            i = idx_of_sid[r["stream"]]
            while done_upto[i] < len(sent[i]) and sent[i][done_upto[i]] <= r["last_request"]:
                if req_of[(sids[i], sent[i][done_upto[i]])] >= (todo[i][0] if todo[i] else 1 << 60):
                    inflight[i] -= 1
                    consumed += 1
                done_upto[i] += 1
            while inflight[i] < QD and nxt[i] < len(todo[i]):
                submit(i, todo[i][nxt[i]])
                nxt[i] += 1
                inflight[i] += 1
    h3 = time.perf_counter()
    closed_reps = reports[n_before:]
    closed_rows = sum(r["rows"] for r in closed_reps)
    st_closed = srv.stats()
    kstats, kticks = srv.profile_read()
    srv.profile(0)
    srv.stop()
    if args.copy_mb > 0:
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    all_committed = all(r["committed"] == 1 for r in reports)

    # the sampled streams' cuts and fits, for the oracle
    sample = sorted(range(n_streams), key=lambda i: streams[i].K0 * streams[i].J * streams[i].R)[:2]
    cuts, fits = {}, {}
    for i in sample:
        mine = sorted((r for r in reports if r["stream"] == sids[i]), key=lambda r: r["step"])
        c, k, prev = [], 0, 0
        for r in mine:
            grp = []
            while k < len(sent[i]) and sent[i][k] <= r["last_request"]:
                grp.append(streams[i].requests[req_of[(sids[i], sent[i][k])]])
                k += 1
            c.append(grp)
        cuts[i], fits[i] = c, [r["fit"] for r in mine]

    # dominant kernel of the closed loop
    kern = max(kstats, key=lambda e: e["ms"]) if kstats else None
    roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None}
    if kern and kern["ms"] > 0:
        ach = kern["bytes"] / (kern["ms"] / 1e3) / 1e9
        roof.update(achieved=ach, frac=ach / HBM_PEAK_GBS, kernel=kern["name"],
                    avg_launch_us=1e3 * kern["ms"] / kern["launches"], launches=kern["launches"],
                    algorithmic_bytes_per_launch=kern["bytes"] / kern["launches"],
                    timing=f"HIP events on the server's stream around every launch of every "
                           f"{args.sample_every}-th tick of the closed loop ({kticks} ticks timed)")
        roof["traffic"] = counter_traffic(kern["name"].split("<")[0], "serve_mixed" if prec else "serve",
                                          kern["bytes"] / kern["launches"])
    ticks_closed = st_closed["ticks"] - st_open["ticks"]
    out = {
        "metric": METRIC,
        "value": closed_rows / (h3 - h2),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": ticks_closed,
        "warmup": st_open["ticks"],
        "ms_per_step": 1e3 * (h3 - h2) / max(ticks_closed, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-mfma/f32" if prec == PREC_MIXED else "f32",
        "data": "synthetic",
        "config": {"workload": SERVE_WORKLOAD.format(n=n_streams, to=T_open, tc=T_closed, qd=args.closed_depth),
                   "streams": n_streams, "rows_closed_loop": closed_rows,
                   "updates_closed_loop": len(closed_reps)},
        "latency_ms": {"p50": float(np.percentile(open_lat, 50)), "p99": float(np.percentile(open_lat, 99)),
                       "note": "open loop at the arrival times: submit of an update's first request to its "
                               "commit seen by the server's loop thread"},
        "open_loop": {"rows_per_s": open_rows / (h1 - h0), "offered_rows_per_s": 2000.0 * n_streams,
                      "updates": len(open_reps), "ticks": st_open["ticks"] - st_warm["ticks"],
                      "submit_lag_ms_p99": 1e3 * float(np.percentile(lag, 99)) if lag else None},
        "closed_loop": {"latency_ms_p50": float(np.percentile([r["latency_us"] for r in closed_reps], 50)) / 1e3,
                        "latency_ms_p99": float(np.percentile([r["latency_us"] for r in closed_reps], 99)) / 1e3,
                        "launches_per_tick": (st_closed["launches"] - st_open["launches"]) / max(ticks_closed, 1)},
        "kernels_closed_loop": [{"name": e["name"], "avg_us": 1e3 * e["ms"] / e["launches"],
                                 "gbps": e["bytes"] / (e["ms"] / 1e3) / 1e9 if e["ms"] > 0 else None}
                                for e in sorted(kstats, key=lambda e: -e["ms"])],
        "roofline": roof,
        "all_committed": all_committed,
        "gen_s": t_gen,
    }
    srv.close()
    del drows, dnew
    torch.cuda.synchronize()
    if not args.no_queue:
        out["queueing"] = serve_queueing(streams[: n_streams], prec, kw_of, to)
    if not args.no_oracle:
        out["fit_check"], out["cpu_baseline"] = serve_oracle_leg(streams, cuts, fits, sample, args.oracle_seconds)
    print(json.dumps(out, default=_json_default), flush=True)


def pcie_phase(g, pcie_batches, dev):
    """Rows handed over from host memory: each update's rows are copied from
    pinned host buffers to the device on torch's null stream, then ingested
    and the update enqueued; the library's blocking stream follows the null
    stream, so copy and update run in turn (no overlap).  Whole-job rows/s
    over these updates, between two synchronisations."""
    import torch
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).pin_memory()
    host = [(pin(b.rows), pin(b.new_rows)) for b in pcie_batches]
    devb = [(torch.empty(hr.shape, dtype=torch.float32, device=dev),
             torch.empty(hn.shape, dtype=torch.float32, device=dev)) for hr, hn in host]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, (hr, hn), (dr, dn) in zip(pcie_batches, host, devb):
        dr.copy_(hr, non_blocking=True)
        dn.copy_(hn, non_blocking=True)
        g.ingest_rows(b.row_ids, b.row_ptr, dr)
        g.ingest_slices(b.new_ptr, dn)
        g.update_async()
    g.wait()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rows = sum(b.M for b in pcie_batches)
    nbytes = sum(hr.numel() * 4 + hn.numel() * 4 for hr, hn in host)
    return {"rows_per_s": rows / (t1 - t0), "updates": len(pcie_batches),
            "h2d_bytes_per_update": nbytes / len(pcie_batches), "ms_per_update": 1e3 * (t1 - t0) / len(pcie_batches),
            "note": "rows copied from pinned host memory on the null stream before each update; copy and "
                    "update run in turn"}


def serve_queueing(streams, prec, kw_of, to, budget=2 << 30, windows=10):
    """Every stream asks for admission under a 2 GB budget; admitted streams
    are initialised, serve their first requests and close, which admits the
    ones waiting."""
    from paper_2305_18376_amd.dash import DashServer
    srv = DashServer(budget)
    t0 = time.perf_counter()
    sids = [srv.open(st.J, st.R, queue=True, **kw_of(st)) for st in streams]
    admitted0 = sum(1 for s in sids if srv.state(s) == srv.OPEN)
    srv.start(0)
    served, peak_used, updates = set(), 0, 0
    while len(served) < len(streams):
        opened = [i for i, s in enumerate(sids) if i not in served and srv.state(s) == srv.OPEN]
        if not opened:
            break
        keep = []
        for i in opened:
            st = streams[i]
            srv.context(sids[i]).init_from_factors(st.init_ptr, to(st.init_X), to(st.init_U),
                                                   to(st.W[: st.K0]), to(st.V))
            rows = to(st.rows)
            newr = to(st.new_rows) if st.new_rows.shape[0] else None
            keep.append((rows, newr))
            for q in st.requests[:windows]:
                kw = {}
                if q.n1 > q.n0:
                    kw = dict(new_ptr=q.new_ptr, new_rows=newr[q.n0:q.n1])
                if q.r1 > q.r0:
                    srv.submit(sids[i], q.row_ids, q.row_ptr, rows[q.r0:q.r1], **kw)
                else:
                    srv.submit(sids[i], **kw)
        srv.drain(120000)
        updates += len(srv.poll())
        peak_used = max(peak_used, srv.stats()["used"])
        for i in opened:
            srv.close_stream(sids[i])
            served.add(i)
        del keep
    srv.stop()
    wall = time.perf_counter() - t0
    srv.close()
    return {"budget_gb": budget / 2 ** 30, "streams": len(streams), "admitted_at_open": admitted0,
            "queued_at_open": len(streams) - admitted0, "served": len(served), "updates": updates,
            "peak_used_gb": peak_used / 2 ** 30, "wall_s": wall}


def study_main(args):
    """Synthetic studies of the update (the paper's update-cycle scalability,
    lambda sensitivity and the static-recompute comparison, on planted data of
    the mid workload's shape: J = 88, R = 10, K0 = 2000)."""
    import torch
    from paper_2305_18376_amd.dash import Dash
    from paper_2305_18376_amd.synth import make_workload
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

    def mean_slice_error(X, U, S, W, V):
        # mean over slices of each slice's mean absolute error |X - U S_k V^T|
        r = np.abs(X - (U * W[S]) @ V.T).mean(axis=1)
        cnt = np.bincount(S)
        tot = np.bincount(S, weights=r)
        has = cnt > 0
        return float(np.mean(tot[has] / cnt[has]))

    def stream(wl, lam, n_steps, cycle=None, scores=False, global_err=None, lagged=False):
        from paper_2305_18376_amd.dash import STATS_EXACT, STATS_LAGGED
        ptr, X, U = wl.init_data(want_u=True)
        if global_err is not None:
            # every row seen, with its U row as the update that brought it computed it
            acc_x, acc_u = [X.astype(np.float64)], [U.astype(np.float64)]
            acc_s = [np.repeat(np.arange(wl.K0), np.diff(ptr))]
        g = Dash(wl.J, wl.R, lam=lam, max_slices=wl.K_max + 64, max_rows=1 << 21, max_groups=1 << 16,
                 stats_mode=STATS_LAGGED if lagged else STATS_EXACT)
        g.init_from_factors(ptr, to(X), to(U), to(wl.W[: wl.K0]), to(wl.V))
        if scores:
            g.anomaly(5)
        g.spans(True)
        out = []
        for s in range(1, n_steps + 1):
            b = wl.step(s)
            if cycle is not None:   # cycle / 5 rows per slice per update (the first ones of the batch)
                keep = np.minimum(np.diff(b.row_ptr), max(1, cycle // 5))
                rows = np.concatenate([b.rows[b.row_ptr[i]:b.row_ptr[i] + keep[i]] for i in range(b.n_groups)])
                rptr = np.concatenate([[0], np.cumsum(keep)]).astype(np.int64)
            else:
                rows, rptr = b.rows, b.row_ptr
            rd, nd = to(rows), to(b.new_rows)
            g.ingest_slices(b.new_ptr, nd)
            g.ingest_rows(b.row_ids, rptr, rd)
            torch.cuda.synchronize()
            rep = g.update()
            out.append((rep, int(rptr[-1] + b.new_ptr[-1])))
            if global_err is not None:
                # the global error of the evaluation section: old rows with their
                # stored U rows, plus this update's rows, both reconstructed
                # with the current S_k and V
                Vc, Wc, Un = (t.cpu().numpy().astype(np.float64) for t in g.get_factors())
                K_old = wl.K_at(s - 1)
                new_x = np.concatenate([b.new_rows, rows]).astype(np.float64)
                new_s = np.concatenate([np.repeat(K_old + np.arange(b.n_new), np.diff(b.new_ptr)),
                                        np.repeat(b.row_ids.astype(np.int64), np.diff(rptr))])
                old = mean_slice_error(np.concatenate(acc_x), np.concatenate(acc_u), np.concatenate(acc_s), Wc, Vc)
                global_err.append(old + mean_slice_error(new_x, Un, new_s, Wc, Vc))
                acc_x.append(new_x)
                acc_u.append(Un)
                acc_s.append(new_s)
        spans = g.spans_read()
        g.spans(False)
        return g, out, spans, (ptr, X)

    res = {"study": args.study, "data": "synthetic", "n_gpus": 1}
    if args.study == "cycle":
        rows = []
        for cycle in (20, 40, 60, 80, 100):
            wl = make_workload("mid", n_steps=12, median=24, lo=11, hi=200)
            wl_cycle = wl
            g, out, spans, _ = stream(wl_cycle, 0.95, 12, cycle=cycle)
            sp = np.array(spans[2:]) * 1e3
            m = np.mean([o[1] for o in out[2:]])
            rows.append({"cycle": cycle, "rows_per_update": m, "update_us_p50": float(np.median(sp)),
                         "rows_per_s": m / (float(np.median(sp)) / 1e6)})
            g.close()
        res["config"] = ("mid shape (J 88, R 10, K0 2000, initial slices median 24): each update brings cycle/5 "
                         "rows of every slice and 20 new slices; device span per update (p50 of updates 3..12)")
        res["points"] = rows
    elif args.study == "lambda":
        rows = []
        for drift in (0.0, 0.05):
            for lam in (0.1, 0.3, 0.5, 0.7, 0.9):
                wl = make_workload("mid", n_steps=16, median=24, lo=11, hi=200, drift=drift)
                ge = []
                g, out, _, _ = stream(wl, lam, 16, scores=True, global_err=ge)
                te = [o[0]["te"] for o in out]
                rows.append({"drift": drift, "lambda": lam, "local_error_mean": float(np.mean(te)),
                             "global_error_mean": float(np.mean(ge)),
                             "fit_lambda_weighted_last": out[-1][0]["fit"]})
                g.close()
        res["config"] = ("mid shape (J 88, R 10, K0 2000, initial slices median 24), 16 updates, planted V "
                         "stationary (drift 0) or moved 5 % of the way to a second planted V per update "
                         "(drift 0.05); local error = te (Definition 2: mean absolute error of the updated "
                         "model on each update's new rows), global error = the evaluation section's sum of "
                         "the mean per-slice absolute errors over the rows seen before the update (their U "
                         "rows as computed on arrival) and over the update's rows, with the current S_k and "
                         "V; both averaged over the updates")
        res["points"] = rows
    elif args.study == "lagged":
        # the same stream under both statistics modes: Lemmas 2-3 evaluated from
        # the exact Y_k, D_k (every slice's Y_k read twice per pass) against
        # Algorithm 1's recursions of c_k, F, G (only the new rows read)
        res_modes = {}
        for shape in ("mid", "batch_r10"):
            n = 24
            for lagged in (False, True):
                wl = make_workload(shape, n_steps=n, median=24, lo=11, hi=200)
                g, out, spans, _ = stream(wl, wl.lam, n, lagged=lagged)
                res_modes[(shape, lagged)] = ([o[0]["fit"] for o in out], np.array(spans[2:]) * 1e3,
                                              [o[1] for o in out])
                g.close()
        rows = []
        for shape in ("mid", "batch_r10"):
            fe, se, me = res_modes[(shape, False)]
            fl, sl, _ = res_modes[(shape, True)]
            d = np.abs(np.array(fe) - np.array(fl))
            rows.append({"workload": shape, "updates": len(fe),
                         "exact_update_us_p50": float(np.median(se)), "lagged_update_us_p50": float(np.median(sl)),
                         "rows_per_update": float(np.mean(me)),
                         "fit_exact_last": fe[-1], "fit_lagged_last": fl[-1],
                         "abs_dfit_first": float(d[0]), "abs_dfit_max": float(d.max()), "abs_dfit_last": float(d[-1])})
        res["config"] = ("mid (J 88, R 10, K0 2000) and batching R 10 (J 128, K0 20000) shapes, initial slices "
                         "median 24, 24 updates each, lambda 0.95, one ALS pass; the same inputs under the exact "
                         "statistics and the lagged recursions; device span per update (p50 of updates 3..24); "
                         "fit as each mode reports it")
        res["points"] = rows
    else:
        wl = make_workload("mid", n_steps=10, median=24, lo=11, hi=200)
        g, out, spans, (ptr, X) = stream(wl, 1.0, 10)
        t_update = float(np.median(np.array(spans) * 1e3))
        # the accumulated tensor: initial rows, then every update's rows, per slice
        K = wl.K_at(10)
        parts = [[X[ptr[k]:ptr[k + 1]]] if k < wl.K0 else [] for k in range(K)]
        for s in range(1, 11):
            b = wl.step(s)
            for l, blk in enumerate(b.new_slices()):
                parts[wl.K_at(s - 1) + l].append(blk)
            for k, blk in b.groups():
                parts[k].append(blk)
        Xa = np.concatenate([np.concatenate(p) for p in parts])
        pa = np.concatenate([[0], np.cumsum([sum(x.shape[0] for x in p) for p in parts])]).astype(np.int64)
        h = Dash(wl.J, wl.R, lam=1.0, max_slices=K + 8, max_rows=1024, max_groups=1024,
                 max_init_rows=int(pa[-1]) + 1, init_max_iter=10)
        Xd = to(Xa)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ir = h.init(pa, Xd, to(wl.V))
        torch.cuda.synchronize()
        t_static = (time.perf_counter() - t0) * 1e6
        res["config"] = ("mid shape, lambda = 1, 10 updates; the static recompute is the GPU PARAFAC2-ALS "
                         "(10 iterations, started from the planted V) over every row seen so far")
        res["points"] = [{"streaming_update_us_p50": t_update, "streaming_fit": out[-1][0]["fit"],
                          "static_recompute_us": t_static, "static_fit": ir["fit"], "static_iters": ir["iters"],
                          "rows_total": int(pa[-1]), "speedup": t_static / t_update}]
        g.close()
        h.close()
    print(json.dumps(res, default=_json_default), flush=True)


if __name__ == "__main__":
    main()
