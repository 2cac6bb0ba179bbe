"""Benchmark of the streaming PARAFAC2 update on one MI355X.

Workload (mid-size dual-way stream): K0 = 2000 slices, I_k log-normal (median
800, clipped to [100, 4000]), J = 88, R = 10, planted low-rank rows + 5 % noise;
every update appends U{1..20} rows to every slice and brings 20 new slices of
U{1..20} rows; lambda = 0.95, one ALS pass per update (Algorithm 1).

A "step" is one update (Lemma 1 rows -> Lemma 2 sweep -> Lemma 3 solve ->
commit) over one batch that is already resident in HBM.  Warm-up updates run
blocking and their fits are checked against the FP64 oracle, which is also
timed on the host as the CPU baseline; the timed updates run back to back
(asynchronously) and are bracketed by stream synchronisation.

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


def algorithmic_bytes(M, K, K_t, J, R, words=1):
    """Bytes one update pass must move (the per-pass model of the design notes):
    new rows read, U_new written, every slice's Y_k / D_k / n_k / W row read,
    touched slices' Y_k / D_k / n_k written, every W row written.  `words` = 2
    counts the compensation word the mixed path keeps beside each Y_k / D_k
    entry."""
    return (M * J * 4 + M * R * 4
            + K * (words * (R * J * 4 + R * R * 4) + 8 + R * 8)
            + K_t * (words * (R * J * 4 + R * R * 4) + 8)
            + K * R * 8)


def _source_digest():
    """SHA-256 of the kernel source the library is built from."""
    import hashlib
    src = os.path.join(ROOT, "paper_2305_18376_amd", "csrc", "dash_kernels.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_traffic(kernel, workload):
    """HBM bytes per dispatch of `kernel` from the committed byte-counter
    summary (profiles/<kernel>_<workload>_counters.md), or None when that
    summary is missing or was taken on a different kernel source."""
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
        return float(vals["traffic_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed updates (mid: 90, others: 20)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up updates (mid: 10, others: 3)")
    ap.add_argument("--workload", default="mid", choices=["mid", "batch_r10", "batch_r20", "precision"],
                    help="mid is the headline workload; the others are the batching and precision ones "
                         "(their initial slices are shorter: the per-update cost does not depend on them)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "mixed"])
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
    ap.add_argument("--serve", action="store_true",
                    help="serving measurement instead: 64 streams of mixed shapes on one device, "
                         "one update per stream per tick; prints its own JSON line")
    ap.add_argument("--ticks", type=int, default=200, help="ticks of the serving measurement")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed region, one plain device copy of this many MiB "
                         "(reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the update would shard by slice with one all-reduce of F, G per pass).", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        return serve_main(args)

    import torch
    from paper_2305_18376_amd.dash import Dash
    from paper_2305_18376_amd.synth import make_workload

    big = args.workload != "mid"
    W_ = args.warmup if args.warmup is not None else (3 if big else 10)
    if args.autotune > 0:
        W_ = max(W_, 8 * args.autotune + 2)   # at most 8 candidate schedules
    K_ = args.steps if args.steps is not None else (20 if big else 90)
    n_total = W_ + K_
    if big:
        # initial slices of log-normal length median 24 (the update cost depends on K, not on them)
        wl = make_workload(args.workload, n_steps=n_total, median=24, lo=1, hi=200)
        wl.init_len = np.maximum(wl.init_len, wl.R + 1)
    else:
        wl = make_workload("mid", n_steps=max(100, n_total))
    t0 = time.time()
    ptr, X, U = wl.init_data(want_u=True)
    batches = [wl.step(s) for s in range(1, n_total + 1)]
    t_gen = time.time() - t0

    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    from paper_2305_18376_amd.dash import PREC_FP32, PREC_MIXED
    max_rows = max(64 * 1024, max(b.M for b in batches) + 1)
    max_groups = max(8192, max(b.n_groups + b.n_new for b in batches) + 1)
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
    bytes_pass, bytes_all = 0, 0
    for i in range(K_):
        b = batches[W_ + i]
        s = W_ + i + 1
        nb = algorithmic_bytes(b.M, wl.K_at(s), b.n_groups + b.n_new, wl.J, wl.R,
                               words=2 if args.precision == "mixed" else 1) * wl.n_iter
        bytes_all += nb
        if args.sample_every > 0 and s % args.sample_every == 0:
            bytes_pass += nb
    pass_ms = prof["pass_ms"]
    achieved = bytes_pass / (pass_ms / 1e3) / 1e9 if pass_ms > 0 else None

    sched = g.schedule()
    kernel = "k_pass_wave" if sched["variant"] == 0 else "k_rows"
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
                     "kernel": kernel, "algorithmic_bytes_per_step": bytes_all / K_},
        "final_fit": last["fit"],
        "gen_s": t_gen,
    }

    tr = counter_traffic(kernel, args.workload + ("" if args.precision == "fp32" else "_mixed"))
    out["roofline"]["traffic"] = tr
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


def serve_streams(n_streams, ticks, seed=5000):
    """Seeded multi-stream workload: per stream J ~ U{32,64,128,256}, R ~ U{8,16,32},
    lambda ~ U[0.8, 0.99], K0 ~ U{100..300} slices of log-normal length (median 30);
    every tick Poisson(50) new rows spread over the slices by Zipf(1.2) popularity
    of a random ranking, and a new slice of U{1..60} rows with probability 0.05."""
    streams = []
    for sidx in range(n_streams):
        rng = np.random.default_rng([seed, sidx])
        J = int(rng.choice([32, 64, 128, 256]))
        R = int(rng.choice([8, 16, 32]))
        lam = float(rng.uniform(0.8, 0.99))
        K0 = int(rng.integers(100, 301))
        K_max = K0 + ticks
        V = rng.standard_normal((J, R))
        W = rng.uniform(0.5, 1.5, size=(K_max, R))

        def rows(ids):
            U = rng.standard_normal((len(ids), R))
            X = (U * W[ids]) @ V.T + 0.05 * rng.standard_normal((len(ids), J))
            return X.astype(np.float32), U

        lens = np.clip(np.round(np.exp(np.log(30) + rng.standard_normal(K0))), R + 1, 400).astype(np.int64)
        ptr0 = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        X0, U0 = rows(np.repeat(np.arange(K0), lens))
        rank = rng.permutation(K_max)
        batches = []
        K = K0
        for t in range(ticks):
            n = int(rng.poisson(50))
            pop = (np.arange(1, K + 1) ** -1.2)[np.argsort(rank[:K])]
            ids = np.sort(rng.choice(K, size=n, p=pop / pop.sum())) if n else np.zeros(0, np.int64)
            uniq, cnt = np.unique(ids, return_counts=True)
            X, _ = rows(ids)
            new = None
            if rng.random() < 0.05:
                m = int(rng.integers(1, 61))
                new = rows(np.full(m, K))[0]
                K += 1
            batches.append((uniq.astype(np.int32), np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64), X, new))
        streams.append(dict(J=J, R=R, lam=lam, K0=K0, K_max=K_max, V=V, W=W[:K0], ptr0=ptr0, X0=X0, U0=U0,
                            batches=batches))
    return streams


def serve_main(args):
    """Closed-loop serving measurement: every tick stages one batch per stream,
    enqueues one update per stream (all concurrent, one HIP stream each) and
    polls until all of them are committed.  Latency = host time from the tick
    that cut an update to the poll that saw it committed."""
    import torch
    from paper_2305_18376_amd.dash import DashServer, PREC_FP32, PREC_MIXED
    n_streams, T = 64, args.ticks
    prec = PREC_MIXED if args.precision == "mixed" else PREC_FP32
    t0 = time.time()
    streams = serve_streams(n_streams, T)
    t_gen = time.time() - t0
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    srv = DashServer(200 << 30)
    views = []
    for d in streams:
        sid, g = srv.open(d["J"], d["R"], lam=d["lam"], max_slices=d["K_max"] + 8, max_rows=4096,
                          max_groups=4096, precision=prec)
        g.init_from_factors(d["ptr0"], to(d["X0"]), to(d["U0"]), to(d["W"]), to(d["V"]))
        dbat = [(ids, ptr, to(X) if X.shape[0] else None, None if new is None else to(new))
                for ids, ptr, X, new in d["batches"]]
        views.append((sid, g, dbat))
    torch.cuda.synchronize()

    def run(sel, ticks, warm):
        lat, rows_done, t_run = [], 0, 0.0
        for t in range(ticks):
            for i in sel:
                _, g, dbat = views[i]
                ids, ptr, X, new = dbat[t]
                if new is not None:
                    g.ingest_slices(np.array([0, new.shape[0]], np.int64), new)
                if X is not None:
                    g.ingest_rows(ids, ptr, X)
            h0 = time.perf_counter()
            srv.tick()
            reps = srv.poll(wait=True)
            dt = time.perf_counter() - h0
            if t >= warm:
                t_run += dt
                lat += [r["latency_us"] for r in reps]
                rows_done += sum(r["rows"] for r in reps)
            assert all(r["committed"] for r in reps)
        return np.array(lat), rows_done, t_run

    warm = 10
    lat, rows_done, t_run = run(range(n_streams), T, warm)
    out = {"metric": "serving: ingested rows/sec with p50/p99 cut-to-commit update latency",
           "value": rows_done / t_run, "unit": "rows/s", "n_gpus": 1, "streams": n_streams,
           "ticks": T - warm, "warmup": warm, "higher_is_better": True,
           "latency_ms": {"p50": float(np.percentile(lat, 50)) / 1e3, "p99": float(np.percentile(lat, 99)) / 1e3},
           "ms_per_tick": 1e3 * t_run / (T - warm),
           "dtype": "f32" if args.precision == "fp32" else "bf16-mfma/f32", "data": "synthetic",
           "config": {"workload": "64 streams, J~U{32,64,128,256}, R~U{8,16,32}, K0~U{100..300}, "
                                  "Poisson(50) rows/tick over Zipf(1.2) slices, new slice p=0.05/tick",
                      "budget_gb": 200, "closed_loop": True},
           "gen_s": t_gen}
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
