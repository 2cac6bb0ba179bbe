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


def algorithmic_bytes(M, K, K_t, J, R):
    """Bytes one update pass must move (the per-pass model of the design notes):
    new rows read, U_new written, every slice's Y_k / D_k / n_k / W row read,
    touched slices' Y_k / D_k / n_k written, every W row written."""
    return (M * J * 4 + M * R * 4
            + K * (R * J * 4 + R * R * 4 + 8 + R * 8)
            + K_t * (R * J * 4 + R * R * 4 + 8)
            + K * R * 8)


def _source_digest():
    """SHA-256 of the kernel source the library is built from."""
    import hashlib
    src = os.path.join(ROOT, "paper_2305_18376_amd", "csrc", "dash_kernels.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from the committed byte-counter
    summary (profiles/<kernel>_mid_counters.md), or None when that summary is
    missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_mid_counters.md")
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
    ap.add_argument("--steps", type=int, default=90)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sample-every", type=int, default=10,
                    help="time the kernels of every N-th update with HIP events (events perturb "
                         "the launches they bracket, so the others run undisturbed)")
    ap.add_argument("--oracle-seconds", type=float, default=25.0,
                    help="bound on the FP64 oracle replay (CPU baseline and fit check)")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="after the timed region, one plain device copy of this many MiB "
                         "(reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the update would shard by slice with one all-reduce of F, G per pass).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_18376_amd.dash import Dash
    from paper_2305_18376_amd.synth import make_workload

    W_, K_ = args.warmup, args.steps
    n_total = W_ + K_
    wl = make_workload("mid", n_steps=max(100, n_total))
    t0 = time.time()
    ptr, X, U = wl.init_data(want_u=True)
    batches = [wl.step(s) for s in range(1, n_total + 1)]
    t_gen = time.time() - t0

    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    g = Dash(wl.J, wl.R, lam=wl.lam, n_iter=wl.n_iter, max_slices=wl.K_max + 64,
             max_rows=64 * 1024, max_groups=8192)
    Xd, Ud = to(X), to(U)
    g.init_from_factors(ptr, Xd, Ud, to(wl.W[: wl.K0]), to(wl.V))
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

    # timed region
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K_)]
    g.profile(args.sample_every)
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    ev0.record(stream)
    for i in range(K_):
        step_ev[i][0].record(stream)
        stage(W_ + i)
        g.update_async()
        step_ev[i][1].record(stream)
    ev1.record(stream)
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
    dev_ms = ev0.elapsed_time(ev1)
    lat = np.array([a.elapsed_time(b) for a, b in step_ev])
    rows = sum(batches[W_ + i].M for i in range(K_))
    value = rows / (dev_ms / 1e3)

    # algorithmic bytes of the sampled (event-timed) passes; update index s = W_ + i + 1
    bytes_pass, bytes_all = 0, 0
    for i in range(K_):
        b = batches[W_ + i]
        s = W_ + i + 1
        nb = algorithmic_bytes(b.M, wl.K_at(s), b.n_groups + b.n_new, wl.J, wl.R) * wl.n_iter
        bytes_all += nb
        if args.sample_every > 0 and s % args.sample_every == 0:
            bytes_pass += nb
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mid dual-way stream: K0=2000 slices, I_k lognormal(median 800, clip 100..4000), "
                               "J=88, R=10, +U{1..20} rows/slice and +20 slices per update, lambda=0.95, 1 ALS pass",
                   "K_final": wl.K_at(n_total), "rows_timed": rows},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "note": "per-update device span, back-to-back updates"},
        "host_ms_per_step": (h1 - h0) * 1e3 / K_,
        "kernel_us_avg": {k: (1e3 * prof[k + "_ms"] / prof[k + "_launches"]) if prof[k + "_launches"] else None
                          for k in ("pass", "solve", "upload")},
        "kernel_timing": f"HIP events around the launches of every {args.sample_every}-th update "
                         f"({prof['updates']} sampled)",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
                     "kernel": "k_pass_wave", "algorithmic_bytes_per_step": bytes_all / K_},
        "final_fit": last["fit"],
        "gen_s": t_gen,
    }

    tr = counter_traffic("k_pass_wave")
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


if __name__ == "__main__":
    main()
