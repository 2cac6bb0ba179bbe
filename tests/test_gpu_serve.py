"""GPU tests of the serving layer: many streams on one device, each with its own
shape and forgetting factor, one update per stream per tick, non-blocking
completion polling.  Streams share nothing, so a stream's factors are bit for
bit those it has alone (and those of a plain context fed the same rows)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def stream_data(seed, J, R, K0, ticks):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((J, R))
    W = rng.uniform(0.5, 1.5, size=(K0 + ticks, R))

    def rows(k, m):
        U = rng.standard_normal((m, R))
        return ((U * W[k]) @ V.T + 0.05 * rng.standard_normal((m, J))).astype(np.float32), U

    init = [rows(k, int(rng.integers(R + 1, 2 * R + 6))) for k in range(K0)]
    batches = []
    K = K0
    for t in range(ticks):
        ids = np.unique(rng.integers(0, K, size=int(rng.integers(3, 12)))).astype(np.int32)
        blocks = [rows(int(k), int(rng.integers(1, 6)))[0] for k in ids]
        ptr = np.concatenate([[0], np.cumsum([b.shape[0] for b in blocks])]).astype(np.int64)
        new = [rows(K, int(rng.integers(1, 5)))[0]] if t % 2 == 0 else []
        if new:
            K += 1
        batches.append((ids, ptr, np.concatenate(blocks), new))
    return dict(J=J, R=R, V=V, W=W[:K0], init=init, batches=batches, lam=0.9)


def init_ctx(g, d):
    X0 = [x for x, _ in d["init"]]
    U0 = [u for _, u in d["init"]]
    ptr = np.concatenate([[0], np.cumsum([x.shape[0] for x in X0])]).astype(np.int64)
    g.init_from_factors(ptr, dev(np.concatenate(X0)), dev(np.concatenate(U0)), dev(d["W"]), dev(d["V"]))


def stage(g, batch, keep):
    ids, ptr, rows, new = batch
    if new:
        nptr = np.array([0, new[0].shape[0]], np.int64)
        nr = dev(new[0])
        keep.append(nr)
        g.ingest_slices(nptr, nr)
    r = dev(rows)
    keep.append(r)
    g.ingest_rows(ids, ptr, r)


SHAPES = [(64, 8), (32, 16), (128, 8), (256, 32), (88, 10), (40, 5), (130, 20), (64, 32)]


def run_server(specs, ticks, budget=1 << 34):
    from paper_2305_18376_amd.dash import DashServer
    srv = DashServer(budget)
    views = {}
    for name, d in specs.items():
        sid, g = srv.open(d["J"], d["R"], lam=d["lam"], max_slices=256, max_rows=4096, max_groups=1024)
        init_ctx(g, d)
        views[name] = (sid, g)
    keep = []
    reports = []
    for t in range(ticks):
        for name, d in specs.items():
            stage(views[name][1], d["batches"][t], keep)
        srv.tick()
        # non-blocking polls until every stream reported this tick's update
        got = []
        while len(got) < len(specs):
            got += srv.poll(wait=False)
        reports += got
        keep.clear()
    out = {}
    for name, (sid, g) in views.items():
        V, W, _ = g.get_factors()
        out[name] = (V.cpu().numpy().copy(), W.cpu().numpy().copy())
    srv.close()
    return out, reports


def test_stream_alone_equals_stream_in_the_mix_bitwise():
    ticks = 4
    specs = {f"s{i}": stream_data(100 + i, J, R, 40, ticks) for i, (J, R) in enumerate(SHAPES)}
    alone, _ = run_server({"s0": specs["s0"], }, ticks)
    mixed, reports = run_server(specs, ticks)
    assert len(reports) == ticks * len(specs)
    assert all(r["committed"] == 1 and r["latency_us"] > 0 for r in reports)
    np.testing.assert_array_equal(alone["s0"][0], mixed["s0"][0])
    np.testing.assert_array_equal(alone["s0"][1], mixed["s0"][1])
    # and a plain context fed the same rows gives the same bits
    from paper_2305_18376_amd.dash import Dash
    d = specs["s0"]
    g = Dash(d["J"], d["R"], lam=d["lam"], max_slices=256, max_rows=4096, max_groups=1024)
    init_ctx(g, d)
    keep = []
    for t in range(ticks):
        stage(g, d["batches"][t], keep)
        g.update()
        keep.clear()
    V, W, _ = g.get_factors()
    np.testing.assert_array_equal(V.cpu().numpy(), mixed["s0"][0])
    np.testing.assert_array_equal(W.cpu().numpy(), mixed["s0"][1])


def test_admission_by_footprint_and_reopen():
    from paper_2305_18376_amd.dash import DashServer, DashError, E_CAPACITY, footprint
    kw = dict(max_slices=256, max_rows=4096, max_groups=1024)
    fp = footprint(J=64, R=8, **kw)
    srv = DashServer(int(1.5 * fp))
    a, _ = srv.open(64, 8, **kw)
    with pytest.raises(DashError) as e:
        srv.open(64, 8, **kw)
    assert e.value.status == E_CAPACITY
    srv.close_stream(a)
    b, g = srv.open(64, 8, **kw)
    d = stream_data(7, 64, 8, 20, 1)
    init_ctx(g, d)
    keep = []
    stage(g, d["batches"][0], keep)
    assert srv.tick() == 1
    reps = srv.poll(wait=True)
    assert len(reps) == 1 and reps[0]["stream"] == b and reps[0]["committed"] == 1
    srv.close()
