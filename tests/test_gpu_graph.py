"""Graph mode (dash_graph): an update's launches replayed from one HIP graph with
the kernel-node parameters rewritten per update.  Every replay must give the
bits of the directly launched update -- blocking updates with the program's
own synchronisations between replays, and back-to-back asynchronous ones."""
import numpy as np
import pytest

from paper_2305_18376_amd.synth import make_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def make(wl, ptr, X, U, graph, n_iter=None):
    from paper_2305_18376_amd.dash import Dash
    g = Dash(wl.J, wl.R, lam=wl.lam, n_iter=n_iter or wl.n_iter, max_slices=wl.K_max + 8, max_rows=1 << 16,
             max_groups=1 << 14)
    g.init_from_factors(ptr, dev(X), dev(U), dev(wl.W[: wl.K0]), dev(wl.V))
    if graph:
        g.graph(True)
    return g


def stage(g, b, keep):
    nr, r = dev(b.new_rows), dev(b.rows)
    keep += [nr, r]
    g.ingest_slices(b.new_ptr, nr)
    g.ingest_rows(b.row_ids, b.row_ptr, r)


@pytest.mark.parametrize("n_iter", [1, 2])
def test_graph_replays_equal_direct_launches(n_iter):
    wl = make_workload("mid", K0=300, n_steps=6)
    ptr, X, U = wl.init_data(want_u=True)
    eager, graph = make(wl, ptr, X, U, False, n_iter), make(wl, ptr, X, U, True, n_iter)
    keep = []
    for s in range(1, 7):
        b = wl.step(s)
        for g in (eager, graph):
            stage(g, b, keep)
        re, rg = eager.update(), graph.update()
        torch.cuda.synchronize()
        assert re["device_us"] > 0 and rg["device_us"] > 0
        re.pop("device_us"), rg.pop("device_us")
        assert re == rg, (s, re, rg)
        fe, fg = eager.get_factors(), graph.get_factors()
        for a, c in zip(fe, fg):
            assert torch.equal(a, c), s


def test_graph_back_to_back_async_equals_direct():
    wl = make_workload("mid", K0=300, n_steps=8)
    ptr, X, U = wl.init_data(want_u=True)
    eager, graph = make(wl, ptr, X, U, False), make(wl, ptr, X, U, True)
    batches = [wl.step(s) for s in range(1, 9)]
    keep = []
    for b in batches:
        stage(eager, b, keep)
        eager.update()
    for b in batches:
        stage(graph, b, keep)
        graph.update_async()
    rg = graph.wait()
    assert rg["committed"] == 1 and rg["step"] == 8
    se, sg = eager.get_state(), graph.get_state()
    for k in se:
        np.testing.assert_array_equal(se[k], sg[k])


def test_autotune_picks_a_schedule_and_stays_exact():
    """Every candidate schedule computes the same update (to the order of FP64
    partial sums); after the trials the best is kept, in graph mode too."""
    from oracle.dash_oracle import DashOracle
    wl = make_workload("mid", K0=300, n_steps=14)
    ptr, X, U = wl.init_data(want_u=True)
    g = make(wl, ptr, X, U, True)
    g.autotune(1)
    o = DashOracle(wl.J, wl.R, wl.lam)
    o.init_from_factors([X[ptr[k]:ptr[k + 1]] for k in range(wl.K0)], [U[ptr[k]:ptr[k + 1]] for k in range(wl.K0)],
                        wl.W[: wl.K0], wl.V)
    keep = []
    for s in range(1, 15):
        b = wl.step(s)
        r = o.update(b.groups(), b.new_slices())
        stage(g, b, keep)
        rep = g.update()
        assert abs(rep["fit"] - r.fit) <= 1e-5, (s, rep["fit"], r.fit)
    sc = g.schedule()
    assert sc["tuned"] == 1 and sc["candidates"] >= 8 and sc["ns_per_kb"] > 0, sc


def test_autotune_cache_reuses_the_schedule_tuned_for_the_same_shape(tmp_path):
    """A finished tuning run stores its winner under the update's shape key; a
    second context of the same shape takes it at its first update, and its
    updates stay exact."""
    import json
    from oracle.dash_oracle import DashOracle
    cache = tmp_path / "tune.jsonl"
    wl = make_workload("mid", K0=300, n_steps=12)
    ptr, X, U = wl.init_data(want_u=True)
    a = make(wl, ptr, X, U, False)
    a.autotune(1, cache=cache)
    keep = []
    for s in range(1, 11):
        stage(a, wl.step(s), keep)
        a.update()
    sa = a.schedule()
    assert sa["tuned"] == 1 and sa["from_cache"] == 0, sa
    lines = [json.loads(x) for x in cache.read_text().splitlines()]
    assert len(lines) == 1 and lines[0]["key"].startswith("gfx950/J88/R10/")
    assert (lines[0]["variant"], lines[0]["spread"], lines[0]["fuse"], lines[0]["solve_div"]) == \
        (sa["variant"], sa["spread"], sa["fused"], sa["solve_div"])
    b = make(wl, ptr, X, U, False)
    b.autotune(1, cache=cache)
    o = DashOracle(wl.J, wl.R, wl.lam)
    o.init_from_factors([X[ptr[k]:ptr[k + 1]] for k in range(wl.K0)], [U[ptr[k]:ptr[k + 1]] for k in range(wl.K0)],
                        wl.W[: wl.K0], wl.V)
    for s in range(1, 4):
        bt = wl.step(s)
        r = o.update(bt.groups(), bt.new_slices())
        stage(b, bt, keep)
        rep = b.update()
        assert abs(rep["fit"] - r.fit) <= 1e-5, (s, rep["fit"], r.fit)
        sb = b.schedule()
        assert sb["tuned"] == 1 and sb["from_cache"] == 1, sb
        assert (sb["variant"], sb["spread"], sb["fused"], sb["solve_div"]) == \
            (sa["variant"], sa["spread"], sa["fused"], sa["solve_div"])
