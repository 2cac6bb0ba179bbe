"""GPU parity of the update path (HIP kernels through the C ABI) against the
FP64 oracle.

Teacher-forced tests start the library and the oracle from the same state
(dash_set_state with the oracle's state) and compare one update element by
element: every element of U_new, Y_k, D_k, n_k, W and V, and the fit, against
its a-priori float32 bound (tests/_bounds.py: the sums of |a||b| of the
element's products times the unit roundoff and the product length, carried
through Lemma 2's and Lemma 3's systems componentwise, so the condition of
each system enters the bound of its solution).  Tests with several ALS
passes per update, or free-running streams, compare normwise: U_new, Y_k,
D_k <= 2e-6, n_k <= 1e-6, W and V <= 1e-5.
"""
import numpy as np
import pytest

from oracle.dash_oracle import DashOracle
from paper_2305_18376_amd.synth import make_workload
from tests._bounds import assert_within, update_bounds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dash():
    from paper_2305_18376_amd.dash import Dash
    return Dash


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def feed(g, groups, news, J):
    """Stage one update on the GPU: new slices first, then row groups; returns
    the ingest-order list of (kind, index) for matching U_new rows."""
    if news:
        ptr = np.concatenate([[0], np.cumsum([X.shape[0] for X in news])]).astype(np.int64)
        g.ingest_slices(ptr, dev(np.concatenate(news)))
    if groups:
        ids = np.array([k for k, _ in groups], dtype=np.int32)
        ptr = np.concatenate([[0], np.cumsum([X.shape[0] for _, X in groups])]).astype(np.int64)
        rows = np.concatenate([X for _, X in groups]) if ptr[-1] else np.zeros((1, J), np.float32)
        g.ingest_rows(ids, ptr, dev(rows))


def oracle_u(r):
    parts = list(r.U_new_slices) + list(r.U_groups)
    parts = [p for p in parts if p.shape[0]]
    return np.concatenate(parts) if parts else np.zeros((0, 1))


def per_slice(groups, news, r, K_old):
    """{slice: X_new}, {slice: U_new} of an update (rows of a slice concatenated
    in ingest order: its new-slice block first, then its groups)."""
    xs, us = {}, {}
    for l, (X, U) in enumerate(zip(news, r.U_new_slices)):
        xs.setdefault(K_old + l, []).append(np.asarray(X, np.float64))
        us.setdefault(K_old + l, []).append(U)
    for (k, X), U in zip(groups, r.U_groups):
        if X.shape[0]:
            xs.setdefault(k, []).append(np.asarray(X, np.float64))
            us.setdefault(k, []).append(U)
    return ({k: np.concatenate(v) for k, v in xs.items()}, {k: np.concatenate(v) for k, v in us.items()})


def check_step(g, o, r, rep, tol_w=1e-5, tag="", pre=None, groups=None, news=None):
    st = g.get_state()
    V, W, U = g.get_factors()
    U = U.cpu().numpy()
    ost = o.state()
    if pre is not None and o.n_iter == 1:
        # element by element against the a-priori bounds
        K_old = pre["W"].shape[0]
        xs, us = per_slice(groups or [], news or [], r, K_old)
        bnd = update_bounds(pre, ost, o.lam, xs, us)
        # U_new bound rows in ingest order: a slice's rows keep their order across groups
        offs = {k: 0 for k in xs}
        rows_b = []
        for l, X in enumerate(news or []):
            k = K_old + l
            rows_b.append(bnd["U"][k][offs[k]:offs[k] + X.shape[0]])
            offs[k] += X.shape[0]
        for k, X in groups or []:
            if X.shape[0]:
                rows_b.append(bnd["U"][k][offs[k]:offs[k] + X.shape[0]])
                offs[k] += X.shape[0]
        worst = {"U": assert_within(f"{tag} U", U, oracle_u(r), np.concatenate(rows_b))}
        for key in ("Y", "D", "n", "W", "V"):
            worst[key] = assert_within(f"{tag} {key}", st[key], ost[key], bnd[key])
        worst["fit"] = abs(rep["fit"] - r.fit) / bnd["fit"] if bnd["fit"] > 0 else 0.0
        print(tag, "error/bound", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
        assert rep["committed"] == 1
        assert worst["fit"] <= 1.0, worst
        return worst
    errs = {
        "U": relerr(U, oracle_u(r)),
        "Y": relerr(st["Y"], ost["Y"]),
        "D": relerr(st["D"], ost["D"]),
        "n": relerr(st["n"], ost["n"]),
        "W": relerr(st["W"], ost["W"]),
        "V": relerr(st["V"], ost["V"]),
        "fit": abs(rep["fit"] - r.fit),
    }
    print(tag, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert rep["committed"] == 1
    assert errs["U"] <= 2e-6 and errs["Y"] <= 2e-6 and errs["D"] <= 2e-6 and errs["n"] <= 1e-6, errs
    assert errs["W"] <= tol_w and errs["V"] <= tol_w, errs
    e_state = max(errs["Y"], errs["D"], errs["n"])
    assert errs["fit"] <= 1e-6 + 4.0 * e_state / max(1.0 - r.fit, 1e-3), errs
    return errs


def random_stream(seed, K0, J, R, steps, lam=0.8, n_iter=1, max_new=4):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((J, R))
    W = rng.uniform(0.5, 1.5, size=(K0 + 3 * steps, R))

    def rows(k, m):
        U = rng.standard_normal((m, R))
        return ((U * W[k]) @ V.T + 0.05 * rng.standard_normal((m, J))).astype(np.float32), U

    init = [rows(k, int(rng.integers(R + 1, 3 * R + 8))) for k in range(K0)]
    batches = []
    K = K0
    for _ in range(steps):
        groups = [(k, rows(k, int(rng.integers(0, max_new + 1)))[0]) for k in range(K)]
        groups = [(k, X) for k, X in groups if X.shape[0]]
        news = [rows(K + l, int(rng.integers(1, max_new + 2)))[0] for l in range(3)]
        batches.append((groups, news))
        K += 3
    return dict(V=V, W=W[:K0], init=init, batches=batches, lam=lam, n_iter=n_iter, J=J, R=R)


def start_pair(cfg, Dash):
    J, R = cfg["J"], cfg["R"]
    X0 = [x for x, _ in cfg["init"]]
    U0 = [u for _, u in cfg["init"]]
    o = DashOracle(J, R, cfg["lam"], n_iter=cfg["n_iter"])
    o.init_from_factors(X0, U0, cfg["W"], cfg["V"])
    g = Dash(J, R, lam=cfg["lam"], n_iter=cfg["n_iter"], max_slices=4096, max_rows=1 << 16, max_groups=4096)
    ptr = np.concatenate([[0], np.cumsum([x.shape[0] for x in X0])]).astype(np.int64)
    g.init_from_factors(ptr, dev(np.concatenate(X0)), dev(np.concatenate(U0)), dev(cfg["W"]), dev(cfg["V"]))
    return o, g


def test_init_from_factors_state_matches_oracle():
    Dash = _dash()
    cfg = random_stream(1, K0=40, J=24, R=6, steps=0)
    o, g = start_pair(cfg, Dash)
    st, ost = g.get_state(), o.state()
    for key in ("Y", "D", "n", "W", "V"):
        assert relerr(st[key], ost[key]) <= 2e-6, key
    rep = g.update()  # nothing staged: no-op, reports the current fit
    assert rep["rows"] == 0
    assert abs(rep["fit"] - o.fit()) <= 1e-6


@pytest.mark.parametrize("variant", ["default", "split"])
@pytest.mark.parametrize("J,R,n_iter", [(1, 1, 1), (7, 3, 2), (20, 5, 3), (64, 8, 1), (65, 5, 1),
                                        (88, 10, 1), (128, 20, 1), (200, 17, 2), (128, 16, 1), (64, 32, 1), (256, 32, 1)])
def test_teacher_forced_update_shapes(J, R, n_iter, variant, monkeypatch):
    """One update from an identical state, every (R, J) register class, with
    the sweep the library picks and with the split sweep (row stage, solve
    stage, F stage; J not a multiple of 4 or 16 takes its own code there)."""
    if variant == "split":
        monkeypatch.setenv("DASH_VARIANT", "1")
    else:
        monkeypatch.delenv("DASH_VARIANT", raising=False)
    Dash = _dash()
    cfg = random_stream(J * 100 + R, K0=37, J=J, R=R, steps=3, n_iter=n_iter)
    o, g = start_pair(cfg, Dash)
    for s, (groups, news) in enumerate(cfg["batches"]):
        ost = o.state()
        g.set_state(ost["V"], ost["W"], ost["Y"], ost["D"], ost["n"])
        feed(g, groups, news, J)
        rep = g.update()
        r = o.update(groups, news)
        check_step(g, o, r, rep, tag=f"J={J} R={R} step={s}", pre=ost, groups=groups, news=news)


def test_free_run_tiny_workload_tracks_oracle():
    """The tiny planted workload (10 updates, 3 ALS passes, lambda 0.9) run
    freely on both sides from the planted factors."""
    Dash = _dash()
    wl = make_workload("tiny")
    ptr, X, U = wl.init_data(want_u=True)
    slices = [X[ptr[k]:ptr[k + 1]] for k in range(wl.K0)]
    o = DashOracle(wl.J, wl.R, wl.lam, n_iter=wl.n_iter)
    o.init_from_factors(slices, [U[ptr[k]:ptr[k + 1]] for k in range(wl.K0)], wl.W[: wl.K0], wl.V)
    g = Dash(wl.J, wl.R, lam=wl.lam, n_iter=wl.n_iter, max_slices=256, max_rows=1 << 14, max_groups=1024)
    g.init_from_factors(ptr, dev(X), dev(U), dev(wl.W[: wl.K0]), dev(wl.V))
    for s in range(1, wl.n_steps + 1):
        b = wl.step(s)
        feed(g, b.groups(), b.new_slices(), wl.J)
        rep = g.update()
        r = o.update(b.groups(), b.new_slices())
        print(s, rep["fit"], r.fit, flush=True)
        assert abs(rep["fit"] - r.fit) <= 1e-5
    st, ost = g.get_state(), o.state()
    assert relerr(st["V"], ost["V"]) <= 1e-4
    assert relerr(st["W"], ost["W"]) <= 1e-4


def test_teacher_forced_mid_workload_reduced():
    """The mid workload's generator at K0=300 (several chunks, ragged rows)."""
    Dash = _dash()
    wl = make_workload("mid", K0=300, n_steps=3)
    ptr, X, U = wl.init_data(want_u=True)
    slices = [X[ptr[k]:ptr[k + 1]] for k in range(wl.K0)]
    o = DashOracle(wl.J, wl.R, wl.lam)
    o.init_from_factors(slices, [U[ptr[k]:ptr[k + 1]] for k in range(wl.K0)], wl.W[: wl.K0], wl.V)
    g = Dash(wl.J, wl.R, lam=wl.lam, max_slices=1024, max_rows=1 << 16, max_groups=2048)
    g.init_from_factors(ptr, dev(X), dev(U), dev(wl.W[: wl.K0]), dev(wl.V))
    for s in range(1, wl.n_steps + 1):
        b = wl.step(s)
        ost = o.state()
        g.set_state(ost["V"], ost["W"], ost["Y"], ost["D"], ost["n"])
        feed(g, b.groups(), b.new_slices(), wl.J)
        rep = g.update()
        r = o.update(b.groups(), b.new_slices())
        check_step(g, o, r, rep, tag=f"mid300 step={s}", pre=ost, groups=b.groups(), news=b.new_slices())


def test_edge_cases_multi_group_new_slice_rows_and_small_blocks():
    """A slice extended by two groups in one update, rows appended to a slice
    created in the same update, blocks with fewer rows than R."""
    Dash = _dash()
    J, R = 12, 5
    cfg = random_stream(5, K0=6, J=J, R=R, steps=0)
    o, g = start_pair(cfg, Dash)
    rng = np.random.default_rng(6)
    blk = lambda m: rng.standard_normal((m, J)).astype(np.float32)
    news = [blk(2), blk(1)]
    groups = [(3, blk(1)), (0, blk(7)), (3, blk(2)), (7, blk(2)), (5, blk(0))]
    feed(g, groups, news, J)
    rep = g.update()
    r = o.update(groups, news)
    check_step(g, o, r, rep, tag="edge")
    # an empty update is a no-op: no forgetting
    before = g.get_state()
    rep = g.update()
    assert rep["rows"] == 0
    after = g.get_state()
    for key in before:
        np.testing.assert_array_equal(before[key], after[key])


@pytest.mark.parametrize("J,R,n_iter", [(130, 20, 1), (96, 24, 2), (256, 32, 1)])
def test_block_variant_long_groups_and_neighbours(J, R, n_iter):
    """The workgroup-per-slice sweep: row groups longer than one staged block
    (64 rows up to J = 128, 32 beyond), a slice extended by two groups,
    consecutive touched slices (the next slice's first block is staged while
    the current one solves), rows appended to a slice created in the same
    update, blocks with fewer rows than R, untouched slices between; J = 130
    takes the scalar row staging, the others float4 loads."""
    Dash = _dash()
    cfg = random_stream(17, K0=12, J=J, R=R, steps=0, n_iter=n_iter)
    o, g = start_pair(cfg, Dash)
    rng = np.random.default_rng(18)
    Vt = cfg["V"]

    def blk(k, m):
        U = rng.standard_normal((m, R))
        return ((U * rng.uniform(0.5, 1.5, R)) @ Vt.T + 0.05 * rng.standard_normal((m, J))).astype(np.float32)

    for step in range(2):
        news = [blk(0, 3), blk(0, 70)]
        K = 12 + 2 * step
        groups = [(1, blk(1, 150)), (2, blk(2, 5)), (3, blk(3, 65)), (4, blk(4, 2)), (1, blk(1, 33)),
                  (7, blk(7, 1)), (8, blk(8, 97)), (K, blk(K, 4)), (K + 1, blk(K + 1, 40))]
        feed(g, groups, news, J)
        rep = g.update()
        r = o.update(groups, news)
        check_step(g, o, r, rep, tag=f"block J={J} R={R} step {step}")


def test_errors_leave_state_unchanged_and_numeric_rollback():
    from paper_2305_18376_amd.dash import DashError, E_INVALID_ARG, E_NUMERIC, E_CAPACITY
    Dash = _dash()
    J, R = 10, 3
    cfg = random_stream(9, K0=5, J=J, R=R, steps=1)
    o, g = start_pair(cfg, Dash)
    before = g.get_state()
    rows = dev(np.ones((2, J)))
    with pytest.raises(DashError) as e:
        g.ingest_rows(np.array([5], np.int32), np.array([0, 2]), rows)   # id 5 does not exist
    assert e.value.status == E_INVALID_ARG
    with pytest.raises(DashError) as e:
        g.ingest_rows(np.array([0], np.int32), np.array([2, 1]), rows)   # decreasing row_ptr
    assert e.value.status == E_INVALID_ARG
    with pytest.raises(DashError) as e:
        g.ingest_slices(np.array([0, 0]), rows)                          # empty new slice
    assert e.value.status == E_INVALID_ARG
    with pytest.raises(DashError) as e:
        g.ingest_rows(np.array([0], np.int32), np.array([0, 1 << 17]), rows)  # capacity
    assert e.value.status == E_CAPACITY
    # non-finite data: the update is rolled back, the context keeps working
    bad = np.ones((3, J), np.float32)
    bad[1, 2] = np.nan
    g.ingest_rows(np.array([1], np.int32), np.array([0, 3]), dev(bad))
    g.ingest_slices(np.array([0, 2]), dev(np.ones((2, J))))
    with pytest.raises(DashError) as e:
        g.update()
    assert e.value.status == E_NUMERIC
    after = g.get_state()
    for key in before:
        np.testing.assert_array_equal(before[key], after[key])
    assert g.dims().K == 5
    groups, news = cfg["batches"][0]
    feed(g, groups, news, J)
    rep = g.update()
    r = o.update(groups, news)
    check_step(g, o, r, rep, tag="after-rollback")


def test_async_updates_equal_blocking_and_are_deterministic():
    Dash = _dash()
    cfg = random_stream(11, K0=50, J=32, R=4, steps=4)
    _, g1 = start_pair(cfg, Dash)
    _, g2 = start_pair(cfg, Dash)
    for groups, news in cfg["batches"]:
        feed(g1, groups, news, cfg["J"])
        g1.update()
    for groups, news in cfg["batches"]:
        feed(g2, groups, news, cfg["J"])
        g2.update_async()
    g2.wait()
    s1, s2 = g1.get_state(), g2.get_state()
    for key in s1:
        np.testing.assert_array_equal(s1[key], s2[key])


def test_checkpoint_roundtrip_resumes_bitwise(tmp_path):
    Dash = _dash()
    cfg = random_stream(13, K0=30, J=16, R=4, steps=4)
    _, g1 = start_pair(cfg, Dash)
    for groups, news in cfg["batches"][:2]:
        feed(g1, groups, news, cfg["J"])
        g1.update()
    path = tmp_path / "ck.bin"
    g1.save(path)
    g2 = Dash(cfg["J"], cfg["R"], lam=cfg["lam"], max_slices=4096, max_rows=1 << 16, max_groups=4096)
    g2.load(path)
    assert g2.dims().step == g1.dims().step
    for groups, news in cfg["batches"][2:]:
        for g in (g1, g2):
            feed(g, groups, news, cfg["J"])
            g.update()
    s1, s2 = g1.get_state(), g2.get_state()
    for key in s1:
        np.testing.assert_array_equal(s1[key], s2[key])
