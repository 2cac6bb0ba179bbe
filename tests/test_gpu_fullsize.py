"""Teacher-forced parity at full size: K0 = 20 000 slices, one update of the
batching and precision workloads' arrival law (truncated Zipf(1.2), 0..200
rows per slice, 20 new slices), every kernel variant and chunking the
benchmark runs at that size.  Initial slices are short (the state, not the
rows that built it, is what an update reads), so the oracle finishes in
seconds.

Every element of U_new, W and V, and of Y_k, D_k, n_k of every slice, is
compared with the FP64 oracle against its a-priori bound (tests/_bounds.py:
float32 products, the fold, the FP64 R x R solves; BF16 products in the mixed
path).
"""
import numpy as np
import pytest

from oracle.dash_oracle import DashOracle
from paper_2305_18376_amd.synth import make_workload
from tests._bounds import assert_within, update_bounds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def oracle_run(name, R_over=None):
    kw = dict(K0=20000, n_steps=1, median=12, lo=1, hi=40)
    if R_over:
        kw["R"] = R_over
    wl = make_workload(name, **kw)
    ptr, X, U = wl.init_data(want_u=True)
    o = DashOracle(wl.J, wl.R, wl.lam)
    o.init_from_factors([X[ptr[k]:ptr[k + 1]] for k in range(wl.K0)], [U[ptr[k]:ptr[k + 1]] for k in range(wl.K0)],
                        wl.W[: wl.K0], wl.V)
    return wl, ptr, X, U, o


def gpu_update(wl, ptr, X, U, pre, precision, variant, monkeypatch):
    from paper_2305_18376_amd.dash import Dash
    # "wave" forces the fused wave sweep even where the default schedule
    # (past four slices per wave) would take the split sweep
    monkeypatch.setenv("DASH_VARIANT", "1" if variant == "split" else "0")
    g = Dash(wl.J, wl.R, lam=wl.lam, max_slices=wl.K_max + 8, max_rows=1 << 20, max_groups=1 << 16,
             precision=precision)
    g.set_state(pre["V"], pre["W"], pre["Y"], pre["D"], pre["n"])
    b = wl.step(1)
    g.ingest_slices(b.new_ptr, dev(b.new_rows))
    g.ingest_rows(b.row_ids, b.row_ptr, dev(b.rows))
    rep = g.update()
    st = g.get_state()
    _, _, Un = g.get_factors()
    out = (rep, st, Un.cpu().numpy().astype(np.float64))
    g.close()
    torch.cuda.synchronize()
    return out


def check(wl, o, pre, r, b, gpu, mixed, tag):
    rep, st, Un = gpu
    post = o.state()
    K_old = wl.K0
    xs, us = {}, {}
    for l, (Xb, Ub) in enumerate(zip(b.new_slices(), r.U_new_slices)):
        xs[K_old + l] = np.asarray(Xb, np.float64)
        us[K_old + l] = Ub
    for (k, Xb), Ub in zip(b.groups(), r.U_groups):
        xs[k] = np.asarray(Xb, np.float64)
        us[k] = Ub
    bnd = update_bounds(pre, post, wl.lam, xs, us, mixed=mixed)
    row_slices = np.concatenate([np.repeat(np.arange(K_old, K_old + b.n_new), np.diff(b.new_ptr)),
                                 np.repeat(b.row_ids, np.diff(b.row_ptr))])
    # U_new rows in ingest order (new slices, then groups)
    ou = np.concatenate(list(r.U_new_slices) + list(r.U_groups))
    bu = np.concatenate([bnd["U"][K_old + l] for l in range(b.n_new)] + [bnd["U"][k] for k, _ in b.groups()])
    worst = {"U": assert_within(f"{tag} U", Un, ou, bu)}
    for key in ("Y", "D", "n", "W", "V"):
        try:
            worst[key] = assert_within(f"{tag} {key}", st[key], post[key], bnd[key])
        except AssertionError:
            if key in ("Y", "D"):
                ratio = np.abs(st[key] - post[key]) / (bnd[key] + 1e-30)
                k = int(np.unravel_index(np.argmax(ratio), ratio.shape)[0])
                bad = np.argwhere(ratio[k] > 1.0)
                print(f"{tag} {key}: slice {k}: rows {xs[k].shape[0] if k in xs else 0}, "
                      f"entries over bound {len(bad)} of {ratio[k].size}: {bad[:12].tolist()}", flush=True)
                print("  max|ref|", float(np.max(np.abs(post[key][k]))), "max|err|",
                      float(np.max(np.abs(st[key][k] - post[key][k]))), flush=True)
                if k in xs:
                    # the GPU's own U_new rows of the slice, fed through the same fold in FP64
                    rows = [i for i, kk in enumerate(row_slices) if kk == k]
                    ug = Un[rows]
                    old = pre[key][k] * wl.lam
                    self_ref = old + (ug.T @ xs[k] if key == "Y" else ug.T @ ug)
                    print("  GPU vs fold of its own U in FP64: max|err|",
                          float(np.max(np.abs(st[key][k] - self_ref))), flush=True)
                    print("  U rows err max", float(np.max(np.abs(ug - us[k]))), "|U| max", float(np.max(np.abs(us[k]))),
                          flush=True)
            raise
    worst["fit"] = abs(rep["fit"] - r.fit) / bnd["fit"]
    print(tag, {k: f"{v:.2e}" for k, v in worst.items()}, f"|dfit|={abs(rep['fit'] - r.fit):.2e}", flush=True)
    assert worst["fit"] <= 1.0
    assert rep["committed"] == 1 and rep["K"] == wl.K0 + wl.new_per_step


@pytest.mark.parametrize("name,variants", [("batch_r10", ("wave", "split")), ("batch_r20", ("split",))])
def test_batching_full_size(name, variants, monkeypatch):
    wl, ptr, X, U, o = oracle_run(name)
    b = wl.step(1)
    gpus = {}
    pre = o.state()
    from paper_2305_18376_amd.dash import PREC_FP32
    for v in variants:
        gpus[v] = gpu_update(wl, ptr, X, U, pre, PREC_FP32, v, monkeypatch)
    # both sides from the float32-rounded state the GPU holds
    st0 = {k: np.asarray(pre[k], np.float64) for k in pre}
    st0["Y"] = st0["Y"].astype(np.float32).astype(np.float64)
    st0["D"] = st0["D"].astype(np.float32).astype(np.float64)
    o2 = DashOracle(wl.J, wl.R, wl.lam)
    o2.init_from_state(st0["V"], st0["W"], st0["Y"], st0["D"], st0["n"])
    r = o2.update(b.groups(), b.new_slices())
    for v in variants:
        check(wl, o2, st0, r, b, gpus[v], False, f"{name} {v}")


def test_precision_full_size_fp32_and_mixed(monkeypatch):
    from paper_2305_18376_amd.dash import PREC_FP32, PREC_MIXED
    wl, ptr, X, U, o = oracle_run("precision")
    b = wl.step(1)
    pre = o.state()
    g32 = gpu_update(wl, ptr, X, U, pre, PREC_FP32, "split", monkeypatch)
    gmx = gpu_update(wl, ptr, X, U, pre, PREC_MIXED, "split", monkeypatch)
    st0 = {k: np.asarray(pre[k], np.float64) for k in pre}
    st32 = dict(st0)
    st32["Y"] = st0["Y"].astype(np.float32).astype(np.float64)
    st32["D"] = st0["D"].astype(np.float32).astype(np.float64)
    o32 = DashOracle(wl.J, wl.R, wl.lam)
    o32.init_from_state(st32["V"], st32["W"], st32["Y"], st32["D"], st32["n"])
    r32 = o32.update(b.groups(), b.new_slices())
    check(wl, o32, st32, r32, b, g32, False, "precision fp32")
    # the mixed path keeps the state's low words: it starts from the FP64 state
    omx = DashOracle(wl.J, wl.R, wl.lam)
    omx.init_from_state(st0["V"], st0["W"], st0["Y"], st0["D"], st0["n"])
    rmx = omx.update(b.groups(), b.new_slices())
    check(wl, omx, st0, rmx, b, gmx, True, "precision mixed")
    # the benchmark's bar on the fit
    assert abs(gmx[0]["fit"] - rmx.fit) <= 1e-3
