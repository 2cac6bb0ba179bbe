"""GPU parity of the lagged statistics mode (Algorithm 1's recursions verbatim:
eq. [obtain_CandC] for c_k, [obtain_FandF] and [obtain_FandG] for F and G)
against the oracle's lagged mode.

Both sides start from one state (the recursions' starting values are the exact
c_k, F, G of that state) and run free; the GPU's reported fit is the closed
form of eq. [new_loss] evaluated with the lagged F and G, which the test forms
from the oracle's lagged F, G.  The lagged and exact modes coincide while V and
S_k stay fixed and drift apart otherwise: the divergence of the two modes over
the stream is printed.
"""
import numpy as np
import pytest

from oracle.dash_oracle import DashOracle
from paper_2305_18376_amd.synth import make_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def lagged_fit(o):
    sn = float(np.sum(o.n))
    loss = sn - 2.0 * float(np.sum(o.V * o.F)) + float(np.sum((o.V.T @ o.V) * o.G))
    return 1.0 - np.sqrt(max(0.0, loss)) / np.sqrt(sn)


@pytest.mark.parametrize("wl_name,precision,n_iter", [("tiny", 0, 3), ("mid", 0, 1), ("mid", 1, 1)])
def test_lagged_stream_tracks_oracle(wl_name, precision, n_iter):
    from paper_2305_18376_amd.dash import Dash, STATS_LAGGED
    kw = dict(K0=300, n_steps=6) if wl_name == "mid" else {}
    wl = make_workload(wl_name, **kw)
    ptr, X, U = wl.init_data(want_u=True)
    slices = [X[ptr[k]:ptr[k + 1]] for k in range(wl.K0)]
    us = [U[ptr[k]:ptr[k + 1]] for k in range(wl.K0)]
    g = Dash(wl.J, wl.R, lam=wl.lam, n_iter=n_iter, max_slices=wl.K_max + 8, max_rows=1 << 16, max_groups=4096,
             precision=precision, stats_mode=STATS_LAGGED)
    g.init_from_factors(ptr, dev(X), dev(U), dev(wl.W[: wl.K0]), dev(wl.V))
    st = g.get_state()
    o = DashOracle(wl.J, wl.R, wl.lam, n_iter=n_iter, mode="lagged")
    o.init_from_state(st["V"], st["W"], st["Y"], st["D"], st["n"])
    ox = DashOracle(wl.J, wl.R, wl.lam, n_iter=n_iter, mode="exact")
    ox.init_from_state(st["V"], st["W"], st["Y"], st["D"], st["n"])
    tol_u, tol_f = (2e-5, 1e-5) if precision == 0 else (3e-2, 1e-3)
    for s in range(1, wl.n_steps + 1):
        b = wl.step(s)
        g.ingest_slices(b.new_ptr, dev(b.new_rows))
        g.ingest_rows(b.row_ids, b.row_ptr, dev(b.rows))
        rep = g.update()
        r = o.update(b.groups(), b.new_slices())
        rx = ox.update(b.groups(), b.new_slices())
        V, W, Un = g.get_factors()
        ou = np.concatenate([u for u in list(r.U_new_slices) + list(r.U_groups) if u.shape[0]])
        # the gauge-free product U_new S_k for the row comparison
        ids = np.concatenate([np.repeat(np.arange(wl.K_at(s - 1), wl.K_at(s)), np.diff(b.new_ptr)),
                              np.repeat(b.row_ids, np.diff(b.row_ptr))])
        us_g = Un.cpu().numpy() * W.cpu().numpy()[ids]
        us_o = ou * o.W[ids]
        e = dict(US=relerr(us_g, us_o), W=relerr(W.cpu().numpy(), o.W), V=relerr(V.cpu().numpy(), o.V),
                 fit=abs(rep["fit"] - lagged_fit(o)), lag_vs_exact_V=relerr(o.V, ox.V),
                 lag_vs_exact_fit=abs(r.fit - rx.fit))
        print(wl_name, precision, s, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
        assert rep["committed"] == 1
        assert e["US"] <= tol_u and e["W"] <= tol_u and e["V"] <= tol_u, e
        assert e["fit"] <= tol_f, e
