"""GPU anomaly scores (Sec. 3.4, Definitions 1-2; window-5 threshold of
Sec. 4.5) against the oracle's slice_errors, tensor_error and
moving_threshold, on a stream with injected anomalies.

Both sides run the same stream; at update 5 the rows of a few slices are
replaced by large noise.  Per update: every slice's se_k (GPU, float32 row
products over the updated factors) within 1e-4 relative of the oracle's, te
likewise, and the flags equal wherever the score is not within 1e-3 of its
threshold; the injected slices must be flagged at update 5, and the tensor
level must flag that update.
"""
import numpy as np
import pytest

from oracle.dash_oracle import DashOracle, moving_threshold
from paper_2305_18376_amd.synth import make_workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(params=["wave", "split"])
def variant(request, monkeypatch):
    if request.param == "split":
        monkeypatch.setenv("DASH_VARIANT", "1")
    else:
        monkeypatch.delenv("DASH_VARIANT", raising=False)
    return request.param


def test_scores_and_thresholds_match_oracle(variant):
    from paper_2305_18376_amd.dash import Dash
    wl = make_workload("mid", K0=200, n_steps=8)
    ptr, X, U = wl.init_data(want_u=True)
    g = Dash(wl.J, wl.R, lam=wl.lam, max_slices=wl.K_max + 8, max_rows=1 << 16, max_groups=4096)
    g.init_from_factors(ptr, dev(X), dev(U), dev(wl.W[: wl.K0]), dev(wl.V))
    st = g.get_state()
    o = DashOracle(wl.J, wl.R, wl.lam)
    o.init_from_state(st["V"], st["W"], st["Y"], st["D"], st["n"])
    g.anomaly(5)
    hist, te_hist = {}, []
    rng = np.random.default_rng(7)
    injected = [3, 50, 120]
    for s in range(1, wl.n_steps + 1):
        b = wl.step(s)
        rows = b.rows.copy()
        if s == 5:
            for k in injected:
                gi = int(np.nonzero(b.row_ids == k)[0][0])
                a0, a1 = b.row_ptr[gi], b.row_ptr[gi + 1]
                rows[a0:a1] = 30.0 * rng.standard_normal((a1 - a0, wl.J)).astype(np.float32)
        groups = [(int(b.row_ids[i]), rows[b.row_ptr[i]:b.row_ptr[i + 1]]) for i in range(b.n_groups)]
        g.ingest_slices(b.new_ptr, dev(b.new_rows))
        g.ingest_rows(b.row_ids, b.row_ptr, dev(rows))
        rep = g.update()
        r = o.update(groups, b.new_slices())
        se_o = o.slice_errors(groups, b.new_slices(), result=r)
        te_o = o.tensor_error(se_o)
        sid, se_g, fl_g = g.slice_errors()
        assert sorted(se_o) == list(sid)
        ref = np.array([se_o[k] for k in sid])
        rel = np.abs(se_g - ref) / ref
        assert float(np.max(rel)) <= 1e-4, (s, float(np.max(rel)))
        assert abs(rep["te"] - te_o) <= 1e-4 * te_o
        thr_te = moving_threshold(te_hist, 5)
        te_hist.append(te_o)
        if abs(te_o - thr_te) > 1e-3 * abs(thr_te):
            assert rep["te_anomaly"] == int(te_o > thr_te), (s, te_o, thr_te)
        n_flag = 0
        for k, se, f in zip(sid, se_g, fl_g):
            h = hist.setdefault(int(k), [])
            thr = moving_threshold(h, 5)
            want = int(se_o[k] > thr)
            if not np.isfinite(thr) or abs(se_o[k] - thr) > 1e-3 * abs(thr):
                assert f == want, (s, int(k), float(se), thr)
            h.append(se_o[k])
            n_flag += int(f)
        assert rep["n_anomalies"] == n_flag
        print(s, variant, f"te={rep['te']:.4g} thr={rep['te_threshold']:.4g} flagged={n_flag} "
              f"max rel se err={float(np.max(rel)):.1e}", flush=True)
        if s == 5:
            flagged = {int(k) for k, f in zip(sid, fl_g) if f}
            assert set(injected) <= flagged
            assert rep["te_anomaly"] == 1
