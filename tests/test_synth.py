"""The seeded input generators (host only): draws are reproducible per update,
and the drift option changes nothing but the planted V that rows are drawn
with."""
import numpy as np

from paper_2305_18376_amd.synth import make_workload


def test_steps_regenerate_on_their_own():
    a = make_workload("mid", n_steps=4, median=24, lo=11, hi=200)
    b = make_workload("mid", n_steps=4, median=24, lo=11, hi=200)
    s3a = a.step(3)
    b.step(1)
    s3b = b.step(3)
    np.testing.assert_array_equal(s3a.rows, s3b.rows)
    np.testing.assert_array_equal(s3a.row_ptr, s3b.row_ptr)


def test_drift_moves_only_the_planted_v():
    base = make_workload("mid", n_steps=30, median=24, lo=11, hi=200)
    dr = make_workload("mid", n_steps=30, median=24, lo=11, hi=200, drift=0.05)
    # the initial tensor and every other draw are those of the stationary stream
    np.testing.assert_array_equal(base.V, dr.V)
    np.testing.assert_array_equal(base.W, dr.W)
    np.testing.assert_array_equal(base.init_data()[1], dr.init_data()[1])
    np.testing.assert_array_equal(dr.V_at(0), dr.V)
    # V_s is the stated interpolation, reaching V_end at s = 20 and staying there
    np.testing.assert_allclose(dr.V_at(4), 0.8 * dr.V + 0.2 * dr.V_end)
    np.testing.assert_array_equal(dr.V_at(20), dr.V_at(30))
    np.testing.assert_allclose(dr.V_at(30), dr.V_end)
    # an update's rows: same arrivals and same u, only V differs
    b0, b1 = base.step(5, want_u=True), dr.step(5, want_u=True)
    np.testing.assert_array_equal(b0.row_ptr, b1.row_ptr)
    np.testing.assert_array_equal(b0.true_u, b1.true_u)
    assert not np.allclose(b0.rows, b1.rows)
    # noise-free check of the V used: rows of a noiseless drifting stream are
    # (u * w_k) V_s^T exactly (up to float32 storage)
    nz = make_workload("mid", n_steps=6, median=24, lo=11, hi=200, drift=0.1, noise=0.0)
    b = nz.step(6, want_u=True)
    ids = np.repeat(b.row_ids.astype(np.int64), np.diff(b.row_ptr))
    x = (b.true_u * nz.W[ids]) @ nz.V_at(6).T
    np.testing.assert_allclose(b.rows, x, rtol=1e-5, atol=1e-5 * np.abs(x).max())
