"""Pins of the oracle's singular-system branches and of the lagged helper
terms built from given factors.

Where a system of Lemma 1 (S_k V^T V S_k), Lemma 2 (V^T V * D_k) or Lemma 3
(G) is singular the oracle takes the eigen pseudo-inverse (reading of the
singular cases: Cholesky when every pivot passes, else the pseudo-inverse with
a 1e-12 relative eigenvalue cutoff).  That choice picks the minimum-norm
least-squares solution of each sub-problem, which ``np.linalg.lstsq`` computes
from an SVD of the explicit design: the pins compare against that, on inputs
built so that the singular branch must be taken, and count the branch entries
so that a pin cannot pass without exercising them.  (A shortcut that inverts
S_k entry-wise with 1/w := 0 for a zero weight fails the zero-weight pin: it
projects with the inverse of all of V^T V instead of that of the kept
columns.)
"""
import numpy as np
import pytest

import oracle.dash_oracle as od
from oracle.dash_oracle import DashOracle


def kr(A, B):
    """Khatri-Rao product, rows indexed (i_A, i_B) with B fastest."""
    return np.stack([np.kron(A[:, r], B[:, r]) for r in range(A.shape[1])], axis=1)


def vec(X):
    return X.flatten(order="F")


@pytest.fixture
def branches(monkeypatch):
    """Counts entries into the pseudo-inverse fallback."""
    count = {"pinv": 0}
    real_pinv = od.pinv_psd

    def pinv(M):
        count["pinv"] += 1
        return real_pinv(M)

    monkeypatch.setattr(od, "pinv_psd", pinv)
    return count


def planted(seed, K0, J, R, m=7):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((J, R))
    W = rng.uniform(0.5, 1.5, size=(K0, R))
    Us = [rng.standard_normal((m + k % 3, R)) for k in range(K0)]
    Xs = [(U * W[k]) @ V.T + 0.05 * rng.standard_normal((U.shape[0], J)) for k, U in enumerate(Us)]
    return rng, V, W, Us, Xs


def history_w_lstsq(blocks, V, lam, now):
    """Brute-force W(k,:): weighted lstsq on the explicit Khatri-Rao design over
    every (step, X, U) block of the slice (proof of Lemma 2); minimum norm."""
    A = np.vstack([np.sqrt(lam ** (now - t)) * kr(V, U) for t, X, U in blocks])
    b = np.concatenate([np.sqrt(lam ** (now - t)) * vec(X) for t, X, U in blocks])
    return np.linalg.lstsq(A, b, rcond=None)[0]


def test_new_slice_of_zero_rows_takes_pinv_and_gets_zero_weight(branches):
    """A new slice whose rows are all zero: its U_new rows are 0, D_k = 0, and
    (V^T V * D_k) = 0 sends Lemma 2 to the pseudo-inverse, whose minimum-norm
    answer w_k = 0 is what lstsq gives on the all-zero Khatri-Rao design.  The
    next update brings real rows to that slice: with S_k = 0 Lemma 1's system
    S_k V^T V S_k is zero too, and U_new = 0 is the minimum-norm least-squares
    solution of x ~ u S_k V^T."""
    rng, V, W, Us, Xs = planted(1, K0=5, J=9, R=3)
    o = DashOracle(9, 3, 0.8)
    o.init_from_factors(Xs, Us, W, V)
    zero = np.zeros((4, 9))
    r = o.update([], [zero])
    k = 5
    np.testing.assert_array_equal(r.U_new_slices[0], np.zeros((4, 3)))
    np.testing.assert_array_equal(o.D[k], np.zeros((3, 3)))
    assert branches["pinv"] >= 1          # Lemma 2 (D_k = 0); Lemma 1 has S_k = I, a regular system
    w_ref = history_w_lstsq([(1, zero, r.U_new_slices[0])], o.V, 0.8, 1)
    np.testing.assert_array_equal(w_ref, np.zeros(3))
    np.testing.assert_array_equal(o.W[k], w_ref)
    # next update: real rows for the zero-weight slice
    X2 = rng.standard_normal((3, 9))
    before = dict(branches)
    r2 = o.update([(k, X2), (0, rng.standard_normal((2, 9)))], [], record=True)
    p = r2.passes[-1]
    assert branches["pinv"] >= before["pinv"] + 2   # Lemma 1 with S_k = 0, Lemma 2
    A = p["V_in"] @ np.diag(p["W_in"][k])
    u_ref = np.linalg.lstsq(A, X2.T, rcond=None)[0].T
    np.testing.assert_allclose(r2.U_groups[0], u_ref, atol=1e-14)
    assert np.max(np.abs(r2.U_groups[0])) <= 1e-12


def test_zero_weight_column_zeroes_u_column_and_solves_by_pinv(branches):
    """A new slice started with a weight vector that has a zero entry r0: Lemma 1's
    S_k V^T V S_k is singular; its pseudo-inverse gives the minimum-norm lstsq
    solution, whose column r0 is 0 (column r0 of the design V S_k is zero) and
    whose other columns project on the kept columns of V only.  D_k then has a zero row and
    column r0, (V^T V * D_k) is singular, and the pseudo-inverse gives w_r0 = 0:
    the minimum-norm lstsq on the Khatri-Rao design, whose column r0 is zero."""
    rng, V, W, Us, Xs = planted(2, K0=6, J=10, R=4)
    o = DashOracle(10, 4, 0.9)
    o.init_from_factors(Xs, Us, W, V)
    o.new_slice_w = np.array([1.2, 0.0, 0.7, 1.0])
    Xn = (rng.standard_normal((6, 4)) * [1.0, 0.5, 1.5, 0.8]) @ V.T
    r = o.update([(1, Xs[1][:2])], [Xn], record=True)
    p = r.passes[-1]
    k = 6
    assert branches["pinv"] >= 2
    A = p["V_in"] @ np.diag(p["W_in"][k])
    u_ref = np.linalg.lstsq(A, Xn.T, rcond=None)[0].T
    np.testing.assert_allclose(r.U_new_slices[0], u_ref, rtol=1e-10, atol=1e-12)
    assert np.max(np.abs(r.U_new_slices[0][:, 1])) <= 1e-12 * np.max(np.abs(r.U_new_slices[0]))
    w_ref = history_w_lstsq([(1, Xn, r.U_new_slices[0])], p["V_in"], 0.9, 1)
    np.testing.assert_allclose(p["W_out"][k], w_ref, rtol=1e-9, atol=1e-12)
    assert abs(p["W_out"][k][1]) <= 1e-12 * np.max(np.abs(p["W_out"][k]))


def test_rank_deficient_V_u_v_and_w_steps_are_minimum_norm(branches):
    """V with two equal columns: V^T V is singular, so with S_k = I Lemma 1's
    system is singular and u = x V (V^T V)^+ is the minimum-norm lstsq solution
    of x ~ u V^T.  Lemma 2's Hadamard systems stay regular here (the Schur
    product of a positive definite D_k with the positive semi-definite V^T V of
    positive diagonal), and every W(k,:) is the weighted lstsq over the slice's
    rows; V = F G^{-1} is the lstsq over the stacked rows."""
    rng = np.random.default_rng(3)
    J, R, K0 = 8, 3, 4
    V = rng.standard_normal((J, R))
    V[:, 2] = V[:, 1]
    W = np.ones((K0, R))
    Us = [rng.standard_normal((6, R)) for _ in range(K0)]
    Xs = [U @ V.T + 0.1 * rng.standard_normal((6, J)) for U in Us]
    o = DashOracle(J, R, 0.7)
    o.init_from_factors(Xs, Us, W, V)
    groups = [(k, rng.standard_normal((3, J))) for k in range(K0)]
    r = o.update(groups, [], record=True)
    p = r.passes[-1]
    assert branches["pinv"] >= K0         # Lemma 1 for every slice
    for (k, X), U in zip(groups, r.U_groups):
        u_ref = np.linalg.lstsq(V, X.T, rcond=None)[0].T
        np.testing.assert_allclose(U, u_ref, rtol=1e-9, atol=1e-11)
    hist = {k: [(0, Xs[k], Us[k])] for k in range(K0)}
    for (k, X), U in zip(groups, r.U_groups):
        hist[k].append((1, X, U))
    for k in range(K0):
        w_ref = history_w_lstsq(hist[k], p["V_in"], 0.7, 1)
        np.testing.assert_allclose(p["W_out"][k], w_ref, rtol=1e-7, atol=1e-9)
    A = np.vstack([np.sqrt(0.7 ** (1 - t)) * (U @ np.diag(p["W_out"][k])) for k in hist for t, X, U in hist[k]])
    B = np.vstack([np.sqrt(0.7 ** (1 - t)) * X for k in hist for t, X, U in hist[k]])
    Vt = np.linalg.lstsq(A, B, rcond=None)[0]
    np.testing.assert_allclose(p["V_out"], Vt.T, rtol=1e-7, atol=1e-9)


def test_rank_deficient_V_with_weights_u_is_minimum_norm(branches):
    """With S_k != I and singular V^T V, Lemma 1's pseudo-inverse solution is the
    minimum-norm least-squares solution of ||x - u S_k V^T|| too."""
    rng = np.random.default_rng(4)
    J, R = 9, 4
    V = rng.standard_normal((J, R))
    V[:, 3] = 2.0 * V[:, 0]
    W = rng.uniform(0.5, 1.5, size=(3, R))
    Us = [rng.standard_normal((5, R)) for _ in range(3)]
    Xs = [(U * W[k]) @ V.T for k, U in enumerate(Us)]
    o = DashOracle(J, R, 0.9)
    o.init_from_factors(Xs, Us, W, V)
    X = rng.standard_normal((4, J))
    r = o.update([(1, X)], [], record=True)
    p = r.passes[-1]
    assert branches["pinv"] >= 1
    A = p["V_in"] @ np.diag(p["W_in"][1])
    u_ref = np.linalg.lstsq(A, X.T, rcond=None)[0].T
    np.testing.assert_allclose(r.U_groups[0], u_ref, rtol=1e-8, atol=1e-10)


def test_singular_G_takes_pinv_and_gives_minimum_norm_V(branches):
    """Every slice with a zero weight in column r0 makes G's row and column r0
    zero: V = F G^+ then has a zero column r0, the minimum-norm lstsq answer."""
    rng = np.random.default_rng(5)
    J, R, K0 = 7, 3, 5
    V = rng.standard_normal((J, R))
    W = rng.uniform(0.5, 1.5, size=(K0, R))
    W[:, 2] = 0.0
    Us = [rng.standard_normal((5, R)) for _ in range(K0)]
    Us = [np.where(np.arange(R) == 2, 0.0, U) for U in Us]
    Xs = [(U * W[k]) @ V.T + 0.1 * rng.standard_normal((5, J)) for k, U in enumerate(Us)]
    o = DashOracle(J, R, 0.8)
    o.init_from_factors(Xs, Us, W, V)
    groups = [(k, rng.standard_normal((2, J))) for k in range(K0)]
    r = o.update(groups, [], record=True)
    p = r.passes[-1]
    assert branches["pinv"] >= 1 + 2 * K0   # Lemma 1 and 2 per slice, Lemma 3
    assert np.max(np.abs(p["V_out"][:, 2])) <= 1e-12 * np.max(np.abs(p["V_out"]))
    hist = {k: [(0, Xs[k], Us[k])] for k in range(K0)}
    for (k, X), U in zip(groups, r.U_groups):
        hist[k].append((1, X, U))
    A = np.vstack([np.sqrt(0.8 ** (1 - t)) * (U @ np.diag(p["W_out"][k])) for k in hist for t, X, U in hist[k]])
    B = np.vstack([np.sqrt(0.8 ** (1 - t)) * X for k in hist for t, X, U in hist[k]])
    Vt = np.linalg.lstsq(A, B, rcond=None)[0]
    np.testing.assert_allclose(p["V_out"], Vt.T, rtol=1e-8, atol=1e-10)


def test_spd_solve_accepts_and_rejects_like_cholesky(branches):
    """The acceptance rule: a matrix whose smallest Cholesky pivot is above 1e-12
    of the largest diagonal entry is solved directly (no pinv); one below it,
    or indefinite, goes to the pseudo-inverse, which returns the minimum-norm
    solution of the consistent system."""
    rng = np.random.default_rng(6)
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    good = Q @ np.diag([4.0, 2.0, 1.0, 1e-6]) @ Q.T
    b = rng.standard_normal(4)
    np.testing.assert_allclose(od.spd_solve(good, b), np.linalg.solve(good, b), rtol=1e-8)
    assert branches["pinv"] == 0
    sing = Q @ np.diag([4.0, 2.0, 1.0, 0.0]) @ Q.T
    bc = sing @ rng.standard_normal(4)            # consistent right-hand side
    x = od.spd_solve(sing, bc)
    assert branches["pinv"] == 1
    np.testing.assert_allclose(x, np.linalg.lstsq(sing, bc, rcond=None)[0], rtol=1e-8, atol=1e-12)
    np.testing.assert_array_equal(od.spd_solve(np.zeros((3, 3)), np.ones(3)), np.zeros(3))
    assert branches["pinv"] == 2


def test_lagged_helpers_from_given_factors_equal_explicit_sums():
    """eq. [updateC_init]-[updateG_init] from caller-given factors: c_k is
    vec(X_k)^T (V kr U_k) on the explicit Khatri-Rao design; F and G are the sums
    over every row x_i, u_i of x_i^T (u_i * w_k) and (u_i * w_k)^T (u_i * w_k)."""
    rng, V, W, Us, Xs = planted(7, K0=5, J=6, R=3)
    o = DashOracle(6, 3, 0.8, mode="lagged")
    o.init_from_factors(Xs, Us, W, V)
    F = np.zeros((6, 3))
    G = np.zeros((3, 3))
    for k, (X, U) in enumerate(zip(Xs, Us)):
        np.testing.assert_allclose(o.c[k], vec(X) @ kr(V, U), rtol=1e-12, atol=1e-12)
        for i in range(X.shape[0]):
            z = U[i] * W[k]
            F += np.outer(X[i], z)
            G += np.outer(z, z)
    np.testing.assert_allclose(o.F, F, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(o.G, G, rtol=1e-12, atol=1e-12)


def test_lagged_update_from_given_factors_equals_history_with_past_factors():
    """Lagged mode started by init_from_factors: after several updates c_k, F, G
    equal the forgetting-weighted sums over all rows evaluated with the factors
    in force when each block arrived (the given ones for the initial rows)."""
    rng, V, W, Us, Xs = planted(8, K0=5, J=7, R=3)
    lam = 0.75
    o = DashOracle(7, 3, lam, mode="lagged")
    o.init_from_factors(Xs, Us, W, V)
    hist = [(k, 0, X, U, V, W[k]) for k, (X, U) in enumerate(zip(Xs, Us))]
    for s in range(1, 4):
        K_old = o.K
        groups = [(k, rng.standard_normal((int(rng.integers(0, 4)), 7))) for k in range(K_old)]
        news = [rng.standard_normal((3, 7))]
        r = o.update(groups, news, record=True)
        p = r.passes[-1]
        for l, (X, U) in enumerate(zip(news, r.U_new_slices)):
            hist.append((K_old + l, s, X, U, p["V_in"], p["W_out"][K_old + l]))
        for (k, X), U in zip(groups, r.U_groups):
            if X.shape[0]:
                hist.append((k, s, X, U, p["V_in"], p["W_out"][k]))
    now = o.steps
    F = sum(lam ** (now - t) * X.T @ U @ np.diag(w) for k, t, X, U, Vt, w in hist)
    G = sum(lam ** (now - t) * np.diag(w) @ U.T @ U @ np.diag(w) for k, t, X, U, Vt, w in hist)
    np.testing.assert_allclose(o.F, F, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(o.G, G, rtol=1e-9, atol=1e-10)
    for k in range(o.K):
        c = sum(lam ** (now - t) * (vec(X) @ kr(Vt, U)) for kk, t, X, U, Vt, w in hist if kk == k)
        np.testing.assert_allclose(o.c[k], c, rtol=1e-9, atol=1e-10)
