"""A-priori, element-wise error bounds for one teacher-forced update of the GPU
path against the FP64 oracle (test helper; not collected).

The GPU starts from the oracle's state rounded to float32 (Y_k, D_k; n_k, W, V
stay float64), runs one ALS pass in float32 (or with BF16 row products in the
mixed-precision path) and solves every R x R system in float64.  Each bound
below is the first-order rounding-error bound of the operation that produces
the element -- the sum of |a||b| over its products times the unit roundoff and
the product length -- propagated through the next operation the same way
(Higham, "Accuracy and Stability of Numerical Algorithms", Sec. 3.1 for sums of
products, Sec. 7.2 for the componentwise perturbation of a linear system).
Every quantity the bounds use comes from the oracle, never from the GPU.

  U_new (Lemma 1):   |dU| <= (J + 4) u |X| |P| / |w|,  P = V (V^T V)^{-1}
                     (BF16 path: + 2 u_b |X| |P| / |w|)
  Y_k, D_k (fold):   |dY| <= u (2 s |Y_old| + |Y|) + (m + 2) u |U|^T |X| + |dU|^T |X|
                     |dD| <= u (2 s |D_old| + |D|) + (m + 2) u |U|^T |U| + |dU|^T |U| + |U|^T |dU|
  c_k:               |dc| <= sum_j (|dY| + u |Y|) |V|
  w_k (Lemma 2):     |dw| <= |M^{-1}| (|dc| + |dM| |w|),  M = V^T V * D_k
  F, G:              |dF| <= sum_k s_k (|dY_k|^T |w_k| + |Y_k|^T |dw_k|),  same for G
  V (Lemma 3):       |dV| <= (|dF| + |V| |dG|) |G^{-1}|
  fit:               |dfit| <= d_loss / (2 sqrt(loss * sum_n))

A safety factor of 4 covers second-order terms; the tests assert each element
against its bound (plus a floor of 1e-30 for exact zeros).
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
UB = 2.0 ** -8        # a product of two BF16-rounded operands (2^-9 each)
UC = 2.0 ** -33       # the mixed path's Y pair: float32 word plus the residual rounded to BF16 (2^-24 * 2^-9)
SAFETY = 4.0


def update_bounds(pre, post, lam, xs, us, mixed=False):
    """pre/post: oracle states (dicts of V, W, Y, D, n) before and after the
    update; xs, us: {slice: X_new}, {slice: U_new} of the update (oracle);
    lam: forgetting factor.  The slices of xs were folded; others decayed.
    Returns a dict of bound arrays shaped like the post state, plus 'U' (a
    dict per slice) and 'fit' (a scalar)."""
    V0 = pre["V"]
    W0 = pre["W"]
    J, R = V0.shape
    K = post["W"].shape[0]
    K_old = pre["W"].shape[0]
    VtV = V0.T @ V0
    P = V0 @ np.linalg.pinv(VtV)
    prod_u = U32 if not mixed else U32 + UB
    bU = {}
    for k, X in xs.items():
        w = W0[k] if k < K_old else np.ones(R)
        w_abs = np.where(np.abs(w) > 0, np.abs(w), np.inf)
        bU[k] = SAFETY * ((J + 4) * U32 + (2 * UB if mixed else 0.0)) * (np.abs(X) @ np.abs(P)) / w_abs
    # state after the fold
    Yp, Dp = post["Y"], post["D"]
    bY = np.zeros_like(Yp)
    bD = np.zeros_like(Dp)
    for k in range(K):
        Y_old = pre["Y"][k] if k < K_old else np.zeros((R, J))
        D_old = pre["D"][k] if k < K_old else np.zeros((R, R))
        if k in xs:
            X, U = xs[k], us[k]
            m = X.shape[0]
            # the mixed path keeps a compensation word: BF16 for Y, float32 for D
            store = UC if mixed else U32
            store_d = 0.0 if mixed else U32
            bY[k] = store * (2 * lam * np.abs(Y_old) + np.abs(Yp[k])) + U32 * np.abs(Yp[k]) \
                + (m + 2) * prod_u * (np.abs(U).T @ np.abs(X)) + bU[k].T @ np.abs(X)
            bD[k] = store_d * (2 * lam * np.abs(D_old) + np.abs(Dp[k])) + U32 * np.abs(Dp[k]) \
                + (m + 2) * prod_u * (np.abs(U).T @ np.abs(U)) + bU[k].T @ np.abs(U) + np.abs(U).T @ bU[k]
        else:
            bY[k] = 2 * U32 * np.abs(Yp[k])
            bD[k] = 2 * U32 * np.abs(Dp[k])
    bY *= SAFETY
    bD *= SAFETY
    # Lemma 2 per slice, with the pass's V (the pre-update V)
    Wp = post["W"]
    bW = np.zeros_like(Wp)
    absV = np.abs(V0)
    for k in range(K):
        M = VtV * Dp[k]
        Minv = np.linalg.pinv(M)
        dc = np.einsum("rj,jr->r", bY[k] + U32 * np.abs(Yp[k]), absV)
        dM = np.abs(VtV) * (bD[k] + U32 * np.abs(Dp[k]))
        bW[k] = SAFETY * np.abs(Minv) @ (dc + dM @ np.abs(Wp[k]))
    # Lemma 3
    sig = np.ones(K)   # every slice's state is already decayed in the oracle's post state
    absW = np.abs(Wp)
    dF = np.einsum("k,krj,kr->jr", sig, bY, absW) + np.einsum("k,krj,kr->jr", sig, np.abs(Yp), bW)
    dG = np.einsum("k,kr,ks,krs->rs", sig, absW, absW, bD) + 2 * np.einsum("k,kr,ks,krs->rs", sig, bW, absW,
                                                                              np.abs(Dp))
    F = np.einsum("krj,kr->jr", Yp, Wp)
    G = np.einsum("kr,ks,krs->rs", Wp, Wp, Dp)
    Vp = post["V"]
    bV = SAFETY * (dF + np.abs(Vp) @ dG) @ np.abs(np.linalg.pinv(G))
    sum_n = float(np.sum(post["n"]))
    VtVp = Vp.T @ Vp
    loss = sum_n - 2 * float(np.sum(Vp * F)) + float(np.sum(VtVp * G))
    d_loss = 2 * float(np.sum(bV * np.abs(F))) + 2 * float(np.sum(np.abs(Vp) * dF)) \
        + float(np.sum((2 * np.abs(Vp).T @ bV) * np.abs(G))) + float(np.sum(np.abs(VtVp) * dG))
    b_fit = SAFETY * d_loss / (2 * np.sqrt(max(loss, 1e-300) * sum_n)) if sum_n > 0 else 0.0
    return dict(U=bU, Y=bY, D=bD, W=bW, V=bV, n=1e-12 * np.abs(post["n"]) + 1e-300, fit=b_fit)


def assert_within(name, got, want, bound, floor=1e-30):
    """Every element: |got - want| <= bound + floor.  Reports the worst ratio."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    bound = np.asarray(bound, dtype=np.float64)
    err = np.abs(got - want)
    ratio = err / (bound + floor)
    worst = float(np.max(ratio)) if ratio.size else 0.0
    assert np.all(np.isfinite(got)), f"{name}: non-finite values"
    assert worst <= 1.0, (f"{name}: worst error/bound {worst:.3g} at {np.unravel_index(np.argmax(ratio), ratio.shape)}"
                          f" err={err.flat[np.argmax(ratio)]:.3g} bound={bound.flat[np.argmax(ratio)]:.3g}")
    return worst
