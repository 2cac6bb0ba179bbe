"""FP64 CPU oracle of the dual-way streaming PARAFAC2 update (DASH).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product (the HIP
library and its Python binding) never does, and shares no code with it.

Plain numpy float64, per-slice Python loops, no blocking, fusion or reordering
beyond the paper's own equations.  Notation follows the paper:

  slices X_k (I_k x J), model X_k ~ U_k S_k V^T with S_k = diag(W(k,:)),
  U_k free (the U_k = Q_k H constraint is dropped, Sec. 2.1), forgetting
  factor lambda (Sec. 3.1, eq. [new_loss]).

State kept between updates (the "helper" terms of Sec. 3.2, stored in the form
that evaluates the lemmas exactly; see ``DashOracle``):

  Y_k = sum over past rows of lambda^age * U_k^T X_k        (R x J)
  D_k = sum over past rows of lambda^age * U_k^T U_k        (R x R)  [obtain_CandD]
  n_k = sum over past rows of lambda^age * ||x||^2

Readings of passages that are silent, ambiguous or garbled (each is also listed
in the design notes of the repository):

  * lambda compounds: data that arrived t updates ago carry weight lambda^t, and
    every slice decays at every (non-empty) update (eq. [obtain_CandC],
    [obtain_CandD], [obtain_FandF], [obtain_FandG]).
  * "exact" stats mode (default): c_k, F and G are evaluated from Y_k, D_k with the
    *current* V and W, which is what Lemmas 2 and 3 state (eq. [updateC],
    [updateF], [updateG]).  "lagged" mode applies Algorithm 1's recursions
    verbatim: the old part of c_k, F, G is the value stored at the previous
    update, scaled by lambda.
  * a new slice's S_k, needed by Lemma 1 before it exists, starts at the identity.
  * singular systems (S_k V^T V S_k of Lemma 1, V^T V * D_k of Lemma 2, G of
    Lemma 3): Cholesky, with the eigen pseudo-inverse (cutoff 1e-12 of the
    largest eigenvalue) when a pivot is not positive enough.  Every solve is
    then the minimum-norm least-squares solution of its sub-problem; in
    particular a zero weight in S_k is not inverted (Lemma 1 is written with
    S_k V^T V S_k, not with S_k^{-1}).
  * an update with no rows is a no-op (no decay).
  * the initial decomposition (Sec. 3.2.1 "Initialization") is PARAFAC2-ALS:
    V0 = top-R eigenvectors of sum_k X_k^T X_k (sign: largest-magnitude entry of
    each column positive), H = I, W = 1, then per iteration the orthogonal
    Procrustes step Q_k = polar(X_k V S_k H^T) and one CP-ALS sweep
    H -> V -> W on Y_k = Q_k^T X_k.
  * the fit is 1 - sqrt(loss)/sqrt(sum_k n_k), loss being eq. [new_loss] with
    compounding weights, evaluated in closed form from the state.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
from scipy.linalg import cho_solve

PIVOT_REL = 1e-12      # Cholesky pivot threshold, relative to the largest diagonal entry
EIG_CUTOFF = 1e-12     # pseudo-inverse / inverse-square-root eigenvalue cutoff (relative)


# ---------------------------------------------------------------------------
# small dense helpers (the R x R inverses of Lemmas 1-3)
# ---------------------------------------------------------------------------
def spd_solve(M: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve M x = b for symmetric positive (semi-)definite M.

    Cholesky when every pivot exceeds PIVOT_REL * max diag(M); otherwise the
    eigen pseudo-inverse with relative cutoff EIG_CUTOFF.  ``b`` may be a vector
    or a matrix of right-hand sides (columns).
    """
    M = np.asarray(M, dtype=np.float64)
    dmax = float(np.max(np.diag(M))) if M.size else 0.0
    if dmax > 0.0:
        try:
            L = np.linalg.cholesky(M)
            if np.min(np.diag(L)) ** 2 > PIVOT_REL * dmax:
                return cho_solve((L, True), b)
        except np.linalg.LinAlgError:
            pass
    return pinv_psd(M) @ b


def pinv_psd(M: np.ndarray) -> np.ndarray:
    lam, Z = np.linalg.eigh(M)
    top = np.max(np.abs(lam)) if lam.size else 0.0
    keep = lam > EIG_CUTOFF * top if top > 0 else np.zeros_like(lam, dtype=bool)
    return (Z[:, keep] / lam[keep]) @ Z[:, keep].T


def inv_sqrt_psd(P: np.ndarray):
    """(P^{+1/2}, Pi) for symmetric PSD P: inverse square root on the retained
    eigenspace and the projector onto it (Pi = P^{+1/2} P P^{+1/2})."""
    lam, Z = np.linalg.eigh(P)
    top = np.max(lam) if lam.size else 0.0
    keep = lam > EIG_CUTOFF * top if top > 0 else np.zeros_like(lam, dtype=bool)
    Zk = Z[:, keep]
    return (Zk / np.sqrt(lam[keep])) @ Zk.T, Zk @ Zk.T


def top_eigvecs(Gm: np.ndarray, R: int) -> np.ndarray:
    """Top-R eigenvectors of a symmetric matrix, descending eigenvalues, each
    column signed so that its entry of largest magnitude is positive."""
    lam, Z = np.linalg.eigh(Gm)
    order = np.argsort(lam)[::-1][:R]
    V = Z[:, order].copy()
    for r in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, r])))
        if V[i, r] < 0:
            V[:, r] = -V[:, r]
    return V


# ---------------------------------------------------------------------------
# initial decomposition: PARAFAC2-ALS (the paper initialises with SPARTan, a
# PARAFAC2-ALS for sparse inputs; Sec. 3.2.1)
# ---------------------------------------------------------------------------
@dataclass
class Parafac2Result:
    V: np.ndarray
    W: np.ndarray
    H: np.ndarray
    Y: list            # Q_k^T X_k from the last Procrustes step
    Pinv_sqrt: list    # (A_k^T A_k)^{+1/2}
    Pi: list           # Q_k^T Q_k (identity when A_k has full column rank)
    A_factor: list     # V diag(w_k) H^T used to form A_k in the last Procrustes step
    losses: list
    iters: int

    def U(self, slices):
        """U_k = Q_k H with Q_k = X_k (V diag(w_k) H^T)(A_k^T A_k)^{+1/2}."""
        return [X @ (self.A_factor[k] @ self.Pinv_sqrt[k]) @ self.H for k, X in enumerate(slices)]


def parafac2_als(slices, R: int, max_iter: int = 10, tol: float = 1e-10, V0=None,
                 W0=None, H0=None) -> Parafac2Result:
    """PARAFAC2-ALS (Kiers, ten Berge & Bro, 1999) on {X_k}."""
    K = len(slices)
    J = slices[0].shape[1]
    X64 = [np.asarray(X, dtype=np.float64) for X in slices]
    if V0 is None:
        Gm = np.zeros((J, J))
        for X in X64:
            Gm += X.T @ X
        V = top_eigvecs(Gm, R)
    else:
        V = np.array(V0, dtype=np.float64)
    H = np.eye(R) if H0 is None else np.array(H0, dtype=np.float64)
    W = np.ones((K, R)) if W0 is None else np.array(W0, dtype=np.float64)
    nrm = [float(np.sum(X * X)) for X in X64]
    losses = []
    Y = Pis = Pi = Af = None
    it = 0
    for it in range(1, max_iter + 1):
        # Procrustes step: Q_k = A_k (A_k^T A_k)^{-1/2}, A_k = X_k V S_k H^T; Y_k = Q_k^T X_k
        Y, Pis, Pi, Af = [], [], [], []
        for k, X in enumerate(X64):
            M = V @ np.diag(W[k]) @ H.T
            A = X @ M
            P = A.T @ A
            E = A.T @ X
            Ps, Pk = inv_sqrt_psd(P)
            Y.append(Ps @ E)
            Pis.append(Ps)
            Pi.append(Pk)
            Af.append(M)
        # CP-ALS sweep on the R x J x K tensor with frontal slices Y_k ~ H S_k V^T
        WtW = W.T @ W
        M1 = np.zeros((R, R))
        for k in range(K):
            M1 += Y[k] @ V @ np.diag(W[k])
        H = spd_solve((V.T @ V) * WtW, M1.T).T
        M2 = np.zeros((J, R))
        for k in range(K):
            M2 += Y[k].T @ H @ np.diag(W[k])
        V = spd_solve((H.T @ H) * WtW, M2.T).T
        Mw = (H.T @ H) * (V.T @ V)
        loss = 0.0
        for k in range(K):
            c = np.diag(H.T @ Y[k] @ V)
            W[k] = spd_solve(Mw, c)
            # ||X_k - Q_k H S_k V^T||^2 expanded with Q_k^T Q_k = Pi_k
            loss += nrm[k] - 2.0 * W[k] @ c + W[k] @ (((H.T @ Pi[k] @ H) * (V.T @ V)) @ W[k])
        losses.append(loss)
        if len(losses) > 1 and abs(losses[-2] - losses[-1]) <= tol * abs(losses[-1]):
            break
    return Parafac2Result(V, W, H, Y, Pis, Pi, Af, losses, it)


# ---------------------------------------------------------------------------
# the streaming update (Algorithm 1 with Lemmas 1-3)
# ---------------------------------------------------------------------------
@dataclass
class UpdateResult:
    U_groups: list           # U_new rows per existing-slice group, ingest order
    U_new_slices: list       # U_new rows per new slice
    first_new_id: int
    fit: float
    loss: float
    sum_n: float
    rows: int
    passes: list = field(default_factory=list)   # per-pass record when requested


class DashOracle:
    """Streaming state and update of DASH in float64.

    ``mode="exact"`` evaluates Lemma 2's c_k and Lemma 3's F, G from the stored
    Y_k, D_k with the current factors; ``mode="lagged"`` uses Algorithm 1's
    recursions (eq. [obtain_CandC], [obtain_FandF], [obtain_FandG]) and keeps
    the exact Y_k only to report the fit.
    """

    def __init__(self, J: int, R: int, lam: float, n_iter: int = 1, mode: str = "exact"):
        assert 0.0 < lam <= 1.0 and J >= 1 and R >= 1 and n_iter >= 1
        assert mode in ("exact", "lagged")
        self.J, self.R, self.lam, self.n_iter, self.mode = J, R, float(lam), n_iter, mode
        self.V = None
        self.W = np.zeros((0, R))
        self.Y, self.D, self.n = [], [], []
        self.c = []
        self.F = np.zeros((J, R))
        self.G = np.zeros((R, R))
        self.steps = 0
        # pin hooks: hold V and/or W fixed during updates; starting S_k of new slices
        self.freeze_V = False
        self.freeze_W = False
        self.new_slice_w = None

    @property
    def K(self) -> int:
        return len(self.Y)

    # ----------------------------------------------------------- initial state
    def init_from_factors(self, slices, U_list, W, V):
        """Helper terms of an initial tensor from given factors (eq. [updateC_init],
        [updateD_init], [updateF_init], [updateG_init])."""
        self.V = np.array(V, dtype=np.float64)
        self.W = np.array(W, dtype=np.float64).reshape(len(slices), self.R)
        self.Y, self.D, self.n, self.c = [], [], [], []
        self.F = np.zeros((self.J, self.R))
        self.G = np.zeros((self.R, self.R))
        for k, X in enumerate(slices):
            X = np.asarray(X, dtype=np.float64)
            U = np.asarray(U_list[k], dtype=np.float64)
            self.Y.append(U.T @ X)
            self.D.append(U.T @ U)
            self.n.append(float(np.sum(X * X)))
            # vec(X)^T (V kr U) = diag(U^T X V) with column-major vec
            self.c.append(np.diag(U.T @ X @ self.V).copy())
            S = np.diag(self.W[k])
            self.F += X.T @ U @ S
            self.G += S @ U.T @ U @ S
        self.steps = 0

    def init_from_state(self, V, W, Y, D, n):
        """Load an arbitrary exact-mode state (teacher forcing for parity tests)."""
        self.V = np.array(V, dtype=np.float64)
        self.W = np.array(W, dtype=np.float64)
        self.Y = [np.array(y, dtype=np.float64) for y in Y]
        self.D = [np.array(d, dtype=np.float64) for d in D]
        self.n = [float(v) for v in n]
        self.c = [np.diag(y @ self.V).copy() for y in self.Y]
        self.F, self.G = self._exact_FG()

    def init_parafac2(self, slices, max_iter: int = 10, tol: float = 1e-10, V0=None):
        """Initial decomposition by PARAFAC2-ALS, then hand-off to the streaming state:
        U_k = Q_k H, Y_k = H^T Q_k^T X_k, D_k = H^T (Q_k^T Q_k) H, n_k = ||X_k||^2."""
        res = parafac2_als(slices, self.R, max_iter=max_iter, tol=tol, V0=V0)
        self.V = res.V.copy()
        self.W = res.W.copy()
        self.Y, self.D, self.n = [], [], []
        for k, X in enumerate(slices):
            self.Y.append(res.H.T @ res.Y[k])
            self.D.append(res.H.T @ res.Pi[k] @ res.H)
            X = np.asarray(X, dtype=np.float64)
            self.n.append(float(np.sum(X * X)))
        self.c = [np.diag(y @ self.V).copy() for y in self.Y]
        self.F, self.G = self._exact_FG()
        self.steps = 0
        return res

    # ------------------------------------------------------------- evaluation
    def _exact_FG(self, W=None):
        W = self.W if W is None else W
        F = np.zeros((self.J, self.R))
        G = np.zeros((self.R, self.R))
        for k in range(self.K):
            F += self.Y[k].T @ np.diag(W[k])
            G += np.diag(W[k]) @ self.D[k] @ np.diag(W[k])
        return F, G

    def loss(self) -> float:
        """Eq. [new_loss] (compounding weights) in closed form from the state:
        sum_k n_k - 2 <V, F> + <V^T V, G> with F, G from Y_k, D_k and the current W."""
        F, G = self._exact_FG()
        return float(sum(self.n) - 2.0 * np.sum(self.V * F) + np.sum((self.V.T @ self.V) * G))

    def fit(self) -> float:
        sn = float(sum(self.n))
        return 1.0 - np.sqrt(max(0.0, self.loss())) / np.sqrt(sn) if sn > 0 else 1.0

    def state(self):
        return dict(V=self.V.copy(), W=self.W.copy(), Y=np.array(self.Y), D=np.array(self.D),
                    n=np.array(self.n))

    # ----------------------------------------------------------------- update
    def update(self, groups=(), new_slices=(), record: bool = False) -> UpdateResult:
        """One update (Algorithm 1).

        ``groups``: [(k, X_block)] new rows of slices, in ingest order (k may name a
        slice created by ``new_slices`` in this same update); ``new_slices``:
        [X_block] whole new slices, which receive ids K, K+1, ... in order.
        Rows of one slice are concatenated in ingest order (new-slice block first).
        """
        groups = [(int(k), np.asarray(X, dtype=np.float64)) for k, X in groups]
        new_slices = [np.asarray(X, dtype=np.float64) for X in new_slices]
        rows = sum(X.shape[0] for _, X in groups) + sum(X.shape[0] for X in new_slices)
        K_old = self.K
        if rows == 0 and not new_slices:
            return UpdateResult([np.zeros((0, self.R)) for _ in groups], [], K_old,
                                self.fit(), self.loss(), float(sum(self.n)), 0)
        lam, R, J = self.lam, self.R, self.J
        # new slices: S_k = I as the starting guess, empty history
        L = len(new_slices)
        for _ in range(L):
            w0 = np.ones((1, R)) if self.new_slice_w is None else np.reshape(self.new_slice_w, (1, R))
            self.W = np.vstack([self.W, w0])
            self.Y.append(np.zeros((R, J)))
            self.D.append(np.zeros((R, R)))
            self.n.append(0.0)
            self.c.append(np.zeros(R))
        K = self.K
        # X_{k,new}: concatenation per slice in ingest order
        parts = {}
        for l, X in enumerate(new_slices):
            parts.setdefault(K_old + l, []).append(X)
        for k, X in groups:
            if not (0 <= k < K):
                raise ValueError(f"slice id {k} out of range")
            parts.setdefault(k, []).append(X)
        Xn = {k: np.concatenate(v, axis=0) for k, v in parts.items() if sum(b.shape[0] for b in v) > 0}
        # old parts, scaled by lambda (the terms loaded "without computation")
        Yo = [lam * y for y in self.Y]
        Do = [lam * d for d in self.D]
        self.n = [lam * v for v in self.n]
        for k, X in Xn.items():
            self.n[k] += float(np.sum(X * X))
        co = [lam * c for c in self.c]
        Fo, Go = lam * self.F, lam * self.G
        passes = []
        Un = {}
        Y, D = list(Yo), list(Do)
        c_new = list(co)
        F = G = None
        for it in range(self.n_iter):
            V_in, W_in = self.V.copy(), self.W.copy()
            VtV = self.V.T @ self.V
            # Lemma 1: U_new = X_new V S_k (S_k V^T V S_k)^{-1}, one R x R system per slice
            Un = {}
            for k, X in Xn.items():
                S = np.diag(self.W[k])
                Un[k] = spd_solve(S @ VtV @ S, (X @ self.V @ S).T).T
            # Lemma 2 with eq. [obtain_CandD]
            Y, D = list(Yo), list(Do)
            for k, U in Un.items():
                Y[k] = Yo[k] + U.T @ Xn[k]
                D[k] = Do[k] + U.T @ U
            c_new = []
            W_out = self.W.copy()
            for k in range(K):
                if self.mode == "exact":
                    ck = np.diag(Y[k] @ self.V).copy()
                else:
                    ck = co[k].copy()
                    if k in Un:
                        ck += np.diag(Un[k].T @ Xn[k] @ self.V)
                c_new.append(ck)
                W_out[k] = spd_solve(VtV * D[k], ck)
            if not self.freeze_W:
                self.W = W_out
            # Lemma 3 with eq. [obtain_FandF], [obtain_FandG]
            if self.mode == "exact":
                F = np.zeros((J, R))
                G = np.zeros((R, R))
                for k in range(K):
                    F += Y[k].T @ np.diag(self.W[k])
                    G += np.diag(self.W[k]) @ D[k] @ np.diag(self.W[k])
            else:
                F, G = Fo.copy(), Go.copy()
                for k, U in Un.items():
                    S = np.diag(self.W[k])
                    F += Xn[k].T @ U @ S
                    G += S @ U.T @ U @ S
            V_out = spd_solve(G, F.T).T
            if not self.freeze_V:
                self.V = V_out
            if record:
                passes.append(dict(V_in=V_in, W_in=W_in, U={k: u.copy() for k, u in Un.items()},
                                   W_out=self.W.copy(), V_out=self.V.copy(), F=F.copy(), G=G.copy(),
                                   Y=[y.copy() for y in Y], D=[d.copy() for d in D], c=[c.copy() for c in c_new]))
        # commit (the U_{k,old} rows are never revisited)
        self.Y, self.D, self.c = Y, D, c_new
        self.F, self.G = F, G
        self.steps += 1
        # outputs in ingest order
        offs = {k: 0 for k in Un}
        U_new_slices = []
        for l, X in enumerate(new_slices):
            k = K_old + l
            m = X.shape[0]
            U_new_slices.append(Un[k][offs[k]:offs[k] + m] if m else np.zeros((0, R)))
            offs[k] = offs.get(k, 0) + m
        U_groups = []
        for k, X in groups:
            m = X.shape[0]
            if m == 0:
                U_groups.append(np.zeros((0, R)))
                continue
            U_groups.append(Un[k][offs[k]:offs[k] + m])
            offs[k] += m
        return UpdateResult(U_groups, U_new_slices, K_old, self.fit(), self.loss(),
                            float(sum(self.n)), rows, passes)

    # ------------------------------------------------------------ application
    def slice_errors(self, groups=(), new_slices=(), result: UpdateResult | None = None):
        """Slice-level reconstruction errors (Definition 1) of the last update's new
        rows, reconstructed with the updated factors U_new S_k V^T; returns
        {k: se_k} over slices that received rows."""
        assert result is not None
        acc = {}
        cnt = {}
        K_old = result.first_new_id
        items = [(K_old + l, X, U) for l, (X, U) in enumerate(zip(new_slices, result.U_new_slices))]
        items += [(k, X, U) for (k, X), U in zip(groups, result.U_groups)]
        for k, X, U in items:
            X = np.asarray(X, dtype=np.float64)
            if X.shape[0] == 0:
                continue
            Xh = U @ np.diag(self.W[k]) @ self.V.T
            acc[k] = acc.get(k, 0.0) + float(np.sum(np.abs(X - Xh)))
            cnt[k] = cnt.get(k, 0) + X.size
        return {k: acc[k] / cnt[k] for k in acc}

    @staticmethod
    def tensor_error(se: dict) -> float:
        """Tensor-level reconstruction error (Definition 2): mean of se over the
        slices that received rows in the update."""
        return float(np.mean(list(se.values()))) if se else 0.0


def moving_threshold(history, window: int = 5) -> float:
    """Anomaly threshold of Sec. 4.5 (Q4): moving mean plus moving standard deviation
    over the previous ``window`` errors (population std)."""
    h = np.asarray(history[-window:], dtype=np.float64)
    if h.size == 0:
        return np.inf
    return float(h.mean() + h.std())
