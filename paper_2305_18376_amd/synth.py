"""Seeded synthetic dual-way streams of irregular tensors.

This module only *draws data*: planted PARAFAC2 factors, ragged slice lengths,
per-update arrival counts and noise.  It contains none of the decomposition's
arithmetic and is shared, as plain input, by the FP64 oracle tests, the GPU
parity tests and the benchmark.

Data model (paper, Sec. 2.1 "PARAFAC2 decomposition" and Problem 1): an
irregular tensor {X_k} with slices X_k of shape I_k x J; each update brings new
rows of existing slices (appended below the old rows) and whole new slices
(ids K, K+1, ... in arrival order).  The paper's datasets are not available;
these generators stand in for them with the shapes of its workloads (J = 85..144,
thousands of slices, ragged row counts, 20 % initial period) scaled to the five
workloads below.

All randomness comes from numpy's PCG64 seeded by ``SeedSequence([seed, tag])``
so every step can be regenerated on its own.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = ["StepBatch", "Workload", "make_workload", "WORKLOADS"]


def _rng(seed: int, *tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *tag])))


@dataclass
class StepBatch:
    """One update's worth of new data, in ingest order.

    ``row_ids[g]`` is the existing slice that group ``g`` extends; its rows are
    ``rows[row_ptr[g]:row_ptr[g+1]]``.  New slices follow, one group each, in
    ``new_rows[new_ptr[l]:new_ptr[l+1]]``.
    """
    row_ids: np.ndarray          # int32 [n]
    row_ptr: np.ndarray          # int64 [n+1]
    rows: np.ndarray             # float32 [row_ptr[-1], J]
    new_ptr: np.ndarray          # int64 [L+1]
    new_rows: np.ndarray         # float32 [new_ptr[-1], J]
    true_u: np.ndarray | None = None      # planted U rows for rows (float64), optional
    true_u_new: np.ndarray | None = None  # planted U rows for new_rows

    @property
    def n_groups(self) -> int:
        return int(self.row_ids.shape[0])

    @property
    def n_new(self) -> int:
        return int(self.new_ptr.shape[0] - 1)

    @property
    def M(self) -> int:
        return int(self.row_ptr[-1] + self.new_ptr[-1])

    def groups(self):
        """[(slice_id, X_block)] for existing slices in ingest order."""
        return [(int(self.row_ids[g]), self.rows[self.row_ptr[g]:self.row_ptr[g + 1]])
                for g in range(self.n_groups)]

    def new_slices(self):
        return [self.new_rows[self.new_ptr[l]:self.new_ptr[l + 1]] for l in range(self.n_new)]


def _ptr(counts) -> np.ndarray:
    p = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(np.asarray(counts, dtype=np.int64), out=p[1:])
    return p


@dataclass
class Workload:
    """A seeded dual-way stream: an initial tensor plus ``n_steps`` updates."""
    name: str
    J: int
    R: int
    lam: float
    n_iter: int
    K0: int
    n_steps: int
    seed: int
    noise: float
    # planted truth
    V: np.ndarray = field(repr=False, default=None)      # J x R
    W: np.ndarray = field(repr=False, default=None)      # K_max x R
    H: np.ndarray | None = field(repr=False, default=None)
    init_len: np.ndarray = field(repr=False, default=None)  # K0
    kind: str = "iid"          # "iid" (free U rows) or "qh" (U_k = Q_k H, tiny workload)
    new_per_step: int = 0
    col_scale: np.ndarray | None = field(repr=False, default=None)
    heavy_tail: bool = False
    arrivals: str = "uniform20"  # or "zipf"
    _tiny: dict | None = field(repr=False, default=None)
    # concept drift: update s draws its rows with V_s = (1 - a) V + a V_end,
    # a = min(1, drift * s); the initial tensor uses V (drift = 0: no drift)
    drift: float = 0.0
    V_end: np.ndarray | None = field(repr=False, default=None)

    @property
    def K_max(self) -> int:
        return self.K0 + self.new_per_step * self.n_steps

    def K_at(self, s: int) -> int:
        """Number of slices after update ``s`` (s = 0 is the initial tensor)."""
        return self.K0 + self.new_per_step * s

    # ------------------------------------------------------------------ rows
    def _draw_u(self, rng, n):
        if self.heavy_tail:
            return rng.standard_t(3.0, size=(n, self.R))
        return rng.standard_normal((n, self.R))

    def V_at(self, s: int) -> np.ndarray:
        """The planted V that update ``s`` draws its rows with (s = 0: the initial tensor)."""
        if self.drift <= 0.0 or s == 0:
            return self.V
        a = min(1.0, self.drift * s)
        return (1.0 - a) * self.V + a * self.V_end

    def _rows_for(self, rng, slice_ids: np.ndarray, want_u: bool, V: np.ndarray | None = None):
        """Draw planted rows x = (u * w_k) V^T + e for each entry of slice_ids."""
        n = int(slice_ids.shape[0])
        if n == 0:
            z = np.zeros((0, self.J), dtype=np.float32)
            return z, (np.zeros((0, self.R)) if want_u else None)
        u = self._draw_u(rng, n)
        w = self.W[slice_ids]
        x = (u * w) @ (self.V if V is None else V).T
        if self.noise > 0:
            sig = self.noise * np.sqrt((w * w).sum(axis=1) * (3.0 if self.heavy_tail else 1.0))
            if self.heavy_tail:
                e = rng.standard_t(3.0, size=x.shape)
            else:
                e = rng.standard_normal(x.shape)
            x += e * sig[:, None]
        if self.col_scale is not None:
            x *= self.col_scale[None, :]
        return x.astype(np.float32), (u if want_u else None)

    # ------------------------------------------------------------ interface
    def init_data(self, want_u: bool = False):
        """Initial tensor: (row_ptr int64[K0+1], X float32[N, J]) [, true U]."""
        if self.kind == "qh":
            t = self._tiny
            X = np.concatenate([t["X"][k][: self.init_len[k]] for k in range(self.K0)]).astype(np.float32)
            ptr = _ptr(self.init_len)
            if want_u:
                U = np.concatenate([t["U"][k][: self.init_len[k]] for k in range(self.K0)])
                return ptr, X, U
            return ptr, X
        ptr = _ptr(self.init_len)
        ids = np.repeat(np.arange(self.K0, dtype=np.int64), self.init_len)
        X = np.empty((int(ptr[-1]), self.J), dtype=np.float32)
        U = np.empty((int(ptr[-1]), self.R)) if want_u else None
        # generate in slice-aligned chunks of ~256k rows to bound temporaries
        bounds = [0]
        acc = 0
        for k in range(self.K0):
            acc += int(self.init_len[k])
            if acc >= 262144:
                bounds.append(k + 1)
                acc = 0
        if bounds[-1] != self.K0:
            bounds.append(self.K0)
        for c in range(len(bounds) - 1):
            a, b = int(ptr[bounds[c]]), int(ptr[bounds[c + 1]])
            x, u = self._rows_for(_rng(self.seed, 1, c), ids[a:b], want_u)
            X[a:b] = x
            if want_u:
                U[a:b] = u
        return (ptr, X, U) if want_u else (ptr, X)

    def init_slices(self):
        ptr, X = self.init_data()
        return [X[ptr[k]:ptr[k + 1]] for k in range(self.K0)]

    def step(self, s: int, want_u: bool = False) -> StepBatch:
        """Update ``s`` (1-based)."""
        assert 1 <= s <= self.n_steps
        if self.kind == "qh":
            return self._tiny_step(s, want_u)
        rng = _rng(self.seed, 2, s)
        K_old = self.K_at(s - 1)
        if self.arrivals == "uniform20":
            cnt = rng.integers(1, 21, size=K_old)
            new_cnt = rng.integers(1, 21, size=self.new_per_step)
        else:
            cnt = _zipf_counts(rng, K_old)
            new_cnt = 1 + _zipf_counts(rng, self.new_per_step)
        keep = np.nonzero(cnt > 0)[0]
        row_ids = keep.astype(np.int32)
        row_ptr = _ptr(cnt[keep])
        ids = np.repeat(keep.astype(np.int64), cnt[keep])
        Vs = self.V_at(s)
        rows, u = self._rows_for(rng, ids, want_u, Vs)
        new_ids = np.repeat(np.arange(K_old, K_old + self.new_per_step, dtype=np.int64), new_cnt)
        new_rows, u_new = self._rows_for(rng, new_ids, want_u, Vs)
        return StepBatch(row_ids, row_ptr, rows, _ptr(new_cnt), new_rows, u, u_new)

    def _tiny_step(self, s, want_u):
        t = self._tiny
        K_old = self.K_at(s - 1)
        row_ids = np.arange(K_old, dtype=np.int32)
        blocks, ublocks = [], []
        for k in range(K_old):
            a = t["shown"][k] + 10 * (s - 1 - t["born"][k])
            blocks.append(t["X"][k][a:a + 10])
            ublocks.append(t["U"][k][a:a + 10])
        row_ptr = _ptr([10] * K_old)
        nb, nu = [], []
        for k in range(K_old, K_old + self.new_per_step):
            nb.append(t["X"][k][: t["shown"][k]])
            nu.append(t["U"][k][: t["shown"][k]])
        new_ptr = _ptr([b.shape[0] for b in nb])
        return StepBatch(row_ids, row_ptr, np.concatenate(blocks).astype(np.float32), new_ptr,
                         np.concatenate(nb).astype(np.float32),
                         np.concatenate(ublocks) if want_u else None,
                         np.concatenate(nu) if want_u else None)


def _zipf_counts(rng, n):
    """Per-slice arrivals with P(c) proportional to (c+1)^-1.2, c in {0..200}."""
    c = np.arange(201)
    p = (c + 1.0) ** -1.2
    p /= p.sum()
    return rng.choice(201, size=n, p=p)


def _lognormal_lengths(rng, n, median, lo, hi, sigma=1.0):
    return np.clip(np.round(np.exp(np.log(median) + sigma * rng.standard_normal(n))), lo, hi).astype(np.int64)


def _tiny(seed=1001, noise=0.01, K0=50, J=20, R=5, n_steps=10, new_per_step=5, lam=0.9, n_iter=3):
    rng = _rng(seed, 0)
    K_max = K0 + new_per_step * n_steps
    H = rng.standard_normal((R, R))
    V = rng.standard_normal((J, R))
    # S_k entries 0.25 + |N(0,1)|: positive, bounded away from zero
    W = 0.25 + np.abs(rng.standard_normal((K_max, R)))
    born = np.zeros(K_max, dtype=np.int64)      # update at which the slice appears (0 = initial)
    shown = np.zeros(K_max, dtype=np.int64)     # rows visible when it appears
    shown[:K0] = rng.integers(50, 201, size=K0)
    for s in range(1, n_steps + 1):
        a = K0 + new_per_step * (s - 1)
        born[a:a + new_per_step] = s
        shown[a:a + new_per_step] = rng.integers(20, 61, size=new_per_step)
    Xs, Us = [], []
    for k in range(K_max):
        # every block a slice shows at once (its initial rows, then each 10-row
        # update) is Q H with its own random orthonormal Q, so the initial tensor
        # is an exact PARAFAC2 tensor (U_k^T U_k = H^T H for all k)
        blocks = [int(shown[k])] + [10] * int(n_steps - born[k])
        U = np.concatenate([np.linalg.qr(rng.standard_normal((m, R)))[0] for m in blocks]) @ H
        X = (U * W[k]) @ V.T
        if noise > 0:
            X = X + noise * rng.standard_normal(X.shape)
        Xs.append(X)
        Us.append(U)
    wl = Workload("tiny", J, R, lam, n_iter, K0, n_steps, seed, noise, V=V, W=W, H=H,
                  init_len=shown[:K0].copy(), kind="qh", new_per_step=new_per_step)
    wl._tiny = {"X": Xs, "U": Us, "born": born, "shown": shown}
    return wl


def _iid(name, seed, J, R, K0, median, lo, hi, lam, n_iter, n_steps, new_per_step, noise,
         arrivals, heavy_tail=False, col_scale=False, drift=0.0):
    rng = _rng(seed, 0)
    K_max = K0 + new_per_step * n_steps
    V = rng.standard_normal((J, R))
    W = rng.uniform(0.5, 1.5, size=(K_max, R))
    init_len = _lognormal_lengths(rng, K0, median, lo, hi)
    cs = 10.0 ** rng.uniform(-3.0, 3.0, size=J) if col_scale else None
    # drawn from a stream of its own, so that the other draws do not depend on it
    V_end = _rng(seed, 7).standard_normal((J, R)) if drift > 0 else None
    return Workload(name, J, R, lam, n_iter, K0, n_steps, seed, noise, V=V, W=W,
                    init_len=init_len, kind="iid", new_per_step=new_per_step, col_scale=cs,
                    heavy_tail=heavy_tail, arrivals=arrivals, drift=drift, V_end=V_end)


WORKLOADS = ("tiny", "mid", "batch_r10", "batch_r20", "precision")


def make_workload(name: str, **kw) -> Workload:
    """Build one of the named workloads; keyword arguments override sizes.

    tiny       planted rank-5 PARAFAC2 (U_k = Q_k H, per-block orthonormal Q), K0=50, I_k~U{50..200}, J=20,
               10 updates of +10 rows per slice and 5 new slices of U{20..60} rows,
               lambda=0.9, 3 ALS passes per update, noise 0.01.
    mid        K0=2000, I_k log-normal (median 800, clip [100,4000]), J=88, R=10,
               100 updates of U{1..20} rows per slice plus 20 new slices, lambda=0.95,
               5 % noise.
    batch_r10  K0=20000, I_k log-normal (median 300, clip [20,5000]), J=128, R=10,
    batch_r20  R=20; truncated-Zipf(1.2) arrivals of 0..200 rows per slice per update.
    precision  as batch with J=256, R=32, Student-t(3) rows and noise, column
               scales 10^U[-3,3].
    drift=d (any iid workload): update s draws its rows with V moved a fraction
               min(1, d s) of the way to a second planted V.
    """
    if name == "tiny":
        return _tiny(**kw)
    base = {
        "mid": dict(seed=1002, J=88, R=10, K0=2000, median=800, lo=100, hi=4000, lam=0.95,
                    n_iter=1, n_steps=100, new_per_step=20, noise=0.05, arrivals="uniform20"),
        "batch_r10": dict(seed=1003, J=128, R=10, K0=20000, median=300, lo=20, hi=5000, lam=0.95,
                          n_iter=1, n_steps=100, new_per_step=20, noise=0.05, arrivals="zipf"),
        "batch_r20": dict(seed=1003, J=128, R=20, K0=20000, median=300, lo=20, hi=5000, lam=0.95,
                          n_iter=1, n_steps=100, new_per_step=20, noise=0.05, arrivals="zipf"),
        "precision": dict(seed=1004, J=256, R=32, K0=20000, median=300, lo=20, hi=5000, lam=0.95,
                          n_iter=1, n_steps=100, new_per_step=20, noise=0.05, arrivals="zipf",
                          heavy_tail=True, col_scale=True),
    }[name]
    base.update(kw)
    return _iid(name, **base)


# --------------------------------------------------------------------------
# Serving workload: many independent streams with Poisson arrivals
# --------------------------------------------------------------------------
@dataclass
class Request:
    """The rows one stream received in one cut window (ingest order): groups
    of existing slices, rows[r0:r1] of the stream's row array, and new slices,
    new_rows[n0:n1] of its new-slice array."""
    t: float                     # window end (seconds of the stream's clock)
    row_ids: np.ndarray          # int32 [n]
    row_ptr: np.ndarray          # int64 [n+1], relative to r0
    r0: int
    r1: int
    new_ptr: np.ndarray          # int64 [L+1], relative to n0
    n0: int
    n1: int

    @property
    def M(self) -> int:
        return (self.r1 - self.r0) + (self.n1 - self.n0)


@dataclass
class ServedStream:
    J: int
    R: int
    lam: float
    K0: int
    V: np.ndarray = field(repr=False)           # J x R
    W: np.ndarray = field(repr=False)           # K_max x R
    init_ptr: np.ndarray = field(repr=False)    # int64 [K0+1]
    init_X: np.ndarray = field(repr=False)      # float32
    init_U: np.ndarray = field(repr=False)      # float64
    rows: np.ndarray = field(repr=False)        # float32 [N, J], every request's rows
    new_rows: np.ndarray = field(repr=False)    # float32 [N_new, J]
    requests: list = field(repr=False, default_factory=list)

    @property
    def K_max(self) -> int:
        return int(self.W.shape[0])


def serving_streams(n_streams=64, seconds=10.0, seed=5000, window=0.025, rate=2000.0, new_rate=2.0,
                    init_median=24, init_hi=200):
    """The serving workload's streams, stream s seeded with seed + s.

    Per stream: J ~ U{32,64,128,256}, R ~ U{8,16,32}, K0 ~ U{500..5000},
    lambda = 0.95; planted rows x = (u * w_k) V^T + 5 % noise (u ~ N(0,1)^R,
    w_k ~ U[0.5,1.5]^R, V ~ N(0,1)).  Rows arrive as a Poisson process of
    `rate` rows per second, each to an existing slice drawn by Zipf(1.2)
    popularity over a random ranking of the slices; new slices arrive as a
    Poisson process of `new_rate` per second with U{1..60} rows.  A request is
    one `window` of a stream's clock (the windows of different streams are
    offset by a random phase).  Initial slices have log-normal lengths of
    median `init_median` (sigma 1, clipped to [R+1, init_hi]): the cost of an
    update depends on the number of slices, not on the rows that built them."""
    out = []
    for s in range(n_streams):
        rng = _rng(seed + s, 0)
        J = int(rng.choice([32, 64, 128, 256]))
        R = int(rng.choice([8, 16, 32]))
        K0 = int(rng.integers(500, 5001))
        n_new_max = int(rng.poisson(new_rate * seconds)) + 1
        K_max = K0 + n_new_max
        V = rng.standard_normal((J, R))
        W = rng.uniform(0.5, 1.5, size=(K_max, R))
        lens = _lognormal_lengths(rng, K0, init_median, R + 1, init_hi)

        def draw(ids, g):
            u = g.standard_normal((len(ids), R))
            w = W[ids]
            x = (u * w) @ V.T
            x += 0.05 * np.sqrt((w * w).sum(axis=1))[:, None] * g.standard_normal(x.shape)
            return x.astype(np.float32), u

        init_ptr = _ptr(lens)
        init_X, init_U = draw(np.repeat(np.arange(K0), lens), _rng(seed + s, 1))
        g = _rng(seed + s, 2)
        rank = g.permutation(K_max)
        # arrival times over the whole run
        n_rows = int(g.poisson(rate * seconds))
        t_rows = np.sort(g.uniform(0.0, seconds, size=n_rows))
        n_new = min(int(g.poisson(new_rate * seconds)), n_new_max)
        t_new = np.sort(g.uniform(0.0, seconds, size=n_new))
        new_len = g.integers(1, 61, size=n_new)
        phase = g.uniform(0.0, window)
        edges = np.arange(phase, seconds + window, window)
        ids_all = np.empty(n_rows, dtype=np.int64)
        reqs = []
        K = K0
        pop_K, cdf = -1, None
        r_at, n_at, i_new = 0, 0, 0
        for e in edges:
            # new slices of this window (they join the ranking at once)
            L0 = i_new
            while i_new < n_new and t_new[i_new] < e:
                i_new += 1
            r_end = int(np.searchsorted(t_rows, e))
            m = r_end - r_at
            if K != pop_K:
                p = (np.argsort(np.argsort(rank[:K])) + 1.0) ** -1.2
                cdf = np.cumsum(p / p.sum())
                pop_K = K
            ids = np.minimum(np.searchsorted(cdf, g.uniform(size=m)), K - 1)
            order = np.argsort(ids, kind="stable")
            ids_all[r_at:r_end] = ids[order]
            uniq, cnt = np.unique(ids, return_counts=True)
            nl = new_len[L0:i_new]
            if m or i_new > L0:
                reqs.append(Request(float(e), uniq.astype(np.int32), _ptr(cnt), r_at, r_end, _ptr(nl), n_at,
                                    n_at + int(nl.sum())))
            r_at = r_end
            n_at += int(nl.sum())
            K += i_new - L0
        rows, _ = draw(ids_all, _rng(seed + s, 3))
        new_ids = np.repeat(np.arange(K0, K0 + n_new), new_len)
        new_rows, _ = draw(new_ids, _rng(seed + s, 4))
        out.append(ServedStream(J, R, 0.95, K0, V, W, init_ptr, init_X, init_U, rows, new_rows, reqs))
    return out
