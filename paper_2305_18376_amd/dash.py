"""Thin ctypes binding of libdash (include/dash.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  PyTorch supplies device memory (input rows, output buffers) and the
stream; host metadata (row pointers, slice ids) is passed as numpy arrays.
The binding refuses to run without the built library -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdash.so")

OK, E_INVALID_ARG, E_OUT_OF_MEMORY, E_BAD_STATE, E_CAPACITY, E_NUMERIC, E_DEVICE, E_IO = range(8)
PREC_FP32, PREC_MIXED = 0, 1
SITE_NONE, SITE_INGEST, SITE_LAUNCH, SITE_COMMIT, SITE_INIT_ALLOC = range(5)   # dash_debug_fail_next
STATS_EXACT, STATS_LAGGED = 0, 1


class DashConfig(C.Structure):
    _fields_ = [
        ("J", C.c_int32), ("R", C.c_int32), ("lam", C.c_double), ("n_iter", C.c_int32),
        ("init_max_iter", C.c_int32), ("init_tol", C.c_double), ("precision", C.c_int32),
        ("stats_mode", C.c_int32), ("max_slices", C.c_int64), ("max_rows_per_update", C.c_int64),
        ("max_groups_per_update", C.c_int64), ("max_init_rows", C.c_int64), ("device", C.c_int32),
        ("stream", C.c_void_p),
    ]


class UpdateReport(C.Structure):
    _fields_ = [("step", C.c_int64), ("rows", C.c_int64), ("K", C.c_int32), ("committed", C.c_int32),
                ("fit", C.c_double), ("loss", C.c_double), ("sum_n", C.c_double), ("device_us", C.c_double),
                ("te", C.c_double), ("te_threshold", C.c_double), ("te_anomaly", C.c_int32),
                ("n_anomalies", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class InitReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("loss", C.c_double), ("fit", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ProfileStats(C.Structure):
    _fields_ = [("updates", C.c_int64), ("pass_launches", C.c_int64), ("reduce_launches", C.c_int64),
                ("solve_launches", C.c_int64), ("commit_launches", C.c_int64), ("upload_launches", C.c_int64),
                ("pass_ms", C.c_double), ("reduce_ms", C.c_double), ("solve_ms", C.c_double),
                ("commit_ms", C.c_double), ("upload_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Dims(C.Structure):
    _fields_ = [("J", C.c_int32), ("R", C.c_int32), ("K", C.c_int32), ("K_pending", C.c_int32),
                ("step", C.c_int64), ("m_last", C.c_int64), ("rows_pending", C.c_int64),
                ("initialized", C.c_int32)]


class Schedule(C.Structure):
    _fields_ = [("variant", C.c_int32), ("spread", C.c_int32), ("fused", C.c_int32), ("solve_div", C.c_int32),
                ("from_cache", C.c_int32), ("tuned", C.c_int32), ("candidates", C.c_int32),
                ("ns_per_kb", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerReport(C.Structure):
    _fields_ = [("stream", C.c_int32), ("committed", C.c_int32), ("step", C.c_int64), ("rows", C.c_int64),
                ("fit", C.c_double), ("latency_us", C.c_double), ("last_request", C.c_int64),
                ("device_us", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double)]

    def as_dict(self):
        return {"name": self.name.decode(), "launches": self.launches, "ms": self.ms, "bytes": self.bytes}


class ServerStats(C.Structure):
    _fields_ = [("ticks", C.c_int64), ("launches", C.c_int64), ("updates", C.c_int64), ("rows", C.c_int64),
                ("budget", C.c_int64), ("used", C.c_int64), ("queued", C.c_int32), ("open", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_SIGS = {
    "dash_config_default": (None, [C.POINTER(DashConfig), C.c_int32, C.c_int32]),
    "dash_create": (C.c_int, [C.POINTER(DashConfig), C.POINTER(_P)]),
    "dash_destroy": (C.c_int, [_P]),
    "dash_init": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.POINTER(InitReport)]),
    "dash_init_from_factors": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P]),
    "dash_init_noalloc": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.POINTER(InitReport)]),
    "dash_init_noalloc_limit": (C.c_size_t, []),
    "dash_ingest_rows": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "dash_ingest_slices": (C.c_int, [_P, C.c_int32, _P, _P, C.POINTER(C.c_int32)]),
    "dash_update": (C.c_int, [_P, C.POINTER(UpdateReport)]),
    "dash_update_async": (C.c_int, [_P]),
    "dash_wait": (C.c_int, [_P, C.POINTER(UpdateReport)]),
    "dash_get_factors": (C.c_int, [_P, _P, _P, _P, C.POINTER(C.c_int64)]),
    "dash_get_dims": (C.c_int, [_P, C.POINTER(Dims)]),
    "dash_get_state": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "dash_set_state": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P]),
    "dash_save": (C.c_int, [_P, C.c_char_p]),
    "dash_load": (C.c_int, [_P, C.c_char_p]),
    "dash_profile": (C.c_int, [_P, C.c_int32]),
    "dash_profile_read": (C.c_int, [_P, C.POINTER(ProfileStats)]),
    "dash_status_string": (C.c_char_p, [C.c_int]),
    "dash_debug_fail_next": (C.c_int, [_P, C.c_int32]),
    "dash_last_error": (C.c_char_p, [_P]),
    "dash_poll": (C.c_int, [_P, C.POINTER(UpdateReport), C.c_int32, C.POINTER(C.c_int32)]),
    "dash_footprint": (C.c_int, [C.POINTER(DashConfig), C.POINTER(C.c_int64)]),
    "dash_anomaly": (C.c_int, [_P, C.c_int32]),
    "dash_get_slice_errors": (C.c_int, [_P, _P, _P, _P, C.c_int32, C.POINTER(C.c_int32)]),
    "dash_spans": (C.c_int, [_P, C.c_int32]),
    "dash_graph": (C.c_int, [_P, C.c_int32]),
    "dash_autotune": (C.c_int, [_P, C.c_int32]),
    "dash_autotune_read": (C.c_int, [_P, C.POINTER(Schedule)]),
    "dash_autotune_cache": (C.c_int, [_P, C.c_char_p]),
    "dash_spans_read": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]),
    "dash_server_create": (C.c_int, [C.c_int32, C.c_int64, C.POINTER(_P)]),
    "dash_server_destroy": (C.c_int, [_P]),
    "dash_server_open": (C.c_int, [_P, C.POINTER(DashConfig), C.c_int32, C.POINTER(C.c_int32)]),
    "dash_server_state": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32)]),
    "dash_server_close": (C.c_int, [_P, C.c_int32]),
    "dash_server_context": (_P, [_P, C.c_int32]),
    "dash_server_submit": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, _P, _P, _P,
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "dash_server_tick": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "dash_server_poll": (C.c_int, [_P, C.c_int32, C.POINTER(ServerReport), C.c_int32, C.POINTER(C.c_int32)]),
    "dash_server_start": (C.c_int, [_P, C.c_int32]),
    "dash_server_stop": (C.c_int, [_P]),
    "dash_server_drain": (C.c_int, [_P, C.c_int32]),
    "dash_server_get_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
    "dash_server_last_error": (C.c_char_p, [_P]),
    "dash_server_profile": (C.c_int, [_P, C.c_int32]),
    "dash_server_profile_read": (C.c_int, [_P, C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int64)]),
}

_lib = None


def lib():
    """Load libdash.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2305_18376_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def make_config(J, R, lam=0.7, n_iter=1, max_slices=65536, max_rows=1 << 20, max_groups=65536,
                max_init_rows=4 << 20, init_max_iter=10, init_tol=1e-10, device=0, precision=PREC_FP32,
                stats_mode=STATS_EXACT):
    cfg = DashConfig()
    lib().dash_config_default(C.byref(cfg), J, R)
    cfg.lam = lam
    cfg.n_iter = n_iter
    cfg.max_slices = max_slices
    cfg.max_rows_per_update = max_rows
    cfg.max_groups_per_update = max_groups
    cfg.max_init_rows = max_init_rows
    cfg.init_max_iter = init_max_iter
    cfg.init_tol = init_tol
    cfg.precision = precision
    cfg.stats_mode = stats_mode
    cfg.device = device
    return cfg


def footprint(**kw):
    """Device bytes of a context with these settings (make_config's keywords)."""
    b = C.c_int64()
    st = lib().dash_footprint(C.byref(make_config(**kw)), C.byref(b))
    if st != OK:
        raise DashError(st, "dash_footprint")
    return b.value


class DashError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} [{lib().dash_status_string(status).decode()}]")
        self.status = status


def _ptr(t) -> int:
    """Device pointer of a contiguous CUDA(HIP) tensor, or host pointer of a numpy array."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags["C_CONTIGUOUS"]
        return t.ctypes.data
    assert t.is_contiguous() and t.is_cuda, "expected a contiguous device tensor"
    return t.data_ptr()


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _init_row_ptr(row_ptr):
    """(K, array) of an initial decomposition's row_ptr: a contiguous int64
    device tensor goes to the library as it is (the library copies it to the
    host), anything else as a host int64 array."""
    if getattr(row_ptr, "is_cuda", False):
        assert str(row_ptr.dtype) == "torch.int64" and row_ptr.dim() == 1, "row_ptr: 1-D int64 tensor"
        return row_ptr.numel() - 1, row_ptr
    rp = _host(row_ptr, np.int64)
    return rp.shape[0] - 1, rp


class Dash:
    """One streaming decomposition (one C context)."""

    def __init__(self, J, R, lam=0.7, n_iter=1, max_slices=65536, max_rows=1 << 20,
                 max_groups=65536, max_init_rows=4 << 20, init_max_iter=10, init_tol=1e-10,
                 device=0, stream=None, precision=PREC_FP32, stats_mode=STATS_EXACT):
        self._owned = True
        cfg = make_config(J, R, lam, n_iter, max_slices, max_rows, max_groups, max_init_rows, init_max_iter,
                          init_tol, device, precision, stats_mode)
        import torch
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        cfg.stream = stream
        h = _P()
        st = L.dash_create(C.byref(cfg), C.byref(h))
        if st != OK:
            raise DashError(st, "dash_create failed")
        self._h = h
        self.J, self.R = J, R
        self.device = device
        self._borrowed = []

    # ------------------------------------------------------------ plumbing
    def _check(self, st, what):
        if st != OK:
            msg = lib().dash_last_error(self._h)
            raise DashError(st, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                lib().dash_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def debug_fail_next(self, site):
        """Make the next call reaching `site` (SITE_INGEST, SITE_LAUNCH,
        SITE_COMMIT, SITE_INIT_ALLOC; SITE_NONE cancels) fail there."""
        self._check(lib().dash_debug_fail_next(self._h, int(site)), "dash_debug_fail_next")

    def dims(self):
        d = Dims()
        self._check(lib().dash_get_dims(self._h, C.byref(d)), "dash_get_dims")
        return d

    # ---------------------------------------------------------------- init
    def init_from_factors(self, row_ptr, X, U, W, V):
        K, rp = _init_row_ptr(row_ptr)
        self._check(lib().dash_init_from_factors(self._h, K, _ptr(rp), _ptr(X), _ptr(U), _ptr(W), _ptr(V)),
                    "dash_init_from_factors")

    def init(self, row_ptr, X, V0=None):
        K, rp = _init_row_ptr(row_ptr)
        rep = InitReport()
        self._check(lib().dash_init(self._h, K, _ptr(rp), _ptr(X), _ptr(V0), C.byref(rep)),
                    "dash_init")
        return rep.as_dict()

    # -------------------------------------------------------------- ingest
    def ingest_rows(self, slice_id, row_ptr, rows):
        sid = _host(slice_id, np.int32)
        rp = _host(row_ptr, np.int64)
        self._check(lib().dash_ingest_rows(self._h, sid.shape[0], _ptr(sid), _ptr(rp), _ptr(rows)),
                    "dash_ingest_rows")
        self._borrowed.append(rows)

    def ingest_slices(self, row_ptr, rows):
        rp = _host(row_ptr, np.int64)
        first = C.c_int32()
        self._check(lib().dash_ingest_slices(self._h, rp.shape[0] - 1, _ptr(rp), _ptr(rows), C.byref(first)),
                    "dash_ingest_slices")
        self._borrowed.append(rows)
        return first.value

    def update(self):
        rep = UpdateReport()
        st = lib().dash_update(self._h, C.byref(rep))
        self._borrowed = []
        self._check(st, "dash_update")
        return rep.as_dict()

    def update_async(self):
        self._check(lib().dash_update_async(self._h), "dash_update_async")

    def autotune(self, trials=2, cache=None):
        """Try every launch schedule `trials` times over the next updates and keep the fastest;
        with `cache` (a file path) a schedule tuned earlier for the same update shape is taken
        at once, and a finished run stores its winner there."""
        self._check(lib().dash_autotune_cache(self._h, str(cache).encode() if cache else None),
                    "dash_autotune_cache")
        self._check(lib().dash_autotune(self._h, int(trials)), "dash_autotune")

    def schedule(self):
        sc = Schedule()
        self._check(lib().dash_autotune_read(self._h, C.byref(sc)), "dash_autotune_read")
        return sc.as_dict()

    def graph(self, enable=True):
        """Replay each update's launches from one HIP graph (node parameters rewritten per update)."""
        self._check(lib().dash_graph(self._h, 1 if enable else 0), "dash_graph")

    def spans(self, enable=True):
        """Record (or stop recording) each update's device span."""
        self._check(lib().dash_spans(self._h, 1 if enable else 0), "dash_spans")

    def spans_read(self, cap=1 << 16):
        buf = (C.c_float * cap)()
        n = C.c_int32()
        self._check(lib().dash_spans_read(self._h, buf, cap, C.byref(n)), "dash_spans_read")
        return np.frombuffer(buf, dtype=np.float32, count=n.value).copy()

    def poll(self, cap=64):
        """Reports of the enqueued updates that have finished (non-blocking)."""
        reps = (UpdateReport * cap)()
        n = C.c_int32()
        st = lib().dash_poll(self._h, reps, cap, C.byref(n))
        out = [reps[i].as_dict() for i in range(n.value)]
        self._check(st, "dash_poll")
        return out

    def wait(self):
        rep = UpdateReport()
        st = lib().dash_wait(self._h, C.byref(rep))
        self._borrowed = []
        self._check(st, "dash_wait")
        return rep.as_dict()

    # ------------------------------------------------------------- outputs
    def get_factors(self):
        import torch
        d = self.dims()
        dev = torch.device("cuda", self.device)
        V = torch.empty((self.J, self.R), dtype=torch.float32, device=dev)
        W = torch.empty((max(d.K, 1), self.R), dtype=torch.float32, device=dev)
        U = torch.empty((max(d.m_last, 1), self.R), dtype=torch.float32, device=dev)
        m = C.c_int64()
        self._check(lib().dash_get_factors(self._h, _ptr(V), _ptr(W), _ptr(U), C.byref(m)), "dash_get_factors")
        return V, W[: d.K], U[: m.value]

    def get_state(self):
        d = self.dims()
        K, J, R = d.K, self.J, self.R
        V = np.empty((J, R))
        W = np.empty((K, R))
        Y = np.empty((K, R, J))
        D = np.empty((K, R, R))
        n = np.empty((K,))
        self._check(lib().dash_get_state(self._h, _ptr(V), _ptr(W), _ptr(Y), _ptr(D), _ptr(n)), "dash_get_state")
        return dict(V=V, W=W, Y=Y, D=D, n=n)

    def set_state(self, V, W, Y, D, n):
        V, W, Y, D, n = (_host(a, np.float64) for a in (V, W, Y, D, n))
        K = W.shape[0]
        assert Y.shape == (K, self.R, self.J) and D.shape == (K, self.R, self.R) and n.shape == (K,)
        self._check(lib().dash_set_state(self._h, K, _ptr(V), _ptr(W), _ptr(Y), _ptr(D), _ptr(n)), "dash_set_state")

    def anomaly(self, window=5):
        """Score every later update (slice-level se_k, tensor-level te, moving
        thresholds over `window` previous scores); 0 turns the scores off."""
        self._check(lib().dash_anomaly(self._h, int(window)), "dash_anomaly")

    def slice_errors(self, cap=1 << 20):
        """(slice ids, se, flags) of the last scored update, ascending slice id."""
        sid = np.empty(cap, np.int32)
        se = np.empty(cap, np.float32)
        fl = np.empty(cap, np.int32)
        n = C.c_int32()
        self._check(lib().dash_get_slice_errors(self._h, _ptr(sid), _ptr(se), _ptr(fl), cap, C.byref(n)),
                    "dash_get_slice_errors")
        return sid[: n.value].copy(), se[: n.value].copy(), fl[: n.value].copy()

    def profile(self, every=1):
        """Time the launches of every `every`-th update (0 or False: stop)."""
        every = int(every) if every is not True else 1
        self._check(lib().dash_profile(self._h, max(0, every)), "dash_profile")

    def profile_read(self):
        st = ProfileStats()
        self._check(lib().dash_profile_read(self._h, C.byref(st)), "dash_profile_read")
        return st.as_dict()

    def save(self, path):
        self._check(lib().dash_save(self._h, str(path).encode()), "dash_save")

    def load(self, path):
        self._check(lib().dash_load(self._h, str(path).encode()), "dash_load")


class DashServer:
    """Many streams on one device (the serving layer of the library).

    Rows go in through submit(); the device buffers of a request are kept
    referenced here until an update of its stream reports them consumed."""

    QUEUED, OPEN = 1, 2

    def __init__(self, budget_bytes, device=0):
        h = _P()
        st = lib().dash_server_create(device, int(budget_bytes), C.byref(h))
        if st != OK:
            raise DashError(st, "dash_server_create")
        self._h = h
        self.device = device
        self._views = {}
        self._held = {}      # stream -> [(request id, tensors)]

    def _check(self, st, what):
        if st != OK:
            msg = lib().dash_server_last_error(self._h)
            raise DashError(st, f"{what}: {msg.decode() if msg else ''}")

    def open(self, J, R, queue=False, **kw):
        """Open a stream; returns its id.  Raises DashError (E_CAPACITY) when its
        footprint does not fit and queue is False; with queue=True it may wait
        for admission (state() == QUEUED)."""
        cfg = make_config(J, R, device=self.device, **kw)
        sid = C.c_int32()
        self._check(lib().dash_server_open(self._h, C.byref(cfg), 1 if queue else 0, C.byref(sid)),
                    "dash_server_open")
        self._held[sid.value] = []
        self._views.pop(sid.value, None)
        return sid.value

    def state(self, sid):
        v = C.c_int32()
        self._check(lib().dash_server_state(self._h, sid, C.byref(v)), "dash_server_state")
        return v.value

    def context(self, sid):
        """A Dash view of an open stream's context (init, get_* only)."""
        if sid not in self._views:
            h = lib().dash_server_context(self._h, sid)
            if not h:
                raise DashError(E_BAD_STATE, f"stream {sid} is not open")
            d = Dash.__new__(Dash)
            d._h, d._owned, d._borrowed = h, False, []
            dims = Dims()
            lib().dash_get_dims(h, C.byref(dims))
            d.J, d.R, d.device = dims.J, dims.R, self.device
            self._views[sid] = d
        return self._views[sid]

    def close_stream(self, sid):
        v = self._views.pop(sid, None)
        if v is not None:
            v._h = None
        self._check(lib().dash_server_close(self._h, sid), "dash_server_close")
        self._held.pop(sid, None)

    def submit(self, sid, slice_id=None, row_ptr=None, rows=None, new_ptr=None, new_rows=None, producer=None):
        """Submit row groups (slice_id, row_ptr host arrays; rows a device tensor)
        and new slices (new_ptr host array; new_rows a device tensor).  producer:
        the HIP stream the tensors were written on (default: torch's current
        stream).  Returns (request id, first new slice id)."""
        ng = 0 if slice_id is None else len(slice_id)
        nn = 0 if new_ptr is None else len(new_ptr) - 1
        sid_a = _host(slice_id, np.int32) if ng else None
        ptr_a = _host(row_ptr, np.int64) if ng else None
        nptr_a = _host(new_ptr, np.int64) if nn else None
        if producer is None:
            import torch
            producer = torch.cuda.current_stream(self.device).cuda_stream
        req = C.c_int64()
        first = C.c_int32()
        st = lib().dash_server_submit(self._h, sid, ng, _ptr(sid_a), _ptr(ptr_a), _ptr(rows) if ng else None, nn,
                                      _ptr(nptr_a), _ptr(new_rows) if nn else None, producer or None,
                                      C.byref(req), C.byref(first))
        self._check(st, "dash_server_submit")
        self._held.setdefault(sid, []).append((req.value, (rows, new_rows)))
        return req.value, first.value

    def _release(self, reps):
        for r in reps:
            held = self._held.get(r["stream"])
            if held:
                self._held[r["stream"]] = [(q, t) for q, t in held if q > r["last_request"]]

    def tick(self):
        n = C.c_int32()
        self._check(lib().dash_server_tick(self._h, C.byref(n)), "dash_server_tick")
        return n.value

    def poll(self, wait=False, cap=4096):
        out = (ServerReport * cap)()
        n = C.c_int32()
        st = lib().dash_server_poll(self._h, 1 if wait else 0, out, cap, C.byref(n))
        reps = [out[i].as_dict() for i in range(n.value)]
        self._release(reps)
        self._check(st, "dash_server_poll")
        return reps

    def start(self, tick_us=0):
        self._check(lib().dash_server_start(self._h, int(tick_us)), "dash_server_start")

    def stop(self):
        self._check(lib().dash_server_stop(self._h), "dash_server_stop")

    def drain(self, timeout_ms=-1):
        self._check(lib().dash_server_drain(self._h, int(timeout_ms)), "dash_server_drain")

    def profile(self, every=10):
        self._check(lib().dash_server_profile(self._h, int(every)), "dash_server_profile")

    def profile_read(self, cap=64):
        out = (KernelStat * cap)()
        n = C.c_int32()
        t = C.c_int64()
        self._check(lib().dash_server_profile_read(self._h, out, cap, C.byref(n), C.byref(t)),
                    "dash_server_profile_read")
        return [out[i].as_dict() for i in range(n.value)], t.value

    def stats(self):
        s = ServerStats()
        self._check(lib().dash_server_get_stats(self._h, C.byref(s)), "dash_server_get_stats")
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            for v in self._views.values():
                v._h = None
            lib().dash_server_destroy(self._h)
            self._h = None
            self._views = {}
            self._held = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
