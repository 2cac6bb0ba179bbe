"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad configurations before touching a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2305_18376_amd import dash as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dash.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dash_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_problem_calls():
    names = declared_functions()
    for call in ("dash_init", "dash_ingest_rows", "dash_ingest_slices", "dash_update", "dash_get_factors"):
        assert call in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(D.LIB_PATH):
        pytest.fail("libdash.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", D.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dash_[a-z_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = D.lib()
    for n in declared_functions():
        assert getattr(L, n) is not None


def test_config_defaults_and_status_strings():
    L = D.lib()
    cfg = D.DashConfig()
    L.dash_config_default(C.byref(cfg), 88, 10)
    assert (cfg.J, cfg.R, cfg.n_iter, cfg.init_max_iter) == (88, 10, 1, 10)
    assert cfg.lam == pytest.approx(0.7)
    for s in range(8):
        assert L.dash_status_string(s)
    assert b"unknown" in L.dash_status_string(99)


@pytest.mark.parametrize("field,value", [("J", 0), ("J", 257), ("R", 0), ("R", 33), ("lam", 0.0),
                                         ("lam", 1.5), ("n_iter", 0), ("max_slices", 0),
                                         ("max_rows_per_update", 0), ("precision", 7), ("stats_mode", 9)])
def test_create_rejects_bad_config_without_a_device(field, value):
    L = D.lib()
    cfg = D.DashConfig()
    L.dash_config_default(C.byref(cfg), 16, 4)
    setattr(cfg, field, value)
    h = C.c_void_p()
    assert L.dash_create(C.byref(cfg), C.byref(h)) == D.E_INVALID_ARG
    assert not h.value


def test_null_arguments():
    L = D.lib()
    assert L.dash_create(None, None) == D.E_INVALID_ARG
    assert L.dash_destroy(None) == D.OK
    assert L.dash_update(None, None) == D.E_INVALID_ARG
    assert L.dash_get_dims(None, None) == D.E_INVALID_ARG
    assert L.dash_last_error(None) == b""
    assert L.dash_debug_fail_next(None, D.SITE_COMMIT) == D.E_INVALID_ARG


def test_footprint_and_admission_without_a_device():
    """Admission is decided from the footprint before any device call."""
    import ctypes as C
    small = D.make_config(32, 8, max_slices=1000, max_rows=10000, max_groups=1000)
    big = D.make_config(32, 8, max_slices=100000, max_rows=10000, max_groups=1000)
    a, b = C.c_int64(), C.c_int64()
    assert D.lib().dash_footprint(C.byref(small), C.byref(a)) == D.OK
    assert D.lib().dash_footprint(C.byref(big), C.byref(b)) == D.OK
    assert 0 < a.value < b.value
    # the state alone: 2 buffers of Y, D, n, W per slice
    ys = (8 * 32 + 63) // 64 * 64
    assert a.value >= 2 * 1000 * (ys * 4 + 64 * 4 + 8 + 8 * 8)
    bad = D.make_config(32, 8)
    bad.R = 0
    assert D.lib().dash_footprint(C.byref(bad), C.byref(a)) == D.E_INVALID_ARG
    srv = C.c_void_p()
    assert D.lib().dash_server_create(0, a.value - 1, C.byref(srv)) == D.OK
    sid = C.c_int32(-1)
    assert D.lib().dash_server_open(srv, C.byref(small), 0, C.byref(sid)) == D.E_CAPACITY
    assert sid.value == -1
    # larger than the whole budget: refused even when it may wait
    assert D.lib().dash_server_open(srv, C.byref(small), 1, C.byref(sid)) == D.E_CAPACITY
    assert sid.value == -1
    st = D.ServerStats()
    assert D.lib().dash_server_get_stats(srv, C.byref(st)) == D.OK
    assert st.open == 0 and st.queued == 0 and st.budget == a.value - 1
    assert D.lib().dash_server_context(srv, 0) is None
    assert D.lib().dash_server_destroy(srv) == D.OK
