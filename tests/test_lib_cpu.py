"""Host-only checks of the C ABI library: it loads, exports every entry point
declared in include/adi.h, and validates arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2006_07583_amd import adi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "adi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(adi_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    L = adi.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(adi.EXPORTS)


def test_params_struct_matches_header():
    p = adi.AdiParams()
    assert adi.lib().adi_params_init(ctypes.byref(p)) == 0
    assert p.struct_size == ctypes.sizeof(adi.AdiParams)
    assert p.sweeps == 6 and p.src_i == -1 and p.kappa0 == 1.0


def _ws(p, **kw):
    n = ctypes.c_size_t()
    return adi.lib().adi_workspace_size(ctypes.byref(p), kw.get("K", 0), kw.get("Rv", 0),
                                        kw.get("Rw", 0), ctypes.byref(n)), n.value


def good(method=adi.CFD, dtype=adi.FP32, n=64):
    return adi.make_params(method, dtype, n, n, 1.0 / n, 0.5 / n, 1.0)


def test_workspace_size_grows_with_materials():
    rc, base = _ws(good())
    assert rc == 0 and base > 0
    rc, full = _ws(good(), K=1, Rv=1, Rw=1)
    assert rc == 0 and full > base
    rc, d = _ws(good(dtype=adi.FP64))
    assert rc == 0 and d > base


@pytest.mark.parametrize("mutate,expect", [
    (lambda p: setattr(p, "sweeps", 7), "even"),
    (lambda p: setattr(p, "sweeps", -2), "even"),
    (lambda p: (setattr(p, "sweeps", 0), setattr(p, "dtype", adi.FP32C)), "compensated"),
    (lambda p: (setattr(p, "sweeps", 0), setattr(p, "dt", 400.0 / 64)), "too large"),
    (lambda p: setattr(p, "nx", 7), ">= 8"),
    (lambda p: setattr(p, "dt", 1.2 / 64), "cfl"),
    (lambda p: setattr(p, "method", 5), "method"),
    (lambda p: setattr(p, "dtype", 9), "dtype"),
    (lambda p: setattr(p, "order", 2), "order"),
    (lambda p: setattr(p, "h", 0.0), "h must"),
    (lambda p: setattr(p, "c_max", 0.0), "c_max"),
    (lambda p: setattr(p, "struct_size", 8), "struct_size"),
    (lambda p: (setattr(p, "src_i", 0), setattr(p, "src_j", 5)), "source"),
    (lambda p: (setattr(p, "src_i", 64), setattr(p, "src_j", 63)), "source"),
])
def test_invalid_parameters_rejected(mutate, expect):
    p = good()
    mutate(p)
    rc, _ = _ws(p)
    assert rc == -1
    assert expect in adi.lib().adi_last_error().decode()
    h = ctypes.c_void_p()
    assert adi.lib().adi_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert not h.value


def test_mfd_cfl_limit_is_lower():
    p = adi.make_params(adi.MFD, adi.FP32, 64, 64, 1.0 / 64, 0.85 / 64, 1.0)
    assert _ws(p)[0] == -1
    p.dt = 0.8 / 64
    assert _ws(p)[0] == 0
    p = adi.make_params(adi.CFD, adi.FP32, 64, 64, 1.0 / 64, 1.1 / 64, 1.0)
    assert _ws(p)[0] == 0


def test_null_arguments():
    L = adi.lib()
    assert L.adi_run(None, 1) == -1
    assert L.adi_bind(None, None, None, None, None, None, None, None, None, 0) == -1
    assert L.adi_destroy(None) == 0
    assert L.adi_status_string(-5) == b"ADI_ENOTREADY"
    assert L.adi_set_tolerance(None, 1e-6, 2) == -1
    n = ctypes.c_int64()
    assert L.adi_sweep_stats(None, ctypes.byref(n), ctypes.byref(n)) == -1


def test_batch_create_validates_arguments_on_the_host():
    L = adi.lib()
    out = ctypes.c_void_p()
    vp = ctypes.c_void_p
    assert L.adi_batch_create(None, 1, None, 0, ctypes.byref(out)) == -1
    arr = (vp * 1)(None)
    assert L.adi_batch_create(arr, 0, None, 0, ctypes.byref(out)) == -1
    assert b"at least one" in L.adi_last_error()
    assert L.adi_batch_create(arr, 1, None, 4, ctypes.byref(out)) == -1
    assert b"flags" in L.adi_last_error()
    assert L.adi_batch_create(arr, 1, None, adi.BATCH_GRAPH, ctypes.byref(out)) == -1
    assert b"stream" in L.adi_last_error()
    assert L.adi_batch_create(arr, 1, None, 0, None) == -1
    assert L.adi_batch_run(None, 1) == -1
    assert L.adi_batch_sync(None) == -1
    n = ctypes.c_int64()
    assert L.adi_batch_launches(None, ctypes.byref(n)) == -1
    assert L.adi_batch_destroy(None) == 0


def test_server_validates_arguments_on_the_host():
    L = adi.lib()
    out = ctypes.c_void_p()
    p = adi.AdiServerParams()
    assert L.adi_server_params_init(ctypes.byref(p)) == 0
    assert p.struct_size == ctypes.sizeof(adi.AdiServerParams) and p.max_active == 256
    assert L.adi_server_create(None, ctypes.byref(out)) == -1
    bad = adi.AdiServerParams(p.struct_size, 0, p.hbm_budget_bytes)
    assert L.adi_server_create(ctypes.byref(bad), ctypes.byref(out)) == -1
    assert b"max_active" in L.adi_last_error()
    bad = adi.AdiServerParams(p.struct_size, 4, 1024)
    assert L.adi_server_create(ctypes.byref(bad), ctypes.byref(out)) == -1
    assert L.adi_server_create(ctypes.byref(p), None) == -1
    t = ctypes.c_uint64()
    assert L.adi_submit(None, None, ctypes.byref(t)) == -1
    st = ctypes.c_int()
    assert L.adi_poll(None, 1, ctypes.byref(st)) == -1
    assert L.adi_wait(None, 1) == -1
    assert L.adi_server_destroy(None) == 0


def test_direct_solves_accept_large_steps_and_size_their_store():
    """sweeps 0 (direct solves) lifts the divergence limit of the sweeps and
    adds the factor store to the workspace, larger for larger steps."""
    n = 1024
    p = good(n=n)
    p.dt = 1.2 / n
    assert _ws(p)[0] == -1
    p.sweeps = 0
    rc, small = _ws(p)
    assert rc == 0
    p.dt = 4.0 / n
    rc, big = _ws(p)
    assert rc == 0 and big > small
    p.sweeps, p.dt = 6, 0.5 / n
    assert _ws(p)[1] < small
