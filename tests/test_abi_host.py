"""Host-side checks of the C ABI: the library loads, exports every entry point
include/di.h declares, and rejects invalid input before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "di.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:di_status|const char\*)\s+(di_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["di_graph_create", "di_graph_destroy", "di_solve", "di_power_solve",
                     "di_solve_batch", "di_server_create", "di_server_add_graph",
                     "di_server_submit", "di_server_poll", "di_server_wait", "di_server_cancel",
                     "di_server_stats", "di_server_destroy", "di_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1202_6158_amd import di
    lib = ctypes.CDLL(di.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(di.EXPORTED)
    assert "gfx950" in di.version()


def _create(n, row_ptr, col_idx, w=None):
    from paper_1202_6158_amd import di
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    rc = di._lib.di_graph_create(n, len(ci), rp.ctypes.data, ci.ctypes.data if len(ci) else None,
                                 wa.ctypes.data if wa is not None else None, None, ctypes.byref(h))
    return rc, di.last_error()


@pytest.mark.parametrize("case", [
    dict(n=0, row_ptr=[0], col_idx=[]),
    dict(n=2, row_ptr=[1, 1, 1], col_idx=[0]),
    dict(n=2, row_ptr=[0, 2, 1], col_idx=[0]),
    dict(n=2, row_ptr=[0, 1, 2], col_idx=[0, 2]),
    dict(n=2, row_ptr=[0, 1, 2], col_idx=[0, -1]),
    dict(n=2, row_ptr=[0, 2, 2], col_idx=[0, 1], w=[0.5, 0.4]),
    dict(n=2, row_ptr=[0, 2, 2], col_idx=[0, 1], w=[1.5, -0.5]),
    dict(n=2, row_ptr=[0, 2, 2], col_idx=[0, 1], w=[np.nan, 1.0]),
])
def test_graph_create_rejects_invalid_input(case):
    from paper_1202_6158_amd import di
    rc, msg = _create(**case)
    assert rc == di.EINVAL and msg


def test_solve_rejects_bad_options_without_device():
    from paper_1202_6158_amd import di
    st = di.Stats()
    for d, tol in [(1.0, 1e-8), (-0.1, 1e-8), (0.85, 0.0), (float("nan"), 1e-8)]:
        o = di.make_opts(d=d, tol=tol)
        rc = di._lib.di_solve(ctypes.c_void_p(1), None, ctypes.byref(o), None, ctypes.byref(st), None)
        assert rc == di.EINVAL
        rc = di._lib.di_power_solve(ctypes.c_void_p(1), None, ctypes.byref(o), None, ctypes.byref(st), None)
        assert rc == di.EINVAL
    o = di.make_opts()
    assert di._lib.di_solve(None, None, ctypes.byref(o), None, ctypes.byref(st), None) == di.EINVAL


def test_binding_has_no_fallback(tmp_path, monkeypatch):
    """Without libdi.so the binding refuses to import (no CPU path)."""
    import importlib.util
    src = os.path.join(ROOT, "paper_1202_6158_amd", "di.py")
    pkg = tmp_path / "fakepkg"
    pkg.mkdir()
    (pkg / "di.py").write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("fakepkg.di", str(pkg / "di.py"))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_autotune_rejects_missing_graph():
    from paper_1202_6158_amd import di
    o = di.make_opts(0.85, 1e-8, "fp32")
    best = di.Tune()
    rc = di._lib.di_autotune(None, di.TUNE_SOLVE, ctypes.byref(o), 0, None, None,
                             ctypes.byref(best), None, 0, None, None)
    assert rc == di.EINVAL and "graph" in di.last_error()


@pytest.mark.parametrize("n,tune,expect", [
    (10_000, None, (8, False)),            # about 512 windows, never below 2^8
    (1_000_000, None, (11, False)),        # 489 windows of 2^11
    (20_000_000, None, (13, False)),       # the LDS tables still fit at 2^13
    (30_000_000, None, (13, True)),        # 3663 windows: tables in global memory
    (134_217_728, None, (13, True)),       # the largest graph: 16384 windows
    (10_000, dict(window_log2=14), (13, False)),  # 2^14 never fits the LDS budget
    (10_000, dict(tables="global"), (8, True)),
])
def test_window_layout(n, tune, expect):
    from paper_1202_6158_amd import di
    t = di.make_tune("mean", 1.0, **tune) if tune else None
    assert di.window_layout(n, t) == expect


@pytest.mark.parametrize("n,tables", [(134_217_729, "auto"), (30_000_000, "lds"), (0, "auto")])
def test_window_layout_rejects_what_does_not_fit(n, tables):
    from paper_1202_6158_amd import di
    with pytest.raises(di.DiError) as e:
        di.window_layout(n, di.make_tune("mean", 1.0, tables=tables))
    assert e.value.status == di.EINVAL


def test_taken_list_switch_is_host_only_and_checked():
    from paper_1202_6158_amd import di
    assert di._lib.di_set_taken_list(2) == di.EINVAL and "enable" in di.last_error()
    assert di._lib.di_set_taken_list(-1) == di.EINVAL
    di.set_taken_list(False)
    di.set_taken_list(True)


def test_persist_wait_setting_is_host_only_and_checked():
    from paper_1202_6158_amd import di
    assert di._lib.di_set_persist_wait(-1.0) == di.EINVAL and "seconds" in di.last_error()
    assert di._lib.di_set_persist_wait(61.0) == di.EINVAL
    di.set_persist_wait(0.5)
    di.set_persist_wait(2.0)
