"""CPU checks of the C ABI: the library loads, exports every declared entry
point, the struct layouts agree, and argument errors are reported without
touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cesmlmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ces_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_13493_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2306_13493_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    from paper_2306_13493_amd import _lib
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


def test_struct_layouts(lib):
    from paper_2306_13493_amd import _lib
    d = _lib.LevelDesc()
    lib.ces_level_desc_default(ctypes.byref(d))
    assert d.struct_size == ctypes.sizeof(_lib.LevelDesc) == 136 and d.mg_cycle == 0
    assert ctypes.sizeof(_lib.PlanInfo) == 72
    assert d.m_fine == 32 and d.cg_rtol == 1e-10 and d.cg_max_iter == 500 and d.f_value == 1.0
    assert abs(d.qoi_x - 7 / 15) < 1e-16 and d.precision == 1 and d.psd_policy == 0


def test_argument_errors_without_device(lib):
    from paper_2306_13493_amd import _lib
    d = _lib.LevelDesc()
    lib.ces_level_desc_default(ctypes.byref(d))
    h = ctypes.c_void_p()
    assert lib.ces_plan_create(None, ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"NULL" in lib.ces_last_error()
    assert lib.ces_sample(None, 0, 0, 4, None, None, None, None, None, None) == -1
    assert lib.ces_normals(0, 0, 0, 0, -1, None, None) == -1
    assert lib.ces_normals(0, 0, 0, 2 ** 32 - 2, 5, ctypes.c_void_p(8), None) == -1
    assert lib.ces_solve(None, 0, 1, None, None, None, None) == -1
    assert lib.ces_plan_info_get(None, None) == -1
    assert lib.ces_plan_destroy(None) == 0
    assert lib.ces_context_destroy(None) == 0


def test_batch_entry_points_reject_bad_arguments(lib):
    from paper_2306_13493_amd import _lib
    assert ctypes.sizeof(_lib.Request) == 72
    assert ctypes.sizeof(_lib.Schedule) == 24
    reqs = (_lib.Request * 1)()
    assert lib.ces_sample_batch(None, reqs, 1, None) == -1
    assert lib.ces_schedule_get(None, None) == -1
    assert lib.ces_schedule_set(None, None) == -1
    assert lib.ces_autotune(None, reqs, 1, None, None, None) == -1
    assert b"NULL" in lib.ces_last_error()


def test_server_entry_points_reject_bad_arguments(lib):
    from paper_2306_13493_amd import _lib
    assert ctypes.sizeof(_lib.ServerStats) == 72
    rid = ctypes.c_int64()
    st = ctypes.c_int32()
    assert lib.ces_server_create(None, 0, 0, None) == -1
    assert lib.ces_server_submit(None, None, 0, 0, 1, None, None, ctypes.byref(rid)) == -1
    assert lib.ces_server_poll(None, 1, ctypes.byref(st), None) == -1
    assert lib.ces_server_drain(None) == -1
    assert lib.ces_server_get_stats(None, None) == -1
    assert lib.ces_server_destroy(None) == 0


def test_mlmc_entry_points(lib):
    from paper_2306_13493_amd import _lib
    o = _lib.MlmcOpts()
    lib.ces_mlmc_opts_default(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(_lib.MlmcOpts) and o.theta == 0.5 and o.n_pilot >= 2
    r = _lib.MlmcResult()
    assert lib.ces_mlmc_run(None, None, None, 1, ctypes.byref(o), None, ctypes.byref(r)) == -1
    d = _lib.LevelDesc()
    lib.ces_level_desc_default(ctypes.byref(d))
    d.nu, d.lambda_ = 0.5, 0.03
    m0 = ctypes.c_int32()
    assert lib.ces_mlmc_coarsest_mesh(ctypes.byref(d), ctypes.byref(m0)) == 0 and m0.value == 32


def test_smoothing_study_entry_points(lib):
    from paper_2306_13493_amd import _lib
    assert ctypes.sizeof(_lib.SmoothingStats) == 56
    r = _lib.SmoothingStats()
    r.struct_size = ctypes.sizeof(r)
    assert lib.ces_smoothing_error(None, None, None, 0, 0, 4, None, ctypes.byref(r)) == -1
    t = ctypes.c_int64()
    assert lib.ces_tau_rule(0, 1.5, 64, 0, 1.0, 1.0, ctypes.byref(t), None) == 0 and 0 <= t.value <= 128 * 128
    assert lib.ces_tau_rule(7, 1.5, 64, 0, 1.0, 1.0, ctypes.byref(t), None) == -1
