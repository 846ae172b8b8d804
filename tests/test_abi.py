"""CPU checks of the C ABI: the library loads and exports every symbol that
include/ga.h declares; host-only calls behave. No compute call is made."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ga.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ga_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["ga_splat", "ga_fft3d", "ga_correlate", "ga_energy_fields", "ga_force_torque", "ga_plan_create"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1711_05017_amd import ga

    lib = ga.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(ga.EXPORTS) == _declared()


def test_host_only_calls():
    from paper_1711_05017_amd import ga

    lib = ga.load()
    assert lib.ga_version().decode().startswith("ga ")
    assert lib.ga_status_str(0).decode() == "ok"
    assert lib.ga_status_str(-1).decode() == "invalid argument"
    for n in (16, 24, 32, 48, 64, 96, 128, 192):
        assert lib.ga_supported_n(n) == 1
    for n in (7, 10, 100, 1000):
        assert lib.ga_supported_n(n) == 0
    # null out-pointer and odd sizes are rejected before touching the device
    assert lib.ga_plan_create(None, 32, 1, 0) == -1
    h = ctypes.c_void_p()
    assert lib.ga_plan_create(ctypes.byref(h), 33, 1, 0) == -1
    assert lib.ga_plan_create(ctypes.byref(h), 32, 0, 0) == -1
    assert lib.ga_plan_create(ctypes.byref(h), 32, 1, 7) == -1
    assert lib.ga_plan_create(ctypes.byref(h), 100, 1, 0) == -6
    assert lib.ga_workspace_size(None, 3, 1, 0) == 0
    assert lib.ga_plan_destroy(None) == -1


def test_library_is_the_in_tree_build():
    from paper_1711_05017_amd import ga

    assert os.path.dirname(ga.LIB_PATH) == os.path.join(ROOT, "paper_1711_05017_amd")
    assert os.path.exists(ga.LIB_PATH)


def test_missing_library_fails_loudly(tmp_path):
    from paper_1711_05017_amd import ga

    saved = ga._lib
    try:
        ga._lib = None
        with pytest.raises(RuntimeError):
            ga.load(str(tmp_path / "nope.so"))
    finally:
        ga._lib = saved
