"""CPU-side checks of the C-ABI boundary: the library loads and exports every
function include/wfa.h declares; host-only calls validate their arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "wfa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wfa_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libwfa():
    from paper_2209_13768_amd import wfa
    return wfa.lib()


def test_exports_every_declared_function(libwfa):
    from paper_2209_13768_amd import wfa
    declared = header_functions()
    assert len(declared) >= 18
    assert sorted(wfa.EXPORTS) == declared
    for name in declared:
        assert hasattr(libwfa, name), name


def test_workspace_bytes_and_validation(libwfa):
    from paper_2209_13768_amd import wfa
    assert wfa.workspace_bytes(0, 4, 4) == 0
    assert wfa.workspace_bytes(4, 4, 4, 7) == 0
    n = 64 * 64 * 64
    f64 = wfa.workspace_bytes(64, 64, 64, wfa.F64)
    f32 = wfa.workspace_bytes(64, 64, 64, wfa.F32)
    ir = wfa.workspace_bytes(64, 64, 64, wfa.F32_IR64)
    assert f64 >= 8 * 8 * n and f32 >= 8 * 4 * n and ir >= (8 + 9 * 4) * n
    assert f32 < f64
    # argument validation happens before any device work
    c = wfa.make_coeffs(h=0.1, dt=0.0)
    out = ctypes.c_void_p()
    rc = libwfa.wfa_grid_create(4, 4, 4, ctypes.byref(c), ctypes.c_void_p(256), 1 << 30,
                                ctypes.byref(out))
    assert rc == wfa.ERR_INVALID and "dt" in wfa.last_error()
    c = wfa.make_coeffs(h=0.1, dt=0.1)
    rc = libwfa.wfa_grid_create(4, 4, 4, ctypes.byref(c), ctypes.c_void_p(256), 16,
                                ctypes.byref(out))
    assert rc == wfa.ERR_NOMEM
    rc = libwfa.wfa_grid_create(4, 4, 4, ctypes.byref(c), ctypes.c_void_p(300), 1 << 30,
                                ctypes.byref(out))
    assert rc == wfa.ERR_INVALID
    c.mode = wfa.COEF_CELL
    rc = libwfa.wfa_grid_create(4, 4, 4, ctypes.byref(c), ctypes.c_void_p(256), 1 << 30,
                                ctypes.byref(out))
    assert rc == wfa.ERR_INVALID and "kappa" in wfa.last_error()


def test_grid_descriptor_host_only(libwfa):
    """A descriptor can be created on a fake (never dereferenced) device
    address: creation, options and tiling are host-only."""
    from paper_2209_13768_amd import wfa
    c = wfa.make_coeffs(h=1 / 257, dt=1e-2, u=(1, 0.5, 0.25))
    out = ctypes.c_void_p()
    nbytes = wfa.workspace_bytes(256, 256, 256, wfa.F64)
    assert libwfa.wfa_grid_create(256, 256, 256, ctypes.byref(c), ctypes.c_void_p(1 << 20),
                                  nbytes, ctypes.byref(out)) == wfa.OK
    v = [ctypes.c_int() for _ in range(4)]
    assert libwfa.wfa_grid_tiling(out, *[ctypes.byref(q) for q in v]) == wfa.OK
    tx, ty, zc, blocks = (q.value for q in v)
    assert tx == 64 and ty % 4 == 0 and 1 <= zc <= 256
    assert blocks == (256 // tx) * (-(-256 // ty)) * (-(-256 // zc))
    assert libwfa.wfa_grid_set_option(out, wfa.OPT_METHOD, 5) == wfa.ERR_INVALID
    assert libwfa.wfa_grid_set_option(out, wfa.OPT_ZCHUNK, 32) == wfa.OK
    assert libwfa.wfa_grid_tiling(out, *[ctypes.byref(q) for q in v]) == wfa.OK
    assert v[2].value == 32
    assert libwfa.wfa_grid_destroy(out) == wfa.OK
