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
    # an empty grid is rejected
    c.mode = wfa.COEF_CONST
    for dims in ((0, 4, 4), (4, 0, 4), (4, 4, 0), (-1, 4, 4)):
        rc = libwfa.wfa_grid_create(*dims, ctypes.byref(c), ctypes.c_void_p(256), 1 << 30,
                                    ctypes.byref(out))
        assert rc == wfa.ERR_INVALID, dims


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
    assert libwfa.wfa_grid_set_option(out, wfa.OPT_METHOD, wfa.METHOD_CG1) == wfa.OK
    # a server-only option is not a grid option
    assert libwfa.wfa_grid_set_option(out, wfa.OPT_CG1_MAX_CELLS, 1000) == wfa.ERR_INVALID
    assert libwfa.wfa_grid_set_option(out, wfa.OPT_ZCHUNK, 32) == wfa.OK
    assert libwfa.wfa_grid_tiling(out, *[ctypes.byref(q) for q in v]) == wfa.OK
    assert v[2].value == 32
    # launch timing: off, every launch, or every n-th launch of each kernel
    for n, rc in ((-1, wfa.ERR_INVALID), ((1 << 20) + 1, wfa.ERR_INVALID), (8, wfa.OK),
                  (1, wfa.OK), (0, wfa.OK)):
        assert libwfa.wfa_grid_set_option(out, wfa.OPT_PROFILE, n) == rc, n
    assert libwfa.wfa_grid_destroy(out) == wfa.OK


def _tiling(libwfa, g):
    v = [ctypes.c_int() for _ in range(4)]
    assert libwfa.wfa_grid_tiling(g, *[ctypes.byref(q) for q in v]) == 0
    return tuple(q.value for q in v)


def test_tuning_table_file_and_grid_creation(libwfa, tmp_path):
    """The tuning table is host-only: a loaded entry sets the tiling of every
    grid created with its key (shape, precision, coefficient mode) and no
    other; save writes what load reads; a malformed file is rejected whole."""
    from paper_2209_13768_amd import wfa
    wfa.tune_clear()
    c = wfa.make_coeffs(h=1 / 97, dt=1e-2)
    nbytes = wfa.workspace_bytes(96, 80, 48, wfa.F64)

    def grid(nx=96, ny=80, nz=48):
        out = ctypes.c_void_p()
        assert libwfa.wfa_grid_create(nx, ny, nz, ctypes.byref(c), ctypes.c_void_p(1 << 20),
                                      nbytes, ctypes.byref(out)) == wfa.OK
        return out

    g = grid()
    default = _tiling(libwfa, g)
    libwfa.wfa_grid_destroy(g)
    table = tmp_path / "tune.txt"
    table.write_text("# comment\n96 80 48 0 0 4 8 123.5\n96 80 48 1 0 1 2 50.0\n")
    wfa.tune_load(str(table))
    g = grid()
    assert _tiling(libwfa, g) == (64, 16, 8, 2 * 5 * 6)   # 4 rows per wave, 8 planes
    libwfa.wfa_grid_destroy(g)
    g = grid(96, 80, 47)                                   # another key: default rule
    assert _tiling(libwfa, g)[1] == default[1]
    libwfa.wfa_grid_destroy(g)
    saved = tmp_path / "saved.txt"
    wfa.tune_save(str(saved))
    rows = [ln.split() for ln in saved.read_text().splitlines() if not ln.startswith("#")]
    assert sorted(r[:7] for r in rows) == sorted([["96", "80", "48", "0", "0", "4", "8"],
                                                  ["96", "80", "48", "1", "0", "1", "2"]])
    wfa.tune_clear()
    g = grid()
    assert _tiling(libwfa, g) == default
    libwfa.wfa_grid_destroy(g)
    for bad in ("96 80 48 0 0 3 8 1.0\n", "96 80 48 0 0 2 49 1.0\n", "96 80 48 0\n",
                "96 80 48 9 0 2 8 1.0\n"):
        table.write_text("96 80 40 0 0 2 4 1.0\n" + bad)
        with pytest.raises(wfa.WfaError):
            wfa.tune_load(str(table))
    g = grid(96, 80, 40)                                   # nothing of a bad file is merged
    assert _tiling(libwfa, g)[2] != 4 or default[2] == 4
    libwfa.wfa_grid_destroy(g)
    with pytest.raises(wfa.WfaError):
        wfa.tune_load(str(tmp_path / "missing.txt"))
    wfa.tune_clear()


def test_bandwidth_probe_kinds_and_validation(libwfa):
    """The probe kinds of the header and the binding agree, and bad kinds,
    sizes and pointers are refused before any device work."""
    from paper_2209_13768_amd import wfa
    text = open(os.path.join(ROOT, "include", "wfa.h")).read()
    kinds = dict((k, int(v)) for k, v in re.findall(r"\bWFA_PROBE_([A-Z0-9_]+)\s*=\s*(\d+)", text))
    assert kinds == {"COPY": wfa.PROBE_COPY, "COPY_PLAIN": wfa.PROBE_COPY_PLAIN,
                     "COPY32": wfa.PROBE_COPY32, "READ": wfa.PROBE_READ,
                     "WRITE": wfa.PROBE_WRITE, "MIX_6R4W": wfa.PROBE_MIX_6R4W,
                     "MIX_3R1W": wfa.PROBE_MIX_3R1W}
    assert len(wfa.PROBE_NAMES) == len(wfa.PROBE_STREAMS) == len(kinds)
    g = ctypes.c_double()
    fake = ctypes.c_void_p(1 << 20)
    for kind, size, src in ((-1, 4096, fake), (7, 4096, fake), (wfa.PROBE_MIX_6R4W, 4104, fake),
                            (wfa.PROBE_MIX_3R1W, 4096, None), (wfa.PROBE_COPY32, 4112, fake),
                            (wfa.PROBE_READ, 1024, fake), (wfa.PROBE_MIX_6R4W, (1 << 40) + 16, fake)):
        rc = libwfa.wfa_bandwidth_probe(kind, 0, src, fake, size, 1, ctypes.byref(g), None)
        assert rc == wfa.ERR_INVALID, (kind, size)
    # unaligned buffers
    rc = libwfa.wfa_bandwidth_probe(wfa.PROBE_MIX_3R1W, 0, ctypes.c_void_p((1 << 20) + 8), fake,
                                    4096, 1, ctypes.byref(g), None)
    assert rc == wfa.ERR_INVALID
