"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every entry
point the public header declares, and its built-in method constants equal the oracle's."""
import ctypes

import pytest

import oracle


def test_library_exports_every_declared_symbol():
    from paper_2009_07515_amd import tpcsf
    lib = tpcsf.load()
    names = tpcsf.header_symbols()
    assert len(names) >= 11
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_default_constants_match_the_oracle():
    from paper_2009_07515_amd import tpcsf
    p = tpcsf.default_params().as_dict()
    for k, v in oracle.DEFAULT_PARAMS.items():
        if k == "c0":
            assert tuple(p[k]) == tuple(v)
        else:
            assert p[k] == pytest.approx(v, rel=0, abs=0), k
    t = tpcsf.default_tuning().as_dict()
    for k, v in oracle.DEFAULT_GRID.items():
        assert t[k] == v, k


def test_create_rejects_bad_geometry_without_touching_the_gpu():
    from paper_2009_07515_amd import tpcsf
    lib = tpcsf.load()
    h = ctypes.c_void_p()
    # rows not increasing -> E_INVALID before any HIP call
    rx = (ctypes.c_float * 3)(1.0, 0.5, 2.0)
    geo = tpcsf.Geometry(36, 3, ctypes.cast(rx, ctypes.c_void_p), 0.5)
    assert lib.tpcsf_create(ctypes.byref(geo), None, None, 0, ctypes.byref(h)) == tpcsf.E_INVALID
    geo = tpcsf.Geometry(36, 2, ctypes.cast(rx, ctypes.c_void_p), 0.5)
    assert lib.tpcsf_create(ctypes.byref(geo), None, None, 0, ctypes.byref(h)) == tpcsf.E_INVALID
    bad_t = tpcsf.default_tuning()
    bad_t.block = 100
    rx2 = (ctypes.c_float * 3)(1.0, 2.0, 3.0)
    geo = tpcsf.Geometry(36, 3, ctypes.cast(rx2, ctypes.c_void_p), 0.5)
    assert lib.tpcsf_create(ctypes.byref(geo), None, ctypes.byref(bad_t), 0, ctypes.byref(h)) == tpcsf.E_INVALID


def test_create_rejects_more_than_255_rows():
    """A tracklet's cluster count fills the 8 high bits of its 32-bit selection weight, so a
    geometry of 256 rows (a 256-cluster tracklet would wrap to 0) is refused before any HIP
    call; 255 rows pass the geometry check."""
    from paper_2009_07515_amd import tpcsf
    lib = tpcsf.load()
    h = ctypes.c_void_p()
    rx = (ctypes.c_float * 256)(*[85.0 + i for i in range(256)])
    geo = tpcsf.Geometry(36, 256, ctypes.cast(rx, ctypes.c_void_p), 0.5)
    assert lib.tpcsf_create(ctypes.byref(geo), None, None, 0, ctypes.byref(h)) == tpcsf.E_INVALID
    assert not h.value
