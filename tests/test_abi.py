"""The C-ABI library loads and exports every symbol declared in
include/gbs_mps.h; host-side argument checks (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbs_mps.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(gbs_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("gbs_mps_build", "gbs_mps_amplitude", "gbs_mps_sample", "gbs_mps_free", "gbs_last_error"):
        assert f in fns


def test_library_exports_every_declared_symbol():
    from paper_2512_10643_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2512_10643_amd import build_lib
        build_lib.build()
    L = ctypes.CDLL(_lib.LIB_PATH)
    for f in declared_functions():
        assert hasattr(L, f), f
    assert set(declared_functions()) == set(_lib.EXPORTED_SYMBOLS)


def test_noalloc_scratch_size_matches_header():
    from paper_2512_10643_amd import _lib
    m = re.search(r"#define GBS_SAMPLE_NOALLOC_SCRATCH_BYTES \((\d+)ll << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.GBS_SAMPLE_NOALLOC_SCRATCH_BYTES


def test_invalid_arguments_rejected_on_host():
    """Argument validation happens before any device work."""
    from paper_2512_10643_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    opts = _lib.BuildOpts(d=4, chi=16, dstar=1.0 + 1e-10, prec=0, flags=0, trunc_rel=0.0)
    fake = ctypes.c_void_p(1)  # never dereferenced: validation fails first
    assert L.gbs_mps_build(fake, 0, ctypes.byref(opts), None, ctypes.byref(h)) == _lib.GBS_E_INVAL
    assert h.value is None
    for bad in (dict(d=0), dict(chi=0), dict(chi=5000), dict(dstar=1.0), dict(prec=9), dict(chi_build=-1),
                dict(chi_build=5000), dict(chi_build=4096)):  # the last: chi_build * d = 16384 > 8192
        o = _lib.BuildOpts(**{**dict(d=4, chi=16, dstar=1.0 + 1e-10, prec=0, flags=0, trunc_rel=0.0), **bad})
        assert L.gbs_mps_build(fake, 4, ctypes.byref(o), None, ctypes.byref(h)) == _lib.GBS_E_INVAL
    assert L.gbs_mps_build(None, 4, ctypes.byref(opts), None, ctypes.byref(h)) == _lib.GBS_E_INVAL
    assert b"NULL" in L.gbs_last_error()
    assert L.gbs_mps_amplitude(None, None, 1, None, None) == _lib.GBS_E_INVAL
    assert L.gbs_mps_sample(None, 1, 0, None, None) == _lib.GBS_E_INVAL
    assert L.gbs_mps_sample_noalloc(None, 1, 0, None, None) == _lib.GBS_E_INVAL
    L.gbs_mps_free(None)


def test_server_and_footprint_host_checks():
    """Server creation arguments and the footprint estimate are validated on
    the host; the estimate grows with chi and with the shot count."""
    from paper_2512_10643_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.gbs_server_create(0, 1 << 30, 16, ctypes.byref(h)) == _lib.GBS_E_INVAL
    assert L.gbs_server_create(4, 0, 16, ctypes.byref(h)) == _lib.GBS_E_INVAL
    assert L.gbs_server_create(4, 1 << 30, 0, ctypes.byref(h)) == _lib.GBS_E_INVAL
    assert not h.value
    o = _lib.BuildOpts(d=8, chi=256, dstar=1.0 + 1e-10, prec=1, flags=0, trunc_rel=0.0)
    f1 = L.gbs_mps_footprint(144, ctypes.byref(o), 0)
    f2 = L.gbs_mps_footprint(144, ctypes.byref(o), 10_000)
    o.chi = 64
    f3 = L.gbs_mps_footprint(144, ctypes.byref(o), 0)
    assert 0 < f3 < f1 < f2
    o.chi_build = 256     # built at 256 states per cut, recompressed to 64
    assert L.gbs_mps_footprint(144, ctypes.byref(o), 0) == f1
    o.chi_build = -1
    assert L.gbs_mps_footprint(144, ctypes.byref(o), 0) == -1
    o.chi_build = 0
    # the C3 build holds its PCO tensors (144 x 8 x 256^2 complex FP64) at least
    assert f1 > 144 * 8 * 256 * 256 * 16
    o.d = 0
    assert L.gbs_mps_footprint(144, ctypes.byref(o), 0) == -1
