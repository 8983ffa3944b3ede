"""The C ABI library loads and exports every symbol include/utd.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "utd.h")) as fh:
        src = fh.read()
    return sorted(set(re.findall(r"\b(utd_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    import paper_2310_10578_amd as utd
    assert sorted(utd.EXPORTS) == declared_symbols()


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2310_10578_amd", "libutd.so")
    if not os.path.exists(path):
        pytest.fail("libutd.so not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_default_options_and_error_paths_without_gpu():
    import paper_2310_10578_amd as utd
    lib = utd.load_library()
    o = utd.Options()
    lib.utd_default_options(ctypes.byref(o))
    assert (o.precision, o.l_enc, o.bodies_occlude, o.lit_branch) == (0, 0, 1, 1)
    assert abs(o.caustic_guard - 1e-6) < 1e-18
    # argument errors are reported before any device work
    b = utd.Bodies()
    s = utd.make_source((0, 0, 0))
    o.l_enc = 7
    st = lib.utd_smooth_field(None, ctypes.byref(b), ctypes.byref(s), None, 0, None, 0, ctypes.byref(o),
                              None, None, None)
    assert st == -1 and b"l_enc" in lib.utd_last_error()
    o.l_enc = 0
    st = lib.utd_smooth_field(None, ctypes.byref(b), ctypes.byref(s), None, -1, None, 0, ctypes.byref(o),
                              None, None, None)
    assert st == -1
    # empty work is a no-op
    st = lib.utd_smooth_field(None, ctypes.byref(b), ctypes.byref(s), None, 0, None, 0, ctypes.byref(o),
                              None, None, None)
    assert st == 0
    # the uniform caustic sum: 0 or 1, forward calls only
    assert o.caustic_uniform == 0
    o.caustic_uniform = 2
    st = lib.utd_smooth_field(None, ctypes.byref(b), ctypes.byref(s), None, 0, None, 0, ctypes.byref(o),
                              None, None, None)
    assert st == -1 and b"caustic_uniform" in lib.utd_last_error()
    o.caustic_uniform = 1
    dummy = ctypes.c_double()
    st = lib.utd_smooth_field_backward(None, ctypes.byref(b), ctypes.byref(s), None, 0, None, 0, ctypes.byref(o),
                                       None, None, None, ctypes.byref(dummy), None)
    assert st == -5 and b"caustic" in lib.utd_last_error()
    state = ctypes.c_void_p()
    st = lib.utd_smooth_field_saved(None, ctypes.byref(b), ctypes.byref(s), None, 0, None, 0, ctypes.byref(o),
                                    None, None, ctypes.byref(state), None)
    assert st == -5 and not state.value
    o.caustic_uniform = 0
    h = ctypes.c_void_p()
    assert lib.utd_scene_create(None, -1, ctypes.byref(h)) == -1
    assert lib.utd_scene_create(None, 0, None) == -1
