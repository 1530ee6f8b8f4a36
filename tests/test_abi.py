"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_2409_01910_amd as bz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bz_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declarations_match_binding_list():
    assert set(_declared()) == set(bz.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = bz.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_create_rejects_bad_parameters_without_a_device():
    lib = bz.load_library()
    h = ctypes.c_void_p()
    for kw in [dict(N=12), dict(L=-1.0), dict(n_theta=3), dict(n_phi=0), dict(n_rho=0), dict(precision=7)]:
        base = dict(N=8, L=4.0, gamma=0.0, n_theta=2, n_phi=4, n_rho=2, R=0.0, precision=0, device=0)
        base.update(kw)
        p = bz.bz_params(**base)
        assert lib.bz_create(ctypes.byref(p), ctypes.byref(h)) == 1  # BZ_EINVAL
        assert not h.value


def test_status_strings():
    lib = bz.load_library()
    assert lib.bz_status_str(0) == b"ok"
    assert lib.bz_status_str(1) == b"invalid argument"
