"""The C-ABI library builds, loads and exports every declared entry point
(CPU only: no compute call is made)."""
from __future__ import annotations

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            names += re.findall(r"^\s*(?:int|void|const char\*)\s+(m2c_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("m2c_create", "m2c_set_state", "m2c_step", "m2c_get_state"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2508_16387_amd as m
    if not os.path.exists(m.lib_path()):
        pytest.fail("libm2c.so not built")
    names = _declared()
    import ctypes
    L = ctypes.CDLL(m.lib_path())
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(m._binding.EXPORTS) == names


def test_config_default_without_gpu():
    import paper_2508_16387_amd as m
    c = m.config_default()
    assert c.struct_size == 156 or c.struct_size > 0
    assert c.rk_order == 2 and abs(c.limiter_alpha - 1.2) < 1e-15
    assert (c.nx, c.ny, c.nz) == (1, 1, 1)


def test_create_rejects_bad_config_without_gpu():
    import ctypes as C
    import paper_2508_16387_amd as m
    c = m.config_default()
    c.nx = 0
    h = C.c_void_p()
    assert m.lib().m2c_create(C.byref(c), C.byref(h)) == m.M2C_ERR_ARG
    c = m.config_default()
    c.bc[0] = m.M2C_BC_PERIODIC        # unpaired periodic side
    assert m.lib().m2c_create(C.byref(c), C.byref(h)) == m.M2C_ERR_ARG
