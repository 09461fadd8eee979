"""The C-ABI library loads on a machine without a GPU and exports every
entry point include/esdg.h declares; host-only pieces are checked here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esdg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(esdg_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("esdg_mesh_create", "esdg_rhs", "esdg_lsrk_step", "esdg_entropy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2605_16684_amd import esdg
    lib = C.CDLL(esdg.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in esdg.SIGNATURES, name
    assert set(esdg.SIGNATURES) == set(_declared())


@pytest.mark.parametrize("N", range(1, 16))
def test_library_lgl_tables_match_oracle(N):
    from paper_2605_16684_amd import esdg
    x, w, D = esdg.lgl_tables(N)
    xo, wo, Do = O.lgl(N)
    assert np.max(np.abs(x - xo)) <= 2.3e-16
    assert np.max(np.abs(w - wo)) <= 4.5e-16
    assert np.max(np.abs(D - Do)) <= 1e-13 * N * N


def test_invalid_arguments_fail_without_touching_the_device():
    from paper_2605_16684_amd import esdg
    d = esdg.MeshDesc()
    d.N = 0
    d.K[:] = [1, 1, 1]
    d.hi[:] = [1.0, 1.0, 1.0]
    d.gamma, d.gas_R = 1.4, 287.0
    h = C.c_void_p()
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "N=0" in esdg.last_error()
    d.N = 4
    d.periodic[:] = [0, 0, 1]
    d.grav = 9.81
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "periodic z" in esdg.last_error()
    d.periodic[:] = [0, 0, 0]
    d.K[:] = [4, 0, 4]  # empty mesh
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "K[1]=0" in esdg.last_error()
    d.K[:] = [2048, 2048, 1024]  # 2^32 elements
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "2^31" in esdg.last_error()
    d.K[:] = [2, 2, 2]
    d.hi[:] = [1.0, 0.0, 1.0]
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    d.hi[:] = [1.0, 1.0, 1.0]
    d.gamma = 1.0
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    d.gamma = 1.4
    d.surface_flux = 7
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    d.surface_flux = 0
    d.precision = 3
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    d.precision = 0
    d.epw = 6  # not a compiled variant at N=4
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "no kernel variant" in esdg.last_error()
    d.epw = 0
    d.curved = 2
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    d.curved = 1
    d.precision = esdg.FP32_MIXED
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "curved" in esdg.last_error()
    d.precision = 0
    d.warp[:] = [0.0, float("nan"), 0.0]
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "warp" in esdg.last_error()
    assert esdg.lib.esdg_rhs(None, None, None, 0.0) == esdg.ESDG_EINVAL
    assert esdg.lib.esdg_lgl_tables(4, None, None, None) == esdg.ESDG_EINVAL  # NULL outputs
    buf = (C.c_double * 256)()
    assert esdg.lib.esdg_lgl_tables(16, buf, buf, buf) == esdg.ESDG_EINVAL  # order above 15
    assert "N=16" in esdg.last_error()


def test_high_orders_are_fp64_affine_and_unpacked():
    from paper_2605_16684_amd import esdg
    assert esdg.epw_options(12) == []
    d = esdg.MeshDesc()
    d.N = 16
    d.K[:] = [1, 1, 1]
    d.hi[:] = [1.0, 1.0, 1.0]
    d.gamma, d.gas_R = 1.4, 287.0
    h = C.c_void_p()
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "N=16" in esdg.last_error()
    d.N = 11
    d.precision = esdg.FP32_MIXED
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    assert "FP64" in esdg.last_error()
    d.precision = esdg.FP64
    d.curved = 1
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
    d.curved = 0
    d.epw = 2
    assert esdg.lib.esdg_mesh_create(C.byref(d), None, C.byref(h)) == esdg.ESDG_EINVAL
