"""The C-ABI library loads and exports every entry point of include/stokes.h (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "stokes.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stk_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    assert "stk_create" in names and "stk_solve" in names and len(names) >= 20


def test_library_exports_all_declared_symbols():
    from paper_2506_04157_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libstokes.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_host_only_entry_points():
    from paper_2506_04157_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libstokes.so not built")
    lib = _lib.load()
    p = _lib.SolverParams()
    lib.stk_default_params(ctypes.byref(p))
    assert (p.sigma, p.omega, p.tol_A, p.m_A, p.deg_A, p.m_V, p.deg_V) == (1.0, 0.3, 1e-2, 3, 2, 1, 1)
    assert (p.tol_vbfbt, p.tol_invmass, p.tol_coarse) == (1e-1, 1e-10, 1e-2)
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    d = _lib.MeshDesc(kind=7, level=1)
    assert lib.stk_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.STK_EINVAL
    assert b"mesh kind" in lib.stk_last_error()
    d = _lib.MeshDesc(kind=0, level=1, min_level=0, bc_inner=2)
    assert lib.stk_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.STK_EINVAL
    assert lib.stk_create(None, None, ctypes.byref(h)) == _lib.STK_EINVAL


def test_node_count_limit_refused_before_device_work():
    """The kernels index nodes with signed 32-bit integers: meshes with 2^31
    or more P2 (or P1) nodes are refused from the closed-form counts before
    any device call (a 15x4 shell at level 5 has 2.37e9 P2 nodes; the 10x2
    shell at level 5, 5.28e8, is below the limit and is not refused for its
    size)."""
    from oracle.mesh import shell_counts
    from paper_2506_04157_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libstokes.so not built")
    lib = _lib.load()
    assert shell_counts(15, 4, 5)[0] >= 2 ** 31 > shell_counts(10, 2, 5)[0]
    h = ctypes.c_void_p()
    d = _lib.MeshDesc(kind=1, n_tan=15, n_rad=4, r_in=0.55, r_out=1.0, level=5, min_level=0, bc_inner=1, bc_outer=2)
    assert lib.stk_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.STK_EINVAL
    assert b"2^31" in lib.stk_last_error()
    d = _lib.MeshDesc(kind=1, n_tan=1000, n_rad=1000, r_in=0.55, r_out=1.0, level=7, min_level=0, bc_inner=1,
                      bc_outer=2)
    assert lib.stk_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.STK_EINVAL
