"""Thin Python layer over the C ABI: torch tensors carry device memory and the
stream; every operation runs in the library's HIP kernels."""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (BC_DIRICHLET, BC_FREESLIP, MESH_CUBE, MESH_SHELL, MeshDesc, Report, SolverParams,
                   check, load)


def default_params(**kw):
    p = SolverParams()
    load().stk_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _prec(t):
    if t.dtype == torch.float64:
        return 64
    if t.dtype == torch.float32:
        return 32
    raise TypeError("vectors must be float64 or float32")


class StokesContext:
    """A mesh hierarchy and its fields on one GPU (see include/stokes.h)."""

    def __init__(self, kind="shell", level=1, min_level=0, n_tan=1, n_rad=1, r_in=0.55, r_out=1.0,
                 bc_inner=BC_DIRICHLET, bc_outer=BC_FREESLIP, device="cuda:0"):
        self.device = torch.device(device)
        self.lib = load()
        d = MeshDesc()
        d.kind = MESH_CUBE if kind == "cube" else MESH_SHELL
        d.n_tan, d.n_rad, d.r_in, d.r_out = n_tan, n_rad, r_in, r_out
        d.level, d.min_level = level, min_level
        d.bc_inner, d.bc_outer = bc_inner, bc_outer
        self.desc = d
        self.level, self.min_level = level, min_level
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            check(self.lib.stk_create(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.params = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.stk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- sizes and node coordinates ------------------------------------------
    def sizes(self, level=None):
        level = self.level if level is None else level
        a, b = ctypes.c_int64(), ctypes.c_int64()
        check(self.lib.stk_sizes(self.h, level, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def coords(self, level=None, which=2):
        level = self.level if level is None else level
        n2, n1 = self.sizes(level)
        n = n2 if which == 2 else n1
        xyz = np.zeros((n, 3))
        flags = np.zeros(n, dtype=np.uint8)
        check(self.lib.stk_coords(self.h, level, which, xyz.ctypes.data_as(ctypes.c_void_p),
                                  flags.ctypes.data_as(ctypes.c_void_p)))
        return xyz, flags

    def zeros_u(self, level=None, dtype=torch.float64):
        return torch.zeros(3 * self.sizes(level)[0], dtype=dtype, device=self.device)

    def zeros_p(self, level=None, dtype=torch.float64):
        return torch.zeros(self.sizes(level)[1], dtype=dtype, device=self.device)

    # -- fields ------------------------------------------------------------------
    def set_fields(self, eta, lnrho=None, params=None):
        self.params = params or default_params()
        check(self.lib.stk_set_fields(self.h, _ptr(eta), _ptr(lnrho), ctypes.byref(self.params)))

    def set_log_viscosity(self, m, lnrho=None, params=None):
        self.params = params or default_params()
        check(self.lib.stk_set_log_viscosity(self.h, _ptr(m), _ptr(lnrho), ctypes.byref(self.params)))

    def set_temperature_viscosity(self, T, eta_base, E_A=4.610, V_A=2.996, l_eta=-1, lnrho=None, params=None):
        """eta(x, T) of the geodynamic model from the P2 temperature T (device,
        FP64); quadrature-point evaluation on levels min_level .. l_eta."""
        self.params = params or default_params()
        base = np.ascontiguousarray(eta_base, dtype=np.float64)
        check(self.lib.stk_set_temperature_viscosity(
            self.h, _ptr(T), _ptr(lnrho), base.ctypes.data_as(ctypes.c_void_p), len(base), float(E_A), float(V_A),
            int(l_eta), ctypes.byref(self.params)))

    def rhs_buoyancy(self, T, scale=1.0, out=None):
        out = self.zeros_u() if out is None else out
        check(self.lib.stk_rhs_buoyancy(self.h, _ptr(T), float(scale), _ptr(out)))
        return out

    # -- operators -------------------------------------------------------------------
    def apply_A(self, x, level=None, bc=3, out=None):
        level = self.level if level is None else level
        out = torch.empty_like(x) if out is None else out
        check(self.lib.stk_apply_A(self.h, level, _prec(x), _ptr(x), _ptr(out), bc))
        return out

    def apply_B(self, u, level=None, with_C=False, bc=1, out=None):
        level = self.level if level is None else level
        out = self.zeros_p(level, u.dtype) if out is None else out
        check(self.lib.stk_apply_B(self.h, level, _prec(u), _ptr(u), _ptr(out), int(with_C), bc))
        return out

    def apply_Bt(self, p, level=None, with_Ct=False, bc=2, out=None):
        level = self.level if level is None else level
        out = self.zeros_u(level, p.dtype) if out is None else out
        check(self.lib.stk_apply_Bt(self.h, level, _prec(p), _ptr(p), _ptr(out), int(with_Ct), bc))
        return out

    def apply_K(self, u, p, transpose=False, bc=3):
        yu, yp = torch.empty_like(u), torch.empty_like(p)
        check(self.lib.stk_apply_K(self.h, _prec(u), _ptr(u), _ptr(p), _ptr(yu), _ptr(yp), int(transpose), bc))
        return yu, yp

    def apply_mass(self, p, level=None):
        level = self.level if level is None else level
        out = torch.empty_like(p)
        check(self.lib.stk_apply_mass(self.h, level, _prec(p), _ptr(p), _ptr(out)))
        return out

    def diag_A(self, level=None):
        level = self.level if level is None else level
        out = self.zeros_u(level)
        check(self.lib.stk_diag_A(self.h, level, _ptr(out)))
        return out

    def cheb_bounds(self, level=None):
        level = self.level if level is None else level
        lo, hi = ctypes.c_double(), ctypes.c_double()
        check(self.lib.stk_cheb_bounds(self.h, level, ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def set_cheb_bounds(self, level, lo, hi):
        check(self.lib.stk_set_cheb_bounds(self.h, level, float(lo), float(hi)))

    def smooth(self, b, x, level=None, degree=2, steps=3):
        level = self.level if level is None else level
        check(self.lib.stk_smooth(self.h, level, _prec(b), _ptr(b), _ptr(x), degree, steps))
        return x

    def prolong(self, ec, level):
        out = self.zeros_u(level, ec.dtype)
        check(self.lib.stk_prolong(self.h, level, _prec(ec), _ptr(ec), _ptr(out)))
        return out

    def restrict(self, rf, level):
        out = self.zeros_u(level - 1, rf.dtype)
        check(self.lib.stk_restrict(self.h, level, _prec(rf), _ptr(rf), _ptr(out)))
        return out

    def vcycle(self, b, params=None, which=0):
        params = params or self.params or default_params()
        x = torch.empty_like(b)
        check(self.lib.stk_vcycle(self.h, ctypes.byref(params), _prec(b), _ptr(b), _ptr(x), which))
        return x

    # -- solves ------------------------------------------------------------------------
    def solve(self, f, g=None, u_dirichlet=None, params=None, allow_noconv=False):
        params = params or self.params or default_params()
        u, p = self.zeros_u(), self.zeros_p()
        rep = Report()
        rc = self.lib.stk_solve(self.h, ctypes.byref(params), _ptr(f), _ptr(g), _ptr(u_dirichlet), _ptr(u),
                                _ptr(p), ctypes.byref(rep))
        if not (allow_noconv and rc == _lib.STK_ENOCONV):
            check(rc)
        return u, p, rep.as_dict()

    def precondition(self, ru, rp, params=None, transpose=False):
        """One application of the block preconditioner to the residual [ru; rp]."""
        params = params or self.params or default_params()
        zu, zp = self.zeros_u(), self.zeros_p()
        check(self.lib.stk_precondition(self.h, ctypes.byref(params), _ptr(ru), _ptr(rp), _ptr(zu), _ptr(zp),
                                        int(transpose)))
        return zu, zp

    def solve_adjoint(self, ju, jp=None, params=None):
        params = params or self.params or default_params()
        jp = self.zeros_p() if jp is None else jp
        lu, lp = self.zeros_u(), self.zeros_p()
        rep = Report()
        check(self.lib.stk_solve_adjoint(self.h, ctypes.byref(params), _ptr(ju), _ptr(jp), _ptr(lu), _ptr(lp),
                                         ctypes.byref(rep)))
        return lu, lp, rep.as_dict()

    def gradient(self, u, lu, scale=1.0):
        gm, gT = self.zeros_p(), torch.zeros(self.sizes()[0], dtype=torch.float64, device=self.device)
        check(self.lib.stk_gradient(self.h, _ptr(u), _ptr(lu), float(scale), _ptr(gm), _ptr(gT)))
        return gm, gT

    def time_apply_A(self, x, y, reps=20, level=None):
        """(ms per A-apply operator, ms per plane-sweep kernel launch)."""
        level = self.level if level is None else level
        ms, mk = ctypes.c_double(), ctypes.c_double()
        check(self.lib.stk_time_apply_A(self.h, level, _prec(x), _ptr(x), _ptr(y), reps, ctypes.byref(ms),
                                        ctypes.byref(mk)))
        return ms.value, mk.value
