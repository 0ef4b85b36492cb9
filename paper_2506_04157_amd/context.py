"""Thin Python layer over the C ABI: torch tensors carry device memory and the
stream; every operation runs in the library's HIP kernels."""
import ctypes
import sys

import numpy as np
import torch

from . import _lib
from ._lib import (BC_DIRICHLET, BC_FREESLIP, MESH_CUBE, MESH_SHELL, MeshDesc, Report, SolverParams,
                   TempParams, TempReport, check, load)


def default_params(**kw):
    p = SolverParams()
    load().stk_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def temp_params(**kw):
    """Parameters of the temperature step (stk_temp_params) with overrides."""
    p = TempParams()
    load().stk_temp_default_params(ctypes.byref(p))
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
    """A mesh hierarchy and its fields on one GPU (see include/stokes.h).

    Every vector argument is checked here (device, contiguity, dtype and
    length) before the library sees its pointer, so a wrong tensor raises
    ValueError instead of reaching a kernel.  Usable as a context manager;
    close() releases the device memory."""

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
        self.generation = 0   # counts field changes (set_fields, set_log_viscosity, ...)

    def close(self):
        if getattr(self, "h", None):
            self.lib.stk_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        # during interpreter shutdown the HIP runtime (and a profiler's hooks)
        # may already be gone: leave the memory to the process exit then
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks ------------------------------------------------------------
    def _vec(self, t, n, dtypes=(torch.float64,), name="vector"):
        """Pointer of a contiguous device tensor with n elements of one of `dtypes`."""
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor")
        if not t.is_cuda or t.device.index != (self.device.index or 0):
            raise ValueError(f"{name}: expected a tensor on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous tensor")
        if t.dtype not in dtypes:
            raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
        if t.numel() != n:
            raise ValueError(f"{name}: {t.numel()} elements, expected {n}")
        return ctypes.c_void_p(t.data_ptr())

    def _u(self, t, level=None, dtypes=(torch.float64,), name="velocity"):
        return self._vec(t, 3 * self.sizes(level)[0], dtypes, name)

    def _p(self, t, level=None, dtypes=(torch.float64,), name="pressure"):
        return self._vec(t, self.sizes(level)[1], dtypes, name)

    def _s2(self, t, level=None, name="P2 scalar"):
        return self._vec(t, self.sizes(level)[0], (torch.float64,), name)

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
        a, b = self._p(eta, name="eta"), self._p(lnrho, name="lnrho")
        self.params = params or default_params()
        self.generation += 1
        check(self.lib.stk_set_fields(self.h, a, b, ctypes.byref(self.params)))

    def set_log_viscosity(self, m, lnrho=None, params=None):
        a, b = self._p(m, name="m"), self._p(lnrho, name="lnrho")
        self.params = params or default_params()
        self.generation += 1
        check(self.lib.stk_set_log_viscosity(self.h, a, b, ctypes.byref(self.params)))

    def set_temperature_viscosity(self, T, eta_base, E_A=4.610, V_A=2.996, l_eta=-1, lnrho=None, params=None):
        """eta(x, T) of the geodynamic model from the P2 temperature T (device,
        FP64); quadrature-point evaluation on levels min_level .. l_eta."""
        a, b = self._s2(T, name="T"), self._p(lnrho, name="lnrho")
        self.params = params or default_params()
        base = np.ascontiguousarray(eta_base, dtype=np.float64)
        self.generation += 1
        check(self.lib.stk_set_temperature_viscosity(
            self.h, a, b, base.ctypes.data_as(ctypes.c_void_p), len(base), float(E_A), float(V_A),
            int(l_eta), ctypes.byref(self.params)))

    def rhs_buoyancy(self, T, scale=1.0, out=None):
        out = self.zeros_u() if out is None else out
        check(self.lib.stk_rhs_buoyancy(self.h, self._s2(T, name="T"), float(scale), self._u(out, name="out")))
        return out

    # -- operators -------------------------------------------------------------------
    def apply_A(self, x, level=None, bc=3, out=None):
        level = self.level if level is None else level
        out = torch.empty_like(x) if out is None else out
        fl = (x.dtype,)
        a = self._u(x, level, (torch.float64, torch.float32), "x")
        check(self.lib.stk_apply_A(self.h, level, _prec(x), a, self._u(out, level, fl, "out"), bc))
        return out

    def apply_A_noalloc(self, x, out, level=None, bc=3):
        """A-apply through the entry point that allocates no device memory
        (its scratch is a fixed per-GPU array); `out` is caller-provided."""
        level = self.level if level is None else level
        a = self._u(x, level, (torch.float64, torch.float32), "x")
        b = self._u(out, level, (x.dtype,), "out")
        check(self.lib.stk_apply_A_noalloc(self.h, level, _prec(x), a, b, bc))
        return out

    def apply_B(self, u, level=None, with_C=False, bc=1, out=None):
        level = self.level if level is None else level
        out = self.zeros_p(level, u.dtype) if out is None else out
        a = self._u(u, level, (torch.float64, torch.float32), "u")
        b = self._p(out, level, (u.dtype,), "out")
        check(self.lib.stk_apply_B(self.h, level, _prec(u), a, b, int(with_C), bc))
        return out

    def apply_Bt(self, p, level=None, with_Ct=False, bc=2, out=None):
        level = self.level if level is None else level
        out = self.zeros_u(level, p.dtype) if out is None else out
        a = self._p(p, level, (torch.float64, torch.float32), "p")
        b = self._u(out, level, (p.dtype,), "out")
        check(self.lib.stk_apply_Bt(self.h, level, _prec(p), a, b, int(with_Ct), bc))
        return out

    def apply_K(self, u, p, transpose=False, bc=3):
        a = self._u(u, None, (torch.float64, torch.float32), "u")
        b = self._p(p, None, (u.dtype,), "p")
        yu, yp = torch.empty_like(u), torch.empty_like(p)
        check(self.lib.stk_apply_K(self.h, _prec(u), a, b, _ptr(yu), _ptr(yp), int(transpose), bc))
        return yu, yp

    def apply_mass(self, p, level=None):
        level = self.level if level is None else level
        a = self._p(p, level, (torch.float64, torch.float32), "p")
        out = torch.empty_like(p)
        check(self.lib.stk_apply_mass(self.h, level, _prec(p), a, _ptr(out)))
        return out

    def apply_vmass(self, u, a=1.0, bc=3, out=None):
        """M_{sqrt eta} u on the finest level (weighted BFBT), element factor a^2
        on the micro-tets touching a Dirichlet boundary."""
        out = torch.empty_like(u) if out is None else out
        x = self._u(u, None, (torch.float64, torch.float32), "u")
        check(self.lib.stk_apply_vmass(self.h, _prec(u), float(a), x, self._u(out, None, (u.dtype,), "out"), bc))
        return out

    def apply_poisson(self, p, level=None, a=1.0, out=None):
        """K_{1/sqrt eta} p on `level` (the weighted BFBT's Poisson operator)."""
        level = self.level if level is None else level
        out = torch.empty_like(p) if out is None else out
        x = self._p(p, level, (torch.float64, torch.float32), "p")
        check(self.lib.stk_apply_poisson(self.h, level, _prec(p), float(a), x,
                                         self._p(out, level, (p.dtype,), "out")))
        return out

    def p1_transfer(self, v, level, restrict=False):
        """Nested P1 prolongation from level-1 to level (restrict: its transpose)."""
        src, dst = (level, level - 1) if restrict else (level - 1, level)
        x = self._p(v, src, (torch.float64, torch.float32), "v")
        out = self.zeros_p(dst, v.dtype)
        check(self.lib.stk_p1_transfer(self.h, level, _prec(v), int(bool(restrict)), x, _ptr(out)))
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
        pb = self._u(b, level, (torch.float64, torch.float32), "b")
        px = self._u(x, level, (b.dtype,), "x")
        check(self.lib.stk_smooth(self.h, level, _prec(b), pb, px, degree, steps))
        return x

    def prolong(self, ec, level, add_to=None):
        """P_v P ec on `level`; add_to: a fine vector that receives += P_v P ec
        in place (and is returned)."""
        a = self._u(ec, level - 1, (torch.float64, torch.float32), "ec")
        if add_to is None:
            out = self.zeros_u(level, ec.dtype)
        else:
            out = add_to
        b = self._u(out, level, (ec.dtype,), "add_to")
        check(self.lib.stk_prolong(self.h, level, _prec(ec), a, b, int(add_to is not None)))
        return out

    def restrict(self, rf, level, minus=None):
        """P_v P^T rf, or P_v P^T P_v (rf - minus) with a fine vector `minus`."""
        a = self._u(rf, level, (torch.float64, torch.float32), "rf")
        t = self._u(minus, level, (rf.dtype,), "minus")
        out = self.zeros_u(level - 1, rf.dtype)
        check(self.lib.stk_restrict(self.h, level, _prec(rf), a, t, _ptr(out)))
        return out

    def vcycle(self, b, params=None, which=0):
        params = params or self.params or default_params()
        a = self._u(b, None, (torch.float64, torch.float32), "b")
        x = torch.empty_like(b)
        check(self.lib.stk_vcycle(self.h, ctypes.byref(params), _prec(b), a, _ptr(x), which))
        return x

    # -- solves ------------------------------------------------------------------------
    def solve(self, f, g=None, u_dirichlet=None, params=None, allow_noconv=False, u0=None, p0=None):
        """u0, p0 (optional): the initial guess of FGMRES (initial_guess = 1)."""
        params = params or self.params or default_params()
        pf, pg = self._u(f, name="f"), self._p(g, name="g")
        pd = self._u(u_dirichlet, name="u_dirichlet")
        u, p = self.zeros_u(), self.zeros_p()
        if u0 is not None or p0 is not None:
            if u0 is not None:
                self._u(u0, name="u0")
                u.copy_(u0)
            if p0 is not None:
                self._p(p0, name="p0")
                p.copy_(p0)
            params = SolverParams.from_buffer_copy(params)
            params.initial_guess = 1
        rep = Report()
        rc = self.lib.stk_solve(self.h, ctypes.byref(params), pf, pg, pd, _ptr(u), _ptr(p), ctypes.byref(rep))
        if not (allow_noconv and rc == _lib.STK_ENOCONV):
            check(rc)
        return u, p, rep.as_dict()

    def precondition(self, ru, rp, params=None, transpose=False):
        """One application of the block preconditioner to the residual [ru; rp]."""
        params = params or self.params or default_params()
        a, b = self._u(ru, name="ru"), self._p(rp, name="rp")
        zu, zp = self.zeros_u(), self.zeros_p()
        check(self.lib.stk_precondition(self.h, ctypes.byref(params), a, b, _ptr(zu), _ptr(zp), int(transpose)))
        return zu, zp

    def solve_adjoint(self, ju, jp=None, params=None, allow_noconv=False):
        params = params or self.params or default_params()
        jp = self.zeros_p() if jp is None else jp
        a, b = self._u(ju, name="ju"), self._p(jp, name="jp")
        lu, lp = self.zeros_u(), self.zeros_p()
        rep = Report()
        rc = self.lib.stk_solve_adjoint(self.h, ctypes.byref(params), a, b, _ptr(lu), _ptr(lp), ctypes.byref(rep))
        if not (allow_noconv and rc == _lib.STK_ENOCONV):
            check(rc)
        return lu, lp, rep.as_dict()

    def gradient(self, u, lu, scale=1.0):
        a, b = self._u(u, name="u"), self._u(lu, name="lu")
        gm, gT = self.zeros_p(), torch.zeros(self.sizes()[0], dtype=torch.float64, device=self.device)
        check(self.lib.stk_gradient(self.h, a, b, float(scale), _ptr(gm), _ptr(gT)))
        return gm, gT

    def time_apply_A(self, x, y, reps=20, level=None):
        """(ms per A-apply operator, ms per plane-sweep kernel launch)."""
        level = self.level if level is None else level
        a = self._u(x, level, (torch.float64, torch.float32), "x")
        b = self._u(y, level, (x.dtype,), "y")
        ms, mk = ctypes.c_double(), ctypes.c_double()
        check(self.lib.stk_time_apply_A(self.h, level, _prec(x), a, b, reps, ctypes.byref(ms), ctypes.byref(mk)))
        return ms.value, mk.value

    def kernel_timer(self, enable):
        """enable=True: start bracketing every finest-level A sweep kernel with
        HIP events; enable=False: stop and return (summed ms, launches)."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        check(self.lib.stk_kernel_timer(self.h, int(bool(enable)), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # -- temperature step (Sec. 3, eq. WeakTemp) --------------------------------------
    def _s1(self, t, name):
        return self._vec(t, self.sizes()[1], (torch.float64,), name)

    def temp_apply(self, x, params, mode=0, u_star=None, lnrho=None, out=None):
        """mode 0: L x; 1: the symmetric part S x; 2: diag(S) (x ignored)."""
        n2 = self.sizes()[0]
        out = torch.empty(n2, dtype=torch.float64, device=self.device) if out is None else out
        check(self.lib.stk_temp_apply(self.h, ctypes.byref(params), int(mode), self._u(u_star, name="u_star"),
                                      self._s1(lnrho, "lnrho"), self._s2(x, name="x"), self._s2(out, name="out")))
        return out

    def temp_rhs(self, That_n, That_nm1, params, u_star=None, lnrho=None, eta=None, out=None):
        n2 = self.sizes()[0]
        out = torch.empty(n2, dtype=torch.float64, device=self.device) if out is None else out
        check(self.lib.stk_temp_rhs(self.h, ctypes.byref(params), self._u(u_star, name="u_star"),
                                    self._s1(lnrho, "lnrho"), self._s1(eta, "eta"), self._s2(That_n, name="That_n"),
                                    self._s2(That_nm1, name="That_nm1"), self._s2(out, name="out")))
        return out

    def mmoc(self, F, u_new, u_old, tau, out=None):
        out = torch.empty_like(F) if out is None else out
        check(self.lib.stk_mmoc(self.h, self._s2(F, name="F"), self._u(u_new, name="u_new"),
                                self._u(u_old, name="u_old"), float(tau), self._s2(out, name="out")))
        return out

    def temp_solve(self, b, params, u_star=None, lnrho=None, T_init=None, allow_noconv=False):
        T = torch.empty_like(b)
        rep = TempReport()
        rc = self.lib.stk_temp_solve(self.h, ctypes.byref(params), self._u(u_star, name="u_star"),
                                     self._s1(lnrho, "lnrho"), self._s2(b, name="b"), self._s2(T_init, name="T_init"),
                                     self._s2(T, name="T"), ctypes.byref(rep))
        if not (allow_noconv and rc == _lib.STK_ENOCONV):
            check(rc)
        return T, rep.as_dict()

    def temperature_step(self, T_n, T_nm1, u_n, u_nm1, eta, params, lnrho=None, traced=False, allow_noconv=False):
        """T^{n+1} (and, with traced=True, the traced history values)."""
        T = torch.empty_like(T_n)
        thn = torch.empty_like(T_n) if traced else None
        thm = torch.empty_like(T_n) if traced else None
        rep = TempReport()
        rc = self.lib.stk_temperature_step(
            self.h, ctypes.byref(params), self._s2(T_n, name="T_n"), self._s2(T_nm1, name="T_nm1"),
            self._u(u_n, name="u_n"), self._u(u_nm1, name="u_nm1"), self._s1(lnrho, "lnrho"), self._s1(eta, "eta"),
            self._s2(T, name="T"), self._s2(thn, name="That_n"), self._s2(thm, name="That_nm1"), ctypes.byref(rep))
        if not (allow_noconv and rc == _lib.STK_ENOCONV):
            check(rc)
        return (T, thn, thm, rep.as_dict()) if traced else (T, rep.as_dict())

    def coupled_step(self, T_n, T_nm1, u_n, u_nm1, eta_base, tparams, params=None, E_A=4.610, V_A=2.996,
                     l_eta=-1, buoyancy_scale=1.0, lnrho=None, p_n=None, allow_noconv=False):
        """One step of the coupled scheme (temperature, then Stokes at the new
        temperature): (T^{n+1}, u^{n+1}, p^{n+1}, temperature report, Stokes report)."""
        params = params or self.params or default_params()
        base = np.ascontiguousarray(eta_base, dtype=np.float64)
        T = torch.empty_like(T_n)
        u, p = self.zeros_u(), self.zeros_p()
        trep, srep = TempReport(), Report()
        rc = self.lib.stk_coupled_step(
            self.h, ctypes.byref(params), ctypes.byref(tparams), base.ctypes.data_as(ctypes.c_void_p), len(base),
            float(E_A), float(V_A), int(l_eta), float(buoyancy_scale), self._s1(lnrho, "lnrho"),
            self._s2(T_n, name="T_n"), self._s2(T_nm1, name="T_nm1"), self._u(u_n, name="u_n"),
            self._u(u_nm1, name="u_nm1"), self._p(p_n, name="p_n"), self._s2(T, name="T_np1"), self._u(u, name="u_np1"),
            self._p(p, name="p_np1"), ctypes.byref(trep), ctypes.byref(srep))
        if not (allow_noconv and rc == _lib.STK_ENOCONV):
            check(rc)
        self.params = params
        self.generation += 1
        return T, u, p, trep.as_dict(), srep.as_dict()
