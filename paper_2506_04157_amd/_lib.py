"""ctypes binding of ``libstokes.so`` (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstokes.so")

STK_OK, STK_EINVAL, STK_ENOMEM, STK_EHIP, STK_ENOCONV, STK_ENOTREADY = 0, -1, -2, -3, -4, -5
MESH_CUBE, MESH_SHELL = 0, 1
BC_DIRICHLET, BC_FREESLIP = 1, 2
UZAWA_SYMMETRIC, UZAWA_INEXACT, UZAWA_ADJOINT = 0, 1, 2
SCHUR_VBFBT, SCHUR_MASS, SCHUR_DIAG_BFBT, SCHUR_WBFBT = 0, 1, 2, 3


class MeshDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_tan", ctypes.c_int), ("n_rad", ctypes.c_int),
                ("r_in", ctypes.c_double), ("r_out", ctypes.c_double), ("level", ctypes.c_int),
                ("min_level", ctypes.c_int), ("bc_inner", ctypes.c_int), ("bc_outer", ctypes.c_int)]


class SolverParams(ctypes.Structure):
    _fields_ = [("tol_rel", ctypes.c_double), ("tol_abs", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("precision", ctypes.c_int), ("sigma", ctypes.c_double),
                ("omega", ctypes.c_double), ("tol_A", ctypes.c_double), ("tol_vbfbt", ctypes.c_double),
                ("tol_invmass", ctypes.c_double), ("tol_coarse", ctypes.c_double), ("m_A", ctypes.c_int),
                ("deg_A", ctypes.c_int), ("m_V", ctypes.c_int), ("deg_V", ctypes.c_int),
                ("max_inner", ctypes.c_int), ("use_Bbar", ctypes.c_int), ("power_its", ctypes.c_int),
                ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double), ("uzawa", ctypes.c_int),
                ("schur", ctypes.c_int), ("a_l", ctypes.c_double), ("a_r", ctypes.c_double),
                ("tol_wbfbt", ctypes.c_double), ("tol_vmass", ctypes.c_double), ("initial_guess", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("abs_residual", ctypes.c_double), ("initial_residual", ctypes.c_double),
                ("a_solves", ctypes.c_int), ("a_cg_its", ctypes.c_int), ("s_solves", ctypes.c_int),
                ("s_cg_its", ctypes.c_int), ("vcycles", ctypes.c_int), ("coarse_its", ctypes.c_int),
                ("mass_its", ctypes.c_int), ("seconds", ctypes.c_double),
                ("history_len", ctypes.c_int), ("history", ctypes.c_double * 256)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "history"}
        d["history"] = list(self.history[: self.history_len])
        return d


class TempParams(ctypes.Structure):
    _fields_ = [("tau1", ctypes.c_double), ("tau0", ctypes.c_double), ("k", ctypes.c_double),
                ("Pe", ctypes.c_double), ("Cp", ctypes.c_double), ("Di", ctypes.c_double),
                ("alpha", ctypes.c_double), ("H", ctypes.c_double), ("Ra", ctypes.c_double),
                ("adv", ctypes.c_double), ("T_in", ctypes.c_double), ("T_out", ctypes.c_double),
                ("tol_abs", ctypes.c_double), ("tol_cg", ctypes.c_double), ("restart", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("max_cg", ctypes.c_int), ("stored_S", ctypes.c_int)]


class TempReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("cg_its", ctypes.c_int), ("converged", ctypes.c_int),
                ("initial_residual", ctypes.c_double), ("abs_residual", ctypes.c_double),
                ("ms_mmoc", ctypes.c_double), ("ms_rhs", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("stored_S", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


TEMP_APPLY, TEMP_SYM, TEMP_DIAG, TEMP_SYM_STORED = 0, 1, 2, 3

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_CTX = ctypes.c_void_p

# name -> argtypes  (every entry point of include/stokes.h)
SIGNATURES = {
    "stk_create": [ctypes.POINTER(MeshDesc), _P, ctypes.POINTER(_CTX)],
    "stk_destroy": [_CTX],
    "stk_default_params": [ctypes.POINTER(SolverParams)],
    "stk_last_error": [],
    "stk_sizes": [_CTX, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "stk_coords": [_CTX, _I, _I, _P, _P],
    "stk_set_fields": [_CTX, _P, _P, ctypes.POINTER(SolverParams)],
    "stk_set_log_viscosity": [_CTX, _P, _P, ctypes.POINTER(SolverParams)],
    "stk_set_temperature_viscosity": [_CTX, _P, _P, _P, _I, _D, _D, _I, ctypes.POINTER(SolverParams)],
    "stk_rhs_buoyancy": [_CTX, _P, _D, _P],
    "stk_apply_A": [_CTX, _I, _I, _P, _P, _I],
    "stk_apply_B": [_CTX, _I, _I, _P, _P, _I, _I],
    "stk_apply_Bt": [_CTX, _I, _I, _P, _P, _I, _I],
    "stk_apply_K": [_CTX, _I, _P, _P, _P, _P, _I, _I],
    "stk_apply_A_noalloc": [_CTX, _I, _I, _P, _P, _I],
    "stk_apply_mass": [_CTX, _I, _I, _P, _P],
    "stk_apply_vmass": [_CTX, _I, _D, _P, _P, _I],
    "stk_apply_poisson": [_CTX, _I, _I, _D, _P, _P],
    "stk_p1_transfer": [_CTX, _I, _I, _I, _P, _P],
    "stk_diag_A": [_CTX, _I, _P],
    "stk_cheb_bounds": [_CTX, _I, ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "stk_set_cheb_bounds": [_CTX, _I, _D, _D],
    "stk_smooth": [_CTX, _I, _I, _P, _P, _I, _I],
    "stk_prolong": [_CTX, _I, _I, _P, _P, _I],
    "stk_restrict": [_CTX, _I, _I, _P, _P, _P],
    "stk_vcycle": [_CTX, ctypes.POINTER(SolverParams), _I, _P, _P, _I],
    "stk_precondition": [_CTX, ctypes.POINTER(SolverParams), _P, _P, _P, _P, _I],
    "stk_solve": [_CTX, ctypes.POINTER(SolverParams), _P, _P, _P, _P, _P, ctypes.POINTER(Report)],
    "stk_solve_adjoint": [_CTX, ctypes.POINTER(SolverParams), _P, _P, _P, _P, ctypes.POINTER(Report)],
    "stk_gradient": [_CTX, _P, _P, _D, _P, _P],
    "stk_time_apply_A": [_CTX, _I, _I, _P, _P, _I, ctypes.POINTER(_D), ctypes.POINTER(_D)],
    "stk_kernel_timer": [_CTX, _I, ctypes.POINTER(_D), ctypes.POINTER(_I)],
    "stk_temp_default_params": [ctypes.POINTER(TempParams)],
    "stk_temp_apply": [_CTX, ctypes.POINTER(TempParams), _I, _P, _P, _P, _P],
    "stk_temp_rhs": [_CTX, ctypes.POINTER(TempParams), _P, _P, _P, _P, _P, _P],
    "stk_mmoc": [_CTX, _P, _P, _P, _D, _P],
    "stk_temp_solve": [_CTX, ctypes.POINTER(TempParams), _P, _P, _P, _P, _P, ctypes.POINTER(TempReport)],
    "stk_temperature_step": [_CTX, ctypes.POINTER(TempParams), _P, _P, _P, _P, _P, _P, _P, _P, _P,
                             ctypes.POINTER(TempReport)],
    "stk_coupled_step": [_CTX, ctypes.POINTER(SolverParams), ctypes.POINTER(TempParams), _P, _I, _D, _D, _I, _D,
                         _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.POINTER(TempReport), ctypes.POINTER(Report)],
}

_lib = None


def load():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "stk_last_error" else (
                None if name in ("stk_default_params", "stk_temp_default_params") else ctypes.c_int)
        _lib = lib
    return _lib


class StokesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc):
    if rc != STK_OK:
        raise StokesError(rc, load().stk_last_error().decode())
    return rc
