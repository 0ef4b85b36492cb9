"""GPU parity of the operator applies against the assembled FP64 oracle.

Bars: FP64 applies 1e-12 relative (Euclidean norm), FP32 applies 1e-5; and
per entry, against the entry's scale sum_j |a_ij x_j| (so that a single wrong
node cannot hide in the norm): 1e-13 for FP64, 1e-5 for FP32.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle.fem import assemble_A, assemble_B, assemble_M_inv_eta, rhs_buoyancy
from tests._util import Pair, relerr, rowerr

pytestmark = pytest.mark.gpu

CASES = [("cube", 2, 1, 1), ("shell", 2, 1, 1), ("shell", 1, 2, 1), ("cube", 3, 1, 1)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-L{c[1]}-{c[2]}x{c[3]}")
def case(request):
    kind, L, nt, nr = request.param
    print(f"\n[case {kind} L{L} {nt}x{nr}]", flush=True)
    P = Pair(kind, L, min_level=0, n_tan=nt, n_rad=nr)
    m = P.meshes[L]
    rng = np.random.default_rng(11)
    eta = rng.uniform(0.1, 10.0, m.n1)
    lnrho = inputs.ln_density(m.X1) if kind == "shell" else m.X1 @ np.array([0.3, -0.5, 0.2])
    P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho))
    A = assemble_A(m, eta)
    B = assemble_B(m)
    C = assemble_B(m, lnrho, only_C=True)
    M = assemble_M_inv_eta(m, eta)
    Pu, Q = P.projector()
    x = inputs.uniform(0, 3 * m.n2)
    p = inputs.uniform(1, m.n1)
    return dict(P=P, m=m, eta=eta, A=A, B=B, C=C, M=M, Pu=Pu, x=x, p=p)


ROW_TOL = {torch.float64: 1e-13, torch.float32: 1e-5}


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
@pytest.mark.parametrize("bc", [0, 3])
def test_apply_A(case, dtype, tol, bc):
    P, A, Pu, x = case["P"], case["A"], case["Pu"], case["x"]
    y = P.u_to_or(P.ctx.apply_A(P.u_to_lib(x, dtype=dtype), bc=bc))
    if bc == 0:
        ref, scale = A @ x, abs(A) @ abs(x)
    else:
        ref, scale = Pu @ (A @ (Pu @ x)), abs(Pu) @ (abs(A) @ (abs(Pu) @ abs(x)))
    assert relerr(y, ref) < tol
    assert rowerr(y, ref, scale) < ROW_TOL[dtype]


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
@pytest.mark.parametrize("with_C", [False, True])
def test_apply_B_and_Bt(case, dtype, tol, with_C):
    P, B, C, Pu, x, p = case["P"], case["B"], case["C"], case["Pu"], case["x"], case["p"]
    Bb = B + C if with_C else B
    aB = abs(B) + abs(C) if with_C else abs(B)
    rt = ROW_TOL[dtype]
    q = P.p_to_or(P.ctx.apply_B(P.u_to_lib(x, dtype=dtype), with_C=with_C, bc=0))
    assert relerr(q, Bb @ x) < tol and rowerr(q, Bb @ x, aB @ abs(x)) < rt
    q = P.p_to_or(P.ctx.apply_B(P.u_to_lib(x, dtype=dtype), with_C=with_C, bc=1))
    assert relerr(q, Bb @ (Pu @ x)) < tol and rowerr(q, Bb @ (Pu @ x), aB @ (abs(Pu) @ abs(x))) < rt
    y = P.u_to_or(P.ctx.apply_Bt(P.p_to_lib(p, dtype=dtype), with_Ct=with_C, bc=0))
    assert relerr(y, Bb.T @ p) < tol and rowerr(y, Bb.T @ p, aB.T @ abs(p)) < rt
    y = P.u_to_or(P.ctx.apply_Bt(P.p_to_lib(p, dtype=dtype), with_Ct=with_C, bc=2))
    assert relerr(y, Pu @ (Bb.T @ p)) < tol and rowerr(y, Pu @ (Bb.T @ p), abs(Pu) @ (aB.T @ abs(p))) < rt


@pytest.mark.parametrize("transpose", [False, True])
def test_apply_K(case, transpose):
    P, A, B, C, Pu, x, p = (case[k] for k in ("P", "A", "B", "C", "Pu", "x", "p"))
    yu, yp = P.ctx.apply_K(P.u_to_lib(x), P.p_to_lib(p), transpose=transpose)
    xp = Pu @ x
    if transpose:
        ru, rp = Pu @ (A @ xp + (B + C).T @ p), B @ xp
    else:
        ru, rp = Pu @ (A @ xp + B.T @ p), (B + C) @ xp
    assert relerr(P.u_to_or(yu), ru) < 1e-12
    assert relerr(P.p_to_or(yp), rp) < 1e-12


def test_mass_and_diag(case):
    P, M, A, p = case["P"], case["M"], case["A"], case["p"]
    for dtype, tol in [(torch.float64, 1e-12), (torch.float32, 1e-5)]:
        q = P.p_to_or(P.ctx.apply_mass(P.p_to_lib(p, dtype=dtype)))
        assert relerr(q, M @ p) < tol and rowerr(q, M @ p, abs(M) @ abs(p)) < ROW_TOL[dtype]
    d = P.u_to_or(P.ctx.diag_A())
    assert relerr(d, A.diagonal()) < 1e-12


def test_rhs_buoyancy(case):
    P, m = case["P"], case["m"]
    T = inputs.uniform(5, m.n2, 0.0, 1.0)
    f = P.u_to_or(P.ctx.rhs_buoyancy(P.s2_to_lib(T), scale=2.5))
    assert relerr(f, rhs_buoyancy(m, T, scale=2.5)) < 1e-12
