"""GPU parity of the quadrature-point viscosity on the coarse levels
(Sec. 5.2.2) with the viscosity model of eq. ViscosityDef, against the oracle.

Levels min_level .. l_eta evaluate eta(x_q, T_h(x_q)) at the quadrature points
from the P2 temperature injected to that level; the levels above take the P1
interpolant of the vertex values.  Synthetic inputs: the spherical-harmonic
temperature of the shell workload and a synthetic radial base profile in
place of the paper's figure; E_A and V_A as in the paper.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle.fem import assemble_A, assemble_A_qp, assemble_B, rhs_buoyancy, viscosity_model
from oracle.system import solve_stokes
from paper_2506_04157_amd import default_params
from tests._util import Pair, relerr

pytestmark = pytest.mark.gpu

E_A, V_A = 4.610, 2.996


def _model(base):
    return lambda X, Tq: viscosity_model(X, Tq, base, E_A, V_A, 0.55, 1.0)


@pytest.fixture(scope="module")
def shell():
    print("\n[qp viscosity shell L2]", flush=True)
    P = Pair("shell", 2, min_level=0, n_tan=1, n_rad=1)
    field = inputs.SHField(2)
    base = inputs.base_viscosity_profile()
    return P, field, base


@pytest.mark.parametrize("l_eta", [0, 1])
def test_operator_and_diagonal_per_level(shell, l_eta):
    P, field, base = shell
    T = field.temperature(P.meshes[2].X2)
    P.ctx.set_temperature_viscosity(P.s2_to_lib(T), base, E_A, V_A, l_eta=l_eta)
    for l, m in sorted(P.meshes.items()):
        Tl = field.temperature(m.X2)
        if l <= l_eta:
            Aref = assemble_A_qp(m, _model(base), Tl)
        else:
            Aref = assemble_A(m, viscosity_model(m.X1, field.temperature(m.X1), base, E_A, V_A, 0.55, 1.0))
        d = P.u_to_or(P.ctx.diag_A(l), l)
        print(l, l_eta, relerr(d, Aref.diagonal()))
        assert relerr(d, Aref.diagonal()) < 1e-12
        x = inputs.uniform(30 + l, 3 * m.n2)
        for dtype, tol in [(torch.float64, 1e-12), (torch.float32, 2e-5)]:
            y = P.u_to_or(P.ctx.apply_A(P.u_to_lib(x, l, dtype), level=l, bc=0), l)
            assert relerr(y, Aref @ x) < tol, (l, dtype)


def test_quadrature_point_viscosity_differs_from_p1_on_coarse_levels(shell):
    """The two coarse operators are not the same (otherwise the parity above
    would not test the quadrature-point path)."""
    P, field, base = shell
    m = P.meshes[0]
    Tl = field.temperature(m.X2)
    Aq = assemble_A_qp(m, _model(base), Tl)
    A1 = assemble_A(m, viscosity_model(m.X1, field.temperature(m.X1), base, E_A, V_A, 0.55, 1.0))
    assert abs(Aq - A1).max() > 1e-2 * abs(A1).max()


@pytest.mark.parametrize("precision", [64, 32])
def test_solve_with_quadrature_point_coarse_viscosity(shell, precision):
    """The finest operator keeps the P1 viscosity, so the solution is the
    oracle's P1 one; only the preconditioner's coarse levels change."""
    P, field, base = shell
    m = P.meshes[2]
    T = field.temperature(m.X2)
    eta1 = viscosity_model(m.X1, field.temperature(m.X1), base, E_A, V_A, 0.55, 1.0)
    lnrho = inputs.ln_density(m.X1)
    f = rhs_buoyancy(m, T)
    A = assemble_A(m, eta1)
    B = assemble_B(m)
    Bb = B + assemble_B(m, lnrho, only_C=True)
    _, Q = P.projector()
    uo, po, _ = solve_stokes(A, Bb, f, np.zeros(m.n1), Q, Bt=B.T)
    its = {}
    for l_eta in (-1, 1):
        params = default_params(tol_rel=1e-9, precision=precision)
        P.ctx.set_temperature_viscosity(P.s2_to_lib(T), base, E_A, V_A, l_eta=l_eta, lnrho=P.p_to_lib(lnrho),
                                        params=params)
        u, p, rep = P.ctx.solve(P.u_to_lib(f), params=params)
        its[l_eta] = (rep["iterations"], rep["a_cg_its"])
        assert rep["rel_residual"] <= 1e-9
        assert relerr(P.u_to_or(u), uo) < 1e-6 and relerr(P.p_to_or(p), po) < 1e-5
    print("FGMRES / A-block CG iterations by l_eta:", its)
