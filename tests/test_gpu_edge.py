"""Degenerate and invalid inputs through the C ABI (GPU): a zero right-hand
side, a one-level hierarchy (the V-cycle is the coarse solve alone), and the
errors the ABI promises."""
import numpy as np
import pytest
import torch

import inputs
from oracle.fem import assemble_A, assemble_B
from oracle.system import solve_stokes
from paper_2506_04157_amd import StokesContext, default_params
from paper_2506_04157_amd._lib import STK_EINVAL, STK_ENOTREADY, StokesError
from tests._util import Pair, relerr

pytestmark = pytest.mark.gpu


def test_zero_right_hand_side_gives_zero_solution():
    sc = StokesContext("shell", level=2, min_level=0)
    n2, n1 = sc.sizes()
    sc.set_fields(torch.ones(n1, dtype=torch.float64, device="cuda"))
    for prec in (64, 32):
        u, p, rep = sc.solve(torch.zeros(3 * n2, dtype=torch.float64, device="cuda"),
                             params=default_params(precision=prec))
        assert rep["iterations"] == 0 and rep["initial_residual"] == 0.0
        assert torch.count_nonzero(u).item() == 0 and torch.count_nonzero(p).item() == 0
    sc.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_one_level_hierarchy(precision):
    print(f"\n[one level cube prec {precision}]", flush=True)
    P = Pair("cube", 2, min_level=2)
    m = P.meshes[2]
    eta = np.exp(inputs.uniform(3, m.n1, -1.0, 1.0))
    f = inputs.uniform(4, 3 * m.n2)
    A, B = assemble_A(m, eta), assemble_B(m)
    _, Q = P.projector()
    uo, po, _ = solve_stokes(A, B, f, np.zeros(m.n1), Q, Bt=B.T)
    params = default_params(tol_rel=1e-10, precision=precision)
    P.ctx.set_fields(P.p_to_lib(eta), params=params)
    u, p, rep = P.ctx.solve(P.u_to_lib(f), params=params)
    assert rep["rel_residual"] <= 1e-10
    assert relerr(P.u_to_or(u), uo) < 1e-7 and relerr(P.p_to_or(p), po) < 1e-6


def test_invalid_inputs_are_refused():
    sc = StokesContext("shell", level=1, min_level=0)
    n2, n1 = sc.sizes()
    with pytest.raises(StokesError) as e:
        sc.solve(torch.zeros(3 * n2, dtype=torch.float64, device="cuda"))
    assert e.value.code == STK_ENOTREADY
    for bad in (0.0, -1.0, float("nan")):
        eta = torch.ones(n1, dtype=torch.float64, device="cuda")
        eta[n1 // 2] = bad
        with pytest.raises(StokesError) as e:
            sc.set_fields(eta)
        assert e.value.code == STK_EINVAL
    sc.set_fields(torch.ones(n1, dtype=torch.float64, device="cuda"))
    x = torch.zeros(3 * n2, dtype=torch.float64, device="cuda")
    with pytest.raises(StokesError) as e:
        sc.apply_A(x, level=5)
    assert e.value.code == STK_EINVAL
    T = torch.zeros(n2, dtype=torch.float64, device="cuda")
    with pytest.raises(StokesError) as e:   # l_eta must be below the finest level
        sc.set_temperature_viscosity(T, inputs.base_viscosity_profile(), l_eta=1)
    assert e.value.code == STK_EINVAL
    with pytest.raises(StokesError) as e:   # a base profile needs two positive samples
        sc.set_temperature_viscosity(T, [1.0], l_eta=0)
    assert e.value.code == STK_EINVAL
    sc.close()
    cube = StokesContext("cube", level=1, min_level=0)
    c2, c1 = cube.sizes()
    with pytest.raises(StokesError) as e:   # quadrature-point viscosity needs the blended shell
        cube.set_temperature_viscosity(torch.zeros(c2, dtype=torch.float64, device="cuda"),
                                       inputs.base_viscosity_profile(), l_eta=0)
    assert e.value.code == STK_EINVAL
    cube.close()


def test_binding_refuses_wrong_tensors_before_the_library():
    """Every raw vector argument is checked for device, contiguity, dtype and
    length in Python: a wrong tensor raises ValueError and no entry point
    runs (the outputs stay untouched)."""
    with StokesContext("shell", level=2, min_level=0) as sc:
        n2, n1 = sc.sizes()
        dev = "cuda"
        sc.set_fields(torch.ones(n1, dtype=torch.float64, device=dev))
        gen = sc.generation
        bad = [
            lambda: sc.set_fields(torch.ones(n1, dtype=torch.float32, device=dev)),          # dtype
            lambda: sc.set_log_viscosity(torch.zeros(n1 - 1, dtype=torch.float64, device=dev)),  # length
            lambda: sc.set_fields(torch.ones(n1, dtype=torch.float64)),                        # host tensor
            lambda: sc.rhs_buoyancy(torch.ones(n2 - 5, dtype=torch.float64, device=dev)),
            lambda: sc.solve(torch.zeros(3 * n2, dtype=torch.float32, device=dev)),
            lambda: sc.solve(torch.zeros(3 * n2, dtype=torch.float64, device=dev),
                             g=torch.zeros(n1 + 1, dtype=torch.float64, device=dev)),
            lambda: sc.solve_adjoint(torch.zeros(3 * n2 + 3, dtype=torch.float64, device=dev)),
            lambda: sc.gradient(torch.zeros(3 * n2, dtype=torch.float64, device=dev),
                                torch.zeros(3 * n2, dtype=torch.float32, device=dev)),
            lambda: sc.apply_A(torch.zeros(3 * n2, dtype=torch.float16, device=dev)),
            lambda: sc.apply_A(torch.zeros(3 * n2 + 1, dtype=torch.float64, device=dev)),
            lambda: sc.apply_A(torch.zeros(3 * n2, dtype=torch.float64, device=dev),
                               out=torch.zeros(3 * n2, dtype=torch.float32, device=dev)),           # mixed dtypes
            lambda: sc.apply_B(torch.zeros(3 * n2, dtype=torch.float64, device=dev),
                               out=torch.zeros(n1 - 1, dtype=torch.float64, device=dev)),
            lambda: sc.apply_Bt(torch.zeros(n1, dtype=torch.float64, device=dev)[::2]),       # not contiguous
            lambda: sc.apply_mass(torch.zeros(n1 + 2, dtype=torch.float64, device=dev)),
            lambda: sc.restrict(torch.zeros(3 * n2 - 3, dtype=torch.float64, device=dev), 2),  # fine size expected
            lambda: sc.prolong(torch.zeros(3 * n2, dtype=torch.float64, device=dev), 2),      # coarse size expected
        ]
        y = torch.full((3 * n2,), 7.0, dtype=torch.float64, device=dev)
        for f in bad:
            with pytest.raises(ValueError):
                f()
        with pytest.raises(ValueError):
            sc.apply_A(torch.zeros(3 * n2 - 3, dtype=torch.float64, device=dev), out=y)
        assert (y == 7.0).all() and sc.generation == gen


def test_backward_after_an_interleaved_forward_uses_its_own_fields():
    """Two differentiable solves on one context, both forwards before either
    backward (a sum of two losses): each backward must use the viscosity of
    its own forward.  Both gradients are checked against the oracle's
    assembled gradient of its own field."""
    from oracle.adjoint import grad_log_eta, grad_temperature
    from oracle.fem import rhs_buoyancy
    from paper_2506_04157_amd import StokesSolve
    P = Pair("shell", 1, min_level=0)
    m = P.meshes[1]
    field = inputs.SHField(2)
    T = field.temperature(m.X2)
    params = default_params(tol_rel=1e-11, precision=64)
    A0, B = None, assemble_B(m)
    _, Q = P.projector()
    ms = [np.log(inputs.viscosity_contrast(field.temperature(m.X1), 1e2)), inputs.uniform(30, m.n1, -1.0, 1.0)]
    tens, outs = [], []
    for mv in ms:
        mt = P.p_to_lib(mv).requires_grad_(True)
        Tt = P.s2_to_lib(T).requires_grad_(True)
        u, p = StokesSolve.apply(mt, Tt, P.ctx, params)
        tens.append((mt, Tt))
        outs.append(u)
    (0.5 * (outs[0] ** 2).sum() + 0.5 * (outs[1] ** 2).sum()).backward()
    f = rhs_buoyancy(m, T)
    for (mt, Tt), mv in zip(tens, ms):
        eta = np.exp(mv)
        A = assemble_A(m, eta)
        uo, _, _ = solve_stokes(A, B, f, np.zeros(m.n1), Q, Bt=B.T)
        lam, _, _ = solve_stokes(A, B, uo, np.zeros(m.n1), Q, Bt=B.T)
        assert relerr(P.p_to_or(mt.grad), grad_log_eta(m, eta, uo, lam)) < 1e-6
        assert relerr(P.s2_to_or(Tt.grad), grad_temperature(m, lam)) < 1e-6
