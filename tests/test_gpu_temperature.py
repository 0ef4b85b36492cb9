"""GPU parity of the temperature step (Sec. 3 splitting, Sec. 6 eq. WeakTemp)
against the oracle: the operators L and S (and diag S), the right-hand side
with history, adiabatic, internal and shear heating terms, the method of
characteristics (analytic point location in the blended shell and on the
cube), the FGMRES + CG solve with Dirichlet values on both spheres, and the
whole step.  Errors are per entry against the entry's own scale.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle.fem import assemble_vector_mass
from oracle.temperature import bdf2, mmoc, solve_dirichlet, symmetric_part, temperature_step, temperature_system
from paper_2506_04157_amd import StokesError, temp_params
from tests._util import Pair, relerr, rowerr

pytestmark = pytest.mark.gpu

COEF = dict(k=0.8, Pe=3.0, Cp=1.1, Di=0.4, alpha=1.3, H=0.7, Ra=30.0)
TAU1, TAU0 = 0.02, 0.026


def _u(seed, X):
    return inputs.smooth_vector_field(seed, X).T.ravel().copy()


@pytest.fixture(scope="module")
def shell():
    print("\n[temperature shell L2]", flush=True)
    P = Pair("shell", 2, min_level=0, n_tan=1, n_rad=1)
    m = P.meshes[2]
    field = inputs.SHField(4)
    T2 = field.temperature(m.X2)
    lnrho = inputs.ln_density(m.X1)
    eta = inputs.viscosity_contrast(field.temperature(m.X1), 1e2)
    return dict(P=P, m=m, T2=T2, lnrho=lnrho, eta=eta, u=_u(31, m.X2), u_old=_u(32, m.X2))


def _params(adv=0.0, **kw):
    kw = {**COEF, **kw}
    return temp_params(tau1=TAU1, tau0=TAU0, adv=adv, **kw)


@pytest.mark.parametrize("adv", [0.0, 1.0])
def test_temperature_operators_match_oracle(shell, adv):
    d = shell
    P, m = d["P"], d["m"]
    prm = _params(adv)
    x = inputs.uniform(41, m.n2)
    z = np.zeros(m.n2)
    Lo, _ = temperature_system(m, d["u"], d["lnrho"], d["eta"], z, z, TAU1, TAU0, adv=adv, **COEF)
    So = symmetric_part(m, d["lnrho"], TAU1, TAU0, k=COEF["k"], Pe=COEF["Pe"], Cp=COEF["Cp"])
    ul, lr = P.u_to_lib(d["u"]), P.p_to_lib(d["lnrho"])
    y = P.s2_to_or(P.ctx.temp_apply(P.s2_to_lib(x), prm, 0, u_star=ul, lnrho=lr))
    ys = P.s2_to_or(P.ctx.temp_apply(P.s2_to_lib(x), prm, 1, lnrho=lr))
    yd = P.s2_to_or(P.ctx.temp_apply(P.s2_to_lib(x), prm, 2, lnrho=lr))
    yst = P.s2_to_or(P.ctx.temp_apply(P.s2_to_lib(x), prm, 3, lnrho=lr))   # stored element matrices
    eL = rowerr(y, Lo @ x, abs(Lo) @ np.abs(x))
    eS = rowerr(ys, So @ x, abs(So) @ np.abs(x))
    eD = rowerr(yd, So.diagonal(), np.abs(So.diagonal()))
    eSt = rowerr(yst, So @ x, abs(So) @ np.abs(x))
    print(f"adv {adv}: L {eL:.2e}  S {eS:.2e}  diag {eD:.2e}  stored S {eSt:.2e}")
    assert eL < 1e-12 and eS < 1e-12 and eD < 1e-13 and eSt < 1e-12


def test_temperature_rhs_matches_oracle(shell):
    d = shell
    P, m = d["P"], d["m"]
    prm = _params()
    Tn = d["T2"]
    Tm = d["T2"] + 0.05 * inputs.uniform(42, m.n2)
    _, bo = temperature_system(m, d["u"], d["lnrho"], d["eta"], Tn, Tm, TAU1, TAU0, **COEF)
    b = P.s2_to_or(P.ctx.temp_rhs(P.s2_to_lib(Tn), P.s2_to_lib(Tm), prm, u_star=P.u_to_lib(d["u"]),
                                  lnrho=P.p_to_lib(d["lnrho"]), eta=P.p_to_lib(d["eta"])))
    s1, s0, sm = bdf2(TAU1, TAU0)
    M = assemble_vector_mass(m, np.ones(m.n1))[:m.n2, :m.n2]
    z = np.zeros(m.n2)
    _, src = temperature_system(m, d["u"], d["lnrho"], d["eta"], z, z, TAU1, TAU0, **COEF)
    # per-entry scale: |M| applied to the history magnitudes plus the source
    # level (the P2 mass has negative entries, so M itself is no scale)
    Ma = abs(M)
    src_level = np.max(np.abs(src) / (Ma @ np.ones(m.n2)))
    scale = Ma @ (s0 * np.abs(Tn) + sm * np.abs(Tm) + src_level)
    e = rowerr(b, bo, scale)
    print(f"rhs {e:.2e}  (heating share {np.abs(src).max() / np.abs(bo).max():.2e})")
    assert e < 1e-12
    # without a velocity only the history and internal heating remain
    b0 = P.s2_to_or(P.ctx.temp_rhs(P.s2_to_lib(Tn), P.s2_to_lib(Tm), prm, lnrho=P.p_to_lib(d["lnrho"])))
    ref = M @ (s0 * Tn - sm * Tm) + TAU1 * COEF["H"] / COEF["Cp"] * (M @ np.ones(m.n2))
    assert rowerr(b0, ref, scale) < 1e-12


@pytest.mark.parametrize("tau", [0.0, 0.03, 0.12])
def test_mmoc_matches_oracle_on_the_shell(shell, tau):
    """Departure points up to several micro-tets away, through macro and
    icosahedral-face boundaries; with tau = 0.12 many boundary nodes trace
    out of the shell and are moved back radially."""
    d = shell
    P, m = d["P"], d["m"]
    F = d["T2"]
    got = P.s2_to_or(P.ctx.mmoc(P.s2_to_lib(F), P.u_to_lib(d["u"]), P.u_to_lib(d["u_old"]), tau))
    ref = mmoc(m, F, d["u"], d["u_old"], tau)
    e = np.abs(got - ref).max() / np.abs(F).max()
    print(f"tau {tau}: max |gpu - oracle| / max|F| = {e:.2e}, moved {np.abs(ref - F).max():.2e}")
    assert e < 1e-11
    if tau == 0.0:
        assert np.abs(got - F).max() < 1e-13


def test_mmoc_on_the_cube_matches_oracle_and_is_exact_for_constant_velocity():
    print("\n[temperature cube L2]", flush=True)
    P = Pair("cube", 2, min_level=0)
    m = P.meshes[2]
    q = lambda x: 1.0 + x[:, 0] * x[:, 1] - 2.0 * x[:, 2] ** 2 + 0.5 * x[:, 0]
    F = q(m.x2)
    c = np.array([0.2, -0.1, 0.15])
    u = np.repeat(c, m.n2)
    got = P.s2_to_or(P.ctx.mmoc(P.s2_to_lib(F), P.u_to_lib(u), P.u_to_lib(u), 0.5))
    dep = m.x2 - 0.5 * c
    inside = np.all((dep >= 0) & (dep <= 1), axis=1)
    assert np.abs(got[inside] - q(dep[inside])).max() < 1e-12
    v = _u(33, m.X2)
    got = P.s2_to_or(P.ctx.mmoc(P.s2_to_lib(F), P.u_to_lib(v), P.u_to_lib(0.5 * v), 0.2))
    assert np.abs(got - mmoc(m, F, v, 0.5 * v, 0.2)).max() < 1e-11
    P.ctx.close()


@pytest.mark.parametrize("adv,stored", [(0.0, 1), (1.0, 1), (1.0, 0)])
def test_temperature_solve_matches_oracle(shell, adv, stored):
    d = shell
    P, m = d["P"], d["m"]
    prm = _params(adv, T_in=1.0, T_out=0.1, tol_abs=1e-15, stored_S=stored)
    Tn = d["T2"]
    Lo, bo = temperature_system(m, d["u"], d["lnrho"], d["eta"], Tn, Tn, TAU1, TAU0, adv=adv, **COEF)
    To = solve_dirichlet(Lo, bo, m.flag2 > 0, np.where(m.flag2 == 2, 0.1, 1.0))
    T, rep = P.ctx.temp_solve(P.s2_to_lib(bo), prm, u_star=P.u_to_lib(d["u"]), lnrho=P.p_to_lib(d["lnrho"]),
                              T_init=P.s2_to_lib(Tn))
    T = P.s2_to_or(T)
    e = np.abs(T - To).max() / np.abs(To).max()
    print(f"adv {adv}: {rep['iterations']} FGMRES its, {rep['cg_its']} CG its, residual {rep['abs_residual']:.2e}, "
          f"max rel diff {e:.2e}")
    assert rep["converged"] == 1 and e < 1e-9 and rep["stored_S"] == stored
    assert np.array_equal(T[m.flag2 == 1], np.ones((m.flag2 == 1).sum()))
    assert np.array_equal(T[m.flag2 == 2], np.full((m.flag2 == 2).sum(), 0.1))


def test_temperature_step_matches_oracle(shell):
    d = shell
    P, m = d["P"], d["m"]
    prm = _params(0.0, T_in=1.0, T_out=0.0, tol_abs=1e-15)
    Tn = d["T2"]
    Tm = d["T2"] + 0.05 * inputs.uniform(43, m.n2)
    To, tho, tmo, _ = temperature_step(m, Tn, Tm, d["u"], d["u_old"], d["lnrho"], d["eta"], TAU1, TAU0, T_in=1.0,
                                       T_out=0.0, **COEF)
    T, thn, thm, rep = P.ctx.temperature_step(
        P.s2_to_lib(Tn), P.s2_to_lib(Tm), P.u_to_lib(d["u"]), P.u_to_lib(d["u_old"]), P.p_to_lib(d["eta"]), prm,
        lnrho=P.p_to_lib(d["lnrho"]), traced=True)
    e_n = np.abs(P.s2_to_or(thn) - tho).max()
    e_m = np.abs(P.s2_to_or(thm) - tmo).max()
    e_T = np.abs(P.s2_to_or(T) - To).max() / np.abs(To).max()
    print(f"traced {e_n:.2e} {e_m:.2e}, T {e_T:.2e}, {rep['iterations']} its, mmoc {rep['ms_mmoc']:.1f} ms, "
          f"solve {rep['ms_solve']:.1f} ms")
    assert e_n < 1e-11 and e_m < 1e-11 and e_T < 1e-9


def test_temperature_errors_and_no_convergence(shell):
    d = shell
    P, m = d["P"], d["m"]
    F = P.s2_to_lib(d["T2"])
    u = P.u_to_lib(d["u"])
    assert P.ctx.lib.stk_mmoc(P.ctx.h, None, None, None, 0.1, None) == -1   # STK_EINVAL before any launch
    with pytest.raises(StokesError):
        P.ctx.mmoc(F, u, u, 0.1, out=F)                       # aliasing refused
    with pytest.raises(StokesError):
        P.ctx.mmoc(F, u, u, -0.1)
    with pytest.raises(StokesError):
        P.ctx.temp_apply(F, temp_params(tau1=0.0), 0)
    prm = _params(1.0, tol_abs=1e-30, max_outer=2, restart=2)
    b = P.s2_to_lib(d["T2"])
    T, rep = P.ctx.temp_solve(b, prm, u_star=u, allow_noconv=True)
    assert rep["converged"] == 0 and rep["iterations"] == 2
    assert torch.isfinite(T).all()


def test_two_coupled_steps_match_oracle(shell):
    """Two steps of the Gauss-Seidel-like alternation (Sec. 3): the Stokes
    solve with the buoyancy of T^n (no-slip inner, free-slip outer,
    compressible; buoyancy scaled by 500 so that the velocity is of order
    one), then the temperature step from T^n, T^{n-1}, u^n, u^{n-1} with a
    step of about a third of a micro-tet's height over max |u|; the library
    (FGMRES to 1e-11, the step's FGMRES to an absolute 1e-14) against the
    oracle's direct solves, starting from T^{-1} = T^0, u^{-1} = u^0.  Bars:
    the velocity within the solve's condition x residual (1e-6), T^{n+1}
    within 1e-7."""
    from oracle.fem import assemble_A, assemble_B, rhs_buoyancy
    from oracle.system import solve_stokes
    from paper_2506_04157_amd import default_params
    d = shell
    P, m = d["P"], d["m"]
    eta, lnrho = d["eta"], d["lnrho"]
    A = assemble_A(m, eta)
    B = assemble_B(m)
    Bb = B + assemble_B(m, lnrho, only_C=True)
    _, Q = P.projector()
    sp_ = default_params(tol_rel=1e-11, precision=64)
    P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho), params=sp_)
    T_o = [d["T2"].copy(), d["T2"].copy()]          # T^{n-1}, T^n
    T_g = [P.s2_to_lib(d["T2"]), P.s2_to_lib(d["T2"])]
    u_o, u_g = [], []
    tau = None
    for step in range(2):
        f = rhs_buoyancy(m, T_o[-1], scale=500.0)
        uo, _, _ = solve_stokes(A, Bb, f, np.zeros(m.n1), Q, Bt=B.T)
        ug, _, rep = P.ctx.solve(P.ctx.rhs_buoyancy(T_g[-1], scale=500.0), params=sp_)
        assert rep["rel_residual"] <= 1e-11
        e_u = relerr(P.u_to_or(ug), uo)
        u_o.append(uo)
        u_g.append(ug)
        if tau is None:
            tau = 0.3 * 0.45 / 8 / np.abs(uo).max()     # a third of a micro-tet height per step
        prm = temp_params(tau1=tau, tau0=tau, adv=0.0, T_in=1.0, T_out=0.0, tol_abs=1e-14, **COEF)
        un_o, unm1_o = u_o[-1], u_o[-2] if step > 0 else u_o[-1]
        un_g, unm1_g = u_g[-1], u_g[-2] if step > 0 else u_g[-1]
        Tn1_o, _, _, _ = temperature_step(m, T_o[-1], T_o[-2], un_o, unm1_o, lnrho, eta, tau, tau, T_in=1.0,
                                          T_out=0.0, **COEF)
        Tn1_g, rep_t = P.ctx.temperature_step(T_g[-1], T_g[-2], un_g, unm1_g, P.p_to_lib(eta), prm,
                                              lnrho=P.p_to_lib(lnrho))
        e_T = np.abs(P.s2_to_or(Tn1_g) - Tn1_o).max() / np.abs(Tn1_o).max()
        moved = np.abs(Tn1_o - T_o[-1]).max()
        print(f"step {step}: u {e_u:.2e} (max|u| {np.abs(uo).max():.2e}, tau {tau:.2e}), T {e_T:.2e}, "
              f"T changed by {moved:.2e}, {rep_t['iterations']} its")
        assert e_u < 1e-6 and e_T < 1e-7 and moved > 1e-4
        T_o.append(Tn1_o)
        T_g.append(Tn1_g)


def test_coupled_step_entry_point_matches_oracle(shell):
    """stk_coupled_step twice (the temperature step with the viscosity of the
    model at the extrapolated temperature, then the Stokes solve with the
    viscosity and buoyancy of the new temperature) against the same sequence
    in the oracle: the model's eta(x_V, T(x_V)) at the vertices, the oracle's
    temperature step and its direct Stokes solve."""
    from oracle.fem import assemble_A, assemble_B, rhs_buoyancy, vertex_p2_nodes, viscosity_model
    from oracle.system import solve_stokes
    from paper_2506_04157_amd import default_params
    d = shell
    P, m = d["P"], d["m"]
    lnrho = d["lnrho"]
    base = inputs.base_viscosity_profile()
    E_A, V_A, scale = 4.610, 2.996, 500.0
    v2 = vertex_p2_nodes(m)
    model = lambda T2: viscosity_model(m.X1, T2[v2], base, E_A, V_A, 0.55, 1.0)
    B = assemble_B(m)
    Bb = B + assemble_B(m, lnrho, only_C=True)
    _, Q = P.projector()
    sp_ = default_params(tol_rel=1e-11, precision=64, max_outer=400)
    # start: T^{-1} = T^0 and the velocity of T^0
    T0 = d["T2"]
    u0, _, _ = solve_stokes(assemble_A(m, model(T0)), Bb, rhs_buoyancy(m, T0, scale=scale), np.zeros(m.n1), Q,
                            Bt=B.T)
    tau = 0.3 * 0.45 / 8 / np.abs(u0).max()
    tp = temp_params(tau1=tau, tau0=tau, T_in=1.0, T_out=0.0, tol_abs=1e-14, **COEF)
    To = [T0, T0]
    uo = [u0, u0]
    Tg = [P.s2_to_lib(T0), P.s2_to_lib(T0)]
    ug = [P.u_to_lib(u0), P.u_to_lib(u0)]
    for step in range(2):
        Ts = 2.0 * To[-1] - To[-2]
        Tn1, _, _, _ = temperature_step(m, To[-1], To[-2], uo[-1], uo[-2], lnrho, model(Ts), tau, tau, T_in=1.0,
                                        T_out=0.0, **COEF)
        un1, pn1, _ = solve_stokes(assemble_A(m, model(Tn1)), Bb, rhs_buoyancy(m, Tn1, scale=scale),
                                   np.zeros(m.n1), Q, Bt=B.T)
        T, u, p, trep, srep = P.ctx.coupled_step(Tg[-1], Tg[-2], ug[-1], ug[-2], base, tp, params=sp_, E_A=E_A,
                                                 V_A=V_A, buoyancy_scale=scale, lnrho=P.p_to_lib(lnrho))
        e_T = np.abs(P.s2_to_or(T) - Tn1).max() / np.abs(Tn1).max()
        e_u = relerr(P.u_to_or(u), un1)
        print(f"coupled step {step}: T {e_T:.2e}, u {e_u:.2e}, {trep['iterations']} temperature its, "
              f"{srep['iterations']} Stokes its, rel {srep['rel_residual']:.1e}")
        assert e_T < 1e-7 and e_u < 1e-6 and srep["rel_residual"] <= 1e-11
        To.append(Tn1)
        uo.append(un1)
        Tg.append(T)
        ug.append(u)
