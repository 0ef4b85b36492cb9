"""Pins of the oracle's temperature step (CPU only): the BDF2 weights, the
advection-diffusion system of eq. (WeakTemp), point location and evaluation in
the blended mesh, and the method of characteristics."""
import numpy as np
import pytest

from oracle.fem import assemble_vector_mass, blend_map
from oracle.mesh import RefinedMesh, cube_macros, shell_macros
from oracle.temperature import (bdf2, evaluate_p2, locate, mmoc, solve_dirichlet, symmetric_part, temperature_step,
                                temperature_system)


@pytest.mark.parametrize("tau1,tau0", [(0.1, 0.1), (0.05, 0.2), (0.3, 0.07)])
def test_bdf2_weights_differentiate_quadratics_exactly(tau1, tau0):
    s1, s0, sm = bdf2(tau1, tau0)
    t = np.array([0.0, -tau1, -tau1 - tau0])
    for f, df in [(lambda x: np.ones_like(x), 0.0), (lambda x: x, 1.0), (lambda x: x * x, 0.0),
                  (lambda x: 3 * x * x - 2 * x + 1, -2.0)]:
        v = f(t)
        assert abs((s1 * v[0] - s0 * v[1] + sm * v[2]) / tau1 - df) < 1e-12
    if tau1 == tau0:
        assert np.allclose([s1, s0, sm], [1.5, 2.0, 0.5])


def _lin(X, a=(0.7, -0.4, 1.1), c=0.3):
    return X @ np.array(a) + c


def test_pure_diffusion_keeps_a_linear_temperature():
    """u* = 0, no sources, constant rho on the affine cube: with both history
    values equal to the interpolant of a linear T and T on the boundary, the
    step returns T (its Laplacian vanishes and the BDF2 weights sum to zero)."""
    m = RefinedMesh(cube_macros(), 2)
    T = _lin(m.x2)
    L, b = temperature_system(m, np.zeros(3 * m.n2), np.full(m.n1, 0.2), np.ones(m.n1), T, T, 0.1, 0.15, k=2.0)
    dmask = m.flag2 > 0
    Tn = solve_dirichlet(L, b, dmask, T)
    assert np.abs(Tn - T).max() < 1e-12


def test_advection_mass_and_diffusion_terms():
    """On the affine cube: with k = 0 the matrix is s^{n+1} M + tau Adv, and
    Adv applied to a linear T is (c . grad T) times int phi_i for a constant
    velocity c; the diffusion annihilates constants for a variable rho, and
    for a constant rho it is K / rho (symmetric, energy |grad T|^2 vol / rho
    for a linear T on interior-supported parts)."""
    m = RefinedMesh(cube_macros(), 1)
    n2 = m.n2
    c = np.array([0.3, -1.2, 0.5])
    u = np.repeat(c, n2)
    T = _lin(m.x2)
    s1, _, _ = bdf2(0.1, 0.2)
    L, _ = temperature_system(m, u, np.zeros(m.n1), np.ones(m.n1), T, T, 0.1, 0.2, k=0.0, adv=1.0)
    M = assemble_vector_mass(m, np.ones(m.n1))[:n2, :n2]
    expect = s1 * (M @ T) + 0.1 * (c @ np.array([0.7, -0.4, 1.1])) * (M @ np.ones(n2))
    assert np.abs(L @ T - expect).max() < 1e-13
    # diffusion only (s^{n+1} M removed), variable rho
    lnrho = m.X1 @ np.array([0.5, -0.2, 0.8])
    Lk, _ = temperature_system(m, np.zeros(3 * n2), lnrho, np.ones(m.n1), T, T, 1.0, 1.0, k=3.0)
    D = Lk - 1.5 * M
    assert np.abs(D @ np.ones(n2)).max() < 1e-13
    assert abs(D - D.T).max() > 1e-6            # grad(w / rho) makes it non-symmetric
    Lc, _ = temperature_system(m, np.zeros(3 * n2), np.full(m.n1, np.log(2.0)), np.ones(m.n1), T, T, 1.0, 1.0, k=3.0)
    Dc = Lc - 1.5 * M
    assert abs(Dc - Dc.T).max() < 1e-14
    assert abs(T @ (Dc @ T) - 3.0 / 2.0 * np.sum(np.square([0.7, -0.4, 1.1]))) < 1e-12


def test_shear_heating_and_adiabatic_source():
    """u = (x, 0, 0): eps = diag(1, 0, 0), div u = 1, tau:eps = 2 eta (1 - 1/3);
    the heating term of the right-hand side is tau Pe Di / (Ra rho Cp) 4 eta / 3
    int phi_i for constant eta and rho; a rigid rotation heats nothing."""
    m = RefinedMesh(cube_macros(), 1)
    n2 = m.n2
    u = np.concatenate([m.x2[:, 0], np.zeros(n2), np.zeros(n2)])
    z = np.zeros(n2)
    M = assemble_vector_mass(m, np.ones(m.n1))[:n2, :n2]
    eta, lr = 2.5, 0.4
    _, b = temperature_system(m, u, np.full(m.n1, lr), np.full(m.n1, eta), z, z, 0.2, 0.2, Pe=3.0, Cp=2.0, Di=0.5,
                              Ra=7.0, H=0.9)
    heat = 0.2 * 3.0 * 0.5 / (7.0 * np.exp(lr) * 2.0) * (4.0 * eta / 3.0) + 0.2 * 0.9 / 2.0
    assert np.abs(b - heat * (M @ np.ones(n2))).max() < 1e-13
    rot = np.concatenate([-m.x2[:, 1], m.x2[:, 0], np.zeros(n2)])
    _, b = temperature_system(m, rot, np.zeros(m.n1), np.ones(m.n1), z, z, 0.2, 0.2, Di=1.0)
    assert np.abs(b).max() < 1e-13


def test_locate_inverts_the_blending_map():
    """Reference points inside known elements of the blended shell, mapped by
    the blending map: point location recovers them (same reference point),
    and a P2 function that is quadratic in the reference coordinates is
    evaluated exactly there."""
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    rng = np.random.default_rng(3)
    e = rng.integers(0, m.ne, 200)
    lam = rng.dirichlet(np.ones(4), 200)
    xt = np.einsum("nk,nkd->nd", lam, m.ev[e])
    X = blend_map(xt, m.blend_g[m.emacro[e]], m.blend_s0[m.emacro[e]])
    e2, lam2 = locate(m, X)
    xt2 = np.einsum("nk,nkd->nd", lam2, m.ev[e2])
    assert np.abs(xt2 - xt).max() < 1e-12
    q = lambda x: 1.0 + x[:, 0] * x[:, 1] - 2.0 * x[:, 2] ** 2 + 0.5 * x[:, 0]
    assert np.abs(evaluate_p2(m, q(m.x2), X)[0] - q(xt)).max() < 1e-12


def test_mmoc_is_exact_for_a_constant_velocity_and_the_identity_for_none():
    """On the affine cube, a constant velocity is represented exactly and the
    Runge-Kutta step is exact for it: the departure point of node x is
    x - tau c, where the P2 interpolant of a quadratic equals the quadratic.
    Without velocity every node is its own departure point."""
    m = RefinedMesh(cube_macros(), 2)
    n2 = m.n2
    q = lambda x: 1.0 + x[:, 0] * x[:, 1] - 2.0 * x[:, 2] ** 2 + 0.5 * x[:, 0]
    F = q(m.x2)
    assert np.abs(mmoc(m, F, np.zeros(3 * n2), np.zeros(3 * n2), 0.3) - F).max() < 1e-13
    c = np.array([0.2, -0.1, 0.15])
    u = np.repeat(c, n2)
    tau = 0.5
    got = mmoc(m, F, u, u, tau)
    dep = m.x2 - tau * c
    inside = np.all((dep >= 0) & (dep <= 1), axis=1)
    assert inside.sum() > n2 // 3
    assert np.abs(got[inside] - q(dep[inside])).max() < 1e-12


def test_mmoc_follows_a_rigid_rotation_on_the_shell():
    """A rigid rotation about z on the blended shell, over a small step: the
    departure points are the nodes rotated back, up to the interpolation
    and Runge-Kutta errors."""
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 2)
    n2 = m.n2
    w = 0.8
    u = np.concatenate([-w * m.X2[:, 1], w * m.X2[:, 0], np.zeros(n2)])
    f = lambda X: X[:, 0] + 0.5 * X[:, 1] ** 2 - X[:, 2]
    tau = 0.05
    got = mmoc(m, f(m.X2), u, u, tau)
    a = -w * tau
    R = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    ref = f(m.X2 @ R.T)
    assert np.abs(got - ref).max() < 5e-3
    assert np.abs(got - f(m.X2)).max() > 1e-2       # it did move


def test_adiabatic_term_against_a_closed_form_integral():
    """g = -X/|X| on the unit cube, u* = c constant, no diffusion: 1^T L 1 =
    s^{n+1} + tau Di alpha / Cp c . int X/|X| dx, where each component of the
    integral is int int sqrt(1 + y^2 + z^2) - sqrt(y^2 + z^2) dy dz (the x
    integral done by hand).  |X| is not polynomial: the bar is the
    quadrature error of the 27-point rule at level 2."""
    from scipy.integrate import dblquad
    I = dblquad(lambda y, z: np.sqrt(1 + y * y + z * z) - np.sqrt(y * y + z * z), 0, 1, 0, 1, epsabs=1e-13)[0]
    m = RefinedMesh(cube_macros(), 2)
    n2 = m.n2
    c = np.array([0.4, -0.9, 0.25])
    s1, _, _ = bdf2(0.1, 0.3)
    L, _ = temperature_system(m, np.repeat(c, n2), np.zeros(m.n1), np.ones(m.n1), np.zeros(n2), np.zeros(n2), 0.1,
                              0.3, k=0.0, Di=1.5, alpha=2.0, Cp=0.5)
    one = np.ones(n2)
    expect = s1 + 0.1 * 1.5 * 2.0 / 0.5 * c.sum() * I
    assert abs(one @ (L @ one) - expect) < 1e-4 * abs(expect - s1)


def test_symmetric_part_is_the_symmetric_mass_and_diffusion():
    """Without velocity and with constant rho the system matrix is exactly
    the preconditioner's (symmetric, positive definite on the free nodes);
    with a variable rho the two differ by the non-symmetric term only."""
    m = RefinedMesh(cube_macros(), 1)
    z = np.zeros(m.n2)
    S = symmetric_part(m, np.full(m.n1, 0.3), 0.1, 0.2, k=2.0)
    L, _ = temperature_system(m, np.zeros(3 * m.n2), np.full(m.n1, 0.3), np.ones(m.n1), z, z, 0.1, 0.2, k=2.0)
    assert abs(S - L).max() < 1e-15
    free = m.flag2 == 0
    assert np.linalg.eigvalsh(S[free][:, free].toarray()).min() > 0
    lr = m.X1 @ np.array([0.5, -0.2, 0.8])
    S = symmetric_part(m, lr, 0.1, 0.2, k=2.0)
    L, _ = temperature_system(m, np.zeros(3 * m.n2), lr, np.ones(m.n1), z, z, 0.1, 0.2, k=2.0)
    assert abs(S - S.T).max() < 1e-15 and abs(L - L.T).max() > 1e-6
    one = np.ones(m.n2)
    assert np.abs((L - S) @ one).max() < 1e-15


def test_splitting_step_transports_a_rotating_field():
    """Pure transport (k = 0, no sources) by a steady rigid rotation about z on
    the blended shell: the exact solution is T(t, X) = f(R(-w t) X), every
    traced history value equals T^{n+1} at the nodes, and the step returns
    the interpolant of T^{n+1} up to the tracing and interpolation errors.
    Counting the advection a second time in the linear system (adv = 1)
    moves the result by a step's worth of advection."""
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 2)
    n2 = m.n2
    w, tau = 0.8, 0.04
    u = np.concatenate([-w * m.X2[:, 1], w * m.X2[:, 0], np.zeros(n2)])
    f = lambda X: X[:, 0] + 0.5 * X[:, 1] ** 2 - X[:, 2]

    def T(t):
        a = -w * t
        R = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
        return f(m.X2 @ R.T)
    dmask = m.flag2 > 0
    kw = dict(k=0.0)
    # the Dirichlet values are the exact ones: pass them through the history
    out = {}
    for adv in (0.0, 1.0):
        ustar = u.copy()
        That_n = mmoc(m, T(1.0), ustar, u, tau)
        That_nm1 = mmoc(m, mmoc(m, T(1.0 - tau), u, u, tau), ustar, u, tau)
        L, b = temperature_system(m, ustar, np.zeros(m.n1), np.ones(m.n1), That_n, That_nm1, tau, tau, adv=adv, **kw)
        out[adv] = solve_dirichlet(L, b, dmask, T(1.0 + tau))
    ex = T(1.0 + tau)
    e0 = np.abs(out[0.0] - ex).max()
    e1 = np.abs(out[1.0] - ex).max()
    assert e0 < 5e-3
    assert e1 > 5 * e0
    # the composed tracing of the step routine is the one used here
    Tn1, Thn, Thnm1, us = temperature_step(m, T(1.0), T(1.0 - tau), u, u, np.zeros(m.n1), np.ones(m.n1), tau, tau,
                                           T_in=0.0, T_out=0.0, k=0.0)
    assert np.abs(us - u).max() == 0.0
    assert np.abs(Thnm1 - mmoc(m, mmoc(m, T(1.0 - tau), u, u, tau), u, u, tau)).max() == 0.0
