"""Taylor-Hood convergence rates of the oracle (textbook pin, CPU only).

Manufactured smooth solution with variable viscosity: u = curl psi (exactly
divergence free), smooth p, f = -div(2 eta eps_dev(u)) + grad p.  Expected
rates for P2/P1: |u - u_h|_L2 = O(h^3), |grad(u - u_h)| = O(h^2),
|p - p_h|_L2 = O(h^2).
"""
import numpy as np
import sympy as sy

from oracle.fem import assemble_A, assemble_B, error_norms, rhs_function
from oracle.mesh import RefinedMesh, cube_macros, shell_macros
from oracle.quadrature import rule_stroud
from oracle.system import solve_stokes, velocity_basis


def _manufactured(psi_expr, p_expr, eta_expr):
    x, y, z = sy.symbols("x y z")
    X = sy.Matrix([x, y, z])
    psi = psi_expr(x, y, z)
    u = sy.Matrix([sy.diff(psi[2], y) - sy.diff(psi[1], z),
                   sy.diff(psi[0], z) - sy.diff(psi[2], x),
                   sy.diff(psi[1], x) - sy.diff(psi[0], y)])
    p = p_expr(x, y, z)
    eta = eta_expr(x, y, z)
    G = u.jacobian(X)
    eps = (G + G.T) / 2 - sy.eye(3) * G.trace() / 3
    tau = 2 * eta * eps
    f = sy.Matrix([-sum(sy.diff(tau[i, j], X[j]) for j in range(3)) + sy.diff(p, X[i]) for i in range(3)])
    lam = lambda e: sy.lambdify((x, y, z), e, "numpy")
    uf, gf, pf, ff, ef = lam(list(u)), lam(G.tolist()), lam(p), lam(list(f)), lam(eta)

    def vec(fn):
        def w(P):
            o = fn(P[:, 0], P[:, 1], P[:, 2])
            return np.stack([np.broadcast_to(np.asarray(v, dtype=float), P[:, 0].shape) for v in o], 1)
        return w

    def grad(P):
        o = gf(P[:, 0], P[:, 1], P[:, 2])
        return np.stack([np.stack([np.broadcast_to(np.asarray(v, dtype=float), P[:, 0].shape)
                                   for v in row], 1) for row in o], 1)

    scal = lambda fn: (lambda P: np.broadcast_to(np.asarray(fn(P[:, 0], P[:, 1], P[:, 2]), float), P[:, 0].shape))
    return vec(uf), grad, scal(pf), vec(ff), scal(ef)


def _errors(mesh, dir_flags, sol):
    uf, gf, pf, ff, ef = sol
    hi = rule_stroud(4)
    A = assemble_A(mesh, ef(mesh.X1))
    B = assemble_B(mesh)
    f = rhs_function(mesh, ff, hi)
    Q, dm, _ = velocity_basis(mesh, dir_flags, set())
    uD = np.zeros(3 * mesh.n2)
    uD[dm] = uf(mesh.X2).T.ravel()[dm]
    uh, ph, mu = solve_stokes(A, B, f, np.zeros(mesh.n1), Q, uD, Bt=B.T)
    return np.array(error_norms(mesh, uh, ph, uf, gf, pf, hi))


def test_rates_cube_variable_viscosity():
    sol = _manufactured(lambda x, y, z: sy.Matrix([sy.sin(2 * y) * z, sy.cos(x + z), x * y * y]),
                        lambda x, y, z: sy.cos(sy.pi * x) * sy.cos(sy.pi * y) * sy.cos(sy.pi * z),
                        lambda x, y, z: 1 + x * x + sy.exp(y))
    e = [_errors(RefinedMesh(cube_macros(), L), {1}, sol) for L in (1, 2, 3)]
    rates = np.log2(np.array(e[1]) / np.array(e[2]))
    assert rates[0] > 2.8 and rates[1] > 1.85 and rates[2] > 1.85, rates


def test_rates_blended_shell():
    sol = _manufactured(lambda x, y, z: sy.Matrix([sy.sin(2 * y) * sy.cos(z), sy.sin(2 * z) * x, sy.cos(x) * y * y]),
                        lambda x, y, z: sy.sin(x + 2 * y) * z,
                        lambda x, y, z: sy.exp(x * y + z))
    e = [_errors(RefinedMesh(shell_macros(2, 1, 0.55, 1.0), L), {1, 2}, sol) for L in (0, 1)]
    rates = np.log2(np.array(e[0]) / np.array(e[1]))
    assert rates[0] > 2.5 and rates[1] > 1.7 and rates[2] > 1.8, rates
