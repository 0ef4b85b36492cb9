"""Pin of the oracle's assembled adjoint gradient by central differences (CPU only)."""
import numpy as np

from oracle.adjoint import grad_log_eta, grad_temperature
from oracle.fem import assemble_A, assemble_B, rhs_buoyancy
from oracle.mesh import RefinedMesh, shell_macros
from oracle.system import solve_stokes, velocity_basis


def test_adjoint_gradient_matches_central_differences():
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    rng = np.random.default_rng(4)
    mvec = rng.uniform(-1, 1, m.n1)
    T = rng.uniform(0, 1, m.n2)
    lnrho = 0.5 * (1 - np.linalg.norm(m.X1, axis=1))
    Q, dm, fs = velocity_basis(m, {1}, {2})
    B = assemble_B(m)
    Bbar = B + assemble_B(m, lnrho, only_C=True)
    uobs = 0.01 * rng.uniform(-1, 1, 3 * m.n2)

    def J(mv, Tv):
        A = assemble_A(m, np.exp(mv))
        u, p, mu = solve_stokes(A, Bbar, rhs_buoyancy(m, Tv), np.zeros(m.n1), Q, Bt=B.T)
        return 0.5 * np.sum((u - uobs) ** 2), u, A

    j0, u, A = J(mvec, T)
    # K^T = [[A, Bbar^T], [B, 0]]
    lam, lp, _ = solve_stokes(A, B, u - uobs, np.zeros(m.n1), Q, Bt=Bbar.T)
    gm = grad_log_eta(m, np.exp(mvec), u, lam)
    gT = grad_temperature(m, lam)
    h = 1e-6
    for _ in range(3):
        dmv, dT = rng.standard_normal(m.n1), rng.standard_normal(m.n2)
        fd_m = (J(mvec + h * dmv, T)[0] - J(mvec - h * dmv, T)[0]) / (2 * h)
        fd_T = (J(mvec, T + h * dT)[0] - J(mvec, T - h * dT)[0]) / (2 * h)
        assert abs(fd_m - gm @ dmv) <= 1e-5 * abs(fd_m)
        assert abs(fd_T - gT @ dT) <= 1e-6 * abs(fd_T)
