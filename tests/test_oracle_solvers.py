"""Pins of the oracle's solver components (CPU only)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.fem import assemble_A, assemble_B
from oracle.mesh import RefinedMesh, cube_macros, shell_macros
from oracle.solvers import (adjoint_uzawa, inexact_uzawa, bfbt, wbfbt, chebyshev, chebyshev_error_polynomial, fgmres, pcg,
                            prolongation, symmetric_uzawa, vcycle, vector_prolongation)
from oracle.system import rigid_rotations, solve_stokes, velocity_basis


def test_chebyshev_matches_closed_form_error_polynomial():
    rng = np.random.default_rng(0)
    lam = rng.uniform(0.05, 2.0, 50)
    A = sp.diags(lam)
    P = sp.identity(50)
    e0 = rng.standard_normal(50)
    lo, hi = 0.2, 2.1
    for deg in (1, 2, 3, 5):
        # solving A x = 0 from x = e0: the error is p_deg(A) e0
        x = chebyshev(A, np.ones(50), P, np.zeros(50), e0, lo, hi, deg, 1)
        assert np.allclose(x, chebyshev_error_polynomial(lam, lo, hi, deg) * e0, atol=1e-13)
    x = chebyshev(A, np.ones(50), P, np.zeros(50), e0, lo, hi, 2, 3)
    assert np.allclose(x, chebyshev_error_polynomial(lam, lo, hi, 2) ** 3 * e0, atol=1e-13)


def test_prolongation_reproduces_quadratics_and_restriction_is_adjoint():
    mac = shell_macros(1, 1, 0.55, 1.0)
    c, f = RefinedMesh(mac, 0), RefinedMesh(mac, 1)
    P = prolongation(c, f)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-14)
    # a quadratic in reference coordinates is in both P2 spaces
    q = lambda x: 1 + x[:, 0] - 2 * x[:, 1] * x[:, 2] + 0.5 * x[:, 0] ** 2
    assert np.allclose(P @ q(c.x2), q(f.x2), atol=1e-13)
    # weights take the values of the P2 basis at the fine nodes
    vals = np.unique(np.round(P.data * 8))
    assert set(vals.tolist()) <= {-1.0, 2.0, 3.0, 4.0, 6.0, 8.0}
    rng = np.random.default_rng(1)
    r, e = rng.standard_normal(f.n2), rng.standard_normal(c.n2)
    assert np.isclose((P.T @ r) @ e, r @ (P @ e), rtol=1e-13)


def _levels(mac, lmax, eta_fn):
    levels = []
    meshes = [RefinedMesh(mac, l) for l in range(lmax + 1)]
    for l, m in enumerate(meshes):
        A = assemble_A(m, eta_fn(m.X1))
        Q, dm, _ = velocity_basis(m, {1}, set())
        Pm = Q @ Q.T
        Dinv = 1.0 / A.diagonal()
        d = dict(A=A, P=Pm, Dinv=Dinv, Q=Q)
        x = np.random.default_rng(5).standard_normal(A.shape[0])
        for _ in range(60):
            x = Pm @ (Dinv * (A @ (Pm @ x)))
            lmax_est = np.linalg.norm(x)
            x /= lmax_est
        d["lo"], d["hi"] = 0.12 * lmax_est, 1.2 * lmax_est
        if l > 0:
            d["Pro"] = vector_prolongation(prolongation(meshes[l - 1], m))
        levels.append(d)
    return levels, meshes


def test_p1_prolongation_reproduces_linear_functions():
    """The nested P1 embedding: a linear function of the reference
    coordinates is interpolated exactly, rows sum to one, and on the shell
    every fine P1 node is a coarse vertex (weight 1) or an edge midpoint
    (weights 1/2, 1/2)."""
    from oracle.solvers import prolongation_p1
    for mac in (cube_macros(), shell_macros(1, 1, 0.55, 1.0)):
        c, f = RefinedMesh(mac, 1), RefinedMesh(mac, 2)
        P = prolongation_p1(c, f)
        g = np.array([0.7, -1.3, 0.4])
        assert np.abs(P @ (c.x1 @ g + 0.2) - (f.x1 @ g + 0.2)).max() < 1e-13
        assert np.abs(np.asarray(P.sum(axis=1)).ravel() - 1.0).max() < 1e-14
        nnz = np.diff(P.indptr)
        assert set(np.unique(nnz)) == {1, 2}
        assert np.allclose(P.data[np.repeat(nnz, nnz) == 2], 0.5)


def test_vcycle_contracts_level_independently():
    eta = lambda X: 1.0 + 9.0 * (X[:, 0] > 0.5)
    factors = []
    for lmax in (2, 3):
        levels, meshes = _levels(cube_macros(), lmax, eta)
        Q0 = levels[0]["Q"]
        A0 = (Q0.T @ levels[0]["A"] @ Q0).tocsc()
        lu = spla.splu(A0)
        cs = lambda b: Q0 @ lu.solve(Q0.T @ b)
        L = levels[lmax]
        Pm = L["P"]
        x = Pm @ np.random.default_rng(3).standard_normal(L["A"].shape[0])
        # error propagation of the V-cycle as a stationary iteration on A e = 0
        for _ in range(6):
            xn = x - vcycle(levels, lmax, Pm @ (L["A"] @ x), cs, 2, 3)
            rho = np.linalg.norm(xn) / np.linalg.norm(x)
            x = xn
        factors.append(rho)
    assert max(factors) < 0.35, factors
    assert abs(factors[0] - factors[1]) < 0.15, factors


def test_bfbt_identity_for_square_B():
    rng = np.random.default_rng(2)
    n = 6
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    B = rng.standard_normal((n, n))
    Ch = rng.standard_normal((n, n))
    Ch = Ch @ Ch.T + n * np.eye(n)                 # any SPD "A-hat"
    Ainv = lambda v: np.linalg.solve(Ch, v)
    BAB = B @ np.linalg.solve(Ch, B.T)
    r = rng.standard_normal(n)
    s = bfbt(r, B, B.T, A, Ainv, lambda v: np.linalg.solve(BAB, v))
    exact = np.linalg.solve(B @ np.linalg.solve(A, B.T), r)
    assert np.allclose(s, exact, rtol=1e-10)


def test_wbfbt_identity_for_square_B_and_exact_poisson_operators():
    """With a square invertible B and the Poisson operators taken exactly as
    K_l = B M_l^-1 B^T, K_r = B M_r^-1 B^T, the weighted BFBT is the exact
    inverse Schur complement for any SPD masses M_l, M_r (different left and
    right weights, as with a_l != a_r); swapping l and r, or dropping one
    mass, breaks it."""
    rng = np.random.default_rng(3)
    n = 6
    X = rng.standard_normal((n, n))
    A = X @ X.T + n * np.eye(n)
    B = rng.standard_normal((n, n))
    Ms = []
    for _ in range(2):
        Y = rng.standard_normal((n, n))
        Ms.append(Y @ Y.T + n * np.eye(n))
    Ml, Mr = Ms
    Kl, Kr = B @ np.linalg.solve(Ml, B.T), B @ np.linalg.solve(Mr, B.T)
    r = rng.standard_normal(n)
    sol = lambda Mat: (lambda v: np.linalg.solve(Mat, v))
    s = wbfbt(r, B, B.T, A, sol(Ml), sol(Mr), sol(Kl), sol(Kr))
    exact = np.linalg.solve(B @ np.linalg.solve(A, B.T), r)
    assert np.allclose(s, exact, rtol=1e-10)
    wrong = wbfbt(r, B, B.T, A, sol(Mr), sol(Ml), sol(Kl), sol(Kr))
    assert not np.allclose(wrong, exact, rtol=1e-3)


def test_fgmres_with_exact_symmetric_uzawa_converges_in_one_step():
    rng = np.random.default_rng(4)
    n, m = 12, 5
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    B = rng.standard_normal((m, n))
    Cc = 0.1 * rng.standard_normal((m, n))
    Bbar = B + Cc
    K = np.block([[A, B.T], [Bbar, np.zeros((m, m))]])
    S = Bbar @ np.linalg.solve(A, B.T)
    b = rng.standard_normal(n + m)

    def prec(v):
        u, p = symmetric_uzawa(v[:n], v[n:], A, B.T, Bbar, lambda r: np.linalg.solve(A, r),
                               lambda r: np.linalg.solve(S, r), 1.0, 1.0)
        return np.concatenate([u, p])

    x, it, hist = fgmres(lambda v: K @ v, b, prec, 1e-12, restart=10)
    assert it <= 2
    assert np.allclose(K @ x, b, atol=1e-10)
    # with an inexact preconditioner FGMRES still converges to the solution
    x, it, hist = fgmres(lambda v: K @ v, b, lambda v: v / 10.0, 1e-11, restart=40)
    assert np.linalg.norm(K @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_inexact_and_adjoint_uzawa_are_the_block_triangular_solves():
    """With exact inner solves and S = Bbar A^-1 B^T, one inexact Uzawa step
    from zero solves the lower block-triangular system [[A, 0], [Bbar, -S/omega]]
    (scaled by sigma) and the adjoint step the upper one [[A, B^T], [0, -S/omega]];
    FGMRES preconditioned by either converges in two iterations."""
    rng = np.random.default_rng(7)
    n, m = 14, 6
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    B = rng.standard_normal((m, n))
    Bbar = B + 0.1 * rng.standard_normal((m, n))
    S = Bbar @ np.linalg.solve(A, B.T)
    K = np.block([[A, B.T], [Bbar, np.zeros((m, m))]])
    Ainv = lambda r: np.linalg.solve(A, r)
    Sinv = lambda r: np.linalg.solve(S, r)
    ru, rp = rng.standard_normal(n), rng.standard_normal(m)
    sigma, omega = 0.8, 0.3
    u, p = inexact_uzawa(ru, rp, Bbar, Ainv, Sinv, sigma, omega)
    lower = np.block([[A / sigma, np.zeros((n, m))], [Bbar, -S / omega]])
    ref = np.linalg.solve(lower, np.concatenate([ru, rp]))
    assert np.allclose(np.concatenate([u, p]), ref, rtol=1e-11, atol=1e-12)
    u, p = adjoint_uzawa(ru, rp, B.T, Ainv, Sinv, sigma, omega)
    upper = np.block([[A / sigma, B.T], [np.zeros((m, n)), -S / omega]])
    ref = np.linalg.solve(upper, np.concatenate([ru, rp]))
    assert np.allclose(np.concatenate([u, p]), ref, rtol=1e-11, atol=1e-12)
    b = rng.standard_normal(n + m)
    for step in (lambda v: inexact_uzawa(v[:n], v[n:], Bbar, Ainv, Sinv, 1.0, 1.0),
                 lambda v: adjoint_uzawa(v[:n], v[n:], B.T, Ainv, Sinv, 1.0, 1.0)):
        x, it, hist = fgmres(lambda v: K @ v, b, lambda v: np.concatenate(step(v)), 1e-12, restart=10)
        assert it <= 2
        assert np.allclose(K @ x, b, atol=1e-10)


def test_pcg_and_direct_solve_agree():
    m = RefinedMesh(cube_macros(), 2)
    A = assemble_A(m, np.ones(m.n1))
    Q, dm, _ = velocity_basis(m, {1}, set())
    QAQ = (Q.T @ A @ Q).tocsr()
    b = np.random.default_rng(0).standard_normal(QAQ.shape[0])
    x, it = pcg(lambda v: QAQ @ v, b, lambda r: r / QAQ.diagonal(), 1e-12)
    assert np.allclose(x, spla.spsolve(QAQ.tocsc(), b), rtol=1e-9, atol=1e-11)


def test_direct_solve_satisfies_constraints_free_slip():
    mac = shell_macros(1, 1, 0.55, 1.0)
    m = RefinedMesh(mac, 1)
    rng = np.random.default_rng(7)
    A = assemble_A(m, np.exp(rng.uniform(-2, 2, m.n1)))
    B = assemble_B(m)
    C = assemble_B(m, 0.5 * (1 - np.linalg.norm(m.X1, axis=1)), only_C=True)
    f = rng.standard_normal(3 * m.n2)
    Q, dm, fs = velocity_basis(m, {1}, {2})
    u, p, mu = solve_stokes(A, B + C, f, np.zeros(m.n1), Q, Bt=B.T)
    assert abs(p.mean()) < 1e-13
    n = m.X2[fs] / np.linalg.norm(m.X2[fs], axis=1, keepdims=True)
    U = u.reshape(3, -1).T
    assert np.abs(np.einsum("kd,kd->k", U[fs], n)).max() < 1e-13
    assert np.abs(u[dm]).max() == 0.0
    Pm = Q @ Q.T
    ru = Pm @ (f - A @ u - B.T @ p)
    rp = (B + C) @ u
    assert np.linalg.norm(ru) < 1e-10 * np.linalg.norm(f)
    assert np.linalg.norm(rp - rp.mean()) < 1e-10 * np.linalg.norm(f)


def _free_slip_both(level=2):
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), level)
    rng = np.random.default_rng(8)
    A = assemble_A(m, np.exp(rng.uniform(-2, 2, m.n1)))
    B = assemble_B(m)
    C = assemble_B(m, 0.5 * (1 - np.linalg.norm(m.X1, axis=1)), only_C=True)
    Q, dm, fs = velocity_basis(m, set(), {1, 2})
    return m, A, B, C, Q, fs, rigid_rotations(m)


def test_rigid_rotations_are_admissible_and_near_null_under_free_slip_on_both_spheres():
    """The rotations e_k x X are tangential at every sphere node (so P_v leaves
    them unchanged), and Q^T A Q has exactly three eigenvalues far below the
    rest: the blended A annihilates the rotations only up to the
    discretisation error, so without a constraint the solution's rotational
    part is set by that error."""
    m, A, B, C, Q, fs, R = _free_slip_both()
    Pm = Q @ Q.T
    assert np.abs(Pm @ R - R).max() < 1e-13 * np.abs(R).max()
    QAQ = (Q.T @ A @ Q).tocsc()
    small = np.sort(spla.eigsh(QAQ, k=5, sigma=-1e-9, which="LM", return_eigenvectors=False))
    big = spla.eigsh(QAQ, k=1, which="LA", return_eigenvectors=False)[0]
    assert small[2] < 1e-5 * big and small[3] > 30 * small[2]


def test_direct_solve_free_slip_on_both_spheres_removes_rotations():
    """The constrained solve: u tangential on both spheres, R^T u = 0, the
    momentum residual in span(R) (its projection vanishes), the continuity
    residual constant; and a body force that is itself a rigid rotation drives
    no flow, while a solve without the constraint does pick up a rotation."""
    m, A, B, C, Q, fs, R = _free_slip_both()
    Bb = B + C
    f = np.random.default_rng(9).standard_normal(3 * m.n2)
    u, p, mu = solve_stokes(A, Bb, f, np.zeros(m.n1), Q, Bt=B.T, rotations=R)
    U = u.reshape(3, -1).T
    n = m.X2[fs] / np.linalg.norm(m.X2[fs], axis=1, keepdims=True)
    assert np.abs(np.einsum("kd,kd->k", U[fs], n)).max() < 1e-13 * np.abs(U).max()
    assert np.abs(R.T @ u).max() < 1e-11 * np.linalg.norm(R, axis=0).max() * np.linalg.norm(u)
    Qr, _ = np.linalg.qr(Q.T @ R)
    ru = Q.T @ (f - A @ u - B.T @ p)
    ru -= Qr @ (Qr.T @ ru)
    rp = Bb @ u
    assert np.linalg.norm(ru) < 1e-10 * np.linalg.norm(f)
    assert np.linalg.norm(rp - rp.mean()) < 1e-10 * np.linalg.norm(f)
    assert abs(p.mean()) < 1e-13 * np.abs(p).max()
    # a rigid-rotation body force
    u0, p0, _ = solve_stokes(A, Bb, R @ np.array([0.3, -1.2, 0.7]), np.zeros(m.n1), Q, Bt=B.T, rotations=R)
    assert np.abs(u0).max() < 1e-10 and np.abs(p0).max() < 1e-10
    # without the constraint the same forcing spins the shell
    u1, _, _ = solve_stokes(A, Bb, f, np.zeros(m.n1), Q, Bt=B.T)
    rot = np.linalg.lstsq(R, u1, rcond=None)[0]
    assert np.linalg.norm(R @ rot) > 10 * np.linalg.norm(u)
