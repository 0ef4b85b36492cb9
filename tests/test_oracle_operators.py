"""Pins of the oracle's element integrals and assembled operators (CPU only)."""
import os
from math import factorial

import numpy as np
import pytest
import sympy as sy

from oracle.fem import (assemble_A, assemble_A_qp, assemble_B, assemble_M_inv_eta, element_A, geometry,
                        rhs_buoyancy, strain_and_div, vertex_p2_nodes, viscosity_model)
from oracle.mesh import RefinedMesh, cube_macros, shell_macros
from oracle.quadrature import rule_q4, rule_stroud


def _mono_integral(a, b, c):
    return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)


@pytest.mark.parametrize("rule,deg", [(rule_q4(), 2), (rule_stroud(4), 7), (rule_stroud(2), 3)])
def test_quadrature_exact_for_monomials(rule, deg):
    xi, w, lam = rule
    assert np.all(w > 0)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                q = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
                assert abs(q - _mono_integral(a, b, c)) < 1e-15


def test_q4_is_not_degree_3():
    xi, w, _ = rule_q4()
    assert abs(np.sum(w * xi[:, 0] ** 3) - _mono_integral(3, 0, 0)) > 1e-5


class _OneTet:
    """A single affine tetrahedron in the RefinedMesh interface."""

    def __init__(self, verts):
        self.ev = np.asarray(verts, dtype=np.float64)[None]
        self.blend_g = None
        self.emacro = np.zeros(1, dtype=np.int64)


def _exact_element_matrices(verts):
    """A (constant eta = 1), B and the P1 mass on one affine tet, integrated
    exactly from the nodal basis written symbolically."""
    x1, x2, x3 = sy.symbols("x1 x2 x3")
    xi = sy.Matrix([x1, x2, x3])
    V = [sy.Matrix([sy.Rational(int(round(c * 8)), 8) for c in v]) for v in verts]
    J = sy.Matrix.hstack(V[1] - V[0], V[2] - V[0], V[3] - V[0])
    detJ = abs(J.det())
    Jit = J.inv().T
    lam = [1 - x1 - x2 - x3, x1, x2, x3]
    edges = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
    N = [lam[i] * (2 * lam[i] - 1) for i in range(4)] + [4 * lam[i] * lam[j] for (i, j) in edges]
    G = [Jit * sy.Matrix([sy.diff(n, v) for v in (x1, x2, x3)]) for n in N]

    def integ(expr):
        p = sy.Poly(sy.expand(expr), x1, x2, x3)
        return sum(coef * sy.Rational(factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))
                   for (a, b, c), coef in p.terms()) * detJ

    A = np.zeros((30, 30))
    for c in range(3):
        for a in range(10):
            for d in range(3):
                for b in range(10):
                    e = (1 if c == d else 0) * (G[a].dot(G[b])) + G[a][d] * G[b][c] \
                        - sy.Rational(2, 3) * G[a][c] * G[b][d]
                    A[c * 10 + a, d * 10 + b] = float(integ(e))
    Bm = np.zeros((4, 30))
    for i in range(4):
        for d in range(3):
            for b in range(10):
                Bm[i, d * 10 + b] = float(integ(-lam[i] * G[b][d]))
    M = np.array([[float(integ(lam[i] * lam[j])) for j in range(4)] for i in range(4)])
    return A, Bm, M


def test_element_matrices_exact_on_affine_tet():
    verts = [[0.125, 0.0, 0.25], [1.0, 0.25, 0.0], [0.25, 1.125, 0.125], [0.0, 0.375, 0.875]]
    A_ex, B_ex, M_ex = _exact_element_matrices(verts)
    W, G2, G1, X, N2, N1 = geometry(_OneTet(verts), np.array([0]))
    A = element_A(W, G2, np.ones((1, 4)))[0]
    assert np.allclose(A, A_ex, rtol=0, atol=1e-13 * np.abs(A_ex).max())
    _, div = strain_and_div(G2)
    B = -np.einsum("eq,qi,eqa->eia", W, N1, div)[0]
    assert np.allclose(B, B_ex, atol=1e-14)
    M = np.einsum("eq,qi,qj->ij", W, N1, N1)
    assert np.allclose(M, M_ex, atol=1e-15)


def _fields(X):
    """10 fields with vanishing deviatoric strain: rigid modes, dilation and
    the special conformal fields 2(b.x)x - |x|^2 b."""
    out = []
    for c in range(3):
        v = np.zeros_like(X)
        v[:, c] = 1.0
        out.append(v)
    for (i, j) in [(0, 1), (0, 2), (1, 2)]:
        v = np.zeros_like(X)
        v[:, i], v[:, j] = X[:, j], -X[:, i]
        out.append(v)
    out.append(X.copy())
    for c in range(3):
        b = np.zeros(3)
        b[c] = 1.0
        out.append(2.0 * (X @ b)[:, None] * X - (X * X).sum(1)[:, None] * b)
    return [v.T.ravel() for v in out]


def test_A_kernel_symmetry_and_definiteness_affine():
    m = RefinedMesh(cube_macros(), 2)
    eta = np.random.default_rng(0).uniform(0.01, 100.0, m.n1)
    A = assemble_A(m, eta)
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    scale = abs(A).max()
    for v in _fields(m.x2):
        assert np.abs(A @ v).max() <= 1e-12 * scale * np.abs(v).max()
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 10               # kernel is exactly 10-dim


def test_literal_formula_reading_breaks_kernel_and_definiteness():
    """The printed formula without eta in the divergence term does not have
    the deviatoric kernel and is indefinite for eta < 1 (reading check)."""
    m = RefinedMesh(cube_macros(), 1)
    eta = np.full(m.n1, 0.25)
    rows = []
    for sel in [np.arange(m.ne)]:
        W, G2, G1, X, N2, N1 = geometry(m, sel)
        eps, div = strain_and_div(G2)
        lit = 2 * np.einsum("eq,eqaij,eqbij->eab", 0.25 * W, eps, eps) \
            - (2.0 / 3.0) * np.einsum("eq,eqa,eqb->eab", W, div, div)
    dil = m.x2.T.ravel()
    d = np.concatenate([m.e2 + c * m.n2 for c in range(3)], axis=1)
    val = np.einsum("ea,eab,eb->", dil[d], lit, dil[d])
    assert val < -1.0                                         # 6 eta - 6 per volume


def test_A_blended_symmetric_translations():
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    eta = np.random.default_rng(1).uniform(0.1, 10.0, m.n1)
    A = assemble_A(m, eta)
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    for c in range(3):
        v = np.zeros((m.n2, 3))
        v[:, c] = 1.0
        assert np.abs(A @ v.T.ravel()).max() <= 1e-12 * abs(A).max()
    x = np.random.default_rng(2).standard_normal(3 * m.n2)
    assert x @ (A @ x) > 0


def test_B_annihilates_constants_and_Bt_of_constant():
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    B = assemble_B(m)
    for c in range(3):
        v = np.zeros((m.n2, 3))
        v[:, c] = 1.0
        assert np.abs(B @ v.T.ravel()).max() < 1e-15
    mc = RefinedMesh(cube_macros(), 2)
    Bc = assemble_B(mc)
    g = Bc.T @ np.ones(mc.n1)
    inner = np.tile(mc.flag2 == 0, 3)
    assert np.abs(g[inner]).max() < 1e-15


def test_C_block():
    """C = 0 for constant ln rho; for linear ln rho = k.x, C u integrates
    -(k.u) psi, so 1^T C u = -int k.u."""
    m = RefinedMesh(cube_macros(), 1)
    C0 = assemble_B(m, np.full(m.n1, 3.0), only_C=True)
    assert abs(C0).max() < 1e-15
    k = np.array([0.3, -0.7, 1.1])
    C = assemble_B(m, m.x1 @ k, only_C=True)
    u = np.tile([1.0, 2.0, -1.0], (m.n2, 1)).T.ravel()
    assert np.isclose(np.ones(m.n1) @ (C @ u), -(k @ [1.0, 2.0, -1.0]), rtol=1e-13)


def test_mass_and_buoyancy():
    m = RefinedMesh(cube_macros(), 1)
    M = assemble_M_inv_eta(m, np.full(m.n1, 2.0))
    assert np.isclose(M.sum(), 0.5, rtol=1e-14)
    # buoyancy: f . I_h(x) = int T r_hat . x = int T |x|; T = 1 on the shell
    errs = []
    exact = np.pi * (1.0 - 0.55 ** 4)
    for L in range(3):
        ms = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), L)
        f = rhs_buoyancy(ms, np.ones(ms.n2))
        errs.append(abs(f @ ms.X2.T.ravel() - exact))
    assert errs[2] < errs[1] < errs[0] and errs[1] / errs[2] > 3.5


def test_quadrature_point_viscosity_assembly():
    """A with eta evaluated at the quadrature points (Sec. 5.2.2): on affine
    (cube) elements an affine eta(x) is its own P1 interpolant, so the
    assembly equals the P1-eta one; a quadratic T is its own P2 interpolant,
    so eta = T_h(x_q) equals eta = T(x_q); on the blended shell a constant
    eta reproduces the constant-eta operator."""
    m = RefinedMesh(cube_macros(), 2)
    k, c0 = np.array([0.3, -0.2, 0.5]), 1.7
    A1 = assemble_A(m, c0 + m.x1 @ k)
    Aq = assemble_A_qp(m, lambda X, Tq: c0 + X @ k, np.zeros(m.n2))
    assert abs(Aq - A1).max() <= 1e-13 * abs(A1).max()
    quad = lambda X: 2.0 + X[..., 0] * X[..., 1] - 0.5 * X[..., 2] ** 2 + X[..., 1]
    AT = assemble_A_qp(m, lambda X, Tq: Tq, quad(m.x2))
    AX = assemble_A_qp(m, lambda X, Tq: quad(X), np.zeros(m.n2))
    assert abs(AT - AX).max() <= 1e-13 * abs(AX).max()
    # the dropped-interpolation mistake is visible: P1 interpolation of the
    # quadratic differs from its quadrature-point values
    assert abs(assemble_A(m, quad(m.x1)) - AX).max() > 1e-3 * abs(AX).max()
    ms = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    Ac = assemble_A_qp(ms, lambda X, Tq: np.full(Tq.shape, 3.0), np.zeros(ms.n2))
    assert abs(Ac - assemble_A(ms, np.full(ms.n1, 3.0))).max() <= 1e-13 * abs(Ac).max()


def test_viscosity_model_and_vertex_nodes():
    """eq. ViscosityDef: eta_base interpolated linearly on its radial grid,
    exp(-E_A T) in temperature, exp(V_A (r_out - r)) in depth; P1 vertices
    map onto P2 nodes at the same place."""
    base = np.array([1.0, 3.0, 2.0])
    x = np.array([[0.55, 0.0, 0.0], [0.0, 0.6625, 0.0], [0.0, 0.0, 1.0], [0.3, 0.4, 0.0]])
    T = np.array([0.0, 0.5, 1.0, 0.2])
    eta = viscosity_model(x, T, base, 4.61, 2.996, 0.55, 1.0)
    b = np.array([1.0, 2.0, 2.0, 1.0])       # r = 0.55, 0.6625 (halfway to 0.775), 1, 0.5 (clamped)
    r = np.array([0.55, 0.6625, 1.0, 0.5])
    assert np.allclose(eta, b * np.exp(-4.61 * T + 2.996 * (1.0 - r)), rtol=1e-15)
    ms = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 2)
    v2 = vertex_p2_nodes(ms)
    assert np.abs(ms.X2[v2] - ms.X1).max() < 1e-15


def _p1_quadrature_points(ev):
    """Barycentric weights, reference points and weights (|K| / 4) of the
    symmetric 4-point rule on each reference element, computed from the
    element's vertices alone: point q has weight a on vertex q and b on the
    others, a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20."""
    a, b = (5.0 + 3.0 * 5 ** 0.5) / 20.0, (5.0 - 5 ** 0.5) / 20.0
    lam = np.full((4, 4), b) + (a - b) * np.eye(4)
    vol = np.abs(np.linalg.det(ev[:, 1:] - ev[:, :1])) / 6.0
    xq = np.einsum("qi,eid->eqd", lam, ev)
    return lam, xq, vol / 4.0


def test_mass_weight_is_reciprocal_viscosity_at_the_points():
    """M_{1/eta} (Sec. 5.2.3, eq. schurMass; reading: consistent mass with
    weight 1/eta_h(x_q)).  On affine (cube) elements an affine eta is its own
    P1 interpolant, so every entry must equal the 4-point quadrature of
    psi_i psi_j / eta(x_q) with eta evaluated analytically at the physical
    points; interpolating 1/eta instead (the other plausible reading) differs."""
    m = RefinedMesh(cube_macros(), 2)
    k, c0 = np.array([2.0, -1.5, 3.0]), 2.0
    eta_fn = lambda X: c0 + X @ k                      # in [0.5, 7] on the unit cube
    M = assemble_M_inv_eta(m, eta_fn(m.x1)).toarray()
    lam, xq, wq = _p1_quadrature_points(m.ev)
    ref = np.zeros((m.n1, m.n1))
    Me = np.einsum("e,eq,qi,qj->eij", wq, 1.0 / eta_fn(xq), lam, lam)
    for i in range(4):
        for j in range(4):
            np.add.at(ref, (m.e1[:, i], m.e1[:, j]), Me[:, i, j])
    assert np.abs(M - ref).max() <= 1e-14 * np.abs(ref).max()
    # negative control: the P1 interpolant of 1/eta at the points
    inv_h = np.einsum("qk,ek->eq", lam, 1.0 / eta_fn(m.x1)[m.e1])
    Mi = np.einsum("e,eq,qi,qj->eij", wq, inv_h, lam, lam)
    alt = np.zeros_like(ref)
    for i in range(4):
        for j in range(4):
            np.add.at(alt, (m.e1[:, i], m.e1[:, j]), Mi[:, i, j])
    assert np.abs(alt - ref).max() > 1e-4 * np.abs(ref).max()


def test_buoyancy_uses_the_p2_temperature_at_the_points():
    """f_i = int T_h r_hat . phi_i (Sec. 5.1 right-hand side, unit scaling):
    T_h is the P2 interpolant on the reference (unblended) mesh, so for T
    quadratic in the reference coordinate x~ it is exact at every quadrature
    point.  The reference is built without the oracle's geometry code: points
    from the element vertices, the blended weight |det J_F| |det J_B| with
    det J_B from central differences of the blending map, r_hat = x~/|x~|
    (the map is radial), and the P2 basis from its barycentric formulas.
    A P1 interpolation of T (a plausible mistake) differs."""
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    Tfn = lambda x: 0.4 + 0.3 * x[..., 0] * x[..., 2] - 0.2 * x[..., 1] ** 2 + 0.5 * x[..., 2]
    f = rhs_buoyancy(m, Tfn(m.x2))
    lam, xq, wq = _p1_quadrature_points(m.ev)
    g, s0 = m.blend_g[m.emacro], m.blend_s0[m.emacro]

    def blend(x):
        s = np.einsum("ed,eqd->eq", g, x) + s0[:, None]
        return x * (s / np.linalg.norm(x, axis=-1))[..., None]

    h = 1e-6
    J = np.empty(xq.shape + (3,))
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        J[..., d] = (blend(xq + e) - blend(xq - e)) / (2 * h)
    detB = np.linalg.det(J)
    rhat = xq / np.linalg.norm(xq, axis=-1, keepdims=True)
    edges = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
    N = np.concatenate([lam * (2 * lam - 1), np.stack([4 * lam[:, i] * lam[:, j] for i, j in edges], 1)], 1)

    def assemble(Tq):
        fe = np.einsum("eq,eq,eq,eqc,qa->eca", wq[:, None] * np.ones((1, 4)), detB, Tq, rhat, N)
        ref = np.zeros(3 * m.n2)
        for c in range(3):
            np.add.at(ref, c * m.n2 + m.e2, fe[:, c, :])
        return ref

    ref = assemble(Tfn(xq))
    assert np.abs(f - ref).max() <= 1e-8 * np.abs(ref).max()
    # negative control: T from its vertex values only (P1 interpolation)
    Tp1 = np.einsum("qk,ek->eq", lam, Tfn(m.x2)[m.e2[:, :4]])
    assert np.abs(assemble(Tp1) - ref).max() > 1e-4 * np.abs(ref).max()


# --- weighted BFBT operators (eq. schurWBFBT) -------------------------------------

def _exact_p2_mass_and_p1_stiffness(verts):
    """The P2 mass int N_a N_b and the P1 stiffness int grad lam_i . grad lam_j
    on one affine tet, integrated exactly from the symbolic basis."""
    x1, x2, x3 = sy.symbols("x1 x2 x3")
    V = [sy.Matrix([sy.Rational(int(round(c * 8)), 8) for c in v]) for v in verts]
    J = sy.Matrix.hstack(V[1] - V[0], V[2] - V[0], V[3] - V[0])
    detJ = abs(J.det())
    Jit = J.inv().T
    lam = [1 - x1 - x2 - x3, x1, x2, x3]
    edges = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
    N = [lam[i] * (2 * lam[i] - 1) for i in range(4)] + [4 * lam[i] * lam[j] for (i, j) in edges]

    def integ(expr):
        p = sy.Poly(sy.expand(expr), x1, x2, x3)
        return sum(coef * sy.Rational(factorial(a) * factorial(b) * factorial(c), factorial(a + b + c + 3))
                   for (a, b, c), coef in p.terms()) * detJ

    M = np.array([[float(integ(N[a] * N[b])) for b in range(10)] for a in range(10)])
    G = [Jit * sy.Matrix([sy.diff(l, v) for v in (x1, x2, x3)]) for l in lam]
    K = np.array([[float(G[i].dot(G[j]) * detJ / 6) for j in range(4)] for i in range(4)])
    return M, K


def test_vector_mass_and_poisson_exact_on_affine_tet():
    """Constant eta = 4 on one affine tet: M_{sqrt eta} is 2 x the exact P2
    mass in each component block (the 27-point rule integrates the degree-4
    integrand exactly) and K_{1/sqrt eta} is 1/2 x the exact P1 stiffness;
    the element factor s_K multiplies them by a and 1/a."""
    from oracle.fem import assemble_poisson_p1, assemble_vector_mass

    verts = [[0.125, 0.0, 0.25], [1.0, 0.25, 0.0], [0.25, 1.125, 0.125], [0.0, 0.375, 0.875]]
    M_ex, K_ex = _exact_p2_mass_and_p1_stiffness(verts)
    one = _OneTet(verts)
    one.e2 = np.arange(10)[None]
    one.e1 = np.arange(4)[None]
    one.n2, one.n1, one.ne = 10, 4, 1
    eta = np.full(4, 4.0)
    M = assemble_vector_mass(one, eta).toarray()
    for c in range(3):
        blk = M[c * 10:(c + 1) * 10, c * 10:(c + 1) * 10]
        assert np.allclose(blk, 2.0 * M_ex, rtol=0, atol=1e-15)
    assert np.abs(M[:10, 10:]).max() == 0.0
    assert np.linalg.matrix_rank(M[:10, :10]) == 10
    K = assemble_poisson_p1(one, eta).toarray()
    assert np.allclose(K, 0.5 * K_ex, rtol=0, atol=1e-14)
    s = np.array([9.0])
    assert np.allclose(assemble_vector_mass(one, eta, s).toarray(), 3.0 * M, atol=1e-15)
    assert np.allclose(assemble_poisson_p1(one, eta, s).toarray(), K / 3.0, atol=1e-15)
    # the 4-point rule of the Stokes blocks would leave the P2 mass singular
    from oracle.quadrature import rule_q4
    assert np.linalg.matrix_rank(assemble_vector_mass(one, eta, rule=rule_q4()).toarray()[:10, :10]) == 4


def test_vector_mass_takes_sqrt_eta_at_the_points_and_poisson_kernel():
    """An affine viscosity (its own P1 interpolant) on affine cube elements:
    M_{sqrt eta} equals the quadrature of sqrt(eta(x_q)) N_a N_b with eta taken
    analytically at the physical points, and differs from the reading that
    interpolates sqrt(eta) nodally.  The Poisson matrix annihilates
    constants, is symmetric, and x^T K x = int |grad x|^2 / sqrt(eta) for a
    linear x."""
    from oracle.fem import assemble_poisson_p1, assemble_vector_mass
    from oracle.quadrature import rule_stroud

    m = RefinedMesh(cube_macros(), 1)
    eta_fn = lambda X: 1.0 + 3.0 * X[..., 0] + 2.0 * X[..., 1] + X[..., 2]
    eta = eta_fn(m.X1)
    M = assemble_vector_mass(m, eta)
    rule = rule_stroud(3)
    ref = np.zeros((m.n2, m.n2))
    W, G2, G1, X, N2, N1 = geometry(m, np.arange(m.ne), rule)
    Me = np.einsum("eq,qa,qb->eab", W * np.sqrt(eta_fn(X)), N2, N2)
    for e in range(m.ne):
        ref[np.ix_(m.e2[e], m.e2[e])] += Me[e]
    assert np.abs(M[:m.n2, :m.n2].toarray() - ref).max() < 1e-15 * np.abs(ref).max() * 100
    # nodal interpolation of sqrt(eta) is a different matrix
    Mi = np.einsum("eq,eq,qa,qb->eab", W, np.einsum("qk,ek->eq", N1, np.sqrt(eta)[m.e1]), N2, N2)
    assert np.abs(Mi - Me).max() > 1e-6 * np.abs(Me).max()
    K = assemble_poisson_p1(m, eta)
    assert np.abs(K @ np.ones(m.n1)).max() < 1e-13 * abs(K).max()
    assert abs(K - K.T).max() < 1e-15 * abs(K).max()
    g = np.array([0.3, -1.1, 0.7])
    x = m.X1 @ g
    W, G2, G1, X, N2, N1 = geometry(m, np.arange(m.ne))
    expect = np.sum(W / np.sqrt(eta_fn(X))) * (g @ g)
    assert abs(x @ (K @ x) - expect) < 1e-12 * expect


def test_dirichlet_element_scale_marks_the_elements_touching_the_dirichlet_sphere():
    from oracle.fem import dirichlet_element_scale
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    s = dirichlet_element_scale(m, {1}, 10.0)
    r = np.linalg.norm(m.X1[m.e1], axis=2)
    touch = (np.abs(r - 0.55) < 1e-12).any(axis=1)
    assert np.array_equal(s == 100.0, touch) and np.all(s[~touch] == 1.0) and touch.any() and (~touch).any()
    assert np.all(dirichlet_element_scale(m, {1}, 1.0) == 1.0)


def test_multicore_spmv_equals_scipy():
    """The oracle's OpenMP CSR product (host timing) sums each row in storage
    order, as scipy does: equal to A @ x up to rounding on an assembled A."""
    from oracle import cspmv
    if not os.path.exists(cspmv.LIB):
        cspmv.build()
    m = RefinedMesh(shell_macros(1, 1, 0.55, 1.0), 1)
    A = assemble_A(m, np.exp(np.linspace(-1.0, 1.0, m.n1)))
    x = np.random.default_rng(7).standard_normal(A.shape[0])
    ref = A @ x
    assert np.abs(cspmv.spmv(A, x) - ref).max() <= 1e-14 * np.abs(ref).max()
