"""GPU parity of the solver components against the oracle's assembled references."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import inputs
from oracle.adjoint import grad_log_eta, grad_temperature
from oracle.fem import assemble_A, assemble_B, rhs_buoyancy
from oracle.solvers import chebyshev, prolongation, vcycle, vector_prolongation
from oracle.system import solve_stokes
from paper_2506_04157_amd import default_params
from tests._util import Pair, relerr

pytestmark = pytest.mark.gpu


def _eta(m, seed=3, lo=-2.0, hi=2.0):
    return np.exp(inputs.uniform(seed, m.n1, lo, hi))


@pytest.mark.parametrize("kind,L,lmin", [("cube", 3, 1), ("shell", 2, 0)])
def test_prolongation_and_restriction(kind, L, lmin):
    print(f"\n[transfers {kind} L{L}]", flush=True)
    P = Pair(kind, L, min_level=lmin)
    for l in range(lmin + 1, L + 1):
        mc, mf = P.meshes[l - 1], P.meshes[l]
        Pro = vector_prolongation(prolongation(mc, mf))
        Pf, _ = P.projector(l)
        Pc, _ = P.projector(l - 1)
        for dtype, tol in [(torch.float64, 1e-14), (torch.float32, 1e-6)]:
            ec = inputs.uniform(7, 3 * mc.n2)
            ef = P.u_to_or(P.ctx.prolong(P.u_to_lib(ec, l - 1, dtype), l), l)
            assert relerr(ef, Pf @ (Pro @ ec)) < tol
            rf = inputs.uniform(8, 3 * mf.n2)
            rc = P.u_to_or(P.ctx.restrict(P.u_to_lib(rf, l, dtype), l), l - 1)
            assert relerr(rc, Pc @ (Pro.T @ rf)) < tol
            # the V-cycle's fused forms: x += P_v P e_c and P_v P^T P_v (b - t)
            x0 = inputs.uniform(9, 3 * mf.n2)
            xs = P.ctx.prolong(P.u_to_lib(ec, l - 1, dtype), l, add_to=P.u_to_lib(x0, l, dtype))
            assert relerr(P.u_to_or(xs, l), x0 + Pf @ (Pro @ ec)) < tol
            tf = inputs.uniform(10, 3 * mf.n2)
            rd = P.ctx.restrict(P.u_to_lib(rf, l, dtype), l, minus=P.u_to_lib(tf, l, dtype))
            assert relerr(P.u_to_or(rd, l - 1), Pc @ (Pro.T @ (Pf @ (rf - tf)))) < tol


def _oracle_levels(P, eta_fine, bounds):
    levels = []
    lmin = min(P.meshes)
    etas = {}
    for l in sorted(P.meshes):
        m = P.meshes[l]
        # nodal injection of the fine viscosity (coarse nodes are fine nodes)
        from scipy.spatial import cKDTree
        idx = cKDTree(P.meshes[P.L].X1).query(m.X1)[1]
        etas[l] = eta_fine[idx]
        A = assemble_A(m, etas[l])
        Pm, Q = P.projector(l)
        d = dict(A=A, P=Pm, Q=Q, Dinv=1.0 / A.diagonal())
        if l in bounds:
            d["lo"], d["hi"] = bounds[l]
        if l > lmin:
            d["Pro"] = vector_prolongation(prolongation(P.meshes[l - 1], m))
        levels.append(d)
    return levels


def _power_bounds(levels, lmin):
    b = {}
    for i, d in enumerate(levels[1:], start=1):
        x = d["P"] @ inputs.uniform(20 + i, d["A"].shape[0])
        for _ in range(30):
            x = d["P"] @ (d["Dinv"] * (d["A"] @ (d["P"] @ x)))
            lam = np.linalg.norm(x)
            x /= lam
        b[lmin + i] = (0.12 * lam, 1.2 * lam)
    return b


def test_spectral_bound_matches_power_iteration_and_covers_the_spectrum():
    """lambda-hat of every level: the library's FP64 power iteration on
    P D^-1 P A P (D = diag(A), no projection) from its splitmix64 start vector
    (Sec. 5.2.2: the Chebyshev smoother's interval; the method is the reading
    of the build).  The oracle repeats the same iteration on its assembled A
    from the same start vector (drawn here with the same published
    generator, in the library's node order) and must agree to 1e-10; and the
    interval's top 1.2 lambda-hat must lie above the largest eigenvalue of
    D^-1 A on range(P), computed by ARPACK."""
    print("\n[lambda-hat shell L2]", flush=True)
    P = Pair("shell", 2, min_level=0)
    m = P.meshes[2]
    eta = _eta(m)
    params = default_params(power_its=15)
    P.ctx.set_fields(P.p_to_lib(eta), params=params)
    levels = _oracle_levels(P, eta, {})
    for l in (1, 2):
        d = levels[l]
        lo, hi = P.ctx.cheb_bounds(l)
        lam_gpu = hi / params.cheb_hi
        assert abs(lo / params.cheb_lo - lam_gpu) <= 1e-14 * lam_gpu
        n = d["A"].shape[0]
        x0 = inputs.splitmix64_uniform(0x9E3779B97F4A7C15 ^ l, n)        # library order
        x = d["P"] @ P.u_to_or(torch.tensor(x0), l)
        x /= np.linalg.norm(x)
        for _ in range(params.power_its):
            x = d["P"] @ (d["Dinv"] * (d["P"] @ (d["A"] @ (d["P"] @ x))))
            lam = np.linalg.norm(x)
            x /= lam
        print(l, lam_gpu, lam, abs(lam_gpu - lam) / lam)
        assert abs(lam_gpu - lam) <= 1e-10 * lam
        op = spla.LinearOperator((n, n), dtype=np.float64,
                                 matvec=lambda v: d["P"] @ (d["Dinv"] * (d["P"] @ (d["A"] @ (d["P"] @ v)))))
        lmax = float(np.max(np.real(spla.eigs(op, k=1, which="LR", tol=1e-10,
                                              v0=np.ones(n), return_eigenvectors=False))))
        print("  lambda_max", lmax, "lambda-hat / lambda_max", lam_gpu / lmax)
        assert hi >= lmax and lam_gpu <= 1.2 * lmax


@pytest.mark.parametrize("kind,L,lmin", [("cube", 3, 1), ("shell", 2, 0)])
def test_chebyshev_smoother(kind, L, lmin):
    print(f"\n[chebyshev {kind} L{L}]", flush=True)
    P = Pair(kind, L, min_level=lmin)
    m = P.meshes[L]
    eta = _eta(m)
    P.ctx.set_fields(P.p_to_lib(eta))
    levels = _oracle_levels(P, eta, {})
    bounds = _power_bounds(levels, lmin)
    lo, hi = bounds[L]
    P.ctx.set_cheb_bounds(L, lo, hi)
    d = levels[-1]
    b = d["P"] @ inputs.uniform(1, 3 * m.n2)
    x0 = d["P"] @ inputs.uniform(2, 3 * m.n2)
    for deg, steps in [(1, 1), (2, 3), (3, 2)]:
        ref = chebyshev(d["A"], d["Dinv"], d["P"], b, x0, lo, hi, deg, steps)
        for dtype, tol in [(torch.float64, 1e-12), (torch.float32, 1e-5)]:
            x = P.u_to_lib(x0, dtype=dtype)
            P.ctx.smooth(P.u_to_lib(b, dtype=dtype), x, degree=deg, steps=steps)
            assert relerr(P.u_to_or(x), ref) < tol, (deg, steps, dtype)


@pytest.mark.parametrize("kind,L,lmin", [("cube", 3, 1), ("shell", 2, 0)])
def test_vcycle_matches_assembled_vcycle(kind, L, lmin):
    print(f"\n[vcycle {kind} L{L}]", flush=True)
    P = Pair(kind, L, min_level=lmin)
    m = P.meshes[L]
    eta = _eta(m)
    levels = _oracle_levels(P, eta, {})
    bounds = _power_bounds(levels, lmin)
    for l, (lo, hi) in bounds.items():
        levels[l - lmin]["lo"], levels[l - lmin]["hi"] = lo, hi
        P.ctx.set_cheb_bounds(l, lo, hi)
    params = default_params(tol_coarse=1e-15, max_inner=2000)
    P.ctx.set_fields(P.p_to_lib(eta), params=params)
    Q0 = levels[0]["Q"]
    lu = spla.splu((Q0.T @ levels[0]["A"] @ Q0).tocsc())
    cs = lambda r: Q0 @ lu.solve(Q0.T @ r)
    b = levels[-1]["P"] @ inputs.uniform(4, 3 * m.n2)
    for which, (steps, deg) in [(0, (3, 2)), (1, (1, 1))]:
        ref = vcycle(levels, L - lmin, b, cs, deg, steps)
        x = P.ctx.vcycle(P.u_to_lib(b), params, which=which)
        assert relerr(P.u_to_or(x), ref) < 1e-9
        x32 = P.ctx.vcycle(P.u_to_lib(b, dtype=torch.float32), params, which=which)
        assert relerr(P.u_to_or(x32), ref) < 1e-4


def test_vcycle_bfbt_step_matches_oracle():
    """The V-cycle BFBT of eq. (schurV) as a component: one symmetric Uzawa
    step whose Schur inverse is (B C^-1 B^T)^-1 (B C^-1 A C^-1 B^T)
    (B C^-1 B^T)^-1 with C^-1 one V-cycle (Chebyshev degree 1, one step,
    exact coarse solve), the two outer solves by CG preconditioned with
    M_{1/eta} to 1e-13, the A-block solve to 1e-12; against the oracle's
    `bfbt` with its assembled V-cycle, a CG to 1e-14 for B C^-1 B^T and exact
    projected solves elsewhere (1×1 shell, level 2, variable eta)."""
    from oracle.fem import assemble_M_inv_eta
    from oracle.solvers import bfbt, pcg, symmetric_uzawa
    from paper_2506_04157_amd._lib import SCHUR_VBFBT, UZAWA_SYMMETRIC
    print("\n[V-cycle BFBT shell L2]", flush=True)
    P = Pair("shell", 2, min_level=0)
    m = P.meshes[2]
    eta = _eta(m)
    levels = _oracle_levels(P, eta, {})
    for l, (lo, hi) in _power_bounds(levels, 0).items():
        levels[l]["lo"], levels[l]["hi"] = lo, hi
        P.ctx.set_cheb_bounds(l, lo, hi)
    params = default_params(precision=64, tol_A=1e-12, tol_vbfbt=1e-13, tol_invmass=1e-14, tol_coarse=1e-15,
                            max_inner=2000, uzawa=UZAWA_SYMMETRIC, schur=SCHUR_VBFBT)
    P.ctx.set_fields(P.p_to_lib(eta), params=params)
    ru = inputs.uniform(61, 3 * m.n2)
    rp = inputs.uniform(62, m.n1)
    zu, zp = P.ctx.precondition(P.u_to_lib(ru), P.p_to_lib(rp), params=params)
    zu, zp = P.u_to_or(zu), P.p_to_or(zp)
    A, Pm, Q = levels[-1]["A"], levels[-1]["P"], levels[-1]["Q"]
    B = assemble_B(m)
    Q0 = levels[0]["Q"]
    lu0 = spla.splu((Q0.T @ levels[0]["A"] @ Q0).tocsc())
    cs = lambda r: Q0 @ lu0.solve(Q0.T @ r)
    V = lambda b: vcycle(levels, 2, Pm @ b, cs, params.deg_V, params.m_V)
    Alu = spla.splu((Q.T @ A @ Q).tocsc())
    Ainv = lambda r: Q @ Alu.solve(Q.T @ r)
    Mlu = spla.splu(assemble_M_inv_eta(m, eta).tocsc())
    mean0 = lambda v: v - v.mean()
    SC = lambda p: mean0(B @ (Pm @ V(Pm @ (B.T @ p))))
    solve_BAB = lambda r: mean0(pcg(SC, mean0(r), lambda v: mean0(Mlu.solve(v)), 1e-14, maxit=2000)[0])
    Sinv = lambda r: bfbt(mean0(r), (B @ Pm).tocsr(), (Pm @ B.T).tocsr(), (Pm @ A @ Pm).tocsr(), V, solve_BAB)
    uo, po = symmetric_uzawa(ru, mean0(rp), A, B.T, B, Ainv, Sinv, params.sigma, params.omega)
    eu, ep = relerr(zu, uo), relerr(zp, mean0(po))
    print(f"V-cycle BFBT step: u {eu:.2e}, p {ep:.2e}")
    assert eu < 1e-8 and ep < 1e-8


def _oracle_solution(P, eta, lnrho, f, uD=None, transpose=False):
    m = P.meshes[P.L]
    A = assemble_A(m, eta)
    B = assemble_B(m)
    Bb = B + assemble_B(m, lnrho, only_C=True) if lnrho is not None else B
    _, Q = P.projector()
    if transpose:
        return solve_stokes(A, B, f, np.zeros(m.n1), Q, uD, Bt=Bb.T), (A, B, Bb, Q)
    return solve_stokes(A, Bb, f, np.zeros(m.n1), Q, uD, Bt=B.T), (A, B, Bb, Q)


@pytest.mark.parametrize("precision", [64, 32])
def test_solve_cube_dirichlet_data(precision):
    print(f"\n[solve cube prec {precision}]", flush=True)
    P = Pair("cube", 3, min_level=1)
    m = P.meshes[3]
    eta = np.exp(2.0 * np.sin(3 * m.X1[:, 0]) * np.cos(2 * m.X1[:, 1]))
    f = inputs.uniform(5, 3 * m.n2)
    uD = inputs.smooth_vector_field(6, m.X2).T.ravel()
    (uo, po, _), (A, B, Bb, Q) = _oracle_solution(P, eta, None, f, uD)
    params = default_params(tol_rel=1e-10, precision=precision)
    P.ctx.set_fields(P.p_to_lib(eta), params=params)
    u, p, rep = P.ctx.solve(P.u_to_lib(f), u_dirichlet=P.u_to_lib(uD), params=params)
    print(rep["iterations"], rep["rel_residual"], rep["seconds"])
    ug, pg = P.u_to_or(u), P.p_to_or(p)
    assert rep["rel_residual"] <= 1e-10
    assert relerr(ug, uo) < 1e-7 and relerr(pg, po) < 1e-6
    # residual of the GPU solution in the oracle's assembled system
    Pm = Q @ Q.T
    ru = Pm @ (f - A @ ug - B.T @ pg)
    assert np.linalg.norm(ru) <= 1e-8 * np.linalg.norm(Pm @ (f - A @ uD))
    dm = np.tile(m.flag2 == 1, 3)
    assert np.allclose(ug[dm], uD[dm], atol=1e-14)


@pytest.mark.parametrize("precision", [64, 32])
def test_solve_shell_freeslip_compressible(precision):
    print(f"\n[solve shell prec {precision}]", flush=True)
    P = Pair("shell", 2, min_level=0, n_tan=1, n_rad=1)
    m = P.meshes[2]
    field = inputs.SHField(2)
    eta = inputs.viscosity_contrast(field.temperature(m.X1), 1e4)
    lnrho = inputs.ln_density(m.X1)
    T = field.temperature(m.X2)
    f = rhs_buoyancy(m, T)
    (uo, po, _), (A, B, Bb, Q) = _oracle_solution(P, eta, lnrho, f)
    params = default_params(tol_rel=1e-10, precision=precision)
    P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho), params=params)
    fl = P.ctx.rhs_buoyancy(P.s2_to_lib(T))
    assert relerr(P.u_to_or(fl), f) < 1e-12
    u, p, rep = P.ctx.solve(fl, params=params)
    print(rep["iterations"], rep["rel_residual"], rep["seconds"], rep["a_cg_its"], rep["s_cg_its"])
    ug, pg = P.u_to_or(u), P.p_to_or(p)
    assert rep["rel_residual"] <= 1e-10
    # the GPU solution solves the oracle's assembled constrained system to the
    # stated residual tolerance ...
    Pm = Q @ Q.T
    ru = Pm @ (f - A @ ug - B.T @ pg)
    rp = Bb @ ug
    rp = rp - rp.mean()
    assert np.hypot(np.linalg.norm(ru), np.linalg.norm(rp)) <= 2e-10 * np.linalg.norm(Pm @ f)
    # ... and is close to its direct solution (error <= condition x residual)
    assert relerr(ug, uo) < 1e-5 and relerr(pg, po) < 1e-5
    assert abs(pg.mean()) < 1e-12 * np.abs(pg).max()


def test_solve_shell_contrast_1e6_mixed_and_fp64():
    """Viscosity contrast 1e6 (depth factor, a seeded slab and the
    temperature factor of the third workload, calibrated on the P1 nodes),
    compressible, no-slip inner / free-slip outer, 1×1 shell at level 2: the
    mixed-precision solve (FP32 V-cycles with FP64 Chebyshev bounds and FP64
    coarse solve inside FP64 FGMRES) and the all-FP64 solve both reach 1e-10
    in the oracle's assembled system, and their solutions differ by no more
    than the residual allows."""
    print("\n[solve shell contrast 1e6]", flush=True)
    P = Pair("shell", 2, min_level=0, n_tan=1, n_rad=1)
    m = P.meshes[2]
    field = inputs.SHField(2)
    eta = inputs.viscosity_1e6(m.X1, field.temperature(m.X1))
    assert eta.max() / eta.min() == pytest.approx(1e6, rel=1e-9)
    lnrho = inputs.ln_density(m.X1)
    T = field.temperature(m.X2)
    f = rhs_buoyancy(m, T)
    (uo, po, _), (A, B, Bb, Q) = _oracle_solution(P, eta, lnrho, f)
    Pm = Q @ Q.T
    sol = {}
    for precision in (32, 64):
        params = default_params(tol_rel=1e-10, precision=precision, max_outer=400)
        P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho), params=params)
        u, p, rep = P.ctx.solve(P.ctx.rhs_buoyancy(P.s2_to_lib(T)), params=params)
        ug, pg = P.u_to_or(u), P.p_to_or(p)
        ru = Pm @ (f - A @ ug - B.T @ pg)
        rp = Bb @ ug
        rp = rp - rp.mean()
        res = np.hypot(np.linalg.norm(ru), np.linalg.norm(rp)) / np.linalg.norm(Pm @ f)
        print(f"precision {precision}: {rep['iterations']} its, rel {rep['rel_residual']:.2e}, oracle-system "
              f"residual {res:.2e}, |u - u_direct| {relerr(ug, uo):.2e}, {rep['seconds']:.1f} s")
        assert rep["rel_residual"] <= 1e-10 and res <= 2e-10
        # error <= condition x residual: the bar of the contrast-1e4 solve test
        assert relerr(ug, uo) < 1e-5 and relerr(pg, po) < 1e-5
        sol[precision] = (ug, pg)
    du = relerr(sol[32][0], sol[64][0])
    dp = relerr(sol[32][1], sol[64][1])
    print(f"mixed vs FP64: u {du:.2e}, p {dp:.2e}")
    assert du < 1e-5 and dp < 1e-5


@pytest.mark.parametrize("precision", [64, 32])
def test_solve_shell_plate_velocity_and_freeslip_cmb(precision):
    """The boundary arrangement of the paper's model (Sec. 2): prescribed
    tangential (plate) velocity at the surface r = 1, free slip at the
    core-mantle boundary r = 0.55; compressible, viscosity contrast 1e4."""
    print(f"\n[solve shell plates prec {precision}]", flush=True)
    P = Pair("shell", 2, min_level=0, n_tan=1, n_rad=1, bc_inner=2, bc_outer=1)
    m = P.meshes[2]
    field = inputs.SHField(2)
    eta = inputs.viscosity_contrast(field.temperature(m.X1), 1e4)
    lnrho = inputs.ln_density(m.X1)
    f = rhs_buoyancy(m, field.temperature(m.X2))
    uS = inputs.plate_velocity(13, m.X2)
    assert np.abs(np.einsum("ij,ij->i", uS, m.X2)).max() < 1e-13   # tangential
    uD = np.where(m.flag2 == 2, uS.T, 0.0).ravel()   # the data lives on the surface nodes
    (uo, po, _), (A, B, Bb, Q) = _oracle_solution(P, eta, lnrho, f, uD)
    params = default_params(tol_rel=1e-10, precision=precision)
    P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho), params=params)
    u, p, rep = P.ctx.solve(P.u_to_lib(f), u_dirichlet=P.u_to_lib(uD), params=params)
    print(rep["iterations"], rep["rel_residual"], rep["seconds"])
    ug, pg = P.u_to_or(u), P.p_to_or(p)
    assert rep["rel_residual"] <= 1e-10
    Pm = Q @ Q.T
    ru = Pm @ (f - A @ ug - B.T @ pg)
    rp = Bb @ ug
    rp = rp - rp.mean()
    scale = np.hypot(np.linalg.norm(Pm @ (f - A @ uD)), np.linalg.norm(Bb @ uD))
    assert np.hypot(np.linalg.norm(ru), np.linalg.norm(rp)) <= 2e-10 * scale
    assert relerr(ug, uo) < 1e-5 and relerr(pg, po) < 1e-5
    # surface nodes carry the plate velocity; core-mantle boundary nodes have u.n = 0
    U = ug.reshape(3, -1).T
    surf, cmb = m.flag2 == 2, m.flag2 == 1
    assert np.abs(U[surf] - uS[surf]).max() <= 1e-14 * np.abs(uS).max()
    nrm = m.X2[cmb] / np.linalg.norm(m.X2[cmb], axis=1)[:, None]
    assert np.abs(np.einsum("ij,ij->i", U[cmb], nrm)).max() <= 1e-12 * np.abs(U).max()


def test_adjoint_solve_and_gradient():
    print("\n[adjoint]", flush=True)
    P = Pair("shell", 2, min_level=0)
    m = P.meshes[2]
    eta = _eta(m, 9, -1.5, 1.5)
    lnrho = inputs.ln_density(m.X1)
    ju = inputs.uniform(10, 3 * m.n2)
    (lo, lpo, _), (A, B, Bb, Q) = _oracle_solution(P, eta, lnrho, ju, transpose=True)
    params = default_params(tol_rel=1e-11)
    P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho), params=params)
    lu, lp, rep = P.ctx.solve_adjoint(P.u_to_lib(ju), params=params)
    assert relerr(P.u_to_or(lu), lo) < 1e-7
    # gradient kernel vs the oracle's assembled gradient (any u, lambda)
    u = inputs.uniform(11, 3 * m.n2)
    lam = inputs.uniform(12, 3 * m.n2)
    gm, gT = P.ctx.gradient(P.u_to_lib(u), P.u_to_lib(lam), scale=1.5)
    assert relerr(P.p_to_or(gm), grad_log_eta(m, eta, u, lam)) < 1e-12
    assert relerr(P.s2_to_or(gT), grad_temperature(m, lam, scale=1.5)) < 1e-12


FD_H = 1e-6
FD_DIRECTIONS, FD_CHUNK = 20, 5


@pytest.fixture(scope="module", params=[64, 32], ids=["fp64", "mixed"])
def fd_problem(request):
    """The gradient-check problem: J = 1/2 |u - u_obs|^2 with u_obs the solution
    for the log-viscosity m + 0.1 zeta (zeta a seeded smooth field, seed 5),
    on the 240-macro shell (n_t = 2, n_r = 1) at level 3, viscosity contrast
    1e4, C = 0; the base solve (1e-13) and the autograd gradient (adjoint solve
    to 1e-12) in the given precision."""
    from paper_2506_04157_amd import StokesContext, StokesSolve
    precision = request.param
    print(f"\n[autograd FD setup prec {precision}]", flush=True)
    sc = StokesContext("shell", level=3, min_level=0, n_tan=2, n_rad=1)
    n2, n1 = sc.sizes()
    X2, _ = sc.coords(which=2)
    X1, _ = sc.coords(which=1)
    field = inputs.SHField(2)
    m0 = np.log(inputs.viscosity_contrast(field.temperature(X1), 1e4))
    T0 = field.temperature(X2)
    zeta = 2.0 * inputs.SHField(5).temperature(X1) - 1.0
    dev = lambda v: torch.tensor(v, dtype=torch.float64, device="cuda")
    p_obs = default_params(tol_rel=1e-13, precision=64, max_outer=300, restart=50)
    sc.set_log_viscosity(dev(m0 + 0.1 * zeta), params=p_obs)
    uobs, _, _ = sc.solve(sc.rhs_buoyancy(dev(T0)), params=p_obs)
    fwd = default_params(tol_rel=1e-13, precision=precision, max_outer=300, restart=50)
    adj = default_params(tol_rel=1e-12, precision=precision, max_outer=300, restart=50)

    sc.set_log_viscosity(dev(m0), params=fwd)
    u0, p0, _ = sc.solve(sc.rhs_buoyancy(dev(T0)), params=fwd)
    ju = (u0 - uobs).contiguous()
    # the adjoint solve (to 1e-12) and the gradient kernel
    sc.set_log_viscosity(dev(m0), params=adj)
    lu, _, rep = sc.solve_adjoint(ju, None, adj)
    gm, gT = sc.gradient(u0, lu)
    # the same gradient through torch.autograd (the backward of StokesSolve)
    mt2, Tt2 = dev(m0).requires_grad_(True), dev(T0).requires_grad_(True)
    u2, _ = StokesSolve.apply(mt2, Tt2, sc, adj)
    (0.5 * ((u2 - uobs) ** 2).sum()).backward()
    g_auto = (mt2.grad.cpu().numpy(), Tt2.grad.cpu().numpy())
    corr = default_params(tol_rel=1e-10, precision=precision, max_outer=300, restart=50)
    yield dict(sc=sc, n1=n1, n2=n2, m0=m0, T0=T0, u0=u0, p0=p0, uobs=uobs, gm=gm.cpu().numpy(),
               gT=gT.cpu().numpy(), g_auto=g_auto, corr=corr, dev=dev)
    sc.close()


@pytest.mark.parametrize("chunk", range(FD_DIRECTIONS // FD_CHUNK))
def test_gradient_matches_central_differences(fd_problem, chunk):
    """dJ/dm and dJ/dT against central differences with h = 1e-6, direction by
    direction: |fd - g.d| <= 1e-6 |fd| for the seeded directions (seed 4) of
    this chunk (20 in all, 5 per test, in FP64 and in mixed precision).

    The perturbed solutions are u0 + du, where du solves K(m +- h d) du =
    b(T) - K(m +- h d) [u0; p0] from the base solution [u0; p0] (to 1e-10
    relative to its own right-hand side): the correction is O(h), so the
    solver's tolerance bounds the error of u+ - u- relative to h |du/dm d|,
    not to |u|, whereas two solves each converged relative to |f| would
    leave their error divided by h in the difference.  u depends on T
    affinely (through the right-hand side only), so its central difference
    equals, for any h, the solution of K du = b(dT) times 2h, which one solve
    gives."""
    P = fd_problem
    sc, dev, u0, p0, uobs, corr = P["sc"], P["dev"], P["u0"], P["p0"], P["uobs"], P["corr"]
    m0, T0 = P["m0"], P["T0"]
    # the autograd backward computes the same gradient as the explicit adjoint path
    assert np.linalg.norm(P["g_auto"][0] - P["gm"]) <= 1e-9 * np.linalg.norm(P["gm"])
    assert np.linalg.norm(P["g_auto"][1] - P["gT"]) <= 1e-9 * np.linalg.norm(P["gT"])
    f0 = sc.rhs_buoyancy(dev(T0))

    def correction(mv):
        sc.set_log_viscosity(dev(mv), params=corr)
        yu, yp = sc.apply_K(u0, p0, bc=3)
        du, _, rep = sc.solve(f0 - yu, g=-yp, params=corr)
        assert rep["rel_residual"] <= 1e-10
        return du

    for k in range(chunk * FD_CHUNK, (chunk + 1) * FD_CHUNK):
        dmv = inputs.normal([4, k], P["n1"])
        dTv = inputs.normal([4, 100 + k], P["n2"])
        dp, dm_ = correction(m0 + FD_H * dmv), correction(m0 - FD_H * dmv)
        # (J+ - J-)/(2h) = (u+ - u-) . ((u+ + u-)/2 - u_obs) / (2h), u+- = u0 + du+-
        fdm = ((dp - dm_) * (u0 + 0.5 * (dp + dm_) - uobs)).sum().item() / (2 * FD_H)
        sc.set_log_viscosity(dev(m0), params=corr)
        dT, _, rep = sc.solve(sc.rhs_buoyancy(dev(dTv)), params=corr)
        assert rep["rel_residual"] <= 1e-10
        fdT = (dT * (u0 - uobs)).sum().item()
        gdm, gdT = P["gm"] @ dmv, P["gT"] @ dTv
        em, eT = abs(fdm - gdm) / abs(fdm), abs(fdT - gdT) / abs(fdT)
        print(k, f"m: fd {fdm:.10e} g.d {gdm:.10e} rel {em:.2e} | T: fd {fdT:.10e} g.d {gdT:.10e} rel {eT:.2e}",
              flush=True)
        assert em <= 1e-6 and eT <= 1e-6, k


def test_coarsest_level_size_limit():
    """The coarse-grid CG keeps the coarsest level's element matrices: a
    coarsest level above the stated size is refused at creation."""
    from paper_2506_04157_amd import StokesContext
    from paper_2506_04157_amd._lib import STK_EINVAL, StokesError
    with pytest.raises(StokesError) as err:
        StokesContext("shell", level=2, min_level=2, n_tan=10, n_rad=2)   # 768,000 coarsest micro-tets
    assert err.value.code == STK_EINVAL and "min_level" in str(err.value)


@pytest.mark.parametrize("precision", [64, 32])
def test_solve_shell_free_slip_on_both_spheres(precision):
    """Free slip on both spheres (NEXT-3): the rigid rotations e_k x X are
    admissible and strain free, so the solves remove them (R^T u = 0, the
    momentum residual projected off span(R)).  The GPU solution solves the
    oracle's constrained system (three rotation multipliers) to the stated
    tolerance and is close to its direct solution; compressible, viscosity
    contrast 1e4."""
    from oracle.system import rigid_rotations
    print(f"\n[solve shell free slip both prec {precision}]", flush=True)
    P = Pair("shell", 2, min_level=0, n_tan=1, n_rad=1, bc_inner=2, bc_outer=2)
    m = P.meshes[2]
    field = inputs.SHField(2)
    eta = inputs.viscosity_contrast(field.temperature(m.X1), 1e4)
    lnrho = inputs.ln_density(m.X1)
    f = rhs_buoyancy(m, field.temperature(m.X2))
    R = rigid_rotations(m)
    A = assemble_A(m, eta)
    B = assemble_B(m)
    Bb = B + assemble_B(m, lnrho, only_C=True)
    _, Q = P.projector()
    uo, po, _ = solve_stokes(A, Bb, f, np.zeros(m.n1), Q, Bt=B.T, rotations=R)
    params = default_params(tol_rel=1e-10, precision=precision)
    P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho), params=params)
    u, p, rep = P.ctx.solve(P.u_to_lib(f), params=params)
    print(rep["iterations"], rep["rel_residual"], rep["seconds"])
    ug, pg = P.u_to_or(u), P.p_to_or(p)
    assert rep["rel_residual"] <= 1e-10
    # no rigid rotation in the solution
    assert np.abs(R.T @ ug).max() <= 1e-12 * np.linalg.norm(R, axis=0).max() * np.linalg.norm(ug)
    # the residual in the oracle's system, with span(R) projected off
    Pm = Q @ Q.T
    Qr, _ = np.linalg.qr(R)
    ru = Pm @ (f - A @ ug - B.T @ pg)
    ru -= Qr @ (Qr.T @ ru)
    rp = Bb @ ug
    rp = rp - rp.mean()
    fr = Pm @ f - Qr @ (Qr.T @ (Pm @ f))
    assert np.hypot(np.linalg.norm(ru), np.linalg.norm(rp)) <= 2e-10 * np.linalg.norm(fr)
    assert relerr(ug, uo) < 1e-5 and relerr(pg, po) < 1e-5
    # tangential on both spheres
    U = ug.reshape(3, -1).T
    bnd = m.flag2 > 0
    nrm = m.X2[bnd] / np.linalg.norm(m.X2[bnd], axis=1)[:, None]
    assert np.abs(np.einsum("ij,ij->i", U[bnd], nrm)).max() <= 1e-12 * np.abs(U).max()


def test_solve_from_an_initial_guess():
    """initial_guess = 1: FGMRES starts from the given (u, p).  From the
    converged solution the solve stops at once (0 iterations, same
    solution); from the solution of a slightly different right-hand side it
    converges in fewer iterations than from zero, to the same solution."""
    print("\n[solve from an initial guess]", flush=True)
    P = Pair("shell", 2, min_level=0, n_tan=1, n_rad=1)
    m = P.meshes[2]
    field = inputs.SHField(2)
    eta = inputs.viscosity_contrast(field.temperature(m.X1), 1e4)
    lnrho = inputs.ln_density(m.X1)
    T = field.temperature(m.X2)
    params = default_params(tol_rel=1e-10, precision=32)
    P.ctx.set_fields(P.p_to_lib(eta), P.p_to_lib(lnrho), params=params)
    f = P.ctx.rhs_buoyancy(P.s2_to_lib(T))
    u, p, rep = P.ctx.solve(f, params=params)
    u2, p2, rep2 = P.ctx.solve(f, params=params, u0=u, p0=p)
    print("from the solution:", rep2["iterations"], rep2["initial_residual"], rep2["abs_residual"])
    assert rep2["iterations"] == 0
    assert relerr(P.u_to_or(u2), P.u_to_or(u)) < 1e-14 and relerr(P.p_to_or(p2), P.p_to_or(p)) < 1e-14
    f2 = P.ctx.rhs_buoyancy(P.s2_to_lib(T + 0.01 * inputs.uniform(5, m.n2)))
    uc, pc, rc = P.ctx.solve(f2, params=params)
    uw, pw, rw = P.ctx.solve(f2, params=params, u0=u, p0=p)
    print("cold", rc["iterations"], "warm", rw["iterations"], relerr(P.u_to_or(uw), P.u_to_or(uc)))
    assert rw["iterations"] < rc["iterations"]
    # both stop at 1e-10 |b|: they agree within condition x residual, the bar
    # of the other solve tests' comparisons
    assert relerr(P.u_to_or(uw), P.u_to_or(uc)) < 1e-6 and relerr(P.p_to_or(pw), P.p_to_or(pc)) < 1e-6
