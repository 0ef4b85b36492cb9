"""GPU parity at the full benchmark size (icosahedral 10x2 shell, 12,000
macro-tets, level 4, N_u = 2.0e8) in the launch configuration the benchmark
times, on sampled outputs the oracle can compute on its own: the rows of A and
B at the nodes inside one macro-tet depend only on that macro's micro-tets, so
a one-macro oracle mesh reproduces them exactly.  The same holds for the fused
K and K^T rows, B^T + C^T, the prolongation at macro-interior fine nodes and
the restriction at macro-interior coarse nodes (a coarse P2 basis function
vanishes on every face that does not hold its node), and for one Chebyshev
step at nodes at least three micro-tet layers inside the macro (the step
reaches two layers).  Inputs are smooth functions of the node coordinates,
evaluated by each side at its own nodes.  Errors are per entry, against the
entry's own scale.  Also the symmetry of the projected A at full size.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch
from scipy.spatial import cKDTree

import inputs
from oracle.fem import assemble_A, assemble_B
from oracle.mesh import MacroMesh, RefinedMesh, shell_macros
from oracle.solvers import chebyshev, prolongation, vector_prolongation
from tests._util import rowerr

pytestmark = pytest.mark.gpu

L, NT, NR = 4, 10, 2


def _eta(X):
    return np.exp(1.5 * np.sin(3.0 * X[:, 0]) * np.cos(2.0 * X[:, 1]) + X[:, 2])


@pytest.fixture(scope="module")
def full():
    print("\n[full size: shell 10x2 level 4]", flush=True)
    from paper_2506_04157_amd import StokesContext
    sc = StokesContext("shell", level=L, min_level=0, n_tan=NT, n_rad=NR)
    X2, _ = sc.coords(which=2)
    X1, _ = sc.coords(which=1)
    sc.set_fields(torch.tensor(_eta(X1), device="cuda"), torch.tensor(inputs.ln_density(X1), device="cuda"))
    yield sc, X2, X1
    sc.close()


def _one_macro(mac_id, level=L):
    mm = shell_macros(NT, NR, 0.55, 1.0)
    t = mm.tets[mac_id]
    one = MacroMesh("shell", mm.vertices[t], [[0, 1, 2, 3]], mm.layer[t], 0.55, 1.0, NR)
    return RefinedMesh(one, level)


def _block_match(Xg, n_block, Xo):
    """Indices into Xg of the points Xo: the macro-interior nodes are numbered
    macro by macro, n_block per macro, so the block is found first."""
    nm = 60 * NT * NT * NR
    means = Xg[:nm * n_block].reshape(nm, n_block, 3).mean(axis=1)
    b = int(np.argmin(np.linalg.norm(means - Xo.mean(axis=0), axis=1)))
    d, j = cKDTree(Xg[b * n_block:(b + 1) * n_block]).query(Xo)
    assert d.max() < 1e-12, "macro-interior nodes not found"
    return b * n_block + j


@pytest.mark.parametrize("mac_id", [0, 5432, 11999])
def test_sampled_rows_of_A_and_B(full, mac_id):
    sc, X2, X1 = full
    m = _one_macro(mac_id)
    n2, n1 = m.n2, m.n1
    # macro-interior nodes of the one-macro mesh (all barycentric weights > 0)
    in2 = (m.keys2[:, 4:] > 0).all(axis=1)
    in1 = (m.keys1[:, 4:] > 0).all(axis=1)
    g2 = _block_match(X2, int(in2.sum()), m.X2[in2])
    g1 = _block_match(X1, int(in1.sum()), m.X1[in1])
    u_or = inputs.smooth_vector_field(7, m.X2).T.ravel()
    A = assemble_A(m, _eta(m.X1))
    B = assemble_B(m)
    # a smooth input makes A u and B u small differences of large terms, so
    # each row's error is measured against its scale sum_j |a_ij u_j|
    yA = (A @ u_or).reshape(3, n2)[:, in2]
    sA = (abs(A) @ abs(u_or)).reshape(3, n2)[:, in2]
    yB = (B @ u_or)[in1]
    sB = (abs(B) @ abs(u_or))[in1]
    N2 = len(X2)
    u = torch.tensor(inputs.smooth_vector_field(7, X2).T.ravel(), device="cuda")
    for dtype, tol in [(torch.float64, 1e-13), (torch.float32, 1e-5)]:
        y = sc.apply_A(u.to(dtype), bc=0).double().cpu().numpy().reshape(3, N2)[:, g2]
        err = np.abs(y - yA) / sA
        print(mac_id, dtype, err.max())
        assert err.max() <= tol, (mac_id, dtype)
    q = sc.apply_B(u, bc=0).cpu().numpy()[g1]
    assert (np.abs(q - yB) / sB).max() <= 1e-13


def test_projected_A_is_symmetric_at_full_size(full):
    sc, X2, X1 = full
    n = 3 * len(X2)
    x = torch.tensor(inputs.uniform(1, n), device="cuda")
    y = torch.tensor(inputs.uniform(2, n), device="cuda")
    xAy = torch.dot(x, sc.apply_A(y, bc=3)).item()
    yAx = torch.dot(y, sc.apply_A(x, bc=3)).item()
    assert abs(xAy - yAx) <= 1e-12 * abs(xAy)


def _interior(m, margin=1):
    """Masks of the P2 and P1 nodes whose barycentric lattice weights are all
    >= margin (P2 lattice units for the P2 nodes, P1 units for the P1 nodes)."""
    return (m.keys2[:, 4:] >= margin).all(axis=1), (m.keys1[:, 4:] >= margin).all(axis=1)


def _scalar(seed, X):
    return inputs.smooth_vector_field(seed, X)[:, 0].copy()


@pytest.mark.parametrize("mac_id", [0, 11999])
def test_sampled_rows_of_K_Kt_and_BtCt(full, mac_id):
    """Fused K = [[A, B^T], [B + C, 0]] and K^T (FP64; no projection) and
    B^T + C^T (FP64 and FP32) at the macro-interior rows."""
    sc, X2, X1 = full
    m = _one_macro(mac_id)
    in2, in1 = _interior(m)
    g2 = _block_match(X2, int(in2.sum()), m.X2[in2])
    g1 = _block_match(X1, int(in1.sum()), m.X1[in1])
    u_or = inputs.smooth_vector_field(7, m.X2).T.ravel()
    p_or = _scalar(8, m.X1)
    A = assemble_A(m, _eta(m.X1))
    B = assemble_B(m)
    C = assemble_B(m, inputs.ln_density(m.X1), only_C=True)
    aA, aB, aC = abs(A), abs(B), abs(C)
    au, ap = abs(u_or), abs(p_or)
    N2 = len(X2)
    u = torch.tensor(inputs.smooth_vector_field(7, X2).T.ravel(), device="cuda")
    p = torch.tensor(_scalar(8, X1), device="cuda")
    sel = lambda v: v.reshape(3, -1)[:, in2]
    for transpose in (False, True):
        yu, yp = sc.apply_K(u, p, transpose=transpose, bc=0)
        yu = yu.cpu().numpy().reshape(3, N2)[:, g2]
        yp = yp.cpu().numpy()[g1]
        if transpose:
            ru, rp = A @ u_or + (B + C).T @ p_or, B @ u_or
            su, sp_ = aA @ au + (aB + aC).T @ ap, aB @ au
        else:
            ru, rp = A @ u_or + B.T @ p_or, (B + C) @ u_or
            su, sp_ = aA @ au + aB.T @ ap, (aB + aC) @ au
        eu, ep = rowerr(yu, sel(ru), sel(su)), rowerr(yp, rp[in1], sp_[in1])
        print(mac_id, "K^T" if transpose else "K", eu, ep)
        assert eu <= 1e-13 and ep <= 1e-13
    ref, scale = sel((B + C).T @ p_or), sel((aB + aC).T @ ap)
    for dtype, tol in [(torch.float64, 1e-13), (torch.float32, 1e-5)]:
        y = sc.apply_Bt(p.to(dtype), with_Ct=True, bc=0).double().cpu().numpy().reshape(3, N2)[:, g2]
        e = rowerr(y, ref, scale)
        print(mac_id, "Bt+Ct", dtype, e)
        assert e <= tol


@pytest.mark.parametrize("mac_id", [0, 11999])
def test_sampled_fp32_transfers_at_full_size(full, mac_id):
    """The V-cycle's FP32 transfers between levels 3 and 4: x += P_v P e_c at
    macro-interior fine nodes and P_v P^T P_v (b - t) at macro-interior coarse
    nodes, against the one-macro prolongation matrix."""
    sc, X2, X1 = full
    X2c, _ = sc.coords(L - 1, 2)
    mf, mc = _one_macro(mac_id), _one_macro(mac_id, L - 1)
    Pro = vector_prolongation(prolongation(mc, mf))
    inf, _ = _interior(mf)
    inc, _ = _interior(mc)
    gf = _block_match(X2, int(inf.sum()), mf.X2[inf])
    gc = _block_match(X2c, int(inc.sum()), mc.X2[inc])
    f32 = lambda seed, X: torch.tensor(inputs.smooth_vector_field(seed, X).T.ravel(), dtype=torch.float32,
                                       device="cuda")
    orv = lambda seed, X: inputs.smooth_vector_field(seed, X).T.ravel()
    # prolongation with accumulation
    xs = sc.prolong(f32(9, X2c), L, add_to=f32(10, X2)).double().cpu().numpy().reshape(3, -1)[:, gf]
    ec, x0 = orv(9, mc.X2), orv(10, mf.X2)
    ref = (x0 + Pro @ ec).reshape(3, -1)[:, inf]
    scale = (abs(x0) + abs(Pro) @ abs(ec)).reshape(3, -1)[:, inf]
    e = rowerr(xs, ref, scale)
    print(mac_id, "prolong-add", e)
    assert e <= 2e-6
    # restriction of a difference
    rc = sc.restrict(f32(11, X2), L, minus=f32(12, X2)).double().cpu().numpy().reshape(3, -1)[:, gc]
    rf, tf = orv(11, mf.X2), orv(12, mf.X2)
    ref = (Pro.T @ (rf - tf)).reshape(3, -1)[:, inc]
    scale = (abs(Pro).T @ (abs(rf) + abs(tf))).reshape(3, -1)[:, inc]
    e = rowerr(rc, ref, scale)
    print(mac_id, "restrict-diff", e)
    assert e <= 2e-6


@pytest.mark.parametrize("mac_id", [5432])
def test_sampled_fp32_chebyshev_step_at_full_size(full, mac_id):
    """One FP32 Chebyshev step of degree 2 on level 4 with the context's own
    interval, at nodes at least three micro-tet layers inside one macro,
    against the oracle's smoother on the one-macro matrix."""
    sc, X2, X1 = full
    lo, hi = sc.cheb_bounds(L)
    m = _one_macro(mac_id)
    deep, _ = _interior(m, margin=6)
    g2 = _block_match(X2, int((m.keys2[:, 4:] > 0).all(axis=1).sum()), m.X2[deep])
    b = torch.tensor(inputs.smooth_vector_field(13, X2).T.ravel(), dtype=torch.float32, device="cuda")
    x = torch.tensor(inputs.smooth_vector_field(14, X2).T.ravel(), dtype=torch.float32, device="cuda")
    sc.smooth(b, x, level=L, degree=2, steps=1)
    xg = x.double().cpu().numpy().reshape(3, -1)[:, g2]
    A = assemble_A(m, _eta(m.X1))
    I = sp.identity(A.shape[0], format="csr")
    ref = chebyshev(A, 1.0 / A.diagonal(), I, inputs.smooth_vector_field(13, m.X2).T.ravel(),
                    inputs.smooth_vector_field(14, m.X2).T.ravel(), lo, hi, 2, 1).reshape(3, -1)[:, deep]
    e = np.abs(xg - ref).max() / np.abs(ref).max()
    print(mac_id, "chebyshev", int(deep.sum()), "nodes", e)
    assert e <= 1e-5


def test_mmoc_rigid_rotation_at_full_size(full):
    """The method of characteristics at full size (66.6 million P2 nodes):
    without velocity every node is its own departure point; for a
    rigid rotation about z the departure point of X is R(-w tau) X, and a
    function linear in the physical coordinates is evaluated there up to the
    blended P2 interpolation error (order h^3) of the velocity and of the
    function: a point located in a wrong micro-tet would be off by order h."""
    sc, X2, _ = full
    Xt = torch.tensor(X2, device="cuda")
    # elementwise (torch's matrix-vector product is not used at this size)
    lin = lambda Y: (0.7 * Y[:, 0] - 0.4 * Y[:, 1] + 1.1 * Y[:, 2] + 0.3).contiguous()
    F = lin(Xt)
    z = torch.zeros(3 * len(X2), dtype=torch.float64, device="cuda")
    got = sc.mmoc(F, z, z, 0.05)
    # exact up to the rounding of the inverse blending and of the barycentric
    # coordinates (node values about 2)
    assert (got - F).abs().max().item() < 2e-12
    w, tau = 1.0, 0.05
    u = torch.cat([-w * Xt[:, 1], w * Xt[:, 0], torch.zeros_like(Xt[:, 0])]).contiguous()
    got = sc.mmoc(F, u, u, tau)
    c, s = np.cos(-w * tau), np.sin(-w * tau)
    Xd = torch.stack([c * Xt[:, 0] - s * Xt[:, 1], s * Xt[:, 0] + c * Xt[:, 1], Xt[:, 2]], dim=1)
    err = (got - lin(Xd)).abs().max().item()
    moved = (F - lin(Xd)).abs().max().item()
    print(f"rotation: max error {err:.2e}, displacement effect {moved:.2e}")
    assert err < 2e-5 and moved > 1e-2


@pytest.mark.parametrize("mac_id", [0, 11999])
def test_sampled_rows_of_the_temperature_operators_at_full_size(full, mac_id):
    """The temperature step's operators at full size (66.6 million P2 nodes,
    the launch shape of the temperature study): the rows of L (advection in
    the system), of S (matrix-free and through the stored element matrices)
    and of the right-hand side at the nodes inside one macro-tet depend only
    on that macro's micro-tets, so the oracle's one-macro assembly
    reproduces them; smooth inputs evaluated by each side at its own nodes,
    errors per entry against the entry's scale."""
    from oracle.temperature import symmetric_part, temperature_system
    from paper_2506_04157_amd import temp_params
    sc, X2, X1 = full
    m = _one_macro(mac_id)
    in2 = (m.keys2[:, 4:] > 0).all(axis=1)
    g2 = _block_match(X2, int(in2.sum()), m.X2[in2])
    coef = dict(k=0.8, Pe=3.0, Cp=1.1, Di=0.4, alpha=1.3, H=0.7, Ra=30.0)
    tau1, tau0 = 0.02, 0.026
    f = lambda X: np.sin(2.0 * X[:, 0]) + X[:, 1] * X[:, 2]
    h = lambda X: np.cos(X[:, 0] + 2.0 * X[:, 2]) - 0.5 * X[:, 1]
    u_or = inputs.smooth_vector_field(7, m.X2).T.ravel()
    lnrho_or = inputs.ln_density(m.X1)
    eta_or = _eta(m.X1)
    Lo, bo = temperature_system(m, u_or, lnrho_or, eta_or, f(m.X2), h(m.X2), tau1, tau0, adv=1.0, **coef)
    So = symmetric_part(m, lnrho_or, tau1, tau0, k=coef["k"], Pe=coef["Pe"], Cp=coef["Cp"])
    x_or = f(m.X2)
    dev = "cuda"
    Xt = torch.tensor(X2, device=dev)
    X1t = torch.tensor(X1, device=dev)
    ft = lambda X: (torch.sin(2.0 * X[:, 0]) + X[:, 1] * X[:, 2]).contiguous()
    ht = lambda X: (torch.cos(X[:, 0] + 2.0 * X[:, 2]) - 0.5 * X[:, 1]).contiguous()
    u = torch.tensor(inputs.smooth_vector_field(7, X2).T.ravel(), device=dev)
    lnrho = torch.tensor(inputs.ln_density(X1), device=dev)
    eta = torch.tensor(_eta(X1), device=dev)
    prm = temp_params(tau1=tau1, tau0=tau0, adv=1.0, **coef)
    x = ft(Xt)
    checks = [("L", sc.temp_apply(x, prm, 0, u_star=u, lnrho=lnrho), Lo @ x_or, abs(Lo) @ np.abs(x_or)),
              ("S", sc.temp_apply(x, prm, 1, lnrho=lnrho), So @ x_or, abs(So) @ np.abs(x_or)),
              ("S stored", sc.temp_apply(x, prm, 3, lnrho=lnrho), So @ x_or, abs(So) @ np.abs(x_or))]
    for name, y, ref, scale in checks:
        err = np.abs(y.cpu().numpy()[g2] - ref[in2]) / scale[in2]
        print(mac_id, name, err.max())
        assert err.max() <= 1e-12, (mac_id, name)
    b = sc.temp_rhs(ft(Xt), ht(Xt), prm, u_star=u, lnrho=lnrho, eta=eta).cpu().numpy()[g2]
    z = np.zeros(m.n2)
    _, src = temperature_system(m, u_or, lnrho_or, eta_or, z, z, tau1, tau0, **coef)
    from oracle.fem import assemble_vector_mass
    from oracle.temperature import bdf2
    _, s0, sm = bdf2(tau1, tau0)
    Ma = abs(assemble_vector_mass(m, np.ones(m.n1))[:m.n2, :m.n2])
    scale = Ma @ (s0 * np.abs(f(m.X2)) + sm * np.abs(h(m.X2)) + np.max(np.abs(src) / (Ma @ np.ones(m.n2))))
    err = np.abs(b - bo[in2]) / scale[in2]
    print(mac_id, "rhs", err.max())
    assert err.max() <= 1e-12
    del Xt, X1t
