"""Element-by-element assembly of the Stokes blocks (Sec. 5.1, FP64).

Definitions (Sec. 5.1, "Linear algebraic formulation"; stress tensor of Sec. 2):

* A_ij = int 2 eta [eps(phi_j) : eps(phi_i) - 1/3 div phi_j div phi_i] dx.
  The printed formula drops eta from the divergence term; the reading here
  keeps it, as follows from tau = 2 eta (sym grad u - div u I / 3), and it is
  the only reading for which A is positive semidefinite for all eta > 0.
* B_ij = - int div phi_j psi_i dx,   C_ij = - int (grad ln rho . phi_j) psi_i dx
* M_{1/eta, ij} = int psi_i psi_j / eta dx      (Sec. 5.2.3, Schur approximation)
* f_i = int T r_hat . phi_i dx                  (buoyancy with unit scaling)
* M_{sqrt eta}: the P2 vector mass with weight sqrt(s_K eta_h) and
  K_{1/sqrt eta}: the P1 Poisson (Neumann) matrix with weight
  (s_K eta_h)^{-1/2}, s_K = a^2 on the elements touching the Dirichlet
  boundary and 1 elsewhere (the weighted BFBT, eq. schurWBFBT and the
  scaled viscosities eta_l, eta_r that follow it)

eta, ln rho are P1 interpolants of nodal values, T is a P2 interpolant; on
the coarse levels up to l_eta the viscosity is instead evaluated at the
quadrature points from T (Sec. 5.2.2, ``assemble_A_qp``).
Integrals on a blended element K = B(F(K^)) are pulled back to the reference
tetrahedron with the Jacobian J = J_B(F(xi)) J_F and the weight
|det J_B| |det J_F| (Sec. 4.1).  Velocity DoFs are stored component-major:
dof (c, node) -> c * n2 + node.
"""
import numpy as np
import scipy.sparse as sp

from .quadrature import rule_q4, rule_stroud

# --- P2 / P1 shape functions in barycentric coordinates -------------------
EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
DLAM_DXI = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def p2_values(lam):
    """(nq, 10) values: vertices lambda_i (2 lambda_i - 1), edges 4 lambda_i lambda_j."""
    v = [lam[:, i] * (2.0 * lam[:, i] - 1.0) for i in range(4)]
    e = [4.0 * lam[:, i] * lam[:, j] for (i, j) in EDGES]
    return np.stack(v + e, axis=1)


def p2_grad_ref(lam):
    """(nq, 10, 3) gradients with respect to the reference coordinates xi."""
    nq = len(lam)
    dl = np.zeros((nq, 10, 4))
    for i in range(4):
        dl[:, i, i] = 4.0 * lam[:, i] - 1.0
    for k, (i, j) in enumerate(EDGES):
        dl[:, 4 + k, i] = 4.0 * lam[:, j]
        dl[:, 4 + k, j] = 4.0 * lam[:, i]
    return dl @ DLAM_DXI


def p1_values(lam):
    return lam.copy()


def p1_grad_ref(nq):
    return np.broadcast_to(DLAM_DXI, (nq, 4, 3)).copy()


# --- blending map ------------------------------------------------------------

def blend_jacobian(xt, g, s0):
    """Closed-form Jacobian of B(x) = s(x) x/|x|, s(x) = g.x + s0.

    With d = x/|x| and alpha = s/|x|:  J_B = d g^T + alpha (I - d d^T),
    det J_B = alpha^2 (g . d).  Shapes: xt (..., 3), g (..., 3), s0 (...).
    """
    r = np.linalg.norm(xt, axis=-1)
    d = xt / r[..., None]
    s = np.einsum("...k,...k->...", g, xt) + s0
    alpha = s / r
    I = np.eye(3)
    J = d[..., :, None] * g[..., None, :] + alpha[..., None, None] * (I - d[..., :, None] * d[..., None, :])
    return J


def blend_map(xt, g, s0):
    s = np.einsum("...k,...k->...", g, xt) + s0
    return xt * (s / np.linalg.norm(xt, axis=-1))[..., None]


# --- per-element geometry at quadrature points ------------------------------

def geometry(mesh, sel, rule=None):
    """Geometry of elements ``sel`` at the rule's points.

    Returns W (ne, nq) = w_q |det J|, G2 (ne, nq, 10, 3) physical P2 gradients,
    G1 (ne, nq, 4, 3) physical P1 gradients, X (ne, nq, 3) physical points,
    N2 (nq, 10), N1 (nq, 4).
    """
    xi, w, lam = rule if rule is not None else rule_q4()
    ev = mesh.ev[sel]                                             # (ne,4,3)
    JF = np.stack([ev[:, 1] - ev[:, 0], ev[:, 2] - ev[:, 0], ev[:, 3] - ev[:, 0]], axis=2)
    xt = ev[:, None, 0, :] + np.einsum("edk,qk->eqd", JF, xi)     # (ne,nq,3)
    nq = len(w)
    if mesh.blend_g is not None:
        m = mesh.emacro[sel]
        g = np.broadcast_to(mesh.blend_g[m][:, None, :], xt.shape)
        s0 = np.broadcast_to(mesh.blend_s0[m][:, None], xt.shape[:2])
        JB = blend_jacobian(xt, g, s0)
        X = blend_map(xt, g, s0)
        J = JB @ JF[:, None]
    else:
        J = np.broadcast_to(JF[:, None], (len(ev), nq, 3, 3))
        X = xt
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    W = np.abs(detJ) * w[None, :]
    # grad_x N = J^{-T} grad_xi N
    G2 = np.einsum("eqkd,qak->eqad", Jinv, p2_grad_ref(lam))
    G1 = np.einsum("eqkd,qak->eqad", Jinv, p1_grad_ref(nq))
    return W, G2, G1, X, p2_values(lam), p1_values(lam)


def _chunks(ne, size=16384):
    for s in range(0, ne, size):
        yield np.arange(s, min(ne, s + size))


def _vec_dofs(mesh, sel):
    """(ne, 30) velocity dof ids, ordered (comp, local node)."""
    n2 = mesh.n2
    e = mesh.e2[sel]
    return np.concatenate([e + c * n2 for c in range(3)], axis=1)


def strain_and_div(G2):
    """Strain tensors eps(phi_{c,a}) and divergences for all 30 vector basis
    functions phi_{c,a} = N_a e_c: eps_ij = (d_ic dN_a/dx_j + d_jc dN_a/dx_i)/2."""
    sh = G2.shape[:-2]
    I = np.eye(3)
    # grad phi_{c,a}: row c holds grad N_a  -> (.., c, a, i, j) = d_ic G_a[j]
    grad = np.einsum("ci,...aj->...caij", I, G2)
    eps = 0.5 * (grad + np.swapaxes(grad, -1, -2))
    div = np.einsum("...caii->...ca", grad)
    return eps.reshape(sh + (30, 3, 3)), div.reshape(sh + (30,))


def element_A(W, G2, eta_q):
    """(ne, 30, 30) element matrices of A with viscosity eta_q (ne, nq)."""
    eps, div = strain_and_div(G2)
    dev = np.einsum("eqaij,eqbij->eqab", eps, eps) - np.einsum("eqa,eqb->eqab", div, div) / 3.0
    return np.einsum("eq,eqab->eab", 2.0 * eta_q * W, dev)


def assemble_A(mesh, eta1, rule=None):
    n = 3 * mesh.n2
    rows, cols, vals = [], [], []
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        eta_q = np.einsum("qk,ek->eq", N1, eta1[mesh.e1[sel]])
        Ae = element_A(W, G2, eta_q)
        d = _vec_dofs(mesh, sel)
        rows.append(np.repeat(d, 30, axis=1).ravel())
        cols.append(np.tile(d, (1, 30)).ravel())
        vals.append(Ae.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def viscosity_model(x, T, eta_base, E_A, V_A, r_in, r_out):
    """Frank-Kamenetskii viscosity of the geodynamic model (Sec. 6, eq.
    ViscosityDef): eta(x, T) = eta_base(|x|) exp(-E_A T + V_A (r_out - |x|)).

    The radial base profile is known only from a figure; the reading here
    takes it as ``len(eta_base)`` samples on a uniform grid of [r_in, r_out],
    linear in between and constant outside."""
    r = np.linalg.norm(np.asarray(x), axis=-1)
    grid = np.linspace(r_in, r_out, len(eta_base))
    return np.interp(r, grid, eta_base) * np.exp(-E_A * np.asarray(T) + V_A * (r_out - r))


def vertex_p2_nodes(mesh):
    """P2 node of every P1 vertex (the element's first four P2 nodes are its
    vertices, in the order of its P1 nodes)."""
    v2 = np.empty(mesh.n1, dtype=np.int64)
    v2[mesh.e1.ravel()] = mesh.e2[:, :4].ravel()
    return v2


def assemble_A_qp(mesh, eta_fn, T2, rule=None):
    """A with the viscosity evaluated at the quadrature points from a P2
    temperature (Sec. 5.2.2, levels up to l_eta): eta_q = eta_fn(x_q, T_h(x_q)),
    x_q the physical quadrature point and T_h the P2 interpolant of T2."""
    n = 3 * mesh.n2
    rows, cols, vals = [], [], []
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        Tq = np.einsum("qa,ea->eq", N2, T2[mesh.e2[sel]])
        Ae = element_A(W, G2, eta_fn(X, Tq))
        d = _vec_dofs(mesh, sel)
        rows.append(np.repeat(d, 30, axis=1).ravel())
        cols.append(np.tile(d, (1, 30)).ravel())
        vals.append(Ae.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def assemble_B(mesh, lnrho1=None, rule=None, with_C=False, only_C=False):
    """B (div part) and/or C (compressibility part), shape (n1, 3 n2)."""
    rows, cols, vals = [], [], []
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        _, div = strain_and_div(G2)                                   # (ne,nq,30)
        Be = np.zeros((len(sel), 4, 30))
        if not only_C:
            Be -= np.einsum("eq,qi,eqa->eia", W, N1, div)
        if with_C or only_C:
            glr = np.einsum("eqkd,ek->eqd", G1, lnrho1[mesh.e1[sel]])  # grad ln rho_h
            # (grad ln rho . phi_{c,a}) = glr_c N_a
            gphi = np.einsum("eqc,qa->eqca", glr, N2).reshape(len(sel), len(W[0]), 30)
            Be -= np.einsum("eq,qi,eqa->eia", W, N1, gphi)
        d = _vec_dofs(mesh, sel)
        p = mesh.e1[sel]
        rows.append(np.repeat(p, 30, axis=1).ravel())
        cols.append(np.tile(d, (1, 4)).ravel())
        vals.append(Be.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh.n1, 3 * mesh.n2)).tocsr()


def assemble_M_inv_eta(mesh, eta1, rule=None):
    """P1 mass with weight 1/eta_h evaluated at the quadrature points."""
    rows, cols, vals = [], [], []
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        eta_q = np.einsum("qk,ek->eq", N1, eta1[mesh.e1[sel]])
        Me = np.einsum("eq,qi,qj->eij", W / eta_q, N1, N1)
        p = mesh.e1[sel]
        rows.append(np.repeat(p, 4, axis=1).ravel())
        cols.append(np.tile(p, (1, 4)).ravel())
        vals.append(Me.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh.n1, mesh.n1)).tocsr()


def dirichlet_element_scale(mesh, dirichlet_flags, a):
    """s_K of the weighted BFBT (eq. schurWBFBT): a^2 on the set D_eta of
    elements whose closure meets the Dirichlet boundary (a vertex on it is
    enough), 1 elsewhere."""
    on = np.isin(mesh.flag1, list(dirichlet_flags)) & (mesh.flag1 != 0)
    return np.where(on[mesh.e1].any(axis=1), a * a, 1.0)


def assemble_vector_mass(mesh, eta1, elem_scale=None, rule=None):
    """M_{sqrt eta}: (c, a), (c', b) entry delta_cc' int sqrt(s_K eta_h) N_a N_b dx
    (component-major velocity layout).  The P2 mass integrand has degree 4,
    so the default rule is the 27-point conical product (degree 5): the
    4-point rule of the Stokes blocks would make the element matrices rank 4
    and the mass singular."""
    rule = rule if rule is not None else rule_stroud(3)
    n2 = mesh.n2
    rows, cols, vals = [], [], []
    for sel in _chunks(mesh.ne, 4096):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        eta_q = np.einsum("qk,ek->eq", N1, eta1[mesh.e1[sel]])
        s_e = 1.0 if elem_scale is None else elem_scale[sel][:, None]
        Me = np.einsum("eq,qa,qb->eab", W * np.sqrt(s_e * eta_q), N2, N2)
        e = mesh.e2[sel]
        for c in range(3):
            d = e + c * n2
            rows.append(np.repeat(d, 10, axis=1).ravel())
            cols.append(np.tile(d, (1, 10)).ravel())
            vals.append(Me.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * n2, 3 * n2)).tocsr()


def assemble_poisson_p1(mesh, eta1, elem_scale=None, rule=None):
    """K_{1/sqrt eta}: int (s_K eta_h)^{-1/2} grad psi_i . grad psi_j dx on the P1
    space, with natural (Neumann) boundary conditions: constants span its
    kernel."""
    rows, cols, vals = [], [], []
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        eta_q = np.einsum("qk,ek->eq", N1, eta1[mesh.e1[sel]])
        s_e = 1.0 if elem_scale is None else elem_scale[sel][:, None]
        Ke = np.einsum("eq,eqid,eqjd->eij", W / np.sqrt(s_e * eta_q), G1, G1)
        p = mesh.e1[sel]
        rows.append(np.repeat(p, 4, axis=1).ravel())
        cols.append(np.tile(p, (1, 4)).ravel())
        vals.append(Ke.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh.n1, mesh.n1)).tocsr()


def rhs_buoyancy(mesh, T2, scale=1.0, rule=None):
    """f_{c,a} = int scale T_h (x/|x|)_c N_a dx, T_h the P2 interpolant."""
    f = np.zeros(3 * mesh.n2)
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        Tq = np.einsum("qa,ea->eq", N2, T2[mesh.e2[sel]])
        rhat = X / np.linalg.norm(X, axis=-1, keepdims=True)
        fe = scale * np.einsum("eq,eq,eqc,qa->eca", W, Tq, rhat, N2).reshape(len(sel), 30)
        np.add.at(f, _vec_dofs(mesh, sel).ravel(), fe.ravel())
    return f


def rhs_function(mesh, func, rule):
    """f_{c,a} = int func(x)_c N_a dx for a vector function of physical x."""
    f = np.zeros(3 * mesh.n2)
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        F = func(X.reshape(-1, 3)).reshape(X.shape)
        fe = np.einsum("eq,eqc,qa->eca", W, F, N2).reshape(len(sel), 30)
        np.add.at(f, _vec_dofs(mesh, sel).ravel(), fe.ravel())
    return f


def volume(mesh, rule=None):
    tot = 0.0
    for sel in _chunks(mesh.ne):
        W = geometry(mesh, sel, rule)[0]
        tot += W.sum()
    return tot


# --- error norms (degree >= 6 rule) -------------------------------------------

def error_norms(mesh, uh, ph, u_func, gradu_func, p_func, rule):
    """L2 and H1-seminorm errors of the P2 velocity and the L2 error of the P1
    pressure after shifting both pressures to zero integral mean."""
    n2 = mesh.n2
    U = uh.reshape(3, n2)
    eu2 = eg2 = 0.0
    pint = phint = vol = 0.0
    parts = []
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        Ue = U[:, mesh.e2[sel]]                                        # (3,ne,10)
        uq = np.einsum("cea,qa->eqc", Ue, N2)
        gq = np.einsum("cea,eqad->eqcd", Ue, G2)
        ue = u_func(X.reshape(-1, 3)).reshape(X.shape)
        ge = gradu_func(X.reshape(-1, 3)).reshape(X.shape + (3,))
        eu2 += np.einsum("eq,eqc->", W, (uq - ue) ** 2)
        eg2 += np.einsum("eq,eqcd->", W, (gq - ge) ** 2)
        pq = np.einsum("qk,ek->eq", N1, ph[mesh.e1[sel]])
        pe = p_func(X.reshape(-1, 3)).reshape(X.shape[:2])
        pint += (W * pe).sum()
        phint += (W * pq).sum()
        vol += W.sum()
        parts.append((W, pq, pe))
    ep2 = 0.0
    for W, pq, pe in parts:
        ep2 += (W * ((pq - phint / vol) - (pe - pint / vol)) ** 2).sum()
    return np.sqrt(eu2), np.sqrt(eg2), np.sqrt(ep2)
