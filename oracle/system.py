"""Constrained saddle-point system and its direct solve (Sec. 5.1).

The inner system eq. (InnerSaddlePointSystem) is the block system restricted
to non-Dirichlet velocities, with the free-slip projection P_v and the
pressure projection P_p applied on both sides.  Its solution in range(P) is
computed here as the solution of a square nonsingular system:

* Dirichlet velocity DoFs take prescribed values u_D (block row
  modification, eq. SaddlePointStructureDirichlet); they move to the
  right-hand side as f - A u_D and g - Bbar u_D.
* at free-slip nodes the velocity is written in an orthonormal tangential
  basis Q_i = [t1, t2], t_k perpendicular to the exact sphere normal x/|x|
  (this is range(P_v), u.n = 0);
* the pressure has arithmetic mean zero (how P_p is implemented, Sec. 5.1);
  a scalar multiplier mu absorbs the constant part of the continuity
  residual that P_p removes.

    [ Q^T A Q   Q^T B^T  0 ] [u~]   [ Q^T (f - A u_D) ]
    [ Bbar Q    0        1 ] [p ] = [ g - Bbar u_D    ]
    [ 0         1^T      0 ] [mu]   [ 0               ]

* with free slip on both spheres (the boundary conditions of Sec. 2 with
  the surface condition also of free-slip type) the rigid rotations
  e_k x X are admissible and strain free, so the problem does not determine
  them (on the blended mesh A annihilates them only up to the discretisation
  error).  They are removed as the pressure constant is: the nodal velocity
  is Euclidean-orthogonal to the three rotation vectors R (R^T u = 0), and
  three more multipliers nu absorb the rotational part of the momentum
  residual (columns Q^T R in the first block row, rows R^T Q below).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def tangent_basis(n):
    """Two orthonormal vectors perpendicular to each unit normal in n (k, 3)."""
    a = np.where(np.abs(n[:, [0]]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(n, a)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n, t1)
    return t1, t2


def velocity_basis(mesh, dirichlet_flags, freeslip_flags):
    """Sparse Q (3 n2 x n_free): columns span the admissible velocities."""
    n2 = mesh.n2
    flag = mesh.flag2
    dir_mask = np.isin(flag, list(dirichlet_flags)) & (flag != 0)
    fs_mask = np.isin(flag, list(freeslip_flags)) & (flag != 0) & ~dir_mask
    free = ~dir_mask & ~fs_mask
    rows, cols, vals = [], [], []
    col = 0
    idx = np.nonzero(free)[0]
    for c in range(3):
        rows.append(c * n2 + idx)
        cols.append(col + np.arange(len(idx)))
        vals.append(np.ones(len(idx)))
        col += len(idx)
    idx = np.nonzero(fs_mask)[0]
    nrm = mesh.X2[idx] / np.linalg.norm(mesh.X2[idx], axis=1, keepdims=True)
    t1, t2 = tangent_basis(nrm)
    for t in (t1, t2):
        for c in range(3):
            rows.append(c * n2 + idx)
            cols.append(col + np.arange(len(idx)))
            vals.append(t[:, c])
        col += len(idx)
    Q = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(3 * n2, col)).tocsr()
    dmask3 = np.tile(dir_mask, 3)
    return Q, dmask3, fs_mask


def projector(mesh, dirichlet_flags, freeslip_flags):
    """Dense-free application of P (velocity part): zero Dirichlet DoFs,
    remove the normal component at free-slip nodes."""
    Q, dmask3, fs = velocity_basis(mesh, dirichlet_flags, freeslip_flags)
    return Q @ Q.T


def rigid_rotations(mesh):
    """The rigid rotations e_k x X at the P2 nodes, k = 0, 1, 2, as the
    columns of a (3 n2, 3) array in the component-major velocity layout."""
    X = mesh.X2
    R = np.zeros((3 * mesh.n2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        R[:, k] = np.cross(e, X).T.ravel()
    return R


def solve_stokes(A, Bbar, f, g, Q, u_D=None, Bt=None, rotations=None):
    """Direct solve of the constrained system; returns (u, p, mu).

    Bt (optional) is the matrix of the gradient block; by default Bbar^T is
    not used: the gradient block is B^T with B = Bbar - C supplied by caller.
    rotations (optional, (3 n2, k)): velocity modes the solution is made
    Euclidean-orthogonal to, each with a multiplier (the rigid rotations
    under free slip on both spheres).
    """
    n1 = Bbar.shape[0]
    if u_D is None:
        u_D = np.zeros(A.shape[0])
    if Bt is None:
        raise ValueError("pass the gradient block Bt = B^T explicitly")
    QAQ = (Q.T @ A @ Q).tocsr()
    QBt = (Q.T @ Bt).tocsr()
    BQ = (Bbar @ Q).tocsr()
    nu = Q.shape[1]
    # The border (the column 1 for mu and the row 1^T for the mean) is dense,
    # which ruins a sparse LU.  Factor instead K0' = K0 + e e^T, with K0 the
    # square saddle-point block and e a unit vector on one pressure DoF, and
    # eliminate the border and the rank-one shift with three solves
    # (bordering / Sherman-Morrison).
    k = nu
    E = sp.csr_matrix(([1.0], ([k], [k])), shape=(nu + n1, nu + n1))
    K0 = sp.bmat([[QAQ, QBt], [BQ, None]], format="csc")
    lu = spla.splu((K0 + E).tocsc())
    b = np.concatenate([Q.T @ (f - A @ u_D), g - Bbar @ u_D])
    e = np.zeros(nu + n1)
    e[k] = 1.0
    # border columns: the pressure mean (c), then the constrained velocity modes
    W = [np.concatenate([np.zeros(nu), np.ones(n1)])]
    if rotations is not None:
        QR = Q.T @ rotations
        W += [np.concatenate([QR[:, j], np.zeros(n1)]) for j in range(QR.shape[1])]
    W = np.array(W).T                                   # (nu + n1, nw)
    ye = lu.solve(e)
    YW = np.column_stack([lu.solve(W[:, j]) for j in range(W.shape[1])])
    # (K0 + e e^T) x - t e + W lam = rm with t = e^T x and W^T x = rb:
    # x = yb + t ye - YW lam; unknowns z = (t, lam)
    cols = np.column_stack([ye, -YW])
    rows = np.vstack([W.T, e])
    Mz = rows @ cols
    Mz[-1, 0] -= 1.0

    def bordered(rm, rb):
        yb = lu.solve(rm)
        z = np.linalg.solve(Mz, np.concatenate([rb, [0.0]]) - rows @ yb)
        return yb + cols @ z, z

    sol, z = bordered(b, np.zeros(W.shape[1]))
    # one step of iterative refinement on K0 x + W lam = b, W^T x = 0: the
    # factorised matrix is nearly singular when rotations are constrained
    dx, dz = bordered(b - (K0 @ sol + W @ z[1:]), -(W.T @ sol))
    sol, z = sol + dx, z + dz
    mu = z[1]
    u = Q @ sol[:nu] + u_D
    p = sol[nu:nu + n1]
    return u, p, mu


def residual(A, Bt, Bbar, u, p, f, g, Pu):
    """Projected residual [P_u (f - A u - Bt p); P_p (g - Bbar u)] (u_D already
    contained in u, rows of Dirichlet DoFs zeroed by Pu)."""
    ru = Pu @ (f - A @ u - Bt @ p)
    rp = g - Bbar @ u
    rp = rp - rp.mean()
    return ru, rp
