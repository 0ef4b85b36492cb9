"""The temperature step (Sec. 3 and Sec. 6 of arXiv 2506.04157), FP64.

Test infrastructure: plain assembled matrices and a brute-force method of
characteristics that the GPU path is compared against.

* ``bdf2``                 the variable-step BDF2 weights s^{n+1}, s^n, s^{n-1}
                           of the difference quotient D[.] (Sec. 3).
* ``temperature_system``   the matrix and right-hand side of the discrete
                           advection-diffusion problem, eq. (WeakTemp), on the
                           P2 space of the blended mesh; Dirichlet values on
                           both spheres.
* ``locate`` / ``evaluate_p2``   point location in the blended mesh (every
                           element tried: the reference point of a physical
                           x in macro m is |x~| = (|x| - s0_m) / (g_m . d) along
                           d = x/|x|, the inverse of the blending map) and
                           evaluation of a P2 function there.
* ``mmoc``                 the modified method of characteristics (Sec. 3):
                           nodes traced backwards over one step with the
                           classical Runge-Kutta method along the velocity
                           linearly interpolated in time, and the field
                           evaluated at the departure points.

Readings (the paper is terse or garbled here):
* eq. (WeakTemp) prints the history terms int s^n T^n w - int s^{n-1} T^{n-1} w
  inside the factor tau^{n+1}; the BDF2 quotient D[T^{n+1}, T^n, T^{n-1}] /
  tau^{n+1} defined just before it puts them beside s^{n+1} T^{n+1}, without
  tau.  The quotient is followed: after multiplying by tau^{n+1} the history
  terms carry no tau.
* eq. (WeakTemp) and the strong form before it both print the advection term
  u* . grad T^{n+1} beside the BDF2 quotient of the traced values, while the
  text says the splitting step solves the energy equation without advection
  and the cost breakdown assigns the advection to the MMOC alone.  With the
  traced values the quotient already approximates the material derivative,
  so the printed term would count the advection twice; it is kept with a
  weight ``adv``, 0 by default (the splitting), 1 for the printed equation.
* the preconditioner's "symmetric mass and diffusion part" is
  s^{n+1} M + tau k / (Pe Cp) int grad T . grad w / rho: the symmetric half of
  the diffusion term (the term -w grad ln rho . grad T / rho is not symmetric).
* the shear heating is tau(u) : eps(u) = 2 eta (eps : eps - (div u)^2 / 3), the
  deviatoric stress of the Stokes blocks.
* the second history value composes the two tracing steps so that the
  characteristic through a node at t^{n+1} is followed back to t^n and then
  to t^{n-1}, as the definition T^(t^{n-1}, x) = T(t^{n-1}, X(t^{n+1}, t^{n-1}, x))
  requires: T^(n-1) = MMOC(MMOC(T^{n-1}, u^n, u^{n-1}, tau^n), u*^{n+1}, u^n,
  tau^{n+1}).  The printed formula nests the two steps the other way round,
  which agrees with the definition only for a velocity constant in time.
* departure points outside the shell are moved radially onto it (onto the
  cube by clamping the coordinates).
* Dirichlet values: T_in on the inner sphere (the whole boundary of the
  cube), T_out on the outer sphere.
"""
import numpy as np
import scipy.sparse as sp

from .fem import EDGES, _chunks, geometry, p2_values, strain_and_div
from .quadrature import rule_stroud


def bdf2(tau1, tau0):
    """(s^{n+1}, s^n, s^{n-1}) for the step tau1 = tau^{n+1} after tau0 = tau^n."""
    s1 = (2.0 * tau1 + tau0) / (tau1 + tau0)
    s0 = (tau1 + tau0) / tau0
    sm = tau1 * tau1 / (tau0 * (tau1 + tau0))
    return s1, s0, sm


def temperature_system(mesh, ustar, lnrho1, eta1, That_n, That_nm1, tau1, tau0, k=1.0, Pe=1.0, Cp=1.0, Di=0.0,
                       alpha=0.0, H=0.0, Ra=1.0, adv=0.0, rule=None):
    """LHS matrix L (n2 x n2) and right-hand side b of eq. (WeakTemp), before
    the Dirichlet rows are imposed:

      L_ij = int s^{n+1} phi_j phi_i
             + tau ( adv int (u* . grad phi_j) phi_i
                     + int k / (Pe Cp) grad phi_j . grad (phi_i / rho)
                     - int Di alpha / Cp phi_j (u* . g) phi_i ),      g = -r_hat
      b_i  = int (s^n That^n - s^{n-1} That^{n-1}) phi_i
             + tau ( int H / Cp phi_i + int Pe Di / (Ra rho Cp) tau(u*):eps(u*) phi_i )

    with rho = exp(ln rho_h), ln rho_h and eta_h the P1 interpolants of the
    nodal values, the P2 functions at the points of the 27-point rule."""
    rule = rule if rule is not None else rule_stroud(3)
    s1, s0, sm = bdf2(tau1, tau0)
    n2 = mesh.n2
    U = ustar.reshape(3, n2)
    rows, cols, vals = [], [], []
    b = np.zeros(n2)
    kap = k / (Pe * Cp)
    for sel in _chunks(mesh.ne, 4096):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        e2 = mesh.e2[sel]
        lr = np.einsum("qk,ek->eq", N1, lnrho1[mesh.e1[sel]])
        glr = np.einsum("eqkd,ek->eqd", G1, lnrho1[mesh.e1[sel]])      # grad ln rho_h
        rho = np.exp(lr)
        etaq = np.einsum("qk,ek->eq", N1, eta1[mesh.e1[sel]])
        uq = np.einsum("cea,qa->eqc", U[:, e2], N2)                      # u* at the points
        rhat = X / np.linalg.norm(X, axis=-1, keepdims=True)
        ug = -np.einsum("eqc,eqc->eq", uq, rhat)                         # u* . g
        mass = np.einsum("eq,qi,qj->eij", W, N2, N2)
        advm = np.einsum("eq,eqd,eqjd,qi->eij", W, uq, G2, N2)
        # grad(phi_i / rho) = (grad phi_i - phi_i grad ln rho) / rho
        dif = np.einsum("eq,eqid,eqjd->eij", W / rho, G2, G2) - np.einsum("eq,qi,eqd,eqjd->eij", W / rho, N2, glr, G2)
        adi = np.einsum("eq,eq,qi,qj->eij", W, ug, N2, N2)
        Le = s1 * mass + tau1 * (adv * advm + kap * dif - (Di * alpha / Cp) * adi)
        rows.append(np.repeat(e2, 10, axis=1).ravel())
        cols.append(np.tile(e2, (1, 10)).ravel())
        vals.append(Le.ravel())
        hist = np.einsum("qa,ea->eq", N2, s0 * That_n[e2] - sm * That_nm1[e2])
        # tau(u):eps(u) = 2 eta (eps:eps - (div u)^2 / 3) from the P2 velocity
        gradu = np.einsum("cea,eqad->eqcd", U[:, e2], G2)
        eps = 0.5 * (gradu + np.swapaxes(gradu, -1, -2))
        divu = np.einsum("eqcc->eq", gradu)
        shear = 2.0 * etaq * (np.einsum("eqcd,eqcd->eq", eps, eps) - divu ** 2 / 3.0)
        src = hist + tau1 * (H / Cp + Pe * Di / (Ra * rho * Cp) * shear)
        np.add.at(b, e2.ravel(), np.einsum("eq,eq,qi->ei", W, src, N2).ravel())
    L = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n2, n2)).tocsr()
    return L, b


def solve_dirichlet(L, b, dmask, Tdir):
    """T with T = Tdir on the Dirichlet nodes (dmask) and the other rows of
    L T = b, by a direct solve."""
    import scipy.sparse.linalg as spla
    free = ~dmask
    T = np.where(dmask, Tdir, 0.0)
    rhs = (b - L @ T)[free]
    T[free] = spla.spsolve(L[free][:, free].tocsc(), rhs)
    return T


# --- point location and evaluation in the blended mesh --------------------------

def _macro_vertices(mesh):
    tets = mesh.macro.tets
    return mesh.macro.vertices[tets]                              # (nm, 4, 3)


def _reference_points(mesh, X, macros):
    """Reference points x~ of the physical points X (n, 3) for each macro in
    `macros` (n, c, 3): the inverse of the blending map of that macro, along
    +X/|X| (NaN where that ray misses the macro's blending, i.e. |x~| <= 0);
    X itself on the cube."""
    if mesh.blend_g is None:
        return np.broadcast_to(X[:, None, :], (len(X), len(macros), 3))
    r = np.linalg.norm(X, axis=1)
    d = X / r[:, None]
    gd = d @ mesh.blend_g[macros].T                                 # (n, c)
    with np.errstate(divide="ignore", invalid="ignore"):
        rt = (r[:, None] - mesh.blend_s0[macros][None, :]) / gd
        rt = np.where(rt > 0.0, rt, np.nan)
        return rt[:, :, None] * d[:, None, :]


def _barycentric(verts, xt):
    """Barycentric coordinates (n, c, 4) of the points xt (n, c, 3) in the
    tetrahedra verts (c, 4, 3)."""
    T = np.stack([verts[:, 1] - verts[:, 0], verts[:, 2] - verts[:, 0], verts[:, 3] - verts[:, 0]], axis=2)
    xi = np.einsum("cij,ncj->nci", np.linalg.inv(T), xt - verts[None, :, 0, :])
    return np.concatenate([1.0 - xi.sum(-1, keepdims=True), xi], axis=-1)


def locate(mesh, X):
    """For physical points X (n, 3) inside the mesh: the element and the
    element-local barycentric coordinates (of the reference point).  Brute
    force in two stages: every macro-tet is tried, the reference point of x in
    macro m being x~ = |x~| d with |x~| = (|x| - s0_m) / (g_m . d) > 0 along
    d = x/|x| (x itself on the cube), and the macro whose smallest barycentric
    coordinate of x~ is largest wins; then every element of that macro is
    tried the same way."""
    X = np.asarray(X, dtype=np.float64)
    n = len(X)
    nm = mesh.macro.n_macros
    mverts = mesh.macro.vertices[mesh.macro.tets]                     # (nm, 4, 3)
    lam_m = _barycentric(mverts, _reference_points(mesh, X, np.arange(nm)))
    mn = np.nan_to_num(lam_m.min(-1), nan=-np.inf)
    best_mac = np.argmax(mn, axis=1)
    assert mn[np.arange(n), best_mac].min() > -1e-8, "point outside the mesh"
    ne_loc = mesh.ne // nm
    best_e = np.zeros(n, dtype=np.int64)
    best_l = np.zeros((n, 4))
    for mac in np.unique(best_mac):
        elems = np.arange(mac * ne_loc, (mac + 1) * ne_loc)
        allp = np.nonzero(best_mac == mac)[0]
        for pts in np.array_split(allp, max(1, len(allp) * ne_loc // 2 ** 20)):
            xt = _reference_points(mesh, X[pts], np.array([mac]))[:, 0, :]
            lam = _barycentric(mesh.ev[elems], np.broadcast_to(xt[:, None, :], (len(pts), ne_loc, 3)))
            j = np.argmax(lam.min(-1), axis=1)
            best_e[pts] = elems[j]
            best_l[pts] = lam[np.arange(len(pts)), j]
    assert best_l.min() > -1e-8, "point outside the mesh"
    return best_e, best_l


def evaluate_p2(mesh, F, X):
    """Values at physical points X of the P2 functions F (k, n2) (rows are
    fields) as an array (k, n)."""
    F = np.atleast_2d(F)
    e, lam = locate(mesh, X)
    N = p2_values(lam)                                            # (n, 10)
    return np.einsum("na,kna->kn", N, F[:, mesh.e2[e]])


def _clamp_to_shell(mesh, X):
    if mesh.blend_g is None:
        return np.clip(X, 0.0, 1.0)
    r = np.linalg.norm(X, axis=1)
    rc = np.clip(r, mesh.macro.r_in, mesh.macro.r_out)
    return X * (rc / r)[:, None]


def mmoc(mesh, F, u_new, u_old, tau):
    """The field F (n2) evaluated at the departure points of the P2 nodes:
    each node is traced backwards over [t - tau, t] with one step of the
    classical Runge-Kutta method along u(s) linearly interpolated between
    u_old at t - tau and u_new at t (Sec. 3), departure points moved onto the
    shell if they leave it."""
    n2 = mesh.n2

    def vel(X, theta):
        """u at the points X and time t - tau + theta tau."""
        uv = evaluate_p2(mesh, np.concatenate([theta * u_new.reshape(3, n2) + (1.0 - theta) * u_old.reshape(3, n2)]),
                         X)
        return uv.T

    X0 = mesh.X2
    k1 = vel(X0, 1.0)
    k2 = vel(_clamp_to_shell(mesh, X0 - 0.5 * tau * k1), 0.5)
    k3 = vel(_clamp_to_shell(mesh, X0 - 0.5 * tau * k2), 0.5)
    k4 = vel(_clamp_to_shell(mesh, X0 - tau * k3), 0.0)
    Xd = _clamp_to_shell(mesh, X0 - tau / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4))
    return evaluate_p2(mesh, F, Xd)[0]


def symmetric_part(mesh, lnrho1, tau1, tau0, k=1.0, Pe=1.0, Cp=1.0, rule=None):
    """The matrix the CG preconditioner solves with: s^{n+1} M + tau k / (Pe Cp)
    K_{1/rho}, K_{1/rho} the P2 stiffness matrix with weight 1/rho_h."""
    rule = rule if rule is not None else rule_stroud(3)
    s1, _, _ = bdf2(tau1, tau0)
    kap = k / (Pe * Cp)
    rows, cols, vals = [], [], []
    for sel in _chunks(mesh.ne, 4096):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        rho = np.exp(np.einsum("qk,ek->eq", N1, lnrho1[mesh.e1[sel]]))
        Le = s1 * np.einsum("eq,qi,qj->eij", W, N2, N2) + tau1 * kap * np.einsum("eq,eqid,eqjd->eij", W / rho, G2, G2)
        e2 = mesh.e2[sel]
        rows.append(np.repeat(e2, 10, axis=1).ravel())
        cols.append(np.tile(e2, (1, 10)).ravel())
        vals.append(Le.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh.n2, mesh.n2)).tocsr()


def dirichlet_values(mesh, T_in, T_out):
    """Mask of the Dirichlet nodes and their values (T_in on flag 1, T_out on
    flag 2)."""
    dmask = mesh.flag2 > 0
    return dmask, np.where(mesh.flag2 == 2, T_out, np.where(mesh.flag2 == 1, T_in, 0.0))


def temperature_step(mesh, T_n, T_nm1, u_n, u_nm1, lnrho1, eta1, tau1, tau0, T_in=1.0, T_out=0.0, **coef):
    """One step of the splitting scheme (Sec. 3): the extrapolated velocity
    u*^{n+1} = u^n + (u^n - u^{n-1}) tau^{n+1} / tau^n (eq. Extrapolation), the
    traced history values by the MMOC, and the Dirichlet solve of eq. (WeakTemp).
    eta1 is the viscosity at the extrapolated temperature, given by the caller.
    Returns T^{n+1}, That^n, That^{n-1} and u*."""
    ustar = u_n + (u_n - u_nm1) * (tau1 / tau0)
    That_n = mmoc(mesh, T_n, ustar, u_n, tau1)
    That_nm1 = mmoc(mesh, mmoc(mesh, T_nm1, u_n, u_nm1, tau0), ustar, u_n, tau1)
    L, b = temperature_system(mesh, ustar, lnrho1, eta1, That_n, That_nm1, tau1, tau0, **coef)
    dmask, Tdir = dirichlet_values(mesh, T_in, T_out)
    return solve_dirichlet(L, b, dmask, Tdir), That_n, That_nm1, ustar
