"""Assembled-matrix references of the solver components (Sec. 5.2).

Plain linear algebra on the oracle's sparse matrices, in FP64:

* ``chebyshev``       Jacobi-preconditioned Chebyshev smoother (Sec. 5.2.2:
                      m pre/post steps of a degree-d polynomial).  The paper
                      cites the method only; the recurrence used is Chebyshev
                      acceleration (Saad, Iterative Methods for Sparse Linear
                      Systems, Sec. 12.3) with the interval of D^-1 A given
                      as [lo, hi]; one "step of degree d" costs d products
                      with A (the first is the residual).
* ``prolongation``    canonical embedding of nested P2 spaces: the coarse basis
                      evaluated at the fine nodes' reference coordinates;
                      restriction is its transpose (Sec. 5.1 mentions both
                      operators and their projections but not their form).
* ``vcycle``          one GMG V-cycle with projections after prolongation and
                      before restriction (Sec. 5.2.2, Fig. ASolverStructure).
* ``pcg``             preconditioned CG stopped on a relative residual.
* ``bfbt``            the BFBT-type Schur approximation, eq. (schurV), with
                      caller-supplied inner operators.
* ``wbfbt``           the weighted BFBT, eq. (schurWBFBT), with its Poisson
                      replacements K_{1/sqrt eta}^-1 (caller-supplied).
* ``symmetric_uzawa``, ``inexact_uzawa``, ``adjoint_uzawa``  one step of
                      eqs. (SymmetricUzawaStep1), (InexactUzawaStep1) and
                      (AdjointInexactUzawaStep1) from zero (Sec. 5.2.1).
* ``fgmres``          right-preconditioned flexible GMRES (Saad 1993).
"""
import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .fem import p2_values


def chebyshev(A, Dinv, P, b, x, lo, hi, degree, steps):
    """``steps`` applications of the degree-``degree`` Chebyshev polynomial in
    P D^-1 P A for A x = b; P projects onto admissible vectors."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    x = x.copy()
    for _ in range(steps):
        r = P @ (b - A @ x)
        d = (P @ (Dinv * r)) / theta
        rho_old = 1.0 / sigma
        for k in range(1, degree + 1):
            x = x + d
            if k == degree:
                break
            r = r - P @ (A @ d)
            rho = 1.0 / (2.0 * sigma - rho_old)
            d = rho * rho_old * d + (2.0 * rho / delta) * (P @ (Dinv * r))
            rho_old = rho
    return x


def chebyshev_error_polynomial(lam, lo, hi, degree):
    """Closed form: T_d((hi+lo-2 lam)/(hi-lo)) / T_d((hi+lo)/(hi-lo))."""
    from numpy.polynomial import chebyshev as C
    c = np.zeros(degree + 1)
    c[-1] = 1.0
    return C.chebval((hi + lo - 2.0 * lam) / (hi - lo), c) / C.chebval((hi + lo) / (hi - lo), c)


def prolongation(coarse, fine):
    """Scalar P2 prolongation (n2_fine x n2_coarse): P[f, c] = phi_c(x~_f)."""
    return _embedding(coarse, fine.x2, coarse.e2, p2_values, coarse.n2)


def prolongation_p1(coarse, fine):
    """Scalar P1 prolongation (n1_fine x n1_coarse): P[f, c] = psi_c(x~_f), the
    nested P1 spaces of the Poisson multigrid in the weighted BFBT."""
    return _embedding(coarse, fine.x1, coarse.e1, lambda lam: lam, coarse.n1)


def _embedding(coarse, xf, enodes, basis, ncoarse):
    """Coarse basis functions (values by `basis` of the barycentric
    coordinates) evaluated at the reference points xf."""
    ev = coarse.ev                                              # (nec,4,3)
    T = np.stack([ev[:, 1] - ev[:, 0], ev[:, 2] - ev[:, 0], ev[:, 3] - ev[:, 0]], axis=2)
    Tinv = np.linalg.inv(T)
    cent = ev.mean(axis=1)
    tree = cKDTree(cent)
    k = min(40, len(cent))
    _, cand = tree.query(xf, k=k)
    cand = cand.reshape(len(xf), k)
    rows, cols, vals = [], [], []
    found = np.zeros(len(xf), dtype=bool)
    for j in range(k):
        todo = np.nonzero(~found)[0]
        if len(todo) == 0:
            break
        e = cand[todo, j]
        xi = np.einsum("nij,nj->ni", Tinv[e], xf[todo] - ev[e, 0])
        lam = np.concatenate([1.0 - xi.sum(1, keepdims=True), xi], axis=1)
        ok = np.all(lam >= -1e-12, axis=1)
        idx = todo[ok]
        if len(idx) == 0:
            continue
        N = basis(lam[ok])                                       # (n, nodes per element)
        found[idx] = True
        for a in range(N.shape[1]):
            rows.append(idx)
            cols.append(enodes[e[ok], a])
            vals.append(N[:, a])
    assert found.all(), "fine node outside the coarse mesh"
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    keep = np.abs(v) > 1e-14
    return sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(len(xf), ncoarse))


def vector_prolongation(Ps):
    return sp.block_diag([Ps, Ps, Ps], format="csr")


def vcycle(levels, l, b, coarse_solve, deg, steps):
    """One V-cycle on level l.  ``levels[l]`` holds A, Dinv, P (projector),
    lo, hi and, for l > 0, Pro (prolongation from l-1)."""
    L = levels[l]
    if l == 0:
        return coarse_solve(b)
    x = chebyshev(L["A"], L["Dinv"], L["P"], b, np.zeros_like(b), L["lo"], L["hi"], deg, steps)
    r = L["P"] @ (b - L["A"] @ x)
    bc = levels[l - 1]["P"] @ (L["Pro"].T @ r)
    ec = vcycle(levels, l - 1, bc, coarse_solve, deg, steps)
    x = x + L["P"] @ (L["Pro"] @ ec)
    x = chebyshev(L["A"], L["Dinv"], L["P"], b, x, L["lo"], L["hi"], deg, steps)
    return x


def pcg(apply_A, b, precond, tol, maxit=10000, x0=None):
    """Preconditioned CG; stops when |r| <= tol |b|.  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = apply_A(p)
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


def bfbt(r, B, Bt, A, Ahat_inv, solve_BAB):
    """eq. (schurV): S^-1 r = (B Ah^-1 B^T)^-1 (B Ah^-1 A Ah^-1 B^T) (B Ah^-1 B^T)^-1 r."""
    y = solve_BAB(r)
    y = B @ Ahat_inv(A @ Ahat_inv(Bt @ y))
    return solve_BAB(y)


def wbfbt(r, B, Bt, A, Ml_inv, Mr_inv, Kl_inv, Kr_inv):
    """The weighted BFBT of eq. schurWBFBT with the Poisson replacements and
    the scaled viscosities that follow it:
    S_w^-1 r = K_l^-1 (B M_l^-1 A M_r^-1 B^T) K_r^-1 r, with M the sqrt(eta)
    vector masses and K the 1/sqrt(eta) Poisson operators of eta_l, eta_r
    (caller-supplied inverses, constraints applied by the caller)."""
    y = Kr_inv(r)
    return Kl_inv(B @ Ml_inv(A @ Mr_inv(Bt @ y)))


def symmetric_uzawa(ru, rp, A, Bt, Bbar, Ahat_inv, Shat_inv, sigma, omega):
    """One step of eq. (SymmetricUzawaStep1) started from (u, p) = (0, 0)."""
    uh = sigma * Ahat_inv(ru)
    p = -omega * Shat_inv(rp - Bbar @ uh)
    u = uh + sigma * Ahat_inv(ru - A @ uh - Bt @ p)
    return u, p


def inexact_uzawa(ru, rp, Bbar, Ahat_inv, Shat_inv, sigma, omega):
    """One step of eq. (InexactUzawaStep1) from (0, 0): velocity first, then
    the pressure from the continuity residual of the new velocity."""
    u = sigma * Ahat_inv(ru)
    p = -omega * Shat_inv(rp - Bbar @ u)
    return u, p


def adjoint_uzawa(ru, rp, Bt, Ahat_inv, Shat_inv, sigma, omega):
    """One step of eq. (AdjointInexactUzawaStep1) from (0, 0): pressure first,
    then the velocity from the momentum residual of the new pressure."""
    p = -omega * Shat_inv(rp)
    u = sigma * Ahat_inv(ru - Bt @ p)
    return u, p


def fgmres(apply_K, b, precond, tol, restart=30, maxit=1000):
    """Right-preconditioned FGMRES; stops when |b - K x| <= tol |b|.

    Returns (x, iterations, residual history)."""
    n = len(b)
    x = np.zeros(n)
    nb = np.linalg.norm(b)
    hist = [1.0]
    it = 0
    while it < maxit:
        r = b - apply_K(x)
        beta = np.linalg.norm(r)
        if beta <= tol * nb:
            break
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        V[0] = r / beta
        g = np.zeros(restart + 1)
        g[0] = beta
        cs, sn = np.zeros(restart), np.zeros(restart)
        j_used = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = apply_K(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_used = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= tol * nb or it >= maxit:
                break
        y = np.linalg.solve(H[:j_used, :j_used], g[:j_used])
        x = x + Z[:j_used].T @ y
        if hist[-1] <= tol:
            break
    return x, it, hist
