"""Assembled adjoint gradient of J = 1/2 |u - u_obs|^2.

Parametrisation: eta_h = sum_k exp(m_k) psi_k (P1 interpolant of the nodal
viscosity, as the viscosity is represented in Sec. 5.2.2), so
d eta_h / d m_k = eta_k psi_k.  The temperature enters through the buoyancy
right-hand side f = int T_h r_hat . phi only.

With K^T lambda = dJ/d(u, p) solved in the same constrained form as the
forward problem (K^T swaps B and Bbar), the gradients are

    dJ/dm_k = - lambda_u^T (dA/dm_k) u,      dJ/dT_k = lambda_u^T (df/dT_k),

where dA/dm_k is assembled element by element from the element matrices of A
with the weight eta_k psi_k in place of eta_h.
"""
import numpy as np

from .fem import _chunks, _vec_dofs, element_A, geometry


def grad_log_eta(mesh, eta1, u, lam, rule=None):
    g = np.zeros(mesh.n1)
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        d = _vec_dofs(mesh, sel)
        ue, le = u[d], lam[d]
        ek = eta1[mesh.e1[sel]]                                   # (ne,4)
        for k in range(4):
            eta_q = ek[:, k:k + 1] * N1[None, :, k]               # eta_k psi_k(q)
            Ak = element_A(W, G2, eta_q)
            val = -np.einsum("ea,eab,eb->e", le, Ak, ue)
            np.add.at(g, mesh.e1[sel][:, k], val)
    return g


def grad_temperature(mesh, lam, scale=1.0, rule=None):
    g = np.zeros(mesh.n2)
    n2 = mesh.n2
    for sel in _chunks(mesh.ne):
        W, G2, G1, X, N2, N1 = geometry(mesh, sel, rule)
        rhat = X / np.linalg.norm(X, axis=-1, keepdims=True)
        le = lam[_vec_dofs(mesh, sel)].reshape(len(sel), 3, 10)   # (ne,c,a)
        lq = np.einsum("eca,qa->eqc", le, N2)                      # lambda_h(q)
        s = scale * np.einsum("eq,eqc,eqc->eq", W, rhat, lq)
        val = np.einsum("eq,qk->ek", s, N2)
        np.add.at(g, mesh.e2[sel].ravel(), val.ravel())
    return g
