"""Quadrature rules on the reference tetrahedron {xi >= 0, xi1 + xi2 + xi3 <= 1}.

The paper does not state its rule (the operator generator picks it).  The
reading used for every operator on the path is the symmetric 4-point rule of
degree 2 (``rule_q4``): the lowest degree that keeps the optimal Taylor-Hood
rates, all weights positive, so A stays symmetric positive semidefinite.
``rule_stroud`` (Gauss-Jacobi conical product) is used only for error norms.
"""
import numpy as np
from scipy.special import roots_jacobi


def rule_q4():
    """Points: barycentric permutations of (a, b, b, b), a = (5+3 sqrt5)/20,
    b = (5 - sqrt5)/20; weights 1/24 each (sum = volume 1/6).

    Returns (xi (4,3), w (4,), lam (4,4)) with lam the barycentric coordinates
    (lambda_0 = 1 - sum xi).  Point q has the large coordinate a on vertex q.
    """
    a = (5.0 + 3.0 * 5.0 ** 0.5) / 20.0
    b = (5.0 - 5.0 ** 0.5) / 20.0
    lam = np.full((4, 4), b)
    np.fill_diagonal(lam, a)
    xi = lam[:, 1:].copy()
    w = np.full(4, 1.0 / 24.0)
    return xi, w, lam


def rule_stroud(k):
    """Conical-product rule with k Gauss-Jacobi points per collapsed direction,
    exact for polynomials of total degree 2k - 1 (Stroud 1971)."""
    def gj(alpha):
        x, w = roots_jacobi(k, alpha, 0.0)
        return (1.0 + x) / 2.0, w / 2.0 ** (alpha + 1)
    u1, w1 = gj(2.0)
    u2, w2 = gj(1.0)
    u3, w3 = gj(0.0)
    U1, U2, U3 = np.meshgrid(u1, u2, u3, indexing="ij")
    W = (w1[:, None, None] * w2[None, :, None] * w3[None, None, :])
    xi1 = U1
    xi2 = (1.0 - U1) * U2
    xi3 = (1.0 - U1) * (1.0 - U2) * U3
    xi = np.stack([xi1.ravel(), xi2.ravel(), xi3.ravel()], axis=1)
    w = W.ravel()
    lam = np.concatenate([1.0 - xi.sum(1, keepdims=True), xi], axis=1)
    return xi, w, lam
