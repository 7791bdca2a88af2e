"""Gaussian quadrature on simplices (the paper only says "Gaussian", Sec. 4.3).

Reading: conical-product (Stroud) Gauss-Jacobi rules with q = p+1 points
per collapsed direction.  Volume rules are exact to degree 2q-1 = 2p+1
(>= 2p, so the MGS inner products of Alg. 1 are exact); face rules likewise.

Reference simplex: vertices 0, e_1, ..., e_d.  In 2D the collapse is
  eta = (1+b)/2,  xi = (1+a)/2 (1-eta),
with a Gauss-Legendre and b Gauss-Jacobi(1,0); weight w_a w_b / 8.
In 3D
  zeta = (1+c)/2,  eta = (1+b)/2 (1-zeta),  xi = (1+a)/2 (1-eta-zeta),
with c Gauss-Jacobi(2,0); weight w_a w_b w_c / 64.  Weights sum to 1/d!.
"""

import numpy as np
from scipy.special import roots_jacobi


def gauss_jacobi(n, alpha, beta):
    """n-point Gauss-Jacobi rule on [-1, 1] for the weight (1-x)^a (1+x)^b."""
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, np.float64), np.asarray(w, np.float64)


def simplex_rule(dim, q):
    """Reference-simplex rule: points (nq, dim), weights (nq,) summing to 1/dim!."""
    a, wa = gauss_jacobi(q, 0.0, 0.0)
    b, wb = gauss_jacobi(q, 1.0, 0.0)
    if dim == 1:
        return ((1 + a) / 2)[:, None], wa / 2
    if dim == 2:
        B, A = np.meshgrid(b, a, indexing="ij")
        WB, WA = np.meshgrid(wb, wa, indexing="ij")
        eta = (1 + B) / 2
        xi = (1 + A) / 2 * (1 - eta)
        pts = np.stack([xi.ravel(), eta.ravel()], axis=-1)
        return pts, (WA * WB).ravel() / 8.0
    c, wc = gauss_jacobi(q, 2.0, 0.0)
    C, B, A = np.meshgrid(c, b, a, indexing="ij")
    WC, WB, WA = np.meshgrid(wc, wb, wa, indexing="ij")
    zeta = (1 + C) / 2
    eta = (1 + B) / 2 * (1 - zeta)
    xi = (1 + A) / 2 * (1 - eta - zeta)
    pts = np.stack([xi.ravel(), eta.ravel(), zeta.ravel()], axis=-1)
    return pts, (WA * WB * WC).ravel() / 64.0


def face_rule(dim, q):
    """Rule on a (dim-1)-simplex face in barycentric form.

    Returns mu (nfq, dim) (barycentric coordinates with respect to the
    face's ordered vertices C_0..C_{dim-1}) and weights (nfq,) summing to 1,
    so that the integral over a face of measure |f| is |f| * sum_r w_r g(x_r)
    with x_r = sum_j mu_rj C_j.
    """
    pts, w = simplex_rule(dim - 1, q)
    mu = np.concatenate([1.0 - pts.sum(axis=1, keepdims=True), pts], axis=1)
    return mu, w / w.sum()
