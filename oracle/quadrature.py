"""Gaussian quadrature on simplices (the paper only says "Gaussian", Sec. 4.3).

Reading: conical-product (Stroud) Gauss-Jacobi rules with q = p+1 points
per collapsed direction.  Volume rules are exact to degree 2q-1 = 2p+1
(>= 2p, so the MGS inner products of Alg. 1 are exact); face rules likewise.
For p = 2 in 3D the operator uses fully symmetric rules of the same degree
5 with fewer points instead (:func:`dg_rules`): 14 points on the
tetrahedron (27 conical) and Radon's 7 points on each triangular face (9).

Reference simplex: vertices 0, e_1, ..., e_d.  In 2D the collapse is
  eta = (1+b)/2,  xi = (1+a)/2 (1-eta),
with a Gauss-Legendre and b Gauss-Jacobi(1,0); weight w_a w_b / 8.
In 3D
  zeta = (1+c)/2,  eta = (1+b)/2 (1-zeta),  xi = (1+a)/2 (1-eta-zeta),
with c Gauss-Jacobi(2,0); weight w_a w_b w_c / 64.  Weights sum to 1/d!.
"""

import itertools
from math import factorial

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


def radon7():
    """Radon's 7-point rule on the triangle, exact to degree 5, in barycentric
    form: the centroid, weight 9/40, and the orbits of (a, a, 1 - 2a) for
    a = (6 - sqrt 15)/21 and (6 + sqrt 15)/21, weights (155 - sqrt 15)/1200
    and (155 + sqrt 15)/1200 (fractions of the area).  Order: centroid, then
    each orbit with 1 - 2a at barycentric index 0, 1, 2."""
    s = np.sqrt(15.0)
    bary = [[1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0]]
    w = [9.0 / 40.0]
    for a, wa in (((6.0 - s) / 21.0, (155.0 - s) / 1200.0), ((6.0 + s) / 21.0, (155.0 + s) / 1200.0)):
        for k in range(3):
            b = [a, a, a]
            b[k] = 1.0 - 2.0 * a
            bary.append(b)
            w.append(wa)
    return np.array(bary), np.array(w)


def _tet14_points(a1, a2, b):
    """Barycentric points (14, 4) of the orbits of (a, a, a, 1 - 3a) for
    a = a1, a2 (1 - 3a at index 0..3 in turn) and of (b, b, 1/2 - b, 1/2 - b)
    (b at the index pairs i < j in lexicographic order)."""
    bary = []
    for a in (a1, a2):
        for k in range(4):
            row = [a] * 4
            row[k] = 1.0 - 3.0 * a
            bary.append(row)
    for i in range(4):
        for j in range(i + 1, 4):
            row = [0.5 - b] * 4
            row[i] = b
            row[j] = b
            bary.append(row)
    return np.array(bary)


def _tet14_moments(x, exps, exact):
    a1, a2, b, w1, w2, w3 = x
    pts = _tet14_points(a1, a2, b)[:, 1:]
    w = np.array([w1] * 4 + [w2] * 4 + [w3] * 6)
    return np.array([np.sum(w * np.prod(pts ** e[None, :], axis=1)) for e in exps]) - exact


def tet14():
    """The 14-point fully symmetric rule on the reference tetrahedron, exact to
    degree 5 with positive weights: two orbits (a, a, a, 1 - 3a) of 4 points
    and the orbit (b, b, 1/2 - b, 1/2 - b) of 6, one weight per orbit.  The
    six parameters are the solution of the moment equations (every monomial
    of degree <= 5 integrated exactly, prod e_i! / (|e| + 3)!), found here by
    Gauss-Newton from rough starting values.  Returns barycentric points
    (14, 4) (order as in :func:`_tet14_points`) and weights summing to 1/6."""
    exps = [np.array(e) for e in itertools.product(range(6), repeat=3) if sum(e) <= 5]
    exact = np.array([np.prod([factorial(k) for k in e]) / factorial(int(sum(e)) + 3) for e in exps])
    x = np.array([0.09, 0.31, 0.05, 0.012, 0.019, 0.007])
    for _ in range(40):
        r = _tet14_moments(x, exps, exact)
        J = np.empty((len(r), 6))
        for k in range(6):
            h = 1e-7 * max(abs(x[k]), 1e-3)
            d = np.zeros(6)
            d[k] = h
            J[:, k] = (_tet14_moments(x + d, exps, exact) - _tet14_moments(x - d, exps, exact)) / (2 * h)
        dx = np.linalg.lstsq(J, -r, rcond=None)[0]
        x = x + dx
        if np.max(np.abs(dx)) < 1e-17:
            break
    a1, a2, b, w1, w2, w3 = x
    return _tet14_points(a1, a2, b), np.array([w1] * 4 + [w2] * 4 + [w3] * 6)


def dg_rules(dim, p):
    """Volume rule (points on the reference simplex, weights summing to
    1/dim!) and face rule (barycentric, weights summing to 1) of the DG
    operator of degree p: the symmetric degree-5 rules for dim = 3, p = 2,
    else the conical-product rules with p + 1 points per direction."""
    if dim == 3 and p == 2:
        bary, w = tet14()
        mu, wf = radon7()
        return bary[:, 1:].copy(), w, mu, wf
    pts, w = simplex_rule(dim, p + 1)
    mu, wf = face_rule(dim, p + 1)
    return pts, w, mu, wf
