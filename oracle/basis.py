"""Orthonormal basis in global Cartesian coordinates (Sec. 4.3, eqs. (basis2),
(basis), Alg. 1 "Basis orthonormalization").

chi_i(x) = prod_a ((x_a - x_{c,a}) / L_a)^{p_a}, centred at the element
centroid and scaled by the half bounding-box extents.  Reading of the garbled
index set of eq. (basis2): all monomials of total degree <= p in graded
order; within a degree, descending power of x, then of y (2D: 1, x, y, x^2,
xy, y^2; 3D: 1, x, y, z, x^2, xy, xz, y^2, yz, z^2).

Reading of Alg. 1: modified Gram-Schmidt against the already orthonormal
psi_j (j < i), normalising once after the inner loop, which gives the form
psi_i = s_i (chi_i + sum_{j<i} c_ij chi_j) of eq. (basis) with s_i > 0.
The inner product <f, g>_E = int_E f g dx uses the volume quadrature, exact
for degree 2p.
"""

import numpy as np


def exponents(dim, p):
    out = []
    for deg in range(p + 1):
        if dim == 2:
            for a in range(deg, -1, -1):
                out.append((a, deg - a))
        else:
            for a in range(deg, -1, -1):
                for b in range(deg - a, -1, -1):
                    out.append((a, b, deg - a - b))
    return np.array(out, dtype=np.int64)


def n_basis(dim, p):
    return len(exponents(dim, p))


def monomials(x, xc, L, exps, grad=False):
    """chi at points.  x (n, npts, d); xc, L (n, d).  Returns (n, npts, N)
    and, with ``grad``, d chi / dx of shape (n, npts, N, d)."""
    z = (x - xc[:, None, :]) / L[:, None, :]
    n, npts, d = x.shape
    N = exps.shape[0]
    val = np.ones((n, npts, N), dtype=z.dtype)
    for i, e in enumerate(exps):
        for a in range(d):
            if e[a]:
                val[..., i] *= z[..., a] ** e[a]
    if not grad:
        return val
    g = np.zeros((n, npts, N, d), dtype=z.dtype)
    for i, e in enumerate(exps):
        for a in range(d):
            if e[a] == 0:
                continue
            t = e[a] * z[..., a] ** (e[a] - 1) / L[:, None, a]
            for b in range(d):
                if b != a and e[b]:
                    t = t * z[..., b] ** e[b]
            g[..., i, a] = t
    return val, g


def mgs_coefficients(gram):
    """Lower-triangular C with psi_i = sum_j C_ij chi_j orthonormal under ``gram``.

    gram (n, N, N) holds <chi_a, chi_b>_E.  Modified Gram-Schmidt: for each
    i, start from chi_i, subtract the projection on each orthonormal psi_j
    (j < i) in turn, then normalise.
    """
    n, N, _ = gram.shape
    C = np.zeros_like(gram)
    for i in range(N):
        c = np.zeros((n, N))
        c[:, i] = 1.0
        for j in range(i):
            w = np.einsum("ea,eab,eb->e", c, gram, C[:, j])
            c = c - w[:, None] * C[:, j]
        nrm = np.sqrt(np.einsum("ea,eab,eb->e", c, gram, c))
        C[:, i] = c / nrm[:, None]
    return C
