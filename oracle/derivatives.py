"""Jacobian-vector products of the DG residual (Sec. 4.4 "Exact Jacobian").

The paper forms the exact Jacobian (eqs. (jac1), (jac2)) with automatic
differentiation of the Riemann flux.  The oracle obtains the same exact
directional derivative by the complex step (Squire & Trapp 1998):
J(u) v = Im R(u + i h v) / h with h = 1e-30, exact to rounding because R
is written with complex-safe abs/max.

The finite-difference Frechet derivative (R(u + eps v) - R(u)) / eps is not
part of the paper; it is the baseline JVP, with
eps = sqrt(2^-52) (1 + ||u||_2) / ||v||_2.
"""

import numpy as np

H_CS = 1e-30
EPS_MACH = 2.0 ** -52


def jvp_cs(op, u, v, h=H_CS):
    return np.imag(op.residual(u + 1j * h * v)) / h


def fd_epsilon(u, v):
    return np.sqrt(EPS_MACH) * (1.0 + np.linalg.norm(u)) / np.linalg.norm(v)


def jvp_fd(op, u, v, R_u=None):
    if R_u is None:
        R_u = op.residual(u)
    eps = fd_epsilon(u, v)
    return (op.residual(u + eps * v) - R_u) / eps


def dense_jacobian(op, u):
    """Dense J (K x K) column by column with the complex step (tiny meshes)."""
    shape = u.shape
    K = u.size
    J = np.zeros((K, K))
    e = np.zeros(K)
    for j in range(K):
        e[j] = 1.0
        J[:, j] = jvp_cs(op, u, e.reshape(shape)).reshape(-1)
        e[j] = 0.0
    return J


def vjp_dense(J, w):
    return (J.T @ w.reshape(-1)).reshape(w.shape)
