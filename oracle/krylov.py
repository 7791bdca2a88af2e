"""Krylov evaluation of phi_k(dt J) b (Sec. 2.2, eqs. (vm), (vm1), (vm2),
(evv), (final1), (final)).

Arnoldi: v_1 = b/||b||, J V_m = V_{m+1} Htilde_m, H_m = V_m^T J V_m.  The
paper does not name its Gram-Schmidt variant; the oracle uses modified
Gram-Schmidt (as in Saad 1992, which the paper cites).  Breakdown: if
h_{j+1,j} <= eta ||J v_j|| the iteration stops with m_eff = j.

phi_k(dt J) b ~= ||b|| V_m phi_k(dt H_m) e_1.  Eq. (final) writes
phi_1(dt H_m) with H_m^{-1}, which fails for singular H_m (the paper notes J
is singular with periodic boundaries); reading: phi_k(dt H_m) e_1 is taken
from the exponential of the augmented matrix
   [[dt H_m, e_1, 0], [0, 0, I_{k-1}], [0, 0, 0]]
(Saad 1992, Sidje 1998), whose top-right block column equals
phi_k(dt H_m) e_1 and which agrees with eq. (final) whenever H_m is
invertible.  The small exponential is scipy.linalg.expm (the paper's
Chebyshev rational approximation is one of several FP64-accurate choices).
"""

import numpy as np
from scipy.linalg import expm


def _norm(x):
    # sqrt(sum x^2) without conjugation, so that complex-step perturbations pass through
    return np.sqrt(np.sum(x * x))


def arnoldi_mgs(matvec, b, m, eta=1e-12):
    """Returns (V (K, m_eff+1), H (m_eff+1, m_eff), beta, m_eff, breakdown)."""
    b = np.asarray(b).reshape(-1)
    dt = np.result_type(b, np.float64)
    K = b.size
    beta = _norm(b)
    V = np.zeros((K, m + 1), dtype=dt)
    H = np.zeros((m + 1, m), dtype=dt)
    if np.real(beta) == 0.0:
        return V[:, :1], H[:1, :0], beta, 0, True
    V[:, 0] = b / beta
    for j in range(m):
        w = np.asarray(matvec(V[:, j])).reshape(-1)
        if np.iscomplexobj(w) and not np.iscomplexobj(V):
            V = V.astype(np.complex128)
            H = H.astype(np.complex128)
        wn = _norm(w)
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = _norm(w)
        if np.real(H[j + 1, j]) <= eta * np.real(wn):
            return V[:, :j + 2], H[:j + 2, :j + 1], beta, j + 1, True
        V[:, j + 1] = w / H[j + 1, j]
    return V, H, beta, m, False


def phi_augmented(A, k):
    """phi_k(A) e_1 from expm of the augmented matrix (k >= 1); k = 0: expm(A) e_1."""
    n = A.shape[0]
    if k == 0:
        return expm(A)[:, 0]
    M = np.zeros((n + k, n + k), dtype=A.dtype)
    M[:n, :n] = A
    M[0, n] = 1.0
    for j in range(1, k):
        M[n + j - 1, n + j] = 1.0
    return expm(M)[:n, n + k - 1]


def arnoldi_phi(matvec, b, dt, k, m, eta=1e-12, return_info=False):
    """phi_k(dt J) b (no dt prefactor) by the Krylov projection of dimension m."""
    shape = np.shape(b)
    V, H, beta, meff, brk = arnoldi_mgs(matvec, b, m, eta)
    if meff == 0:
        out = np.zeros(shape, dtype=V.dtype)
    else:
        y = phi_augmented(dt * H[:meff, :meff], k)
        out = (beta * (V[:, :meff] @ y)).reshape(shape)
    if return_info:
        return out, dict(beta=beta, m_eff=meff, breakdown=brk,
                         h_last=H[meff, meff - 1] if meff > 0 else 0.0)
    return out


def dense_phi(A, b, dt, k):
    """phi_k(dt A) b for a dense A: expm of [[dt A, b, 0], [0, 0, I_{k-1}], [0, 0, 0]]."""
    A = np.asarray(A)
    b = np.asarray(b).reshape(-1)
    n = A.shape[0]
    if k == 0:
        return expm(dt * A) @ b
    M = np.zeros((n + k, n + k), dtype=np.result_type(A, b))
    M[:n, :n] = dt * A
    M[:n, n] = b
    for j in range(1, k):
        M[n + j - 1, n + j] = 1.0
    return expm(M)[:n, n + k - 1]


def phi1_with_error(H, beta, h_next, dt):
    """phi_1(dt H) e_1 and the a-posteriori relative error estimate of the
    Krylov approximation of phi_1 (Saad 1992): the leading error term of
    beta V phi_1(dt H) e_1 is beta dt h_{m+1,m} [phi_2(dt H) e_1]_m v_{m+1}, so
    err = dt h_{m+1,m} |[phi_2(dt H) e_1]_m| / |phi_1(dt H) e_1|.
    Both functions from the exponential of the augmented matrix with k = 2."""
    m = H.shape[0]
    M = np.zeros((m + 2, m + 2), dtype=H.dtype)
    M[:m, :m] = dt * H
    M[0, m] = 1.0
    M[m, m + 1] = 1.0
    E = expm(M)
    p1 = E[:m, m]
    p2 = E[:m, m + 1]
    n1 = np.sqrt(np.sum(np.real(p1) ** 2))
    err = float(dt * abs(np.real(h_next)) * abs(np.real(p2[m - 1])) / n1) if n1 > 0 else 0.0
    return p1, err


def adaptive_dimension(H, beta, meff, dt, tol, check_every):
    """Adaptive Krylov dimension (the Krylov tolerance of Sec. 5 read as a
    stopping rule): the smallest j with j % check_every == 0 and
    1 <= j < meff whose error estimate (phi1_with_error, with h_{j+1,j} of
    the Arnoldi relation) at dt is <= tol; meff when there is none.  The
    first j columns of an Arnoldi process do not depend on later iterations,
    so checking the finished relation equals stopping the process at j.
    Returns (m_eff, stopped)."""
    if check_every <= 0:
        return meff, False
    for j in range(check_every, meff, check_every):
        _, err = phi1_with_error(H[:j, :j], beta, H[j, j - 1], dt)
        if err <= tol:
            return j, True
    return meff, False


def arnoldi_phi1_controlled(matvec, b, dt, m, tol, eta=1e-12, max_halvings=40, check_every=0,
                            dt_control=True):
    """dt * phi_1(dt J) b with the Krylov tolerance: the dimension is first
    chosen by adaptive_dimension (check_every > 0), then, if dt_control, dt
    is halved until the error estimate is <= tol.
    Returns (x, dt_used, err, halvings, info)."""
    shape = np.shape(b)
    V, H, beta, meff, brk = arnoldi_mgs(matvec, b, m, eta)
    if meff == 0:
        return np.zeros(shape), dt, 0.0, 0, dict(m_eff=0)
    meff, stopped = adaptive_dimension(H, beta, meff, dt, tol, check_every)
    if stopped:
        brk = False
    h_next = 0.0 if brk else H[meff, meff - 1]
    halv = 0
    while True:
        y, err = phi1_with_error(H[:meff, :meff], beta, h_next, dt)
        if not dt_control or err <= tol or halv >= max_halvings:
            break
        dt *= 0.5
        halv += 1
    x = dt * (beta * (V[:, :meff] @ y)).reshape(shape)
    return x, dt, err, halv, dict(m_eff=meff, breakdown=brk)
