"""Analytic flow fields, seeded perturbations and random directions.

Fields are evaluated at points supplied by the caller (each side of the
comparison evaluates them at its own quadrature points).  Conserved
variables are ordered (rho, rho*u, rho*v, [rho*w], rho*E).
Non-dimensionalisation: rho_inf = 1, p_inf = 1, T = p / rho, c_inf = sqrt(gamma).
"""

import numpy as np

GAMMA = 1.4


def freestream_prim(dim, mach=0.5, angle_deg=45.0, gamma=GAMMA):
    """Primitive free stream (rho, u, v, [w], p) with rho = p = 1."""
    c = np.sqrt(gamma)
    speed = mach * c
    a = np.deg2rad(angle_deg)
    vel = [speed * np.cos(a), speed * np.sin(a)] + ([0.0] if dim == 3 else [])
    return np.array([1.0] + vel + [1.0], dtype=np.float64)


def prim_to_cons(prim, gamma=GAMMA):
    """(..., rho, vel..., p) -> (..., rho, rho*vel..., rho*E)."""
    prim = np.asarray(prim, dtype=np.float64)
    rho = prim[..., :1]
    vel = prim[..., 1:-1]
    p = prim[..., -1:]
    rhoE = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1, keepdims=True)
    return np.concatenate([rho, rho * vel, rhoE], axis=-1)


def uniform_state(points, prim, gamma=GAMMA):
    """Constant conserved state at every point: (n, dim) -> (n, dim+2)."""
    points = np.asarray(points)
    cons = prim_to_cons(prim, gamma)
    return np.broadcast_to(cons, points.shape[:-1] + cons.shape).copy()


def _wrap(d, period):
    if period is None:
        return d
    period = np.asarray(period, dtype=np.float64)
    out = d.copy()
    for a in range(min(d.shape[-1], period.shape[0])):
        if period[a] > 0:
            out[..., a] = d[..., a] - period[a] * np.round(d[..., a] / period[a])
    return out


def isentropic_vortex(points, t=0.0, center=(5.0, 5.0), period=None, strength=5.0,
                      uinf=None, gamma=GAMMA):
    """Isentropic vortex of strength ``strength`` advected by the free stream.

    In 2D (or as a column along z in 3D): r^2 = |x - x_v(t)|^2 in the xy-plane,
    du = -eps/(2 pi) (y - y_v) e^{(1-r^2)/2}, dv = eps/(2 pi) (x - x_v) e^{(1-r^2)/2},
    T = 1 - (gamma-1) eps^2 / (8 gamma pi^2) e^{1-r^2}, rho = T^{1/(gamma-1)},
    p = rho T.  The vortex centre moves with the free-stream velocity and is
    wrapped into the periodic box (nearest image).
    """
    points = np.asarray(points, dtype=np.float64)
    dim = points.shape[-1]
    if uinf is None:
        uinf = freestream_prim(dim)[1:-1]
    uinf = np.asarray(uinf, dtype=np.float64)
    xc = np.zeros(dim)
    xc[:2] = center[:2]
    xc = xc + uinf * t
    d = _wrap(points - xc, period)
    dx, dy = d[..., 0], d[..., 1]
    r2 = dx * dx + dy * dy
    eps = strength
    g = np.exp(0.5 * (1.0 - r2))
    du = -eps / (2.0 * np.pi) * dy * g
    dv = eps / (2.0 * np.pi) * dx * g
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * np.pi ** 2) * g * g
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    vel = np.zeros(points.shape[:-1] + (dim,))
    vel[..., 0] = uinf[0] + du
    vel[..., 1] = uinf[1] + dv
    if dim == 3:
        vel[..., 2] = uinf[2]
    prim = np.concatenate([rho[..., None], vel, p[..., None]], axis=-1)
    return prim_to_cons(prim, gamma)


def paper_vortex(points, t=0.0, beta=0.2, R=0.05, center=(0.05, 0.05), length=0.1,
                 mach=0.5, gamma=GAMMA):
    """The vortex of the paper's temporal-accuracy test in non-dimensional form.

    Velocity U0 = U(1 - beta (y-yc)/R e^{-r^2/2}), V0 = U beta (x-xc)/R e^{-r^2/2},
    with r = |x - x_c| / R; temperature chosen for radial equilibrium,
    T0 = T_inf - (beta U)^2 / (2 c_p) e^{-r^2} (c_p = gamma/(gamma-1) with
    R_gas = 1, T_inf = 1, rho_inf = 1); entropy is uniform.  The free stream
    is (U, 0) with U = mach * sqrt(gamma); the box is periodic with side ``length``.
    """
    points = np.asarray(points, dtype=np.float64)
    U = mach * np.sqrt(gamma)
    xc = np.array([center[0] + U * t, center[1]])
    d = _wrap(points[..., :2] - xc, np.array([length, length]))
    r2 = (d[..., 0] ** 2 + d[..., 1] ** 2) / R ** 2
    g = np.exp(-0.5 * r2)
    u = U * (1.0 - beta * d[..., 1] / R * g)
    v = U * beta * d[..., 0] / R * g
    cp = gamma / (gamma - 1.0)
    T = 1.0 - (beta * U) ** 2 / (2.0 * cp) * g * g
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    prim = np.stack([rho, u, v, p], axis=-1)
    return prim_to_cons(prim, gamma)


def perturbation(shape, seed, amplitude=1e-6):
    """Absolute i.i.d. U(-a, a) values (numpy PCG64 stream of ``seed``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amplitude, amplitude, size=shape)


def random_directions(n_dir, shape, seed, norm=1.0):
    """``n_dir`` N(0,1) arrays of ``shape``, each rescaled to 2-norm ``norm``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = rng.standard_normal(size=(n_dir,) + tuple(shape))
    for k in range(n_dir):
        out[k] *= norm / np.linalg.norm(out[k])
    return out


def random_unit_vector(shape, seed):
    """One N(0,1) array of ``shape`` rescaled to unit 2-norm."""
    return random_directions(1, shape, seed, 1.0)[0]
