"""Pins of the oracle's quadrature, basis, fluxes and DG residual against
closed forms, identities and special cases (Sec. 4)."""

from math import factorial

import numpy as np
import pytest

import workloads as W
from oracle import quadrature, basis, euler
from oracle.dg import DG

GAMMA = 1.4


# ------------------------------------------------------------- quadrature
def _exact_simplex_monomial(e):
    # int over the unit simplex of prod x_a^{e_a} = prod e_a! / (|e| + d)!
    return np.prod([factorial(k) for k in e]) / factorial(sum(e) + len(e))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_simplex_rule_exactness(dim, q):
    pts, w = quadrature.simplex_rule(dim, q)
    assert abs(w.sum() - 1.0 / factorial(dim)) < 1e-15
    deg = 2 * q - 1
    for tot in range(deg + 1):
        for e in basis.exponents(dim, tot):
            if sum(e) != tot:
                continue
            got = np.sum(w * np.prod(pts ** e[None, :], axis=1))
            assert abs(got - _exact_simplex_monomial(e)) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_face_rule_exactness(dim, q):
    mu, w = quadrature.face_rule(dim, q)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(mu.sum(axis=1), 1.0)
    # int over the unit (d-1)-simplex normalised to measure 1: (d-1)! prod e!/(|e|+d-1)!
    for tot in range(2 * q):
        for e in basis.exponents(dim - 1, tot) if dim == 3 else [(tot,)]:
            e = np.array(e)
            if e.sum() != tot:
                continue
            got = np.sum(w * np.prod(mu[:, 1:] ** e[None, :], axis=1))
            want = factorial(dim - 1) * np.prod([factorial(k) for k in e]) / factorial(tot + dim - 1)
            assert abs(got - want) < 1e-15


def _moment_errors(pts, w, deg):
    """Largest error of the rule over the monomials of each degree <= deg on
    the reference simplex (closed-form integrals)."""
    dim = pts.shape[1]
    errs = []
    for tot in range(deg + 1):
        e_tot = 0.0
        for e in basis.exponents(dim, tot):
            if sum(e) != tot:
                continue
            got = np.sum(w * np.prod(pts ** np.asarray(e)[None, :], axis=1))
            e_tot = max(e_tot, abs(got - _exact_simplex_monomial(e)))
        errs.append(e_tot)
    return errs


def test_symmetric_degree5_rules():
    """Radon's 7-point triangle rule and the 14-point tetrahedron rule: exact
    on every monomial of degree <= 5 and not on degree 6, positive weights,
    points strictly inside, and each orbit invariant under the vertex
    permutations."""
    bary, w = quadrature.radon7()
    assert bary.shape == (7, 3) and np.all(w > 0) and np.all(bary > 0)
    assert np.allclose(bary.sum(axis=1), 1.0, atol=1e-15)
    errs = _moment_errors(bary[:, 1:], w / 2.0, 6)
    assert max(errs[:6]) < 1e-16 and errs[6] > 1e-6
    bary, w = quadrature.tet14()
    assert bary.shape == (14, 4) and np.all(w > 0) and np.all(bary > 0)
    assert np.allclose(bary.sum(axis=1), 1.0, atol=1e-15)
    errs = _moment_errors(bary[:, 1:], w, 6)
    assert max(errs[:6]) < 2e-16 and errs[6] > 1e-7
    for perm in ([1, 0, 2, 3], [1, 2, 3, 0]):
        pb = bary[:, perm]
        for a in range(14):
            j = int(np.argmin(np.abs(bary - pb[a]).sum(axis=1)))
            assert np.abs(bary[j] - pb[a]).max() < 1e-15 and w[j] == w[a]


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_dg_rules_degree(dim, p):
    """The operator's rules integrate degree 2p + 1 exactly (degree 5 for
    p = 2; the 3D P2 volume rule has 14 points, its face rule 7)."""
    pts, w, mu, wf = quadrature.dg_rules(dim, p)
    assert max(_moment_errors(pts, w, 2 * p + 1)) < 1e-15
    assert abs(wf.sum() - 1.0) < 1e-15 and np.allclose(mu.sum(axis=1), 1.0, atol=1e-15)
    if dim == 3:
        ferr = max(_moment_errors(mu[:, 1:], wf / 2.0, 2 * p + 1))
    else:
        ferr = max(abs(np.sum(wf * mu[:, 1] ** k) - 1.0 / (k + 1)) for k in range(2 * p + 2))
    assert ferr < 1e-15
    if (dim, p) == (3, 2):
        assert len(w) == 14 and len(wf) == 7


# ------------------------------------------------------------------ basis
def _meshes():
    return [
        ("sq3", W.periodic_square(3, 10.0), 45.0),
        ("sq4j", W.periodic_square(4, 10.0, 0.15, 11), 45.0),
        ("cube3", W.periodic_cube(3, 10.0), 45.0),
        ("chan", W.channel_bump(8, 4, height=0.1, seed=5), 0.0),
        ("box3", W.box_cube(3, 10.0, 0.1, 7), 0.0),
    ]


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("name,m,ang", _meshes()[:3])
def test_basis_orthonormal(name, m, ang, p):
    g = DG(m, p, "lf")
    c = g._build(slice(0, g.nE))
    M = np.einsum("eq,eqi,eqj->eij", c.W, c.psi, c.psi)
    assert np.max(np.abs(M - np.eye(g.N))) < 1e-12
    # psi_1 = |E|^{-1/2}
    assert np.max(np.abs(c.psi[:, :, 0] * np.sqrt(g.mesh.vol)[:, None] - 1)) < 1e-13
    # lower triangular in chi with s_i > 0 (eq. (basis))
    assert np.all(np.abs(np.triu(g.C, 1)) == 0)
    assert np.all(np.diagonal(g.C, axis1=1, axis2=2) > 0)


def test_basis_monomial_order_invariance():
    """The projected field does not depend on the order of the monomials."""
    m = W.periodic_square(4, 10.0, 0.15, 7)
    g = DG(m, 2, "lf")
    f = lambda x: W.isentropic_vortex(x, center=(5.0, 5.0), period=m.period)
    u = g.project(f)
    U1 = g.evaluate(u)
    g2 = DG(m, 2, "lf")
    g2.exps = g2.exps[[0, 2, 1, 5, 4, 3]]
    from oracle.mesh import affine_map
    for s in g2._chunks():
        x = affine_map(g2.mesh, g2.ref_pts, s)
        Wt = g2._weights(s)
        chi = basis.monomials(x, g2.mesh.centroid[s], g2.mesh.half_ext[s], g2.exps)
        g2.C[s] = basis.mgs_coefficients(np.einsum("eq,eqa,eqb->eab", Wt, chi, chi))
    g2._cache = None
    U2 = g2.evaluate(g2.project(f))
    assert np.max(np.abs(U1 - U2)) < 1e-12


def test_mgs_equals_cholesky():
    """MGS of Alg. 1 (reading: against orthonormal psi_j) = inverse Cholesky factor."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 6, 6))
    G = A @ np.transpose(A, (0, 2, 1)) + 6 * np.eye(6)
    C = basis.mgs_coefficients(G)
    L = np.linalg.cholesky(G)
    assert np.allclose(C, np.linalg.inv(L), atol=1e-13)


# ------------------------------------------------------------------ fluxes
def _states(n, dim, seed=0):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    vel = rng.uniform(-1.0, 1.0, (n, dim))
    p = rng.uniform(0.5, 2.0, n)
    U = W.prim_to_cons(np.concatenate([rho[:, None], vel, p[:, None]], axis=1))
    nrm = rng.standard_normal((n, dim))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return U, nrm


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("flux", [euler.lax_friedrichs, euler.roe])
def test_flux_consistency_and_antisymmetry(dim, flux):
    UL, n = _states(200, dim, 1)
    UR, _ = _states(200, dim, 2)
    assert np.allclose(flux(UL, UL, n, GAMMA), euler.normal_flux(UL, n, GAMMA), atol=1e-13)
    assert np.allclose(flux(UL, UR, n, GAMMA), -flux(UR, UL, -n, GAMMA), atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_roe_property(dim):
    """Roe 1981: F(U_R).n - F(U_L).n = A(U~)(U_R - U_L) with A the exact flux
    Jacobian at the Roe-averaged state (built here from the physical flux)."""
    UL, n = _states(50, dim, 3)
    UR, _ = _states(50, dim, 4)
    rL, vL, pL = euler.primitives(UL, GAMMA)
    rR, vR, pR = euler.primitives(UR, GAMMA)
    HL, HR = (UL[:, -1] + pL) / rL, (UR[:, -1] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    ut = (sL[:, None] * vL + sR[:, None] * vR) / (sL + sR)[:, None]
    Ht = (sL * HL + sR * HR) / (sL + sR)
    rt = sL * sR
    Et = (Ht + (GAMMA - 1) * 0.5 * np.sum(ut * ut, 1)) / GAMMA
    Ut = np.concatenate([rt[:, None], rt[:, None] * ut, (rt * Et)[:, None]], 1)
    nv = dim + 2
    A = np.zeros((50, nv, nv))
    for j in range(nv):
        e = np.zeros(nv)
        e[j] = 1e-30
        A[:, :, j] = np.imag(euler.normal_flux(Ut + 1j * e, n, GAMMA)) / 1e-30
    lhs = euler.normal_flux(UR, n, GAMMA) - euler.normal_flux(UL, n, GAMMA)
    rhs = np.einsum("eij,ej->ei", A, UR - UL)
    assert np.allclose(lhs, rhs, atol=1e-12)


def test_roe_supersonic_upwinding():
    """All Roe wave speeds positive (negative) => F~ = F(U_L).n (F(U_R).n)."""
    dim = 2
    n = np.tile([1.0, 0.0], (20, 1))
    rng = np.random.default_rng(5)
    prim = lambda u: np.concatenate([rng.uniform(0.8, 1.2, (20, 1)), np.full((20, 1), u),
                                     rng.uniform(-0.2, 0.2, (20, 1)), rng.uniform(0.8, 1.2, (20, 1))], 1)
    UL, UR = W.prim_to_cons(prim(4.0)), W.prim_to_cons(prim(4.0))
    assert np.allclose(euler.roe(UL, UR, n, GAMMA), euler.normal_flux(UL, n, GAMMA), atol=1e-12)
    UL, UR = W.prim_to_cons(prim(-4.0)), W.prim_to_cons(prim(-4.0))
    assert np.allclose(euler.roe(UL, UR, n, GAMMA), euler.normal_flux(UR, n, GAMMA), atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_ghost_states(dim):
    UL, n = _states(30, dim, 8)
    G = euler.slip_wall_ghost(UL, n, GAMMA)
    # mirror: same density, energy, tangential momentum; reversed normal momentum
    assert np.allclose(G[:, 0], UL[:, 0]) and np.allclose(G[:, -1], UL[:, -1])
    mG, mL = G[:, 1:1 + dim], UL[:, 1:1 + dim]
    gn, ln = np.sum(mG * n, 1), np.sum(mL * n, 1)
    assert np.allclose(gn, -ln)
    assert np.allclose(mG - gn[:, None] * n, mL - ln[:, None] * n, atol=1e-13)
    # far field: the free stream is its own ghost
    prim = W.freestream_prim(dim, angle_deg=0.0)
    Uinf = np.tile(W.prim_to_cons(prim), (30, 1))
    assert np.allclose(euler.farfield_ghost(Uinf, n, prim, GAMMA), Uinf, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_lf_dissipation_is_max_wave_speed(dim):
    """The local Lax-Friedrichs dissipation coefficient recovered from the flux,
    (1/2)(F_L + F_R).n - F~ = (alpha/2)(U_R - U_L) in every component, equals
    the largest |eigenvalue| of the exact flux Jacobians at U_L and U_R
    (complex-step Jacobian, numpy eigenvalues)."""
    UL, n = _states(40, dim, 11)
    UR, _ = _states(40, dim, 12)
    D = 0.5 * (euler.normal_flux(UL, n, GAMMA) + euler.normal_flux(UR, n, GAMMA)) \
        - euler.lax_friedrichs(UL, UR, n, GAMMA)
    alpha = 2.0 * D / (UR - UL)
    assert np.allclose(alpha, alpha[:, :1], rtol=1e-9)
    nv = dim + 2

    def max_speed(U):
        A = np.zeros((len(U), nv, nv))
        for j in range(nv):
            e = np.zeros(nv)
            e[j] = 1e-30
            A[:, :, j] = np.imag(euler.normal_flux(U + 1j * e, n, GAMMA)) / 1e-30
        return np.max(np.abs(np.linalg.eigvals(A)), axis=1)

    want = np.maximum(max_speed(UL), max_speed(UR))
    assert np.allclose(alpha[:, 0], want, rtol=1e-10)


def _prims(U):
    rho = U[:, 0]
    v = U[:, 1:-1] / rho[:, None]
    p = (GAMMA - 1.0) * (U[:, -1] - 0.5 * rho * np.sum(v * v, 1))
    return rho, v, p


@pytest.mark.parametrize("dim", [2, 3])
def test_farfield_characteristics(dim):
    """Riemann-invariant far field, checked on the ghost state it returns:
    for subsonic normal flow the ghost carries the interior's outgoing
    invariant v.n + 2c/(g-1) and the free stream's incoming one
    v.n - 2c/(g-1), and the entropy p/rho^g and tangential velocity of the
    upwind side (interior if the ghost's v.n >= 0); supersonic outflow returns
    the interior state, supersonic inflow the free stream."""
    rng = np.random.default_rng(21)
    N = 60
    n = rng.standard_normal((N, dim))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    rho = rng.uniform(0.7, 1.4, N)
    p = rng.uniform(0.7, 1.4, N)
    c = np.sqrt(GAMMA * p / rho)
    t = rng.standard_normal((N, dim))
    t -= np.sum(t * n, 1)[:, None] * n
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    vn = rng.uniform(-0.8, 0.8, N) * c
    v = vn[:, None] * n + rng.uniform(-0.5, 0.5, (N, 1)) * t
    UL = W.prim_to_cons(np.concatenate([rho[:, None], v, p[:, None]], 1))
    prim = W.freestream_prim(dim, mach=0.5, angle_deg=30.0)
    G = euler.farfield_ghost(UL, n, prim, GAMMA)
    rb, vb, pb = _prims(G)
    cb = np.sqrt(GAMMA * pb / rb)
    vnb = np.sum(vb * n, 1)
    vinf = np.asarray(prim[1:-1])
    cinf = np.sqrt(GAMMA * prim[-1] / prim[0])
    vninf = n @ vinf
    assert np.allclose(vnb + 2 * cb / (GAMMA - 1), vn + 2 * c / (GAMMA - 1), atol=1e-12)
    assert np.allclose(vnb - 2 * cb / (GAMMA - 1), vninf - 2 * cinf / (GAMMA - 1), atol=1e-12)
    out = vnb >= 0
    assert 5 < out.sum() < N - 5
    s_up = np.where(out, p / rho ** GAMMA, prim[-1] / prim[0] ** GAMMA)
    assert np.allclose(pb / rb ** GAMMA, s_up, rtol=1e-12)
    vt_up = np.where(out[:, None], v - vn[:, None] * n, vinf - vninf[:, None] * n)
    assert np.allclose(vb - vnb[:, None] * n, vt_up, atol=1e-12)
    # supersonic outflow and inflow
    for sgn, want in ((1.5, UL), (-1.5, np.tile(W.prim_to_cons(prim), (N, 1)))):
        vs = (sgn * c)[:, None] * n
        US = W.prim_to_cons(np.concatenate([rho[:, None], vs, p[:, None]], 1))
        GS = euler.farfield_ghost(US, n, prim, GAMMA)
        assert np.allclose(GS, US if sgn > 0 else want, atol=1e-13)


def test_appendix_flux_jacobian():
    """Appendix eq. (dfdu) at omega = 0 with a_1 = gamma E - a_0 (= H; the printed
    'gamma e' is an erratum): grad(psi).dF/dU against the complex-step derivative."""
    dim = 3
    U, _ = _states(40, dim, 9)
    g = np.random.default_rng(10).standard_normal((40, dim))
    g1 = 1.4
    rho, vel, p = euler.primitives(U, g1)
    u, v, w = vel.T
    E = U[:, -1] / rho
    a0 = 0.5 * (g1 - 1) * (u * u + v * v + w * w)
    a1 = g1 * E - a0
    a2, a3 = g1 - 1, g1 - 2
    px, py, pz = g.T
    B1 = u * px + v * py + w * pz
    B2 = 0.0
    M = np.zeros((40, 5, 5))
    M[:, 0] = np.stack([-B2 + 0 * u, px, py, pz, 0 * u], 1)
    M[:, 1] = np.stack([a0 * px - B1 * u, B1 - B2 - a3 * u * px, u * py - a2 * v * px, u * pz - a2 * w * px, a2 * px], 1)
    M[:, 2] = np.stack([a0 * py - B1 * v, v * px - a2 * u * py, B1 - B2 - a3 * v * py, v * pz - a2 * w * py, a2 * py], 1)
    M[:, 3] = np.stack([a0 * pz - B1 * w, w * px - a2 * u * pz, w * py - a2 * v * pz, B1 - B2 - a3 * w * pz, a2 * pz], 1)
    M[:, 4] = np.stack([(a0 - a1) * B1, a1 * px - a2 * B1 * u, a1 * py - a2 * v * B1, a1 * pz - a2 * B1 * w, g1 * B1 - B2], 1)
    A = np.zeros((40, 5, 5))
    for j in range(5):
        e = np.zeros(5)
        e[j] = 1e-30
        A[:, :, j] = np.imag(np.einsum("ekd,ed->ek", euler.physical_flux(U + 1j * e, g1), g)) / 1e-30
    assert np.allclose(A, M, atol=1e-12)


# --------------------------------------------------------------- residual
@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("flux", ["lf", "roe"])
@pytest.mark.parametrize("name,m,ang", _meshes())
def test_free_stream_preservation(name, m, ang, flux, p):
    if name == "chan":
        m = W.channel_bump(8, 4, height=0.0, seed=5)   # flat walls: the free stream is exact
    prim = W.freestream_prim(m.dim, angle_deg=ang)
    g = DG(m, p, flux, farfield_prim=prim)
    u = g.project(lambda x: W.uniform_state(x, prim))
    R = g.residual(u)
    Fscale = np.max(np.abs(W.prim_to_cons(prim))) * np.max(g.mesh.area) / np.sqrt(np.min(g.mesh.vol))
    assert np.max(np.abs(R)) < 1e-13 * Fscale


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("flux", ["lf", "roe"])
@pytest.mark.parametrize("name,m,ang", _meshes()[:3])
def test_discrete_conservation(name, m, ang, flux, p):
    """Periodic domain: sum_E |E|^{1/2} R_{E,k,1} = 0 (the totals are invariant;
    this is also why J is singular, Sec. 2.2)."""
    g = DG(m, p, flux)
    u = g.project(lambda x: W.isentropic_vortex(x, center=(5.0, 5.0), period=m.period))
    u += W.perturbation(u.shape, 3, 1e-3)
    R = g.residual(u)
    tot = np.sum(np.sqrt(g.mesh.vol)[:, None] * R[:, :, 0], axis=0)
    assert np.max(np.abs(tot)) < 1e-12 * np.sum(np.abs(np.sqrt(g.mesh.vol)[:, None] * R[:, :, 0]))


@pytest.mark.parametrize("flux", ["lf", "roe"])
def test_p0_is_finite_volume(flux):
    """p = 0: R_E = -|E|^{-1/2} sum_f |f| F~(U_E, U_N, n_f) (first-order FV)."""
    m = W.periodic_square(4, 10.0, 0.15, 21)
    g = DG(m, 0, flux)
    rng = np.random.default_rng(1)
    Ucell = W.prim_to_cons(np.concatenate([rng.uniform(0.8, 1.2, (g.nE, 1)), rng.uniform(-.3, .3, (g.nE, 2)),
                                           rng.uniform(0.8, 1.2, (g.nE, 1))], 1))
    u = (Ucell * np.sqrt(g.mesh.vol)[:, None])[:, :, None]
    R = g.residual(u)[:, :, 0]
    fl = euler.lax_friedrichs if flux == "lf" else euler.roe
    want = np.zeros_like(Ucell)
    for f in range(3):
        want -= g.mesh.area[:, f, None] * fl(Ucell, Ucell[g.mesh.nbr[:, f]], g.mesh.normal[:, f], GAMMA)
    want /= np.sqrt(g.mesh.vol)[:, None]
    assert np.allclose(R, want, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2])
def test_residual_consistency_order(p):
    """For the translating vortex U(x,t), R(Pi U) approximates Pi dU/dt; the
    error ||R(Pi U) - Pi dU/dt||_2 falls at least like h^p."""
    errs = []
    for n in (16, 32, 64):
        m = W.periodic_square(n, 10.0)
        g = DG(m, p, "roe")
        f = lambda x, t=0.0: W.isentropic_vortex(x, t=t, center=(5.0, 5.0), period=m.period)
        u = g.project(f)
        dt = 1e-5
        dudt = (g.project(lambda x: f(x, dt)) - g.project(lambda x: f(x, -dt))) / (2 * dt)
        errs.append(np.linalg.norm(g.residual(u) - dudt))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p - 0.3) and rates[-1] > p - 0.1, (errs, rates)


@pytest.mark.parametrize("p", [1, 2])
def test_projection_convergence(p):
    """L2 projection error of the smooth vortex converges at order p+1."""
    errs = []
    for n in (16, 32, 64):
        m = W.periodic_square(n, 10.0)
        g = DG(m, p, "lf")
        f = lambda x: W.isentropic_vortex(x, center=(5.0, 5.0), period=m.period)
        from oracle.diagnostics import l2_error
        errs.append(l2_error(g, g.project(f), f))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p + 1 - 0.1), (errs, rates)
