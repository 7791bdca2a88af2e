"""Pins of the stiff stretched-mesh vortex workload (Sec. 5.1, the paper's
second temporal-accuracy test): the clustered mesh against the spacings the
paper prints, the vortex against radial equilibrium, and the oracle's DG
operator on the stretched mesh against free-stream preservation."""

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG

GAMMA = 1.4


def test_stretched_mesh_spacing_matches_paper():
    """x_j = (1 - xi^3)/2 x_L + (1 + xi^3)/2 x_R, j = 1..N+1, N = 24 on [0, 0.1]:
    the paper prints a minimal spacing of 3e-5 and a maximal one of 0.0115
    (closed forms 0.05 (1/12)^3 and 0.05 (1 - (11/12)^3)); the mesh is
    periodic, symmetric about the centre and clustered there."""
    m = W.stretched_square(24, 0.1)
    x = np.unique(np.round(m.vert[:, 0], 15))
    assert x.size == 25 and abs(x[0]) < 1e-18 and abs(x[-1] - 0.1) < 1e-15
    dx = np.diff(x)
    assert abs(dx.min() - 0.05 / 12 ** 3) < 1e-15 and abs(dx.min() - 3e-5) < 0.5e-5
    assert abs(dx.max() - 0.05 * (1 - (11 / 12) ** 3)) < 1e-15 and abs(dx.max() - 0.0115) < 0.5e-4
    assert np.allclose(dx, dx[::-1], rtol=0, atol=1e-15)
    assert np.argmin(dx) in (11, 12)
    y = np.unique(np.round(m.vert[:, 1], 15))
    assert np.allclose(x, y, rtol=0, atol=1e-15)
    assert m.n_elem == 2 * 24 * 24


def test_paper_vortex_radial_equilibrium():
    """In the frame moving with the free stream the vortex is a steady Euler
    solution: uniform entropy and dp/dr = rho v_theta^2 / r (central
    differences of the closed-form fields along rays)."""
    U = 0.5 * np.sqrt(GAMMA)
    for ang in (0.3, 1.9, 4.0):
        r = np.linspace(0.004, 0.045, 60)
        h = 1e-7
        def fields(rr):
            pts = np.stack([0.05 + rr * np.cos(ang), 0.05 + rr * np.sin(ang)], axis=-1)
            q = W.paper_vortex(pts)
            rho = q[:, 0]
            u = q[:, 1] / rho - U
            v = q[:, 2] / rho
            p = (GAMMA - 1) * (q[:, 3] - 0.5 * rho * (u * u + v * v + 2 * U * u + U * U))
            vth = -u * np.sin(ang) + v * np.cos(ang)
            vr = u * np.cos(ang) + v * np.sin(ang)
            return rho, p, vth, vr
        rho, p, vth, vr = fields(r)
        assert np.max(np.abs(vr)) < 1e-12 * U
        s = p / rho ** GAMMA
        assert np.max(np.abs(s / s[0] - 1)) < 1e-12
        dpdr = (fields(r + h)[1] - fields(r - h)[1]) / (2 * h)
        rhs = rho * vth ** 2 / r
        assert np.max(np.abs(dpdr - rhs)) < 1e-6 * np.max(np.abs(rhs))


@pytest.mark.parametrize("p", [1, 2])
def test_free_stream_preserved_on_stretched_mesh(p):
    """Aspect ratios up to ~400 do not spoil free-stream preservation: the
    residual of the uniform state stays at rounding level (about 5e-13 here),
    far below that of the vortex on the same mesh (0.18)."""
    m = W.stretched_square(6, 0.1)
    g = DG(m, p, "roe")
    prim = W.freestream_prim(2, angle_deg=0.0)
    u = g.project(lambda x: W.uniform_state(x, prim))
    R = g.residual(u)
    assert np.max(np.abs(R)) < 1e-11
