"""Pseudo-time iteration of Sec. 5 in the oracle (eq. (cfl) ramp, eq. (x3d) dt)."""

import numpy as np
import pytest

import workloads as W
from oracle.dg import DG
from oracle.integrators import ExactJacobian, steady_iterations, res_rho_norm, cfl_ramp
from tests.helpers import mesh_case, vortex_state


def test_free_stream_is_a_fixed_point():
    m, _ = mesh_case("chan_flat")
    prim = W.freestream_prim(2, angle_deg=0.0)
    g = DG(m, 1, "roe", farfield_prim=prim)
    u = g.project(lambda x: W.uniform_state(x, prim))
    u1, hist = steady_iterations(g, ExactJacobian(g), u, 2, 1000.0, 10)
    assert hist[0] < 1e-13
    assert np.max(np.abs(u1 - u)) < 1e-12


@pytest.mark.slow
def test_channel_converges_below_1e10():
    """P1 Roe on the 12x4 bump channel from the perturbed free stream: with
    m = 30 and CFL_max = 1000 the rho residual norm falls below 1e-10 within
    60 iterations and the ramp is at CFL_max from the start (r^-3 > 1000)."""
    m, _ = mesh_case("chan")
    prim = W.freestream_prim(2, angle_deg=0.0)
    g = DG(m, 1, "roe", farfield_prim=prim)
    u = vortex_state(g, m, 1e-3)
    r0 = res_rho_norm(g, g.residual(u))
    assert cfl_ramp(1, r0, 1, 1000.0) == 1000.0
    u1, hist = steady_iterations(g, ExactJacobian(g), u, 60, 1000.0, 30)
    assert min(hist) < 1e-10
    assert res_rho_norm(g, g.residual(u1)) < 1e-10


@pytest.mark.slow
def test_open_channel_p2_converges_with_krylov_tolerance():
    """P2 Roe on the 12x4 bump channel with a far-field top, from the uniform
    free stream, with the paper's steady settings (PCEXP, m = 30, the eq. (cfl)
    ramp to CFL_max 1000, Krylov tolerance 1e-5 on the predictor's dt): the
    rho residual norm falls below 1e-10 within 200 iterations, and the
    tolerance is what makes it stable (the predictor halves dt)."""
    m = W.channel_bump(12, 4, height=0.1, seed=5, top_bc=W.BC_FARFIELD)
    prim = W.freestream_prim(2, angle_deg=0.0)
    g = DG(m, 2, "roe", farfield_prim=prim)
    u = g.project(lambda x: W.uniform_state(x, prim))
    u1, hist = steady_iterations(g, ExactJacobian(g), u, 200, 1000.0, 30, krylov_tol=1e-5)
    first = next(i for i, h in enumerate(hist) if h <= 1e-10)
    assert first < 200
    assert res_rho_norm(g, g.residual(u1)) < 1e-10
