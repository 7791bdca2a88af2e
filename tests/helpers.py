"""Shared test fixtures: seeded meshes/states and the oracle <-> device plumbing.

Inputs come from the ``workloads`` generators; expected values come only from
``oracle``.  The device path is reached only through the C ABI binding.
"""

import numpy as np

import workloads as W


def mesh_case(name):
    if name == "sq3":
        return W.periodic_square(3, 10.0), 45.0
    if name == "sq4j":
        return W.periodic_square(4, 10.0, 0.15, 11), 45.0
    if name == "sq16":
        return W.periodic_square(16, 10.0), 45.0
    if name == "sq8j":
        return W.periodic_square(8, 10.0, 0.15, 23), 45.0
    if name == "cube3":
        return W.periodic_cube(3, 10.0), 45.0
    if name == "box3":
        return W.box_cube(3, 10.0, 0.1, 7), 0.0
    if name == "chan":
        return W.channel_bump(12, 4, height=0.1, seed=5), 0.0
    if name == "chan_flat":
        return W.channel_bump(12, 4, height=0.0, seed=5), 0.0
    raise KeyError(name)


def vortex_state(dg, mesh, amp=1e-6, seed=101, uinf=None):
    """Oracle projection of the isentropic vortex (or the free stream for a
    non-periodic mesh) plus a seeded perturbation, shape (nE, nv, Nb)."""
    if mesh.period[0] > 0:
        c = 0.5 * mesh.period[0]
        f = lambda x: W.isentropic_vortex(x, center=(c, c), period=mesh.period, uinf=uinf)
    else:
        prim = W.freestream_prim(mesh.dim, angle_deg=0.0)
        f = lambda x: W.uniform_state(x, prim)
    u = dg.project(f)
    return u + W.perturbation(u.shape, seed, amp)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
