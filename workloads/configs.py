"""The five benchmark workloads (sizes and parameters as plain data).

Unstated parameters take the following values: vortex strength 5 on the
free stream (rho, p) = (1, 1), Mach 0.5 at 45 degrees; square/cube splits as
in :mod:`workloads.meshes`; the channel spans x in [-3, 3], y in
[y_b(x), 2] with a Gaussian bump of height 0.1 and width 0.25, a slip wall
along the bump and characteristic far-field boundaries at inflow, outflow
and top (with a second slip wall at the top, the duct's transverse
acoustic modes near cut-off decay so slowly that pseudo-time stepping
needs about ten times longer to reach the residual target), and
pseudo-time with the Krylov tolerance 1e-5 the paper states; the 3D
vortex column is parallel to z through (5, 5) with w_inf = 0.
"""

from .meshes import periodic_square, channel_bump, periodic_cube, BC_FARFIELD

CONFIGS = {
    "vortex2d_p1_16x16_lf": dict(name="vortex2d_p1_16x16_lf", mesh=("periodic_square", dict(n=16, length=10.0)),
            dim=2, p=1, flux="lf", m=20, cfl=5.0, steps=10, prec="f64",
            vortex_center=(5.0, 5.0), pert_seed=101),
    "vortex2d_p2_128x128_jitter_roe": dict(name="vortex2d_p2_128x128_jitter_roe",
            mesh=("periodic_square", dict(n=128, length=20.0, jitter=0.15, seed=202)),
            dim=2, p=2, flux="roe", m=30, cfl=20.0, steps=50, prec="f64",
            vortex_center=(10.0, 10.0), pert_seed=201),
    "channel_bump_p2_384x128": dict(name="channel_bump_p2_384x128",
            mesh=("channel_bump", dict(nx=384, ny=128, height=0.1, jitter=0.15, seed=302, top_bc=BC_FARFIELD)),
            dim=2, p=2, flux="roe", m=30, cfl_max=1000.0, krylov_tol=1e-5, steps=None, prec="mixed",
            mach=0.5, angle_deg=0.0, target_residual=1e-10),
    "vortex3d_p2_48cube_lf": dict(name="vortex3d_p2_48cube_lf", mesh=("periodic_cube", dict(n=48, length=10.0)),
            dim=3, p=2, flux="lf", m=30, cfl=10.0, steps=20, prec="mixed",
            vortex_center=(5.0, 5.0), pert_seed=401),
    "adjoint_vortex2d_p2_128x128_roe": dict(name="adjoint_vortex2d_p2_128x128_roe",
            mesh=("periodic_square", dict(n=128, length=20.0, jitter=0.15, seed=202)),
            dim=2, p=2, flux="roe", m=30, cfl=20.0, steps=40, checkpoint_every=8,
            prec="f64", vortex_center=(10.0, 10.0), pert_seed=201, dir_seed=501,
            n_dirs=16, fd_h=1e-6),
}

_GEN = dict(periodic_square=periodic_square, channel_bump=channel_bump,
            periodic_cube=periodic_cube)


def get_config(name):
    """A copy of the workload's parameters, by its name."""
    return dict(CONFIGS[name])


def build_mesh(cfg, **override):
    kind, kw = cfg["mesh"]
    kw = dict(kw)
    kw.update(override)
    return _GEN[kind](**kw)
