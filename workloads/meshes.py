"""Seeded mesh generators (vertex and element arrays only).

Every generator returns a :class:`MeshArrays` with positively oriented
simplices.  Periodic meshes keep duplicated image vertices on the periodic
boundary (so that every element has its own true coordinates) and give
``vert_canon``: for each vertex, the index of the vertex it is a periodic
image of.  Two element faces whose canonical vertex sets coincide are the
same face of the periodic domain.  Boundary faces of non-periodic meshes are
listed in ``bface`` with a tag in ``bface_tag``.
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

BC_SLIP = 1
BC_FARFIELD = 2


@dataclass
class MeshArrays:
    dim: int
    vert: np.ndarray                      # (n_vert, dim) float64
    elem: np.ndarray                      # (n_elem, dim+1) int32
    vert_canon: Optional[np.ndarray]      # (n_vert,) int32 or None
    bface: np.ndarray                     # (n_bface, dim) int32
    bface_tag: np.ndarray                 # (n_bface,) int32
    period: np.ndarray                    # (dim,) float64, 0 = not periodic
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_elem(self):
        return int(self.elem.shape[0])

    @property
    def n_vert(self):
        return int(self.vert.shape[0])


def _orient(vert, elem):
    """Reorder vertices of negatively oriented simplices (swap the last two)."""
    d = vert.shape[1]
    X = vert[elem]                                   # (E, d+1, d)
    A = X[:, 1:, :] - X[:, :1, :]                    # rows = edge vectors
    det = np.linalg.det(A)
    neg = det < 0
    if np.any(neg):
        e = elem[neg].copy()
        e[:, [d - 1, d]] = e[:, [d, d - 1]]
        elem = elem.copy()
        elem[neg] = e
    return elem


def _split_squares(nx, ny, vid):
    """Split each square (i, j) along its '\\' diagonal into 2 triangles.

    Corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1); the diagonal joins
    d and b.  Squares are numbered row-major (i fastest), two triangles each.
    """
    tris = np.empty((ny, nx, 2, 3), dtype=np.int64)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    a = vid(i, j)
    b = vid(i + 1, j)
    c = vid(i + 1, j + 1)
    d = vid(i, j + 1)
    tris[:, :, 0] = np.stack([a, b, d], axis=-1)
    tris[:, :, 1] = np.stack([b, c, d], axis=-1)
    return tris.reshape(-1, 3)


def periodic_square(n, length, jitter=0.0, seed=None, name=""):
    """Periodic [0, L]^2 with n x n squares, each split into 2 triangles.

    ``jitter`` is the half-width of the uniform vertex displacement as a
    fraction of h = L/n; the displacement is drawn per canonical vertex and
    applied identically to all of its periodic images.
    """
    h = length / n
    nv1 = n + 1
    vid = lambda i, j: j * nv1 + i
    jj, ii = np.meshgrid(np.arange(nv1), np.arange(nv1), indexing="ij")
    vert = np.stack([ii * h, jj * h], axis=-1).reshape(-1, 2).astype(np.float64)
    canon_ij = vid(ii % n, jj % n).reshape(-1)
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        disp = rng.uniform(-jitter * h, jitter * h, size=(n * n, 2))
        cidx = ((jj % n) * n + (ii % n)).reshape(-1)
        # image vertices = canonical vertex + integer multiples of the period
        base = np.stack([(ii % n) * h, (jj % n) * h], axis=-1).reshape(-1, 2)
        wrap = np.stack([(ii // n) * length, (jj // n) * length], axis=-1).reshape(-1, 2)
        vert = base + disp[cidx] + wrap
    elem = _split_squares(n, n, vid).astype(np.int32)
    elem = _orient(vert, elem).astype(np.int32)
    return MeshArrays(dim=2, vert=vert, elem=elem,
                      vert_canon=canon_ij.astype(np.int32),
                      bface=np.zeros((0, 2), np.int32),
                      bface_tag=np.zeros((0,), np.int32),
                      period=np.array([length, length], np.float64),
                      name=name or f"periodic_square_{n}",
                      meta=dict(n=n, length=length, h=h, jitter=jitter, seed=seed))


def stretched_square(n, length, name=""):
    """Periodic [0, L]^2 clustered mesh x_j = (1-xi^3)/2 x_L + (1+xi^3)/2 x_R.

    xi_j = 2 (j-1)/n - 1 for j = 1..n+1 (n cells per direction); same
    clustering in y; each cell split into two triangles.
    """
    j = np.arange(1, n + 2)
    xi = 2.0 * (j - 1) / n - 1.0
    x = 0.5 * (1 - xi ** 3) * 0.0 + 0.5 * (1 + xi ** 3) * length
    nv1 = n + 1
    vid = lambda i, jj: jj * nv1 + i
    jj, ii = np.meshgrid(np.arange(nv1), np.arange(nv1), indexing="ij")
    vert = np.stack([x[ii], x[jj]], axis=-1).reshape(-1, 2)
    canon = vid(ii % n, jj % n).reshape(-1)
    elem = _orient(vert, _split_squares(n, n, vid).astype(np.int32)).astype(np.int32)
    return MeshArrays(dim=2, vert=vert, elem=elem, vert_canon=canon.astype(np.int32),
                      bface=np.zeros((0, 2), np.int32), bface_tag=np.zeros((0,), np.int32),
                      period=np.array([length, length], np.float64),
                      name=name or f"stretched_square_{n}", meta=dict(n=n, length=length))


def bump_height(x, height=0.1, width=0.25):
    """Gaussian bump y_b(x) = height * exp(-x^2 / (2 width^2))."""
    return height * np.exp(-x ** 2 / (2.0 * width ** 2))


def channel_bump(nx, ny, height=0.1, jitter=0.15, seed=None, x0=-3.0, x1=3.0,
                 y_top=2.0, top_bc=BC_SLIP, name=""):
    """Channel x in [x0, x1], y in [y_b(x), y_top] with a Gaussian bump.

    Structured (x, eta) grid mapped by y = y_b(x) + eta (y_top - y_b(x));
    interior vertices are jittered by U(-jitter, jitter) of the local
    spacing in x and in eta.  The bottom (with the bump) is a slip wall, the
    top boundary y = y_top has the tag ``top_bc`` (a slip wall by default),
    left and right are far-field boundaries.
    """
    xs = np.linspace(x0, x1, nx + 1)
    es = np.linspace(0.0, 1.0, ny + 1)
    jj, ii = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = xs[ii].astype(np.float64)
    E = es[jj].astype(np.float64)
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        hx = (x1 - x0) / nx
        he = 1.0 / ny
        dx = rng.uniform(-jitter * hx, jitter * hx, size=X.shape)
        de = rng.uniform(-jitter * he, jitter * he, size=E.shape)
        interior = (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny)
        X = np.where(interior, X + dx, X)
        E = np.where(interior, E + de, E)
    yb = bump_height(X, height)
    Y = yb + E * (y_top - yb)
    vert = np.stack([X, Y], axis=-1).reshape(-1, 2)
    vid = lambda i, j: j * (nx + 1) + i
    elem = _orient(vert, _split_squares(nx, ny, vid).astype(np.int32)).astype(np.int32)
    i = np.arange(nx)
    j = np.arange(ny)
    bottom = np.stack([vid(i, 0), vid(i + 1, 0)], axis=-1)
    top = np.stack([vid(i, ny), vid(i + 1, ny)], axis=-1)
    left = np.stack([vid(0, j), vid(0, j + 1)], axis=-1)
    right = np.stack([vid(nx, j), vid(nx, j + 1)], axis=-1)
    bface = np.concatenate([bottom, top, left, right]).astype(np.int32)
    tag = np.concatenate([np.full(nx, BC_SLIP), np.full(nx, top_bc),
                          np.full(ny, BC_FARFIELD), np.full(ny, BC_FARFIELD)]).astype(np.int32)
    return MeshArrays(dim=2, vert=vert, elem=elem, vert_canon=None, bface=bface,
                      bface_tag=tag, period=np.zeros(2), name=name or f"channel_{nx}x{ny}",
                      meta=dict(nx=nx, ny=ny, height=height, jitter=jitter, seed=seed, top_bc=top_bc))


def box_cube(n, length, jitter=0.0, seed=None, name=""):
    """[0, L]^3 with n^3 cubes, each split into 6 tetrahedra as in
    :func:`periodic_cube`, without periodic identification.  The faces on
    x = 0 and x = L are far-field boundaries, those on the other four sides
    slip walls.  ``jitter`` displaces interior vertices by U(-jitter,
    jitter) of h in each coordinate."""
    h = length / n
    nv1 = n + 1
    kk, jj, ii = np.meshgrid(np.arange(nv1), np.arange(nv1), np.arange(nv1), indexing="ij")
    vert = np.stack([ii * h, jj * h, kk * h], axis=-1).reshape(-1, 3).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        interior = ((ii > 0) & (ii < n) & (jj > 0) & (jj < n) & (kk > 0) & (kk < n)).reshape(-1)
        disp = rng.uniform(-jitter * h, jitter * h, size=vert.shape)
        vert = np.where(interior[:, None], vert + disp, vert)
    ref = periodic_cube(n, length)
    elem = _orient(vert, np.asarray(ref.elem, np.int32)).astype(np.int32)
    # boundary faces: the element faces whose three vertices lie on one side of the box
    faces = np.concatenate([elem[:, [1, 2, 3]], elem[:, [0, 2, 3]], elem[:, [0, 1, 3]], elem[:, [0, 1, 2]]])
    ijk = np.stack([ii, jj, kk], axis=-1).reshape(-1, 3)
    fi = ijk[faces]                                              # (nF, 3 vertices, 3 axes)
    bf, tags = [], []
    for ax in range(3):
        for side in (0, n):
            on = np.all(fi[:, :, ax] == side, axis=1)
            bf.append(faces[on])
            tags.append(np.full(int(on.sum()), BC_FARFIELD if ax == 0 else BC_SLIP))
    return MeshArrays(dim=3, vert=vert, elem=elem, vert_canon=None,
                      bface=np.concatenate(bf).astype(np.int32), bface_tag=np.concatenate(tags).astype(np.int32),
                      period=np.zeros(3, np.float64),
                      name=name or f"box_cube_{n}", meta=dict(n=n, length=length, h=h, jitter=jitter, seed=seed))


def periodic_cube(n, length, name=""):
    """Periodic [0, L]^3 with n^3 cubes, each split into 6 tetrahedra.

    The split is the Kuhn (path) triangulation along the cube diagonal
    from (1,0,0) to (0,1,1), i.e. the standard one reflected in x; it is
    conforming under translation.  Cubes are numbered with i fastest.
    """
    h = length / n
    nv1 = n + 1
    kk, jj, ii = np.meshgrid(np.arange(nv1), np.arange(nv1), np.arange(nv1), indexing="ij")
    vert = np.stack([ii * h, jj * h, kk * h], axis=-1).reshape(-1, 3).astype(np.float64)
    vid = lambda i, j, k: (k * nv1 + j) * nv1 + i
    canon = vid(ii % n, jj % n, kk % n).reshape(-1)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    local = []
    for p in perms:
        path = [np.zeros(3, int)]
        for ax in p:
            nxt = path[-1].copy()
            nxt[ax] += 1
            path.append(nxt)
        # reflect x: local corner offset (ox, oy, oz) -> (1 - ox, oy, oz)
        local.append([(1 - q[0], q[1], q[2]) for q in path])
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for t, corners in enumerate(local):
        for c, (ox, oy, oz) in enumerate(corners):
            tets[:, t, c] = vid(i + ox, j + oy, k + oz)
    elem = _orient(vert, tets.reshape(-1, 4).astype(np.int32)).astype(np.int32)
    return MeshArrays(dim=3, vert=vert, elem=elem, vert_canon=canon.astype(np.int32),
                      bface=np.zeros((0, 3), np.int32), bface_tag=np.zeros((0,), np.int32),
                      period=np.array([length] * 3, np.float64),
                      name=name or f"periodic_cube_{n}", meta=dict(n=n, length=length, h=h))
