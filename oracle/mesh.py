"""Mesh connectivity and geometry (Sec. 4.2-4.3, Sec. 5 eq. (x3d)).

Local face f of a simplex is the face opposite its local vertex f; its
vertices are the remaining local vertices in increasing local order.

Face point placement (a reading the paper leaves open): the face shared by
elements E and N is parametrised by its *owner*, the element of smaller
index (a boundary face by its only element); the canonical face vertices
are the owner's local face vertices in increasing local order.  Both sides
integrate over the same physical points.  Across a periodic boundary the
non-owner sees the points translated by the period, i.e. it evaluates its
own (global-Cartesian) basis at its own image of the point.
"""

from dataclasses import dataclass
from math import factorial

import numpy as np


@dataclass
class Mesh:
    dim: int
    X: np.ndarray          # (nE, d+1, d) vertex coordinates of each element
    vol: np.ndarray        # (nE,)
    centroid: np.ndarray   # (nE, d)
    half_ext: np.ndarray   # (nE, d)  L_x, L_y, (L_z)
    nbr: np.ndarray        # (nE, d+1) neighbour element, -1 on a boundary
    nbr_face: np.ndarray   # (nE, d+1) neighbour's local face index
    bc: np.ndarray         # (nE, d+1) 0 interior, else boundary tag
    owner: np.ndarray      # (nE, d+1) True if this element owns the face
    face_verts: np.ndarray  # (nE, d+1, d, d) canonical face vertices, in this element's frame
    nbr_shift: np.ndarray  # (nE, d+1, d) x_in_nbr_frame = x_in_own_frame + shift
    normal: np.ndarray     # (nE, d+1, d) outward unit normal
    area: np.ndarray       # (nE, d+1) face measure
    h: np.ndarray          # (nE,) 2 d |E| / |dE|   (eq. (x3d))
    volume_total: float


def face_local(dim):
    """(d+1, d) local vertex indices of each local face."""
    return np.array([[j for j in range(dim + 1) if j != f] for f in range(dim + 1)])


def build_mesh(m):
    """Connectivity + geometry from a ``workloads.MeshArrays``."""
    d = m.dim
    elem = np.asarray(m.elem, dtype=np.int64)
    vert = np.asarray(m.vert, dtype=np.float64)
    nE = elem.shape[0]
    canon = np.arange(vert.shape[0]) if m.vert_canon is None else np.asarray(m.vert_canon, np.int64)
    X = vert[elem]
    A = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))     # columns = edges
    detA = np.linalg.det(A)
    if np.any(detA <= 0):
        raise ValueError("element with non-positive orientation")
    vol = detA / factorial(d)
    centroid = X.mean(axis=1)
    half_ext = 0.5 * (X.max(axis=1) - X.min(axis=1))
    FL = face_local(d)
    ce = canon[elem]                                             # (nE, d+1)
    srt = np.sort(ce, axis=1)
    if np.any(srt[:, 1:] == srt[:, :-1]):
        raise ValueError("element touches its own periodic image")

    # --- match faces by their canonical vertex sets
    keys = np.sort(ce[:, FL], axis=2).reshape(nE * (d + 1), d)  # (M, d)
    order = np.lexsort(keys.T[::-1])
    ks = keys[order]
    new = np.ones(len(ks), bool)
    new[1:] = np.any(ks[1:] != ks[:-1], axis=1)
    gid = np.cumsum(new) - 1
    counts = np.bincount(gid)
    if np.any(counts > 2):
        raise ValueError("face shared by more than two elements")
    nbr = -np.ones(nE * (d + 1), np.int64)
    nbr_face = -np.ones(nE * (d + 1), np.int64)
    bc = np.zeros(nE * (d + 1), np.int64)
    pair_first = np.where(new & (counts[gid] == 2))[0]
    a, b = order[pair_first], order[pair_first + 1]
    nbr[a], nbr_face[a] = b // (d + 1), b % (d + 1)
    nbr[b], nbr_face[b] = a // (d + 1), a % (d + 1)
    single = order[new & (counts[gid] == 1)]
    btag = {tuple(sorted(canon[fv].tolist())): int(t)
            for fv, t in zip(np.asarray(m.bface), np.asarray(m.bface_tag))}
    for s in single:
        key = tuple(keys[s].tolist())
        if key not in btag:
            raise ValueError(f"unmatched face {key}")
        bc[s] = btag[key]
    nbr = nbr.reshape(nE, d + 1)
    nbr_face = nbr_face.reshape(nE, d + 1)
    bc = bc.reshape(nE, d + 1)

    eid = np.arange(nE)[:, None].repeat(d + 1, 1)
    owner = (nbr < 0) | (eid < nbr)

    # --- canonical face vertices in each element's own frame
    face_verts = X[:, FL, :].copy()                              # owner's own face vertices
    nbr_shift = np.zeros((nE, d + 1, d))
    ie, jf = np.nonzero(nbr >= 0)
    n_ = nbr[ie, jf]
    fn = nbr_face[ie, jf]
    # vertex of the neighbour that is the image of each local vertex of my face
    myloc = FL[jf]                                               # (M, d)
    cid = ce[ie[:, None], myloc]                                 # (M, d)
    kn = np.argmax(ce[n_][:, None, :] == cid[:, :, None], axis=2)  # (M, d)
    shift = X[n_, kn[:, 0]] - X[ie, myloc[:, 0]]                # own -> nbr frame
    nbr_shift[ie, jf] = shift
    no = ~owner[ie, jf]
    # for non-owned faces use the neighbour's (owner's) vertex order, moved into my frame
    oloc = FL[fn[no]]
    face_verts[ie[no], jf[no]] = X[n_[no][:, None], oloc] - shift[no][:, None, :]

    normal = np.zeros((nE, d + 1, d))
    area = np.zeros((nE, d + 1))
    for f in range(d + 1):
        P = X[:, FL[f]]
        if d == 2:
            t = P[:, 1] - P[:, 0]
            nv = np.stack([t[:, 1], -t[:, 0]], axis=-1)
            ar = np.linalg.norm(nv, axis=-1)
        else:
            nv = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
            ar = 0.5 * np.linalg.norm(nv, axis=-1)
        nv = nv / np.linalg.norm(nv, axis=-1, keepdims=True)
        outward = np.sum(nv * (P[:, 0] - X[:, f]), axis=-1) > 0
        nv[~outward] *= -1
        normal[:, f] = nv
        area[:, f] = ar
    h = 2.0 * d * vol / area.sum(axis=1)
    return Mesh(dim=d, X=X, vol=vol, centroid=centroid, half_ext=half_ext, nbr=nbr,
                nbr_face=nbr_face, bc=bc, owner=owner, face_verts=face_verts,
                nbr_shift=nbr_shift, normal=normal, area=area, h=h,
                volume_total=float(vol.sum()))


def affine_map(mesh, ref_pts, sel=slice(None)):
    """Physical points x = X_0 + sum_j xi_j (X_j - X_0): (nE, npts, d)."""
    X = mesh.X[sel]
    E = X[:, 1:, :] - X[:, :1, :]                      # (nE, d, d) rows = edges
    return X[:, None, 0, :] + np.einsum("qj,ejd->eqd", ref_pts, E)
