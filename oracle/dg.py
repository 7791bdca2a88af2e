"""DG residual R(u) of the Euler equations (Sec. 4.2, eq. (euler3), with the
orthonormal basis of Sec. 4.3 so that the mass matrix is the identity).

For element E, basis function psi_i and variable k:

  R_{E,k,i} = sum_q W_q F_k(U_h(x_q)) . grad psi_i(x_q)
            - sum_f |f| sum_r w_r psi_i(x_r) Ftilde_k(U_L(x_r), U_R(x_r), n_f)

with U_L the trace of E ("host cell L" of eqs. (jac1)/(jac2)), U_R the trace
of the neighbour across f (or the ghost state on a boundary face), n_f the
outward normal of E.  Omega = 0, so the source term vanishes.

Coefficient layout: u[E, k, i] (element, conserved variable, basis function).
"""

from dataclasses import dataclass
from math import factorial

import numpy as np

from . import quadrature, basis, euler
from .mesh import build_mesh, affine_map


@dataclass
class _Cache:
    W: np.ndarray       # (n, Nq)
    psi: np.ndarray     # (n, Nq, N)
    gpsi: np.ndarray    # (n, Nq, N, d)
    psiL: np.ndarray    # (n, F, Nfq, N)
    psiR: np.ndarray    # (n, F, Nfq, N)


class DG:
    """Plain DG operator on a ``workloads.MeshArrays`` mesh."""

    def __init__(self, mesh_arrays, p, flux="lf", gamma=1.4, farfield_prim=None,
                 chunk=8192, cache_limit=4e7):
        self.m = mesh_arrays
        self.mesh = build_mesh(mesh_arrays)
        self.d = d = self.mesh.dim
        self.p = p
        self.nv = d + 2
        self.flux = flux
        self.gamma = gamma
        self.farfield_prim = None if farfield_prim is None else np.asarray(farfield_prim, np.float64)
        self.exps = basis.exponents(d, p)
        self.N = len(self.exps)
        self.nE = self.mesh.X.shape[0]
        self.ref_pts, self.ref_w, self.mu, self.wf = quadrature.dg_rules(d, p)
        self.Nq = len(self.ref_w)
        self.Nfq = len(self.wf)
        self.chunk = chunk
        self.C = np.zeros((self.nE, self.N, self.N))
        for s in self._chunks():
            x = affine_map(self.mesh, self.ref_pts, s)
            W = self._weights(s)
            chi = basis.monomials(x, self.mesh.centroid[s], self.mesh.half_ext[s], self.exps)
            gram = np.einsum("eq,eqa,eqb->eab", W, chi, chi)
            self.C[s] = basis.mgs_coefficients(gram)
        per = self.Nq * self.N * (1 + d) + 2 * (d + 1) * self.Nfq * self.N
        self._cache = None
        if self.nE * per <= cache_limit:
            self._cache = {i: self._build(s) for i, s in enumerate(self._chunks())}

    @property
    def K(self):
        return self.nE * self.nv * self.N

    def _chunks(self):
        for a in range(0, self.nE, self.chunk):
            yield slice(a, min(a + self.chunk, self.nE))

    def _weights(self, s):
        detA = self.mesh.vol[s] * factorial(self.d)
        return self.ref_w[None, :] * detA[:, None]

    def psi(self, x, elems, grad=False):
        """Basis of the elements ``elems`` at their own points x (n, npts, d)."""
        C = self.C[elems]
        out = basis.monomials(x, self.mesh.centroid[elems], self.mesh.half_ext[elems],
                              self.exps, grad=grad)
        if not grad:
            return np.einsum("eqa,eia->eqi", out, C)
        v, g = out
        return np.einsum("eqa,eia->eqi", v, C), np.einsum("eqad,eia->eqid", g, C)

    def face_points(self, s):
        """Face quadrature points of elements s in their own frame: (n, F, Nfq, d)."""
        return np.einsum("rj,efjd->efrd", self.mu, self.mesh.face_verts[s])

    def _build(self, s):
        idx = np.arange(self.nE)[s]
        x = affine_map(self.mesh, self.ref_pts, s)
        psi, gpsi = self.psi(x, idx, grad=True)
        xf = self.face_points(s)
        n, F, R, d = xf.shape
        psiL = self.psi(xf.reshape(n, F * R, d), idx).reshape(n, F, R, self.N)
        nb = self.mesh.nbr[s]
        nbv = np.where(nb >= 0, nb, 0)
        xr = xf + self.mesh.nbr_shift[s][:, :, None, :]
        psiR = self.psi(xr.reshape(n * F, R, d), nbv.reshape(-1)).reshape(n, F, R, self.N)
        psiR[nb < 0] = 0.0
        return _Cache(self._weights(s), psi, gpsi, psiL, psiR)

    def _data(self, i, s):
        if self._cache is not None:
            return self._cache[i]
        return self._build(s)

    def numflux(self, UL, UR, n):
        if self.flux == "lf":
            return euler.lax_friedrichs(UL, UR, n, self.gamma)
        if self.flux == "roe":
            return euler.roe(UL, UR, n, self.gamma)
        raise ValueError(self.flux)

    def residual(self, u):
        """R(u) for coefficients u (nE, nv, N), real or complex."""
        u = np.asarray(u)
        R = np.zeros(u.shape, dtype=u.dtype)
        for i, s in enumerate(self._chunks()):
            c = self._data(i, s)
            us = u[s]
            U = np.einsum("eqi,eki->eqk", c.psi, us)
            Fp = euler.physical_flux(U, self.gamma)
            Rv = np.einsum("eq,eqkd,eqid->eki", c.W, Fp, c.gpsi)
            UL = np.einsum("efri,eki->efrk", c.psiL, us)
            nb = self.mesh.nbr[s]
            UR = np.einsum("efri,efki->efrk", c.psiR, u[np.where(nb >= 0, nb, 0)])
            nrm = np.broadcast_to(self.mesh.normal[s][:, :, None, :], UL.shape[:-1] + (self.d,))
            bc = self.mesh.bc[s]
            if np.any(bc > 0):
                UR = UR.copy()
                for tag, fn in ((1, self._slip), (2, self._far)):
                    mask = bc == tag
                    if np.any(mask):
                        UR[mask] = fn(UL[mask], nrm[mask])
            Fn = self.numflux(UL, UR, nrm)
            wa = self.mesh.area[s][:, :, None] * self.wf[None, None, :]
            Rf = np.einsum("efr,efrk,efri->eki", wa, Fn, c.psiL)
            R[s] = Rv - Rf
        return R

    def _slip(self, UL, n):
        return euler.slip_wall_ghost(UL, n, self.gamma)

    def _far(self, UL, n):
        return euler.farfield_ghost(UL, n, self.farfield_prim, self.gamma)

    # ---------------------------------------------------------------- helpers
    def quad_points(self):
        return np.concatenate([affine_map(self.mesh, self.ref_pts, s) for s in self._chunks()])

    def project(self, values):
        """L2 projection (mass = I): u_{E,k,i} = sum_q W_q psi_i(x_q) U_k(x_q).

        ``values`` is (nE, Nq, nv) at ``quad_points()`` or a callable of points."""
        out = np.zeros((self.nE, self.nv, self.N))
        for i, s in enumerate(self._chunks()):
            c = self._data(i, s)
            if callable(values):
                x = affine_map(self.mesh, self.ref_pts, s)
                V = values(x.reshape(-1, self.d)).reshape(x.shape[0], self.Nq, self.nv)
            else:
                V = values[s]
            out[s] = np.einsum("eq,eqi,eqk->eki", c.W, c.psi, V)
        return out

    def evaluate(self, u):
        """U_h at the volume quadrature points: (nE, Nq, nv)."""
        out = np.zeros((self.nE, self.Nq, self.nv), dtype=np.asarray(u).dtype)
        for i, s in enumerate(self._chunks()):
            c = self._data(i, s)
            out[s] = np.einsum("eqi,eki->eqk", c.psi, u[s])
        return out

    def evaluate_at(self, u, x_ref):
        """U_h at reference points x_ref (npts, d) of every element: (nE, npts, nv)."""
        x = affine_map(self.mesh, x_ref)
        ps = self.psi(x, np.arange(self.nE))
        return np.einsum("eqi,eki->eqk", ps, u)

    def integrate(self, g):
        """sum_E sum_q W_q g(E, q) for values g (nE, Nq, ...)."""
        out = 0.0
        for i, s in enumerate(self._chunks()):
            c = self._data(i, s)
            out = out + np.einsum("eq,eq...->...", c.W, g[s])
        return out
