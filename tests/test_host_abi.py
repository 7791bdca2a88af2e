"""CPU tests of the C-ABI library and its host-side set-up (no GPU needed).

* libpcexp.so loads and exports every function include/pcexp.h declares;
* the host set-up (independent of the oracle) agrees with the oracle on the
  quadrature nodes, face connectivity and face point placement, and its
  change of basis Q_E is orthogonal;
* malformed meshes and bad arguments are rejected before any GPU work.
"""

import ctypes
import os
import re

import numpy as np
import pytest
from scipy.special import roots_jacobi

import workloads as W
from oracle.dg import DG

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1801_06300_amd")
HEADER = os.path.join(ROOT, "include", "pcexp.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pcexp_[a-z_]+)\s*\(", text)))


def _lib(name):
    path = os.path.join(PKG, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not built")
    return ctypes.CDLL(path)


def test_library_exports_every_declared_symbol():
    lib = _lib("libpcexp.so")
    names = _declared()
    assert "pcexp_step" in names and "pcexp_arnoldi_phi" in names and "pcexp_vjp" in names
    for n in names:
        assert hasattr(lib, n), n


def _probe():
    lib = _lib("libpcexp_setup_probe.so")
    lib.pcexp_probe_setup.restype = ctypes.c_int
    return lib


def _run_probe(m, p):
    lib = _probe()
    vert = np.ascontiguousarray(m.vert, np.float64)
    elem = np.ascontiguousarray(m.elem, np.int32)
    canon = None if m.vert_canon is None else np.ascontiguousarray(m.vert_canon, np.int32)
    bf = np.ascontiguousarray(m.bface, np.int32)
    bt = np.ascontiguousarray(m.bface_tag, np.int32)
    sizes = np.zeros(8, np.int64)
    err = ctypes.create_string_buffer(256)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None
    rc = lib.pcexp_probe_setup(ctypes.c_int(m.dim), ctypes.c_longlong(vert.shape[0]), P(vert),
                               ctypes.c_longlong(elem.shape[0]), P(elem), P(canon), ctypes.c_longlong(bf.shape[0]),
                               P(bf), P(bt), ctypes.c_int(p), P(sizes), None, None, None, None, None, None, None,
                               None, None, None, err, 256)
    if rc != 0:
        return rc, err.value.decode(), None
    nb, nq, nfq, nori, nf, Epad, nE, d = [int(x) for x in sizes]
    out = dict(nb=nb, nq=nq, nfq=nfq, nori=nori, nf=nf, Epad=Epad, nE=nE, d=d,
               ref_pts=np.zeros(nq * d), wq=np.zeros(nq), fpts=np.zeros(nf * nori * nfq * d), wf=np.zeros(nfq),
               Q=np.zeros(nE * nb * nb), nbr=np.zeros(nf * Epad, np.int32), finfo=np.zeros(nf * Epad, np.int32),
               sdet=np.zeros(Epad))
    rc = lib.pcexp_probe_setup(ctypes.c_int(m.dim), ctypes.c_longlong(vert.shape[0]), P(vert),
                               ctypes.c_longlong(elem.shape[0]), P(elem), P(canon), ctypes.c_longlong(bf.shape[0]),
                               P(bf), P(bt), ctypes.c_int(p), None, P(out["ref_pts"]), P(out["wq"]), P(out["fpts"]),
                               P(out["wf"]), P(out["Q"]), P(out["nbr"]), P(out["finfo"]), P(out["sdet"]), None, None,
                               err, 256)
    assert rc == 0
    return 0, "", out


@pytest.mark.parametrize("n,a,b", [(1, 0, 0), (3, 0, 0), (4, 1, 0), (5, 2, 0), (2, 2, 0)])
def test_host_gauss_jacobi_matches_scipy(n, a, b):
    lib = _probe()
    x = np.zeros(n)
    w = np.zeros(n)
    lib.pcexp_probe_gauss_jacobi(ctypes.c_int(n), ctypes.c_double(a), ctypes.c_double(b),
                                 x.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p))
    xs, ws = roots_jacobi(n, a, b)
    assert np.max(np.abs(x - xs)) < 1e-14 and np.max(np.abs(w - ws)) < 1e-14 * ws.max()


@pytest.mark.parametrize("name,p", [("sq4j", 2), ("cube3", 2), ("chan", 1), ("sq3", 3), ("box3", 2)])
def test_host_setup_against_oracle(name, p):
    from tests.helpers import mesh_case
    m, _ = mesh_case(name)
    rc, msg, S = _run_probe(m, p)
    assert rc == 0, msg
    g = DG(m, p, "lf")
    d, nE, Ep, nf, nfq, nori, nb = S["d"], S["nE"], S["Epad"], S["nf"], S["nfq"], S["nori"], S["nb"]
    # same volume rule
    assert np.max(np.abs(S["ref_pts"].reshape(-1, d) - g.ref_pts)) < 1e-14
    assert np.max(np.abs(S["wq"] - g.ref_w)) < 1e-15
    # Q_E orthogonal
    Q = S["Q"].reshape(nE, nb, nb)
    assert np.max(np.abs(np.einsum("eij,ekj->eik", Q, Q) - np.eye(nb))) < 1e-12
    # connectivity and face point placement: physical points seen from each side agree with the oracle's
    nbr = S["nbr"].reshape(nf, Ep)[:, :nE].T
    assert np.array_equal(nbr, np.where(g.mesh.nbr >= 0, g.mesh.nbr, -1))
    finfo = S["finfo"].reshape(nf, Ep)[:, :nE].T
    assert np.array_equal((finfo >> 8) & 3, np.where(g.mesh.nbr >= 0, 0, g.mesh.bc))
    fpts = S["fpts"].reshape(nf, nori, nfq, d)
    X = g.mesh.X
    A = X[:, 1:, :] - X[:, :1, :]
    xo = g.face_points(slice(None))                       # oracle: own frame
    for f in range(nf):
        oE = (finfo[:, f] >> 5) & 7
        xi = fpts[f][oE]                                  # (nE, nfq, d)
        x = X[:, None, 0, :] + np.einsum("erj,ejc->erc", xi, A)
        assert np.max(np.abs(x - xo[:, f])) < 1e-12
        has = nbr[:, f] >= 0
        if np.any(has):
            nb_ = nbr[has, f]
            fN = finfo[has, f] & 3
            oN = (finfo[has, f] >> 2) & 7
            xiN = fpts[fN, oN]
            xN = X[nb_, None, 0, :] + np.einsum("erj,ejc->erc", xiN, A[nb_])
            want = xo[has, f] + g.mesh.nbr_shift[has, f][:, None, :]
            assert np.max(np.abs(xN - want)) < 1e-12


def test_host_rejects_malformed_meshes():
    m = W.periodic_square(3, 10.0)
    bad = W.MeshArrays(**{**m.__dict__})
    bad.elem = m.elem.copy()
    bad.elem[0, [1, 2]] = bad.elem[0, [2, 1]]            # clockwise triangle
    assert _run_probe(bad, 1)[0] == -2
    bad2 = W.MeshArrays(**{**m.__dict__})
    bad2.vert_canon = None                               # periodic faces left unmatched
    rc, msg, _ = _run_probe(bad2, 1)
    assert rc == -2 and "unmatched" in msg
    two = W.periodic_square(2, 10.0)                     # faces shared by more than two elements
    assert _run_probe(two, 1)[0] == -2


def test_abi_rejects_bad_arguments_without_gpu():
    """Validation returns before any HIP call (these run on a CPU-only host)."""
    lib = _lib("libpcexp.so")
    from paper_1801_06300_amd.binding import MeshDesc, DiscDesc, _SIGS
    for n, (res, args) in _SIGS.items():
        getattr(lib, n).restype = res
        getattr(lib, n).argtypes = args
    m = W.periodic_square(3, 10.0)
    vert = np.ascontiguousarray(m.vert)
    elem = np.ascontiguousarray(m.elem.copy())
    elem[0, [1, 2]] = elem[0, [2, 1]]
    canon = np.ascontiguousarray(m.vert_canon)
    md = MeshDesc()
    md.dim, md.n_vert, md.n_elem, md.n_bface = 2, vert.shape[0], elem.shape[0], 0
    md.vert = vert.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    md.elem = elem.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    md.vert_canon = canon.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    dd = DiscDesc()
    dd.p, dd.flux, dd.gamma = 1, 0, 1.4
    ctx = ctypes.c_void_p()
    assert lib.pcexp_create(ctypes.byref(md), ctypes.byref(dd), None, ctypes.byref(ctx)) == -2
    assert not ctx
    dd.p = 7
    assert lib.pcexp_create(ctypes.byref(md), ctypes.byref(dd), None, ctypes.byref(ctx)) in (-2, -7)
    dd.p, dd.flux = 1, 5
    assert lib.pcexp_create(ctypes.byref(md), ctypes.byref(dd), None, ctypes.byref(ctx)) == -1
    assert lib.pcexp_create(None, ctypes.byref(dd), None, ctypes.byref(ctx)) == -1
    assert lib.pcexp_create_dense(0, None, None, None, ctypes.byref(ctx)) == -1
    assert lib.pcexp_create_dense(5000, None, None, None, ctypes.byref(ctx)) == -1
    assert lib.pcexp_step(None, None, 0.1, 0.0, 10, 0, 0, 0, None, 0, None, None) == -1
    assert lib.pcexp_workspace_bytes(None, 10, 1, 0, 0) == 0
