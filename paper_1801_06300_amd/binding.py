"""Thin ctypes binding of libpcexp (include/pcexp.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device memory and streams come from PyTorch (tensors on a HIP device and the
current stream); there is no CPU fallback -- if libpcexp.so is missing or the
tensors are not on the GPU, the calls raise.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcexp.so")

OK = 0
STATUS = {0: "OK", -1: "E_ARG", -2: "E_MESH", -3: "E_HIP", -4: "E_WORKSPACE", -5: "E_NONFINITE",
          -6: "E_UNPHYSICAL", -7: "E_UNSUPPORTED"}
FLUX = {"lf": 0, "roe": 1}
PREC = {"f64": 0, "mixed": 1}
JVP = {"tangent": 0, "fd": 1, "zero": 2}
SCHEME = {"pcexp": 0, "exp1": 1}

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_vert", ctypes.c_int64), ("vert", c_double_p),
                ("n_elem", ctypes.c_int64), ("elem", c_int32_p), ("vert_canon", c_int32_p),
                ("n_bface", ctypes.c_int64), ("bface", c_int32_p), ("bface_tag", c_int32_p)]


class DiscDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("flux", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("farfield_prim", ctypes.c_double * 5)]


class KrylovInfo(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("h_last", ctypes.c_double), ("m_eff", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("err_est", ctypes.c_double), ("dt_halvings", ctypes.c_int32),
                ("pad", ctypes.c_int32)]

    def as_dict(self):
        return dict(beta=self.beta, h_last=self.h_last, m_eff=self.m_eff, breakdown=bool(self.breakdown),
                    err_est=self.err_est, dt_halvings=self.dt_halvings)


class StepInfo(ctypes.Structure):
    _fields_ = [("k1", KrylovInfo), ("k2", KrylovInfo), ("dt", ctypes.c_double),
                ("res_rho_norm", ctypes.c_double), ("flags", ctypes.c_uint32), ("t_advanced", ctypes.c_double)]

    def as_dict(self):
        return dict(k1=self.k1.as_dict(), k2=self.k2.as_dict(), dt=self.dt,
                    res_rho_norm=self.res_rho_norm, flags=int(self.flags), t_advanced=self.t_advanced)


class SteadyInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("res_rho_norm0", ctypes.c_double), ("res_rho_norm", ctypes.c_double)]

    def as_dict(self):
        return dict(iterations=self.iterations, converged=bool(self.converged),
                    res_rho_norm0=self.res_rho_norm0, res_rho_norm=self.res_rho_norm)


_VP = ctypes.c_void_p
_SIGS = {
    "pcexp_create": (ctypes.c_int, [ctypes.POINTER(MeshDesc), ctypes.POINTER(DiscDesc), _VP, ctypes.POINTER(_VP)]),
    "pcexp_create_dense": (ctypes.c_int, [ctypes.c_int64, _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    "pcexp_destroy": (None, [_VP]),
    "pcexp_sizes": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "pcexp_last_error": (ctypes.c_char_p, [_VP]),
    "pcexp_workspace_bytes": (ctypes.c_size_t, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "pcexp_quad_points": (ctypes.c_int, [_VP, _VP, _VP]),
    "pcexp_project": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "pcexp_evaluate": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "pcexp_residual": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "pcexp_jvp": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP]),
    "pcexp_vjp": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "pcexp_vjp2": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "pcexp_step_vjp_workspace_bytes": (ctypes.c_size_t, [_VP, ctypes.c_int32]),
    "pcexp_pressure_functional": (ctypes.c_int, [_VP, _VP, ctypes.c_double, c_double_p, _VP, _VP]),
    "pcexp_pressure_functional_acc": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_double, _VP, _VP, _VP]),
    "pcexp_step_vjp": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP,
                                      ctypes.c_size_t, _VP]),
    "pcexp_stable_dt": (ctypes.c_int, [_VP, _VP, ctypes.c_double, c_double_p, _VP]),
    "pcexp_conserved_totals": (ctypes.c_int, [_VP, _VP, c_double_p, _VP]),
    "pcexp_arnoldi_phi": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, _VP, _VP, ctypes.c_size_t,
                                         ctypes.POINTER(KrylovInfo), _VP]),
    "pcexp_profile": (ctypes.c_int, [_VP, ctypes.c_int32, c_double_p]),
    "pcexp_set_krylov_tol": (ctypes.c_int, [_VP, ctypes.c_double]),
    "pcexp_set_krylov_adapt": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "pcexp_step_etd2": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_int32, _VP, ctypes.c_size_t, _VP, _VP]),
    "pcexp_steady": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                    ctypes.c_size_t, ctypes.POINTER(SteadyInfo), _VP]),
    "pcexp_step": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_size_t,
                                  ctypes.POINTER(StepInfo), _VP]),
    "pcexp_step_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(StepInfo), _VP]),
    "pcexp_advance": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_size_t,
                                     ctypes.POINTER(StepInfo), _VP]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libpcexp.so and declare its signatures (raises if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1801_06300_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PcexpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class PCEXP:
    """A libpcexp context for one mesh and discretisation (or a dense test operator)."""

    def __init__(self, mesh=None, p=1, flux="lf", gamma=1.4, farfield_prim=None, device="cuda",
                 _dense=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("libpcexp needs a HIP device tensor")
        self.ctx = ctypes.c_void_p()
        self._ws = {}
        with torch.cuda.device(self.device):
            st = self._stream()
            if _dense is not None:
                Aj, Ar = _dense
                self._Aj, self._Ar = Aj, Ar
                s = self.lib.pcexp_create_dense(Aj.shape[0], _ptr(Aj), _ptr(Ar), st, ctypes.byref(self.ctx))
            else:
                self.mesh = mesh
                self._vert = np.ascontiguousarray(mesh.vert, dtype=np.float64)
                self._elem = np.ascontiguousarray(mesh.elem, dtype=np.int32)
                self._canon = None if mesh.vert_canon is None else np.ascontiguousarray(mesh.vert_canon, np.int32)
                self._bf = np.ascontiguousarray(mesh.bface, dtype=np.int32)
                self._bt = np.ascontiguousarray(mesh.bface_tag, dtype=np.int32)
                md = MeshDesc()
                md.dim = mesh.dim
                md.n_vert = self._vert.shape[0]
                md.vert = self._vert.ctypes.data_as(c_double_p)
                md.n_elem = self._elem.shape[0]
                md.elem = self._elem.ctypes.data_as(c_int32_p)
                md.vert_canon = self._canon.ctypes.data_as(c_int32_p) if self._canon is not None else None
                md.n_bface = self._bf.shape[0]
                md.bface = self._bf.ctypes.data_as(c_int32_p) if self._bf.size else None
                md.bface_tag = self._bt.ctypes.data_as(c_int32_p) if self._bt.size else None
                dd = DiscDesc()
                dd.p = p
                dd.flux = FLUX[flux]
                dd.gamma = gamma
                ff = np.zeros(5)
                if farfield_prim is not None:
                    ff[:len(farfield_prim)] = farfield_prim
                for i in range(5):
                    dd.farfield_prim[i] = ff[i]
                s = self.lib.pcexp_create(ctypes.byref(md), ctypes.byref(dd), st, ctypes.byref(self.ctx))
        if s != OK:
            raise PcexpError(s, "pcexp_create failed")
        sz = (ctypes.c_int64 * 8)()
        self.lib.pcexp_sizes(self.ctx, sz)
        self.K, self.nE, self.dim, self.nv, self.nb, self.nq, self.nfq, self.p = [int(x) for x in sz]
        self.shape = (self.nE, self.nv, self.nb) if _dense is None else (self.K,)

    @classmethod
    def dense(cls, A_jac, A_res, device="cuda"):
        """Test operator R(u) = A_res u, J v = A_jac v (FP64 device matrices)."""
        import torch
        Aj = torch.as_tensor(A_jac, dtype=torch.float64, device=device).contiguous()
        Ar = torch.as_tensor(A_res, dtype=torch.float64, device=device).contiguous()
        return cls(device=device, _dense=(Aj, Ar))

    def __del__(self):
        try:
            if self.ctx:
                self.lib.pcexp_destroy(self.ctx)
                self.ctx = ctypes.c_void_p()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, s, what):
        if s != OK:
            raise PcexpError(s, f"{what}: {self.lib.pcexp_last_error(self.ctx).decode()}")

    def _vec(self, x, shape=None):
        t = self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t

    def empty(self):
        return self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)

    def workspace(self, m, k=1, prec="f64", jvp="tangent"):
        key = (m, k, prec)
        nbytes = self.lib.pcexp_workspace_bytes(self.ctx, m, k, PREC[prec], JVP[jvp])
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws, nbytes

    # ------------------------------------------------------------ entry points
    def quad_points(self):
        out = self.torch.empty((self.nE, self.nq, self.dim), dtype=self.torch.float64, device=self.device)
        self._check(self.lib.pcexp_quad_points(self.ctx, _ptr(out), self._stream()), "quad_points")
        return out

    def project(self, U_qp):
        U = self._vec(U_qp, (self.nE, self.nq, self.nv))
        u = self.empty()
        self._check(self.lib.pcexp_project(self.ctx, _ptr(U), _ptr(u), self._stream()), "project")
        return u

    def evaluate(self, u):
        u = self._vec(u, self.shape)
        out = self.torch.empty((self.nE, self.nq, self.nv), dtype=self.torch.float64, device=self.device)
        self._check(self.lib.pcexp_evaluate(self.ctx, _ptr(u), _ptr(out), self._stream()), "evaluate")
        return out

    def residual(self, u, out=None):
        u = self._vec(u, self.shape)
        R = self.empty() if out is None else out
        self._check(self.lib.pcexp_residual(self.ctx, _ptr(u), _ptr(R), self._stream()), "residual")
        return R

    def jvp(self, u, v, kind="tangent", prec="f64", out=None):
        """J(u) v; v and the result are float64 for prec="f64" and float32 for
        prec="mixed" (the library's FP32 boundary)."""
        u = self._vec(u, self.shape)
        if prec == "mixed":
            v = self.torch.as_tensor(v, device=self.device).to(self.torch.float32).contiguous().reshape(self.shape)
            Jv = self.torch.empty(self.shape, dtype=self.torch.float32, device=self.device) if out is None else out
            if Jv.dtype != self.torch.float32:
                raise ValueError("mixed-precision jvp writes a float32 output")
        else:
            v = self._vec(v, self.shape)
            Jv = self.empty() if out is None else out
        self._check(self.lib.pcexp_jvp(self.ctx, _ptr(u), _ptr(v), _ptr(Jv), JVP[kind], PREC[prec],
                                       self._stream()), "jvp")
        return Jv

    def vjp(self, u, w, out=None):
        u = self._vec(u, self.shape)
        w = self._vec(w, self.shape)
        out = self.empty() if out is None else out
        self._check(self.lib.pcexp_vjp(self.ctx, _ptr(u), _ptr(w), _ptr(out), self._stream()), "vjp")
        return out

    def vjp2(self, u, v, w):
        """(J(u)^T w, d/deps [J(u + eps v)^T w]) in one pass."""
        u = self._vec(u, self.shape)
        v = self._vec(v, self.shape)
        w = self._vec(w, self.shape)
        out, out_d = self.empty(), self.empty()
        self._check(self.lib.pcexp_vjp2(self.ctx, _ptr(u), _ptr(v), _ptr(w), _ptr(out), _ptr(out_d),
                                        self._stream()), "vjp2")
        return out, out_d

    def pressure_functional(self, u, p_ref=1.0, grad=False):
        """int (p_h - p_ref)^2 dx, and its gradient with respect to u if grad."""
        u = self._vec(u, self.shape)
        val = ctypes.c_double()
        g = self.empty() if grad else None
        self._check(self.lib.pcexp_pressure_functional(self.ctx, _ptr(u), float(p_ref), ctypes.byref(val),
                                                       _ptr(g) if grad else None, self._stream()),
                    "pressure_functional")
        return (val.value, g) if grad else val.value

    def pressure_functional_acc(self, u, scale, p_ref=1.0, value_acc=None, grad_acc=None):
        """value_acc += scale P(u) and grad_acc += scale dP/du on the device
        (contiguous FP64 device tensors: a 0-dim scalar and a state-shaped
        vector; either may be None), asynchronously."""
        for t in (u, value_acc, grad_acc):
            if t is not None and not (t.is_cuda and t.dtype == self.torch.float64 and t.is_contiguous()):
                raise ValueError("pressure_functional_acc: pass contiguous float64 device tensors")
        if grad_acc is not None and tuple(grad_acc.shape) != tuple(self.shape):
            raise ValueError("grad_acc must have the state's shape")
        self._check(self.lib.pcexp_pressure_functional_acc(
            self.ctx, _ptr(u), float(p_ref), float(scale), _ptr(value_acc) if value_acc is not None else None,
            _ptr(grad_acc) if grad_acc is not None else None, self._stream()), "pressure_functional_acc")

    def step_vjp(self, u, ubar, dt, m=30, scheme="pcexp", out=None):
        """(d u_{n+1} / d u_n)^T ubar for the step from u with fixed dt (FP64, tangent JVP)."""
        u = self._vec(u, self.shape)
        ubar = self._vec(ubar, self.shape)
        nbytes = self.lib.pcexp_step_vjp_workspace_bytes(self.ctx, m)
        key = ("rev", m)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
            self._ws[key] = ws
        out = self.empty() if out is None else out
        self._check(self.lib.pcexp_step_vjp(self.ctx, _ptr(u), float(dt), m, SCHEME[scheme], _ptr(ubar), _ptr(out),
                                            _ptr(ws), nbytes, self._stream()), "step_vjp")
        return out

    def stable_dt(self, u, cfl):
        u = self._vec(u, self.shape)
        dt = ctypes.c_double()
        self._check(self.lib.pcexp_stable_dt(self.ctx, _ptr(u), cfl, ctypes.byref(dt), self._stream()), "stable_dt")
        return dt.value

    def conserved_totals(self, u):
        u = self._vec(u, self.shape)
        out = (ctypes.c_double * self.nv)()
        self._check(self.lib.pcexp_conserved_totals(self.ctx, _ptr(u), out, self._stream()), "totals")
        return np.array(out[:])

    def arnoldi_phi(self, u_lin, b, dt, k=1, m=30, prec="f64", jvp="tangent", info=False, out=None):
        u_lin = self._vec(u_lin, self.shape)
        b = self._vec(b, self.shape)
        out = self.empty() if out is None else out
        ws, nbytes = self.workspace(m, k, prec, jvp)
        inf = KrylovInfo()
        self._check(self.lib.pcexp_arnoldi_phi(self.ctx, _ptr(u_lin), _ptr(b), float(dt), k, m, PREC[prec],
                                               JVP[jvp], _ptr(out), _ptr(ws), nbytes,
                                               ctypes.byref(inf) if info else None, self._stream()),
                    "arnoldi_phi")
        return (out, inf.as_dict()) if info else out

    PROFILE_CLASSES = ("residual", "jvp", "gs_reduce", "gs_close", "gs_update", "hess_phi", "combine", "other")

    def profile(self, op):
        """op 'start' (enable + reset), 'stop', or 'read' -> {class: (ms, launches, bytes)}."""
        if op == "start":
            self._check(self.lib.pcexp_profile(self.ctx, 1, None), "profile")
            return None
        if op == "stop":
            self._check(self.lib.pcexp_profile(self.ctx, 0, None), "profile")
            return None
        out = (ctypes.c_double * 24)()
        self._check(self.lib.pcexp_profile(self.ctx, 2, out), "profile")
        return {name: (out[3 * i], int(out[3 * i + 1]), out[3 * i + 2])
                for i, name in enumerate(self.PROFILE_CLASSES)}

    def set_krylov_tol(self, tol):
        """Predictor dt control by the Krylov error estimate (0 disables)."""
        self._check(self.lib.pcexp_set_krylov_tol(self.ctx, float(tol)), "set_krylov_tol")

    def set_krylov_adapt(self, check_every):
        """Adaptive Krylov dimension: with a tolerance set, check the estimate every
        `check_every` Arnoldi iterations and stop once it is met (0 disables)."""
        self._check(self.lib.pcexp_set_krylov_adapt(self.ctx, int(check_every)), "set_krylov_adapt")

    def steady(self, u, cfl_max=1000.0, tol=1e-10, max_iter=500, check_every=10, m=30, scheme="pcexp",
               prec="f64", jvp="tangent"):
        """Pseudo-time iteration with the CFL ramp of eq. (cfl), u updated in place; returns the info dict."""
        if not (u.is_cuda and u.dtype == self.torch.float64 and u.is_contiguous()):
            raise ValueError("steady updates u in place: pass a contiguous float64 device tensor")
        ws, nbytes = self.workspace(m, 1, prec, jvp)
        inf = SteadyInfo()
        self._check(self.lib.pcexp_steady(self.ctx, _ptr(u), float(cfl_max), float(tol), int(max_iter),
                                          int(check_every), m, SCHEME[scheme], PREC[prec], JVP[jvp], _ptr(ws),
                                          nbytes, ctypes.byref(inf), self._stream()), "steady")
        return inf.as_dict()

    def step_etd2(self, u, u_prev, r_prev, have_prev, dt, m=30, jvp="tangent", info=False):
        """ETD2 step (eq. (s7)) in place; u_prev / r_prev hold u_{n-1}, R(u_{n-1})
        when have_prev and are refreshed with u_n, R(u_n) (all contiguous FP64
        device tensors of the state's shape)."""
        for t in (u, u_prev, r_prev):
            if not (t.is_cuda and t.dtype == self.torch.float64 and t.is_contiguous()):
                raise ValueError("step_etd2: pass contiguous float64 device tensors")
        ws, nbytes = self.workspace(m, 1, "f64", jvp)
        inf = StepInfo()
        self._check(self.lib.pcexp_step_etd2(self.ctx, _ptr(u), _ptr(u_prev), _ptr(r_prev), int(bool(have_prev)),
                                             float(dt), m, JVP[jvp], _ptr(ws), nbytes,
                                             ctypes.byref(inf) if info else None, self._stream()), "step_etd2")
        return inf.as_dict() if info else None

    def advance(self, u, nsteps, dt=0.0, cfl=0.0, m=30, scheme="pcexp", prec="f64", jvp="tangent", info=False):
        """nsteps steps in place with u in the internal basis between them
        (u must be a contiguous FP64 device tensor); info describes the last step."""
        if not (u.is_cuda and u.dtype == self.torch.float64 and u.is_contiguous()):
            raise ValueError("advance updates u in place: pass a contiguous float64 device tensor")
        ws, nbytes = self.workspace(m, 1, prec, jvp)
        inf = StepInfo()
        self._check(self.lib.pcexp_advance(self.ctx, _ptr(u), int(nsteps), float(dt), float(cfl), m, SCHEME[scheme],
                                           PREC[prec], JVP[jvp], _ptr(ws), nbytes,
                                           ctypes.byref(inf) if info else None, self._stream()), "advance")
        return inf.as_dict() if info else None

    def step_noalloc(self, u, dt=0.0, cfl=0.0, m=30, scheme="pcexp", prec="f64", jvp="tangent", info=False):
        """pcexp_step with the library's fixed per-GPU workspace (no allocation
        by the call or by this method)."""
        if not (u.is_cuda and u.dtype == self.torch.float64 and u.is_contiguous()):
            raise ValueError("step_noalloc updates u in place: pass a contiguous float64 device tensor")
        inf = StepInfo()
        self._check(self.lib.pcexp_step_noalloc(self.ctx, _ptr(u), float(dt), float(cfl), m, SCHEME[scheme],
                                                PREC[prec], JVP[jvp], ctypes.byref(inf) if info else None,
                                                self._stream()), "step_noalloc")
        return inf.as_dict() if info else None

    def step(self, u, dt=0.0, cfl=0.0, m=30, scheme="pcexp", prec="f64", jvp="tangent", info=False):
        """u_n -> u_{n+1} in place (u must be a contiguous FP64 device tensor)."""
        if not (u.is_cuda and u.dtype == self.torch.float64 and u.is_contiguous()):
            raise ValueError("step updates u in place: pass a contiguous float64 device tensor")
        ws, nbytes = self.workspace(m, 1, prec, jvp)
        inf = StepInfo()
        self._check(self.lib.pcexp_step(self.ctx, _ptr(u), float(dt), float(cfl), m, SCHEME[scheme], PREC[prec],
                                        JVP[jvp], _ptr(ws), nbytes, ctypes.byref(inf) if info else None,
                                        self._stream()), "step")
        return inf.as_dict() if info else None
