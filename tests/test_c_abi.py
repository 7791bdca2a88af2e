"""The library driven from plain C (tests/c/pcexp_c_driver.c): the C ABI of
include/pcexp.h with device memory from the HIP runtime's C interface, no
Python or torch in the caller.  The CPU test compiles and links the driver
with gcc; the GPU test runs it on a 4x4 jittered periodic P2 Roe mesh and
compares its residual and one FP64 tangent PCEXP step with the oracle (the
residual of eq. (euler3) and eqs. (s9)-(s10)) at the FP64 bar 1e-11."""

import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1801_06300_amd")
SRC = os.path.join(ROOT, "tests", "c", "pcexp_c_driver.c")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(out):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    if not os.path.exists(os.path.join(LIBDIR, "libpcexp.so")):
        pytest.skip("libpcexp.so not built")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}", SRC, f"-L{LIBDIR}", "-lpcexp",
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{ROCM}/lib", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr


def test_c_driver_compiles_and_links(tmp_path):
    exe = str(tmp_path / "pcexp_c_driver")
    _compile(exe)
    assert os.path.exists(exe)


@pytest.mark.gpu
def test_c_driver_matches_oracle(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from oracle.dg import DG
    from oracle.integrators import ExactJacobian, pcexp_step, stable_dt

    exe = str(tmp_path / "pcexp_c_driver")
    _compile(exe)
    mesh = W.periodic_square(4, 10.0, 0.15, 3)
    g = DG(mesh, 2, "roe")
    u0 = g.project(lambda x: W.isentropic_vortex(x, center=(5.0, 5.0), period=mesh.period))
    u0 = u0 + W.perturbation(u0.shape, 101, 1e-6)
    dt = stable_dt(g, u0, 5.0)
    m = 8
    vert = np.ascontiguousarray(mesh.vert, np.float64)
    elem = np.ascontiguousarray(mesh.elem, np.int32)
    canon = None if mesh.vert_canon is None else np.ascontiguousarray(mesh.vert_canon, np.int32)
    u = np.ascontiguousarray(u0, np.float64).ravel()
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(inp, "wb") as f:
        f.write(struct.pack("=iq", mesh.dim, vert.shape[0]))
        f.write(vert.tobytes())
        f.write(struct.pack("=q", elem.shape[0]))
        f.write(elem.tobytes())
        f.write(struct.pack("=i", 0 if canon is None else 1))
        if canon is not None:
            f.write(canon.tobytes())
        f.write(struct.pack("=iidq", 2, 1, 1.4, u.size))
        f.write(u.tobytes())
        f.write(struct.pack("=di", dt, m))
    print(f"\n[case] C driver: 4x4 jittered periodic P2 Roe, K={u.size}, dt={dt:.3e}, m={m}", flush=True)
    r = subprocess.run([exe, inp, outp], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(outp, "rb").read()
    K = u.size
    R = np.frombuffer(raw, np.float64, K, 0).reshape(u0.shape)
    un = np.frombuffer(raw, np.float64, K, 8 * K).reshape(u0.shape)
    m1, m2 = struct.unpack_from("=ii", raw, 16 * K)
    Ro = g.residual(u0)
    want = pcexp_step(ExactJacobian(g), u0, dt, m)
    e_res = np.linalg.norm(R - Ro) / np.linalg.norm(Ro)
    e_step = np.linalg.norm(un - want) / np.linalg.norm(want)
    print(f"[c-abi] residual rel err {e_res:.2e}, step rel err {e_step:.2e}, m_eff {m1},{m2}", flush=True)
    assert m1 == m and m2 == m
    assert e_res < 1e-11 and e_step < 1e-11
