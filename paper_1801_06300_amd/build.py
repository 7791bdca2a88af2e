"""Build libpcexp.so (HIP for gfx950) in-tree.

Every HIP translation unit is compiled with hipcc for gfx950 with packed FP32
instructions disabled; the object files are linked into
``paper_1801_06300_amd/libpcexp.so``.  Compilation runs in parallel.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpcexp.so")
PROBE = os.path.join(HERE, "libpcexp_setup_probe.so")

HIP_SOURCES = ["pcexp.hip", "dg2.hip", "dg3.hip", "krylov_kernels.hip", "elem_kernels.hip"]
HOST_SOURCES = ["setup.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run_parallel(cmds, verbose):
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 target feature: harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append((cmd, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + t for c, t in failed)
        raise RuntimeError("libpcexp build failed:\n" + msg)


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    objs, cmds = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(OUT_DIR, src + ".o")
        objs.append(obj)
        cmds.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    for src in HOST_SOURCES:
        obj = os.path.join(OUT_DIR, src + ".o")
        objs.append(obj)
        cmds.append(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    probe_obj = os.path.join(OUT_DIR, "setup_probe.cpp.o")
    cmds.append(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, "setup_probe.cpp"), "-o", probe_obj])
    _run_parallel(cmds, verbose)
    tmp = LIB + ".tmp"
    _run_parallel([[HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]],
                  verbose)
    os.replace(tmp, LIB)
    tmp = PROBE + ".tmp"
    _run_parallel([["g++", "-shared", "-fPIC", "-o", tmp, probe_obj,
                    os.path.join(OUT_DIR, "setup.cpp.o"), "-lpthread"]], verbose)
    os.replace(tmp, PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
