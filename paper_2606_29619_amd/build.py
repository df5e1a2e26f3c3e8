"""Build step of the HIP library: hipcc for gfx950 over the solver (differenced and analytic
porosity-derivative halves) and the request-server sources, compiled in parallel and then
linked; in-tree output."""
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRCS = [os.path.join(PKG, "csrc", f) for f in ("lbm.hip", "lbm_analytic.hip", "lbm_server.hip")]
LIB = os.path.join(PKG, "liblbm.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    # expressions are evaluated exactly as written (FP64 results match the CPU reference)
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile every source for gfx950 and link liblbm.so.  hipcc compiles the device code of
    a source first and its host code afterwards, reading the headers a second time; the
    sources are therefore copied to a private directory first, so that both halves (and all
    three sources) see the same text even if the tree changes while the build runs."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmpdir:
        src_dir = os.path.join(tmpdir, "csrc")
        inc_dir = os.path.join(tmpdir, "include")
        shutil.copytree(os.path.join(PKG, "csrc"), src_dir)
        shutil.copytree(os.path.join(ROOT, "include"), inc_dir)
        objs, procs = [], []
        for src in SRCS:
            name = os.path.basename(src)
            obj = os.path.join(tmpdir, os.path.splitext(name)[0] + ".o")
            cmd = [hipcc, *HIPCC_FLAGS, "-I", inc_dir, "-c", "-o", obj,
                   os.path.join(src_dir, name)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd))
            objs.append(obj)
        codes = [p.wait() for p in procs]
        if any(codes):
            raise subprocess.CalledProcessError(max(codes, key=abs), "hipcc -c")
        tmp = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
