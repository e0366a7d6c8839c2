"""Compile the HIP sources into the in-tree shared library libsesm.so (gfx950).

The library exposes only the C ABI declared in include/sesm.h; it links the
HIP runtime and nothing from PyTorch.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsesm.so")
SOURCES = ["sesm_core.hip", "sesm_dense.hip", "sesm_gmres.hip", "sesm_accel.hip", "sesm_field.hip",
           "sesm_adjoint.hip"]
ARCH = os.environ.get("SESM_OFFLOAD_ARCH", "gfx950")


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-shared", "-fPIC", "-pthread",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-fvisibility=hidden", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", LIB + ".tmp"] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if out.strip() and verbose:
        print(out)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
