"""Build ``libnis.so`` (the HIP library behind include/nis.h) for gfx950.

Each source is compiled with hipcc for gfx950 only; the host runtime file is
compiled with -ffp-contract=off (its double-precision set-up values must be
rounded term by term), the kernels with -O3.  Packed FP32 instructions are
disabled for all device code.  Objects are compiled in parallel and linked
into ``paper_2401_14051_amd/libnis.so``.
"""

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libnis.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["--offload-arch=" + ARCH, "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
SOURCES = {
    "nis_api.cpp": ["-O2", "-ffp-contract=off", "-x", "hip"],
    "server.cpp": ["-O2", "-ffp-contract=off", "-x", "hip"],
    "k_frame.hip": ["-O3"],
    "k_volume.hip": ["-O3"],
    "k_features.hip": ["-O3"],
    "k_mlp.hip": ["-O3"],
    "k_modules.hip": ["-O3"],
}


def _compile(src, extra):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    return obj, out


def build(verbose=False):
    """Compile every source and link libnis.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        futs = [ex.submit(_compile, s, e) for s, e in SOURCES.items()]
        objs = []
        for f in futs:
            obj, out = f.result()
            if verbose and out.strip():
                print(out, file=sys.stderr)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
