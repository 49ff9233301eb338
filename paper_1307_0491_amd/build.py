"""Build step of the HIP library: compiles every source under csrc/ for
gfx950 (one hipcc process per source, objects under _build/) and links
paper_1307_0491_amd/libsve.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsve.so")
SOURCES = ["sve_api.hip", "sve_adjoint.hip", "sve_ensemble.hip", "sve_noalloc.hip",
           "sve_order2.hip", "sve_fused1d.hip"]
COMPILE_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-Wno-unused-result"]
LINK_FLAGS = ["--offload-arch=gfx950", "-fPIC", "-shared"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    procs = []
    for src, obj in zip(srcs, objs):
        cmd = [hipcc(), *COMPILE_FLAGS, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                      text=True))
    failed = False
    for p in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(err)
            failed = True
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    cmd = [hipcc(), *LINK_FLAGS, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
