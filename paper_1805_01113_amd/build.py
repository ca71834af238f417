"""Build the HIP library libmls_hip.so in-tree for gfx950 (hipcc)."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmls_hip.so")
SOURCES = ["mls_api.hip", "mls_build.hip", "mls_transfer.hip", "mls_step.hip", "mls_mlp.hip", "mls_tune.hip",
           "mls_collide.hip", "mls_refine.hip", "mls_grad.hip"]

# -packed-fp32-ops: no packed FP32 instructions are generated (plain VALU FP32)
COMPILE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-fast-math", "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
]


def source_sha256() -> str:
    """SHA-256 over the library's HIP sources and the C-ABI header, file by
    file in name order (name, then contents).  build() stamps it into
    mls_version(), so a loaded library names the sources it was built from."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*"))) + [os.path.join(ROOT, "include", "mls.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose: bool = True, jobs: int = 4) -> str:
    """Compile every source to an object (in parallel) and link the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    stamp = ["-DMLS_SOURCE_SHA256=\"%s\"" % source_sha256()]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = ["hipcc", *COMPILE_FLAGS, *stamp, "-c", *inc, os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode(errors="replace"))
            raise RuntimeError("hipcc failed on %s" % src)
        if verbose and out.strip():
            sys.stderr.write(out.decode(errors="replace"))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
