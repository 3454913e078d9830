"""Build the HIP library ``liblbm.so`` for gfx950 (in-tree, next to this file).

    python -m paper_2107_14774_amd.build

Every source under ``csrc/`` is compiled with hipcc for gfx950 and linked
into one shared library exposing the C ABI of ``include/lbm.h``.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ("lbm_api.hip", "lbm_forward.hip", "lbm_adjoint.hip",
           "lbm_step_f32.hip", "lbm_step_f16.hip", "lbm_step_bf16.hip", "lbm_step_bf16sr.hip",
           "lbm_adjoint_step_f32.hip", "lbm_adjoint_step_f16.hip", "lbm_adjoint_step_bf16.hip")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=True, jobs=None):
    """Compile every source in parallel, then link liblbm.so.  Always rebuilds."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for src, pr in procs:
        out, _ = pr.communicate()
        if out and (pr.returncode != 0 or verbose):
            sys.stdout.write(out.decode(errors="replace"))
        if pr.returncode != 0:
            failed = True
            print("compile failed:", src, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
