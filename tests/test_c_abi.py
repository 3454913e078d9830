"""The C ABI used from C alone: examples/c_taylor_green.c builds with the host
compiler against include/lbm.h and liblbm.so (CPU), and on a GPU its final
velocity field equals the Python binding's bit for bit (same kernels, same
inputs); the FP64 totals agree to their summation rounding (they are
accumulated with atomics, in no fixed order)."""

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "examples", "c_taylor_green.c")
PKG = os.path.join(ROOT, "paper_2107_14774_amd")
ROCM = "/opt/rocm"


def _build(out_dir):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.exists(os.path.join(PKG, "liblbm.so")):
        pytest.skip("no host C compiler or no built library")
    exe = os.path.join(out_dir, "c_taylor_green")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{ROOT}/include", SRC, f"-L{PKG}", "-llbm", f"-L{ROCM}/lib", "-lamdhip64",
           f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib", "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


def test_c_example_builds_against_the_header_and_library(tmp_path):
    assert os.access(_build(str(tmp_path)), os.X_OK)


@pytest.mark.gpu
def test_c_example_matches_python_binding(tmp_path):
    import paper_2107_14774_amd as P
    import workloads as W
    exe = _build(str(tmp_path))
    nx, ny, nz, steps = 64, 48, 32, 60
    u0 = np.ascontiguousarray(W.taylor_green(nx, ny, nz, 1.0, 0.5, 0.05)
                              + W.random_modes(nx, ny, nz, 1.0, 0.5, 3, 0.01, 81))
    ufile = os.path.join(str(tmp_path), "u0.bin")
    u0.astype(np.float64).tofile(ufile)
    print("running", exe, flush=True)
    uout = os.path.join(str(tmp_path), "u_final.bin")
    res = subprocess.run([exe, str(nx), str(ny), str(nz), str(steps), ufile, uout], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    c_sums = [float(v) for v in res.stdout.split()]
    c_u = torch.from_numpy(np.fromfile(uout, dtype=np.float32).reshape(3, nz, ny, nx))
    cs2, nu = 1.0 / 12.0, 0.016
    lat = P.Lattice(nx, ny, nz, r=1.0, s=0.5, cs2=cs2, omega_nu=1.0 / (nu / cs2 + 0.5),
                    omega_xi=1.0 / (1.5 * nu / cs2 + 0.5), storage="f32", corr="local")
    a, b = lat.new_state(), lat.new_state()
    lat.init(a, u=torch.from_numpy(u0).cuda())
    cur, _ = lat.step(a, b, steps)
    m = lat.moments(cur)
    py_sums = m.sums.cpu().tolist()
    print("C:", c_sums, "\nPython:", py_sums, flush=True)
    sys.stdout.flush()
    assert torch.equal(c_u, m.u.cpu())
    scale = [py_sums[0]] + [0.05 * py_sums[0]] * 3 + [py_sums[4]]
    for c, py, sc in zip(c_sums, py_sums, scale):
        assert abs(c - py) <= 1e-13 * sc
