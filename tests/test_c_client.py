"""The C ABI from a plain C99 program (tests/c_client/nsasm_client.c): it
compiles against include/nsasm.h and the HIP runtime API with gcc alone (CPU
test), and, on the GPU, its FP64 right-hand side and velocity VJP equal the
oracle's on a jittered, relabelled mesh."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2403_08777_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_client", "nsasm_client.c")
LIBDIR = os.path.join(ROOT, "paper_2403_08777_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(out_dir):
    exe = os.path.join(out_dir, "nsasm_client")
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", exe, f"-L{LIBDIR}", "-lnsasm",
           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_c_client_compiles(tmp_path):
    assert os.path.exists(os.path.join(LIBDIR, "libnsasm.so")), "build the library first"
    assert os.access(_compile(str(tmp_path)), os.X_OK)


@pytest.mark.gpu
def test_c_client_matches_oracle(tmp_path):
    exe = _compile(str(tmp_path))
    m = synth.cube_mesh(6, jitter=True, permute=True)
    u, p = synth.taylor_green(m)
    lam = synth.adjoint(m.n_nodes)
    rho, mu, cs, f = 1.3, 1e-2, 0.1, (0.1, -0.2, 0.3)
    d = str(tmp_path)
    for name, a, dt in (("coords", m.coords, np.float64), ("conn", m.conn, np.int32), ("u", u, np.float64),
                        ("p", p, np.float64), ("lam", lam, np.float64),
                        ("params", np.array([rho, mu, cs, *f]), np.float64)):
        np.ascontiguousarray(a, dtype=dt).tofile(os.path.join(d, f"{name}.bin"))
    r = subprocess.run([exe, d, str(m.n_nodes), str(m.n_elems)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rhs = np.fromfile(os.path.join(d, "rhs.bin"), dtype=np.float64).reshape(-1, 3)
    grad = np.fromfile(os.path.join(d, "grad.bin"), dtype=np.float64).reshape(-1, 3)
    prm = oracle.Params(rho, mu, cs, f)
    er = oracle.rel_l2(rhs, oracle.rhs(m.coords, m.conn, u, p, prm))
    eg = oracle.rel_l2(grad, oracle.vjp(m.coords, m.conn, u, lam, prm))
    print(f"C client: rhs rel_l2 {er:.2e}, vjp {eg:.2e}", flush=True)
    assert er <= 1e-12 and eg <= 1e-12
