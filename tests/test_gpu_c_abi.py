"""The C ABI used from C alone (GPU tier): tests/c_abi_gradient.c, built with the system C
compiler against include/hmc.h, the built library and the HIP runtime (no Python binding, no
torch in that process), evaluates the gradient of the n=20000, p=1000, K=10 FP32 workload on
the GPU; its log K and G must match the FP64 oracle at the FP32 parity bar, and a workspace one
byte short must be refused with HMC_ERR_WORKSPACE (the program checks that itself)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from gradbound import UNIT_ROUNDOFF, assert_elementwise
from workloads import make_problem, make_random_state

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_c_program_gradient_matches_oracle(lib, tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    libdir = os.path.dirname(lib.LIB_PATH)
    exe = tmp_path / "c_abi_gradient"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "c_abi_gradient.c"), "-L", libdir, "-lhmc",
                        "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{libdir}",
                        f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    prob = make_problem("c2_f32")
    B = make_random_state(prob, 0.05).astype(np.float32)
    inp, outp = tmp_path / "problem.bin", tmp_path / "result.bin"
    with open(inp, "wb") as fh:
        fh.write(np.array([prob.n, prob.p, prob.K], dtype=np.int64).tobytes())
        fh.write(np.ascontiguousarray(prob.X, dtype=np.float32).tobytes())
        fh.write(np.ascontiguousarray(prob.y, dtype=np.int32).tobytes())
        fh.write(np.ascontiguousarray(B).tobytes())
    print(f"[c abi] running {exe.name} on n={prob.n} p={prob.p} K={prob.K}", flush=True)
    r = subprocess.run([str(exe), str(inp), str(outp)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    print(f"[c abi] {r.stdout.strip()}", flush=True)
    raw = outp.read_bytes()
    logk = float(np.frombuffer(raw[:8], dtype=np.float64)[0])
    G = np.frombuffer(raw[8:], dtype=np.float32).reshape(prob.p, prob.K).astype(np.float64)
    B64 = B.astype(np.float64)
    lk_o, G_o = oracle.log_kernel_and_grad(prob.X64, prob.y, B64, prob.prior, prob.prior_scale, 1)
    err = float(np.linalg.norm(G - G_o) / np.linalg.norm(G_o))
    assert err <= 1e-5, f"gradient rel-L2 {err:.3e}"
    assert_elementwise(G, G_o, prob.X64, prob.y, B64, prob.prior, prob.prior_scale, 1,
                       UNIT_ROUNDOFF["f32"])
    assert abs(logk - lk_o) <= 1e-6 * abs(lk_o)
    assert np.all(G[:, -1] == 0)
