"""The boundary header is plain C: a C99 program that includes include/hmc.h compiles with
every warning as an error, links against the built library and calls its host-side entry
points (no GPU needed: these calls do no device work)."""
import os
import shutil
import subprocess

import pytest

import paper_1402_4089_amd as hmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "hmc.h"

int main(void) {
  hmc_problem prob;
  size_t bytes = 0;
  memset(&prob, 0, sizeof prob);
  prob.n = 100; prob.p = 0; prob.K = 3; prob.xfmt = HMC_X_F32; prob.ldx = 8;
  /* p = 0 is a shape error, reported on the host before any device work */
  hmc_status st = hmc_workspace_bytes(&prob, &bytes);
  printf("%lld %d %s\n", (long long)hmc_max_p(HMC_X_F32, 10), (int)st, hmc_status_string(st));
  return st == HMC_ERR_SHAPE ? 0 : 1;
}
"""


def test_header_compiles_as_c99_and_links(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(hmc.LIB_PATH):
        pytest.fail("libhmc.so is not built: run python -m paper_1402_4089_amd.build")
    src = tmp_path / "prog.c"
    src.write_text(PROGRAM)
    libdir = os.path.dirname(hmc.LIB_PATH)
    exe = tmp_path / "prog"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I", os.path.join(ROOT, "include"), str(src), "-L", libdir, "-lhmc",
                        f"-Wl,-rpath,{libdir}", "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    max_p, status, msg = r.stdout.split(maxsplit=2)
    assert int(max_p) == hmc.hmc_max_p(hmc.HMC_X_F32, 10) and int(status) == -2 and msg.strip()
