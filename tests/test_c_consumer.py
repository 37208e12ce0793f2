"""The boundary is a plain C ABI: a C99 program that includes include/pwf.h compiles with
-Wall -Wextra -pedantic -Werror, links against libpwf.so and makes host-only calls (no GPU):
the version, the status strings, the rejection of an unsupported grid and of a null
batch, and the tile settings."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2503_20146_amd")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "pwf.h"

int main(void) {
  pwf_problem p;
  memset(&p, 0, sizeof(p));
  p.geom.nx = 100;                 /* not a supported side */
  p.geom.ny = 100;
  p.geom.pixel_m = 1e-6;
  p.geom.wavelength_m = 5e-11;
  p.geom.z1_m = 5e-3;
  p.geom.z2_m = 0.2;
  printf("version %d\n", (int)pwf_version());
  printf("size %s\n", pwf_status_string(PWF_ERR_SIZE));
  printf("workspace %lu\n", (unsigned long)pwf_workspace_size(&p, 1));
  printf("null_batch %lu\n", (unsigned long)pwf_workspace_size(NULL, 0));
  printf("bad_tile %d\n", (int)pwf_set_column_tile(1024, -1, 3));
  printf("tile %d\n", (int)pwf_column_tile(1024, 11));
  return 0;
}
"""


def test_c_program_uses_the_library(tmp_path):
    gcc = shutil.which("gcc")
    lib = os.path.join(PKG, "libpwf.so")
    if gcc is None or not os.path.exists(lib):
        pytest.skip("gcc or the built library missing")
    src = tmp_path / "consumer.c"
    src.write_text(PROGRAM)
    exe = str(tmp_path / "consumer")
    res = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                          "-I", os.path.join(ROOT, "include"), str(src), "-o", exe,
                          "-L", PKG, "-lpwf", f"-Wl,-rpath,{PKG}"], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    got = dict(line.split(" ", 1) for line in out.stdout.strip().splitlines())
    assert int(got["version"]) >= 10000
    assert "unsupported grid size" in got["size"]
    assert got["workspace"] == "0" and got["null_batch"] == "0"
    assert got["bad_tile"] == "-1"
    assert got["tile"] == "16"
