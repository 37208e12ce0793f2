"""Host-side AddressSanitizer and UndefinedBehaviorSanitizer run of the C ABI (no GPU).

The API and tomography translation units, which hold the library's host code
(argument validation, workspace layout, batch grouping, tuning settings, the
host fits), are rebuilt with both sanitizers on their host pass only and
linked with the device objects of the regular build; the ABI tests then run
against that library in a child process with the compiler's ASan runtime
(which carries the UBSan handlers) preloaded.  A heap or stack overflow, use
after free, double free, signed overflow, misaligned or null access, or
out-of-range shift in any host path those tests reach fails this test with
the sanitizer's report.
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2503_20146_amd import build as B  # noqa: E402

HOST_UNITS = ("pwf_api.hip", "pwf_tomo.hip")


def _asan_runtime() -> str | None:
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.timeout(900)
def test_abi_suite_under_host_asan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime in the ROCm LLVM tree")
    objs = sorted(glob.glob(os.path.join(B.BUILD, "*.o")))
    names = {os.path.basename(o) for o in objs}
    if not {os.path.basename(s)[:-4] + ".o" for s in B.sources()} <= names:
        pytest.skip("regular build objects missing (run __graft_entry__.build() first)")
    hipcc = B._hipcc()
    linked = [o for o in objs if os.path.basename(o)[:-2] + ".hip" not in HOST_UNITS]
    for unit in HOST_UNITS:
        out = str(tmp_path / (unit[:-4] + ".o"))
        cmd = [hipcc, *B.FLAGS, "-O1", "-g",
               "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
               "-c", os.path.join(B.CSRC, unit), "-o", out]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        linked.append(out)
    lib = str(tmp_path / "libpwf_asan.so")
    # the sanitizer's symbols resolve against the preloaded runtime at load time
    res = subprocess.run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-o", lib, *linked],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]

    driver = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2503_20146_amd._lib as L\n"
        "L.LIB_PATH = %r\n"
        "import pytest\n"
        "sys.exit(pytest.main(['-q', '-x', '-m', 'not gpu', '-p', 'no:cacheprovider', %r]))\n"
    ) % (ROOT, lib, os.path.join(ROOT, "tests", "test_abi.py"))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-c", driver], capture_output=True, text=True, env=env, cwd=ROOT,
                         timeout=600)
    report = res.stdout[-4000:] + res.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in report, report
    assert "runtime error:" not in report, report
    assert res.returncode == 0, report
    assert " passed" in res.stdout, report
