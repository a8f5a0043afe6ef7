"""libmgr's host code under the host sanitizers: every source is compiled
with AddressSanitizer and UBSan on its host side only (the device code is
built as usual), linked with tests/lib_host_driver.cpp, and the driver runs
every path that needs no device: option defaults and validation, the argument
checks of every entry point, status strings and the per-thread error text.
It must exit cleanly with no sanitizer report.  CPU only (the library loads
without a GPU; none of these calls reaches one)."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1801_08464_amd", "csrc")
SOURCES = ["k_util.hip", "k_setup.hip", "k_fine.hip", "k_solve.hip", "k_krylov.hip", "k_ncp.hip", "mgr_host.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
# sanitizers on the host half of each compile and link only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang++ not installed")
    out = tmp_path_factory.mktemp("host_asan")
    inc = os.path.join(ROOT, "include")

    def compile_one(src):
        obj = str(out / src.replace(".hip", ".o"))
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN, "-I", inc, "-c",
               os.path.join(CSRC, src), "-o", obj]
        subprocess.run(cmd, check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(4) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv_o = str(out / "lib_host_driver.o")
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", inc, "-c", os.path.join(ROOT, "tests", "lib_host_driver.cpp"), "-o", drv_o],
                   check=True, capture_output=True)
    exe = str(out / "lib_host_driver")
    subprocess.run([HIPCC, "--hip-link", "--offload-arch=gfx950", *HOST_SAN[:4], drv_o, *objs, "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_library_host_paths_clean_under_asan_and_ubsan(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=97",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
    p = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    report = p.stdout + p.stderr
    assert p.returncode == 0, report[-4000:]
    assert "host paths ok" in p.stdout
    assert "runtime error" not in report and "AddressSanitizer" not in report and "LeakSanitizer" not in report, \
        report[-4000:]
