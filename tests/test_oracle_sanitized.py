"""The oracle's C sources under the host sanitizers: a standalone driver
(oracle/sanitize_driver.c) built with gcc -fsanitize=address,undefined runs
every oracle entry point on a small seeded NCP system (the two-phase disk of
Section 6 on a 12x10 grid) under six option sets, and must exit cleanly with
no sanitizer report.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from conftest import ROOT
from synth import make_system

ORACLE = os.path.join(ROOT, "oracle")
SOURCES = ["sanitize_driver.c", "sparse.c", "amg.c", "mgr.c"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-Wall", "-Wno-unused-function", "-o", exe]
    cmd += [os.path.join(ORACLE, s) for s in SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True)
    return exe


def write_system(path, s, bs=3):
    with open(path, "wb") as f:
        np.array([s.n, s.nnz], dtype="<i8").tofile(f)
        np.array([bs], dtype="<i4").tofile(f)
        s.indptr.astype("<i8").tofile(f)
        s.indices.astype("<i4").tofile(f)
        s.data.astype("<f8").tofile(f)
        s.labels.astype("<i4").tofile(f)
        s.b.astype("<f8").tofile(f)


def run(driver, path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=97",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
    return subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=300)


@pytest.mark.parametrize("grid,frac,seed", [((12, 10), 0.4, 3), ((5, 4, 4), 0.35, 8)])
def test_oracle_is_clean_under_asan_and_ubsan(driver, tmp_path, grid, frac, seed):
    s = make_system(grid, 1.5, "disk" if len(grid) == 2 else "ball", frac, seed)
    assert (s.labels == 2).any() and (s.labels == 0).any()
    path = str(tmp_path / "sys.bin")
    write_system(path, s)
    p = run(driver, path)
    report = p.stderr
    assert p.returncode == 0, report[-4000:]
    assert "runtime error" not in report and "AddressSanitizer" not in report, report[-4000:]
    # all six option sets reached the end of their solve
    assert report.count("status ") == 6, report
