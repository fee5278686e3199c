"""The library's host-side planning (argument checks, workspace layout,
traversal orders, coarse block tables, the autotuner's shape cache and its
file format: paper_2103_05034_amd/csrc/plan.cpp)
built with AddressSanitizer and UBSan into a host program that exercises it on
many shapes and edge inputs; then the planned workspace sizes against what
libdwf.so reports for the same shapes (the library links the same source)."""

import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2103_05034_amd", "csrc")


@pytest.fixture(scope="module")
def checks_output(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("host_san") / "plan_checks"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "plan.cpp"), os.path.join(ROOT, "tests", "host", "plan_checks.cpp"),
           "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(out), str(out.parent)], capture_output=True, text=True, env=env, timeout=120)
    return run


def test_plan_checks_clean_under_sanitizers(checks_output):
    r = checks_output
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "all checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]


def test_planned_totals_match_library(checks_output):
    import paper_2103_05034_amd as dwf

    if not os.path.exists(dwf.LIB_PATH):
        from paper_2103_05034_amd import build

        build.build()
    lib = dwf.load_library()
    fn = lib.dwf_workspace_bytes
    rows = [line.split()[1:] for line in checks_output.stdout.splitlines() if line.startswith("total ")]
    assert len(rows) > 100
    for row in rows:
        X, Y, Z, T, Ls, prec, max_nrhs, max_cg_rhs, total = (int(v) for v in row)
        dims = (ctypes.c_int * 4)(X, Y, Z, T)
        assert fn(dims, Ls, prec, max_nrhs, max_cg_rhs) == total, row
