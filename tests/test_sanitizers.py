"""AddressSanitizer + UndefinedBehaviorSanitizer builds, on the CPU, of
  * the C oracle (oracle.c, march.c, shade.c), driven by tests/c/oracle_sanitize.c
    over thousands of small random maps and rays, and
  * the library's HIP-free planning layer (csrc/tc_plan.cpp: column, view
    and edit validation, map layout, upload-table layout), driven by
    tests/c/plan_sanitize.cpp over random and invalid inputs.
Any memory error or undefined behaviour aborts the driver; the drivers also
check that the entry points agree with each other and that every planned
table fits its buffer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(tmp_path, compiler, flags, sources, args):
    if shutil.which(compiler) is None:
        pytest.skip("%s not available" % compiler)
    exe = str(tmp_path / "driver")
    subprocess.check_call([compiler] + flags + SAN + ["-o", exe] + sources)
    r = subprocess.run([exe] + args, capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout, r.stdout
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    o = os.path.join(ROOT, "oracle")
    out = _build_and_run(
        tmp_path, "gcc", ["-std=gnu11", "-ffp-contract=off", "-pthread"],
        [os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"), os.path.join(o, "oracle.c"),
         os.path.join(o, "march.c"), os.path.join(o, "shade.c"), "-lm"],
        ["3000", "20261203"])
    print(out)


def test_planning_layer_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2608_17390_amd", "csrc")
    out = _build_and_run(
        tmp_path, "g++", ["-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + csrc],
        [os.path.join(ROOT, "tests", "c", "plan_sanitize.cpp"), os.path.join(csrc, "tc_plan.cpp")],
        ["5000", "20261203"])
    print(out)
