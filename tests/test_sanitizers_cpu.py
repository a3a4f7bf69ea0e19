"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds tests/sanitize_driver.cpp with the library's host analysis
(paper_2306_14337_amd/csrc/analyze.cpp) and the oracle (oracle/oracle.c)
using gcc/g++ -fsanitize=address,undefined (no recovery), and runs it: the
analysis, the batch merge, CSR validation and every oracle phase on seeded
random matrices of many shapes.  Any memory error or undefined behaviour
aborts the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-ffp-contract=off", "-mfma"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                    reason="no host compilers")
def test_host_code_under_sanitizers(tmp_path):
    ana = tmp_path / "analyze.o"
    ora = tmp_path / "oracle.o"
    drv = tmp_path / "driver.o"
    exe = tmp_path / "sanitize_driver"
    run = lambda cmd: subprocess.run(cmd, check=True, capture_output=True, text=True)  # noqa: E731
    run(["g++", "-std=c++17", *FLAGS, "-c",
         os.path.join(ROOT, "paper_2306_14337_amd", "csrc", "analyze.cpp"), "-o", str(ana)])
    run(["gcc", "-std=c11", *FLAGS, "-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(ora)])
    run(["g++", "-std=c++17", *FLAGS, "-c", os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
         "-o", str(drv)])
    run(["g++", *FLAGS, str(drv), str(ana), str(ora), "-o", str(exe), "-pthread", "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert res.stdout.strip().startswith("ok"), res.stdout
    print(res.stdout.strip())
