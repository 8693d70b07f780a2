"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle's whole C interface on many small inputs, and the C-ABI argument
checks on valid and invalid arguments.  Each driver prints "ok"; any
sanitizer report aborts it (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, exe):
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300, env=env)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout[-3000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    _run(["gcc", *SAN, "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=gnu11", "-o", exe,
          os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"), os.path.join(ROOT, "oracle", "lw_oracle.c"),
          "-lm"], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_abi_argument_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "validate_check")
    csrc = os.path.join(ROOT, "paper_1709_06816_amd", "csrc")
    _run(["g++", *SAN, "-std=c++17", "-I", csrc, "-I", os.path.join(ROOT, "include"), "-o", exe,
          os.path.join(ROOT, "tests", "native", "validate_check.cpp"), os.path.join(csrc, "hac_validate.cpp")], exe)
