"""Host C/C++ code under AddressSanitizer + UndefinedBehaviorSanitizer: the
exact-state codec of the library (host-only code) and the oracle's binned C
sum, driven by tests/sanitize_host.cpp.  Built with g++/gcc for the CPU only;
no device code is involved."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_host_code_is_clean_under_sanitizers(tmp_path):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no host compiler")
    obj = str(tmp_path / "bins.o")
    exe = str(tmp_path / "sanitize_host")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-c", os.path.join(ROOT, "oracle", "bins.c"),
                    "-o", obj] + SAN, check=True)
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-I" + os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize_host.cpp"),
                    "-x", "c++", os.path.join(ROOT, "paper_1605_05436_amd", "csrc", "xsum_state.hip"),
                    "-x", "none", obj, "-o", exe, "-lpthread"] + SAN, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("OK")
