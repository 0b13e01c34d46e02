"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code that
runs without a GPU (CPU only, gcc/g++):

* the oracle (oracle/oracle.c) driven through every entry point on small
  shapes and edge cases, with exactly sized heap buffers
  (tests/sanitize/oracle_driver.c);
* the library's plan-cache reader (paper_1710_11593_amd/csrc/plan.hip, pure
  host C++) fed malformed and mutated cache files
  (tests/sanitize/plan_driver.cpp).

Each is compiled with -fsanitize=address,undefined -fno-sanitize-recover=all,
so any report ends the program with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, cwd, timeout=300):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=ENV)
    return r.returncode, r.stdout + r.stderr


@pytest.fixture(scope="module")
def sanitizers(tmp_path_factory):
    cc, cxx = shutil.which("gcc"), shutil.which("g++")
    if not cc or not cxx:
        pytest.skip("gcc / g++ not available")
    d = tmp_path_factory.mktemp("san")
    probe = d / "probe.c"
    probe.write_text("int main(void) { return 0; }\n")
    rc, out = _run([cc] + SAN + ["-o", str(d / "probe"), str(probe)], str(d))
    if rc != 0:
        pytest.skip("compiler without sanitizer runtimes: " + out[-300:])
    return cc, cxx, d


def test_oracle_under_asan_ubsan(sanitizers):
    cc, _, d = sanitizers
    exe = str(d / "oracle_san")
    rc, out = _run([cc] + SAN + ["-o", exe, os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                                 os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], str(d))
    assert rc == 0, out
    rc, out = _run([exe], str(d))
    assert rc == 0 and "all calls clean" in out, out


def test_plan_reader_under_asan_ubsan(sanitizers):
    _, cxx, d = sanitizers
    exe = str(d / "plan_san")
    rc, out = _run([cxx] + SAN + ["-std=c++17", "-o", exe, os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"),
                                  "-x", "c++", os.path.join(ROOT, "paper_1710_11593_amd", "csrc", "plan.hip")],
                   str(d))
    assert rc == 0, out
    rc, out = _run([exe, str(d)], str(d))
    assert rc == 0 and "all cases clean" in out, out
