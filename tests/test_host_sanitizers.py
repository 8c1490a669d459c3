"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the oracle's C sources and the library's blocked cuckoo table
(paper_2001_08250_amd/csrc/cuckoo.cpp, the host working copy) with gcc/g++
and -fsanitize=address,undefined into one executable with the driver in
tests/sanitize/, runs it, and requires a clean exit: every check of the
driver passed and neither sanitizer reported anything (both abort on their
first report).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no gcc/g++")
def test_oracle_and_cuckoo_table_under_sanitizers(tmp_path):
    objs = []
    for src in ("pir_oracle.c", "cuckoo_oracle.c", "mask_oracle.c", "codec_oracle.c"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run(["gcc", "-std=c11", "-pthread", *SAN, "-c", os.path.join(ROOT, "oracle", src), "-o", obj],
                       check=True)
        objs.append(obj)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    for src in (os.path.join(ROOT, "paper_2001_08250_amd", "csrc", "cuckoo.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", "-std=c++17", *SAN, *inc, "-c", src, "-o", obj], check=True)
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    subprocess.run(["g++", *SAN, "-pthread", "-o", exe, *objs], check=True)
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = run.stdout + run.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert run.returncode == 0, report[-4000:]
    assert "host driver: ok" in run.stdout
