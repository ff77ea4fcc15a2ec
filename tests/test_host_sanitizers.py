"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the regular-expression text front end
and the compiler (random and malformed patterns and ASTs), and the C oracle (single- and multi-threaded runs
that must agree).  Built with the host compilers only (g++ / gcc); no device code is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1108_3126_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_front_end_compiler_and_oracle_under_sanitizers(tmp_path):
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "driver")
    subprocess.run(["gcc", "-std=c11", *SAN, "-c", os.path.join(ROOT, "oracle", "rx_oracle.c"), "-o", obj],
                   check=True, capture_output=True, text=True)
    r = subprocess.run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        os.path.join(ROOT, "tests", "sanitize_driver.cpp"), os.path.join(CSRC, "rx_compile.cpp"),
                        os.path.join(CSRC, "rx_parse.cpp"), obj, "-pthread", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert run.stdout.startswith("ok "), run.stdout
