"""The host term-list builder under AddressSanitizer, UBSan and LeakSanitizer:
termlist.cpp (plain C++, no device code) and a driver that calls the term-list
C ABI (tests/host_sanitize_driver.cpp) are compiled with g++ and run; any
memory error, undefined behaviour or leak fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_term_list_builder_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1301_4895_amd", "csrc"),
           os.path.join(ROOT, "paper_1301_4895_amd", "csrc", "termlist.cpp"),
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", exe]
    built = subprocess.run(cmd, capture_output=True, text=True)
    if built.returncode != 0 and "sanitizer" in built.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + built.stderr[-300:])
    assert built.returncode == 0, built.stderr[-2000:]
    # the environment is passed on unchanged apart from the sanitizer options
    # (a library preloaded by the environment may precede the ASan runtime)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert run.stdout.rstrip().endswith("done"), out[-2000:]
    # the invalid inputs were refused, the valid ones built
    assert "n_src must be 1, 2 or 3" in out and "at most one Lambda" in out
    assert "Lambda + p + n NR" in out and "3n NR 3src" in out and "(loaded)" in out
