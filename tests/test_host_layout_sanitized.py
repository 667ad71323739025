"""The host runtime's layout builder and input validation
(paper_1708_07954_amd/csrc/dba_layout.cpp, plain C++) built on the CPU with
g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on the
edge-case layouts of tests/host_layout_check.cpp, which checks every
invariant the kernels rely on.  No GPU involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_07954_amd", "csrc")


def test_layout_builder_under_address_and_ub_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "host_layout_check"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "dba_layout.cpp"), os.path.join(ROOT, "tests", "host_layout_check.cpp"), "-o", str(exe)]
    subprocess.check_call(cmd)
    # verify_asan_link_order=0: the environment may preload a library ahead
    # of the sanitizer runtime, which is left as it is
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.startswith("ok ")
