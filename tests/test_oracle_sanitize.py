"""The oracle's C code under the address and undefined-behaviour sanitizers
(host build with gcc): a driver runs every routine on small inputs, with
conversion round trips and solver convergence checked, and any invalid
access, leak or undefined arithmetic ends the run with an error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    srcs = [os.path.join(ROOT, "tests", "oracle_sanitize.c"),
            os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "selector.c")]
    flags = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cc = subprocess.run(["gcc"] + flags + srcs + ["-lm", "-o", exe], capture_output=True, text=True)
    if cc.returncode != 0 and "asan" in cc.stderr.lower():
        pytest.skip("sanitizer runtime not installed: " + cc.stderr[-200:])
    assert cc.returncode == 0, cc.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "oracle sanitize run ok" in run.stdout
