"""The external sorts' parallel host copy (csrc/host_copy.h), built with g++
and ThreadSanitizer on the host: byte-exact copies of many sizes with the
thread team reused between copies, and no data race reported."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_copy_team_exact_and_race_free(tmp_path):
    exe = str(tmp_path / "host_copy_check")
    src = os.path.join(HERE, "native", "host_copy_check.cpp")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-pthread", "-o", exe, src], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env={**os.environ, "TSAN_OPTIONS": "halt_on_error=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
    assert "WARNING: ThreadSanitizer" not in r.stderr
