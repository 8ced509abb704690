"""Host-only C++ test of the autotuner's tuning-cache reader and writer
(csrc/tuning_cache.hpp), compiled with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run on the CPU."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tuning_cache_under_sanitizers(tmp_path):
    exe = tmp_path / "tuning_cache_test"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{ROOT / 'paper_2003_01282_amd' / 'csrc'}",
           str(ROOT / "tests" / "native" / "tuning_cache_test.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, timeout=120,
                       env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "PATH": "/usr/bin:/bin"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok (0 failures)" in r.stdout
