"""Host-only checks of the serving loop's bookkeeping, no GPU: the arena that
places request blocks inside the server's reserved HBM budget and the
admission rule (head-of-line requests keep their room, smaller ones pass
within the rest, nothing starves).  The C++ check program is built with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and run on a seeded
random workload."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "serve_host_check.cpp")
INC = os.path.join(ROOT, "paper_1505_01998_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ missing")
def test_arena_and_admission_under_sanitizers(tmp_path):
    exe = tmp_path / "serve_host_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-I", INC, "-o", str(exe), SRC], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "OK"
