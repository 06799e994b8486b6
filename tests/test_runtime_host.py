"""Host-only parts of the batch and server runtime, built with g++ from the
same header the library uses: the first-fit arena that admits requests into a
server's device budget, and the longest-first stream assignment of batches."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_and_stream_assignment(tmp_path):
    exe = tmp_path / "runtime_host_check"
    src = os.path.join(ROOT, "tests", "host", "runtime_host_check.cpp")
    inc = os.path.join(ROOT, "paper_1402_1720_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", inc, src, "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"
