"""The octree builder's host thread pool (csrc/hostpool.h), compiled on its
own with the host compiler: coverage of [0, n) around the chunk and
single-call boundaries, exceptions rethrown on the caller, concurrent
callers serialised."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1503_04544_amd", "csrc")


def test_hostpool(tmp_path):
    exe = tmp_path / "hostpool_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", CSRC, os.path.join(HERE, "hostpool_check.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr


def test_hostpool_thread_sanitizer(tmp_path):
    # the spin-then-sleep hand-off under ThreadSanitizer (host code only)
    exe = tmp_path / "hostpool_check_tsan"
    build = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=thread", "-I", CSRC,
                            os.path.join(HERE, "hostpool_check.cpp"), "-o", str(exe)], capture_output=True, text=True)
    if build.returncode != 0:
        import pytest
        pytest.skip("no ThreadSanitizer runtime: " + build.stderr[-200:])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok") and "WARNING: ThreadSanitizer" not in r.stderr, \
        r.stdout + r.stderr[-2000:]
