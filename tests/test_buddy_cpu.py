"""The server's arena allocator (host C++, shared with the library through
its header) built with g++ and checked by tests/buddy_check.cpp."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1801_05857_amd", "csrc")


def test_buddy_allocator(tmp_path):
    exe = tmp_path / "buddy_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe),
                           os.path.join(HERE, "buddy_check.cpp")])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout
