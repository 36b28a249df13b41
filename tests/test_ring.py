"""The serving loop's ring allocator (host C++), compiled with g++ and fuzzed on the CPU."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_ring_allocator_fuzz(tmp_path):
    exe = str(tmp_path / "ring_fuzz")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-o", exe, os.path.join(HERE, "cpp", "ring_fuzz.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok")
