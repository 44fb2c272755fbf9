"""The server's range allocator (admission and eviction accounting), built
from its header with the host compiler and run on the CPU."""
import os
import subprocess


def test_arena_allocator(tmp_path):
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "arena_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fsanitize=address,undefined", "-o", exe,
                    os.path.join(here, "native", "arena_test.cpp")], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "arena ok" in out.stdout
