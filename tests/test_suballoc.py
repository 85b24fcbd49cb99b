"""The device sub-allocator's logic (csrc/suballoc.h: best fit, split,
coalesce, trim) on the CPU over a malloc backend."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2212_00977_amd", "csrc")


def test_suballoc_random_ops(tmp_path):
    exe = str(tmp_path / "suballoc_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, "-o", exe,
                    os.path.join(HERE, "suballoc_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:")
