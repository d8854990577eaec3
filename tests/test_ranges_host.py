"""CPU: the device pool's free-range bookkeeping (csrc/ranges.h) under random take / give sequences,
checked against a plain model by tests/ranges_check.cpp (built here with g++)."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_range_map_against_model():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "ranges_check")
        subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_2510_15204_amd", "csrc"),
                        os.path.join(ROOT, "tests", "ranges_check.cpp"), "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
