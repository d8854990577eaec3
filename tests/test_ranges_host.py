"""CPU: the device pool's free-range bookkeeping (csrc/ranges.h) under random take / give sequences,
checked against a plain model by tests/ranges_check.cpp, and the RI product's closed-form tile order
(csrc/ri_tiles.h) against the plainly built list by tests/ri_tiles_check.cpp (both built here with
g++)."""
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


def test_ri_tile_order_against_list():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "ri_tiles_check")
        subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_2510_15204_amd", "csrc"),
                        os.path.join(ROOT, "tests", "ri_tiles_check.cpp"), "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
