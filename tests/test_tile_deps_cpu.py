"""The dependency rule of the tile-ordered persistent pool form, checked on
the CPU: tests/c/tile_deps_check.cpp includes the same constexpr header the
kernel uses (csrc/tile_deps.hpp) and verifies, over some 6,200 slot
geometries (whole-row tiles of every width, column tiles of 1 to 512 columns,
ragged last tiles, grids of one or two rows), that every tile owning a node a
tile's iteration reads is among the tiles that tile waits for."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_read_dependency_is_waited_for(tmp_path):
    exe = str(tmp_path / "tile_deps_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror",
                    "-I" + os.path.join(ROOT, "paper_2303_08163_amd", "csrc"),
                    os.path.join(ROOT, "tests", "c", "tile_deps_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.startswith("ok "), out.stdout + out.stderr
