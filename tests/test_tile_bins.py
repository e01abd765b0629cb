"""CPU test of the tile-scratch invariant: whatever tiling a team holds when a
call runs, a query's tile count stays within the bins its scratch was sized for
and its tiles fit the launch's LDS (the arithmetic of csrc/mrv_tiles.hpp, which
k_query_info and the host share)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2604_23960_amd", "csrc")


def test_tile_bins_invariant(tmp_path):
    exe = str(tmp_path / "tile_bins_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "tile_bins_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
