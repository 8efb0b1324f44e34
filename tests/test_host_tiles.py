"""Host logic of the LDS tile builder (no GPU): compiled with g++ from the
library's host sources and run on several meshes and tile geometries."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1908_07038_amd", "csrc")


@pytest.fixture(scope="module")
def checker():
    d = tempfile.mkdtemp(prefix="tiles_check_")
    exe = os.path.join(d, "halo_tiles_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", exe, os.path.join(HERE, "host", "halo_tiles_check.cpp"),
                    os.path.join(CSRC, "mesh_build.cpp")], check=True)
    return exe


# (N, nlev, tile_rows, sweep_bands, ring, col_bytes, row_bytes, budget): FP32
# and FP64 column sizes, level chunks, tiny budgets (a tile per node or two),
# one-row tiles, one band per sweep, tiles taller than the mesh
GEOMS = [(16, 70, 32, 16, 1, 280, 80, 49152), (16, 137, 4, 8, 2, 280, 240, 49152),
         (32, 137, 32, 16, 1, 548, 80, 24576), (32, 137, 32, 16, 2, 368, 144, 65536),
         (1, 5, 1, 1, 1, 40, 144, 8192), (2, 70, 32, 16, 2, 16, 240, 16384),
         (8, 33, 1, 1, 1, 264, 144, 2600), (8, 33, 1000, 1000, 2, 132, 144, 8192),
         (64, 137, 7, 3, 1, 1096, 144, 65536)]


@pytest.mark.parametrize("geom", GEOMS, ids=[f"O{g[0]}-r{g[4]}-{g[7]}" for g in GEOMS])
def test_halo_tiles(checker, geom):
    r = subprocess.run([checker] + [str(v) for v in geom], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")


def test_node_too_large_for_budget(checker):
    # a 7-column stencil of 1 KiB columns cannot fit 4 KiB
    r = subprocess.run([checker, "4", "137", "32", "16", "1", "1024", "144", "4096"], capture_output=True, text=True)
    assert r.returncode == 3 and "REFUSED" in r.stdout, r.stdout
