"""The tiles' geometry, checked on the CPU: the geometry structs of the
two-step and the single-step tile are host-callable, so host programs
(tests/native/tile2_geometry_check.hip and tile_geometry_check.hip, built
with hipcc as host code only, nothing runs on a GPU) enumerate every thread
of every tile of ragged and row-padded shapes, for the single-problem tile
shapes and every batch width class, and verify
bounds, alignment, the node held by every LDS slot (or register) a stencil
reads, and that every interior node is stored exactly once."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "native", "tile2_geometry_check.hip")
SRC1 = os.path.join(HERE, "native", "tile_geometry_check.hip")
CSRC = os.path.join(ROOT, "paper_2608_11882_amd", "csrc")


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
              shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(hipcc() is None, reason="hipcc not available")
def test_two_step_tile_geometry(tmp_path):
    exe = str(tmp_path / "tile2_geometry_check")
    subprocess.run([hipcc(), "-O1", "-std=c++17", "--offload-arch=gfx950", "-I" + CSRC, SRC,
                    "-o", exe], check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert res.returncode == 0 and res.stdout.strip().endswith("ALL OK"), res.stdout[-3000:]


@pytest.mark.skipif(hipcc() is None, reason="hipcc not available")
def test_single_step_tile_geometry(tmp_path):
    exe = str(tmp_path / "tile_geometry_check")
    subprocess.run([hipcc(), "-O1", "-std=c++17", "--offload-arch=gfx950", "-I" + CSRC, SRC1,
                    "-o", exe], check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert res.returncode == 0 and res.stdout.strip().endswith("ALL OK"), res.stdout[-3000:]


@pytest.mark.skipif(hipcc() is None, reason="hipcc not available")
@pytest.mark.parametrize("old,new", [
    # a ring column node is picked from the wrong element of its aligned load
    ("rsel = ri % VEC;", "rsel = (ri + 1) % VEC;"),
    # the x+ neighbour of a lane's last node is read one slot too far
    ("xp_slot = gl == TXL - 1 ? rowb + TX + 1 : own_slot + 1;",
     "xp_slot = gl == TXL - 1 ? rowb + TX + 1 : own_slot + 2;"),
    # the last interior row is left out of the update mask
    ("st[v] = (ia + v >= 1) && (ia + v <= nx - 2) && (j <= ny - 2);",
     "st[v] = (ia + v >= 1) && (ia + v <= nx - 2) && (j <= ny - 3);"),
])
def test_single_step_checker_catches_a_planted_mistake(tmp_path, old, new):
    inc = tmp_path / "inc"
    shutil.copytree(CSRC, inc)
    hdr = inc / "heat_tile.hpp"
    text = hdr.read_text()
    assert text.count(old) == 1
    hdr.write_text(text.replace(old, new))
    exe = str(tmp_path / "check_mutant")
    subprocess.run([hipcc(), "-O1", "-std=c++17", "--offload-arch=gfx950", "-I" + str(inc), SRC1,
                    "-o", exe], check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert res.returncode != 0 and "FAIL" in res.stdout


@pytest.mark.skipif(hipcc() is None, reason="hipcc not available")
@pytest.mark.parametrize("old,new", [

    # the right inner-ring column takes its own slot as its right neighbour
    ("r1xp_u = side == 0 ? rb + 2 : rb + 3 + TX;", "r1xp_u = side == 0 ? rb + 2 : rb + 2 + TX;"),
    # the lower outer-ring row is read one row too high
    ("const int rj = row == 0 ? max(j0 - 2, 0) : min(j0 + BY + 1, ny - 1);",
     "const int rj = row == 0 ? max(j0 - 2, 0) : min(j0 + BY, ny - 1);"),
    # an inner-ring column is updated on the last row
    ("r1st[0] = (ri_u >= 1) && (ri_u <= nx - 2) && (rj_u <= ny - 2);",
     "r1st[0] = (ri_u >= 1) && (ri_u <= nx - 2) && (rj_u <= ny - 1);"),
    # a run's march starts one plane late (its last plane is never written)
    ("const int start = ke - m * zb + 1;", "const int start = ke - m * zb + 2;"),
    # the early start is allowed to reach the Dirichlet plane 0
    ("if (start >= 1) return {start, m, ke + 1};", "if (start >= 0) return {start, m, ke + 1};"),
])
def test_checker_catches_a_planted_geometry_mistake(tmp_path, old, new):
    inc = tmp_path / "inc"
    shutil.copytree(CSRC, inc)
    hdr = inc / "heat_tile2.hpp"
    text = hdr.read_text()
    assert text.count(old) == 1
    hdr.write_text(text.replace(old, new))
    exe = str(tmp_path / "check_mutant")
    subprocess.run([hipcc(), "-O1", "-std=c++17", "--offload-arch=gfx950", "-I" + str(inc), SRC,
                    "-o", exe], check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert res.returncode != 0 and "FAIL" in res.stdout
