"""Host check of the tile sweeps' index geometry (no GPU needed).

Compiles tests/tile_geometry_check.hip, which includes the library's
sv_apply.hip and replays the tile kernels' index arithmetic on the CPU with
the tile arguments the library builds (plain, spread and strided layouts,
every tile shape), and runs it: every tile of states up to 7 qubits above
the tile, and a sample of 64 tiles of states up to 34 qubits (targets up to
the top qubit).  A layout that drops, duplicates or misplaces an amplitude,
or puts a group member anywhere but its base plus its target bits, fails
here before any kernel runs with it.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_tile_geometry_covers_every_amplitude_once(tmp_path):
    exe = str(tmp_path / "tile_geometry_check")
    csrc = os.path.join(ROOT, "paper_2308_01999_amd", "csrc")
    cmd = [HIPCC, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
           os.path.join(ROOT, "tests", "tile_geometry_check.hip"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "fails 0" in r.stdout
