"""Host check of the batched autotuner's cache file (no GPU needed).

Compiles tests/tune_cache_check.cpp with the host compiler against the
library's sv_tune_cache.h and runs it: records round-trip through the file,
merge by (architecture, qubit count), partial records keep the other part,
and malformed or foreign lines are skipped.  The file it leaves must parse
as JSON with one entry per record.
"""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = shutil.which("g++") or shutil.which("c++")


@pytest.mark.skipif(CXX is None, reason="no host C++ compiler")
def test_tune_cache_file(tmp_path):
    exe = str(tmp_path / "tune_cache_check")
    b = subprocess.run([CXX, "-O1", "-std=c++17", "-Wall", "-Werror", os.path.join(ROOT, "tests", "tune_cache_check.cpp"),
                        "-o", exe, "-pthread"], capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0 and "fails 0" in r.stdout, r.stdout[-4000:]
    doc = json.load(open(tmp_path / "tune.json"))
    assert doc["sv_autotune"] == 1
    got = {(e["arch"], e["n"]): e for e in doc["entries"]}
    assert set(got) == {("gfx950:sramecc+:xnack-", 10), ("gfx950:sramecc+:xnack-", 15), ("gfx942", 20)}
    assert got[("gfx950:sramecc+:xnack-", 15)]["tiles_per_wg"] == 2
    assert all(e["dtype"] == "c64" for e in doc["entries"])
