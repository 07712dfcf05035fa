"""CPU checks of bench.py's host logic: the multi-GPU refusal and the
recorded HBM counters (used only while the kernel sources they were taken
on are unchanged)."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_follows_the_kernel_source():
    for kernel, rec in bench.PMC_TRAFFIC.items():
        current = True
        for path, digest in rec["sources"].items():
            with open(os.path.join(ROOT, path), "rb") as f:
                current &= hashlib.sha256(f.read()).hexdigest() == digest
        t = bench.pmc_traffic(kernel, rec["n"])
        if current:
            # 2 x FETCH_SIZE + WRITE_SIZE, within 0.1% of the algorithmic
            # read + write of a 2^n state
            abytes = 16 if "c128" in kernel else 8
            alg = 2 * (1 << rec["n"]) * abytes
            assert abs(t / alg - 1.0) < 1e-3, (kernel, t, alg)
        else:
            assert t is None
        assert bench.pmc_traffic(kernel, rec["n"] + 1) is None
    assert bench.pmc_traffic("no_such_kernel", 30) is None


def test_dominant_kernel_names():
    assert bench.dominant_kernel_name("c64", 5, 30) == "k_tile_c64_k5"
    assert bench.dominant_kernel_name("c128", 5, 30) == "k_tile_c128_k5"
    assert bench.dominant_kernel_name("c64", 6, 30) == "k_tile_c64_k6"
    assert bench.dominant_kernel_name("c128", 6, 30) == "k_tile_c128_k6"
    assert bench.dominant_kernel_name("c64", 5, 10) == "k_apply_mfma_c64_k5"
    assert bench.dominant_kernel_name("c128", 3, 30) == "k_apply_dense<double, 3>"
