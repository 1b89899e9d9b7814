"""Host-side checks of bench.py (no GPU): the per-cell algorithmic bytes the
roofline figures rest on, the roofline arithmetic of the persistent solve and
of the two-right-hand-side solve, the measured-traffic gate, and the refusal
of more than one GPU."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bytes_per_cell_iteration():
    # mixed: A 56 + b 8 + x 8 + L 16 + y 4 forward, U 12 + y 4 + x 8 + x 8 backward
    assert bench.FWD_BYTES["mixed"] == 92 and bench.BWD_BYTES["mixed"] == 32
    # FP64: the factors and y in FP64
    assert bench.FWD_BYTES["fp64"] == 112 and bench.BWD_BYTES["fp64"] == 48
    assert bench.SOLVE_BYTES_MIXED == 124
    # a pair shares A and the factors: A 56 + L 16 + 2 (b 8 + x 8 + y 4); U 12 + 2 (y 4 + x 8 + x 8)
    assert bench.PAIR_FWD_BYTES == 112 and bench.PAIR_BWD_BYTES == 52


def test_persistent_solve_roofline():
    cells, n, ms = 256 ** 3, 4069, 3100.0
    r = bench.persist_roofline(cells, n, ms)
    alg = ((n + 1) * 92 + n * 32) * cells
    assert r["achieved"] == pytest.approx(alg / (ms * 1e-3) / 1e9, abs=0.06)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    # measured traffic only for the workload, iteration count and kernel source it was taken with
    assert r["traffic"] is None
    m = bench.MEASURED["single"]
    r = bench.persist_roofline(cells, m["iterations"], ms, workload="single")
    if bench.kernels_sha256() == bench.MEASURED["kernels_sha256"]:
        assert r["traffic"] == pytest.approx(m["persist_bytes"] / (ms * 1e-3) / 1e9, abs=0.06)
    else:
        assert r["traffic"] is None
    assert bench.persist_roofline(cells, m["iterations"] + 1, ms, workload="single")["traffic"] is None


def test_pair_roofline():
    cells, ms = 256 ** 3, 5500.0
    r = bench.pair_roofline(cells, [4069, 6023], ms)
    alg = ((4069 + 1) * 112 + 4069 * 52 + (1954 + 1) * 92 + 1954 * 32) * cells
    assert r["achieved"] == pytest.approx(alg / (ms * 1e-3) / 1e9, abs=0.06)
    # the order of the two right-hand sides does not matter
    assert bench.pair_roofline(cells, [6023, 4069], ms)["achieved"] == r["achieved"]
    # both stop together: the pair launch alone, no continuation
    r = bench.pair_roofline(cells, [100, 100], 10.0)
    assert r["achieved"] == pytest.approx((101 * 112 + 100 * 52) * cells / 1e-2 / 1e9, abs=0.06)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_working_set_flag():
    # 256^3 mixed: 104 B per cell resident, far beyond the 256 MiB last-level cache
    assert bench.working_set(256 ** 3) == {"working_set_mib": 1664.0, "cache_resident": False}
    assert bench.working_set(64 ** 3)["cache_resident"] is True
