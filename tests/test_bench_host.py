"""Host-side parts of bench.py (no GPU): the algorithmic cell counts behind the
GB/s metric, the multiply-add peak, and the refusal of more than one GPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


# (l, z, n) -> cells of one TFT (z = operand length) and of the ITFT (z = n, f = 0),
# counted from the top-level loops of Alg. 1 and Alg. 2 with the paper's split
@pytest.mark.parametrize("l,z,n,tft,itft", [
    (10, 500, 999, 3547, 4046),
    (13, 3000, 5999, 21031, 24030),
    (17, 50000, 99999, 350703, 400702),
    (11, 977, 1953, 6898, 7874),
])
def test_algorithmic_cells(l, z, n, tft, itft):
    assert bench.alg_cells_tft(l, z, n) == tft
    assert bench.alg_cells_itft(l, n, n, 0) == itft


def test_large_product_bytes():
    cells = 2 * bench.alg_cells_tft(17, 50000, 99999) + bench.alg_cells_itft(17, 99999, 99999, 0)
    assert cells == 1102108 and cells * 8192 == 9028468736


def test_full_transform_reads_and_writes_every_cell_twice():
    # z = n = L: every column and every row pass reads and writes all L cells
    for l in (4, 7, 10):
        L = 1 << l
        assert bench.alg_cells_tft(l, L, L) == 4 * L
        assert bench.alg_cells_itft(l, L, L, 0) == 4 * L


def test_issue_rate_and_cycles_are_inverse():
    # a full-rate wave64 instruction (4 clocks) on 256 CUs x 4 SIMDs at 2.4 GHz
    assert abs(bench.lane_ops_peak(4) - 256 * 4 * 2.4e9 * 16) < 1
    for c in (4, 8, 16, 5.5):
        assert abs(bench.cycles_per_wave_instr(bench.lane_ops_peak(c)) - c) < 1e-9


def test_host_threads_capped():
    nproc, used = bench.host_threads()
    assert nproc >= 1 and 1 <= used <= min(nproc, bench.CPU_THREAD_CAP)


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_pointwise_limb_macs_follow_the_products_method():
    """The pointwise roofline counts the multiply-accumulates the library
    performs: 64 inner products of 96 x 96 (N = 65536) or 64 x 64 (N = 32768)
    limbs for the sizes with one more Schoenhage-Strassen level, (N/32)^2
    otherwise."""
    import bench
    assert bench.pointwise_limb_macs(65536)[0] == 64 * 96 * 96
    assert bench.pointwise_limb_macs(32768)[0] == 64 * 64 * 64
    assert bench.pointwise_limb_macs(131072)[0] == 64 * 160 * 160
    assert bench.pointwise_limb_macs(8192)[0] == 256 * 256
    assert bench.pointwise_limb_macs(65536)[0] * 7 < (65536 // 32) ** 2
