"""Host check of the addresses of the persistent leaf executor.

tests/native/leaf2_addr_check.cpp includes the kernel's own address header
(paper_0810_3203_amd/csrc/leaf2_addr.hpp) and checks, for every element size
the kernel serves (256 to 2048 limbs), both global layouts and every leaf size
it accepts, that the quad copies, the rotated reads of every lane, rotation
and word, and the limb positions stay inside the LDS allocation and the job's
cells, and that the copies move each dword exactly once.  It also shows that
the rotated-read base of a layout without the guard block falls below the
allocation, the condition that led the earlier out-of-line butterflies out of
the LDS aperture.
"""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_leaf2_addresses(tmp_path):
    exe = str(tmp_path / "leaf2_addr_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_0810_3203_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "leaf2_addr_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    last = r.stdout.strip().splitlines()[-1].split()
    assert last[0] == "checks" and int(last[1]) > 10_000_000 and last[3] == "0"
    assert int(last[5]) > 0  # unguarded bases do fall below the allocation
