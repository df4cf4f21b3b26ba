"""Host run of the leaf executor's arithmetic under a lockstep wave emulation.

tests/native/leaf2_ops_emu.cpp compiles the kernel's wave-level code
(paper_0810_3203_amd/csrc/fermat_leaf2_ops.hpp) for the host, with 64 threads
as the lanes of one wavefront, and runs every base case of Alg. 1 and Alg. 2
(L = 2) on two cells for elements of 256 to 2048 limbs: random operands, 0,
1, 2^N, 2^N - 1, operands filling one half, whole lane chunks of zeros or
ones, single limbs and long runs of ones, with twist exponents at every
rotation boundary.  Each result is compared here, with Python integers, with
the base case's definition in Z/(2^N+1) (tests/base_case_defs.py).

The emulation reproduces the source's meaning, not the compiler's output: a
wrong carry that the compiler introduced on the device (it once merged the
last limb of a dropped-carry chain into the next chain) shows up only in
tests/test_gpu_base_cases.py, which runs the same cases on the GPU.
"""

import os
import subprocess

import pytest

from tests.base_case_defs import expect

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("emu") / "leaf2_ops_emu")
    subprocess.check_call(["g++", "-O2", "-std=c++20", "-pthread", "-I",
                           os.path.join(ROOT, "paper_0810_3203_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "leaf2_ops_emu.cpp"), "-o", exe])
    return exe


@pytest.mark.parametrize("C,cases,seed", [(4, 300, 1), (8, 200, 2), (16, 120, 3), (32, 80, 4)])
def test_base_cases_emulated(emu_exe, C, cases, seed):
    r = subprocess.run([emu_exe, str(C), str(cases), str(seed)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.strip().splitlines()
    assert len(lines) == cases
    bad = []
    for ln in lines:
        f = ln.split()
        c, code, s = int(f[0]), int(f[1]), int(f[2])
        N = 32 * 64 * c
        x0 = int(f[3], 16) + (int(f[4]) << N)
        x1 = int(f[5], 16) + (int(f[6]) << N)
        y0 = int(f[7], 16) + (int(f[8]) << N)
        y1 = int(f[9], 16) + (int(f[10]) << N)
        e0, e1 = expect(code, N, s, x0, x1)
        canon = all(v <= (1 << N) and (v >> N == 0 or v == 1 << N) for v in (y0, y1))
        if y0 != e0 or (e1 is not None and y1 != e1) or not canon:
            bad.append((code, s, hex(x0)[:20], hex(x1)[:20]))
    assert not bad, "%d of %d base cases wrong, first: %s" % (len(bad), cases, bad[:5])


def _emulate_plan(emu_exe, N, direction, l, s, z, n, f, leaf, cells):
    """Runs an exported plan's jobs, pass after pass, on the emulated wave."""
    import paper_0810_3203_amd as T
    W = N // 32
    L = 1 << l
    e = T.Plan(T.fermat_ring(N), direction, l, s, z, n, f, 0, leaf).export()
    ops = [(code | (i0 << 4) | (i1 << 18), (b & 0xFFFFFFF) | (alog << 28)) for code, i0, i1, alog, b in e["ops"]]
    jobs = []
    for jb, jc, _ in e["passes"]:
        jobs.extend(e["jobs"][jb:jb + jc])
    lines = ["%d %d %d %d %d %d" % (L, e["ord"], len(e["progs"]), len(e["steps"]), len(ops), len(jobs))]
    lines += ["%d %d %d" % p for p in e["progs"]]
    lines += ["%d %d" % t for t in e["steps"]]
    lines += ["%d %d" % o for o in ops]
    lines += ["%d %d %d %d %d %d" % j for j in jobs]
    for v in cells:
        lines.append("%0*x %d" % (W * 8, v & ((1 << N) - 1), v >> N))
    r = subprocess.run([emu_exe, "plan", str(W // 64)], input="\n".join(lines) + "\n", capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    out = []
    for ln in r.stdout.strip().splitlines():
        h, t = ln.split()
        out.append(int(h, 16) + (int(t) << N))
    return out


@pytest.mark.parametrize("kind,s", [("sparse", 7), ("random", 1000)])
def test_leaf_programs_emulated(emu_exe, kind, s):
    """Whole transforms (two passes of 8-cell leaves) on the emulated wave: TFT
    (Alg. 1) against eq. (1), and the ITFT (Alg. 2) of eq. (1)'s values against
    L times the input.  Sparse inputs (half-width values) keep long zero runs, so
    carries cross many lanes."""
    import random
    from oracle import tft_oracle as O
    N, l, z, n = 8192, 6, 32, 63
    ring = O.FermatRing(N)
    L = 1 << l
    rng = random.Random(s)
    a = [rng.getrandbits(N // 2) if kind == "sparse" else rng.randrange(ring.p) for _ in range(z)]
    a[0] = ring.p - 1
    got = _emulate_plan(emu_exe, N, 0, l, s, z, n, 0, 3, a + [0] * (L - z))
    assert got[:n] == O.tft(ring, L, s, z, n, a)
    inputs, expect = O.itft_case(ring, L, s, n, n, 0, a + [0] * (n - z))
    got = _emulate_plan(emu_exe, N, 1, l, s, n, n, 0, 3, list(inputs) + [0] * (L - n))
    assert got[:n] == expect
